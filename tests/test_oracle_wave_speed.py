"""Pins of the wave speed of the local Lax-Friedrichs interface dissipation.

The dissipation is -(lam / (2 w_end)) (q_i - q_nu) with lam the larger of the two sides' largest
characteristic speeds in the averaged face metric nbar (interface SAT of the linear
convection-diffusion section, entropy-stable variant).  Nothing in the residual's other pins fixes
the size of lam (the entropy budget holds for any lam >= 0), so it is checked here against
quantities computed without the oracle's sound-speed formula:

* the spectral radius of the Euler flux Jacobian d(F(q) . n)/dq, taken by complex step of the
  nodal flux and a numerical eigendecomposition, for random states, gases and unnormalised n;
* c^2 = dP/drho at constant specific entropy (complex step of P(rho) along an isentrope);
* the dissipation the residual actually applies at face-centre nodes, recovered from the
  difference of the residual with and without it, against the eigenvalue-based speed of both
  sides in the averaged metric nbar = (A_l,i + A_l,nu) / 2.
A speed without gamma, or one scaled by |A_l,i| instead of |nbar|, fails these checks.
"""
import numpy as np

import workloads as W
from helpers import Case
from oracle import gas as G
from oracle import residual as R


def _random_states(rng, n, gas):
    rho = rng.uniform(0.3, 3.0, n)
    u = rng.uniform(-2.0, 2.0, (3, n))
    P = rng.uniform(0.2, 5.0, n)
    return np.stack([rho, rho * u[0], rho * u[1], rho * u[2],
                     P / (gas.gamma - 1.0) + 0.5 * rho * (u * u).sum(0)])


def _jacobian_spectral_radius(q, n, gas):
    """max |eig(d(F(q) . n)/dq)| per column of q (complex step, numpy eig)."""
    out = np.zeros(q.shape[1])
    h = 1e-30
    for j in range(q.shape[1]):
        A = np.zeros((5, 5))
        for b in range(5):
            qc = q[:, j:j + 1].astype(np.complex128)
            qc[b] += 1j * h
            A[:, b] = np.imag(G.contract(G.euler_flux(qc, gas), n[:, j:j + 1].astype(np.complex128))[:, 0]) / h
        out[j] = np.abs(np.linalg.eigvals(A)).max()
    return out


def test_wave_speed_is_the_flux_jacobian_spectral_radius():
    rng = np.random.Generator(np.random.PCG64(2024))
    for gamma, Rg in ((1.4, 1.0), (5.0 / 3.0, 287.0), (1.3, 0.5)):
        gas = G.Gas(gamma, Rg)
        q = _random_states(rng, 80, gas)
        n = rng.normal(size=(3, 80)) * rng.uniform(0.1, 5.0, 80)
        ref = _jacobian_spectral_radius(q, n, gas)
        got = G.max_wave_speed(q, n, gas)
        assert np.all(np.abs(got - ref) <= 1e-13 * ref), np.abs(got / ref - 1).max()


def test_sound_speed_squared_is_the_isentropic_pressure_derivative():
    rng = np.random.Generator(np.random.PCG64(2025))
    for gamma, Rg in ((1.4, 1.0), (5.0 / 3.0, 287.0)):
        gas = G.Gas(gamma, Rg)
        q = _random_states(rng, 50, gas)
        rho0 = q[0]
        s0 = G.entropy(q, gas)   # s = R/(gamma-1) log T - R log rho
        h = 1e-30
        rho = rho0 + 1j * h
        T = np.exp((s0 + Rg * np.log(rho)) * (gamma - 1.0) / Rg)
        dPdrho = np.imag(rho * Rg * T) / h
        c = G.sound_speed(q, gas)
        assert np.all(np.abs(c * c - dPdrho) <= 1e-13 * dPdrho)


def test_lax_friedrichs_dissipation_in_the_residual_uses_the_spectral_radius():
    """At nodes on exactly one face the dissipation is -(lam/(2 w_end)) (q_i - q_nu); lam recovered
    from the residual equals max over both sides of the Jacobian spectral radius in nbar."""
    c = Case(W.make_problem(p=2, E=2, L=2.0, A=0.12, mu=0.0, seed=41, u_rms=0.4))
    q = c.jumpy(0.2, seed=3)
    elems = np.arange(c.prob.K)
    on = R.inviscid_sat(q, c.metric, c.nbr, elems, c.sbp, R.Params(iface_diss=1))
    off = R.inviscid_sat(q, c.metric, c.nbr, elems, c.sbp, R.Params(iface_diss=0))
    diss = on - off
    w_end = c.sbp.w[0]
    N = c.sbp.N
    gas = c.prm.gas
    checked = 0
    for e in range(c.prob.K):
        for l in range(3):
            for side in (0, 1):
                il = 0 if side == 0 else N - 1
                nb = c.nbr[e, 2 * l + side]
                # face-centre node: index il along direction l, 1 along the other two
                idx = [1, 1, 1]
                idx[l] = il
                jdx = list(idx)
                jdx[l] = N - 1 - il
                own = (e, idx[2], idx[1], idx[0])
                par = (nb, jdx[2], jdx[1], jdx[0])
                qi, qn = q[(slice(None),) + own], q[(slice(None),) + par]
                Ai = c.metric[(slice(3 * l, 3 * l + 3),) + own]
                An = c.metric[(slice(3 * l, 3 * l + 3),) + par]
                nbar = 0.5 * (Ai + An)
                lam_ref = max(_jacobian_spectral_radius(qi[:, None], nbar[:, None], gas)[0],
                              _jacobian_spectral_radius(qn[:, None], nbar[:, None], gas)[0])
                dq = qi - qn
                k = int(np.argmax(np.abs(dq)))
                lam = -2.0 * w_end * diss[(k,) + own] / dq[k]
                assert abs(lam - lam_ref) <= 1e-12 * lam_ref, (lam, lam_ref)
                # and the dissipation is that multiple of the jump in every component
                assert np.allclose(diss[(slice(None),) + own], -(lam_ref / (2 * w_end)) * dq,
                                   rtol=1e-11, atol=1e-14 * np.abs(diss).max())
                checked += 1
    assert checked == 6 * c.prob.K
