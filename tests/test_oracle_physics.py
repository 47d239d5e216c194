"""Pins of the pointwise physics: logarithmic mean, two-point fluxes, entropy variables, C_mj."""
import math

import mpmath
import numpy as np
import pytest

from oracle import gas as G

GAS = G.Gas(gamma=1.4, R=0.7, mu=0.013, Pr=0.72)


def rand_states(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = rng.uniform(0.5, 2.0, n)
    u = rng.normal(0, 0.5, (3, n))
    P = rng.uniform(0.5, 2.0, n)
    E = P / (GAS.gamma - 1) + 0.5 * rho * (u * u).sum(0)
    return np.stack([rho, rho * u[0], rho * u[1], rho * u[2], E])


def euler_flux_from_primitives(q):
    """Eq. ns_iflux written from primitives independently of the oracle."""
    rho = q[0]
    u = q[1:4] / q[0]
    P = (GAS.gamma - 1) * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0])
    H = (q[4] + P) / rho
    return np.stack([np.stack([rho * u[m], rho * u[m] * u[0] + (m == 0) * P,
                               rho * u[m] * u[1] + (m == 1) * P, rho * u[m] * u[2] + (m == 2) * P,
                               rho * u[m] * H]) for m in range(3)])


def test_log_mean_closed_forms():
    assert abs(G.log_mean(np.array(math.e), np.array(1.0)) - (math.e - 1)) < 1e-15
    a = np.array([0.3, 1.0, 7.5])
    assert np.all(G.log_mean(a, a) == a)


def test_log_mean_vs_mpmath():
    mpmath.mp.dps = 40
    rng = np.random.Generator(np.random.PCG64(3))
    b = rng.uniform(0.1, 10, 400)
    rel = np.concatenate([10 ** rng.uniform(-12, 0.5, 300), rng.uniform(-2e-3, 2e-3, 100)])
    a = b * (1 + rel)
    a = np.where(a > 0, a, b)
    L = G.log_mean(a, b)
    for ai, bi, Li in zip(a, b, L):
        A, B = mpmath.mpf(float(ai)), mpmath.mpf(float(bi))
        ex = A if A == B else (A - B) / (mpmath.log(A) - mpmath.log(B))
        assert abs(Li - float(ex)) <= 4e-16 * float(ex)


def test_log_mean_long_double_series_accuracy():
    b = np.longdouble(1.3)
    for d in [1e-4, 5e-4, 9.9e-4 * 2]:
        a = b * (1 + np.longdouble(d))
        ex = (a - b) / np.log1p((a - b) / b)
        assert abs(G.log_mean(a, b) - ex) / ex < 1e-18


@pytest.mark.parametrize("flux", [G.chandrashekar_flux, G.kennedy_gruber_flux, G.central_flux])
def test_two_point_consistency_and_symmetry(flux):
    qi, qj = rand_states(50, 1), rand_states(50, 2)
    F = flux(qi, qi, GAS)
    assert np.abs(F - euler_flux_from_primitives(qi)).max() < 1e-13
    assert np.abs(flux(qi, qj, GAS) - flux(qj, qi, GAS)).max() < 1e-14


def test_chandrashekar_tadmor_condition():
    """(w_i - w_j) . F#_m = psi_m,i - psi_m,j with the entropy flux potential psi_m = R rho U_m."""
    qi, qj = rand_states(200, 4), rand_states(200, 5)
    # include nearly equal states (series branch of the log mean)
    qj[:, :50] = qi[:, :50] * (1 + 1e-5 * rand_states(50, 6) / rand_states(50, 6).mean())
    F = G.chandrashekar_flux(qi, qj, GAS)
    dw = G.entropy_variables(qi, GAS) - G.entropy_variables(qj, GAS)
    for m in range(3):
        lhs = (dw * F[m]).sum(0)
        rhs = GAS.R * (qi[1 + m] - qj[1 + m])
        assert np.abs(lhs - rhs).max() < 1e-13


def test_entropy_variables_are_gradient_of_entropy_function():
    q = rand_states(20, 7)
    W = G.entropy_variables(q, GAS)
    h = 1e-30
    for c in range(5):
        dq = np.zeros_like(q, dtype=complex)
        dq[c] = 1j * h
        dS = G.entropy_function(q + dq, GAS).imag / h
        assert np.abs(dS - W[c]).max() < 1e-13 * (1 + np.abs(W[c]).max())


def _dW_dQ(q):
    """Jacobian dW/dQ per node by the complex step, shape (5, 5, n)."""
    h = 1e-30
    cols = []
    for c in range(5):
        dq = np.zeros_like(q, dtype=complex)
        dq[c] = 1j * h
        cols.append(G.entropy_variables(q + dq, GAS).imag / h)
    return np.stack(cols, axis=1)


def test_viscous_blocks_match_stress_and_heat_flux():
    """F^V_m = sum_j C_mj dW/dx_j equals [0, tau_1m, tau_2m, tau_3m, tau_im U_i + kappa dT/dx_m]
    (eqs. Fv, tau; Fourier heat flux) for random primitive gradients."""
    n = 30
    q = rand_states(n, 8)
    rng = np.random.Generator(np.random.PCG64(9))
    drho, du, dT = rng.normal(size=(3, n)), rng.normal(size=(3, 3, n)), rng.normal(size=(3, n))  # [j], [k][j]
    rho = q[0]
    u = q[1:4] / rho
    P = (GAS.gamma - 1) * (q[4] - 0.5 * rho * (u * u).sum(0))
    T = P / (rho * GAS.R)
    cv = GAS.R / (GAS.gamma - 1)
    # dQ/dx_j from the primitive gradients: E = rho (cv T + |u|^2/2)
    dQ = np.stack([np.stack([drho[j],
                             drho[j] * u[0] + rho * du[0, j], drho[j] * u[1] + rho * du[1, j],
                             drho[j] * u[2] + rho * du[2, j],
                             drho[j] * (cv * T + 0.5 * (u * u).sum(0))
                             + rho * (cv * dT[j] + (u * du[:, j]).sum(0))]) for j in range(3)])
    dWdQ = _dW_dQ(q)
    gW = np.einsum("ab...,jb...->ja...", dWdQ, dQ)
    FV = G.viscous_flux(q, gW, GAS)
    mu, kap = GAS.mu, GAS.kappa
    div = du[0, 0] + du[1, 1] + du[2, 2]
    for m in range(3):
        tau = [mu * (du[i, m] + du[m, i] - (2 / 3) * (i == m) * div) for i in range(3)]
        ref = np.stack([0 * rho, tau[0], tau[1], tau[2],
                        tau[0] * u[0] + tau[1] * u[1] + tau[2] * u[2] + kap * dT[m]])
        assert np.abs(FV[m] - ref).max() < 1e-12 * (1 + np.abs(ref).max())


def test_viscous_blocks_symmetric_psd():
    q = rand_states(25, 10)
    C = G.viscous_blocks(q, GAS)
    assert np.abs(C - np.swapaxes(np.swapaxes(C, 0, 1), 2, 3)).max() < 1e-15
    big = np.transpose(C, (4, 0, 2, 1, 3)).reshape(25, 15, 15)
    ev = np.linalg.eigvalsh(big)
    assert ev.min() > -1e-14 * ev.max()
