"""Oracle pins for wall boundary faces (slip wall -2, adiabatic no-slip wall -3).

* A gas at rest with uniform density and pressure stays at rest between walls (warped mesh).
* Entropy: with walls the total entropy rate is the interface dissipation of interior faces plus,
  on wall faces, one-sided dissipation written in closed form (LLF) or with the matrix operator;
  with entropy-conservative interfaces the walls produce no entropy at all (inviscid).  The viscous
  budget with adiabatic no-slip walls is the volume dissipation plus the interior-penalty terms,
  with no boundary term: the wall passes no heat and does no work.
* Conservation: walls keep mass, and energy (adiabatic), exactly.
* A slip wall is a mirror: on an affine mesh the residual next to slip walls equals that of the
  doubled periodic domain holding the mirror image of the state.
* The wall-bounded manufactured solution converges under h-refinement (truncation error).
"""
import numpy as np
import pytest
import torch

import workloads as W
from workloads import mms
from oracle import gas as G
from oracle import geometry, operators, residual as R


class WallCase:
    def __init__(self, prob, amp=0.03, seed=1):
        self.prob = prob
        self.sbp = operators.SBP1D(prob.p)
        self.x = W.coords(prob, self.sbp.x).numpy()
        self.metric = geometry.curl_metrics(self.x, self.sbp.D)
        self.jac = geometry.jacobian(self.x, self.sbp.D)
        self.nbr = W.problem_neighbours(prob)
        q = W.state(prob, torch.as_tensor(self.x)).numpy()
        rng = np.random.Generator(np.random.PCG64(seed))
        q[0] *= 1.0 + amp * rng.uniform(-1, 1, q[0].shape)
        q[1:4] += amp * rng.uniform(-1, 1, q[1:4].shape)
        q[4] *= 1.0 + amp * rng.uniform(-1, 1, q[4].shape)
        self.q = q
        self.prm = R.Params.of(prob)
        self.gas = self.prm.gas

    def residual(self, q=None, prm=None):
        return R.residual(self.q if q is None else q, self.metric, self.jac, self.nbr, self.sbp,
                          self.prm if prm is None else prm)

    def wj(self):
        w = self.sbp.w
        return np.einsum("i,j,k->ijk", w, w, w) * self.jac

    def faces(self, fn_interior, fn_wall):
        """sum over interior node pairs (once each) of w_t fn_interior(...) plus sum over wall face
        nodes of w_t fn_wall(qi, Ai, Ji, kind)."""
        wt = np.einsum("i,j->ij", self.sbp.w, self.sbp.w)
        q, tot = self.q, 0.0
        for l, s, f, own, nb in R._faces(self.sbp.p):
            nb_e = self.nbr[:, f]
            inn = nb_e >= 0
            Al = self.metric[3 * l:3 * l + 3]
            qi, Ai, Ji = R._take(q, own, l), R._take(Al, own, l), R._take(self.jac, own, l)
            if inn.any() and fn_interior is not None:
                e = np.nonzero(inn)[0]
                qn = R._take(q[:, nb_e[e]], nb, l)
                An = R._take(Al[:, nb_e[e]], nb, l)
                Jn = R._take(self.jac[nb_e[e]], nb, l)
                v = fn_interior(qi[:, e], qn, 0.5 * (Ai[:, e] + An), Ai[:, e], An, Ji[e], Jn)
                tot += 0.5 * (wt * v).sum()
            for kind in (-2, -3):
                e = np.nonzero(nb_e == kind)[0]
                if len(e):
                    tot += (wt * fn_wall(qi[:, e], Ai[:, e], Ji[e], kind)).sum()
        return tot


def ghost(qi, A, kind):
    """The wall's ghost state written out: momentum reflected about the face (slip) or reversed
    (no-slip)."""
    g = qi.copy()
    if kind == -2:
        mn = (qi[1:4] * A).sum(0) / (A * A).sum(0)
        g[1:4] = qi[1:4] - 2.0 * mn * A
    else:
        g[1:4] = -qi[1:4]
    return g


def _wall_prob(p, E, kind, mu, diss, A=0.1, eta=1.0, box=None, seed=3):
    return W.make_problem(p=p, E=E, L=2.0, A=A, mu=mu, eta=eta, iface_diss=diss, seed=seed,
                          u_rms=0.3, box=box if box is not None else (kind, None, kind))


# ------------------------------------------------------------------ rest state
@pytest.mark.parametrize("kind,mu", [(-2, 0.0), (-3, 0.0), (-3, 0.02)])
def test_gas_at_rest_between_walls_stays_at_rest(kind, mu):
    prob = W.make_problem(p=3, E=3, L=2.0, A=0.12, mu=mu, init="constant", const=(1.2, 0.0, 0.0, 0.0, 0.9),
                          box=(kind, kind, kind))
    c = WallCase(prob, amp=0.0)
    r = c.residual()
    assert np.abs(r).max() < 1e-12


# ------------------------------------------------------------------ entropy, inviscid
@pytest.mark.parametrize("kind", [-2, -3])
def test_walls_produce_no_entropy_with_conservative_interfaces(kind):
    c = WallCase(_wall_prob(4, 3, kind, 0.0, 0))
    r = c.residual()
    w = G.entropy_variables(c.q, c.gas)
    tot = (c.wj() * (w * r).sum(0)).sum()
    mag = (c.wj() * np.abs(w * r).sum(0)).sum()
    assert abs(tot) < 1e-14 * mag


@pytest.mark.parametrize("kind", [-2, -3])
def test_wall_entropy_identity_lax_friedrichs(kind):
    c = WallCase(_wall_prob(3, 3, kind, 0.0, 1))
    gas = c.gas
    lhs = (c.wj() * (G.entropy_variables(c.q, gas) * c.residual()).sum(0)).sum()

    def lam(qx, n):
        rho, u, P, T = G.primitives(qx, gas)
        return np.abs((u * n).sum(0)) + G.sound_speed(qx, gas) * np.sqrt((n * n).sum(0))

    def interior(qi, qn, nbar, Ai, An, Ji, Jn):
        dw = G.entropy_variables(qi, gas) - G.entropy_variables(qn, gas)
        return -np.maximum(lam(qi, nbar), lam(qn, nbar)) / 2 * (dw * (qi - qn)).sum(0)

    def wall(qi, A, J, k):
        rho, u, P, T = G.primitives(qi, gas)
        # w . (q_i - q_ghost): only the momentum differs, by 2 (m.n)n (slip) or 2m (no-slip),
        # and the momentum entropy variables are U/T
        un2 = ((u * A).sum(0)) ** 2 / (A * A).sum(0) if k == -2 else (u * u).sum(0)
        return -lam(qi, A) / 2 * (2.0 * rho * un2 / T)

    rhs = c.faces(interior, wall)
    assert rhs < 0
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


@pytest.mark.parametrize("kind", [-2, -3])
def test_wall_entropy_identity_matrix_dissipation(kind):
    c = WallCase(_wall_prob(3, 3, kind, 0.0, 2))
    gas = c.gas
    lhs = (c.wj() * (G.entropy_variables(c.q, gas) * c.residual()).sum(0)).sum()

    def interior(qi, qn, nbar, Ai, An, Ji, Jn):
        dw = G.entropy_variables(qi, gas) - G.entropy_variables(qn, gas)
        return -0.5 * (dw * G.matrix_dissipation(qi, qn, nbar, gas)).sum(0)

    wall_terms = []

    def wall(qi, A, J, k):
        v = -0.5 * (G.entropy_variables(qi, gas) * G.matrix_dissipation(qi, ghost(qi, A, k), A, gas)).sum(0)
        wall_terms.append(v)
        return v

    rhs = c.faces(interior, wall)
    assert all((v <= 1e-15).all() for v in wall_terms)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


# ------------------------------------------------------------------ entropy, viscous
@pytest.mark.parametrize("eta", [0.0, 1.0])
def test_adiabatic_wall_viscous_entropy_budget(eta):
    """sum wJ w.(dq/dt)_visc = -sum wJ g C g - eta (interior pairs + wall nodes) penalties, with no
    boundary term."""
    box = (None, -3, -3)
    c = WallCase(_wall_prob(3, 3, -3, 0.02, 0, eta=eta, box=box))
    gas = c.gas
    rv = c.residual() - c.residual(prm=R.Params(mu=0.0, iface_diss=0))
    w = G.entropy_variables(c.q, gas)
    lhs = (c.wj() * (w * rv).sum(0)).sum()
    th = R.gradient_theta(c.q, c.metric, c.nbr, np.arange(c.prob.K), c.sbp, c.prm)
    g = np.stack([sum(c.metric[3 * a + j] * th[a] for a in range(3)) / c.jac for j in range(3)])
    vol = -(c.wj() * (g * G.viscous_flux(c.q, g, gas)).sum(axis=(0, 1))).sum()

    def interior(qi, qn, nbar, Ai, An, Ji, Jn):
        Lm = 0.5 * (R.chat_ll(qi, Ai, Ji, gas) + R.chat_ll(qn, An, Jn, gas))
        dw = G.entropy_variables(qi, gas) - G.entropy_variables(qn, gas)
        return -eta * np.einsum("a...,ab...,b...->...", dw, Lm, dw)

    def wall(qi, A, J, k):
        qg = ghost(qi, A, k)
        Lm = 0.5 * (R.chat_ll(qi, A, J, gas) + R.chat_ll(qg, A, J, gas))
        wi = G.entropy_variables(qi, gas)
        return -eta * np.einsum("a...,ab...,b...->...", wi, Lm, wi - G.entropy_variables(qg, gas))

    pen = c.faces(interior, wall)
    assert vol < 0 and pen <= 0
    assert abs(lhs - (vol + pen)) < 1e-12 * abs(vol + pen)


# ------------------------------------------------------------------ conservation
@pytest.mark.parametrize("kind,mu,diss", [(-2, 0.0, 1), (-2, 0.0, 2), (-3, 0.0, 1), (-3, 0.03, 1), (-3, 0.03, 2)])
def test_walls_conserve_mass_and_energy(kind, mu, diss):
    c = WallCase(_wall_prob(3, 3, kind, mu, diss, box=(kind, kind, None)))
    r = c.residual()
    tot = (c.wj() * r).sum(axis=(1, 2, 3, 4))
    mag = (c.wj() * np.abs(r)).sum(axis=(1, 2, 3, 4))
    assert abs(tot[0]) < 1e-14 * mag[0]
    assert abs(tot[4]) < 1e-14 * mag[4]
    # the walls push on the gas: momentum normal to them is not conserved
    assert abs(tot[1]) > 1e-6 * mag[1]


# ------------------------------------------------------------------ slip wall = mirror
@pytest.mark.parametrize("diss,two_point", [(1, 0), (2, 0), (1, 2), (0, 0)])
def test_slip_wall_equals_mirrored_domain(diss, two_point):
    p, E = 2, 2
    prob = W.make_problem(p=p, E=E, L=2.0, A=0.0, mu=0.0, iface_diss=diss, two_point=two_point,
                          seed=11, u_rms=0.3, box=(-2, None, None))
    c = WallCase(prob)
    half = c.residual()
    # doubled domain: 2E elements along x_1 over [0, 2L]; element e1' = 2E-1-e1 holds the mirror
    # image of element e1 about x_1 = L (node i1 -> N-1-i1, x_1 -> 2L - x_1, m_1 -> -m_1)
    N, K, L = prob.N, prob.K, prob.L
    e = np.arange(K)
    e1, e2, e3 = e % E, (e // E) % E, e // (E * E)
    K2 = 2 * K
    x2 = np.zeros((3, K2, N, N, N))
    q2 = np.zeros((5, K2, N, N, N))
    new = e1 + 2 * E * e2 + 2 * E * E * e3
    mir = (2 * E - 1 - e1) + 2 * E * e2 + 2 * E * E * e3
    x2[:, new], q2[:, new] = c.x, c.q
    xm = c.x[..., ::-1].copy()
    xm[0] = 2 * L - xm[0]
    qm = c.q[..., ::-1].copy()
    qm[1] = -qm[1]
    x2[:, mir], q2[:, mir] = xm, qm
    sbp = c.sbp
    metric2, jac2 = geometry.curl_metrics(x2, sbp.D), geometry.jacobian(x2, sbp.D)
    ee = np.arange(K2)
    a1, a2, a3 = ee % (2 * E), (ee // (2 * E)) % E, ee // (2 * E * E)

    def idx(b1, b2, b3):
        return (b1 % (2 * E)) + 2 * E * (b2 % E) + 2 * E * E * (b3 % E)

    nbr2 = np.stack([idx(a1 - 1, a2, a3), idx(a1 + 1, a2, a3), idx(a1, a2 - 1, a3),
                     idx(a1, a2 + 1, a3), idx(a1, a2, a3 - 1), idx(a1, a2, a3 + 1)], axis=1)
    full = R.residual(q2, metric2, jac2, nbr2, sbp, c.prm)
    assert np.abs(full[:, new] - half).max() < 1e-13 * np.abs(half).max()


# ------------------------------------------------------------------ accuracy
@pytest.mark.parametrize("A", [0.0, 0.05])
@pytest.mark.parametrize("p,min_rate,bound", [(2, 1.6, 0.15), (3, 2.3, 0.02)])
def test_channel_truncation_error_converges(A, p, min_rate, bound):
    errs = []
    for E in (2, 4, 8):
        prob = W.channel_problem(p, E, A=A)
        sbp = operators.SBP1D(p)
        x = W.coords(prob, sbp.x).numpy()
        metric, jac = geometry.curl_metrics(x, sbp.D), geometry.jacobian(x, sbp.D)
        q = mms.conservative(x, kind="channel")
        S = mms.source(x, kind="channel")
        r = R.residual(q, metric, jac, W.problem_neighbours(prob), sbp, R.Params.of(prob),
                       source=S, chunk=256)
        scale = np.abs(S).max(axis=(1, 2, 3, 4))[:, None, None, None, None]
        err = np.abs(r) / scale
        errs.append(err.max())
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < bound, errs
    assert rates[-1] > min_rate, (errs, rates)
    # the elements along the walls are no less accurate than the rest
    e2 = (np.arange(8 ** 3) // 8) % 8
    at_wall = (e2 == 0) | (e2 == 7)
    assert err[:, at_wall].max() < 1.5 * err[:, ~at_wall].max()


def test_channel_data_satisfies_the_wall_conditions():
    g = np.linspace(0.0, 1.0, 7)
    for x2 in (0.0, 1.0):
        X = np.stack(np.meshgrid(g, [x2], g, indexing="ij"))
        rho, u, P = mms.primitives(X, "channel")
        assert np.abs(u).max() < 1e-15
        h = 1e-6
        Xp, Xm = X.copy(), X.copy()
        Xp[1] += h
        Xm[1] -= h
        T = lambda Y: mms.primitives(Y, "channel")[2] / (mms.primitives(Y, "channel")[0] * mms.CHANNEL_R)  # noqa
        assert np.abs((T(Xp) - T(Xm)) / (2 * h)).max() < 1e-8


def test_invalid_wall_uses_are_errors():
    prob = _wall_prob(1, 2, -2, 0.01, 1)
    c = WallCase(prob)
    with pytest.raises(ValueError):
        c.residual()   # slip walls with viscosity
    c.nbr = c.nbr.copy()
    c.nbr[0, 0] = -7
    with pytest.raises(ValueError):
        c.residual(prm=R.Params(mu=0.0))
