"""Pins of the oracle residual: identities the method is built to satisfy (entropy conservation and
stability, conservation, freestream), the literal dense-matrix form, the linear split form, the
paper's stationary isentropic vortex and symbolic derivatives of the continuous equations."""
import math

import numpy as np
import pytest
import sympy as sp
import torch

import workloads as W
from helpers import Case, rel_err
from oracle import dense, gas as G, jvp, operators, residual as R
from oracle.geometry import apply_D


def face_sum(c, q, fn):
    """sum over interface node pairs (each counted once) of w_t * fn(qi, qn, nbar, Ai, An, Ji, Jn)."""
    tot = 0.0
    wt = np.einsum("i,j->ij", c.sbp.w, c.sbp.w)
    for l, s, f, own, nb in R._faces(c.sbp.p):
        qi = R._take(q, own, l)
        qn = R._take(q[:, c.nbr[:, f]], nb, l)
        Ai = R._take(c.metric[3 * l:3 * l + 3], own, l)
        An = R._take(c.metric[3 * l:3 * l + 3][:, c.nbr[:, f]], nb, l)
        Ji, Jn = R._take(c.jac, own, l), R._take(c.jac[c.nbr[:, f]], nb, l)
        tot += 0.5 * (wt * fn(qi, qn, 0.5 * (Ai + An), Ai, An, Ji, Jn)).sum()
    return tot


# ------------------------------------------------------------------ dense literal form (pin 9)
@pytest.mark.parametrize("p,E,mu,diss", [(1, 2, 0.0, 1), (2, 2, 0.02, 1), (2, 3, 0.02, 0), (1, 3, 0.05, 1)])
def test_dense_literal_form_matches(p, E, mu, diss):
    c = Case(W.make_problem(p=p, E=E, L=2.0, A=0.12, mu=mu, iface_diss=diss, seed=3, u_rms=0.3))
    q = c.jumpy(0.03, seed=p + E)
    r = c.residual(q)
    mesh = dense.DenseMesh(c.x, c.metric, c.jac, c.sbp, c.prob.L)
    rd = dense.residual(q, mesh, c.prm)
    assert rel_err(r, rd) < 1e-13


# ------------------------------------------------------------------ freestream (pin V)
@pytest.mark.parametrize("p,E,A", [(3, 3, 0.1), (4, 2, 0.15), (7, 2, 0.1)])
def test_freestream_preservation(p, E, A):
    c = Case(W.make_problem(p=p, E=E, L=2.0, A=A, init="constant", mu=0.01))
    r = c.residual()
    # size of the individual flux-differencing terms, for a roundoff-relative bound
    F = G.euler_flux(c.q, c.prm.gas)
    scale = np.abs(F).max() * np.abs(c.metric).max() * np.abs(c.sbp.D).max() / c.jac.min()
    assert np.abs(r).max() < 1e-13 * scale * p


# ------------------------------------------------------------------ conservation (pin IV)
@pytest.mark.parametrize("mu,diss", [(0.0, 1), (0.03, 1)])
def test_conservation(mu, diss):
    c = Case(W.make_problem(p=3, E=3, L=2.0, A=0.1, mu=mu, iface_diss=diss, seed=5, u_rms=0.3))
    q = c.jumpy(0.02, 1)
    r = c.residual(q)
    wj = c.weights3d() * c.jac
    tot = (wj * r).sum(axis=(1, 2, 3, 4))
    mag = (wj * np.abs(r)).sum(axis=(1, 2, 3, 4))
    assert np.all(np.abs(tot) < 1e-14 * mag.max())


# ------------------------------------------------------------------ entropy (pins I, II, III)
def test_entropy_conservation_inviscid():
    c = Case(W.make_problem(p=4, E=3, L=2.0, A=0.12, mu=0.0, iface_diss=0, seed=6, u_rms=0.3))
    q = c.jumpy(0.03, 2)
    r = c.residual(q)
    w = G.entropy_variables(q, c.prm.gas)
    wj = c.weights3d() * c.jac
    assert abs((wj * (w * r).sum(0)).sum()) < 1e-14 * (wj * np.abs(w * r).sum(0)).sum()


def test_entropy_stability_identity_inviscid():
    """sum wJ w.dq/dt = -sum_pairs w_t lam/2 (w_i - w_nu).(q_i - q_nu) <= 0, as an equality."""
    c = Case(W.make_problem(p=3, E=3, L=2.0, A=0.1, mu=0.0, iface_diss=1, seed=7, u_rms=0.3))
    q = c.jumpy(0.03, 3)
    gas = c.prm.gas
    r = c.residual(q)
    w = G.entropy_variables(q, gas)
    lhs = (c.weights3d() * c.jac * (w * r).sum(0)).sum()

    def diss(qi, qn, nbar, Ai, An, Ji, Jn):
        nn = np.sqrt((nbar ** 2).sum(0))
        sp_ = lambda qx: np.abs((G.primitives(qx, gas)[1] * nbar).sum(0)) + G.sound_speed(qx, gas) * nn  # noqa
        lam = np.maximum(sp_(qi), sp_(qn))
        dw = G.entropy_variables(qi, gas) - G.entropy_variables(qn, gas)
        return -lam / 2 * (dw * (qi - qn)).sum(0)

    rhs = face_sum(c, q, diss)
    assert rhs < 0
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_viscous_entropy_budget_identity():
    """sum wJ w.(dq/dt)_visc = -sum wJ g_m^T C_mj g_j - eta sum_pairs w_t dw^T L dw <= 0 (equality)."""
    c = Case(W.make_problem(p=3, E=3, L=2.0, A=0.1, mu=0.02, eta=1.0, iface_diss=0, seed=8, u_rms=0.3))
    q = c.jumpy(0.02, 4)
    gas = c.prm.gas
    rv = c.residual(q) - c.residual(q, prm=R.Params(mu=0.0, iface_diss=0))
    w = G.entropy_variables(q, gas)
    wj = c.weights3d() * c.jac
    lhs = (wj * (w * rv).sum(0)).sum()
    th = R.gradient_theta(q, c.metric, c.nbr, np.arange(c.prob.K), c.sbp, c.prm)
    g = np.stack([sum(c.metric[3 * a + j] * th[a] for a in range(3)) / c.jac for j in range(3)])
    vol = -(wj * (g * G.viscous_flux(q, g, gas)).sum(axis=(0, 1))).sum()

    def ip(qi, qn, nbar, Ai, An, Ji, Jn):
        Lm = 0.5 * (R.chat_ll(qi, Ai, Ji, gas) + R.chat_ll(qn, An, Jn, gas))
        dw = G.entropy_variables(qi, gas) - G.entropy_variables(qn, gas)
        return -c.prm.eta * np.einsum("a...,ab...,b...->...", dw, Lm, dw)

    pen = face_sum(c, q, ip)
    assert vol < 0 and pen < 0
    assert abs(lhs - (vol + pen)) < 1e-12 * abs(vol + pen)


# ------------------------------------------------------------------ split form (pin 7)
@pytest.mark.parametrize("A", [0.0, 0.1])
def test_central_flux_reduces_to_split_form(A):
    """With F# = (F_i + F_j)/2: volume term = 1/2 sum_l [D_l (A_l.F) + A_l.(D_l F)] when the discrete
    GCL holds (the split form of eq. convectionsplitdisctele), i.e. D_l (A_l.F) on affine meshes."""
    c = Case(W.make_problem(p=3, E=2, L=2.0, A=A, seed=9, u_rms=0.3, two_point=1))
    q = c.jumpy(0.02, 5)
    V = R.volume_term(q, c.metric, c.sbp, c.prm)
    F = G.euler_flux(q, c.prm.gas)
    ref = 0
    for l in range(3):
        Al = c.metric[3 * l:3 * l + 3]
        ref = ref + 0.5 * (apply_D(c.sbp.D, G.contract(F, Al), l)
                           + sum(Al[m] * apply_D(c.sbp.D, F[m], l) for m in range(3)))
    assert rel_err(V, ref) < 1e-12
    if A == 0.0:
        ref2 = sum(apply_D(c.sbp.D, G.contract(F, c.metric[3 * l:3 * l + 3]), l) for l in range(3))
        assert rel_err(V, ref2) < 1e-12


# ------------------------------------------------------------------ Kennedy-Gruber form (SF-KG)
def _quad(D, a, b, l):
    """sum_j 2 D_ij abar_ij bbar_ij along xi_l, written as the quadratic split derivative
    (a D b + b D a + D(ab)) / 2."""
    return 0.5 * (a * apply_D(D, b, l) + b * apply_D(D, a, l) + apply_D(D, a * b, l))


def _cubic(D, a, b, c, l):
    """sum_j 2 D_ij abar bbar cbar along xi_l, written as the cubic split derivative of Kennedy and
    Gruber: [D(abc) + a D(bc) + b D(ac) + c D(ab) + bc D a + ac D b + ab D c] / 4."""
    d = lambda f: apply_D(D, f, l)  # noqa: E731
    return 0.25 * (d(a * b * c) + a * d(b * c) + b * d(a * c) + c * d(a * b)
                   + b * c * d(a) + a * c * d(b) + a * b * d(c))


def test_kennedy_gruber_volume_is_the_split_derivative_form():
    """On an affine mesh, flux differencing with the product-of-averages flux equals the split
    derivative form of Kennedy and Gruber term by term (the SF-KG form of the comparison)."""
    c = Case(W.make_problem(p=3, E=2, L=2.0, A=0.0, seed=15, u_rms=0.3, two_point=2))
    q = c.jumpy(0.03, 11)
    V = R.volume_term(q, c.metric, c.sbp, c.prm)
    rho, u, P, _ = G.primitives(q, c.prm.gas)
    e = q[4] / rho
    D = c.sbp.D
    ref = np.zeros_like(q)
    for l in range(3):
        for m in range(3):
            F = [_quad(D, rho, u[m], l)]
            F += [_cubic(D, rho, u[m], u[k], l) + (apply_D(D, P, l) if k == m else 0.0) for k in range(3)]
            F += [_cubic(D, rho, u[m], e, l) + _quad(D, P, u[m], l)]
            ref += c.metric[3 * l + m] * np.stack(F)
    assert rel_err(V, ref) < 1e-12
    # the central flux is not this form (the test can tell them apart)
    Vc = R.volume_term(q, c.metric, c.sbp, R.Params(two_point=1))
    assert rel_err(Vc, ref) > 1e-4


@pytest.mark.parametrize("two_point,preserves", [(2, True), (0, True), (1, False)])
def test_kinetic_energy_conserved_at_uniform_pressure(two_point, preserves):
    """Kinetic-energy-preserving two-point fluxes (momentum flux = mass flux times the mean velocity
    plus a mean pressure) leave the total discrete kinetic energy unchanged on a periodic curvilinear
    mesh without interface dissipation when the pressure is uniform: the convective part cancels by
    skew-symmetry and the pressure part by the discrete GCL. Both SF-KG and ES-C are of this kind;
    the central flux is not."""
    c = Case(W.make_problem(p=4, E=2, L=2.0, A=0.12, mu=0.0, iface_diss=0, seed=16, u_rms=0.3,
                            two_point=two_point))
    q = c.jumpy(0.05, 12)
    gas = c.prm.gas
    rho, u = q[0], q[1:4] / q[0]
    q[4] = 1.0 / (gas.gamma - 1.0) + 0.5 * rho * (u * u).sum(0)
    r = c.residual(q)
    wj = c.weights3d() * c.jac
    ke = (u * r[1:4]).sum(0) - 0.5 * (u * u).sum(0) * r[0]
    mag = (wj * np.abs(u * r[1:4]).sum(0)).sum()
    rel = abs((wj * ke).sum()) / mag
    if preserves:
        assert rel < 1e-13
    else:
        assert rel > 1e-6


# ------------------------------------------------------------------ subsets, chunks, precision
def test_element_subset_matches_full():
    c = Case(W.make_problem(p=2, E=4, L=2.0, A=0.1, mu=0.02, seed=10, u_rms=0.3))
    q = c.jumpy(0.02, 6)
    full = c.residual(q)
    sel = np.array([0, 5, 17, 63, 42])
    assert np.array_equal(c.residual(q, elems=sel), full[:, sel])
    assert np.array_equal(c.residual(q, chunk=7), full)


def test_long_double_noise_floor():
    prob = W.make_problem(p=3, E=3, L=2.0, A=0.1, mu=0.02, seed=11, u_rms=0.3)
    c = Case(prob)
    LD = np.longdouble
    r = c.residual()
    rl = R.residual(c.q.astype(LD), c.metric.astype(LD), c.jac.astype(LD), c.nbr,
                    operators.SBP1D(prob.p, LD), c.prm)
    assert rel_err(r, rl.astype(np.float64)) < 2e-14


def test_complex_step_matches_central_difference():
    c = Case(W.make_problem(p=3, E=2, L=2.0, A=0.1, mu=0.02, seed=12, u_rms=0.3))
    q = c.jumpy(0.02, 7)
    v = W.direction(torch.as_tensor(q), 3).numpy()
    jv = jvp.jvp(q, v, c.metric, c.jac, c.nbr, c.sbp, c.prm)
    h = 1e-6
    fd = (c.residual(q + h * v) - c.residual(q - h * v)) / (2 * h)
    assert rel_err(fd, jv) < 1e-7


# ------------------------------------------------------------------ RK4
def test_rk4_linear_system_is_fourth_order_taylor():
    rng = np.random.Generator(np.random.PCG64(1))
    M = rng.normal(size=(6, 6))
    q = rng.normal(size=6)
    dt = 0.1
    out = R.rk4_step(lambda y: M @ y, q, dt)
    ref = sum(np.linalg.matrix_power(dt * M, k) @ q / math.factorial(k) for k in range(5))
    assert np.abs(out - ref).max() < 1e-14


# ------------------------------------------------------------------ paper's isentropic vortex
@pytest.mark.slow
def test_stationary_isentropic_vortex_converges():
    """The stationary isentropic vortex (beta = 5, Ma = 0.5, T_inf = 1) is an exact steady solution
    of the Euler equations: the discrete residual must vanish under h-refinement at high order."""
    errs = []
    for E in (6, 12):
        prob = W.make_problem(p=4, E=E, L=12.0, A=0.05, mu=0.0, init="vortex", Ma=0.5,
                              R=1.0 / (1.4 * 0.25), iface_diss=1)
        c = Case(prob)
        r = c.residual()
        errs.append(np.abs(r).max())
    rate = math.log2(errs[0] / errs[1])
    assert rate > 3.0, (errs, rate)


# ------------------------------------------------------------------ continuous equations (pin 8)
def _symbolic_ns_rhs(gamma, Rg, mu, Pr):
    x = sp.symbols("x1 x2 x3")
    pi = sp.pi
    rho = 1 + sp.Rational(1, 10) * sp.sin(pi * x[0]) * sp.cos(pi * x[1]) + sp.Rational(1, 20) * sp.cos(pi * x[2])
    u = [sp.Rational(1, 5) * sp.sin(pi * (x[1] + x[2])), sp.Rational(1, 10) * sp.cos(pi * (x[0] - x[2])),
         sp.Rational(3, 20) * sp.sin(pi * x[0]) * sp.sin(pi * x[1])]
    P = 1 + sp.Rational(1, 10) * sp.cos(pi * (x[0] + x[1])) * sp.sin(pi * x[2])
    T = P / (rho * Rg)
    Et = P / (gamma - 1) + rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2) / 2
    cp = gamma * Rg / (gamma - 1)
    kap = mu * cp / Pr
    div = sum(sp.diff(u[i], x[i]) for i in range(3))
    tau = [[mu * (sp.diff(u[i], x[j]) + sp.diff(u[j], x[i]) - sp.Rational(2, 3) * int(i == j) * div)
            for j in range(3)] for i in range(3)]
    rhs = []
    for c in range(5):
        tot = 0
        for m in range(3):
            Fi = [rho * u[m], rho * u[m] * u[0] + int(m == 0) * P, rho * u[m] * u[1] + int(m == 1) * P,
                  rho * u[m] * u[2] + int(m == 2) * P, (Et + P) * u[m]][c]
            Fv = [0, tau[0][m], tau[1][m], tau[2][m],
                  sum(tau[i][m] * u[i] for i in range(3)) + kap * sp.diff(T, x[m])][c]
            tot += -sp.diff(Fi, x[m]) + sp.diff(Fv, x[m])
        rhs.append(sp.lambdify(x, tot, "numpy"))
    prim = [sp.lambdify(x, e, "numpy") for e in (rho, u[0], u[1], u[2], P)]
    return rhs, prim


@pytest.mark.slow
@pytest.mark.parametrize("A,min_rate", [(0.0, 3.5), (0.08, 2.5)])
def test_navier_stokes_residual_converges_to_continuous_rhs(A, min_rate):
    """p = 5: pointwise residual error against -dF/dx + dF^V/dx of the continuous equations
    (eq. compressible_ns with eqs. ns_iflux, Fv, tau) falls at about order p - 1 (viscous part)."""
    gamma, Rg, mu, Pr = 1.4, 1.0, 0.05, 0.72
    rhs, prim = _symbolic_ns_rhs(gamma, Rg, mu, Pr)
    errs = []
    for E in (4, 8):
        prob = W.make_problem(p=5, E=E, L=2.0, A=A, mu=mu, Pr=Pr, gamma=gamma, R=Rg, iface_diss=1)
        c = Case(prob)
        X = [c.x[0], c.x[1], c.x[2]]
        rho, u1, u2, u3, P = [f(*X) * np.ones_like(X[0]) for f in prim]
        q = np.stack([rho, rho * u1, rho * u2, rho * u3, P / (gamma - 1) + 0.5 * rho * (u1 ** 2 + u2 ** 2 + u3 ** 2)])
        r = c.residual(q)
        ex = np.stack([f(*X) * np.ones_like(X[0]) for f in rhs])
        errs.append([np.abs(r[k] - ex[k]).max() for k in range(5)])
    rates = [math.log2(errs[0][k] / errs[1][k]) for k in range(5)]
    assert min(rates) > min_rate, (errs, rates)


# ------------------------------------------------------------------------------------------ DC form
def test_dc_volume_is_derivative_of_nodal_flux_on_affine_mesh():
    """Standard DC: on an affine mesh, D applied to the nodal flux equals the central-flux
    flux-differencing form (both are D_l(A_l . F) there)."""
    c = Case(W.make_problem(p=3, E=2, L=2.0, A=0.0, seed=13, u_rms=0.3, two_point=3))
    q = c.jumpy(0.02, 8)
    V_dc = R.volume_term(q, c.metric, c.sbp, c.prm)
    V_c = R.volume_term(q, c.metric, c.sbp, R.Params(two_point=1))
    assert rel_err(V_dc, V_c) < 1e-12


def test_dc_conservation_and_freestream():
    c = Case(W.make_problem(p=3, E=3, L=2.0, A=0.1, mu=0.02, seed=14, u_rms=0.3, two_point=3))
    r = c.residual(c.jumpy(0.02, 9))
    wj = c.weights3d() * c.jac
    tot = (wj * r).sum(axis=(1, 2, 3, 4))
    mag = (wj * np.abs(r)).sum(axis=(1, 2, 3, 4))
    assert np.all(np.abs(tot) < 1e-13 * mag.max())
    cf = Case(W.make_problem(p=3, E=3, L=2.0, A=0.1, init="constant", two_point=3))
    F = G.euler_flux(cf.q, cf.prm.gas)
    scale = np.abs(F).max() * np.abs(cf.metric).max() * np.abs(cf.sbp.D).max() / cf.jac.min()
    assert np.abs(cf.residual()).max() < 1e-13 * scale * 3


@pytest.mark.slow
def test_dc_converges_on_isentropic_vortex():
    errs = []
    for E in (6, 12):
        prob = W.make_problem(p=4, E=E, L=12.0, A=0.05, mu=0.0, init="vortex", Ma=0.5,
                              R=1.0 / (1.4 * 0.25), iface_diss=1, two_point=3)
        errs.append(np.abs(Case(prob).residual()).max())
    assert math.log2(errs[0] / errs[1]) > 2.5, errs
