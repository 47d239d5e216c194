"""Pins of the entropy-stable matrix interface dissipation (iface_diss = 2).

* At equal states the operator times dw/dq is |nbar| |A_n|: the absolute value of the Euler flux
  Jacobian in the face normal, computed here independently (complex-step Jacobian of the nodal flux,
  numpy eigendecomposition).  Nearby states approach it linearly.
* The operator is symmetric positive semi-definite, so w-weighted it only removes entropy; the
  residual's entropy budget is minus the sum of those quadratic forms over face pairs, as an equality.
"""
import numpy as np

import workloads as W
from helpers import Case
from oracle import gas as G
from test_oracle_residual import face_sum

GAS = G.Gas(1.4, 1.0, 0.0, 0.72)


def _state(rng, n):
    rho = rng.uniform(0.6, 1.4, n)
    u = rng.uniform(-0.6, 0.6, (3, n))
    p = rng.uniform(0.5, 1.5, n)
    return np.stack([rho, rho * u[0], rho * u[1], rho * u[2], p / 0.4 + 0.5 * rho * (u * u).sum(0)])


def _abs_jacobian(q, nbar):
    """|d(F(q).nbar)/dq| by complex step and eigendecomposition, shape (5, 5, n)."""
    n = q.shape[1]
    out = np.zeros((5, 5, n))
    for j in range(n):
        A = np.zeros((5, 5))
        for b in range(5):
            qc = q[:, j:j + 1].astype(np.complex128)
            qc[b] += 1e-30j
            A[:, b] = np.imag(G.contract(G.euler_flux(qc, GAS), nbar[:, j:j + 1].astype(np.complex128))[:, 0]) / 1e-30
        lam, V = np.linalg.eig(A)
        out[:, :, j] = np.real(V @ np.diag(np.abs(lam)) @ np.linalg.inv(V))
    return out


def _dw_dq(q):
    n = q.shape[1]
    out = np.zeros((5, 5, n))
    for b in range(5):
        qc = q.astype(np.complex128)
        qc[b] += 1e-30j
        out[:, b] = np.imag(G.entropy_variables(qc, GAS)) / 1e-30
    return out


def test_equal_states_give_the_roe_matrix():
    rng = np.random.Generator(np.random.PCG64(11))
    q = _state(rng, 6)
    nbar = rng.normal(size=(3, 6))
    M = G.matrix_dissipation_operator(q, q, nbar, GAS)
    got = np.einsum("ab...,bc...->ac...", M, _dw_dq(q))
    ref = _abs_jacobian(q, nbar)
    for j in range(6):
        assert np.abs(got[:, :, j] - ref[:, :, j]).max() < 1e-12 * np.abs(ref[:, :, j]).max()


def test_nearby_states_approach_the_roe_dissipation():
    rng = np.random.Generator(np.random.PCG64(12))
    q = _state(rng, 4)
    nbar = rng.normal(size=(3, 4))
    d = rng.normal(size=q.shape) * q
    errs = []
    for eps in (1e-3, 1e-4):
        qn = q + eps * d
        got = G.matrix_dissipation(q, qn, nbar, GAS)
        ref = np.einsum("ab...,b...->a...", _abs_jacobian(0.5 * (q + qn), nbar), q - qn)
        errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    assert errs[1] < 2e-4 and errs[1] < errs[0] / 5.0


def test_operator_is_symmetric_psd():
    rng = np.random.Generator(np.random.PCG64(13))
    qi, qn = _state(rng, 8), _state(rng, 8)
    M = G.matrix_dissipation_operator(qi, qn, rng.normal(size=(3, 8)), GAS)
    for j in range(8):
        m = M[:, :, j]
        assert np.abs(m - m.T).max() < 1e-13 * np.abs(m).max()
        assert np.linalg.eigvalsh(0.5 * (m + m.T)).min() > -1e-12 * np.abs(m).max()


def test_entropy_budget_with_matrix_dissipation():
    """sum wJ w.dq/dt = -sum_pairs w_t (1/2) dw^T M dw <= 0, as an equality."""
    c = Case(W.make_problem(p=3, E=3, L=2.0, A=0.1, mu=0.0, iface_diss=2, seed=7, u_rms=0.3))
    q = c.jumpy(0.03, 3)
    gas = c.prm.gas
    r = c.residual(q)
    w = G.entropy_variables(q, gas)
    lhs = (c.weights3d() * c.jac * (w * r).sum(0)).sum()

    def diss(qi, qn, nbar, Ai, An, Ji, Jn):
        dw = G.entropy_variables(qi, gas) - G.entropy_variables(qn, gas)
        return -0.5 * (dw * G.matrix_dissipation(qi, qn, nbar, gas)).sum(0)

    rhs = face_sum(c, q, diss)
    assert rhs < 0
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_dissipation_is_odd_in_the_states_and_even_in_the_normal():
    """M(q_i, q_nu, n) = -M(q_nu, q_i, n) = M(q_i, q_nu, -n): the two sides of a face carry
    opposite terms, whatever the sign of the normal each side sees."""
    rng = np.random.default_rng(12)
    qi, qn = _state(rng, 40), _state(rng, 40)
    nbar = rng.normal(size=(3, 40))
    M = G.matrix_dissipation(qi, qn, nbar, GAS)
    assert np.abs(M + G.matrix_dissipation(qn, qi, nbar, GAS)).max() < 1e-13 * np.abs(M).max()
    assert np.abs(M - G.matrix_dissipation(qi, qn, -nbar, GAS)).max() < 1e-13 * np.abs(M).max()


def test_complex_step_of_the_dissipation_matches_central_differences():
    """The complex step through the dissipation (|.| continued by the sign of the real part, log
    means, square roots) gives the same directional derivative as central differences."""
    rng = np.random.default_rng(13)
    qi, qn = _state(rng, 30), _state(rng, 30)
    nbar = rng.normal(size=(3, 30))
    for side in (0, 1):
        v = rng.normal(size=qi.shape) * np.array([0.1, 0.1, 0.1, 0.1, 0.5])[:, None]
        h = 1e-30
        args = [qi.astype(np.complex128), qn.astype(np.complex128)]
        args[side] = args[side] + 1j * h * v
        cs = np.imag(G.matrix_dissipation(*args, nbar, GAS)) / h
        e = 1e-6
        ap, am = [qi, qn], [qi, qn]
        ap[side] = ap[side] + e * v
        am[side] = am[side] - e * v
        fd = (G.matrix_dissipation(*ap, nbar, GAS) - G.matrix_dissipation(*am, nbar, GAS)) / (2 * e)
        assert np.abs(cs - fd).max() < 1e-7 * np.abs(cs).max()
