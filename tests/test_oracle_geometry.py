"""Pins of the curl-form metric terms and the Jacobian (linear convection-diffusion section,
eqs. GCL and discGCLconvection)."""
import math

import numpy as np
import pytest

import workloads as W
from helpers import Case
from oracle import geometry


@pytest.mark.parametrize("p,E", [(1, 2), (3, 3), (5, 2)])
def test_affine_metrics_exact(p, E):
    prob = W.make_problem(p=p, E=E, L=2.0, A=0.0)
    c = Case(prob)
    h = prob.L / E
    for l in range(3):
        for m in range(3):
            ref = (h / 2) ** 2 if l == m else 0.0
            assert np.abs(c.metric[3 * l + m] - ref).max() < 1e-14 * p * p
    assert np.abs(c.jac - (h / 2) ** 3).max() < 1e-14 * p


@pytest.mark.parametrize("p,E,A", [(3, 4, 0.1), (7, 2, 0.15), (4, 3, 0.1)])
def test_discrete_gcl(p, E, A):
    c = Case(W.make_problem(p=p, E=E, L=2.0, A=A))
    scale = np.abs(c.metric).max()
    assert np.abs(geometry.gcl_residual(c.metric, c.sbp.D)).max() < 1e-13 * scale * p
    assert c.jac.min() > 0


def analytic_metrics(prob, x_ref):
    """J dxi_l/dx_m and J from the derivative of the warp map (cofactors of dx/dxi)."""
    E, N, L, A = prob.E, prob.N, prob.L, prob.A
    h = L / E
    ev = np.arange(E)
    g1d = h * (ev[:, None] + (x_ref[None, :] + 1) / 2)
    g = [np.broadcast_to(g1d[None, None, :, None, None, :], (E, E, E, N, N, N)),
         np.broadcast_to(g1d[None, :, None, None, :, None], (E, E, E, N, N, N)),
         np.broadcast_to(g1d[:, None, None, :, None, None], (E, E, E, N, N, N))]
    w = 2 * math.pi / L
    s = [np.sin(w * gg) for gg in g]
    c = [np.cos(w * gg) for gg in g]
    amp = A * L / 2
    dbump = [amp * w * c[0] * s[1] * s[2], amp * w * s[0] * c[1] * s[2], amp * w * s[0] * s[1] * c[2]]
    # dx_m/dxi_i = (delta_mi + dbump_i) h/2
    F = [[(float(mm == i) + dbump[i]) * h / 2 for i in range(3)] for mm in range(3)]
    J = (F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0])
         + F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]))
    # J dxi_l/dx_m = cofactor(F)[m][l]
    cof = lambda a, b: (F[(a + 1) % 3][(b + 1) % 3] * F[(a + 2) % 3][(b + 2) % 3]  # noqa: E731
                        - F[(a + 1) % 3][(b + 2) % 3] * F[(a + 2) % 3][(b + 1) % 3])
    met = np.stack([cof(m, l) for l in range(3) for m in range(3)]).reshape(9, E ** 3, N, N, N)
    return met, J.reshape(E ** 3, N, N, N)


def test_metrics_converge_to_analytic():
    errs = []
    for p in (2, 4, 8, 12):
        prob = W.make_problem(p=p, E=2, L=2.0, A=0.1)
        c = Case(prob)
        met, J = analytic_metrics(prob, c.sbp.x)
        errs.append((np.abs(c.metric - met).max(), np.abs(c.jac - J).max()))
    assert errs[-1][0] < 1e-7 and errs[-1][1] < 1e-10
    assert errs[-1][0] < 1e-2 * errs[0][0]


@pytest.mark.parametrize("A", [0.1, 0.15])
def test_positive_jacobian_at_workload_amplitudes(A):
    c = Case(W.make_problem(p=7, E=2, L=2.0, A=A))
    assert c.jac.min() > 0
