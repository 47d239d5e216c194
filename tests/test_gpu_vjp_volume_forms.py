"""Hand-written VJP with the central flux-differencing form (two_point = 1) and the standard DC form
(two_point = 3: SBP derivative of the nodal fluxes, central interface flux with the own-flux part
of the SAT kept), against the oracle: the extended-precision complex-step Jacobian on small meshes
(periodic, walls, Dirichlet data, rotated elements, viscous and inviscid), the dot-product identity
with the oracle's complex-step J v for p up to 8, and central differences of the GPU residual."""
import numpy as np
import pytest
import torch

import paper_1911_10966_amd as P
import workloads as W
from gpu_helpers import from_dev, require_gpu, to_dev
from helpers import rel_err
from oracle import jvp, operators
from test_gpu_vjp_boundaries import BCase

pytestmark = pytest.mark.gpu
TOL = 1e-12

FULL = [
    # p, E, mu, box, rotate, two_point, iface_diss
    (1, 2, 0.0, (None, None, None), False, 3, 1),
    (1, 2, 0.03, (-3, None, None), False, 3, 1),
    (2, 2, 0.02, (None, None, None), True, 3, 0),
    (1, 2, 0.0, (-2, None, -1), False, 1, 1),
    (2, 2, 0.02, (None, -3, None), True, 1, 1),
]


@pytest.mark.parametrize("p,E,mu,box,rotate,tp,diss", FULL)
def test_volume_form_vjp_matches_full_jacobian(p, E, mu, box, rotate, tp, diss):
    require_gpu()
    print(f"vjp full jacobian p={p} E={E} mu={mu} box={box} rotate={rotate} tp={tp} diss={diss}", flush=True)
    c = BCase(p, E, mu, box, rotate, seed=60 + 10 * p + tp, diss=diss, tp=tp)
    LD = np.longdouble
    kw = c.kw()
    if kw["bc"] is not None:
        kw["bc"] = kw["bc"].astype(LD)
    Jm = jvp.full_jacobian(c.q, c.metric.astype(LD), c.jac.astype(LD), c.nbr, operators.SBP1D(p, LD),
                           c.prm, ctype=np.clongdouble, **kw)
    gb = np.random.Generator(np.random.PCG64(6)).standard_normal(c.q.shape)
    ref = (Jm.T @ gb.ravel().astype(LD)).reshape(c.q.shape).astype(np.float64)
    err = rel_err(c.vjp(c.q, gb), ref)
    print(f"  gpu vs extended-precision J^T gbar: {err:.2e}")
    assert err < TOL


DOT = [
    # p, E, mu, box, rotate, two_point
    (3, 2, 0.02, (None, None, None), False, 3),
    (4, 2, 0.01, (-3, None, -1), False, 3),
    (5, 2, 0.0, (None, None, None), True, 3),
    (8, 2, 0.01, (None, -3, None), False, 3),
    (4, 2, 0.02, (None, None, None), False, 1),
    (7, 2, 0.0, (-2, None, None), True, 1),
]


@pytest.mark.parametrize("p,E,mu,box,rotate,tp", DOT)
def test_volume_form_vjp_dot_product(p, E, mu, box, rotate, tp):
    require_gpu()
    print(f"vjp dot p={p} E={E} mu={mu} box={box} rotate={rotate} tp={tp}", flush=True)
    c = BCase(p, E, mu, box, rotate, seed=70 + p, tp=tp)
    rng = np.random.Generator(np.random.PCG64(p))
    gb = rng.standard_normal(c.q.shape)
    v = W.direction(torch.as_tensor(c.q), 5).numpy()
    jv = jvp.jvp(c.q, v, c.metric, c.jac, c.nbr, c.sbp, c.prm, **c.kw())
    qb = c.vjp(c.q, gb)
    lhs, rhs = (gb * jv).sum(), (qb * v).sum()
    scale = np.abs(gb * jv).sum()
    print(f"  dot: rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) < TOL * scale


def test_dc_vjp_central_difference():
    require_gpu()
    c = BCase(4, 3, 0.02, (None, -1, None), False, seed=81, tp=3)
    gb = np.random.Generator(np.random.PCG64(81)).standard_normal(c.q.shape)
    v = W.direction(torch.as_tensor(c.q), 7).numpy()
    ps = P.ProblemSet([c.device()])
    h = 1e-6
    rp = from_dev(ps.residual(to_dev(c.q + h * v)), c.q.shape)
    rm = from_dev(ps.residual(to_dev(c.q - h * v)), c.q.shape)
    fd = (gb * (rp - rm)).sum() / (2 * h)
    qb = c.vjp(c.q, gb)
    assert abs(fd - (qb * v).sum()) < 1e-6 * np.abs(gb * (rp - rm) / (2 * h)).sum()
