"""Oracle pins for Dirichlet boundary faces and the manufactured-solution forcing.

* The forcing of the manufactured solution (symbolic, ``workloads.mms``) agrees with central finite
  differences of the oracle's own nodal inviscid and viscous fluxes at scattered points.
* The residual of the exact manufactured state plus the forcing (its truncation error) converges
  under h-refinement at about the degree p, on Cartesian and warped meshes with every box face a
  Dirichlet boundary.
* A constant state with matching boundary data stays constant (free-stream preservation with
  boundaries, warped mesh, viscous).
* On an affine mesh, turning the x1 faces of a periodic box into boundaries whose data is the
  periodic neighbour's state gives the periodic inviscid residual: the ghost partner reproduces an
  interface exactly.
"""
import numpy as np
import pytest
import torch

import workloads as W
from workloads import mms
from oracle import gas as G
from oracle import geometry, operators, residual as R


def _mesh(prob):
    sbp = operators.SBP1D(prob.p)
    x = W.coords(prob, sbp.x).numpy()
    return sbp, x, geometry.curl_metrics(x, sbp.D), geometry.jacobian(x, sbp.D)


def test_mms_forcing_matches_finite_differences_of_the_fluxes():
    rng = np.random.Generator(np.random.PCG64(3))
    pts = rng.uniform(0.1, 0.9, size=(3, 6))
    gas = G.Gas(mms.GAMMA, mms.R_GAS, mms.MU, mms.PR)
    h = 1e-4

    def at(x):
        return mms.conservative(x)

    div_inv = np.zeros((5, pts.shape[1]))
    div_visc = np.zeros((5, pts.shape[1]))
    for m in range(3):
        e = np.zeros((3, 1))
        e[m] = h
        div_inv += (G.euler_flux(at(pts + e), gas)[m] - G.euler_flux(at(pts - e), gas)[m]) / (2 * h)

        def fv(x):
            # viscous flux from the oracle's C_mj blocks and finite-difference entropy-variable gradients
            grad = np.stack([(G.entropy_variables(at(x + np.eye(3)[j][:, None] * h), gas)
                              - G.entropy_variables(at(x - np.eye(3)[j][:, None] * h), gas)) / (2 * h)
                             for j in range(3)])
            return G.viscous_flux(at(x), grad, gas)[m]

        div_visc += (fv(pts + e) - fv(pts - e)) / (2 * h)
    S = mms.source(pts)
    S_inv = mms.source(pts, mu=0.0)
    for c in range(5):
        scale = np.abs(S_inv[c]).max()
        assert np.abs(S_inv[c] - div_inv[c]).max() < 1e-6 * scale
    # the viscous part is small (Re = 4e6); nested differences leave ~1e-3 relative error
    for c in range(1, 5):
        vs = S_inv[c] - S[c]
        assert np.abs(vs - div_visc[c]).max() < 2e-3 * np.abs(vs).max() + 1e-9 * np.abs(S_inv[c]).max()


@pytest.mark.parametrize("A", [0.0, 0.05])
@pytest.mark.parametrize("p,min_rate", [(2, 1.7), (3, 2.3)])
def test_mms_truncation_error_converges(A, p, min_rate):
    errs = []
    for E in (2, 4, 8):
        prob = W.mms_problem(p, E, A=A)
        sbp, x, metric, jac = _mesh(prob)
        q, S = mms.conservative(x), mms.source(x)
        r = R.residual(q, metric, jac, W.neighbours(E, periodic=False), sbp, R.Params.of(prob),
                       bc=q, source=S, chunk=256)
        errs.append(max(np.abs(r[c]).max() / np.abs(S[c]).max() for c in range(5)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.04
    assert rates[-1] > min_rate, rates


def test_constant_state_with_boundaries_is_steady():
    prob = W.make_problem(p=3, E=3, L=1.0, A=0.05, mu=0.01, init="constant", periodic=False)
    sbp, x, metric, jac = _mesh(prob)
    q = W.state(prob, torch.as_tensor(x)).numpy()
    r = R.residual(q, metric, jac, W.neighbours(3, periodic=False), sbp, R.Params.of(prob), bc=q)
    assert np.abs(r).max() < 1e-11


def test_boundary_ghost_reproduces_periodic_interface():
    prob = W.make_problem(p=2, E=3, L=2.0, A=0.0, mu=0.0, seed=9, u_rms=0.3)
    sbp, x, metric, jac = _mesh(prob)
    q = W.state(prob, torch.as_tensor(x)).numpy()
    nbr = W.neighbours(3)
    ref = R.residual(q, metric, jac, nbr, sbp, R.Params.of(prob))
    # xi_1 faces of the box become boundaries carrying the periodic neighbour's face state
    nb2 = nbr.copy()
    bc = np.zeros_like(q)
    E, N = 3, prob.N
    for e in range(E ** 3):
        e1 = e % E
        for side, f, own, mirror in ((0, 0, 0, N - 1), (1, 1, N - 1, 0)):
            if (side == 0 and e1 == 0) or (side == 1 and e1 == E - 1):
                bc[:, e, :, :, own] = q[:, nbr[e, f], :, :, mirror]
                nb2[e, f] = -1
    out = R.residual(q, metric, jac, nb2, sbp, R.Params.of(prob), bc=bc)
    scale = np.abs(ref).max()
    assert np.abs(out - ref).max() < 1e-13 * scale


def test_source_is_added_to_dqdt():
    prob = W.make_problem(p=2, E=2, L=2.0, A=0.1, mu=0.01, seed=4, u_rms=0.3)
    sbp, x, metric, jac = _mesh(prob)
    q = W.state(prob, torch.as_tensor(x)).numpy()
    nbr = W.neighbours(2)
    S = np.random.Generator(np.random.PCG64(1)).standard_normal(q.shape)
    a = R.residual(q, metric, jac, nbr, sbp, R.Params.of(prob))
    b = R.residual(q, metric, jac, nbr, sbp, R.Params.of(prob), source=S)
    assert np.array_equal(b, a + S)


def test_missing_boundary_data_is_an_error():
    prob = W.make_problem(p=1, E=2, L=1.0, A=0.0, mu=0.0, init="constant", periodic=False)
    sbp, x, metric, jac = _mesh(prob)
    q = W.state(prob, torch.as_tensor(x)).numpy()
    with pytest.raises(ValueError):
        R.residual(q, metric, jac, W.neighbours(2, periodic=False), sbp, R.Params.of(prob))
