"""Oracle pins for unstructured face orientation.

Turning every element's local axes by its own rotation of the cube relabels the nodes and changes
which faces meet and how their node grids lie on each other, but not the discretization: the
residual on the relabelled mesh (metrics recomputed from the relabelled coordinates, face table
found from the coordinates) must be the relabelled residual of the aligned mesh, for every flux,
dissipation and the viscous terms, with walls too.
"""
import numpy as np
import pytest
import torch

import workloads as W
from workloads import unstructured as U
from helpers import rel_err
from oracle import geometry, operators, residual as R


def test_connectivity_of_an_aligned_grid_is_the_structured_table():
    for E in (2, 3):   # (a single element across the period would match itself in several ways)
        prob = W.make_problem(p=2, E=E, L=2.0, A=0.1)
        sbp = operators.SBP1D(prob.p)
        x = W.coords(prob, sbp.x).numpy()
        nbr, orient = U.connectivity(x, prob.L)
        assert np.array_equal(nbr, W.neighbours(E))
        assert np.array_equal(orient, np.tile(np.array([1, 0, 3, 2, 5, 4]), (E ** 3, 1)))


def test_rotations_are_the_24_proper_ones():
    Rs = U.cube_rotations()
    assert len(Rs) == 24
    assert len({M.tobytes() for M in Rs}) == 24
    for M in Rs:
        assert round(np.linalg.det(M)) == 1


def _rotated(prob, seed, amp=0.03, box=None):
    sbp = operators.SBP1D(prob.p)
    x = W.coords(prob, sbp.x).numpy()
    q = W.state(prob, torch.as_tensor(x)).numpy()
    rng = np.random.Generator(np.random.PCG64(seed))
    q[0] *= 1.0 + amp * rng.uniform(-1, 1, q[0].shape)
    q[1:4] += amp * rng.uniform(-1, 1, q[1:4].shape)
    q[4] *= 1.0 + amp * rng.uniform(-1, 1, q[4].shape)
    rots = rng.integers(0, 24, prob.K)
    xr = U.rotate_elements(x, rots)
    qr = U.rotate_elements(q, rots)
    return sbp, x, q, xr, qr, rots


@pytest.mark.parametrize("p,E,mu,diss,tp", [(2, 3, 0.0, 1, 0), (3, 2, 0.02, 1, 0), (2, 2, 0.02, 2, 0),
                                            (3, 2, 0.0, 0, 2), (2, 2, 0.0, 1, 3), (4, 2, 0.01, 0, 0)])
def test_residual_is_invariant_under_element_rotations(p, E, mu, diss, tp):
    prob = W.make_problem(p=p, E=E, L=2.0, A=0.1, mu=mu, iface_diss=diss, two_point=tp, seed=4,
                          u_rms=0.3)
    sbp, x, q, xr, qr, rots = _rotated(prob, seed=p * 10 + E)
    prm = R.Params.of(prob)
    r0 = R.residual(q, geometry.curl_metrics(x, sbp.D), geometry.jacobian(x, sbp.D), W.neighbours(E),
                    sbp, prm)
    nbr, orient = U.connectivity(xr, prob.L)
    assert len(set((orient // 8).ravel().tolist())) > 1   # several orientations occur
    r1 = R.residual(qr, geometry.curl_metrics(xr, sbp.D), geometry.jacobian(xr, sbp.D), nbr, sbp, prm,
                    orient=orient)
    assert rel_err(r1, U.rotate_elements(r0, rots)) < 1e-12


def test_rotated_mesh_with_walls():
    E = 2
    prob = W.make_problem(p=3, E=E, L=2.0, A=0.1, mu=0.02, iface_diss=1, seed=6, u_rms=0.3,
                          box=(None, -3, None))
    sbp, x, q, xr, qr, rots = _rotated(prob, seed=8)
    prm = R.Params.of(prob)
    r0 = R.residual(q, geometry.curl_metrics(x, sbp.D), geometry.jacobian(x, sbp.D),
                    W.problem_neighbours(prob), sbp, prm)
    # no period in x_2: the box faces there stay unmatched and become walls
    nbr, orient = U.connectivity(xr, prob.L, boundary=-3, periods=(prob.L, None, prob.L))
    r1 = R.residual(qr, geometry.curl_metrics(xr, sbp.D), geometry.jacobian(xr, sbp.D), nbr, sbp, prm,
                    orient=orient)
    assert rel_err(r1, U.rotate_elements(r0, rots)) < 1e-12


def test_orientation_table_is_used():
    """A wrong orientation code changes the residual (the table is not ignored)."""
    prob = W.make_problem(p=2, E=2, L=2.0, A=0.1, mu=0.01, seed=4, u_rms=0.3)
    sbp, x, q, xr, qr, rots = _rotated(prob, seed=3)
    nbr, orient = U.connectivity(xr, prob.L)
    m, j = geometry.curl_metrics(xr, sbp.D), geometry.jacobian(xr, sbp.D)
    prm = R.Params.of(prob)
    r1 = R.residual(qr, m, j, nbr, sbp, prm, orient=orient)
    bad = orient.copy()
    bad[0, 0] ^= 8 * 6
    r2 = R.residual(qr, m, j, nbr, sbp, prm, orient=bad)
    assert rel_err(r2, r1) > 1e-6
