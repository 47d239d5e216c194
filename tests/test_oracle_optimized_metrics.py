"""Pins of the optimised metric terms (oracle.geometry.optimized_metrics, reading of the paragraph after
eq. discGCLconvection: analytic surface metrics, volume metrics closest to the analytic ones under the
discrete GCL).

* The closed-form mapping derivative (workloads.mapping_jacobian) against the collocation derivative
  of the node coordinates at high degree (spectral agreement), and the analytic metrics against the
  adjugate identity A (dx/dxi) = J I.
* The result satisfies the discrete GCL to rounding, shares its face-normal values between the two
  elements of every face, closes the LGL surface integral of every element, and equals the
  analytic metrics on affine elements.
* Both corrections are minimum-norm: the volume change lies in the row space of the GCL operator on
  the moved entries, the surface change in the row space of the compatibility conditions (KKT
  conditions of the two least-norm problems, checked with their own least-squares solves).
* The optimised metrics converge to the analytic ones under h-refinement at about order p.
* With them the residual preserves a uniform flow and conserves entropy (entropy-conservative
  interfaces, inviscid, periodic warped mesh)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import geometry as Gm, operators, residual as R
from oracle import gas as G


def _mesh(p, E, A=0.1, L=2.0):
    prob = W.make_problem(p=p, E=E, L=L, A=A)
    sbp = operators.SBP1D(p)
    return prob, sbp, W.mapping_jacobian(prob, sbp.x)


def test_mapping_jacobian_matches_the_collocation_derivative_of_the_coordinates():
    prob, sbp, F = _mesh(12, 2, A=0.1)
    x = W.coords(prob, sbp.x).numpy()
    Fd = geometry_jacobian = Gm.jacobian_matrix(x, sbp.D)
    err = max(np.abs(F[m, i] - Fd[m][i]).max() for m in range(3) for i in range(3))
    assert err < 1e-9 * np.abs(F).max()


def test_analytic_metrics_are_the_adjugate():
    prob, sbp, F = _mesh(3, 3, A=0.12)
    A, J = Gm.analytic_metrics(F)
    assert (J > 0).all()
    for l in range(3):
        for i in range(3):
            s = sum(A[3 * l + m] * F[m, i] for m in range(3))
            assert np.abs(s - (J if l == i else 0.0)).max() < 1e-14 * np.abs(J).max()


@pytest.mark.parametrize("p,E,A", [(2, 4, 0.12), (3, 3, 0.1), (4, 3, 0.15), (5, 2, 0.1), (7, 2, 0.1)])
def test_gcl_faces_closure(p, E, A):
    prob, sbp, F = _mesh(p, E, A)
    m, J = Gm.optimized_metrics(F, W.neighbours(E), sbp)
    scale = np.abs(m).max()
    assert np.abs(Gm.gcl_residual(m, sbp.D)).max() < 1e-13 * scale
    assert np.abs(Gm.surface_closure(m, sbp.w)).max() < 1e-14 * scale
    nbr = W.neighbours(E)
    N = sbp.N
    for l in range(3):
        own = m[3 * l:3 * l + 3][Gm._face_slice(l, 1, N)]                # + faces, (3, K, b, a)
        par = m[3 * l:3 * l + 3][:, nbr[:, 2 * l + 1]][Gm._face_slice(l, 0, N)]
        assert np.array_equal(own, par)
    assert (J > 0).all()


def test_affine_elements_keep_the_analytic_metrics():
    prob, sbp, F = _mesh(4, 3, A=0.0)
    m, J = Gm.optimized_metrics(F, W.neighbours(3), sbp)
    a, Ja = Gm.analytic_metrics(F)
    assert np.abs(m - a).max() < 1e-15 * np.abs(a).max()
    assert np.array_equal(J, Ja)


def test_both_corrections_are_minimum_norm():
    prob, sbp, F = _mesh(3, 4, A=0.12)
    nbr = W.neighbours(4)
    a0, _ = Gm.analytic_metrics(F)
    surf, xs = Gm.surface_metrics(a0, sbp, nbr)
    m, _ = Gm.optimized_metrics(F, nbr, sbp)
    M, held, pinv, Y = Gm.gcl_operator(sbp.D)
    K, n = prob.K, sbp.N ** 3
    flat = lambda arr, mm: np.concatenate([arr[3 * l + mm].reshape(K, n) for l in range(3)], axis=1)  # noqa
    Mf = M[:, ~held]
    for mm in range(3):
        # volume step: held entries untouched, the change of the others in the row space of M_free
        assert np.array_equal(flat(m, mm)[:, held], flat(surf, mm)[:, held])
        d = (flat(m, mm) - flat(surf, mm))[:, ~held]
        lam, *_ = np.linalg.lstsq(Mf.T, d.T, rcond=None)
        assert np.abs(Mf.T @ lam - d.T).max() < 1e-12 * max(np.abs(d).max(), 1e-300)
    # surface step: its correction is in the row space of the mesh's compatibility system G, and
    # the corrected values meet every condition
    G, cols, _ = Gm.surface_system(sbp, nbr)
    Gd = G.toarray()
    for mm in range(3):
        x = xs[mm]
        assert np.abs(x).max() > 0
        y, *_ = np.linalg.lstsq(Gd.T, x, rcond=None)
        assert np.abs(Gd.T @ y - x).max() < 1e-12 * np.abs(x).max()
        vals = np.zeros(G.shape[1])
        vals[cols.ravel()] = flat(surf, mm)[:, held].ravel()
        assert np.abs(Gd @ vals).max() < 1e-14 * np.abs(vals).max()


@pytest.mark.parametrize("p,Es", [(3, (3, 6)), (4, (4, 8))])
def test_converges_to_the_analytic_metrics(p, Es):
    """The distance to the analytic metrics (relative to their size, which scales as h^2) falls at
    about order p under h-refinement."""
    errs = []
    for E in Es:
        prob, sbp, F = _mesh(p, E, A=0.1)
        m, _ = Gm.optimized_metrics(F, W.neighbours(E), sbp)
        a, _ = Gm.analytic_metrics(F)
        errs.append(np.abs(m - a).max() / np.abs(a).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > p - 0.5, (errs, rate)


def _residual_case(p=3, E=3, A=0.12, mu=0.0, diss=0):
    prob, sbp, F = _mesh(p, E, A)
    nbr = W.neighbours(E)
    metric, J = Gm.optimized_metrics(F, nbr, sbp)
    x = W.coords(prob, sbp.x).numpy()
    return prob, sbp, metric, J, nbr, x


def test_freestream_preserved():
    prob, sbp, metric, J, nbr, x = _residual_case(mu=0.01)
    q = np.zeros((5,) + J.shape)
    q[0], q[1], q[2], q[3], q[4] = 1.2, 0.3, -0.2, 0.1, 3.0
    prm = R.Params(1.4, 1.0, 0.01, 0.72, 1.0, 1, 0)
    r = R.residual(q, metric, J, nbr, sbp, prm)
    assert np.abs(r).max() < 1e-13


def test_entropy_conservation_and_conservation():
    prob, sbp, metric, J, nbr, x = _residual_case()
    q = W.state(W.make_problem(p=prob.p, E=prob.E, L=2.0, A=0.12, seed=3, u_rms=0.3), torch.as_tensor(x)).numpy()
    rng = np.random.Generator(np.random.PCG64(1))
    q = q * (1.0 + 0.02 * rng.uniform(-1, 1, q.shape))
    prm = R.Params(1.4, 1.0, 0.0, 0.72, 1.0, 0, 0)
    r = R.residual(q, metric, J, nbr, sbp, prm)
    w3 = np.einsum("i,j,k->ijk", sbp.w, sbp.w, sbp.w)
    wJ = w3[None] * J
    wv = G.entropy_variables(q, prm.gas)
    rate = (wJ * (wv * r).sum(0)).sum()
    scale = (wJ * np.abs(wv * r).sum(0)).sum()
    assert abs(rate) < 1e-13 * scale
    tot = (wJ[None] * r).reshape(5, -1).sum(1)
    mag = (wJ[None] * np.abs(r)).reshape(5, -1).sum(1)
    assert np.all(np.abs(tot) < 1e-13 * mag)


def test_one_element_periodic_mesh_needs_no_surface_correction():
    """With one element, periodic, each pair of opposite faces is one face: x_+ - x_- vanishes in
    every compatibility condition, so no condition constrains the surface values.  The correction
    must then be exactly zero (the face values stay the means of the analytic ones), and the result
    still satisfies the discrete GCL."""
    prob, sbp, F = _mesh(4, 1, A=0.1)
    nbr = W.neighbours(1)
    a0, _ = Gm.analytic_metrics(F)
    surf, xs = Gm.surface_metrics(a0, sbp, nbr)
    assert np.array_equal(xs, np.zeros_like(xs))
    m, _ = Gm.optimized_metrics(F, nbr, sbp)
    assert np.abs(Gm.gcl_residual(m, sbp.D)).max() < 1e-13 * np.abs(m).max()
