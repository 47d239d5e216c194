"""GPU residual with the optimised metric terms (analytic surface metrics, volume metrics closest to
the analytic ones under the discrete GCL; built by the oracle from the closed-form mapping
derivative) against the oracle, on every kernel path; and, on the GPU output alone, uniform flow
preserved and entropy conserved with entropy-conservative interfaces."""
import time

import numpy as np
import pytest
import torch

import paper_1911_10966_amd as P
import workloads as W
from gpu_helpers import DEV, device_problem, from_dev, require_gpu, to_dev
from helpers import Case, rel_err
from oracle import gas as G
from oracle import geometry as Gm, operators, residual as R

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _case(p, E, A, mu, diss, tp=0):
    c = Case(W.make_problem(p=p, E=E, L=2.0, A=A, mu=mu, iface_diss=diss, two_point=tp, seed=60 + p,
                            u_rms=0.3))
    F = W.mapping_jacobian(c.prob, c.sbp.x)
    c.metric, c.jac = Gm.optimized_metrics(F, c.nbr, c.sbp)
    return c


def _bar(c, q, ref):
    LD = np.longdouble
    ref_ld = R.residual(q.astype(LD), c.metric.astype(LD), c.jac.astype(LD), c.nbr,
                        operators.SBP1D(c.prob.p, LD), c.prm)
    return max(TOL, 4.0 * rel_err(ref, ref_ld))


@pytest.mark.parametrize("p,E,A,mu,diss,tp", [(2, 3, 0.12, 0.02, 1, 0), (3, 3, 0.1, 0.0, 1, 0),
                                             (4, 3, 0.1, 0.01, 1, 0), (4, 2, 0.15, 0.01, 2, 0),
                                             (6, 2, 0.1, 0.01, 1, 2), (9, 2, 0.1, 0.01, 1, 0)])
def test_residual_with_optimized_metrics(p, E, A, mu, diss, tp):
    require_gpu()
    print(f"optimised metrics p={p} E={E} mu={mu} diss={diss} two_point={tp}", flush=True)
    c = _case(p, E, A, mu, diss, tp)
    q = c.jumpy(0.02, seed=p)
    ref = c.residual(q)
    ps = P.ProblemSet([device_problem(c)])
    out = from_dev(ps.residual(to_dev(q)), q.shape)
    assert ps.status() == 0
    err, bar = rel_err(out, ref), _bar(c, q, ref)
    print(f"  err {err:.2e} bar {bar:.1e}")
    assert err < bar


def test_freestream_and_entropy_conservation_on_the_gpu():
    require_gpu()
    c = _case(4, 6, 0.12, 0.0, 0)
    ps = P.ProblemSet([device_problem(c)])
    # uniform flow
    q0 = np.zeros_like(c.q)
    q0[0], q0[1], q0[2], q0[3], q0[4] = 1.1, 0.2, -0.1, 0.3, 2.9
    r0 = from_dev(ps.residual(to_dev(q0)), q0.shape)
    assert np.abs(r0).max() < 1e-13
    # entropy-conservative interfaces, inviscid, periodic: sum w J w.dq/dt = 0
    q = c.jumpy(0.03, seed=4)
    r = from_dev(ps.residual(to_dev(q)), q.shape)
    assert ps.status() == 0
    wJ = c.weights3d()[None] * c.jac
    wv = G.entropy_variables(q, c.prm.gas)
    rate = (wJ * (wv * r).sum(0)).sum()
    scale = (wJ * np.abs(wv * r).sum(0)).sum()
    print(f"entropy rate {rate:.2e} of {scale:.2e}")
    assert abs(rate) < 1e-13 * scale


# ------------------------------------------------------------------------------------------------
# The GPU constructor (sbp_metrics_optimized) against the oracle's optimized_metrics
# ------------------------------------------------------------------------------------------------
MET_TOL = 1e-13   # the two sides solve the same least-norm problems with different bases and orders


def _mapping(p, E, A):
    prob = W.make_problem(p=p, E=E, L=2.0, A=A)
    sbp = operators.SBP1D(p)
    return prob, sbp, W.mapping_jacobian(prob, sbp.x)


def _gpu_optimized(p, nbr, F):
    m, j = P.metrics_optimized(p, torch.as_tensor(np.ascontiguousarray(nbr), device=DEV),
                               torch.as_tensor(np.ascontiguousarray(F.reshape(9, -1)), device=DEV))
    N = p + 1
    K = nbr.shape[0]
    return (m.cpu().numpy().reshape(9, K, N, N, N), j.cpu().numpy().reshape(K, N, N, N))


def _shared_faces_identical(m, nbr, N):
    for l in range(3):
        f = 2 * l + 1
        inner = nbr[:, f] >= 0
        own = m[3 * l:3 * l + 3][Gm._face_slice(l, 1, N)][:, inner]
        par = m[3 * l:3 * l + 3][:, nbr[inner, f]][Gm._face_slice(l, 0, N)]
        if not np.array_equal(own, par):
            return False
    return True


@pytest.mark.parametrize("p,E,A,box", [(2, 3, 0.12, None), (3, 3, 0.1, None), (4, 3, 0.15, None),
                                       (5, 2, 0.1, None), (7, 2, 0.1, None), (8, 2, 0.12, None),
                                       (4, 1, 0.1, None), (2, 7, 0.1, None),
                                       (3, 4, 0.1, (None, -3, None)), (4, 3, 0.12, (-1, -2, -3))])
def test_gpu_constructor_matches_the_oracle(p, E, A, box):
    require_gpu()
    print(f"optimised-metric constructor p={p} E={E} A={A} box={box}", flush=True)
    prob, sbp, F = _mapping(p, E, A)
    nbr = W.neighbours(E, box=box) if box is not None else W.neighbours(E)
    ref, Jr = Gm.optimized_metrics(F, nbr, sbp)
    got, J = _gpu_optimized(p, nbr, F)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    jerr = np.abs(J - Jr).max() / np.abs(Jr).max()
    gcl = np.abs(Gm.gcl_residual(got, sbp.D)).max() / np.abs(got).max()
    print(f"  metric err {err:.2e}, J err {jerr:.2e}, GCL {gcl:.2e}")
    assert err < MET_TOL and jerr < 1e-15 and gcl < 1e-13
    assert _shared_faces_identical(got, nbr, sbp.N)


@pytest.mark.parametrize("p,E", [(12, 2), (15, 2)])
def test_gpu_constructor_properties_at_high_degree(p, E):
    """Degrees whose dense oracle solve is out of reach: GCL to rounding, identical face values,
    closed element surfaces, and within the quadrature error of the analytic metrics."""
    require_gpu()
    prob, sbp, F = _mapping(p, E, 0.1)
    nbr = W.neighbours(E)
    got, J = _gpu_optimized(p, nbr, F)
    a, Ja = Gm.analytic_metrics(F)
    scale = np.abs(got).max()
    assert np.abs(Gm.gcl_residual(got, sbp.D)).max() < 1e-13 * scale
    assert np.abs(Gm.surface_closure(got, sbp.w)).max() < 1e-13 * scale
    assert _shared_faces_identical(got, nbr, sbp.N)
    assert np.abs(got - a).max() < 1e-6 * scale
    assert np.array_equal(J, Ja) or np.abs(J - Ja).max() < 1e-15 * np.abs(Ja).max()


def test_gpu_constructor_on_the_taylor_green_mesh():
    """The full Taylor-Green mesh of the benchmark (p = 4, 32^3 elements, warped, periodic): no
    dense oracle at this size, so the result is checked through what defines it: GCL to rounding,
    identical face values, closed surfaces, order-p closeness to the analytic metrics, and
    sampled elements against the oracle's per-element volume step (the least-norm GCL projection
    of the GPU's own face values, computed with the oracle's pseudo-inverse)."""
    require_gpu()
    p, E = 4, 32
    prob = W.make_problem(p=p, E=E, L=2.0 * np.pi, A=0.1)
    sbp = operators.SBP1D(p)
    F = W.mapping_jacobian(prob, sbp.x)
    nbr = W.neighbours(E)
    _gpu_optimized(p, W.neighbours(2), _mapping(p, 2, 0.1)[2])     # tables built, kernels loaded
    t0 = time.perf_counter()
    got, J = _gpu_optimized(p, nbr, F)
    print(f"Taylor-Green mesh: constructor incl. transfers {time.perf_counter() - t0:.3f} s")
    a, Ja = Gm.analytic_metrics(F)
    scale = np.abs(got).max()
    gcl = np.abs(Gm.gcl_residual(got, sbp.D)).max() / scale
    print(f"Taylor-Green mesh: GCL {gcl:.2e}, distance to analytic {np.abs(got - a).max() / scale:.2e}")
    assert gcl < 1e-13
    assert np.abs(Gm.surface_closure(got, sbp.w)).max() < 1e-13 * scale
    assert _shared_faces_identical(got, nbr, sbp.N)
    assert np.abs(got - a).max() < 1e-5 * scale
    assert np.abs(J - Ja).max() < 1e-15 * np.abs(Ja).max()
    # volume step on sampled elements: from the GPU's face values, the oracle's least-norm
    # projection must reproduce the GPU's volume values
    M, held, pinv, _ = Gm.gcl_operator(sbp.D)
    rng = np.random.Generator(np.random.PCG64(11))
    n = sbp.N ** 3
    for e in rng.choice(prob.K, 24, replace=False):
        for m in range(3):
            start = np.concatenate([a[3 * l + m, e].reshape(n) for l in range(3)])
            fin = np.concatenate([got[3 * l + m, e].reshape(n) for l in range(3)])
            start[held] = fin[held]
            start[~held] += pinv @ (-(M @ start))
            assert np.abs(start - fin).max() < 1e-14 * scale


def test_gpu_residual_with_gpu_built_metrics():
    """The residual evaluated with the GPU-built optimised metrics against the oracle residual
    with the oracle-built ones."""
    require_gpu()
    c = _case(4, 3, 0.12, 0.01, 1)
    F = W.mapping_jacobian(c.prob, c.sbp.x)
    m, j = P.metrics_optimized(4, torch.as_tensor(c.nbr, device=DEV).contiguous(),
                               torch.as_tensor(np.ascontiguousarray(F.reshape(9, -1)), device=DEV))
    q = c.jumpy(0.02, seed=9)
    ref = c.residual(q)
    prob = device_problem(c)
    prob.metric, prob.jac = m, j
    ps = P.ProblemSet([prob])
    out = from_dev(ps.residual(to_dev(q)), q.shape)
    err, bar = rel_err(out, ref), _bar(c, q, ref)
    print(f"residual with GPU-built metrics: err {err:.2e} bar {bar:.1e}")
    assert err < max(bar, 1e-12)


def test_gpu_constructor_rejects_unpaired_faces():
    require_gpu()
    prob, sbp, F = _mapping(3, 3, 0.1)
    nbr = W.neighbours(3).copy()
    nbr[5, 1] = 7                      # element 5's + xi_1 face names element 7, which does not pair back
    with pytest.raises(P.SBPError):
        _gpu_optimized(3, nbr, F)
    nbr = W.neighbours(3).copy()
    nbr[2, 3] = 27                     # out of range
    with pytest.raises(P.SBPError):
        _gpu_optimized(3, nbr, F)
