"""GPU residual with Dirichlet boundary faces and a source term (the manufactured-solution problem of
the viscous error-vs-cost study) against the oracle, element by element."""
import numpy as np
import pytest
import torch

import paper_1911_10966_amd as P
import workloads as W
from workloads import mms
from gpu_helpers import DEV, device_problem, from_dev, require_gpu, to_dev
from helpers import Case, rel_err, rk4_increment_check
from oracle import operators, residual as R

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _mms_case(p, E, A, two_point=0, mu=None, iface_diss=1):
    c = Case(W.mms_problem(p, E, A=A, two_point=two_point, mu=mu, iface_diss=iface_diss))
    c.nbr = W.neighbours(E, periodic=False)
    c.bc = mms.conservative(c.x)
    c.src = mms.source(c.x, mu=c.prob.mu)
    return c


def _tol(c, q, ref, **kw):
    """max(TOL, 4 x the FP64 floor of this case: double oracle against long-double oracle on the
    same inputs).  The supersonic state (|U| ~ 1400, P ~ 1e5) cancels strongly in the residual."""
    LD = np.longdouble
    ref_ld = R.residual(q.astype(LD), c.metric.astype(LD), c.jac.astype(LD), c.nbr,
                        operators.SBP1D(c.prob.p, LD), c.prm,
                        bc=None if kw.get("bc") is None else kw["bc"].astype(LD),
                        source=None if kw.get("source") is None else kw["source"].astype(LD))
    return max(TOL, 4.0 * rel_err(ref, ref_ld))


def _dev_problem(c, bc=True, src=True):
    dp = device_problem(c)
    dp.nbr = torch.as_tensor(c.nbr, device=DEV).contiguous()
    if bc:
        dp.bc_state = to_dev(c.bc)
    if src:
        dp.source = to_dev(c.src)
    return dp


CASES = [
    # p, E, A, two_point, mu (None: the study's), iface_diss
    (2, 3, 0.05, 0, None, 1),
    (3, 2, 0.0, 3, 0.0, 1),
    (4, 2, 0.05, 2, 1e-2, 0),
    (6, 2, 0.05, 0, 1e-2, 1),
    (10, 2, 0.0, 0, 1e-2, 1),
]


@pytest.mark.parametrize("p,E,A,tp,mu,diss", CASES)
def test_boundary_residual_matches_oracle(p, E, A, tp, mu, diss):
    require_gpu()
    print(f"case p={p} E={E} A={A} two_point={tp} mu={mu}", flush=True)
    c = _mms_case(p, E, A, tp, mu, diss)
    q = c.jumpy(0.01, seed=p)
    ref = R.residual(q, c.metric, c.jac, c.nbr, c.sbp, c.prm, bc=c.bc)
    ps = P.ProblemSet([_dev_problem(c, src=False)])
    out = from_dev(ps.residual(to_dev(q)), q.shape)
    assert ps.status() == 0
    assert rel_err(out, ref) < _tol(c, q, ref, bc=c.bc)
    # with the forcing: the same plus the source, node by node
    ps2 = P.ProblemSet([_dev_problem(c)])
    out2 = from_dev(ps2.residual(to_dev(q)), q.shape)
    ref2 = ref + c.src
    scale = np.abs(ref).reshape(5, -1).max(1)[:, None]
    assert np.all(np.abs((out2 - ref2).reshape(5, -1)) <= 4 * _tol(c, q, ref, bc=c.bc) * scale + 1e-15 * np.abs(c.src).reshape(5, -1))


def test_mms_rk4_step_matches_oracle():
    require_gpu()
    c = _mms_case(2, 3, 0.05)
    dt = 0.25 * (1.0 / 3) / (9 * mms.speed_max())
    ps = P.ProblemSet([_dev_problem(c)])
    q0 = c.jumpy(0.01, 7)
    qd = to_dev(q0)
    ps.rk_step(qd, torch.tensor([dt], dtype=torch.float64, device=DEV), 1)
    assert ps.status() == 0
    out = from_dev(qd, q0.shape)

    def rhs(dtype):
        m, j, sbp = c.metric.astype(dtype), c.jac.astype(dtype), operators.SBP1D(c.prob.p, dtype)
        bc, src = c.bc.astype(dtype), c.src.astype(dtype)
        return lambda y: R.residual(y, m, j, c.nbr, sbp, c.prm, bc=bc, source=src)

    # compare the increments (the state itself is large)
    err, bar = rk4_increment_check(rhs(np.float64), rhs(np.longdouble), q0, dt, 1, out)
    print(f"  RK4 increment err {err:.2e} bar {bar:.1e}")
    assert err < bar


def test_batch_of_periodic_and_boundary_problems():
    require_gpu()
    cb = _mms_case(3, 2, 0.05)
    cp = Case(W.make_problem(p=3, E=2, L=2.0, A=0.1, mu=1e-3, seed=33, u_rms=0.3))
    ps = P.ProblemSet([_dev_problem(cb), device_problem(cp)])
    qb, qp = cb.jumpy(0.01, 1), cp.jumpy(0.01, 2)
    out = ps.residual(torch.cat([to_dev(qb), to_dev(qp)])).cpu().numpy()
    assert ps.status() == 0
    n = qb.size
    ref_b = R.residual(qb, cb.metric, cb.jac, cb.nbr, cb.sbp, cb.prm, bc=cb.bc)
    ref_p = cp.residual(qp)
    assert rel_err(out[n:].reshape(qp.shape), ref_p) < TOL
    # the boundary problem's output minus its forcing is its residual
    d = (out[:n].reshape(qb.shape) - cb.src - ref_b).reshape(5, -1)
    scale = np.abs(ref_b).reshape(5, -1).max(1)[:, None]
    tol = _tol(cb, qb, ref_b, bc=cb.bc)
    assert np.all(np.abs(d) <= 4 * tol * scale + 2e-16 * np.abs(cb.src).reshape(5, -1))


def test_boundary_without_data_is_a_mesh_error():
    require_gpu()
    c = _mms_case(2, 2, 0.0)
    ps = P.ProblemSet([_dev_problem(c, bc=False, src=False)])
    ps.residual(to_dev(c.q))
    with pytest.raises(P.SBPError):
        ps.status()
