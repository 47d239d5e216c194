"""GPU residual with wall boundary faces (slip -2, adiabatic no-slip -3, mixed with Dirichlet -1)
against the oracle, element by element, on every kernel path: per-node faces (N <= 5), face work
items (N = 6..8), the plane passes (N >= 10), matrix dissipation, the SF-KG and DC forms; then an
RK4 step, a batch mixing wall and periodic problems, conservation at a large size, and the errors
(the VJP with walls: test_gpu_vjp_boundaries)."""
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


def _case(p, E, A, box, mu, diss, tp, seed=5):
    c = Case(W.make_problem(p=p, E=E, L=2.0, A=A, mu=mu, iface_diss=diss, two_point=tp, seed=seed,
                            u_rms=0.3, box=box))
    c.nbr = W.problem_neighbours(c.prob)
    c.bc = c.jumpy(0.02, seed + 100) if -1 in box else None
    return c


def _tol(c, q, ref):
    """max(TOL, 4 x the FP64 floor of this case: double oracle against long-double oracle on the
    same inputs)."""
    LD = np.longdouble
    ref_ld = R.residual(q.astype(LD), c.metric.astype(LD), c.jac.astype(LD), c.nbr,
                        operators.SBP1D(c.prob.p, LD), c.prm,
                        bc=None if c.bc is None else c.bc.astype(LD))
    return max(TOL, 4.0 * rel_err(ref, ref_ld))


def _rhs(c, dtype=np.float64):
    """The oracle residual of case c as a function of the state, in `dtype` arithmetic."""
    m, j, sbp = c.metric.astype(dtype), c.jac.astype(dtype), operators.SBP1D(c.prob.p, dtype)
    bc = None if c.bc is None else c.bc.astype(dtype)
    return lambda y: R.residual(y, m, j, c.nbr, sbp, c.prm, bc=bc)


def _dev_problem(c):
    dp = device_problem(c)
    if c.bc is not None:
        dp.bc_state = to_dev(c.bc)
    return dp


CASES = [
    # p, E, A, box (per direction: None periodic, else the boundary kind), mu, iface_diss, two_point
    (2, 3, 0.1, (-2, None, -2), 0.0, 1, 0),
    (3, 2, 0.1, (-3, -3, None), 0.02, 1, 0),
    (4, 2, 0.1, (None, -3, -3), 0.02, 2, 0),
    (4, 2, 0.05, (-1, -3, None), 0.02, 1, 0),
    (3, 2, 0.0, (-2, None, None), 0.0, 1, 3),
    (5, 2, 0.05, (-3, None, -3), 0.01, 1, 2),
    (7, 2, 0.1, (-2, -2, -2), 0.0, 2, 0),
    (6, 2, 0.05, (-3, -1, -3), 0.01, 0, 0),
    (9, 2, 0.05, (-3, -3, -3), 0.01, 1, 0),
    (10, 2, 0.0, (-2, -2, -2), 0.0, 2, 0),
    (11, 1, 0.05, (-3, -1, -3), 0.01, 1, 0),
]


@pytest.mark.parametrize("p,E,A,box,mu,diss,tp", CASES)
def test_wall_residual_matches_oracle(p, E, A, box, mu, diss, tp):
    require_gpu()
    print(f"case p={p} E={E} A={A} box={box} mu={mu} diss={diss} two_point={tp}", flush=True)
    c = _case(p, E, A, box, mu, diss, tp)
    q = c.jumpy(0.02, seed=p)
    ref = R.residual(q, c.metric, c.jac, c.nbr, c.sbp, c.prm, bc=c.bc)
    ps = P.ProblemSet([_dev_problem(c)])
    out = from_dev(ps.residual(to_dev(q)), q.shape)
    assert ps.status() == 0
    assert rel_err(out, ref) < _tol(c, q, ref)


def test_wall_rk4_step_in_a_batch_with_a_periodic_problem():
    require_gpu()
    cw = _case(3, 3, 0.1, (None, -3, -3), 0.01, 1, 0)
    cp = Case(W.make_problem(p=3, E=2, L=2.0, A=0.1, mu=1e-3, seed=33, u_rms=0.3))
    ps = P.ProblemSet([_dev_problem(cw), device_problem(cp)])
    qw, qp = cw.jumpy(0.01, 1), cp.jumpy(0.01, 2)
    qd = torch.cat([to_dev(qw), to_dev(qp)])
    dts = torch.tensor([2e-3, 3e-3], dtype=torch.float64, device=DEV)
    ps.rk_step(qd, dts, 2)
    assert ps.status() == 0
    out = qd.cpu().numpy()
    n = qw.size
    cp.bc = None
    for c, q, dt, got in ((cw, qw, 2e-3, out[:n]), (cp, qp, 3e-3, out[n:])):
        err, bar = rk4_increment_check(_rhs(c), _rhs(c, np.longdouble), q, dt, 2, got.reshape(q.shape))
        print(f"  2-step RK4 increment err {err:.2e} bar {bar:.1e}")
        assert err < bar


@pytest.mark.parametrize("p,E", [(4, 16), (7, 8)])
def test_channel_conserves_mass_and_energy_at_size(p, E):
    """Adiabatic no-slip walls: sum_nodes w J (dq/dt)_c vanishes for mass and energy (any size)."""
    require_gpu()
    prob = W.channel_problem(p, E, A=0.05)
    c = Case(prob)
    c.nbr = W.problem_neighbours(prob)
    q = c.jumpy(0.01, 3)
    ps = P.ProblemSet([device_problem(c)])
    out = from_dev(ps.residual(to_dev(q)), q.shape)
    assert ps.status() == 0
    wj = c.weights3d() * c.jac
    tot = (wj * out).sum(axis=(1, 2, 3, 4))
    mag = (wj * np.abs(out)).sum(axis=(1, 2, 3, 4))
    assert abs(tot[0]) < 1e-12 * mag[0]
    assert abs(tot[4]) < 1e-12 * mag[4]
    # sampled elements against the oracle
    rng = np.random.Generator(np.random.PCG64(p))
    elems = np.sort(rng.choice(prob.K, size=24, replace=False))
    ref = R.residual(q, c.metric, c.jac, c.nbr, c.sbp, c.prm, elems=elems)
    LD = np.longdouble
    ref_ld = R.residual(q.astype(LD), c.metric.astype(LD), c.jac.astype(LD), c.nbr,
                        operators.SBP1D(p, LD), c.prm, elems=elems)
    err, bar = rel_err(out[:, elems], ref_ld), max(TOL, 4.0 * rel_err(ref, ref_ld))
    print(f"  sampled elements at size: err {err:.2e} bar {bar:.1e}")
    assert err < bar


def test_channel_manufactured_solution_residual_matches_oracle():
    require_gpu()
    prob = W.channel_problem(3, 4, A=0.05)
    c = Case(prob)
    c.nbr = W.problem_neighbours(prob)
    q = mms.conservative(c.x, kind="channel")
    src = mms.source(c.x, kind="channel")
    dp = device_problem(c)
    dp.source = to_dev(src)
    ps = P.ProblemSet([dp])
    out = from_dev(ps.residual(to_dev(q)), q.shape)
    assert ps.status() == 0
    ref = R.residual(q, c.metric, c.jac, c.nbr, c.sbp, c.prm, source=src)
    scale = np.abs(src).reshape(5, -1).max(1)[:, None]
    assert np.all(np.abs((out - ref).reshape(5, -1)) <= 1e-12 * scale)


def test_slip_wall_on_a_viscous_problem_is_a_mesh_error():
    require_gpu()
    c = _case(2, 2, 0.0, (-2, None, None), 0.01, 1, 0)
    ps = P.ProblemSet([_dev_problem(c)])
    ps.residual(to_dev(c.q))
    with pytest.raises(P.SBPError):
        ps.status()
