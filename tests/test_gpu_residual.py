"""GPU residual against the oracle, element by element (relative error per component,
max |dq/dt_gpu - dq/dt_oracle| / max |dq/dt_oracle| <= 1e-12)."""
import numpy as np
import pytest
import torch

import paper_1911_10966_amd as P
import workloads as W
from gpu_helpers import DEV, device_problem, from_dev, require_gpu, to_dev
from helpers import Case, rel_err
from oracle import residual as R

pytestmark = pytest.mark.gpu
TOL = 1e-12

CASES = [
    # p, E, mu, iface_diss, two_point, A, eta
    (1, 3, 0.0, 1, 0, 0.1, 1.0),
    (1, 2, 0.02, 1, 0, 0.1, 1.0),
    (2, 3, 0.0, 0, 0, 0.12, 1.0),
    (2, 3, 0.02, 1, 0, 0.12, 1.0),
    (3, 3, 0.0, 1, 0, 0.1, 1.0),
    (3, 2, 0.03, 1, 0, 0.1, 0.0),
    (4, 3, 0.01, 1, 0, 0.1, 1.0),
    (4, 2, 0.0, 1, 1, 0.1, 1.0),
    (4, 2, 0.0, 1, 2, 0.1, 1.0),
    (4, 2, 0.01, 0, 2, 0.1, 1.0),
    (5, 2, 0.01, 1, 0, 0.15, 1.0),
    (6, 2, 0.01, 1, 0, 0.1, 1.0),
    (7, 2, 0.02, 1, 0, 0.15, 1.0),
    (8, 2, 0.01, 1, 0, 0.1, 1.0),
    (1, 3, 0.0, 1, 3, 0.1, 1.0),
    (3, 3, 0.02, 1, 3, 0.12, 1.0),
    (4, 2, 0.0, 0, 3, 0.1, 1.0),
    (7, 2, 0.01, 1, 3, 0.1, 1.0),
    (2, 3, 0.01, 1, 2, 0.1, 1.0),
    (5, 2, 0.02, 1, 0, 0.1, 0.0),
    (6, 2, 0.0, 0, 2, 0.1, 1.0),
    (8, 2, 0.0, 1, 1, 0.12, 1.0),
    (6, 2, 0.01, 0, 0, 0.1, 1.0),
    # degrees 9..15 run as plane passes
    (9, 2, 0.01, 1, 0, 0.1, 1.0),
    (10, 3, 0.0, 1, 0, 0.12, 1.0),
    (11, 2, 0.02, 0, 2, 0.1, 1.0),
    (12, 2, 0.01, 1, 3, 0.1, 1.0),
    (13, 2, 0.0, 1, 1, 0.1, 1.0),
    (14, 2, 0.01, 1, 0, 0.1, 0.0),
    (15, 2, 0.01, 1, 0, 0.1, 1.0),
    (15, 2, 0.0, 0, 3, 0.1, 1.0),
    # entropy-stable matrix interface dissipation
    (3, 3, 0.02, 2, 0, 0.1, 1.0),
    (4, 2, 0.0, 2, 2, 0.12, 1.0),
    (2, 3, 0.01, 2, 2, 0.1, 1.0),
    (6, 2, 0.0, 2, 0, 0.1, 1.0),
    (11, 2, 0.01, 2, 0, 0.1, 1.0),
]


@pytest.mark.parametrize("p,E,mu,diss,tp,A,eta", CASES)
def test_residual_matches_oracle(p, E, mu, diss, tp, A, eta):
    require_gpu()
    print(f"case p={p} E={E} mu={mu} diss={diss} two_point={tp}", flush=True)
    c = Case(W.make_problem(p=p, E=E, L=2.0, A=A, mu=mu, iface_diss=diss, two_point=tp, eta=eta,
                            seed=100 + p, u_rms=0.3))
    q = c.jumpy(0.02, seed=p)
    ref = c.residual(q)
    ps = P.ProblemSet([device_problem(c)])
    out = from_dev(ps.residual(to_dev(q)), q.shape)
    assert ps.status() == 0
    assert rel_err(out, ref) < TOL


def test_euler_p3_e4_workload_full():
    """The Euler workload (p = 3, 4^3 warped elements, smooth random state), every node."""
    require_gpu()
    c = Case(W.config("euler_p3_e4"))
    ref = c.residual()
    ps = P.ProblemSet([device_problem(c)])
    out = from_dev(ps.residual(to_dev(c.q)), c.q.shape)
    assert rel_err(out, ref) < TOL


def test_bitwise_deterministic():
    require_gpu()
    c = Case(W.make_problem(p=4, E=3, L=2.0, A=0.1, mu=0.01, seed=5, u_rms=0.3))
    ps = P.ProblemSet([device_problem(c)])
    qd = to_dev(c.jumpy(0.02, 1))
    a = ps.residual(qd).clone()
    b = ps.residual(qd).clone()
    assert torch.equal(a, b)


def test_nonphysical_state_is_flagged():
    require_gpu()
    c = Case(W.make_problem(p=2, E=2, L=2.0, A=0.1, mu=0.0, seed=6, u_rms=0.3))
    ps = P.ProblemSet([device_problem(c)])
    q = c.q.copy()
    q[0, 3, 1, 1, 1] = -1.0
    ps.residual(to_dev(q))
    with pytest.raises(P.SBPError) as ei:
        ps.status()
    assert ei.value.code == -4
    # cleared after reporting
    ps.residual(to_dev(c.q))
    assert ps.status() == 0


def test_bad_neighbour_is_flagged_not_read():
    require_gpu()
    c = Case(W.make_problem(p=2, E=2, L=2.0, A=0.1, mu=0.01, seed=7, u_rms=0.3))
    dp = device_problem(c)
    dp.nbr[1, 3] = 999
    ps = P.ProblemSet([dp])
    ps.residual(to_dev(c.q))
    with pytest.raises(P.SBPError) as ei:
        ps.status()
    assert ei.value.code == -3


def test_metrics_match_oracle():
    require_gpu()
    for p, E, A in [(3, 3, 0.1), (4, 2, 0.15), (8, 2, 0.1), (1, 3, 0.1), (9, 2, 0.1), (11, 2, 0.15),
                    (15, 2, 0.1)]:
        c = Case(W.make_problem(p=p, E=E, L=2.0, A=A))
        x = torch.as_tensor(np.ascontiguousarray(c.x.reshape(3, -1)), device=DEV)
        m, j = P.metrics(p, x)
        torch.cuda.synchronize()
        m = m.cpu().numpy().reshape(c.metric.shape)
        j = j.cpu().numpy().reshape(c.jac.shape)
        assert np.abs(m - c.metric).max() < 1e-13 * np.abs(c.metric).max() * p
        assert np.abs(j - c.jac).max() < 1e-13 * np.abs(c.jac).max() * p


def test_profiled_launches_recorded_without_waiting():
    """profile_residual(wait=False) records events only; profile_collect returns their number and
    total duration, and the result equals the plain residual."""
    require_gpu()
    c = Case(W.make_problem(p=4, E=3, L=2.0, A=0.1, mu=0.01, seed=8, u_rms=0.3))
    ps = P.ProblemSet([device_problem(c)])
    qd = to_dev(c.q)
    out = torch.empty_like(qd)
    P.profile_collect()
    for _ in range(3):
        assert ps.profile_residual(qd, out, wait=False) is None
    n, total = P.profile_collect()
    assert n == 3 and total > 0.0
    assert P.profile_collect() == (0, 0.0)
    assert ps.profile_residual(qd, out) > 0.0
    assert torch.equal(out, ps.residual(qd))
