"""Cached launch plans and RK4 graphs are released with their workspace: explicit release counts,
results unchanged after a release, and many problem sets made and dropped in turn without growth of
device memory."""
import pytest
import torch

import paper_1911_10966_amd as P
import workloads as W
from gpu_helpers import DEV, device_problem, require_gpu, to_dev
from helpers import Case

pytestmark = pytest.mark.gpu


def test_release_counts_plans_and_graphs_and_results_stay():
    require_gpu()
    c = Case(W.make_problem(p=3, E=2, L=2.0, A=0.1, mu=0.01, seed=3, u_rms=0.3))
    ps = P.ProblemSet([device_problem(c)])
    q = to_dev(c.q)
    r0 = ps.residual(q).clone()
    dt = torch.tensor([1e-3], dtype=torch.float64, device=DEV)
    qa = q.clone()
    ps.rk_step(qa, dt, 1)
    assert ps.release() == 2          # one plan, one graph
    assert ps.release() == 0
    assert torch.equal(ps.residual(q), r0)
    qb = q.clone()
    ps.rk_step(qb, dt, 1)
    assert torch.equal(qa, qb)
    assert ps.status() == 0


def test_many_problem_sets_do_not_grow_device_memory():
    require_gpu()
    c = Case(W.make_problem(p=2, E=2, L=2.0, A=0.1, mu=0.01, seed=4, u_rms=0.3))
    q = to_dev(c.q)
    out = torch.empty_like(q)
    dt = torch.tensor([1e-3], dtype=torch.float64, device=DEV)

    def cycle(i):
        dp = device_problem(c)
        dp.eta = 1.0 + 1e-3 * i          # a distinct problem set every time (its own plan)
        ps = P.ProblemSet([dp])
        ps.residual(q, out)
        qq = q.clone()
        ps.rk_step(qq, dt, 1)
        del ps, qq

    for i in range(20):
        cycle(i)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for i in range(20, 520):
        cycle(i)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"device memory free before {free0} after {free1}")
    assert free1 >= free0 - (8 << 20)
