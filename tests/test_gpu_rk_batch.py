"""RK4 steps and the batched (several problems per call) path against the oracle."""
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


@pytest.mark.parametrize("p,E,mu,steps", [(3, 2, 0.02, 1), (4, 3, 0.01, 2), (2, 3, 0.0, 3)])
def test_rk4_step_matches_oracle(p, E, mu, steps):
    require_gpu()
    print(f"rk p={p} E={E} mu={mu} steps={steps}", flush=True)
    prob = W.make_problem(p=p, E=E, L=2.0, A=0.1, mu=mu, seed=20 + p, u_rms=0.3)
    c = Case(prob)
    dt = W.cfl_dt(prob, torch.as_tensor(c.x))
    q = c.q.copy()
    for _ in range(steps):
        q = R.rk4_step(lambda y: c.residual(y), q, dt)
    ps = P.ProblemSet([device_problem(c)])
    qd = to_dev(c.q)
    dtd = torch.tensor([dt], dtype=torch.float64, device=DEV)
    ps.rk_step(qd, dtd, steps)
    out = from_dev(qd, c.q.shape)
    assert ps.status() == 0
    assert rel_err(out - c.q, q - c.q) < TOL


def test_rk4_graph_replay_is_consistent():
    """Repeated calls replay the recorded graph; two single steps equal one call of two steps."""
    require_gpu()
    prob = W.make_problem(p=3, E=2, L=2.0, A=0.1, mu=0.02, seed=31, u_rms=0.3)
    c = Case(prob)
    ps = P.ProblemSet([device_problem(c)])
    dtd = torch.tensor([W.cfl_dt(prob, torch.as_tensor(c.x))], dtype=torch.float64, device=DEV)
    qa = to_dev(c.q)
    ps.rk_step(qa, dtd, 1)
    torch.cuda.synchronize()
    ps.rk_step(qa, dtd, 1)
    qb = to_dev(c.q)
    ps.rk_step(qb, dtd, 2)
    torch.cuda.synchronize()
    assert torch.equal(qa, qb)


def test_batched_residual_matches_oracle_per_problem():
    require_gpu()
    probs = [W.make_problem(p=p, E=E, L=2.0, A=0.05 + 0.02 * i, mu=1e-3 * (i % 2), seed=40 + i, u_rms=0.3)
             for i, (p, E) in enumerate([(2, 3), (5, 2), (3, 2), (8, 2), (4, 3), (1, 3), (6, 2), (7, 2)])]
    cases = [Case(pr) for pr in probs]
    ps = P.ProblemSet([device_problem(c) for c in cases])
    qs = [c.jumpy(0.01, i) for i, c in enumerate(cases)]
    qd = torch.cat([to_dev(q) for q in qs])
    out = ps.residual(qd).cpu().numpy()
    off = 0
    for c, q in zip(cases, qs):
        n = q.size
        assert rel_err(out[off:off + n].reshape(q.shape), c.residual(q)) < TOL
        off += n


def test_batched_rk4_matches_oracle_per_problem():
    require_gpu()
    probs = [W.make_problem(p=p, E=E, L=2.0, A=0.1, mu=1e-3, seed=60 + i, u_rms=0.3)
             for i, (p, E) in enumerate([(2, 2), (4, 2), (3, 3), (9, 2)])]
    cases = [Case(pr) for pr in probs]
    dts = [W.cfl_dt(pr, torch.as_tensor(c.x)) for pr, c in zip(probs, cases)]
    ps = P.ProblemSet([device_problem(c) for c in cases])
    qd = torch.cat([to_dev(c.q) for c in cases])
    ps.rk_step(qd, torch.tensor(dts, dtype=torch.float64, device=DEV), 2)
    out = qd.cpu().numpy()
    off = 0
    for c, dt in zip(cases, dts):
        q = c.q
        for _ in range(2):
            q = R.rk4_step(lambda y: c.residual(y), q, dt)
        n = q.size
        assert rel_err(out[off:off + n].reshape(q.shape) - c.q, q - c.q) < TOL
        off += n


def test_every_schedule_gives_bitwise_identical_results():
    """Each schedule (elements per workgroup, persistent grid) computes each element identically."""
    require_gpu()
    probs = [W.make_problem(p=p, E=E, L=2.0, A=0.1, mu=mu, seed=120 + p, u_rms=0.3)
             for p, E, mu in [(1, 3, 0.01), (2, 3, 0.0), (3, 3, 0.01), (4, 2, 0.01), (5, 2, 0.0),
                              (6, 2, 0.01), (7, 2, 0.01), (8, 2, 0.0), (10, 3, 0.01), (15, 2, 0.0)]]
    cases = [Case(pr) for pr in probs]
    ps = P.ProblemSet([device_problem(c) for c in cases])
    qd = torch.cat([to_dev(c.jumpy(0.01, i)) for i, c in enumerate(cases)])
    ref = ps.residual(qd).clone()
    dt = torch.tensor([1e-4] * len(probs), dtype=torch.float64, device=DEV)
    q_rk = qd.clone()
    ps.rk_step(q_rk, dt, 1)
    for p in [pr.p for pr in probs]:
        for v in range(P.schedule_count(p)):
            ps.set_schedule(p, v)
            assert torch.equal(ps.residual(qd), ref), (p, v)
            q2 = qd.clone()
            ps.rk_step(q2, dt, 1)
            assert torch.equal(q2, q_rk), (p, v)
        ps.set_schedule(p, 0)
    chosen = ps.autotune(qd, reps=1)
    assert len(chosen) == len(probs)
    assert torch.equal(ps.residual(qd), ref)
