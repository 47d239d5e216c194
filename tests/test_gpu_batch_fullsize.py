"""The heterogeneous batch workload (256 periodic problems, p ~ U{2..8}, 2^3..12^3 elements) in the
launch configuration the benchmark times: sampled problems and elements against the oracle,
conservation over 10 graph-replayed RK4 steps for every problem, and the 10-step RK4 increments of
five of its small problems against the oracle's RK4."""
import numpy as np
import pytest
import torch

import paper_1911_10966_amd as P
import workloads as W
from gpu_helpers import DEV, require_gpu
from helpers import rel_err, rk4_increment_check
from oracle import geometry, operators, residual as R

pytestmark = pytest.mark.gpu
TOL = 1e-12


def build_batch(oracle_for=()):
    probs = W.batch_config()
    dps, qs, dts, host = [], [], [], {}
    for b, pr in enumerate(probs):
        x1d = P.lgl_operator(pr.p)[0]
        x = W.coords(pr, x1d, device=DEV)
        if b in oracle_for:
            sbp = operators.SBP1D(pr.p)
            xo = W.coords(pr, sbp.x).numpy()
            metric = torch.as_tensor(geometry.curl_metrics(xo, sbp.D).reshape(9, -1), device=DEV)
            jac = torch.as_tensor(geometry.jacobian(xo, sbp.D).reshape(-1), device=DEV)
            host[b] = (sbp, xo)
        else:
            metric, jac = P.metrics(pr.p, x.reshape(3, -1).contiguous())
        q = W.state(pr, x)
        dts.append(W.cfl_dt(pr, x))
        dps.append(P.Problem(p=pr.p, n_elem=pr.K, nbr=torch.as_tensor(W.neighbours(pr.E), device=DEV),
                             metric=metric, jac=jac, gamma=pr.gamma, R=pr.R, mu=pr.mu, Pr=pr.Pr, eta=pr.eta))
        qs.append(q.reshape(-1))
    return probs, dps, torch.cat(qs), dts, host


def test_batch_sampled_against_oracle():
    require_gpu()
    rng = np.random.Generator(np.random.PCG64(44))
    sampled = [int(b) for b in rng.choice(256, 5, replace=False)]
    probs, dps, qd, dts, host = build_batch(oracle_for=sampled)
    ps = P.ProblemSet(dps)
    print(f"batch: {len(probs)} problems, {ps.total_nodes} nodes", flush=True)
    out = ps.residual(qd).cpu().numpy()
    assert ps.status() == 0
    offs = np.concatenate([[0], np.cumsum([5 * d.nodes for d in dps])])
    for b in sampled:
        pr = probs[b]
        sbp, xo = host[b]
        q = qd[offs[b]:offs[b + 1]].cpu().numpy().reshape(5, pr.K, pr.N, pr.N, pr.N)
        sel = np.unique(np.concatenate([[0, pr.K - 1], rng.integers(0, pr.K, 4)]))
        metric = dps[b].metric.cpu().numpy().reshape((9,) + q.shape[1:])
        jac = dps[b].jac.cpu().numpy().reshape(q.shape[1:])
        ref = R.residual(q, metric, jac, W.neighbours(pr.E), sbp, R.Params.of(pr), elems=sel)
        got = out[offs[b]:offs[b + 1]].reshape(q.shape)[:, sel]
        err = rel_err(got, ref)
        print(f"  problem {b}: p={pr.p} E={pr.E} err {err:.2e}")
        assert err < TOL


def test_batch_rk4_ten_steps_conserves_every_problem():
    require_gpu()
    probs, dps, qd, dts, _ = build_batch()
    ps = P.ProblemSet(dps)
    offs = np.concatenate([[0], np.cumsum([5 * d.nodes for d in dps])])

    def totals(q):
        out = []
        for b, (pr, d) in enumerate(zip(probs, dps)):
            w = torch.as_tensor(P.lgl_operator(pr.p)[1], device=DEV)
            w3 = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)
            wj = (w3[None, :] * d.jac.reshape(pr.K, -1)).reshape(-1)
            qq = q[offs[b]:offs[b + 1]].reshape(5, -1)
            out.append(((qq * wj).sum(1), (qq.abs() * wj).sum(1)))
        return out

    before = totals(qd)
    ps.autotune(qd, reps=1)
    ps.rk_step(qd, torch.tensor(dts, dtype=torch.float64, device=DEV), 10)
    assert ps.status() == 0
    after = totals(qd)
    for (t0, s0), (t1, s1) in zip(before, after):
        assert torch.all((t1 - t0).abs() <= 1e-13 * s1)


def test_batch_rk4_ten_steps_matches_oracle_on_small_problems():
    """The whole batch advanced 10 RK4 steps in one graph-replayed call with the autotuned schedules;
    problems 8, 44, 36, 5 and 70 (p = 3, 4, 6, 8, 2 on 2^3 or 3^3 elements) are checked against ten
    oracle RK4 steps, increment by increment, to max(1e-12, 4 x the FP64 floor)."""
    require_gpu()
    picks = [8, 44, 36, 5, 70]
    probs, dps, qd, dts, host = build_batch(oracle_for=picks)
    ps = P.ProblemSet(dps)
    ps.autotune(qd, reps=1)
    q0 = qd.cpu().numpy()
    ps.rk_step(qd, torch.tensor(dts, dtype=torch.float64, device=DEV), 10)
    assert ps.status() == 0
    q10 = qd.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum([5 * d.nodes for d in dps])])
    LD = np.longdouble
    for b in picks:
        pr = probs[b]
        sbp, _ = host[b]
        shape = (5, pr.K, pr.N, pr.N, pr.N)
        metric = dps[b].metric.cpu().numpy().reshape((9,) + shape[1:])
        jac = dps[b].jac.cpu().numpy().reshape(shape[1:])
        nbr = W.neighbours(pr.E)
        prm = R.Params.of(pr)
        sbp_ld = operators.SBP1D(pr.p, LD)
        m_ld, j_ld = metric.astype(LD), jac.astype(LD)
        f = lambda y: R.residual(y, metric, jac, nbr, sbp, prm)  # noqa: E731
        f_ld = lambda y: R.residual(y, m_ld, j_ld, nbr, sbp_ld, prm)  # noqa: E731
        err, bar = rk4_increment_check(f, f_ld, q0[offs[b]:offs[b + 1]].reshape(shape), dts[b], 10,
                                       q10[offs[b]:offs[b + 1]].reshape(shape))
        print(f"  problem {b}: p={pr.p} E={pr.E} 10-step increment err {err:.2e} bar {bar:.1e}")
        assert err < bar
