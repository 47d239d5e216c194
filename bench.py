#!/usr/bin/env python
"""Benchmark of the ES-C SBP-SAT residual path on one MI355X.

A step is one pass of the hot path over the Taylor-Green workload (compressible Navier-Stokes,
p = 4, 32^3 warped hexahedra, FP64): one residual evaluation plus one classical RK4 step (four
more residual evaluations and the stage updates).  The metric is node-residual evaluations per
second (one node's 5-component dq/dt, evaluated once), in millions.

Prints one JSON line.  The CPU baseline is the plain NumPy oracle, single-threaded, timed on a
bounded sample of elements of the same workload in a child process.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mdof-residual evals/s FP64 (plain vs batched vs VJP) at <=1e-12 rel err; % FP64 peak"
UNIT = "Mdof-residual evals/s"
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 64 FP64 FMA lanes/clk x 2 flop x 2.4 GHz


# ------------------------------------------------------------------------------------------
# Algorithmic work of the main residual kernel (per launch).
# Bytes: the compulsory 160 B per node (q 40 + metric 72 + J 8 read, dq/dt 40 written).  The face
# traces of the contravariant viscous flux that the kernel writes for its neighbours' SAT^V are an
# implementation choice and are reported separately, not counted as algorithmic.
# FP64: the oracle's own operations, counted by oracle/opcount.py (each +, -, *, /, sqrt, log is one
# operation; the branch not taken and structural zeros are not counted): per unordered volume pair
# (3 N^2 lines x N(N-1)/2 pairs per element) and for the rest of the residual per element.
# tests/test_oracle_opcount.py checks this table against the counter.
# ------------------------------------------------------------------------------------------
BYTES_NODE = 160
ORACLE_OPS = {  # (p, viscous): (operations per volume pair, operations of the rest per element)
    (3, False): (183, 29504),
    (4, True): (183, 249591),
    (4, False): (183, 46225),
    (7, True): (183, 828840),
}


def algorithmic_flops(p, K, viscous):
    """Oracle-counted FP64 operations of one residual, or None if the table has no entry."""
    ops = ORACLE_OPS.get((p, viscous))
    if ops is None:
        return None
    N = p + 1
    return K * (3 * N * N * N * (N - 1) // 2 * ops[0] + ops[1])


def algorithmic_bytes(p, K):
    return K * (p + 1) ** 3 * BYTES_NODE


def trace_bytes(p, K, viscous):
    """Face traces of the contravariant viscous flux written per launch (implementation-added)."""
    N = p + 1
    return K * 6 * N * N * 4 * 8 if viscous else 0


# rocprofv3 measurements of the main residual kernel on one workload, valid only for the kernel
# source they were taken on (sha256 of KERNEL_SOURCES); copied from profiles/ (the summary there
# gives the commands).  Per residual schedule index:
#   bytes:    HBM bytes per launch, FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB per dispatch x 1024; the
#             factors are those counters' readings for a plain 512 MiB device copy);
#   trace_ms: average duration from --kernel-trace --stats;
#   hw_flops: hardware FP64 operations per launch, (ADD + MUL + 2 FMA + TRANS) F64 x 64 lanes.
KERNEL_PROFILE = {
    "sha256": "07cc4c09914efe8e4fba15a57dcbc949f35359ac64a3cdf87ab237ab54b1568d",
    "workload": "ns_tgv_p4_e32",
    "bytes": {0: 1297725400, 1: 1291463624, 2: 1319203480, 3: 1238697688, 4: 1297378928,
              5: 1295309520, 6: 1258448944},
    "trace_ms": {0: 0.4249, 1: 0.4953, 2: 0.5811, 3: 0.5587, 4: 0.4349, 5: 0.4372, 6: 0.4275},
    "hw_flops": {0: 10234101760, 1: 10234101760, 2: 10221912064, 3: 10221912064, 4: 10234101760,
                 5: 10234101760, 6: 10234101760},
}
KERNEL_SOURCES = ("paper_1911_10966_amd/csrc/sbp_kernels.hip", "paper_1911_10966_amd/csrc/sbp_device.h")


def kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profiled(workload, key, schedule):
    if KERNEL_PROFILE["sha256"] != kernel_sha() or workload != KERNEL_PROFILE["workload"]:
        return None
    return KERNEL_PROFILE[key].get(schedule)


def traffic_for_current_kernel(workload, schedule):
    return _profiled(workload, "bytes", schedule)


def trace_ms_for_current_kernel(workload, schedule):
    return _profiled(workload, "trace_ms", schedule)


def hw_flops_for_current_kernel(workload, schedule):
    return _profiled(workload, "hw_flops", schedule)


# ------------------------------------------------------------------------------------------
_CPU = {}


def _oracle_chunk(elems):
    from oracle import residual as R
    c = _CPU
    R.residual(c["q"], c["metric"], c["jac"], c["nbr"], c["sbp"], c["prm"], elems=elems, chunk=1024)
    return len(elems)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(workload: str, n_sample: int, workers: int):
    """The plain NumPy oracle on the first `n_sample` elements of the workload (all by default), as
    `workers` contiguous blocks evaluated by forked processes of one thread each; one block is
    first evaluated alone on one process (the single-core figure)."""
    import multiprocessing
    import numpy as np
    import torch

    import workloads as W
    from oracle import geometry, operators, residual as R

    prob = W.config(workload)
    sbp = operators.SBP1D(prob.p)
    x = W.coords(prob, sbp.x).numpy()
    q = W.state(prob, torch.as_tensor(x)).numpy()
    nbr = W.neighbours(prob.E)
    n_sample = min(n_sample, prob.K)
    S = np.arange(n_sample)
    ring = np.unique(np.concatenate([S, nbr[S].ravel(), nbr[nbr[S].ravel()].ravel()]))
    metric = np.zeros((9,) + x.shape[1:])
    jac = np.ones(x.shape[1:])
    metric[:, ring] = geometry.curl_metrics(x[:, ring], sbp.D)
    jac[ring] = geometry.jacobian(x[:, ring], sbp.D)
    _CPU.update(q=q, metric=metric, jac=jac, nbr=nbr, sbp=sbp, prm=R.Params.of(prob))
    N3 = prob.N ** 3
    blocks = [b for b in np.array_split(S, workers) if len(b)]
    t0 = time.perf_counter()
    _oracle_chunk(blocks[0])
    t1 = time.perf_counter() - t0
    with multiprocessing.get_context("fork").Pool(len(blocks)) as pool:
        pool.map(_oracle_chunk, [b[:1] for b in blocks])   # workers started and warm
        t0 = time.perf_counter()
        pool.map(_oracle_chunk, blocks, chunksize=1)
        tw = time.perf_counter() - t0
    print(json.dumps({"value": n_sample * N3 / tw / 1e6, "seconds": tw, "elems": int(n_sample),
                      "nodes": int(n_sample * N3), "workers": len(blocks),
                      "single_value": len(blocks[0]) * N3 / t1 / 1e6, "single_seconds": t1,
                      "single_elems": int(len(blocks[0]))}))


def run_cpu_baseline(workload: str, n_sample: int):
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = os.cpu_count() or 1
    workers = max(1, min(16, avail))
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    env["CUDA_VISIBLE_DEVICES"] = ""
    env["HIP_VISIBLE_DEVICES"] = ""
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", "--workload", workload,
           "--cpu-sample", str(n_sample), "--cpu-workers", str(workers)]
    res = subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=ROOT)
    if res.returncode != 0:
        sys.stderr.write(res.stderr)
        return None
    out = json.loads(res.stdout.strip().splitlines()[-1])
    out["nproc"] = os.cpu_count()
    out["cpu_model"] = cpu_model()
    return out


# ------------------------------------------------------------------------------------------
# Device setup and the secondary measurements (plain residual per workload, batched RK4, VJP)
# ------------------------------------------------------------------------------------------
def device_problem(P, W, prob, dev):
    import torch
    x1d, _, _ = P.lgl_operator(prob.p)
    coords = W.coords(prob, x1d, device=dev)
    metric, jac = P.metrics(prob.p, coords.reshape(3, -1).contiguous())
    q = W.state(prob, coords).reshape(-1).contiguous()
    dt = W.cfl_dt(prob, coords)
    dp = P.Problem(p=prob.p, n_elem=prob.K, nbr=torch.as_tensor(W.problem_neighbours(prob), device=dev),
                   metric=metric, jac=jac, gamma=prob.gamma, R=prob.R, mu=prob.mu, Pr=prob.Pr,
                   eta=prob.eta, iface_diss=prob.iface_diss, two_point=prob.two_point)
    return dp, q, dt


def timed(fn, reps, warm=2):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(torch.cuda.current_stream())
    for _ in range(reps):
        fn()
    e1.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def plain_rate(P, W, name, dev, reps):
    import torch
    prob = W.config(name)
    dp, q, _ = device_problem(P, W, prob, dev)
    ps = P.ProblemSet([dp])
    ps.autotune(q, reps=2)
    out = torch.empty_like(q)
    ms = timed(lambda: ps.residual(q, out), reps)
    ps.status()
    return {"Mdof_res_per_s": round(prob.n_nodes / (ms * 1e-3) / 1e6, 1), "ms": round(ms, 4),
            "nodes": prob.n_nodes, "p": prob.p}


def vjp_rate(P, W, dev, reps, iface_diss=None):
    """VJP and residual of the adjoint workload (p = 4, 16^3 elements); ``iface_diss`` replaces
    its interface dissipation (2: matrix dissipation)."""
    import dataclasses
    import torch
    prob = W.config("vjp_p4_e16")
    if iface_diss is not None:
        prob = dataclasses.replace(prob, iface_diss=iface_diss)
    dp, q, _ = device_problem(P, W, prob, dev)
    ps = P.ProblemSet([dp])
    ps.autotune(q, reps=2)
    gb = W.cotangent(prob, 5, device=dev).reshape(-1).contiguous()
    out = torch.empty_like(q)
    ms_r = timed(lambda: ps.residual(q, out), reps)
    ms_v = timed(lambda: ps.residual_vjp(q, gb, out), reps)
    ps.status()
    # algorithmic HBM bytes of a VJP: q, gbar, metrics and J read, qbar written (200 B per node)
    vjp_bytes = prob.n_nodes * (BYTES_NODE + 40)
    return {"Mdof_vjp_per_s": round(prob.n_nodes / (ms_v * 1e-3) / 1e6, 1), "ms": round(ms_v, 4),
            "residual_ms": round(ms_r, 4), "vjp_over_residual_cost": round(ms_v / ms_r, 3),
            "nodes": prob.n_nodes,
            "hbm_GBps_algorithmic": round(vjp_bytes / (ms_v * 1e-3) / 1e9, 1),
            "hbm_frac": round(vjp_bytes / (ms_v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def mesh_variants_rate(P, W, dev, reps, E=16):
    """The Taylor-Green problem (p = 4) on E^3 elements with every element turned by a random
    rotation of the cube (unstructured faces: neighbour face and orientation table), against the
    same mesh aligned with the default and the autotuned schedule; and the wall-bounded channel
    (adiabatic no-slip walls on two faces) of the same size."""
    import dataclasses
    import numpy as np
    import torch
    from workloads import unstructured as U
    prob = dataclasses.replace(W.config("ns_tgv_p4_e32"), E=E, name=f"ns_tgv_p4_e{E}")
    out_n = lambda ms: round(prob.n_nodes / (ms * 1e-3) / 1e6, 1)  # noqa: E731
    x1d, _, _ = P.lgl_operator(prob.p)
    x = W.coords(prob, x1d).numpy()
    q0 = W.state(prob, torch.as_tensor(x)).numpy()
    rots = np.random.Generator(np.random.PCG64(17)).integers(0, 24, prob.K)
    xr = U.rotate_elements(x, rots)
    nbr, orient = U.connectivity(xr, prob.L)
    metric, jac = P.metrics(prob.p, torch.as_tensor(xr.reshape(3, -1), device=dev).contiguous())
    q = torch.as_tensor(U.rotate_elements(q0, rots).reshape(-1), device=dev).contiguous()
    dp = P.Problem(p=prob.p, n_elem=prob.K, nbr=torch.as_tensor(nbr, device=dev), metric=metric, jac=jac,
                   gamma=prob.gamma, R=prob.R, mu=prob.mu, Pr=prob.Pr, eta=prob.eta,
                   face_orient=torch.as_tensor(orient, device=dev))
    ps = P.ProblemSet([dp])
    out = torch.empty_like(q)
    ms_rot = timed(lambda: ps.residual(q, out), reps)
    ps.status()
    dp0, qa, _ = device_problem(P, W, prob, dev)
    ps0 = P.ProblemSet([dp0])
    ps0.set_schedule(prob.p, 0)
    ms_al0 = timed(lambda: ps0.residual(qa, out), reps)
    ps0.autotune(qa, reps=2)
    ms_al = timed(lambda: ps0.residual(qa, out), reps)
    ps0.status()
    ch = W.channel_problem(prob.p, E, A=0.05)
    dpc, qc, _ = device_problem(P, W, ch, dev)
    psc = P.ProblemSet([dpc])
    psc.autotune(qc, reps=2)
    ms_ch = timed(lambda: psc.residual(qc, out), reps)
    psc.status()
    return {"unstructured": {"Mdof_res_per_s": out_n(ms_rot), "ms": round(ms_rot, 4),
                             "aligned_default_schedule_ms": round(ms_al0, 4),
                             "aligned_autotuned_ms": round(ms_al, 4), "nodes": prob.n_nodes,
                             "orientation_codes": len(set((orient // 8).ravel().tolist()))},
            "channel_adiabatic_walls": {"Mdof_res_per_s": out_n(ms_ch), "ms": round(ms_ch, 4),
                                        "nodes": ch.n_nodes}}


def batched_rate(P, W, dev, steps, loop_baseline=True):
    """The heterogeneous batch, `steps` RK4 steps in one graph-replayed call, against advancing
    the same problems one problem at a time with the plain per-problem path."""
    import torch
    probs = W.batch_config()
    dps, qs, dts = [], [], []
    for pr in probs:
        dp, q, dt = device_problem(P, W, pr, dev)
        dps.append(dp)
        qs.append(q)
        dts.append(dt)
    q = torch.cat(qs)
    del qs
    ps = P.ProblemSet(dps)
    ps.autotune(q, reps=2)
    dtd = torch.tensor(dts, dtype=torch.float64, device=dev)
    nodes = ps.total_nodes
    q_work = q.clone()
    ms = timed(lambda: ps.rk_step(q_work, dtd, steps), 1, warm=1)
    ps.status()
    res = {"problems": len(probs), "nodes": nodes, "rk4_steps": steps, "ms": round(ms, 3),
           "Mdof_res_per_s": round(4 * steps * nodes / (ms * 1e-3) / 1e6, 1)}
    if loop_baseline:
        singles = [P.ProblemSet([d]) for d in dps]
        offs = [0]
        for d in dps:
            offs.append(offs[-1] + 5 * d.nodes)
        views = [q_work[offs[b]:offs[b + 1]] for b in range(len(dps))]
        dtv = [dtd[b:b + 1] for b in range(len(dps))]

        def loop():
            for b, s_ in enumerate(singles):
                s_.rk_step(views[b], dtv[b], steps)

        ms_loop = timed(loop, 1, warm=1)
        res["per_problem_loop_ms"] = round(ms_loop, 3)
        res["batched_speedup_vs_loop"] = round(ms_loop / ms, 2)
    return res


def cost_experiment(P, W, dev, steps):
    """The paper's cost-of-entropy-stability test on one MI355X: Taylor-Green vortex (Re = 1600,
    Ma = 0.05, periodic box of side 2 pi, Cartesian elements) at 256^3 DOFs for p = 1, 3, 7, 15 with the
    ES-C (Chandrashekar), SF-KG (Kennedy-Gruber) and DC volume terms; time per residual and per
    classical RK4 step.  The paper's figures (64 Haswell cores, DOPRI5 steps) are quoted as
    context."""
    import math
    import torch
    paper = {1: {"ES-C": 3.1798, "SF-KG": 2.8634, "DC": 2.7771},
             3: {"ES-C": 2.5059, "SF-KG": 2.01675, "DC": 1.9593},
             7: {"ES-C": 2.6099, "SF-KG": 1.73415, "DC": 1.5335},
             15: {"ES-C": 3.5589, "SF-KG": 1.9914, "DC": 1.4830}}
    out = {"dofs": 256 ** 3, "box": "2pi periodic, Cartesian", "Ma": 0.05, "Re": 1600, "results": []}
    for p in (1, 3, 7, 15):
        E = 256 // (p + 1)
        for name, tp in (("ES-C", 0), ("SF-KG", 2), ("DC", 3)):
            Ma = 0.05
            prob = W.make_problem(name=f"tgv_p{p}", p=p, E=E, L=2.0 * math.pi, A=0.0, gamma=1.4,
                                  R=1.0 / (1.4 * Ma * Ma), mu=1.0 / 1600.0, Pr=0.72, init="tgv",
                                  Ma=Ma, two_point=tp)
            dp, q, dt0 = device_problem(P, W, prob, dev)
            ps = P.ProblemSet([dp])
            sched = ps.autotune(q, reps=2)[0] if tp == 0 else 0
            out_t = torch.empty_like(q)
            ms_res = timed(lambda: ps.residual(q, out_t), 5)
            dt = torch.tensor([dt0], dtype=torch.float64, device=dev)
            ms_rk = timed(lambda: ps.rk_step(q, dt, steps), 1, warm=1) / steps
            ps.status()
            out["results"].append({"p": p, "elements": prob.K, "scheme": name, "schedule": sched,
                                   "ms_per_residual": round(ms_res, 3),
                                   "ms_per_rk4_step": round(ms_rk, 3),
                                   "Mdof_res_per_s": round(prob.n_nodes / (ms_res * 1e-3) / 1e6, 1),
                                   "paper_s_per_dopri5_step_64_haswell_cores": paper[p][name]})
            print(json.dumps(out["results"][-1]), file=sys.stderr, flush=True)
            del ps, dp, q, out_t
            torch.cuda.empty_cache()
    return out


def tgv_robustness(P, W, dev, meshes, degrees, t_final, cfl, budget_s, chunk=1000,
                   only=("ES-C", "SF-KG", "DC")):
    """The paper's robustness study of the Taylor-Green vortex (Re = 1600, Ma = 0.05, Cartesian
    periodic box of side 2 pi, t_f = 20): for each mesh of E^3 elements and degree p, the ES-C,
    SF-KG and DC discretizations are advanced together as one batched problem set (three graph
    branches) with classical RK4 under CFL control: every `chunk` steps the time step is set again
    to dt = cfl (L/E) / ((p+1)^2 max(|U| + c)) from the current states (the smallest over the
    schemes still running, so that they stay at one time), and the last steps are shortened to end
    at t_f.  A run has failed when its state holds a non-finite value or a non-positive density or
    pressure; failed runs leave the set.  Reports, per run, success or the time of failure and, for
    runs that reach t_f, the kinetic energy relative to its initial value.  `only` selects the
    schemes (a scheme run alone takes its time step from its own states)."""
    import math
    import torch
    Ma = 0.05
    gam = 1.4
    schemes = tuple(s for s in (("ES-C", 0), ("SF-KG", 2), ("DC", 3)) if s[0] in only)
    if not schemes:
        raise ValueError(f"no scheme selected from {only}")
    out = {"t_final": t_final, "cfl": cfl, "Ma": Ma, "Re": 1600,
           "integrator": f"classical RK4, dt from the current max(|U|+c) every {chunk} steps",
           "results": []}
    t_start = time.time()
    for E in meshes:
        for p in degrees:
            if time.time() - t_start > budget_s:
                for name, _ in schemes:
                    out["results"].append({"E": E, "p": p, "scheme": name, "result": "not run (time budget)"})
                continue
            probs = [W.make_problem(name=f"tgv_robust_p{p}_e{E}", p=p, E=E, L=2.0 * math.pi, A=0.0,
                                    gamma=gam, R=1.0 / (gam * Ma * Ma), mu=1.0 / 1600.0, Pr=0.72,
                                    init="tgv", Ma=Ma, two_point=tp) for _, tp in schemes]
            built = [device_problem(P, W, pr, dev) for pr in probs]
            h = probs[0].L / E
            _, w, _ = P.lgl_operator(p)
            wt = torch.as_tensor(w, dtype=torch.float64, device=dev)
            w3 = (wt[None, None, :, None, None] * wt[None, None, None, :, None] * wt[None, None, None, None, :])
            wJ = (w3.reshape(1, 1, -1) * built[0][0].jac.reshape(probs[0].K, -1)[None]).reshape(-1)

            def prim(qq):
                q5 = qq.reshape(5, -1)
                u2 = (q5[1] ** 2 + q5[2] ** 2 + q5[3] ** 2) / q5[0] ** 2
                return q5, u2, (gam - 1.0) * (q5[4] - 0.5 * q5[0] * u2)

            def kinetic(qq):
                q5, u2, _ = prim(qq)
                return float(((0.5 * q5[0] * u2) * wJ).sum() / wJ.sum())

            def healthy(qq):
                q5, _, pr_ = prim(qq)
                return bool(torch.isfinite(q5).all()) and bool((q5[0] > 0).all()) and bool((pr_ > 0).all())

            def speed_max(qq):
                q5, u2, pr_ = prim(qq)
                return float((torch.sqrt(u2) + torch.sqrt(gam * pr_ / q5[0])).max())

            qs = [b[1].reshape(-1).clone() for b in built]
            ek0 = kinetic(qs[0])
            alive = list(range(len(schemes)))
            fail = {}
            t = 0.0
            steps = 0
            dts = []
            t0 = time.time()
            ps, qcat, key = None, None, None
            while t < t_final * (1.0 - 1e-12) and alive:
                if key != tuple(alive):
                    key = tuple(alive)
                    ps = P.ProblemSet([built[i][0] for i in alive])
                    qcat = torch.cat([qs[i] for i in alive])
                dt = cfl * h / ((p + 1) ** 2 * max(speed_max(qs[i]) for i in alive))
                n = int(math.ceil((t_final - t) / dt))
                if n > chunk:
                    n = chunk
                else:
                    dt = (t_final - t) / n
                dts.append(dt)
                dtd = torch.full((len(alive),), dt, dtype=torch.float64, device=dev)
                ps.rk_step(qcat, dtd, n)
                try:
                    ps.status()
                except P.SBPError:
                    pass
                t += n * dt
                steps += n
                if steps % (10 * chunk) == 0:
                    print(f"robustness E={E} p={p}: t = {t:.3f}, {steps} steps", file=sys.stderr, flush=True)
                off = 0
                for i in list(alive):
                    m = qs[i].numel()
                    qs[i] = qcat[off:off + m]
                    off += m
                    if not healthy(qs[i]):
                        fail[i] = t
                for i in fail:
                    if i in alive:
                        alive.remove(i)
                        qs[i] = qs[i].clone()
            secs = time.time() - t0
            for i, (name, _) in enumerate(schemes):
                r = {"E": E, "p": p, "scheme": name, "steps": steps, "dt_min": min(dts), "dt_max": max(dts)}
                if i in fail:
                    r.update(result="failure", t_fail_before=round(fail[i], 4))
                else:
                    r.update(result="success", kinetic_energy_ratio=round(kinetic(qs[i]) / ek0, 5))
                out["results"].append(r)
            print(f"robustness E={E} p={p}: steps {steps}, {secs:.1f} s, failed "
                  f"{[schemes[i][0] for i in sorted(fail)]}", file=sys.stderr, flush=True)
            print(json.dumps({"tgv_robustness_run": out["results"][-len(schemes):]}), file=sys.stderr,
                  flush=True)
            del ps, qcat, built, qs
            torch.cuda.empty_cache()
    return out


def mms_error_vs_cost(P, W, dev, degrees, meshes_of, t_end, cfl, budget_s):
    """The paper's viscous error-vs-cost study (manufactured supersonic solution on the unit cube,
    Dirichlet data on every face, Re = 4e6, Ma = 2.14): for ES-C and DC and each degree and mesh,
    classical RK4 from the exact nodal state to t_end (several passages of the slowest wave through
    the cube), then the L2 error of the density against the exact solution, the GPU time of the
    time stepping and the remaining residual (how steady the end state is)."""
    import math
    import torch
    from workloads import mms
    out = {"t_end": t_end, "cfl": cfl, "Re": mms.RE, "Ma": round(800.0 / math.sqrt(1.4e5), 3),
           "integrator": "classical RK4, fixed dt", "results": []}
    smax = mms.speed_max()
    t_start = time.time()
    for p in degrees:
        for E in meshes_of(p):
            for name, tp in (("ES-C", 0), ("DC", 3)):
                if time.time() - t_start > budget_s:
                    out["results"].append({"p": p, "E": E, "scheme": name, "result": "not run (time budget)"})
                    continue
                prob = W.mms_problem(p, E, two_point=tp)
                x1d, w1d, _ = P.lgl_operator(p)
                x = W.coords(prob, x1d, device=dev)
                metric, jac = P.metrics(p, x.reshape(3, -1).contiguous())
                qex = torch.as_tensor(mms.conservative(x), device=dev).reshape(-1).contiguous()
                src = torch.as_tensor(mms.source(x), device=dev).reshape(-1).contiguous()
                dp = P.Problem(p=p, n_elem=prob.K,
                               nbr=torch.as_tensor(W.neighbours(E, periodic=False), device=dev),
                               metric=metric, jac=jac, gamma=prob.gamma, R=prob.R, mu=prob.mu,
                               Pr=prob.Pr, eta=prob.eta, iface_diss=1, two_point=tp,
                               bc_state=qex, source=src)
                ps = P.ProblemSet([dp])
                dt0 = cfl * (1.0 / E) / ((p + 1) ** 2 * smax)
                n = int(math.ceil(t_end / dt0))
                dt = torch.tensor([t_end / n], dtype=torch.float64, device=dev)
                q = qex.clone()
                ps.rk_step(q, dt, 1)
                torch.cuda.synchronize()
                q = qex.clone()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                ps.rk_step(q, dt, n)
                e1.record()
                torch.cuda.synchronize()
                secs = e0.elapsed_time(e1) / 1e3
                failed = False
                try:
                    ps.status()
                except P.SBPError:
                    failed = True
                w = torch.as_tensor(w1d, dtype=torch.float64, device=dev)
                w3 = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)
                wJ = (w3[None, :] * jac.reshape(prob.K, -1)).reshape(-1)
                q5, x5 = q.reshape(5, -1), qex.reshape(5, -1)
                err = float(torch.sqrt((wJ * (q5[0] - x5[0]) ** 2).sum() / wJ.sum()))
                r = ps.residual(q).reshape(5, -1)
                res = float(torch.sqrt((wJ * (r * r).sum(0)).sum() / (wJ * (src.reshape(5, -1) ** 2).sum(0)).sum()))
                out["results"].append({"p": p, "E": E, "scheme": name, "dofs": prob.n_nodes,
                                       "steps": n, "gpu_s": round(secs, 3),
                                       "result": "failure" if failed or not math.isfinite(err) else "ok",
                                       "l2_error_rho": err, "residual_rel": res})
                print(f"mms p={p} E={E} {name}: dofs {prob.n_nodes}, {n} steps, {secs:.2f} s, "
                      f"L2(rho) {err:.3e}, residual {res:.1e}", file=sys.stderr, flush=True)
                del ps, dp, q, qex, src, metric, jac
                torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ns_tgv_p4_e32")
    ap.add_argument("--cpu-sample", type=int, default=32768,
                    help="elements in the oracle sample run on all host cores (at most 16)")
    ap.add_argument("--cpu-workers", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--kernel-reps", type=int, default=0,
                    help="extra profiled residual launches after the timed region")
    ap.add_argument("--vjp", action="store_true",
                    help="only the VJP of the adjoint workload (Lax-Friedrichs and matrix dissipation)")
    ap.add_argument("--cost-experiment", action="store_true",
                    help="run only the ES-C / SF-KG / DC cost comparison at 256^3 DOFs and print it")
    ap.add_argument("--robustness", action="store_true",
                    help="run only the Taylor-Green robustness study (ES-C / SF-KG / DC to t = 20)")
    ap.add_argument("--robust-meshes", default="3", help="comma-separated E of the E^3 meshes")
    ap.add_argument("--robust-degrees", default="1-15", help="degrees, e.g. 1-15 or 1,3,7")
    ap.add_argument("--robust-t-final", type=float, default=20.0)
    ap.add_argument("--robust-cfl", type=float, default=0.5)
    ap.add_argument("--robust-budget", type=float, default=900.0, help="seconds before skipping runs")
    ap.add_argument("--robust-schemes", default="ES-C,SF-KG,DC",
                    help="comma-separated subset of ES-C, SF-KG, DC advanced together")
    ap.add_argument("--mms", action="store_true",
                    help="run only the manufactured-solution error-vs-cost study (ES-C / DC)")
    ap.add_argument("--mms-degrees", default="1,3,5,7")
    ap.add_argument("--mms-t-end", type=float, default=0.02)
    ap.add_argument("--mms-budget", type=float, default=600.0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the plain/batched/VJP secondary measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()

    if args.cpu_leg:
        cpu_leg(args.workload, args.cpu_sample, args.cpu_workers)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the library "
              "runs each problem set on a single GPU (a multi-GPU run would shard element blocks "
              "across GPUs and exchange face traces, which the library does not implement)",
              file=sys.stderr)
        return 2

    import torch

    import paper_1911_10966_amd as P
    import workloads as W

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.cost_experiment:
        print(json.dumps({"cost_of_entropy_stability": cost_experiment(P, W, dev, 5)}), flush=True)
        return 0
    if args.vjp:
        print(json.dumps({"vjp_p4_e16": vjp_rate(P, W, dev, 10),
                          "vjp_matrix_dissipation_p4_e16": vjp_rate(P, W, dev, 10, iface_diss=2)}),
              flush=True)
        return 0
    if args.mms:
        meshes = {1: (4, 8, 16, 32, 64), 2: (2, 4, 8, 16, 32), 3: (2, 4, 8, 16), 4: (2, 4, 8, 16),
                  5: (2, 4, 8), 6: (2, 4, 8), 7: (2, 4, 8)}
        res = mms_error_vs_cost(P, W, dev, [int(v) for v in args.mms_degrees.split(",")],
                                lambda p: meshes.get(p, (2, 4)), args.mms_t_end, 0.5, args.mms_budget)
        print(json.dumps({"mms_error_vs_cost": res}), flush=True)
        return 0
    if args.robustness:
        def int_list(spec):
            vals = []
            for part in spec.split(","):
                a, _, b = part.partition("-")
                vals += list(range(int(a), int(b) + 1)) if b else [int(a)]
            return vals
        res = tgv_robustness(P, W, dev, int_list(args.robust_meshes), int_list(args.robust_degrees),
                             args.robust_t_final, args.robust_cfl, args.robust_budget,
                             only=tuple(args.robust_schemes.split(",")))
        print(json.dumps({"tgv_robustness": res}), flush=True)
        return 0
    prob = W.config(args.workload)
    dp, q, dt0 = device_problem(P, W, prob, dev)
    dt = torch.tensor([dt0], dtype=torch.float64, device=dev)
    ps = P.ProblemSet([dp])
    schedule = ps.autotune(q, reps=3)[0]
    out = torch.empty_like(q)

    def step(record):
        if record:
            # events around the main residual kernel on its launch stream, read after the loop
            ps.profile_residual(q, out, wait=False)
        else:
            ps.residual(q, out)
        ps.rk_step(q, dt, 1)

    for _ in range(args.warmup):
        step(False)
    ps.status()
    P.profile_collect()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step(True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    n_live, live_total = P.profile_collect()
    ps.status()
    ms_step = ms_total / args.steps
    res_per_step = 5
    node_res = res_per_step * prob.n_nodes
    value = node_res * args.steps / (ms_total * 1e-3) / 1e6

    # dominant kernel: the fused residual kernel, timed with events on its launch stream in every
    # timed step (plus optional extra launches after the timed region)
    for _ in range(args.kernel_reps):
        ps.profile_residual(q, out, wait=False)
    n_extra, extra_total = P.profile_collect()
    kmean = (live_total + extra_total) / (n_live + n_extra)
    visc = prob.mu > 0
    flops = algorithmic_flops(prob.p, prob.K, visc)
    nbytes = algorithmic_bytes(prob.p, prob.K)
    hbm = nbytes / (kmean * 1e-3) / 1e9
    alu = flops / (kmean * 1e-3) / 1e12 if flops is not None else None
    if alu is not None and alu / FP64_VALU_PEAK_TFLOPS >= hbm / HBM_PEAK_GBS:
        roof = {"bound": "alu", "achieved": round(alu, 3), "peak": FP64_VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(alu / FP64_VALU_PEAK_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm / HBM_PEAK_GBS, 4)}
    roof["traffic"] = traffic_for_current_kernel(args.workload, schedule)
    roof["schedule"] = schedule
    roof["kernel"] = "k_residual"
    roof["kernel_ms"] = round(kmean, 4)
    roof["kernel_launches_timed"] = n_live + n_extra
    roof["kernel_ms_trace"] = trace_ms_for_current_kernel(args.workload, schedule)
    roof["bytes_algorithmic"] = nbytes
    roof["bytes_implementation_added"] = trace_bytes(prob.p, prob.K, visc)
    roof["hbm_GBps_algorithmic"] = round(hbm, 1)
    roof["hbm_frac"] = round(hbm / HBM_PEAK_GBS, 4)
    roof["fp64_ops_oracle_count"] = flops
    roof["fp64_TFLOPs_algorithmic"] = round(alu, 3) if alu is not None else None
    roof["fp64_frac"] = round(alu / FP64_VALU_PEAK_TFLOPS, 4) if alu is not None else None
    roof["fp64_hw_flops"] = hw_flops_for_current_kernel(args.workload, schedule)

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    extra = None
    if not args.no_extra:
        extra = {
            "schedule_variant": schedule,
            "plain_euler_p3_e4": plain_rate(P, W, "euler_p3_e4", dev, 50),
            "plain_ns_tgv_p4_e32": plain_rate(P, W, "ns_tgv_p4_e32", dev, 10),
            "plain_ns_p7_e16": plain_rate(P, W, "ns_p7_e16", dev, 10),
            "vjp_p4_e16": vjp_rate(P, W, dev, 10),
            "vjp_matrix_dissipation_p4_e16": vjp_rate(P, W, dev, 10, iface_diss=2),
            "batched_256_rk4x10": batched_rate(P, W, dev, 10),
        }
        extra.update({k + "_p4_e16": v for k, v in mesh_variants_rate(P, W, dev, 10).items()})

    cpu = None
    if not args.no_cpu_baseline:
        r = run_cpu_baseline(args.workload, args.cpu_sample)
        if r is not None:
            which = (f"all {r['elems']} elements" if r["elems"] >= prob.K
                     else f"{r['elems']} randomly chosen elements")
            cpu = {"value": round(r["value"], 4), "unit": UNIT, "cores": r["workers"], "kind": "oracle",
                   "sample": f"one residual of {which} ({r['nodes']} nodes) of {args.workload} split "
                             f"into {r['workers']} contiguous blocks on as many processes of one "
                             f"thread, {r['seconds']:.1f} s; one block ({r['single_elems']} elements) "
                             f"alone on one process: {r['single_seconds']:.1f} s",
                   "single_core_value": round(r["single_value"], 4),
                   "nproc": r["nproc"], "cpu_model": r["cpu_model"]}

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "p": prob.p, "elements": prob.K,
                   "nodes": prob.n_nodes, "step": "1 residual + 1 RK4 step (5 residual evaluations)",
                   "Re": prob.Re, "Ma": prob.Ma, "parallelism": "none (1 GPU)"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "sub": extra,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
