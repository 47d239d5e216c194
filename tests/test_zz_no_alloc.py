"""The allocation-free residual (sbp_residual_noalloc, library-owned scratch) against the workspace
residual (sbp_residual) through the C ABI: two calls in a row, the second with a smaller input, on
viscous problems (face traces in the scratch), a plane-pass problem (per-node scratch) and an
inviscid one; the caller's status word receives the flags."""
import numpy as np
import pytest
import torch

import paper_1911_10966_amd as P
import workloads as W
from gpu_helpers import DEV, device_problem, require_gpu, to_dev
from helpers import Case, rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _set(specs):
    cases = [Case(W.make_problem(p=p, E=E, L=2.0, A=0.1, mu=mu, seed=500 + i, u_rms=0.3))
             for i, (p, E, mu) in enumerate(specs)]
    ps = P.ProblemSet([device_problem(c) for c in cases])
    q = torch.cat([to_dev(c.jumpy(0.02, i)) for i, c in enumerate(cases)])
    return cases, ps, q


def _compare(specs):
    cases, ps, q = _set(specs)
    ref = ps.residual(q).clone()
    assert ps.status() == 0
    out = torch.full_like(q, float("nan"))
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    P.lib()  # the C ABI directly, as a caller that cannot allocate would use it
    rc = P._lib.lib().sbp_residual_noalloc(ps._arr, ps.n, q.data_ptr(), out.data_ptr(), status.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    off = 0
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    for c in cases:
        n = c.q.size
        err = rel_err(a[off:off + n].reshape(c.q.shape), b[off:off + n].reshape(c.q.shape))
        print(f"  p={c.prob.p} E={c.prob.E} mu={c.prob.mu}: noalloc vs workspace residual {err:.2e}")
        assert err < TOL
        off += n
    print(f"  bitwise equal: {torch.equal(out, ref)}")


def test_noalloc_matches_workspace_residual_on_two_calls():
    require_gpu()
    # first call: p = 4 on 6^3 and p = 9 on 2^3 (plane passes) viscous, p = 2 inviscid
    _compare([(4, 6, 0.01), (9, 2, 0.01), (2, 3, 0.0)])
    # second call, smaller: one viscous p = 3 problem on 2^3 elements (the scratch keeps the first
    # call's contents)
    _compare([(3, 2, 0.02)])


def test_noalloc_flags_reach_the_callers_status_word():
    require_gpu()
    c = Case(W.make_problem(p=2, E=2, L=2.0, A=0.1, mu=0.01, seed=9, u_rms=0.3))
    ps = P.ProblemSet([device_problem(c)])
    q = c.q.copy()
    q[0, 1, 1, 1, 1] = -1.0
    out, status = ps.residual_noalloc(to_dev(q))
    torch.cuda.synchronize()
    assert int(status.item()) & 1
    out, status = ps.residual_noalloc(to_dev(c.q))
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(out, ps.residual(to_dev(c.q)))
    assert np.isfinite(out.cpu().numpy()).all()
