"""GPU residual with the optimised metric terms (analytic surface metrics, volume metrics closest to
the analytic ones under the discrete GCL; built by the oracle from the closed-form mapping
derivative) against the oracle, on every kernel path; and, on the GPU output alone, uniform flow
preserved and entropy conserved with entropy-conservative interfaces."""
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
