"""Hand-written vector-Jacobian product against the oracle: element by element against the full
complex-step Jacobian on small meshes, the dot-product identity gbar.(J v) = qbar.v with the
oracle's complex-step J v, central differences, and the autograd wrapper."""
import numpy as np
import pytest
import torch

import paper_1911_10966_amd as P
import workloads as W
from gpu_helpers import DEV, device_problem, from_dev, require_gpu, to_dev
from helpers import Case, rel_err
from oracle import jvp, operators, residual as R

pytestmark = pytest.mark.gpu
TOL = 1e-12


def gpu_vjp(c, q, gb):
    ps = P.ProblemSet([device_problem(c)])
    out = from_dev(ps.residual_vjp(to_dev(q), to_dev(gb)), q.shape)
    assert ps.status() == 0
    return out


@pytest.mark.parametrize("p,E,mu,diss,eta", [(1, 2, 0.0, 1, 1.0), (1, 2, 0.03, 1, 1.0), (2, 2, 0.02, 1, 1.0),
                                            (1, 3, 0.05, 0, 2.0)])
def test_vjp_matches_full_jacobian(p, E, mu, diss, eta):
    """J^T gbar from the complex-step Jacobian of the oracle evaluated in extended precision (the
    double-precision oracle Jacobian itself carries rounding errors of a few 1e-12 here)."""
    require_gpu()
    print(f"vjp full jacobian p={p} E={E} mu={mu}", flush=True)
    c = Case(W.make_problem(p=p, E=E, L=2.0, A=0.1, mu=mu, iface_diss=diss, eta=eta, seed=70 + p, u_rms=0.3))
    q = c.jumpy(0.03, 2)
    LD = np.longdouble
    Jm = jvp.full_jacobian(q, c.metric.astype(LD), c.jac.astype(LD), c.nbr, operators.SBP1D(p, LD),
                           c.prm, ctype=np.clongdouble)
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(2):
        gb = rng.standard_normal(q.shape)
        ref = (Jm.T @ gb.ravel().astype(LD)).reshape(q.shape).astype(np.float64)
        err = rel_err(gpu_vjp(c, q, gb), ref)
        print(f"  gpu vs extended-precision J^T gbar: {err:.2e}")
        assert err < TOL


@pytest.mark.parametrize("p,E,mu", [(3, 3, 0.02), (4, 2, 0.0), (5, 2, 0.01), (6, 2, 0.01), (7, 2, 0.02), (8, 2, 0.01)])
def test_vjp_dot_product_with_complex_step_jvp(p, E, mu):
    require_gpu()
    print(f"vjp dot p={p} E={E} mu={mu}", flush=True)
    c = Case(W.make_problem(p=p, E=E, L=2.0, A=0.12, mu=mu, seed=80 + p, u_rms=0.3))
    q = c.jumpy(0.02, 3)
    rng = np.random.Generator(np.random.PCG64(p))
    gb = rng.standard_normal(q.shape)
    v = W.direction(torch.as_tensor(q), 5).numpy()
    jv = jvp.jvp(q, v, c.metric, c.jac, c.nbr, c.sbp, c.prm)
    qb = gpu_vjp(c, q, gb)
    lhs, rhs = (gb * jv).sum(), (qb * v).sum()
    scale = np.abs(gb * jv).sum()
    assert abs(lhs - rhs) < TOL * scale


def test_vjp_central_difference():
    require_gpu()
    c = Case(W.make_problem(p=4, E=2, L=2.0, A=0.1, mu=0.02, seed=90, u_rms=0.3))
    q = c.jumpy(0.02, 4)
    rng = np.random.Generator(np.random.PCG64(9))
    gb = rng.standard_normal(q.shape)
    v = W.direction(torch.as_tensor(q), 6).numpy()
    ps = P.ProblemSet([device_problem(c)])
    h = 1e-6
    rp = from_dev(ps.residual(to_dev(q + h * v)), q.shape)
    rm = from_dev(ps.residual(to_dev(q - h * v)), q.shape)
    fd = (gb * (rp - rm)).sum() / (2 * h)
    qb = from_dev(ps.residual_vjp(to_dev(q), to_dev(gb)), q.shape)
    assert abs(fd - (qb * v).sum()) < 1e-6 * np.abs(gb * (rp - rm) / (2 * h)).sum()


def test_autograd_backward_uses_vjp():
    require_gpu()
    c = Case(W.make_problem(p=3, E=2, L=2.0, A=0.1, mu=0.02, seed=91, u_rms=0.3))
    q = c.jumpy(0.02, 5)
    ps = P.ProblemSet([device_problem(c)])
    qd = to_dev(q).requires_grad_(True)
    r = P.SBPResidual.apply(qd, ps)
    gb = torch.randn_like(r)
    (r * gb).sum().backward()
    direct = ps.residual_vjp(to_dev(q), gb.contiguous())
    assert torch.equal(qd.grad, direct)
    assert torch.equal(r.detach(), ps.residual(to_dev(q)))


def test_vjp_full_size_dot_product():
    """The adjoint workload (p = 4, 16^3 warped elements, Ma = 0.2, Re = 500) in its full launch:
    cotangent supported on sampled elements, J v from the oracle's complex step there."""
    require_gpu()
    from oracle import geometry, operators
    prob = W.config("vjp_p4_e16")
    sbp = operators.SBP1D(prob.p)
    x = W.coords(prob, sbp.x, device=DEV)
    qd = W.state(prob, x)
    xc = x.cpu().numpy()
    nbr = W.neighbours(prob.E)
    rng = np.random.Generator(np.random.PCG64(5))
    S = np.unique(rng.integers(0, prob.K, 6))
    ring = np.unique(np.concatenate([S, nbr[S].ravel(), nbr[nbr[S].ravel()].ravel()]))
    metric = geometry.curl_metrics(xc, sbp.D)
    jac = geometry.jacobian(xc, sbp.D)
    q = qd.cpu().numpy()
    gb = np.zeros_like(q)
    gb[:, S] = W.cotangent(prob, 5).numpy()[:, S]
    v = W.direction(torch.as_tensor(q), 6).numpy()
    jv = jvp.jvp(q, v, metric, jac, nbr, sbp, R.Params.of(prob), elems=S)
    dp = P.Problem(p=prob.p, n_elem=prob.K, nbr=torch.as_tensor(nbr, device=DEV),
                   metric=torch.as_tensor(metric.reshape(9, -1), device=DEV),
                   jac=torch.as_tensor(jac.reshape(-1), device=DEV), gamma=prob.gamma, R=prob.R,
                   mu=prob.mu, Pr=prob.Pr, eta=prob.eta)
    ps = P.ProblemSet([dp])
    qb = ps.residual_vjp(qd.reshape(-1).contiguous(), to_dev(gb)).cpu().numpy().reshape(q.shape)
    assert ps.status() == 0
    lhs = (gb[:, S] * jv).sum()
    rhs = (qb * v).sum()
    scale = np.abs(gb[:, S] * jv).sum()
    print(f"full-size dot: {lhs:.15e} {rhs:.15e} rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) < TOL * scale
    # the cotangent reaches at most two element layers beyond its support
    outside = np.setdiff1d(np.arange(prob.K), ring)
    assert np.all(qb[:, outside] == 0.0)
