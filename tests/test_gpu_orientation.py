"""GPU residual on unstructured meshes: every element turned by its own rotation of the cube, the
face table (neighbour face and orientation) found from the coordinates.  Parity with the oracle on
every kernel path (per-node faces N <= 5, face work items N = 6..8, plane passes N >= 10), with
walls, matrix dissipation and the SF-KG form; invariance against the aligned mesh at a larger size;
an RK4 step; and invalid table entries (the VJP on such meshes: test_gpu_vjp_boundaries)."""
import numpy as np
import pytest
import torch

import paper_1911_10966_amd as P
import workloads as W
from workloads import unstructured as U
from gpu_helpers import DEV, from_dev, require_gpu, to_dev
from helpers import rel_err, rk4_increment_check
from oracle import geometry, operators, residual as R

pytestmark = pytest.mark.gpu
TOL = 1e-12


class RotCase:
    def __init__(self, prob, seed, amp=0.02, periods=None, boundary=-1):
        self.prob = prob
        self.sbp = operators.SBP1D(prob.p)
        x = W.coords(prob, self.sbp.x).numpy()
        q = W.state(prob, torch.as_tensor(x)).numpy()
        rng = np.random.Generator(np.random.PCG64(seed))
        q[0] *= 1.0 + amp * rng.uniform(-1, 1, q[0].shape)
        q[1:4] += amp * rng.uniform(-1, 1, q[1:4].shape)
        q[4] *= 1.0 + amp * rng.uniform(-1, 1, q[4].shape)
        self.rots = rng.integers(0, 24, prob.K)
        self.x0, self.q0 = x, q
        self.x = U.rotate_elements(x, self.rots)
        self.q = U.rotate_elements(q, self.rots)
        self.metric = geometry.curl_metrics(self.x, self.sbp.D)
        self.jac = geometry.jacobian(self.x, self.sbp.D)
        self.nbr, self.orient = U.connectivity(self.x, prob.L, boundary=boundary, periods=periods)
        self.prm = R.Params.of(prob)

    def rhs(self, dtype=np.float64):
        """The oracle residual of this mesh as a function of the state, in `dtype` arithmetic."""
        m, j, sbp = self.metric.astype(dtype), self.jac.astype(dtype), operators.SBP1D(self.prob.p, dtype)
        return lambda y: R.residual(y, m, j, self.nbr, sbp, self.prm, orient=self.orient)

    def device(self, orient=True):
        pr = self.prob
        return P.Problem(p=pr.p, n_elem=pr.K, nbr=torch.as_tensor(self.nbr, device=DEV).contiguous(),
                         metric=to_dev(self.metric).reshape(9, -1), jac=to_dev(self.jac),
                         gamma=pr.gamma, R=pr.R, mu=pr.mu, Pr=pr.Pr, eta=pr.eta,
                         iface_diss=pr.iface_diss, two_point=pr.two_point,
                         face_orient=torch.as_tensor(self.orient, device=DEV).contiguous() if orient else None)


def _tol(c, ref):
    LD = np.longdouble
    ref_ld = R.residual(c.q.astype(LD), c.metric.astype(LD), c.jac.astype(LD), c.nbr,
                        operators.SBP1D(c.prob.p, LD), c.prm, orient=c.orient)
    return max(TOL, 4.0 * rel_err(ref, ref_ld))


CASES = [
    # p, E, mu, iface_diss, two_point, walls in x_2
    (2, 3, 0.0, 1, 0, False),
    (3, 2, 0.02, 1, 0, False),
    (4, 2, 0.02, 2, 0, False),
    (4, 2, 0.02, 1, 0, True),
    (5, 2, 0.01, 1, 2, False),
    (7, 2, 0.01, 1, 0, True),
    (6, 2, 0.0, 2, 0, False),
    (9, 2, 0.01, 1, 0, False),
    (10, 2, 0.0, 1, 0, True),
    (11, 2, 0.01, 2, 0, False),
]


@pytest.mark.parametrize("p,E,mu,diss,tp,walls", CASES)
def test_rotated_mesh_residual_matches_oracle(p, E, mu, diss, tp, walls):
    require_gpu()
    print(f"case p={p} E={E} mu={mu} diss={diss} two_point={tp} walls={walls}", flush=True)
    prob = W.make_problem(p=p, E=E, L=2.0, A=0.1, mu=mu, iface_diss=diss, two_point=tp, seed=4,
                          u_rms=0.3)
    c = RotCase(prob, seed=p + 10 * E, periods=(2.0, None, 2.0) if walls else None, boundary=-3)
    assert (c.orient // 8).max() > 0
    ref = R.residual(c.q, c.metric, c.jac, c.nbr, c.sbp, c.prm, orient=c.orient)
    ps = P.ProblemSet([c.device()])
    out = from_dev(ps.residual(to_dev(c.q)), c.q.shape)
    assert ps.status() == 0
    assert rel_err(out, ref) < _tol(c, ref)


@pytest.mark.parametrize("p,E", [(4, 10), (7, 6)])
def test_rotated_mesh_is_the_aligned_mesh_relabelled_at_size(p, E):
    require_gpu()
    prob = W.make_problem(p=p, E=E, L=2.0, A=0.1, mu=1e-3, seed=7, u_rms=0.3)
    c = RotCase(prob, seed=p)
    ps = P.ProblemSet([c.device()])
    out = from_dev(ps.residual(to_dev(c.q)), c.q.shape)
    assert ps.status() == 0
    m0, j0 = geometry.curl_metrics(c.x0, c.sbp.D), geometry.jacobian(c.x0, c.sbp.D)
    ps0 = P.ProblemSet([P.Problem(p=p, n_elem=prob.K, nbr=torch.as_tensor(W.neighbours(E), device=DEV),
                                  metric=to_dev(m0).reshape(9, -1), jac=to_dev(j0), gamma=prob.gamma,
                                  R=prob.R, mu=prob.mu, Pr=prob.Pr, eta=prob.eta)])
    out0 = from_dev(ps0.residual(to_dev(c.q0)), c.q0.shape)
    rot0 = U.rotate_elements(out0, c.rots)
    # the metrics of the two meshes differ by rounding: the oracle's own difference between the
    # two meshes, over every element, is the floor of the comparison
    prm = R.Params.of(prob)
    o1 = R.residual(c.q, c.metric, c.jac, c.nbr, c.sbp, prm, orient=c.orient)
    o0 = R.residual(c.q0, m0, j0, W.neighbours(E), c.sbp, prm)
    rot_o0 = U.rotate_elements(o0, c.rots)
    floor = rel_err(o1, rot_o0)
    err = rel_err(out, rot0)
    print(f"  rotated vs aligned relabelled: gpu {err:.2e}, oracle floor {floor:.2e}")
    assert err < max(TOL, 4 * floor)
    # and the rotated mesh against the oracle on sampled elements, to the FP64 floor
    rng = np.random.Generator(np.random.PCG64(p))
    el = np.sort(rng.choice(prob.K, size=16, replace=False))
    LD = np.longdouble
    o1_ld = R.residual(c.q.astype(LD), c.metric.astype(LD), c.jac.astype(LD), c.nbr,
                       operators.SBP1D(p, LD), prm, elems=el, orient=c.orient)
    assert rel_err(out[:, el], o1[:, el]) < max(TOL, 4 * rel_err(o1[:, el], o1_ld))


def test_rotated_mesh_rk4_step():
    require_gpu()
    prob = W.make_problem(p=3, E=2, L=2.0, A=0.1, mu=0.01, seed=2, u_rms=0.3)
    c = RotCase(prob, seed=12)
    ps = P.ProblemSet([c.device()])
    qd = to_dev(c.q)
    ps.rk_step(qd, torch.tensor([2e-3], dtype=torch.float64, device=DEV), 1)
    assert ps.status() == 0
    out = from_dev(qd, c.q.shape)
    err, bar = rk4_increment_check(c.rhs(), c.rhs(np.longdouble), c.q, 2e-3, 1, out)
    print(f"  rotated RK4 increment err {err:.2e} bar {bar:.1e}")
    assert err < bar


def test_invalid_orientation_entry_is_a_mesh_error():
    require_gpu()
    c = RotCase(W.make_problem(p=2, E=2, L=2.0, A=0.1, mu=0.01, seed=1, u_rms=0.3), seed=1)
    c.orient = c.orient.copy()
    c.orient[3, 2] = 6 + 8 * 1      # face index 6 does not exist
    ps = P.ProblemSet([c.device()])
    ps.residual(to_dev(c.q))
    with pytest.raises(P.SBPError):
        ps.status()


def test_batch_of_rotated_and_aligned_problems():
    """A rotated and an aligned problem of the same degree in one set (two launch groups), one
    residual and one RK4 step, each against its own oracle."""
    require_gpu()
    from helpers import Case
    from gpu_helpers import device_problem
    pr = W.make_problem(p=3, E=2, L=2.0, A=0.1, mu=0.01, seed=5, u_rms=0.3)
    cr = RotCase(pr, seed=9)
    ca = Case(W.make_problem(p=3, E=2, L=2.0, A=0.1, mu=0.01, seed=6, u_rms=0.3))
    ps = P.ProblemSet([cr.device(), device_problem(ca)])
    qa = ca.jumpy(0.01, 2)
    q = torch.cat([to_dev(cr.q), to_dev(qa)])
    out = ps.residual(q).cpu().numpy()
    assert ps.status() == 0
    n = cr.q.size
    ref_r = R.residual(cr.q, cr.metric, cr.jac, cr.nbr, cr.sbp, cr.prm, orient=cr.orient)
    assert rel_err(out[:n].reshape(cr.q.shape), ref_r) < _tol(cr, ref_r)
    assert rel_err(out[n:].reshape(qa.shape), ca.residual(qa)) < 1e-12
    ps.rk_step(q, torch.tensor([2e-3, 2e-3], dtype=torch.float64, device=DEV), 1)
    assert ps.status() == 0
    q1 = q.cpu().numpy()
    err, bar = rk4_increment_check(cr.rhs(), cr.rhs(np.longdouble), cr.q, 2e-3, 1, q1[:n].reshape(cr.q.shape))
    assert err < bar
    LD = np.longdouble
    m_ld, j_ld, s_ld = ca.metric.astype(LD), ca.jac.astype(LD), operators.SBP1D(ca.prob.p, LD)
    f_ld = lambda y: R.residual(y, m_ld, j_ld, ca.nbr, s_ld, ca.prm)  # noqa: E731
    err, bar = rk4_increment_check(ca.residual, f_ld, qa, 2e-3, 1, q1[n:].reshape(qa.shape))
    assert err < bar
