"""Shared test helpers: build a problem's oracle inputs from the seeded generators."""
import numpy as np
import torch

import workloads as W
from oracle import operators, geometry, residual as R


class Case:
    def __init__(self, prob, dtype=np.float64):
        self.prob = prob
        self.sbp = operators.SBP1D(prob.p, dtype)
        self.x = W.coords(prob, operators.SBP1D(prob.p).x).numpy().astype(dtype)
        self.metric = geometry.curl_metrics(self.x, self.sbp.D)
        self.jac = geometry.jacobian(self.x, self.sbp.D)
        self.nbr = W.neighbours(prob.E)
        self.q = W.state(prob, torch.as_tensor(self.x.astype(np.float64))).numpy().astype(dtype)
        self.prm = R.Params.of(prob)

    def residual(self, q=None, prm=None, elems=None, chunk=None):
        return R.residual(self.q if q is None else q, self.metric, self.jac, self.nbr, self.sbp,
                          self.prm if prm is None else prm, elems=elems, chunk=chunk)

    def weights3d(self):
        w = self.sbp.w
        return np.einsum("i,j,k->ijk", w, w, w)

    def jumped(self, seed=0, amp=0.5):
        """Density and pressure scaled node by node by exp(U[-amp, amp]) (workloads.jumped_state)."""
        return W.jumped_state(self.prob, torch.as_tensor(self.x.astype(np.float64)), seed, amp).numpy()

    def jumpy(self, amp=0.02, seed=0):
        """The state with independent per-node noise, so interface values jump."""
        rng = np.random.Generator(np.random.PCG64(seed))
        q = self.q.copy()
        q[0] *= 1.0 + amp * rng.uniform(-1, 1, q[0].shape)
        q[1:4] += amp * rng.uniform(-1, 1, q[1:4].shape)
        q[4] *= 1.0 + amp * rng.uniform(-1, 1, q[4].shape)
        return q


def rel_err(a, b):
    """max over components of |a_c - b_c|_inf / |b_c|_inf."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return max(float(np.abs(a[c] - b[c]).max() / max(np.abs(b[c]).max(), 1e-300)) for c in range(a.shape[0]))


def far_pair_fractions(q, nbr, gamma, u_min=1e-2):
    """Fractions of the line pairs and of the interface pairs (aligned periodic meshes) whose
    averaged rho and beta = rho / (2P) are taken between far-apart values: u = ((a-b)/(a+b))^2 >=
    u_min, where the kernels evaluate the logarithmic mean from logarithms instead of a series.
    Returns {"line_rho", "line_beta", "face_rho", "face_beta"}."""
    rho = q[0]
    P = (gamma - 1.0) * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho)
    beta = rho / (2.0 * P)
    N = rho.shape[-1]
    out = {}
    for name, v in (("rho", rho), ("beta", beta)):
        far = tot = 0
        for ax in (1, 2, 3):
            for a in range(N):
                for b in range(a + 1, N):
                    va, vb = np.take(v, a, axis=ax), np.take(v, b, axis=ax)
                    u = ((va - vb) / (va + vb)) ** 2
                    far += int((u >= u_min).sum())
                    tot += u.size
        out["line_" + name] = far / tot
        far = tot = 0
        for l in range(3):
            ax = 3 - l                        # axis of direction l in (K, i3, i2, i1)
            own = np.take(v, N - 1, axis=ax)  # + face
            par = np.take(v[nbr[:, 2 * l + 1]], 0, axis=ax)
            u = ((own - par) / (own + par)) ** 2
            far += int((u >= u_min).sum())
            tot += u.size
        out["face_" + name] = far / tot
    return out


def rk4_increment_check(f, f_ld, q0, dt, steps, got):
    """Error and bar of a GPU state `got` reached from q0 by `steps` classical RK4 steps of size dt.
    The increment got - q0 is compared with the oracle's increment evaluated in long double
    (f_ld: the oracle residual on long-double inputs); the bar is max(1e-12, 4 x the error of the
    same increment computed by the double oracle f), i.e. the FP64 rounding floor of the problem.
    Returns (err, bar)."""
    from oracle import residual as R_
    LD = np.longdouble
    qd, ql = q0.copy(), q0.astype(LD)
    for _ in range(steps):
        qd = R_.rk4_step(f, qd, dt)
        ql = R_.rk4_step(f_ld, ql, LD(dt))
    inc_ld = (ql - q0.astype(LD)).astype(np.float64)
    floor = rel_err(qd - q0, inc_ld)
    err = rel_err(got - q0, inc_ld)
    return err, max(1e-12, 4.0 * floor)
