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
