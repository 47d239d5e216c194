"""Helpers of the GPU tests: device problems built from the same seeded inputs the oracle sees."""
import numpy as np
import torch

import paper_1911_10966_amd as P
from helpers import Case

DEV = "cuda:0"


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    P.lib()


def device_problem(case: Case, metric=None, jac=None):
    prob = case.prob
    m = case.metric if metric is None else metric
    j = case.jac if jac is None else jac
    return P.Problem(p=prob.p, n_elem=prob.K,
                     nbr=torch.as_tensor(case.nbr, device=DEV).contiguous(),
                     metric=torch.as_tensor(np.ascontiguousarray(m.reshape(9, -1)), device=DEV),
                     jac=torch.as_tensor(np.ascontiguousarray(j.reshape(-1)), device=DEV),
                     gamma=prob.gamma, R=prob.R, mu=prob.mu, Pr=prob.Pr, eta=prob.eta,
                     iface_diss=prob.iface_diss, two_point=prob.two_point)


def to_dev(q):
    return torch.as_tensor(np.ascontiguousarray(q.reshape(-1)), device=DEV)


def from_dev(t, shape):
    return t.detach().cpu().numpy().reshape(shape)
