"""Directional derivatives of the oracle residual by the complex step (Squire and Trapp, 1998):
J v = Im f(q + i h v) / h with h = 1e-30, free of subtractive cancellation."""
from __future__ import annotations

import numpy as np

from .residual import residual


def jvp(q, v, metric, jac, nbr, sbp, prm, elems=None, h=1e-30, chunk=None, ctype=np.complex128,
        **kw):
    """J v by the complex step; ``ctype`` = numpy.clongdouble evaluates it in extended precision
    (then ``metric``, ``jac`` and ``sbp`` should be long double too).  ``kw`` (boundary data,
    orientation table) goes to the residual; boundary data is not perturbed."""
    real = np.longdouble if ctype == np.clongdouble else np.float64
    qc = q.astype(ctype) + 1j * real(h) * v.astype(real)
    return residual(qc, metric, jac, nbr, sbp, prm, elems=elems, chunk=chunk, **kw).imag / real(h)


def full_jacobian(q, metric, jac, nbr, sbp, prm, h=1e-30, ctype=np.complex128, **kw):
    """Dense Jacobian d(dq/dt)/dq of a tiny problem, one complex-step column per input entry."""
    n = q.size
    cols = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        cols.append(jvp(q, e.reshape(q.shape), metric, jac, nbr, sbp, prm, h=h, ctype=ctype,
                        **kw).ravel())
    return np.stack(cols, axis=1)
