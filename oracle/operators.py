"""1-D diagonal-norm SBP operator on Legendre-Gauss-Lobatto nodes (Notation section, Definition "SBP").

The operator of degree p on N = p+1 LGL nodes in [-1, 1]:
  * nodes: -1, +1 and the roots of P_p' (derivative of the Legendre polynomial);
  * norm P = diag(w), w_i = 2 / (p (p+1) P_p(x_i)^2)  (LGL quadrature weights);
  * D = P^{-1} Q is the collocation derivative: D_ij = P_p(x_i) / (P_p(x_j) (x_i - x_j)), i != j,
    D_00 = -p(p+1)/4, D_pp = +p(p+1)/4, other diagonal entries zero;
  * Q = P D, E = diag(-1, 0, ..., 0, 1), S = Q - E/2 (skew-symmetric).
Roots are found by Newton's method in extended precision (numpy.longdouble).
"""
from __future__ import annotations

import numpy as np

LD = np.longdouble


def legendre(p: int, x):
    """P_p(x) and P_p'(x) by the three-term recurrence (x may be an array)."""
    x = np.asarray(x, dtype=LD)
    p0 = np.ones_like(x)
    if p == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for n in range(1, p):
        p0, p1 = p1, ((2 * n + 1) * x * p1 - n * p0) / (n + 1)
    # derivative from (x^2 - 1) P_p' = p (x P_p - P_{p-1}), valid for |x| < 1
    with np.errstate(divide="ignore", invalid="ignore"):
        dp = p * (x * p1 - p0) / (x * x - 1)
    return p1, dp


def lgl_nodes(p: int) -> np.ndarray:
    """LGL nodes in increasing order, extended precision."""
    if p < 1:
        raise ValueError("p >= 1")
    N = p + 1
    # Chebyshev-Gauss-Lobatto points as initial guesses for the interior roots of P_p'
    x = -np.cos(np.pi * np.arange(N, dtype=LD) / p).astype(LD)
    xi = x[1:-1].copy()
    for _ in range(100):
        P, dP = legendre(p, xi)
        # P_p'' from the Legendre equation (1-x^2) P'' - 2x P' + p(p+1) P = 0
        d2P = (2 * xi * dP - p * (p + 1) * P) / (1 - xi * xi)
        step = dP / d2P
        xi = xi - step
        if np.all(np.abs(step) < LD(1e-30)):
            break
    x[1:-1] = xi
    x[0], x[-1] = LD(-1), LD(1)
    return x


def lgl_weights(p: int, x=None) -> np.ndarray:
    if x is None:
        x = lgl_nodes(p)
    P, _ = legendre(p, x)
    return LD(2) / (p * (p + 1) * P * P)


def lgl_derivative(p: int, x=None) -> np.ndarray:
    if x is None:
        x = lgl_nodes(p)
    N = p + 1
    P, _ = legendre(p, x)
    D = np.zeros((N, N), dtype=LD)
    for i in range(N):
        for j in range(N):
            if i != j:
                D[i, j] = P[i] / (P[j] * (x[i] - x[j]))
    D[0, 0] = -LD(p * (p + 1)) / 4
    D[p, p] = LD(p * (p + 1)) / 4
    return D


class SBP1D:
    """The degree-p LGL SBP operator as float64 (and long double) matrices."""

    def __init__(self, p: int, dtype=np.float64):
        self.p = p
        self.N = p + 1
        x = lgl_nodes(p)
        self.x_ld = x
        self.w_ld = lgl_weights(p, x)
        self.D_ld = lgl_derivative(p, x)
        self.x = x.astype(dtype)
        self.w = self.w_ld.astype(dtype)
        self.D = self.D_ld.astype(dtype)
        self.P = np.diag(self.w)
        self.Q = self.P @ self.D
        self.E = np.zeros((self.N, self.N), dtype=dtype)
        self.E[0, 0], self.E[-1, -1] = -1, 1
        self.S = self.Q - 0.5 * self.E

    def astype(self, dtype):
        return SBP1D(self.p, dtype)
