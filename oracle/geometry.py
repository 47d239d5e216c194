"""Metric terms J*dxi_l/dx_m and the Jacobian J on curvilinear hexahedra.

The paper stores the metric terms as diagonal matrices [A_lm] (linear convection-diffusion
section) and requires the discrete geometric conservation law sum_l D_l [A_lm] 1 = 0
(eq. discGCLconvection). Its own metrics come from an optimisation procedure published
elsewhere; this oracle uses the conservative curl form instead (Kopriva, J. Sci. Comput. 26,
2006), which satisfies that discrete law exactly because tensor-product derivative
operators commute:

    J dxi_i/dx_n = -[ curl_xi ( X_l grad_xi X_m ) ]_i,   (n, m, l) cyclic,

with every xi-derivative taken by the collocation derivative D on nodal values.
J = det(dx/dxi) with dx_m/dxi_i = D_i X_m.
"""
from __future__ import annotations

import numpy as np


def apply_D(D, u, l):
    """Apply the 1-D matrix D along direction xi_l of element arrays u[..., e, i3, i2, i1]."""
    ax = u.ndim - 1 - l
    moved = np.moveaxis(u, ax, 0)
    out = np.tensordot(D, moved, axes=(1, 0))
    return np.moveaxis(out, 0, ax)


def jacobian_matrix(x, D):
    """dx_m/dxi_i as an array [m][i] of nodal arrays."""
    return [[apply_D(D, x[m], i) for i in range(3)] for m in range(3)]


def jacobian(x, D):
    a = jacobian_matrix(x, D)
    return (a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1])
            - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
            + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]))


def curl_metrics(x, D):
    """Metric terms, shape (9, K, N, N, N); entry 3*l + m is J dxi_l/dx_m."""
    A = [[None] * 3 for _ in range(3)]
    for n in range(3):
        m, l = (n + 1) % 3, (n + 2) % 3
        V = [x[l] * apply_D(D, x[m], i) for i in range(3)]
        curl = [apply_D(D, V[2], 1) - apply_D(D, V[1], 2),
                apply_D(D, V[0], 2) - apply_D(D, V[2], 0),
                apply_D(D, V[1], 0) - apply_D(D, V[0], 1)]
        for i in range(3):
            A[i][n] = -curl[i]
    return np.stack([A[l][m] for l in range(3) for m in range(3)])


def gcl_residual(metric, D):
    """sum_l D_l [A_lm] 1 for m = 1..3 (eq. discGCLconvection); zero for exact metrics."""
    return np.stack([sum(apply_D(D, metric[3 * l + m], l) for l in range(3)) for m in range(3)])
