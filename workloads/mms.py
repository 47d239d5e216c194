"""Manufactured solutions: problem data (exact fields and the forcing that makes them steady).

``kind="table"``: the supersonic flow of the viscous error-vs-cost study (section "Viscous flow:
3D manufactured solution", eq. mms with the constants of Table tab_3dmms_ns) on the unit cube with
Dirichlet data on every face.

``kind="channel"``: a subsonic flow on the unit cube, periodic in x_1 and x_3, between the planes
x_2 = 0 and x_2 = 1 on which the velocity and the normal temperature gradient vanish: the data of
adiabatic no-slip walls there (this one is not from the paper; it exercises the wall boundaries).

The exact primitive fields are sums and products of sines and cosines. The forcing that makes
them a steady solution of the compressible Navier-Stokes equations,

    S = d F_m / d x_m - d F^V_m / d x_m,

is derived here by symbolic differentiation of the continuous fluxes (inviscid flux of the
compressible Navier-Stokes section; viscous flux with the Stokes stress and the Fourier heat flux
+kappa dT/dx) and evaluated at the nodes. This is problem data, the same input for every
discretization; nothing here evaluates any part of a discretization.

Readings of the table: the x_3 term of U_1 carries U_1's own constants (the printed formula names
U_3^{x_3} there), and P^{x_3} = 2/3 as printed. Re = rho_0 U_0 L / mu with rho_0 = 1, U_0 = 800,
L = 1 (so mu = 2e-4 at Re = 4e6) and Ma = U_0 / c_0 = 2.14; the gas constant R cancels from the
residual (every term is written in rho, U, P) and is set to 287; Pr = 0.72.
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as sp
import torch

# (phi0, phi_x1, phi_x2, phi_x3, alpha_x1, alpha_x2, alpha_x3) and the trig function per direction
_TABLE = {
    "rho": ((1.0, 3 / 20, -1 / 10, 1 / 5, 1.0, 1 / 2, 1.0), ("sin", "cos", "sin")),
    "u1": ((800.0, 50.0, -30.0, 50.0, 3 / 2, 3 / 5, 1.0), ("sin", "cos", "cos")),
    "u2": ((800.0, -75.0, 40.0, 10.0, 1 / 2, 3 / 2, 3 / 2), ("cos", "sin", "sin")),
    "u3": ((800.0, 15.0, -25.0, 20.0, 3 / 2, 1 / 2, 5 / 4), ("sin", "sin", "cos")),
    "p": ((1.0e5, 2.0e4, 5.0e4, 2 / 3, 1.0, 3 / 2, 1.0), ("sin", "sin", "cos")),
}
L_REF = 1.0
GAMMA = 1.4
R_GAS = 287.0
PR = 0.72
RE = 4.0e6
MU = 1.0 * 800.0 * L_REF / RE


def _field_expr(name, X):
    (f0, a1, a2, a3, k1, k2, k3), fn = _TABLE[name]
    trig = {"sin": sp.sin, "cos": sp.cos}
    amps, ks = (a1, a2, a3), (k1, k2, k3)
    e = sp.Float(f0)
    for d in range(3):
        e = e + sp.Float(amps[d]) * trig[fn[d]](sp.Float(ks[d]) * sp.pi * X[d] / L_REF)
    return e


# channel solution: R = 1, T_0 = 1 (c_0 = 1.18), velocities up to 0.36, mu = 0.01
CHANNEL_R = 1.0
CHANNEL_MU = 0.01


def _table_fields(X, R):
    rho = _field_expr("rho", X)
    U = [_field_expr(n, X) for n in ("u1", "u2", "u3")]
    return rho, U, _field_expr("p", X)


def _channel_fields(X, R):
    s, c, pi = sp.sin, sp.cos, sp.pi
    x1, x2, x3 = X
    rho = 1 + sp.Rational(1, 10) * s(2 * pi * x1) * s(2 * pi * x3) + sp.Rational(1, 20) * c(pi * x2)
    U = [sp.Rational(3, 10) * s(pi * x2) * (1 + sp.Rational(1, 5) * c(2 * pi * x1)),
         sp.Rational(1, 10) * s(pi * x2) ** 2 * s(2 * pi * x1),
         sp.Rational(1, 5) * s(pi * x2) * c(2 * pi * x3)]
    T = 1 + sp.Rational(1, 10) * c(pi * x2) + sp.Rational(1, 20) * s(2 * pi * x1) * c(2 * pi * x3)
    return rho, U, rho * R * T


_FIELDS = {"table": _table_fields, "channel": _channel_fields}


@functools.lru_cache(maxsize=None)
def _symbolic(kind: str, mu: float, gamma: float, Pr: float, R: float):
    X = sp.symbols("x1 x2 x3", real=True)
    rho, U, P = _FIELDS[kind](X, R)
    T = P / (rho * R)
    rhoE = P / (gamma - 1) + rho * (U[0] ** 2 + U[1] ** 2 + U[2] ** 2) / 2
    kappa = mu * gamma * R / ((gamma - 1) * Pr)
    div = sum(sp.diff(U[k], X[k]) for k in range(3))
    tau = [[mu * (sp.diff(U[i], X[j]) + sp.diff(U[j], X[i])) - (sp.Rational(2, 3) * mu * div if i == j else 0)
            for j in range(3)] for i in range(3)]
    S = [0, 0, 0, 0, 0]
    for m in range(3):
        F = [rho * U[m]] + [rho * U[m] * U[c] + (P if c == m else 0) for c in range(3)] + [U[m] * (rhoE + P)]
        FV = [0] + [tau[m][c] for c in range(3)] + [sum(tau[m][k] * U[k] for k in range(3)) + kappa * sp.diff(T, X[m])]
        for c in range(5):
            S[c] = S[c] + sp.diff(F[c], X[m]) - sp.diff(FV[c], X[m])
    prim = [rho, U[0], U[1], U[2], P]
    f_prim = sp.lambdify(X, prim, "numpy")
    f_src = sp.lambdify(X, S, "numpy")
    return f_prim, f_src


def _as_np(x):
    return x.detach().cpu().numpy() if isinstance(x, torch.Tensor) else np.asarray(x)


def _defaults(kind, mu, R):
    if kind == "table":
        return (MU if mu is None else mu), (R_GAS if R is None else R)
    return (CHANNEL_MU if mu is None else mu), (CHANNEL_R if R is None else R)


def primitives(x, kind="table", R=None):
    """(rho, U (3,...), P) of the manufactured solution at coordinates x (3, ...)."""
    mu, R = _defaults(kind, None, R)
    f_prim, _ = _symbolic(kind, mu, GAMMA, PR, R)
    xn = _as_np(x)
    vals = [np.array(np.broadcast_to(np.asarray(v, dtype=np.float64), xn.shape[1:]))
            for v in f_prim(xn[0], xn[1], xn[2])]
    return vals[0], np.stack(vals[1:4]), vals[4]


def conservative(x, gamma=GAMMA, kind="table", R=None) -> np.ndarray:
    """q = [rho, rho U, rho E] of the manufactured solution, shape (5, ...)."""
    rho, u, p = primitives(x, kind, R)
    return np.stack([rho, rho * u[0], rho * u[1], rho * u[2],
                     p / (gamma - 1.0) + 0.5 * rho * (u * u).sum(0)])


def source(x, mu=None, gamma=GAMMA, Pr=PR, R=None, kind="table") -> np.ndarray:
    """Forcing S (5, ...) that makes the manufactured solution steady."""
    mu, R = _defaults(kind, mu, R)
    _, f_src = _symbolic(kind, mu, gamma, Pr, R)
    xn = _as_np(x)
    return np.stack([np.broadcast_to(np.asarray(v, dtype=np.float64), xn.shape[1:])
                     for v in f_src(xn[0], xn[1], xn[2])])


def speed_max(kind="table") -> float:
    """An upper bound of |U| + c over the unit cube (for time-step selection)."""
    g = np.linspace(0.0, 1.0, 41)
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"))
    rho, u, p = primitives(x, kind)
    return float((np.sqrt((u * u).sum(0)) + np.sqrt(GAMMA * p / rho)).max())
