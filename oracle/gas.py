"""Pointwise physics of the compressible Navier-Stokes equations (section "Discretization of the
compressible Navier-Stokes equations").

All functions take nodal arrays with the component axis first and work for any NumPy
scalar type. Branches on values (log-mean series, absolute values, maxima) decide on the
real part, so a complex-step perturbation follows the real computation.
"""
from __future__ import annotations

import numpy as np


class Gas:
    """Ideal gas with constant viscosity: gamma, R, mu, Pr (kappa = mu c_p / Pr)."""

    def __init__(self, gamma=1.4, R=1.0, mu=0.0, Pr=0.72):
        self.gamma, self.R, self.mu, self.Pr = gamma, R, mu, Pr

    @property
    def cp(self):
        return self.gamma * self.R / (self.gamma - 1.0)

    @property
    def kappa(self):
        return self.mu * self.cp / self.Pr


def primitives(q, gas: Gas):
    """rho, u (3,...), P, T from q = [rho, rho U, rho E] with P = (gamma-1)(rho E - rho|U|^2/2),
    P = rho R T (constituent relations)."""
    rho = q[0]
    u = q[1:4] / rho
    P = (gas.gamma - 1.0) * (q[4] - 0.5 * rho * (u * u).sum(0))
    T = P / (rho * gas.R)
    return rho, u, P, T


def entropy(q, gas: Gas):
    """Specific entropy s = R/(gamma-1) log T - R log rho (reference T and rho set to 1)."""
    rho, u, P, T = primitives(q, gas)
    return gas.R / (gas.gamma - 1.0) * np.log(T) - gas.R * np.log(rho)


def entropy_function(q, gas: Gas):
    """Entropy function S = -rho s."""
    return -q[0] * entropy(q, gas)


def entropy_variables(q, gas: Gas):
    """W = dS/dQ = (1/T) [c_p T - T s - |U|^2/2, U_1, U_2, U_3, -1]."""
    rho, u, P, T = primitives(q, gas)
    s = gas.R / (gas.gamma - 1.0) * np.log(T) - gas.R * np.log(rho)
    k = (u * u).sum(0)
    w1 = (gas.cp * T - T * s - 0.5 * k) / T
    return np.stack([w1, u[0] / T, u[1] / T, u[2] / T, -1.0 / T])


def euler_flux(q, gas: Gas):
    """Inviscid fluxes F_m (eq. ns_iflux), shape (3, 5, ...):
    [rho U_m, rho U_m U + delta_m P, rho U_m H], H = c_p T + |U|^2/2."""
    rho, u, P, T = primitives(q, gas)
    H = gas.cp * T + 0.5 * (u * u).sum(0)
    out = []
    for m in range(3):
        mom = [rho * u[m] * u[c] + (P if c == m else 0.0) for c in range(3)]
        out.append(np.stack([rho * u[m], *mom, rho * u[m] * H]))
    return np.stack(out)


def log_mean(a, b):
    """Logarithmic mean (a - b)/(log a - log b), with its limit a at a = b.

    With z = (a-b)/(a+b), log(a/b) = 2 artanh z, so the mean equals
    (a+b) / (2 (1 + z^2/3 + z^4/5 + z^6/7 + ...)); for |z| < 1e-3 the series is cut
    after z^6 (remainder below 1e-24 relative), otherwise (a-b)/log1p((a-b)/b) is used.
    """
    z = (a - b) / (a + b)
    small = np.abs(np.real(z)) < 1e-3
    z2 = z * z
    series = (a + b) / (2.0 * (1.0 + z2 / 3.0 + z2 * z2 / 5.0 + z2 * z2 * z2 / 7.0))
    d = np.where(small, np.ones_like(a), a - b)
    bb = np.where(small, np.ones_like(b), b)
    with np.errstate(all="ignore"):
        direct = d / np.log1p(d / bb)
    return np.where(small, series, direct)


def chandrashekar_flux(qi, qj, gas: Gas):
    """Chandrashekar's two-point entropy-conservative flux F_m(Q_i, Q_j), shape (3, 5, ...).

    rho_hat, beta_hat: logarithmic means; bars: arithmetic means; beta = 1/(2RT);
    P_tilde = R rho_bar T_i T_j / T_bar; the energy component is
    rho_hat U_bar_m (1/(2(gamma-1) beta_hat) - mean(|U|^2)/2) + U_bar . M, with M the three
    momentum components of the same flux.
    """
    ri, ui, Pi, Ti = primitives(qi, gas)
    rj, uj, Pj, Tj = primitives(qj, gas)
    bi = 1.0 / (2.0 * gas.R * Ti)
    bj = 1.0 / (2.0 * gas.R * Tj)
    rho_hat = log_mean(ri, rj)
    beta_hat = log_mean(bi, bj)
    rho_bar = 0.5 * (ri + rj)
    u_bar = 0.5 * (ui + uj)
    T_bar = 0.5 * (Ti + Tj)
    P_tilde = gas.R * rho_bar * Ti * Tj / T_bar
    k_mean = 0.5 * ((ui * ui).sum(0) + (uj * uj).sum(0))
    out = []
    for m in range(3):
        f_rho = rho_hat * u_bar[m]
        M = [f_rho * u_bar[c] + (P_tilde if c == m else 0.0) for c in range(3)]
        f_E = (f_rho * (1.0 / (2.0 * (gas.gamma - 1.0) * beta_hat) - 0.5 * k_mean)
               + u_bar[0] * M[0] + u_bar[1] * M[1] + u_bar[2] * M[2])
        out.append(np.stack([f_rho, *M, f_E]))
    return np.stack(out)


def kennedy_gruber_flux(qi, qj, gas: Gas):
    """Kennedy-Gruber split-form two-point flux (SF-KG), shape (3, 5, ...):
    [rho_bar U_bar_m, rho_bar U_bar_m U_bar + delta_m P_bar, rho_bar U_bar_m E_bar + P_bar U_bar_m]."""
    ri, ui, Pi, Ti = primitives(qi, gas)
    rj, uj, Pj, Tj = primitives(qj, gas)
    rho_bar = 0.5 * (ri + rj)
    u_bar = 0.5 * (ui + uj)
    P_bar = 0.5 * (Pi + Pj)
    E_bar = 0.5 * (qi[4] / ri + qj[4] / rj)
    out = []
    for m in range(3):
        f = rho_bar * u_bar[m]
        mom = [f * u_bar[c] + (P_bar if c == m else 0.0) for c in range(3)]
        out.append(np.stack([f, *mom, f * E_bar + P_bar * u_bar[m]]))
    return np.stack(out)


def central_flux(qi, qj, gas: Gas):
    """Arithmetic mean of the nodal Euler fluxes (used only to pin the flux-differencing form)."""
    return 0.5 * (euler_flux(qi, gas) + euler_flux(qj, gas))


# Two-point fluxes by option: 0 Chandrashekar (ES-C), 1 central, 2 Kennedy-Gruber (SF-KG).
# Option 3 is the standard DC discretization: its volume term is not a two-point form; its
# interface flux is the central flux (plus the optional Lax-Friedrichs dissipation).
TWO_POINT = {0: chandrashekar_flux, 1: central_flux, 2: kennedy_gruber_flux, 3: central_flux}


def matrix_dissipation_operator(qi, qn, nbar, gas: Gas):
    """The 5x5 matrix |nbar| R |Lambda| T R^T of the entropy-stable matrix interface dissipation
    (shape (5, 5, ...)): the dissipative part of a Roe-type flux written in entropy variables, with
    the eigenvectors R of the flux Jacobian in the unit normal n = nbar/|nbar| scaled by T so that
    R T R^T = dq/dw (the matrix-dissipation operators of Barth, Chandrashekar and Winters et al.),
    and the states averaged as in the Chandrashekar flux:

    rho_hat, beta_hat logarithmic means; beta_bar, U_bar, |U|^2_bar arithmetic means;
    p_hat = rho_bar / (2 beta_bar);  a_hat = sqrt(gamma p_hat / rho_hat);
    h_hat = gamma / (2 (gamma-1) beta_hat) + |U_bar|^2 - |U|^2_bar / 2;
    acoustic  r = [1, U_bar -+ a_hat n, h_hat -+ a_hat U_bar.n],  |U_bar.n -+ a_hat|,  rho_hat/(2 gamma)
    entropy   r = [1, U_bar, |U_bar|^2/2],                        |U_bar.n|,          rho_hat (gamma-1)/gamma
    shear     r = [0, t, U_bar.t] for the two unit tangents t,   |U_bar.n|,          p_hat
    (the shear pair is B^T (I - n n^T) B with B = [0 | I | U_bar], so no tangents are needed).
    Our entropy variables are R times the standard ones, so the scaling enters divided by R.
    """
    ri, ui, Pi, Ti = primitives(qi, gas)
    rn, un, Pn, Tn = primitives(qn, gas)
    g, R = gas.gamma, gas.R
    bi, bn = 1.0 / (2.0 * R * Ti), 1.0 / (2.0 * R * Tn)
    rho_hat = log_mean(ri, rn)
    beta_hat = log_mean(bi, bn)
    beta_bar = 0.5 * (bi + bn)
    ub = 0.5 * (ui + un)
    kbar = 0.5 * ((ui * ui).sum(0) + (un * un).sum(0))
    p_hat = 0.5 * (ri + rn) / (2.0 * beta_bar)
    a_hat = np.sqrt(g * p_hat / rho_hat)
    ubsq = (ub * ub).sum(0)
    h_hat = g / (2.0 * (g - 1.0) * beta_hat) + ubsq - 0.5 * kbar
    nn = np.sqrt((nbar * nbar).sum(0))
    n = nbar / nn
    vn = (ub * n).sum(0)
    # |x| continued analytically (sign of the real part), so that the complex step differentiates it
    cabs = lambda x: np.where(np.real(x) >= 0, x, -x)  # noqa: E731
    one, zero = np.ones_like(vn), np.zeros_like(vn)
    M = np.zeros((5, 5) + vn.shape, dtype=np.result_type(vn, np.float64))
    for sgn in (-1.0, 1.0):
        r = np.stack([one, ub[0] + sgn * a_hat * n[0], ub[1] + sgn * a_hat * n[1],
                      ub[2] + sgn * a_hat * n[2], h_hat + sgn * a_hat * vn])
        M = M + (cabs(vn + sgn * a_hat) * rho_hat / (2.0 * g * R)) * r[:, None] * r[None, :]
    r = np.stack([one, ub[0], ub[1], ub[2], 0.5 * ubsq])
    M = M + (cabs(vn) * rho_hat * (g - 1.0) / (g * R)) * r[:, None] * r[None, :]
    B = np.zeros((3, 5) + vn.shape, dtype=M.dtype)
    for k in range(3):
        B[k, k + 1] = one
        B[k, 4] = ub[k]
    P = np.stack([np.stack([(1.0 if i == j else 0.0) - n[i] * n[j] for j in range(3)]) for i in range(3)])
    M = M + (cabs(vn) * p_hat / R) * np.einsum("ka...,kl...,lb...->ab...", B, P, B)
    return nn * M


def matrix_dissipation(qi, qn, nbar, gas: Gas):
    """|nbar| R |Lambda| T R^T (w_i - w_nu), shape (5, ...) (see matrix_dissipation_operator)."""
    dw = entropy_variables(qi, gas) - entropy_variables(qn, gas)
    return np.einsum("ab...,b...->a...", matrix_dissipation_operator(qi, qn, nbar, gas), dw)


def contract(F, n):
    """sum_m F_m n_m for F of shape (3, 5, ...) and n of shape (3, ...)."""
    return F[0] * n[0] + F[1] * n[1] + F[2] * n[2]


def sound_speed(q, gas: Gas):
    """c = sqrt(gamma P / rho) (ideal gas)."""
    rho, u, P, T = primitives(q, gas)
    return np.sqrt(gas.gamma * P / rho)


def max_wave_speed(q, n, gas: Gas):
    """|U . n| + c |n|: the largest characteristic speed of the Euler flux contracted with the
    (unnormalised) vector n, i.e. the spectral radius of d(F(q) . n)/dq.  This is the wave speed of
    the local Lax-Friedrichs interface dissipation (absolute value decided on the real part)."""
    rho, u, P, T = primitives(q, gas)
    un = (u * n).sum(0)
    aun = np.where(np.real(un) >= 0, un, -un)
    return aun + sound_speed(q, gas) * np.sqrt((n * n).sum(0))


def viscous_blocks(q, gas: Gas):
    """The 5x5 blocks C_mj with F^V_m = sum_j C_mj dW/dx_j (eq. Fxment), shape (3, 3, 5, 5, ...).

    Written out from the viscous flux (eq. Fv, with the Fourier heat flux +kappa dT/dx_m) and the
    stresses (eq. tau), using dU_k = T (dW_{k+1} + U_k dW_5) and dT = T^2 dW_5.
    """
    rho, u, P, T = primitives(q, gas)
    mt = gas.mu * T
    kt = gas.kappa * T * T
    k = (u * u).sum(0)
    zero = np.zeros_like(mt)
    C = np.empty((3, 3, 5, 5) + mt.shape, dtype=np.result_type(q.dtype, np.float64))
    C[...] = 0.0
    d = lambda a, b: 1.0 if a == b else 0.0  # noqa: E731
    for m in range(3):
        for j in range(3):
            for i in range(3):
                for kk in range(3):
                    C[m, j, i + 1, kk + 1] = mt * (d(m, j) * d(i, kk) + d(i, j) * d(m, kk)
                                                   - 2.0 / 3.0 * d(i, m) * d(j, kk))
                C[m, j, i + 1, 4] = mt * (d(m, j) * u[i] + d(i, j) * u[m] - 2.0 / 3.0 * d(i, m) * u[j])
                C[m, j, 4, i + 1] = mt * (d(m, j) * u[i] + d(m, i) * u[j] - 2.0 / 3.0 * d(j, i) * u[m])
            C[m, j, 4, 4] = mt * (d(m, j) * k + u[m] * u[j] / 3.0) + kt * d(m, j) + zero
    return C


def viscous_flux(q, grad_w, gas: Gas):
    """F^V_m = sum_j C_mj grad_w[j] for grad_w of shape (3, 5, ...) (j, component); returns (3, 5, ...)."""
    C = viscous_blocks(q, gas)
    return np.einsum("mjab...,jb...->ma...", C, grad_w)
