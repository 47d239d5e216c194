"""Seeded synthetic inputs of the shapes and value distributions of the paper's workloads.

Storage conventions (shared by every consumer of these arrays):

* Elements of a periodic ``E x E x E`` box ``[0, L]^3`` are numbered
  ``e = e1 + E*e2 + E*E*e3``.
* Nodes of an element are numbered ``i1 + N*i2 + N*N*i3`` (xi_1 fastest), N = p + 1.
  Arrays are returned with shape ``(C, K, N, N, N)`` and axes ``(c, e, i3, i2, i1)``,
  so ``reshape(C, K*N**3)`` gives the structure-of-arrays layout.
* Face ``f`` of an element is ``2*l + (0 for the xi_l = -1 side, 1 for the +1 side)``,
  l = 0, 1, 2; ``neighbours(E)[e, f]`` is the element across that face.

Nothing here evaluates any part of the discretization: the caller supplies the
1-D reference node positions at which the mesh map is sampled.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import torch

F64 = torch.float64


@dataclasses.dataclass
class Problem:
    """One compressible Navier-Stokes problem on a warped box (periodic unless stated)."""

    name: str
    p: int
    E: int
    L: float = 2.0
    A: float = 0.1               # warp: x = g + A*(L/2)*prod_k sin(2*pi*g_k/L) per coordinate
    gamma: float = 1.4
    R: float = 1.0
    mu: float = 0.0              # constant dynamic viscosity; 0 -> Euler
    Pr: float = 0.72
    eta: float = 1.0             # interior-penalty coefficient
    iface_diss: int = 1          # 1 -> local Lax-Friedrichs interface dissipation
    two_point: int = 0           # 0 -> Chandrashekar flux, 1 -> central (test only)
    init: str = "random"         # random | tgv | constant | vortex | shear | mms
    periodic: bool = True        # False: the six box faces are Dirichlet boundaries
    box: Optional[tuple] = None  # per direction: None periodic, or a boundary kind (see neighbours)
    seed: int = 0
    Ma: float = 0.3
    u_rms: Optional[float] = None  # per-component rms velocity of the random state
    rho_amp: float = 0.2
    p0: float = 1.0
    p_amp: float = 0.1
    const: tuple = (1.0, 0.3, -0.2, 0.1, 1.0)   # (rho, u1, u2, u3, p) of the constant state
    Re: Optional[float] = None

    @property
    def N(self) -> int:
        return self.p + 1

    @property
    def K(self) -> int:
        return self.E ** 3

    @property
    def n_nodes(self) -> int:
        return self.K * self.N ** 3


def make_problem(name="custom", **kw) -> Problem:
    return Problem(name=name, **kw)


# ----------------------------------------------------------------------------------
# Named configurations of the five benchmark workloads (sizes as stated for each).
# ----------------------------------------------------------------------------------
CONFIG_NAMES = ("euler_p3_e4", "ns_tgv_p4_e32", "ns_p7_e16", "batch256", "vjp_p4_e16")


def _random_ns(name, p, E, A, Ma, Re, seed, L=2.0):
    c0 = math.sqrt(1.4 * 1.0 / 1.0)
    u_rms_mag = Ma * c0
    mu = 1.0 * u_rms_mag * 1.0 / Re
    return Problem(name=name, p=p, E=E, L=L, A=A, R=1.0, mu=mu, init="random",
                   seed=seed, Ma=Ma, u_rms=u_rms_mag / math.sqrt(3.0), Re=Re)


def mms_problem(p: int, E: int, A: float = 0.0, two_point: int = 0, iface_diss: int = 1,
                mu: Optional[float] = None) -> Problem:
    """The manufactured-solution problem of the viscous error-vs-cost study on the unit cube,
    Dirichlet boundaries on all faces (see ``workloads.mms``)."""
    from . import mms
    return Problem(name=f"mms_p{p}_e{E}", p=p, E=E, L=1.0, A=A, gamma=mms.GAMMA, R=mms.R_GAS,
                   mu=mms.MU if mu is None else mu, Pr=mms.PR, init="mms", periodic=False,
                   two_point=two_point, iface_diss=iface_diss, Ma=800.0 / math.sqrt(1.4e5),
                   Re=mms.RE)


def channel_problem(p: int, E: int, A: float = 0.0, iface_diss: int = 1,
                    mu: Optional[float] = None, two_point: int = 0) -> Problem:
    """The wall-bounded manufactured solution (``workloads.mms``, kind "channel") on the unit cube:
    periodic in x_1 and x_3, adiabatic no-slip walls on the x_2 faces."""
    from . import mms
    return Problem(name=f"channel_p{p}_e{E}", p=p, E=E, L=1.0, A=A, gamma=mms.GAMMA,
                   R=mms.CHANNEL_R, mu=mms.CHANNEL_MU if mu is None else mu, Pr=mms.PR,
                   init="channel", box=(None, -3, None), two_point=two_point,
                   iface_diss=iface_diss, Ma=0.3)


def problem_neighbours(prob: Problem) -> np.ndarray:
    """The neighbour table of a problem's box (periodic, Dirichlet or walls as it states)."""
    return neighbours(prob.E, prob.periodic, prob.box)


def config(name: str) -> Problem:
    """The single-problem workloads by name (the batch is ``batch_config``)."""
    if name == "euler_p3_e4":
        # Euler, p = 3, 4^3 elements on [0,2]^3 warped with amplitude 0.1; rho = 1+0.2*smooth,
        # velocity components smooth with rms 0.3, pressure 1 + 0.1*smooth.
        return Problem(name=name, p=3, E=4, L=2.0, A=0.1, mu=0.0, init="random", seed=1,
                       u_rms=0.3)
    if name == "ns_tgv_p4_e32":
        # Taylor-Green vortex at Ma = 0.1, Re = 1600 on [0, 2pi]^3, p = 4, 32^3 warped elements.
        Ma = 0.1
        return Problem(name=name, p=4, E=32, L=2.0 * math.pi, A=0.1, gamma=1.4,
                       R=1.0 / (1.4 * Ma * Ma), mu=1.0 / 1600.0, Pr=0.72, init="tgv",
                       seed=2, Ma=Ma, Re=1600.0)
    if name == "ns_p7_e16":
        return _random_ns(name, p=7, E=16, A=0.15, Ma=0.3, Re=1000.0, seed=3)
    if name == "vjp_p4_e16":
        return _random_ns(name, p=4, E=16, A=0.1, Ma=0.2, Re=500.0, seed=5)
    raise KeyError(name)


def batch_config(n_prob: int = 256, seed_base: int = 4000, p_range=(2, 8), e_range=(2, 12)):
    """Heterogeneous batch: p ~ U{2..8}, E ~ U{2..12}, A ~ U[0.05, 0.15], mu = 1e-3."""
    rng = np.random.Generator(np.random.PCG64(seed_base))
    probs = []
    for b in range(n_prob):
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        E = int(rng.integers(e_range[0], e_range[1] + 1))
        A = float(rng.uniform(0.05, 0.15))
        c0 = math.sqrt(1.4)
        probs.append(Problem(name=f"batch{b}", p=p, E=E, L=2.0, A=A, R=1.0, mu=1e-3,
                             init="random", seed=seed_base + 1 + b, Ma=0.3,
                             u_rms=0.3 * c0 / math.sqrt(3.0)))
    return probs


# ----------------------------------------------------------------------------------
# Mesh
# ----------------------------------------------------------------------------------
def neighbours(E: int, periodic: bool = True, box=None) -> np.ndarray:
    """[K, 6] int32 face-neighbour table of the E^3 grid.

    ``box`` = (k1, k2, k3) says per direction what lies beyond the two box faces normal to it:
    None for periodic wrap-around, or a negative boundary kind written into the table (-1
    Dirichlet, -2 slip wall, -3 adiabatic no-slip wall).  ``periodic=False`` without ``box``
    makes every box face a Dirichlet boundary."""
    if box is None:
        box = (None, None, None) if periodic else (-1, -1, -1)
    e = np.arange(E ** 3)
    pos = (e % E, (e // E) % E, e // (E * E))
    cols = []
    for d in range(3):
        for step in (-1, 1):
            c = [pos[0], pos[1], pos[2]]
            c[d] = c[d] + step
            n = (c[0] % E) + E * (c[1] % E) + E * E * (c[2] % E)
            if box[d] is not None:
                out = (c[d] < 0) | (c[d] >= E)
                n = np.where(out, int(box[d]), n)
            cols.append(n)
    return np.stack(cols, axis=1).astype(np.int32)


def coords(prob: Problem, xi1d, device="cpu") -> torch.Tensor:
    """Physical node coordinates, shape (3, K, N, N, N), for reference nodes ``xi1d`` in [-1, 1].

    Reference point (element (e1,e2,e3), xi) maps to g_d = (L/E)*(e_d + (xi_d + 1)/2) and then
    x_d = g_d + A*(L/2)*sin(2 pi g_1/L) sin(2 pi g_2/L) sin(2 pi g_3/L).
    """
    E, N, L = prob.E, prob.N, prob.L
    xi = torch.as_tensor(np.asarray(xi1d, dtype=np.float64), dtype=F64, device=device)
    assert xi.numel() == N
    h = L / E
    ev = torch.arange(E, dtype=F64, device=device)
    g1d = h * (ev[:, None] + (xi[None, :] + 1.0) * 0.5)          # (E, N)
    # axes (e3, e2, e1, i3, i2, i1)
    g1 = g1d[None, None, :, None, None, :].expand(E, E, E, N, N, N)
    g2 = g1d[None, :, None, None, :, None].expand(E, E, E, N, N, N)
    g3 = g1d[:, None, None, :, None, None].expand(E, E, E, N, N, N)
    w = 2.0 * math.pi / L
    bump = prob.A * (L / 2.0) * torch.sin(w * g1) * torch.sin(w * g2) * torch.sin(w * g3)
    x = torch.stack([g1 + bump, g2 + bump, g3 + bump])
    return x.reshape(3, E ** 3, N, N, N).contiguous()


def mapping_jacobian(prob: Problem, xi1d) -> np.ndarray:
    """dx_m/dxi_i of the mapping of coords() at the nodes, evaluated from its closed form, shape
    (3, 3, K, N, N, N) (entry [m][i]).  With g_d = (L/E)(e_d + (xi_d + 1)/2) and
    x_d = g_d + b(g), b = A (L/2) sin(w g_1) sin(w g_2) sin(w g_3), w = 2 pi/L:
    dx_m/dxi_i = (L/(2E)) (delta_mi + A (L/2) w cos(w g_i) prod_{j != i} sin(w g_j))."""
    E, N, L = prob.E, prob.N, prob.L
    xi = np.asarray(xi1d, dtype=np.float64)
    assert xi.size == N
    h = L / E
    g1d = h * (np.arange(E, dtype=np.float64)[:, None] + (xi[None, :] + 1.0) * 0.5)
    g = [np.broadcast_to(g1d[None, None, :, None, None, :], (E, E, E, N, N, N)),
         np.broadcast_to(g1d[None, :, None, None, :, None], (E, E, E, N, N, N)),
         np.broadcast_to(g1d[:, None, None, :, None, None], (E, E, E, N, N, N))]
    w = 2.0 * math.pi / L
    sn = [np.sin(w * gi) for gi in g]
    cs = [np.cos(w * gi) for gi in g]
    out = np.zeros((3, 3, E, E, E, N, N, N))
    for i in range(3):
        db = prob.A * (L / 2.0) * w * cs[i] * sn[(i + 1) % 3] * sn[(i + 2) % 3]
        for m in range(3):
            out[m, i] = 0.5 * h * ((1.0 if m == i else 0.0) + db)
    return out.reshape(3, 3, E ** 3, N, N, N)


# ----------------------------------------------------------------------------------
# Fields
# ----------------------------------------------------------------------------------
_KVEC = None


def _half_space_wavevectors():
    global _KVEC
    if _KVEC is None:
        ks = []
        for a in range(-2, 3):
            for b in range(-2, 3):
                for c in range(-2, 3):
                    k = (a, b, c)
                    if max(abs(a), abs(b), abs(c)) == 0:
                        continue
                    first = next(v for v in k if v != 0)
                    if first > 0:
                        ks.append(k)
        _KVEC = np.array(ks, dtype=np.float64)
    return _KVEC


class SmoothField:
    """phi(x) = sum_k a_k cos(2 pi k.x / L + phase_k) / sum_k |a_k|, 1 <= |k|_inf <= 2.

    a_k ~ N(0,1)/|k|^2 and phase_k ~ U[0, 2pi) from a PCG64 stream; |phi| <= 1 everywhere,
    and the box-mean of phi^2 is ``rms**2`` (closed form).
    """

    def __init__(self, seed: int, L: float):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.k = _half_space_wavevectors()
        kn = np.linalg.norm(self.k, axis=1)
        self.a = rng.standard_normal(len(self.k)) / kn ** 2
        self.phase = rng.uniform(0.0, 2.0 * math.pi, len(self.k))
        self.L = L
        s = np.abs(self.a).sum()
        self.a = self.a / s
        self.rms = math.sqrt(float((self.a ** 2).sum()) / 2.0)

    def __call__(self, x: torch.Tensor) -> torch.Tensor:
        w = 2.0 * math.pi / self.L
        out = torch.zeros_like(x[0])
        for kk, a, ph in zip(self.k, self.a, self.phase):
            arg = w * (kk[0] * x[0] + kk[1] * x[1] + kk[2] * x[2]) + ph
            out += a * torch.cos(arg)
        return out


def primitive_state(prob: Problem, x: torch.Tensor):
    """(rho, u (3,...), p) of the problem's initial condition at coordinates x (3, ...)."""
    if prob.init == "random":
        base = prob.seed * 16
        f_rho = SmoothField(base + 0, prob.L)
        f_u = [SmoothField(base + 1 + d, prob.L) for d in range(3)]
        f_p = SmoothField(base + 4, prob.L)
        rho = 1.0 + prob.rho_amp * f_rho(x)
        urms = prob.u_rms if prob.u_rms is not None else 0.3
        u = torch.stack([urms * f(x) / f.rms for f in f_u])
        p = prob.p0 + prob.p_amp * prob.p0 * f_p(x)
        return rho, u, p
    if prob.init == "tgv":
        # Taylor-Green vortex initial condition, section on the cost of entropy stability
        # (rho0 = U0 = T0 = 1, R = 1/(gamma Ma^2)).
        g, Ma = prob.gamma, prob.Ma
        x1, x2, x3 = x[0], x[1], x[2]
        rho = 1.0 + g * Ma * Ma / 16.0 * (torch.cos(2 * x1) + torch.cos(2 * x2)) * (torch.cos(2 * x3) + 2.0)
        u = torch.stack([torch.sin(x1) * torch.cos(x2) * torch.cos(x3),
                         -torch.cos(x1) * torch.sin(x2) * torch.cos(x3),
                         torch.zeros_like(x1)])
        T = torch.ones_like(x1)
        p = rho * prob.R * T
        return rho, u, p
    if prob.init in ("mms", "channel"):
        from . import mms
        rho, u, p = mms.primitives(x, "table" if prob.init == "mms" else "channel")
        return (torch.as_tensor(rho, dtype=F64, device=x.device), torch.as_tensor(u, dtype=F64, device=x.device),
                torch.as_tensor(p, dtype=F64, device=x.device))
    if prob.init == "constant":
        r, a, b, c, pp = prob.const
        one = torch.ones_like(x[0])
        return r * one, torch.stack([a * one, b * one, c * one]), pp * one
    if prob.init == "vortex":
        # Stationary isentropic vortex of the isentropic-vortex section (beta = 5, T_inf = 1),
        # axis parallel to x_3 through the box centre; R = 1/(gamma Ma^2) makes it steady.
        g, Ma, beta = prob.gamma, prob.Ma, 5.0
        c = prob.L / 2.0
        d1, d2 = x[0] - c, x[1] - c
        r2 = d1 * d1 + d2 * d2
        T = 1.0 - (g - 1.0) * Ma * Ma * beta * beta / (8.0 * math.pi ** 2) * torch.exp(1.0 - r2)
        rho = T ** (1.0 / (g - 1.0))
        ut = beta / (2.0 * math.pi) * torch.exp((1.0 - r2) / 2.0)     # U_t / r
        u = torch.stack([-ut * d2, ut * d1, torch.zeros_like(d1)])
        p = rho * prob.R * T
        return rho, u, p
    if prob.init == "shear":
        one = torch.ones_like(x[0])
        eps = prob.Ma
        u1 = eps * torch.sin(2.0 * math.pi * x[1] / prob.L)
        return one, torch.stack([u1, 0 * one, 0 * one]), prob.p0 * one
    raise KeyError(prob.init)


def state(prob: Problem, x: torch.Tensor) -> torch.Tensor:
    """Conservative state (5, K, N, N, N) = [rho, rho u, p/(gamma-1) + rho |u|^2 / 2]."""
    rho, u, p = primitive_state(prob, x)
    m = rho[None] * u
    Et = p / (prob.gamma - 1.0) + 0.5 * rho * (u * u).sum(0)
    return torch.cat([rho[None], m, Et[None]]).contiguous()


def jumped_state(prob: Problem, x: torch.Tensor, seed: int, amp: float = 0.5) -> torch.Tensor:
    """The problem's state with density and pressure each multiplied, node by node, by an
    independent factor exp(U[-amp, amp]) (velocity unchanged): neighbouring nodes then differ by up
    to a factor e^(2 amp), so most two-point averages of rho and rho/(2P) are taken between far-apart
    values.  Shape (5, K, N, N, N)."""
    rho, u, p = primitive_state(prob, x)
    rng = np.random.Generator(np.random.PCG64(seed))
    fr = torch.as_tensor(np.exp(rng.uniform(-amp, amp, tuple(rho.shape))), dtype=F64, device=x.device)
    fp = torch.as_tensor(np.exp(rng.uniform(-amp, amp, tuple(p.shape))), dtype=F64, device=x.device)
    rho = rho * fr
    p = p * fp
    m = rho[None] * u
    Et = p / (prob.gamma - 1.0) + 0.5 * rho * (u * u).sum(0)
    return torch.cat([rho[None], m, Et[None]]).contiguous()


def cfl_dt(prob: Problem, x: torch.Tensor, cfl: float = 0.25) -> float:
    """dt = cfl * (L/E) / ((p+1)^2 * max(|u| + c)) from the initial primitive fields."""
    rho, u, p = primitive_state(prob, x)
    c = torch.sqrt(prob.gamma * p / rho)
    smax = float((torch.sqrt((u * u).sum(0)) + c).max())
    return cfl * (prob.L / prob.E) / ((prob.p + 1) ** 2 * smax)


def cotangent(prob: Problem, seed: int, device="cpu") -> torch.Tensor:
    """Seeded N(0,1) cotangent of shape (5, K, N, N, N)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((5, prob.K, prob.N, prob.N, prob.N))
    return torch.as_tensor(g, dtype=F64, device=device)


def direction(q: torch.Tensor, seed: int) -> torch.Tensor:
    """Seeded N(0,1) direction scaled per component by the rms of that component of q."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = torch.as_tensor(rng.standard_normal(tuple(q.shape)), dtype=F64, device=q.device)
    rms = torch.sqrt((q.reshape(q.shape[0], -1) ** 2).mean(1))
    return v * rms.reshape(-1, *([1] * (q.dim() - 1)))
