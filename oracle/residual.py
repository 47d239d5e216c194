"""Semi-discrete residual dq/dt of the entropy-stable SBP-SAT discretization (ES-C) of the
compressible Navier-Stokes equations on conforming curvilinear hexahedra.

Follows eq. discEL (inviscid flux differencing), eq. NSL with eq. MacroForm (viscous
operator in entropy variables, LDG/BR1 gradient, interior penalty), the Chandrashekar
two-point flux, and SATs for conforming periodic interfaces. Readings of passages that
are garbled or that defer to other papers:

* volume term: sum_l sum_j D_l(i,j) (A_l,i + A_l,j) . F#(q_i, q_j), with no factor 1/2 and
  the metric [A_lm] in both terms (the only reading consistent with the linear split
  form, eq. convectionsplitdisc);
* inviscid interface SAT at a node i on face (l, s) of an element, partner node nu on the
  neighbour, n = (A_l,i + A_l,nu)/2, w_end the end weight of the 1-D norm:
      -(s / w_end) [ F#(q_i, q_nu) . n - F(q_i) . A_l,i ]
  plus local Lax-Friedrichs dissipation -(lam / (2 w_end)) (q_i - q_nu),
  lam = max over the two sides of |U . n| + c |n| (iface_diss = 1), or the matrix dissipation
  -(1 / (2 w_end)) |n| R |Lambda| T R^T (w_i - w_nu) (iface_diss = 2, ``gas.matrix_dissipation``);
* viscous operator with theta_a = D_a w + (s/(2 w_end)) (w_nu - w_i) on faces of direction a,
  g_j = sum_a A_aj theta_a / J, F^V_m = sum_j C_mj g_j, fhat_l = sum_m A_lm F^V_m, and
      sum_l D_l fhat_l + (s/(2 w_end)) (fhat_l,nu - fhat_l,i)
      - (eta / w_end) (Chat_ll,i + Chat_ll,nu)/2 (w_i - w_nu),
  Chat_ll = sum_{m,j} A_lm C_mj A_lj / J (eq. Chatij with the summation index fixed);
* the output is dq/dt: the sum of the terms divided by J, plus an optional source term (the
  forcing of a manufactured solution, given per node);
* a boundary face is an interface with a ghost element whose face node carries a ghost state and
  the own node's metrics and J; the inviscid SAT, dissipation, SAT^theta and interior penalty keep
  their interface form with the ghost data.  The neighbour index names the boundary kind:
  -1 Dirichlet: the ghost state is the prescribed state; SAT^V vanishes (the boundary viscous
     flux is the interior one).  A far field is this kind with free-stream data.
  -2 slip wall (inviscid problems only): the ghost is the own state with the momentum reflected
     about the face, m - 2 (m . n) n with n the unit normal A_l / |A_l|; the shared flux then
     carries the pressure alone.
  -3 adiabatic no-slip wall: the ghost is the own state with the momentum reversed, (rho, -m,
     rho E), so that the face averages hold zero velocity and the own temperature; the shared
     flux carries the pressure alone, and SAT^V sets the boundary viscous flux to the own
     momentum flux with zero energy flux (no heat flux, no work at rest):
     -(s / w_end) fhat_l,i[energy] on the energy equation.
  These wall terms follow from the entropy analysis of the interface terms (the wall SATs of the
  references the paper cites are not given in it); the oracle's tests pin their entropy budget.
* faces of neighbouring elements may meet in any of the eight relative orientations of a square
  (unstructured hexahedral meshes): ``orient[e, f] = f' + 8 * code`` names the neighbour's face f'
  (direction l', side s') and how its face-node grid lies on the own one.  With own face-node
  coordinates (a, b) (the two tangential indices in increasing direction order), the partner node
  has (a', b') = (F_a(x), F_b(y)) with (x, y) = (b, a) if bit 0 of code is set, else (a, b), and
  F_a, F_b reversals (N - 1 - .) when bits 1, 2 are set.  The partner's metric row and viscous
  flux are those of its direction l', times -s s' (so that they point as the own direction l
  does).  ``orient=None`` is the aligned case f' = f xor 1, code 0.
"""
from __future__ import annotations

import numpy as np

from . import gas as G
from .geometry import apply_D


class Params:
    """Problem constants: the gas, interior-penalty coefficient eta, the interface dissipation
    (0 none, 1 local Lax-Friedrichs, 2 entropy-stable matrix dissipation), and the inviscid volume form: 0 Chandrashekar (ES-C), 1 central, 2
    Kennedy-Gruber (SF-KG) two-point fluxes, or 3 the standard DC form."""

    def __init__(self, gamma=1.4, R=1.0, mu=0.0, Pr=0.72, eta=1.0, iface_diss=1, two_point=0):
        self.gas = G.Gas(gamma, R, mu, Pr)
        self.eta = eta
        self.iface_diss = iface_diss
        self.two_point = two_point

    @classmethod
    def of(cls, prob):
        return cls(prob.gamma, prob.R, prob.mu, prob.Pr, prob.eta, prob.iface_diss, prob.two_point)


def _take(u, idx, l):
    """Slice of element arrays at index idx along direction xi_l (the axis is removed)."""
    return np.take(u, idx, axis=u.ndim - 1 - l)


def _index(ndim, idx, l):
    sl = [slice(None)] * ndim
    sl[ndim - 1 - l] = idx
    return tuple(sl)


def _faces(p):
    """(l, s, face id, own index, neighbour index) for the six faces of an element."""
    out = []
    for l in range(3):
        for side, s in ((0, -1.0), (1, 1.0)):
            own = 0 if s < 0 else p
            out.append((l, s, 2 * l + side, own, p - own))
    return out


def volume_term(q, metric, sbp, prm: Params):
    """sum_l sum_j D(i_l, j_l) (A_l,i + A_l,j) . F#(q_i, q_j) over the nodes j on the xi_l line
    through i (eq. discEL), for element arrays q (5, n, N, N, N).

    For the standard DC form (option 3) the SBP derivative is applied to the nodal inviscid fluxes
    (eq. ns_iflux) in strong conservation form: sum_l D_l (sum_m [A_lm] F_m)."""
    if prm.two_point == 3:
        F = G.euler_flux(q, prm.gas)
        return sum(apply_D(sbp.D, G.contract(F, metric[3 * l:3 * l + 3]), l) for l in range(3))
    flux = G.TWO_POINT[prm.two_point]
    V = np.zeros_like(q)
    N = sbp.N
    for l in range(3):
        Al = metric[3 * l:3 * l + 3]
        for a in range(N):
            qa, Aa = _take(q, a, l), _take(Al, a, l)
            acc = np.zeros_like(qa)
            for b in range(N):
                if sbp.D[a, b] == 0.0:
                    continue
                qb, Ab = _take(q, b, l), _take(Al, b, l)
                acc = acc + sbp.D[a, b] * G.contract(flux(qa, qb, prm.gas), Aa + Ab)
            V[_index(V.ndim, a, l)] += acc
    return V


DIRICHLET, SLIP_WALL, NOSLIP_WALL = -1, -2, -3


def _face_links(nbr, orient, elems, f):
    """Neighbour element, neighbour face f' and orientation code across face f of ``elems``."""
    nb_e = nbr[elems, f]
    if orient is None:
        return nb_e, np.full(nb_e.shape, f ^ 1), np.zeros(nb_e.shape, dtype=int)
    o = orient[elems, f]
    return nb_e, o % 8, o // 8


def _reorient(face, code):
    """Partner values in the own face-node layout from the neighbour's face slice (trailing axes
    (b', a'))."""
    N = face.shape[-1]
    b, a = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    x, y = (b, a) if code & 1 else (a, b)
    ap = N - 1 - x if code & 2 else x
    bp = N - 1 - y if code & 4 else y
    return face[..., bp, ap]


def _nbr_face(arr_of_dir, nb_e, fp, code, f, p, signed=False):
    """Face-node values of the neighbours ``nb_e`` (all >= 0) across face f, in the own layout.
    ``arr_of_dir(l')`` gives the element array to take the neighbour's face l' from; ``signed``
    multiplies by -s s' (metric rows and contravariant fluxes of direction l')."""
    s = 1.0 if f & 1 else -1.0
    out = None
    for fv, cv in sorted(set(zip(fp.tolist(), code.tolist()))):
        sel = (fp == fv) & (code == cv)
        lp, sp = fv >> 1, (1.0 if fv & 1 else -1.0)
        src = arr_of_dir(lp)
        v = _reorient(_take(src[..., nb_e[sel], :, :, :], p if fv & 1 else 0, lp), cv)
        if signed:
            v = (-s * sp) * v
        if out is None:
            out = np.zeros(src.shape[:-4] + (len(nb_e),) + v.shape[-2:], dtype=v.dtype)
        out[..., sel, :, :] = v
    return out


def _partner(arr_of_dir, nbr, orient, elems, f, own, l, own_vals, signed=False):
    """Face-node values of the partner across face f (direction l) for the elements ``elems``: the
    neighbour's matching face node, or, on boundary faces, ``own_vals`` (the own face node's)."""
    nb_e, fp, code = _face_links(nbr, orient, elems, f)
    out = own_vals.copy()
    inn = nb_e >= 0
    if inn.any():
        out[..., inn, :, :] = _nbr_face(arr_of_dir, nb_e[inn], fp[inn], code[inn], f,
                                        own_vals.shape[-1] - 1, signed)
    return out


def _metric_rows(metric_all):
    return lambda lp: metric_all[3 * lp:3 * lp + 3]


def _slip_ghost(q, A):
    """Own state with the momentum reflected about the face with normal direction A."""
    mn = (q[1:4] * A).sum(0) / (A * A).sum(0)
    g = q.copy()
    g[1:4] = q[1:4] - 2.0 * mn * A
    return g


def _noslip_ghost(q):
    """Own state with the momentum reversed."""
    g = q.copy()
    g[1:4] = -q[1:4]
    return g


def _partner_state(q_all, metric_all, nbr, orient, elems, f, own, l, bc, gas):
    """Partner state across face f (direction l) for the elements ``elems``: the neighbour's node,
    or the ghost state of the boundary kind the neighbour index names."""
    nb_e = nbr[elems, f]
    bnd = nb_e < 0
    qi = _take(q_all[:, elems], own, l)
    qn = _partner(lambda lp: q_all, nbr, orient, elems, f, own, l, qi)
    if not bnd.any():
        return qn
    Ai = _take(metric_all[3 * l:3 * l + 3, elems], own, l)
    for code in np.unique(nb_e[bnd]):
        sel = nb_e == code
        if code == DIRICHLET:
            if bc is None:
                raise ValueError("Dirichlet boundary face without boundary data")
            qn[:, sel] = _take(bc[:, elems[sel]], own, l)
        elif code == SLIP_WALL:
            if gas.mu != 0.0:
                raise ValueError("slip walls are defined for inviscid problems only")
            qn[:, sel] = _slip_ghost(qi[:, sel], Ai[:, sel])
        elif code == NOSLIP_WALL:
            qn[:, sel] = _noslip_ghost(qi[:, sel])
        else:
            raise ValueError(f"unknown boundary kind {code}")
    return qn


def _partner_metric(metric_all, nbr, orient, elems, f, own, l):
    """Partner metric row of direction l (the neighbour's row l', signed; own row on boundaries)."""
    Ai = _take(metric_all[3 * l:3 * l + 3, elems], own, l)
    return Ai, _partner(_metric_rows(metric_all), nbr, orient, elems, f, own, l, Ai, signed=True)


def _partner_jac(jac_all, nbr, orient, elems, f, own, l):
    Ji = _take(jac_all[elems], own, l)
    return Ji, _partner(lambda lp: jac_all, nbr, orient, elems, f, own, l, Ji)


def inviscid_sat(q_all, metric_all, nbr, elems, sbp, prm: Params, bc=None, orient=None):
    """Interface SAT and local Lax-Friedrichs dissipation for the elements ``elems``; ``bc`` is
    the state prescribed on Dirichlet boundary faces."""
    flux = G.TWO_POINT[prm.two_point]
    gas = prm.gas
    q = q_all[:, elems]
    out = np.zeros_like(q)
    w_end = sbp.w[0]
    for l, s, f, own, nb in _faces(sbp.p):
        qi = _take(q, own, l)
        qn = _partner_state(q_all, metric_all, nbr, orient, elems, f, own, l, bc, gas)
        Ai, An = _partner_metric(metric_all, nbr, orient, elems, f, own, l)
        nbar = 0.5 * (Ai + An)
        sat = -(s / w_end) * (G.contract(flux(qi, qn, gas), nbar) - G.contract(G.euler_flux(qi, gas), Ai))
        if prm.iface_diss == 2:
            sat = sat - G.matrix_dissipation(qi, qn, nbar, gas) / (2.0 * w_end)
        elif prm.iface_diss:
            li, ln = G.max_wave_speed(qi, nbar, gas), G.max_wave_speed(qn, nbar, gas)
            lam = np.where(np.real(li) >= np.real(ln), li, ln)
            sat = sat - (lam / (2.0 * w_end)) * (qi - qn)
        out[_index(out.ndim, own, l)] += sat
    return out


def gradient_theta(q_all, metric_all, nbr, elems, sbp, prm: Params, bc=None, orient=None):
    """theta_a = D_a w + SAT^theta for the elements ``elems``, shape (3, 5, n, N, N, N)."""
    gas = prm.gas
    w = G.entropy_variables(q_all[:, elems], gas)
    th = np.stack([apply_D(sbp.D, w, a) for a in range(3)])
    w_end = sbp.w[0]
    for a, s, f, own, nb in _faces(sbp.p):
        wi = _take(w, own, a)
        wn = G.entropy_variables(_partner_state(q_all, metric_all, nbr, orient, elems, f, own, a, bc, gas), gas)
        th[a][_index(w.ndim, own, a)] += (s / (2.0 * w_end)) * (wn - wi)
    return th


def contravariant_viscous_flux(q_all, metric_all, jac_all, nbr, elems, sbp, prm: Params, bc=None,
                               orient=None):
    """fhat_l = sum_m A_lm F^V_m with F^V_m = sum_j C_mj g_j and g_j = sum_a A_aj theta_a / J;
    shape (3, 5, n, N, N, N)."""
    th = gradient_theta(q_all, metric_all, nbr, elems, sbp, prm, bc, orient)
    A = metric_all[:, elems]
    J = jac_all[elems]
    g = np.stack([sum(A[3 * a + j] * th[a] for a in range(3)) / J for j in range(3)])
    FV = G.viscous_flux(q_all[:, elems], g, prm.gas)
    return np.stack([sum(A[3 * l + m] * FV[m] for m in range(3)) for l in range(3)])


def chat_ll(q, A_l, J, gas):
    """Chat_ll = sum_{m,j} A_lm C_mj A_lj / J as 5x5 blocks, shape (5, 5, ...)."""
    C = G.viscous_blocks(q, gas)
    return sum(A_l[m] * C[m, j] * A_l[j] for m in range(3) for j in range(3)) / J


def viscous_term(q_all, metric_all, jac_all, nbr, elems, sbp, prm: Params, bc=None, orient=None):
    """sum_l D_l fhat_l + SAT^V + IP for the elements ``elems`` (eq. NSL, eq. MacroForm)."""
    gas = prm.gas
    elems = np.asarray(elems)
    ring = np.unique(np.concatenate([elems, nbr[elems].ravel()]))
    ring = ring[ring >= 0]
    pos = {int(e): i for i, e in enumerate(ring)}
    fh_ring = contravariant_viscous_flux(q_all, metric_all, jac_all, nbr, ring, sbp, prm, bc, orient)
    own_pos = np.array([pos[int(e)] for e in elems])
    fh = fh_ring[:, :, own_pos]
    out = sum(apply_D(sbp.D, fh[l], l) for l in range(3))
    w_end = sbp.w[0]
    q = q_all[:, elems]
    w = G.entropy_variables(q, gas)
    for l, s, f, own, nb in _faces(sbp.p):
        nb_e, fp, code = _face_links(nbr, orient, elems, f)
        bnd = nb_e < 0
        fi = _take(fh[l], own, l)
        fn = fi.copy()
        if (~bnd).any():
            ring_nb = np.array([pos[int(e)] for e in nb_e[~bnd]])
            fn[:, ~bnd] = _nbr_face(lambda lp: fh_ring[lp], ring_nb, fp[~bnd], code[~bnd], f, sbp.p,
                                    signed=True)
        sat_v = (s / (2.0 * w_end)) * (fn - fi)
        sat_v[:, bnd] = 0.0   # Dirichlet: the boundary viscous flux is the own one
        wall = nb_e == NOSLIP_WALL
        sat_v[4, wall] = -(s / w_end) * fi[4, wall]   # adiabatic wall: zero energy flux
        # interior penalty
        qi = _take(q, own, l)
        qn = _partner_state(q_all, metric_all, nbr, orient, elems, f, own, l, bc, gas)
        wi, wn = _take(w, own, l), G.entropy_variables(qn, gas)
        Ai, An = _partner_metric(metric_all, nbr, orient, elems, f, own, l)
        Ji, Jn = _partner_jac(jac_all, nbr, orient, elems, f, own, l)
        Lm = 0.5 * (chat_ll(qi, Ai, Ji, gas) + chat_ll(qn, An, Jn, gas))
        ip = -(prm.eta / w_end) * np.einsum("ab...,b...->a...", Lm, wi - wn)
        out[_index(out.ndim, own, l)] += sat_v + ip
    return out


def residual(q_all, metric_all, jac_all, nbr, sbp, prm: Params, elems=None, chunk=None, bc=None,
             source=None, orient=None):
    """dq/dt for the elements ``elems`` (all by default), shape (5, n, N, N, N).

    ``chunk`` splits the element list into groups evaluated one after another (memory only).
    ``bc`` (shape of q) holds the state read at the face nodes of Dirichlet boundary faces
    (neighbour index -1; walls, -2 and -3, need no data); ``source`` (shape of q) is added to
    dq/dt; ``orient`` ([K, 6], f' + 8 code) gives the neighbour face and orientation of every
    interior face (None: aligned faces).
    """
    K = q_all.shape[1]
    if elems is None:
        elems = np.arange(K)
    elems = np.asarray(elems)
    if chunk is not None and len(elems) > chunk:
        return np.concatenate([residual(q_all, metric_all, jac_all, nbr, sbp, prm,
                                        elems[i:i + chunk], bc=bc, source=source, orient=orient)
                               for i in range(0, len(elems), chunk)], axis=1)
    q = q_all[:, elems]
    rhs = -volume_term(q, metric_all[:, elems], sbp, prm)
    rhs = rhs + inviscid_sat(q_all, metric_all, nbr, elems, sbp, prm, bc, orient)
    if prm.gas.mu != 0.0:
        rhs = rhs + viscous_term(q_all, metric_all, jac_all, nbr, elems, sbp, prm, bc, orient)
    out = rhs / jac_all[elems]
    if source is not None:
        out = out + source[:, elems]
    return out


def rk4_step(f, q, dt):
    """Classical fourth-order Runge-Kutta step with fixed dt for dq/dt = f(q)."""
    k1 = f(q)
    k2 = f(q + 0.5 * dt * k1)
    k3 = f(q + 0.5 * dt * k2)
    k4 = f(q + dt * k3)
    return q + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
