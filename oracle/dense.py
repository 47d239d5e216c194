"""Literal matrix form of the residual on tiny meshes (eqs. discEL, NSL, Chatij).

Independent of ``residual.py`` in everything but the pointwise physics:
* nodes are ordered as in the paper's tensor products (xi_3 fastest), with
  D_xi1 = D (x) I (x) I, D_xi2 = I (x) D (x) I, D_xi3 = I (x) I (x) D as explicit matrices;
* the inviscid volume term is ((D_l A_lm + A_lm D_l) o F_m) 1 with the full matrix F_m of
  two-point fluxes between every pair of nodes of the element;
* the viscous term is sum_{l,a} D_l [Chat_la] theta_a with the explicit 5x5 blocks
  Chat_la = sum_{m,j} A_lm C_mj A_aj / J;
* interface partners are found from the physical coordinates of the face nodes (modulo the
  period), not from a neighbour table.
Only sensible for a few hundred nodes.
"""
from __future__ import annotations

import numpy as np

from . import gas as G


def _to_paper(u, N):
    """(..., K, i3, i2, i1) -> (..., K, N^3) with local index i3 + N i2 + N^2 i1."""
    v = np.swapaxes(u, -1, -3)
    return v.reshape(v.shape[:-3] + (N ** 3,))


def _from_paper(v, N):
    u = v.reshape(v.shape[:-1] + (N, N, N))
    return np.swapaxes(u, -1, -3)


class DenseMesh:
    def __init__(self, x, metric, jac, sbp, L):
        N = sbp.N
        self.N, self.p, self.sbp = N, sbp.p, sbp
        I = np.eye(N)
        self.Dl = [np.kron(np.kron(sbp.D, I), I), np.kron(np.kron(I, sbp.D), I),
                   np.kron(np.kron(I, I), sbp.D)]
        self.x = _to_paper(x, N)            # (3, K, N^3)
        self.A = _to_paper(metric, N)       # (9, K, N^3)
        self.J = _to_paper(jac, N)          # (K, N^3)
        self.K = self.J.shape[0]
        loc = np.arange(N ** 3)
        self.ijk = [loc // (N * N), (loc // N) % N, loc % N]   # i1, i2, i3 of each local node
        self.pairs = self._match_faces(L)

    def _face_nodes(self, l, s):
        target = 0 if s < 0 else self.p
        return np.nonzero(self.ijk[l] == target)[0]

    def _match_faces(self, L):
        tol = 1e-8 * L

        def mod_close(d):
            return np.all(np.abs(d - L * np.round(d / L)) < tol, axis=0)

        pairs = []
        for l in range(3):
            for s in (-1.0, 1.0):
                own = self._face_nodes(l, s)
                opp = self._face_nodes(l, -s)
                for e in range(self.K):
                    c = self.x[:, e, own].mean(axis=1)
                    partner = None
                    for e2 in range(self.K):
                        c2 = self.x[:, e2, opp].mean(axis=1)
                        if mod_close((c - c2)[:, None])[0]:
                            partner = e2
                            break
                    assert partner is not None, "no matching face"
                    for i in own:
                        d = self.x[:, partner, opp] - self.x[:, e, i][:, None]
                        hit = np.nonzero(mod_close(d))[0]
                        assert len(hit) == 1
                        pairs.append((e, int(i), l, s, partner, int(opp[hit[0]])))
        return pairs


def residual(q_storage, mesh: DenseMesh, prm):
    gas = prm.gas
    flux = G.TWO_POINT[prm.two_point]
    N, K = mesh.N, mesh.K
    q = _to_paper(q_storage, N)                         # (5, K, N^3)
    w_end = mesh.sbp.w[0]
    ones = np.ones(N ** 3)
    rhs = np.zeros_like(q)
    # inviscid volume: ((D_l A_lm + A_lm D_l) o F_m) 1
    for e in range(K):
        qe = q[:, e]
        F = flux(qe[:, :, None], qe[:, None, :], gas)     # (3, 5, N^3, N^3)
        for l in range(3):
            for m in range(3):
                Alm = np.diag(mesh.A[3 * l + m, e])
                Mat = mesh.Dl[l] @ Alm + Alm @ mesh.Dl[l]
                for c in range(5):
                    rhs[c, e] -= (Mat * F[m, c]) @ ones
    # inviscid interface coupling
    for (e, i, l, s, e2, i2) in mesh.pairs:
        qi, qn = q[:, e, i], q[:, e2, i2]
        Ai, An = mesh.A[3 * l:3 * l + 3, e, i], mesh.A[3 * l:3 * l + 3, e2, i2]
        nbar = 0.5 * (Ai + An)
        sat = -(s / w_end) * (G.contract(flux(qi, qn, gas), nbar) - G.contract(G.euler_flux(qi, gas), Ai))
        if prm.iface_diss:
            nn = np.sqrt(np.dot(nbar, nbar))
            lam = []
            for qx in (qi, qn):
                rho, u, P, T = G.primitives(qx, gas)
                un = np.dot(u, nbar)
                lam.append((un if np.real(un) >= 0 else -un) + G.sound_speed(qx, gas) * nn)
            lm = lam[0] if np.real(lam[0]) >= np.real(lam[1]) else lam[1]
            sat = sat - lm / (2.0 * w_end) * (qi - qn)
        rhs[:, e, i] += sat
    if gas.mu != 0.0:
        w = G.entropy_variables(q, gas)                     # (5, K, N^3)
        theta = np.stack([np.stack([(mesh.Dl[a] @ w[:, e].T).T for e in range(K)], axis=1)
                          for a in range(3)])               # (3, 5, K, N^3)
        for (e, i, l, s, e2, i2) in mesh.pairs:
            theta[l, :, e, i] += (s / (2.0 * w_end)) * (w[:, e2, i2] - w[:, e, i])
        C = G.viscous_blocks(q, gas)                        # (3, 3, 5, 5, K, N^3)
        A = mesh.A
        Chat = np.zeros((3, 3, 5, 5, K, N ** 3), dtype=np.result_type(q.dtype, np.float64))
        for l in range(3):
            for a in range(3):
                Chat[l, a] = sum(A[3 * l + m] * C[m, j] * A[3 * a + j]
                                 for m in range(3) for j in range(3)) / mesh.J
        fh = np.einsum("lacd...,ad...->lc...", Chat, theta)  # (3, 5, K, N^3)
        for e in range(K):
            for l in range(3):
                rhs[:, e] += (mesh.Dl[l] @ fh[l, :, e].T).T
        for (e, i, l, s, e2, i2) in mesh.pairs:
            rhs[:, e, i] += (s / (2.0 * w_end)) * (fh[l, :, e2, i2] - fh[l, :, e, i])
            Lm = 0.5 * (Chat[l, l, :, :, e, i] + Chat[l, l, :, :, e2, i2])
            rhs[:, e, i] -= (prm.eta / w_end) * Lm @ (w[:, e, i] - w[:, e2, i2])
    return _from_paper(rhs / mesh.J, N)
