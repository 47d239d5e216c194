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


# ------------------------------------------------------------------------------------------
# Optimised metric terms (section on the linear convection-diffusion equation, the paragraph after
# eq. discGCLconvection): the surface metric terms are the analytic ones, and the volume metric
# terms are the solution of the discrete GCL closest to the analytic volume metrics.  The paper
# defers the procedure to another work; the reading implemented here:
#  1. analytic metrics A_l = a_{l+1} x a_{l+2} (a_i = dx/dxi_i, cyclic) and J = det(dx/dxi) at every
#     node, from the closed-form mapping derivative;
#  2. with the normal components on the faces (A_lm at the nodes of the faces xi_l = -1, +1) held,
#     the GCL sum_l D_l [A_lm] 1 = 0 of an element can be met only if those values satisfy eight
#     linear conditions (the left null space of the GCL operator restricted to the other entries,
#     spanned by tensor products of P 1 and the left null vector of D along each direction; the P 1
#     x P 1 x P 1 condition says that the LGL quadrature of the outward normal metrics over the
#     element surface vanishes).  The analytic values meet them only up to quadrature errors, so
#     the surface metric terms are the analytic ones plus the minimum-norm correction, over all
#     face-node values of the mesh (one value per face node, shared by the two elements of an
#     interior face), for which every element meets its conditions;
#  3. in every element, for each m, the remaining entries move by the minimum-norm amount that
#     makes the GCL hold.
# Degrees p >= 2 (at p = 1 every node is a face node and nothing is left to optimise).
# ------------------------------------------------------------------------------------------
def analytic_metrics(dxdxi):
    """Metric terms (9, K, N, N, N), entry 3l + m = (a_{l+1} x a_{l+2})_m, and J = det(dx/dxi), from
    dxdxi[m][i] = dx_m/dxi_i."""
    a = [np.stack([dxdxi[m][i] for m in range(3)]) for i in range(3)]   # covariant basis vectors
    rows = []
    for l in range(3):
        u, v = a[(l + 1) % 3], a[(l + 2) % 3]
        rows.append(np.stack([u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2],
                              u[0] * v[1] - u[1] * v[0]]))
    J = (a[0] * rows[0]).sum(0)
    return np.concatenate(rows), J


def _face_slice(l, side, N):
    """Index of the face xi_l = -1 (side 0) or +1 (side 1) in element arrays (..., i3, i2, i1)."""
    sl = [slice(None)] * 3
    sl[2 - l] = (N - 1) if side else 0
    return (Ellipsis,) + tuple(sl)


def surface_closure(metric, w):
    """Per element and m, the LGL quadrature of the outward normal metric over the element surface:
    sum over faces (l, s) of s * sum_face w_a w_b A_lm; shape (K, 3)."""
    N = w.size
    W2 = np.outer(w, w)
    c = np.zeros((metric.shape[1], 3), dtype=metric.dtype)
    for l in range(3):
        for side, s in ((0, -1.0), (1, 1.0)):
            for m in range(3):
                face = metric[3 * l + m][_face_slice(l, side, N)]    # (K, b, a)
                c[:, m] += s * (face * W2).sum(axis=(1, 2))
    return c


def gcl_operator(D):
    """For one element, with a = (A_1m, A_2m, A_3m) flattened (node index i1 + N i2 + N^2 i3 in each
    block), M a = sum_l D_l A_lm.  Returns M, the mask of the held entries (normal components on
    the faces), the pseudo-inverse of M on the other entries, and a basis Y of the left null space
    of M on the other entries (the compatibility conditions Y^T M a = 0 on the held entries)."""
    N = D.shape[0]
    I = np.eye(N)
    Ds = [np.kron(np.kron(I, I), D), np.kron(np.kron(I, D), I), np.kron(np.kron(D, I), I)]
    M = np.hstack(Ds)
    n = N ** 3
    idx = np.indices((N, N, N)).reshape(3, -1)          # (i3, i2, i1) of each flattened node
    held = np.zeros(3 * n, dtype=bool)
    for l in range(3):
        il = idx[2 - l]
        held[l * n:(l + 1) * n] = (il == 0) | (il == N - 1)
    U, S, Vt = np.linalg.svd(M[:, ~held], full_matrices=True)
    rank = int((S > 1e-12 * S[0]).sum())
    pinv = (Vt[:rank].T / S[:rank]) @ U[:, :rank].T
    Y = U[:, rank:]
    return M, held, pinv, Y


def surface_system(sbp, nbr):
    """The compatibility conditions of all elements as one linear system on the face-node values of
    the mesh: G (sparse, 8 rows per element) acting on one value per face node (faces numbered in
    order of first appearance, N^2 values each), and cols[e, j], the face-node value that held
    entry j of element e stands for."""
    import scipy.sparse as sp
    N = sbp.N
    n = N ** 3
    K = nbr.shape[0]
    M, held, _, Y = gcl_operator(sbp.D)
    C = Y.T @ M[:, held]                                  # (conditions, held entries)
    k = C.shape[0]
    held_idx = np.nonzero(held)[0]
    # held entry -> (face f of the element, tangential index t = ta + N tb)
    idx = np.indices((N, N, N)).reshape(3, -1)
    ent_face = np.empty(held_idx.size, dtype=np.int64)
    ent_t = np.empty(held_idx.size, dtype=np.int64)
    for h, j in enumerate(held_idx):
        l, node = divmod(int(j), n)
        i3, i2, i1 = idx[:, node]
        il = (i1, i2, i3)[l]
        ta, tb = [v for d, v in enumerate((i1, i2, i3)) if d != l]
        ent_face[h] = 2 * l + (1 if il == N - 1 else 0)
        ent_t[h] = ta + N * tb
    face_id = -np.ones((K, 6), dtype=np.int64)
    nf = 0
    for e in range(K):
        for f in range(6):
            if face_id[e, f] >= 0:
                continue
            face_id[e, f] = nf
            nb = int(nbr[e, f])
            if nb >= 0:
                assert face_id[nb, f ^ 1] < 0 and int(nbr[nb, f ^ 1]) == e, "aligned conforming faces only"
                face_id[nb, f ^ 1] = nf
            nf += 1
    cols = face_id[:, ent_face] * (N * N) + ent_t[None, :]          # (K, held entries)
    rows = np.arange(K * k).reshape(K, k)
    G = sp.csr_matrix((np.broadcast_to(C[None], (K, k, held_idx.size)).ravel(),
                       (np.repeat(rows, held_idx.size, axis=1).ravel(),
                        np.broadcast_to(cols[:, None, :], (K, k, held_idx.size)).ravel())),
                      shape=(K * k, nf * N * N))
    return G, cols, held


def surface_metrics(metric, sbp, nbr):
    """Step 2: the metric terms with the normal components at the face nodes replaced by one value
    per face node of the mesh: the mean of the values of the elements sharing the node (they differ
    by rounding only) plus the minimum-norm correction for which every element meets its
    compatibility conditions.  Also returns the corrections, (3, face-node values)."""
    N = sbp.N
    n = N ** 3
    K = metric.shape[1]
    G, cols, held = surface_system(sbp, nbr)
    # minimum-norm solution x = G^T y, (G G^T) y = rhs, with the eigenvalues of G G^T below 1e-12 of
    # the squared norm of one element's conditions dropped (directions the constraints cannot move;
    # rounding noise of rhs along them would otherwise be amplified).  The scale is that of the
    # conditions themselves, not the largest eigenvalue of the mesh's G G^T: on a mesh where every
    # condition vanishes identically (one element, periodic: its opposite faces are one face) all
    # eigenvalues are rounding noise and none may be kept.  Dense: meant for the mesh sizes of the
    # tests.
    M, held_e, _, Y = gcl_operator(sbp.D)
    c_scale = np.linalg.norm(Y.T @ M[:, held_e], 2) ** 2
    gram = (G @ G.T).toarray()
    lam, V = np.linalg.eigh(gram)
    keep = lam > 1e-12 * c_scale
    count = np.zeros(G.shape[1])
    np.add.at(count, cols.ravel(), 1.0)
    out = metric.copy()
    xs = []
    for m in range(3):
        a = np.concatenate([metric[3 * l + m].reshape(K, n) for l in range(3)], axis=1)
        base = np.zeros(G.shape[1])
        np.add.at(base, cols.ravel(), a[:, held].ravel())
        base /= count
        rhs = -(G @ base)
        y = V[:, keep] @ ((V[:, keep].T @ rhs) / lam[keep])
        x = G.T @ y
        a[:, held] = (base + x)[cols]
        for l in range(3):
            out[3 * l + m] = a[:, l * n:(l + 1) * n].reshape(K, N, N, N)
        xs.append(x)
    return out, np.stack(xs)


def optimized_metrics(dxdxi, nbr, sbp):
    """Metric terms (9, K, N, N, N) and J by steps 1-3 above, for aligned conforming meshes."""
    metric, J = analytic_metrics(dxdxi)
    metric, _ = surface_metrics(metric, sbp, nbr)
    M, held, pinv, _ = gcl_operator(sbp.D)
    free = ~held
    K = metric.shape[1]
    N = sbp.N
    n = N ** 3
    for m in range(3):
        a = np.concatenate([metric[3 * l + m].reshape(K, n) for l in range(3)], axis=1)  # (K, 3n)
        r = -(a @ M.T)                                   # (K, n)
        a[:, free] += r @ pinv.T
        for l in range(3):
            metric[3 * l + m] = a[:, l * n:(l + 1) * n].reshape(K, N, N, N)
    return metric, J
