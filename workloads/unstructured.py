"""Unstructured relabelling of hexahedral meshes (mesh bookkeeping only, no arithmetic of the method).

* ``cube_rotations()``: the 24 rotations of the reference cube as signed permutation matrices M
  (new reference coordinates xi' = M xi; det M = +1, so J stays positive).
* ``relabel(arr, M)``: an element array with axes (..., i3, i2, i1) seen in the turned frame.
* ``rotate_elements(arr, rots)``: every element turned by its own rotation.
* ``connectivity(x, L)``: the face table of a mesh found from the node coordinates (modulo the
  period L): for face f = 2 l + side of element e, the neighbour element, and
  ``orient[e, f] = f' + 8 code`` with f' the neighbour's face and code its orientation.  With the
  own face-node coordinates (a, b) (tangential indices in increasing direction order), the partner
  node has (a', b') = (F_a(x), F_b(y)), (x, y) = (b, a) if bit 0 of code is set, else (a, b), and
  F_a, F_b reversals (N - 1 - .) when bits 1, 2 are set.
"""
from __future__ import annotations

import itertools

import numpy as np


def cube_rotations():
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3), dtype=int)
            for r in range(3):
                M[r, perm[r]] = signs[r]
            if round(np.linalg.det(M)) == 1:
                out.append(M)
    return out


def relabel(arr, M):
    """arr (..., N, N, N) with axes (i3, i2, i1) -> the same nodes indexed in the frame xi' = M xi."""
    nd = arr.ndim
    axes = list(range(nd))
    flips = []
    for r in range(3):
        c = int(np.nonzero(M[r])[0][0])
        axes[nd - 1 - r] = nd - 1 - c
        if M[r, c] < 0:
            flips.append(nd - 1 - r)
    out = np.transpose(arr, axes)
    if flips:
        out = np.flip(out, axis=tuple(flips))
    return np.ascontiguousarray(out)


def rotate_elements(arr, rots):
    """arr (..., K, N, N, N): element e relabelled by cube_rotations()[rots[e]]."""
    R = cube_rotations()
    out = np.empty_like(arr)
    for e in range(arr.shape[-4]):
        out[..., e, :, :, :] = relabel(arr[..., e, :, :, :], R[rots[e]])
    return out


def _face(x, f):
    """Face-node slice (..., K, b, a) of face f."""
    l, side = f >> 1, f & 1
    idx = x.shape[-1] - 1 if side else 0
    return np.take(x, idx, axis=x.ndim - 1 - l)


def orient_face(face, code):
    """A neighbour's face slice (..., b', a') laid out in the own face-node order."""
    N = face.shape[-1]
    b, a = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    xx, yy = (b, a) if code & 1 else (a, b)
    ap = N - 1 - xx if code & 2 else xx
    bp = N - 1 - yy if code & 4 else yy
    return face[..., bp, ap]


def connectivity(x, L, boundary=-1, periods=None):
    """(nbr, orient) of the mesh with node coordinates x (3, K, N, N, N), faces matched modulo the
    period of each coordinate (``periods``, default L for all three; None: not periodic);
    unmatched faces get the neighbour index ``boundary``."""
    K = x.shape[1]
    P = [L, L, L] if periods is None else list(periods)
    faces = [_face(x, f) for f in range(6)]        # (3, K, N, N) each
    res = 1 << 20

    def wrap(v, d):
        return v if P[d] is None else v - P[d] * np.round(v / P[d])

    def key(e, f):
        c = faces[f][:, e].reshape(3, -1).mean(axis=1)
        k = []
        for d in range(3):
            if P[d] is None:
                k.append(int(np.round(c[d] / L * res)))
            else:
                k.append(int(np.round((c[d] / P[d]) % 1.0 * res)) % res)
        return tuple(k)

    table = {}
    for e in range(K):
        for f in range(6):
            table.setdefault(key(e, f), []).append((e, f))
    nbr = np.full((K, 6), boundary, dtype=np.int32)
    orient = np.zeros((K, 6), dtype=np.int32)
    tol = 1e-9 * L

    def same(u, v):
        return all(np.all(np.abs(wrap(u[d] - v[d], d)) < tol) for d in range(3))

    for ents in table.values():
        if len(ents) == 1:
            continue
        assert len(ents) == 2, "a face shared by more than two elements"
        for (e, f), (e2, f2) in (ents, ents[::-1]):
            codes = [c for c in range(8) if same(faces[f][:, e], orient_face(faces[f2][:, e2], c))]
            assert len(codes) == 1, "faces do not conform"
            nbr[e, f] = e2
            orient[e, f] = f2 + 8 * codes[0]
    return nbr, orient
