"""Python entry points over the C ABI.  Every step of the residual runs in the HIP library; torch
provides device memory and the current stream only."""
from __future__ import annotations

import ctypes
import sys
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

F64 = torch.float64


def lgl_operator(p: int):
    """(x, w, D) of the degree-p LGL SBP operator, computed by the library (host)."""
    N = p + 1
    x = np.zeros(N)
    w = np.zeros(N)
    D = np.zeros(N * N)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().sbp_lgl_operator(p, x.ctypes.data_as(dp), w.ctypes.data_as(dp), D.ctypes.data_as(dp)),
          "sbp_lgl_operator")
    return x, w, D.reshape(N, N)


def schedule_count(p: int) -> int:
    return int(lib().sbp_schedule_count(p))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, name):
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")


def metrics(p: int, coords: torch.Tensor):
    """Curl-form metric terms (9, nodes) and Jacobian (nodes,) from device coordinates (3, nodes)."""
    N3 = (p + 1) ** 3
    if coords.numel() == 0 or coords.numel() % (3 * N3) != 0:
        raise ValueError(f"coords has {coords.numel()} entries, not a positive multiple of "
                         f"3 (p+1)^3 = {3 * N3}")
    _need(coords, F64, "coords")
    nodes = coords.numel() // 3
    K = nodes // N3
    metric = torch.empty((9, nodes), dtype=F64, device=coords.device)
    jac = torch.empty((nodes,), dtype=F64, device=coords.device)
    check(lib().sbp_metrics(p, K, _ptr(coords), _ptr(metric), _ptr(jac), _stream()), "sbp_metrics")
    return metric, jac


def metrics_optimized(p: int, nbr: torch.Tensor, dxdxi: torch.Tensor):
    """Optimised metric terms (9, nodes) and Jacobian (nodes,) from the mapping derivative at the
    nodes (9, nodes), entry 3 m + i = dx_m/dxi_i, on the aligned conforming mesh of the neighbour
    table nbr (K, 6): analytic face values corrected so that every element can meet the discrete
    GCL, then the least-norm volume correction that meets it."""
    N3 = (p + 1) ** 3
    if dxdxi.numel() == 0 or dxdxi.numel() % (9 * N3) != 0:
        raise ValueError(f"dxdxi has {dxdxi.numel()} entries, not a positive multiple of "
                         f"9 (p+1)^3 = {9 * N3}")
    _need(dxdxi, F64, "dxdxi")
    nodes = dxdxi.numel() // 9
    K = nodes // N3
    _need(nbr, torch.int32, "nbr")
    if nbr.numel() != 6 * K:
        raise ValueError(f"nbr has {nbr.numel()} entries, expected 6 K = {6 * K}")
    if nbr.device != dxdxi.device:
        raise ValueError("nbr and dxdxi are on different devices")
    metric = torch.empty((9, nodes), dtype=F64, device=dxdxi.device)
    jac = torch.empty((nodes,), dtype=F64, device=dxdxi.device)
    check(lib().sbp_metrics_optimized(p, K, _ptr(nbr), _ptr(dxdxi), _ptr(metric), _ptr(jac),
                                      _stream()), "sbp_metrics_optimized")
    return metric, jac


@dataclass
class Problem:
    """One problem on the device: degree, element count, neighbour table (negative entries are
    boundary kinds), metrics, constants, and optionally Dirichlet boundary data, a source term and
    the face-orientation table of an unstructured mesh."""

    p: int
    n_elem: int
    nbr: torch.Tensor       # int32 (K, 6)
    metric: torch.Tensor    # float64 (9, nodes)
    jac: torch.Tensor       # float64 (nodes,)
    gamma: float = 1.4
    R: float = 1.0
    mu: float = 0.0
    Pr: float = 0.72
    eta: float = 1.0
    iface_diss: int = 1
    two_point: int = 0
    bc_state: Optional[torch.Tensor] = None   # float64 (5, nodes): Dirichlet state, faces with nbr -1
    source: Optional[torch.Tensor] = None     # float64 (5, nodes): added to dq/dt
    face_orient: Optional[torch.Tensor] = None  # int32 (K, 6): f' + 8 code per face; None aligned

    @property
    def nodes(self) -> int:
        return self.n_elem * (self.p + 1) ** 3

    def arrays(self):
        """(name, tensor, dtype, expected entries) of every device array of the problem."""
        out = [("nbr", self.nbr, torch.int32, 6 * self.n_elem), ("metric", self.metric, F64, 9 * self.nodes),
               ("jac", self.jac, F64, self.nodes)]
        for name in ("bc_state", "source"):
            if getattr(self, name) is not None:
                out.append((name, getattr(self, name), F64, 5 * self.nodes))
        if self.face_orient is not None:
            out.append(("face_orient", self.face_orient, torch.int32, 6 * self.n_elem))
        return out

    def c_struct(self) -> _lib.sbp_problem:
        """The C struct; raises ValueError for arrays of the wrong size, dtype, layout or device
        (the library reads them through raw pointers and cannot check their extent)."""
        if self.n_elem <= 0:
            raise ValueError("n_elem must be positive")
        arrs = self.arrays()
        for name, t, dtype, n in arrs:
            if t.numel() != n:
                raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
        for name, t, dtype, n in arrs:
            _need(t, dtype, name)
        if len({t.device for _, t, _, _ in arrs}) != 1:
            raise ValueError("the arrays of a problem must be on one device")
        extra = [None if t is None else t.data_ptr() for t in (self.bc_state, self.source, self.face_orient)]
        return _lib.sbp_problem(self.p, self.iface_diss, self.n_elem, self.nbr.data_ptr(),
                                self.metric.data_ptr(), self.jac.data_ptr(), self.gamma, self.R,
                                self.mu, self.Pr, self.eta, self.two_point, 0, *extra)


class ProblemSet:
    """Problems evaluated together (n = 1: plain path; n > 1: batched path) with their workspace."""

    def __init__(self, problems: Sequence[Problem]):
        self.problems: List[Problem] = list(problems)
        n = len(self.problems)
        self._arr = (_lib.sbp_problem * n)(*[p.c_struct() for p in self.problems])
        self.n = n
        self.ws_bytes = int(lib().sbp_workspace_bytes(self._arr, n))
        if self.ws_bytes == 0:
            raise _lib.SBPError(_lib.SBP_ERR_ARG, "sbp_workspace_bytes")
        dev = self.problems[0].metric.device
        if any(p.metric.device != dev for p in self.problems):
            raise ValueError("the problems of a set must be on one device")
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.total_nodes = sum(p.nodes for p in self.problems)

    def release(self) -> int:
        """Drops the library's cached launch plans and RK4 graphs of this set (they are made again
        on the next call); returns how many were released.  Also done when the set is collected."""
        ws = getattr(self, "ws", None)
        if ws is None:
            return 0
        rc = lib().sbp_release(_ptr(ws))
        if rc < 0:
            check(rc, "sbp_release")
        return rc

    def __del__(self):
        if sys.is_finalizing() or getattr(self, "ws", None) is None:
            return
        try:
            self.release()
        except Exception:  # pragma: no cover - runtime already torn down
            pass

    def state_numel(self) -> int:
        return 5 * self.total_nodes

    def _check_state(self, t, name):
        _need(t, F64, name)
        if t.device != self.ws.device:
            raise ValueError(f"{name} is on {t.device}, the problem set on {self.ws.device}")
        if t.numel() != self.state_numel():
            raise ValueError(f"{name} has {t.numel()} entries, expected {self.state_numel()}")

    def residual(self, q: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check_state(q, "q")
        if out is None:
            out = torch.empty_like(q)
        self._check_state(out, "out")
        check(lib().sbp_residual(self._arr, self.n, _ptr(q), _ptr(out), _ptr(self.ws), self.ws_bytes,
                                 _stream()), "sbp_residual")
        return out

    def residual_noalloc(self, q: torch.Tensor, out: Optional[torch.Tensor] = None,
                         status: Optional[torch.Tensor] = None):
        """The residual through sbp_residual_noalloc: no workspace (the library's own device scratch
        instead) and no allocation inside the call.  ``status`` is a device int32 tensor of one
        entry that receives the flag bits (zeroed here if not given).  Returns (out, status)."""
        self._check_state(q, "q")
        if out is None:
            out = torch.empty_like(q)
        self._check_state(out, "out")
        if status is None:
            status = torch.zeros(1, dtype=torch.int32, device=q.device)
        _need(status, torch.int32, "status")
        check(lib().sbp_residual_noalloc(self._arr, self.n, _ptr(q), _ptr(out), _ptr(status), _stream()),
              "sbp_residual_noalloc")
        return out, status

    def profile_residual(self, q: torch.Tensor, out: torch.Tensor, wait: bool = True):
        """Runs the residual once with HIP events around the main kernel.  wait=True returns its
        duration in ms; wait=False only records the events (read later by profile_collect())."""
        self._check_state(q, "q")
        self._check_state(out, "out")
        ms = ctypes.c_float(0.0)
        check(lib().sbp_profile_residual(self._arr, self.n, _ptr(q), _ptr(out), _ptr(self.ws),
                                         self.ws_bytes, _stream(), ctypes.byref(ms) if wait else None),
              "sbp_profile_residual")
        return float(ms.value) if wait else None

    def autotune(self, q: torch.Tensor, reps: int = 3):
        """Times every residual schedule on these inputs and keeps the fastest per group; returns
        the schedule index chosen for each problem."""
        self._check_state(q, "q")
        out = torch.empty_like(q)
        chosen = (ctypes.c_int32 * self.n)()
        check(lib().sbp_autotune(self._arr, self.n, _ptr(q), _ptr(out), _ptr(self.ws), self.ws_bytes,
                                 _stream(), reps, chosen), "sbp_autotune")
        return list(chosen)

    def set_schedule(self, p: int, variant: int):
        check(lib().sbp_set_schedule(self._arr, self.n, _ptr(self.ws), self.ws_bytes, p, variant),
              "sbp_set_schedule")

    def rk_step(self, q: torch.Tensor, dt: torch.Tensor, n_steps: int = 1) -> torch.Tensor:
        """In-place classical RK4 steps; dt is a device float64 tensor with one entry per problem."""
        self._check_state(q, "q")
        _need(dt, F64, "dt")
        if dt.device != self.ws.device:
            raise ValueError(f"dt is on {dt.device}, the problem set on {self.ws.device}")
        if dt.numel() != self.n:
            raise ValueError("dt needs one entry per problem")
        check(lib().sbp_rk_step(self._arr, self.n, _ptr(q), _ptr(dt), n_steps, _ptr(self.ws),
                                self.ws_bytes, _stream()), "sbp_rk_step")
        return q

    def residual_vjp(self, q: torch.Tensor, gbar: torch.Tensor, out: Optional[torch.Tensor] = None):
        self._check_state(q, "q")
        self._check_state(gbar, "gbar")
        if out is None:
            out = torch.empty_like(q)
        self._check_state(out, "out")
        check(lib().sbp_residual_vjp(self._arr, self.n, _ptr(q), _ptr(gbar), _ptr(out), _ptr(self.ws),
                                     self.ws_bytes, _stream()), "sbp_residual_vjp")
        return out

    def status(self) -> int:
        """Waits for the stream; raises SBPError if a non-physical state or bad neighbour was seen."""
        flags = ctypes.c_int32(0)
        rc = lib().sbp_status(_ptr(self.ws), _stream(), ctypes.byref(flags))
        check(rc, "sbp_status")
        return flags.value


def profile_collect():
    """(count, total ms) of the main-kernel launches recorded with profile_residual(wait=False)
    since the last call; waits for them."""
    n = ctypes.c_int32(0)
    tot = ctypes.c_double(0.0)
    check(lib().sbp_profile_collect(ctypes.byref(n), ctypes.byref(tot)), "sbp_profile_collect")
    return int(n.value), float(tot.value)


class SBPResidual(torch.autograd.Function):
    """dq/dt = residual(q) with the hand-written vector-Jacobian product as its backward."""

    @staticmethod
    def forward(ctx, q, pset: ProblemSet):
        ctx.pset = pset
        ctx.save_for_backward(q)
        return pset.residual(q.contiguous())

    @staticmethod
    def backward(ctx, gbar):
        (q,) = ctx.saved_tensors
        return ctx.pset.residual_vjp(q.contiguous(), gbar.contiguous()), None
