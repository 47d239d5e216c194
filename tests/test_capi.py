"""The C-ABI library loads on a host without a GPU and exports every symbol of include/sbp.h;
host-only entry points (the 1-D operator, argument checks) work without a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1911_10966_amd as P
from paper_1911_10966_amd import _lib
from oracle import operators

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sbp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*\*?(sbp_\w+)\s*\(", src, re.M)))


def test_header_matches_binding():
    assert declared_functions() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = P.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.sbp_version() >= 100


@pytest.mark.parametrize("p", list(range(1, 16)))
def test_lgl_operator_matches_oracle(p):
    x, w, D = P.lgl_operator(p)
    o = operators.SBP1D(p)
    assert np.abs(x - o.x).max() < 1e-15
    assert np.abs(w - o.w).max() < 1e-15
    assert np.abs(D - o.D).max() < 1e-13 * p * p


def test_lgl_operator_rejects_bad_degree():
    dp = ctypes.POINTER(ctypes.c_double)
    assert P.lib().sbp_lgl_operator(0, None, None, None) == _lib.SBP_ERR_DEGREE
    assert P.lib().sbp_lgl_operator(16, None, None, None) == _lib.SBP_ERR_DEGREE


def test_argument_errors_on_host():
    L = P.lib()
    pr = _lib.sbp_problem(3, 1, 8, 64, 64, 64, 1.4, 1.0, 0.0, 0.72, 1.0, 0, 0)
    arr = (_lib.sbp_problem * 1)(pr)
    assert L.sbp_workspace_bytes(arr, 1) > 0
    bad = (_lib.sbp_problem * 1)(_lib.sbp_problem(_lib.SBP_MAX_P + 1, 1, 8, 64, 64, 64, 1.4, 1.0, 0.0, 0.72,
                                                  1.0, 0, 0))
    assert L.sbp_workspace_bytes(bad, 1) == 0
    assert L.sbp_residual(bad, 1, 64, 128, 256, 1 << 20, None) == _lib.SBP_ERR_DEGREE
    # degrees above the VJP's range (the residual itself accepts them)
    hi = (_lib.sbp_problem * 1)(_lib.sbp_problem(_lib.SBP_MAX_VJP_P + 1, 1, 8, 64, 64, 64, 1.4, 1.0, 0.0, 0.72,
                                                 1.0, 0, 0))
    assert L.sbp_workspace_bytes(hi, 1) > 0
    assert L.sbp_residual_vjp(hi, 1, 64, 128, 192, 256, 1 << 22, None) == _lib.SBP_ERR_DEGREE
    # workspace too small
    assert L.sbp_residual(arr, 1, 64, 128, 256, 8, None) == _lib.SBP_ERR_WORKSPACE
    # aliasing output
    assert L.sbp_residual(arr, 1, 64, 64, 256, 1 << 20, None) == _lib.SBP_ERR_ARG
    # misaligned metric
    mis = (_lib.sbp_problem * 1)(_lib.sbp_problem(3, 1, 8, 64, 65, 64, 1.4, 1.0, 0.0, 0.72, 1.0, 0, 0))
    assert L.sbp_residual(mis, 1, 64, 128, 256, 1 << 20, None) == _lib.SBP_ERR_ARG
    # bad option
    opt = (_lib.sbp_problem * 1)(_lib.sbp_problem(3, 1, 8, 64, 64, 64, 1.4, 1.0, 0.0, 0.72, 1.0, 7, 0))
    assert L.sbp_residual(opt, 1, 64, 128, 256, 1 << 20, None) == _lib.SBP_ERR_ARG
    diss = (_lib.sbp_problem * 1)(_lib.sbp_problem(3, 3, 8, 64, 64, 64, 1.4, 1.0, 0.0, 0.72, 1.0, 0, 0))
    assert L.sbp_residual(diss, 1, 64, 128, 256, 1 << 20, None) == _lib.SBP_ERR_ARG
    # matrix dissipation with the DC volume form is not offered
    mdc = (_lib.sbp_problem * 1)(_lib.sbp_problem(3, 2, 8, 64, 64, 64, 1.4, 1.0, 0.0, 0.72, 1.0, 3, 0))
    assert L.sbp_residual(mdc, 1, 64, 128, 256, 1 << 20, None) == _lib.SBP_ERR_ARG
    # misaligned boundary data
    bcm = (_lib.sbp_problem * 1)(_lib.sbp_problem(3, 1, 8, 64, 64, 64, 1.4, 1.0, 0.0, 0.72, 1.0, 0, 0, 68, 0))
    assert L.sbp_residual(bcm, 1, 64, 128, 256, 1 << 20, None) == _lib.SBP_ERR_ARG
    assert P.lib().sbp_error_string(_lib.SBP_ERR_WORKSPACE).decode().startswith("workspace")


def _prob(**kw):
    f = dict(p=3, iface_diss=1, n_elem=8, nbr=64, metric=64, jac=64, gamma=1.4, R=1.0, mu=0.0, Pr=0.72,
             eta=1.0, two_point=0, reserved=0, bc_state=None, source=None, face_orient=None)
    f.update(kw)
    return (_lib.sbp_problem * 1)(_lib.sbp_problem(**f))


@pytest.mark.parametrize("kw", [
    dict(n_elem=0), dict(n_elem=-3),                         # empty or negative element count
    dict(gamma=1.0), dict(R=0.0), dict(mu=-1e-3), dict(eta=-1.0),  # gas and penalty constants
    dict(mu=1e-3, Pr=0.0),                                    # viscous problem without Prandtl number
    dict(reserved=1), dict(two_point=4), dict(iface_diss=-1),
    dict(iface_diss=2, two_point=1),                          # matrix dissipation needs ES-C or SF-KG
    dict(nbr=None), dict(nbr=66), dict(jac=None),             # missing or misaligned arrays
    dict(face_orient=66), dict(source=68),
])
def test_invalid_problems_are_rejected_before_any_device_work(kw):
    L = P.lib()
    arr = _prob(**kw)
    assert L.sbp_workspace_bytes(arr, 1) == 0
    for rc in (L.sbp_residual(arr, 1, 64, 128, 256, 1 << 20, None),
               L.sbp_rk_step(arr, 1, 64, 128, 1, 256, 1 << 20, None),
               L.sbp_residual_vjp(arr, 1, 64, 128, 192, 256, 1 << 22, None)):
        assert rc in (_lib.SBP_ERR_ARG, _lib.SBP_ERR_DEGREE), (kw, rc)


def test_empty_problem_list_is_rejected():
    L = P.lib()
    arr = _prob()
    assert L.sbp_residual(arr, 0, 64, 128, 256, 1 << 20, None) == _lib.SBP_ERR_ARG
    assert L.sbp_residual(None, 1, 64, 128, 256, 1 << 20, None) == _lib.SBP_ERR_ARG
    assert L.sbp_workspace_bytes(arr, 0) == 0


def test_release_rejects_a_null_workspace():
    assert P.lib().sbp_release(None) == _lib.SBP_ERR_ARG


def _host_problem(**over):
    import torch
    p, K = 2, 4
    nodes = K * (p + 1) ** 3
    f = dict(p=p, n_elem=K, nbr=torch.zeros(K, 6, dtype=torch.int32),
             metric=torch.zeros(9, nodes, dtype=torch.float64), jac=torch.ones(nodes, dtype=torch.float64))
    f.update(over)
    return P.Problem(**f)


@pytest.mark.parametrize("name,shape", [("nbr", (4, 5)), ("metric", (9, 107)), ("metric", (8, 108)),
                                        ("jac", (107,)), ("bc_state", (5, 100)), ("source", (4, 108)),
                                        ("face_orient", (3, 6))])
def test_binding_rejects_arrays_of_the_wrong_size(name, shape):
    """The library reads problem arrays through raw pointers, so the binding checks their extent."""
    import torch
    dtype = torch.int32 if name in ("nbr", "face_orient") else torch.float64
    pr = _host_problem(**{name: torch.zeros(shape, dtype=dtype)})
    with pytest.raises(ValueError, match="entries"):
        pr.c_struct()


def test_binding_rejects_host_arrays_and_bad_coordinate_counts():
    import torch
    with pytest.raises(ValueError, match="device tensor"):
        _host_problem().c_struct()
    with pytest.raises(ValueError, match="must be torch.int32"):
        _host_problem(nbr=torch.zeros(4, 6, dtype=torch.int64)).c_struct()
    with pytest.raises(ValueError, match="multiple"):
        P.metrics(2, torch.zeros(3 * 27 + 3, dtype=torch.float64))
    with pytest.raises(ValueError, match="multiple"):
        P.metrics(2, torch.zeros(0, dtype=torch.float64))


def test_noalloc_rejects_oversize_sets_and_bad_arguments_on_host():
    """sbp_residual_noalloc checks sizes against its fixed scratch before any device work."""
    L = P.lib()
    # viscous p = 4 on 100^3 elements: 4.8 GB of face traces, far beyond the scratch
    big = _prob(p=4, n_elem=100 ** 3, mu=1e-3)
    assert L.sbp_residual_noalloc(big, 1, 64, 128, 256, None) == _lib.SBP_ERR_SCRATCH
    assert P.lib().sbp_error_string(_lib.SBP_ERR_SCRATCH).decode().startswith("problem set too large")
    # the limit is the scratch size: 1 + (64 MiB - 64 KiB) // (192 N^2) elements of p = 4 do not fit
    limit = ((_lib.SBP_NOALLOC_SCRATCH_BYTES - (64 << 10)) // (192 * 25)) + 1
    assert L.sbp_residual_noalloc(_prob(p=4, n_elem=limit, mu=1e-3), 1, 64, 128, 256, None) == _lib.SBP_ERR_SCRATCH
    ok = _prob()
    assert L.sbp_residual_noalloc(ok, 0, 64, 128, 256, None) == _lib.SBP_ERR_ARG
    many = (_lib.sbp_problem * (_lib.SBP_NOALLOC_MAX_PROBLEMS + 1))(*([ok[0]] * (_lib.SBP_NOALLOC_MAX_PROBLEMS + 1)))
    assert L.sbp_residual_noalloc(many, _lib.SBP_NOALLOC_MAX_PROBLEMS + 1, 64, 128, 256, None) == _lib.SBP_ERR_ARG
    assert L.sbp_residual_noalloc(ok, 1, 64, 128, None, None) == _lib.SBP_ERR_ARG      # no status word
    assert L.sbp_residual_noalloc(ok, 1, 64, 64, 256, None) == _lib.SBP_ERR_ARG        # aliasing output
    assert L.sbp_residual_noalloc(_prob(p=16), 1, 64, 128, 256, None) == _lib.SBP_ERR_DEGREE


def test_optimized_metrics_rejects_bad_degree_and_arguments_on_host():
    """Checked before the neighbour table is read or any device work starts (fake aligned
    addresses are never dereferenced)."""
    import torch
    L = P.lib()
    for p in (1, _lib.SBP_MAX_P + 1):
        assert L.sbp_metrics_optimized(p, 8, 64, 128, 256, 512, None) == _lib.SBP_ERR_DEGREE
    assert L.sbp_metrics_optimized(3, 0, 64, 128, 256, 512, None) == _lib.SBP_ERR_ARG
    assert L.sbp_metrics_optimized(3, 8, None, 128, 256, 512, None) == _lib.SBP_ERR_ARG
    assert L.sbp_metrics_optimized(3, 8, 64, 129, 256, 512, None) == _lib.SBP_ERR_ARG
    assert L.sbp_metrics_optimized(3, 8, 66, 128, 256, 512, None) == _lib.SBP_ERR_ARG
    with pytest.raises(ValueError, match="multiple"):
        P.metrics_optimized(2, torch.zeros(6, dtype=torch.int32), torch.zeros(9 * 27 + 9, dtype=torch.float64))
    with pytest.raises(ValueError, match="device tensor"):
        P.metrics_optimized(2, torch.zeros(6, dtype=torch.int32), torch.zeros(9 * 27, dtype=torch.float64))
