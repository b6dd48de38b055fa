"""Randomized approximate PSD projection on AMD MI355X (gfx950).

Thin ctypes binding of libpsdproj (the C ABI in include/psdproj.h).  Functions keep the
C names; arguments are device pointers, sizes and a HIP stream handle.  PyTorch is used
only to own device memory and streams: every step of the projection runs in the HIP
kernels of the library.  Importing this package fails loudly when the library has not
been built (python -m paper_2410_19208_amd.build) -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "PLAIN", "SCALED", "FLAG_SRHT", "FLAG_CSR", "psdproj_srht_matrix", "psdproj_run_csr", "FP64", "FP32", "BF16X3", "Desc", "Result", "Layout", "PsdprojError", "SdlsDesc",
    "SdlsInfo", "sdls_desc", "psdproj_sdls_workspace", "psdproj_sdls_solve", "psdproj_exact_workspace",
    "psdproj_exact",
    "lib", "psdproj_plan", "psdproj_plan_destroy", "psdproj_plan_layout", "psdproj_run", "psdproj_run_static",
    "psdproj_static_scratch_bytes",
    "psdproj_batch_workspace", "psdproj_batch", "psdproj_graph_create", "psdproj_graph_launch",
    "psdproj_graph_destroy", "psdproj_graph_stats", "psdproj_tile_override", "psdproj_server_create", "psdproj_submit",
    "psdproj_poll", "psdproj_wait", "psdproj_server_times", "psdproj_server_destroy",
    "psdproj_philox_words", "psdproj_gaussian", "psdproj_status_str", "psdproj_abi_version",
    "EXPORTED", "LIB_PATH",
]

PLAIN, SCALED = 0, 1
FLAG_SRHT = 1          # desc.flags: structured (subsampled randomized Hadamard) test matrix
FLAG_CSR = 2           # desc.flags: sparse A (CSR), run with psdproj_run_csr
FP64, FP32, BF16X3 = 0, 1, 2
(OK, E_INVALID, E_ALPHA, E_NONFINITE, E_BREAKDOWN, E_NOMEM, E_BUDGET, E_DEVICE, E_PENDING, E_TIMEOUT,
 E_SCRATCH) = range(11)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpsdproj.so")


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("alpha", ctypes.c_double), ("alpha_iters", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("r_plus", ctypes.c_int32), ("alpha_used", ctypes.c_double),
                ("sigma1", ctypes.c_double), ("sigma2", ctypes.c_double)]


class Layout(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("r_pad", ctypes.c_int32), ("panel_ld", ctypes.c_int32),
                ("split_k", ctypes.c_int32), ("panel_elem_bytes", ctypes.c_int32),
                ("omega", ctypes.c_size_t), ("q_panel", ctypes.c_size_t), ("compressed", ctypes.c_size_t),
                ("evals", ctypes.c_size_t), ("weights", ctypes.c_size_t), ("factor", ctypes.c_size_t),
                ("power_vec", ctypes.c_size_t), ("y_panel", ctypes.c_size_t), ("gram", ctypes.c_size_t),
                ("total", ctypes.c_size_t)]


class SdlsDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int32), ("k", ctypes.c_int32), ("p", ctypes.c_int32),
                ("q", ctypes.c_int32), ("scal", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("alpha_iters", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("rho", ctypes.c_double), ("beta", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class SdlsInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("grad_norm", ctypes.c_double)]


class PsdprojError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {psdproj_status_str(status)} (status {status})")


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2410_19208_amd/build.py` "
                      "(the projection has no non-HIP path)")
try:
    # PyTorch bundles its own HIP runtime under the same soname; load it first so that the
    # library binds to that one and the process holds a single HIP runtime.
    import torch  # noqa: F401
except ImportError:  # host-only use (planning, validation) works without PyTorch
    pass
lib = ctypes.CDLL(LIB_PATH)

_vp, _i32, _i64, _u32, _u64, _dbl, _sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                           ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t)
_SIGS = {
    "psdproj_plan": (_i32, [ctypes.POINTER(Desc), ctypes.POINTER(_vp), ctypes.POINTER(_sz)]),
    "psdproj_plan_destroy": (None, [_vp]),
    "psdproj_plan_layout": (_i32, [_vp, ctypes.POINTER(Layout)]),
    "psdproj_run": (_i32, [_vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp]),
    "psdproj_run_csr": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp]),
    "psdproj_run_static": (_i32, [_vp, _vp, _i64, _vp, _i64, _vp, _vp]),
    "psdproj_static_scratch_bytes": (_i32, [_vp, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "psdproj_batch_workspace": (_i32, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_sz)]),
    "psdproj_batch": (_i32, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i64),
                             ctypes.POINTER(_vp), ctypes.POINTER(_i64), _vp, _sz, _vp, _vp]),
    "psdproj_graph_create": (_i32, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i64),
                                    ctypes.POINTER(_vp), ctypes.POINTER(_i64), _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "psdproj_graph_launch": (_i32, [_vp, _vp]),
    "psdproj_graph_destroy": (None, [_vp]),
    "psdproj_graph_stats": (_i32, [ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "psdproj_tile_override": (_i32, [_i32, _i32]),
    "psdproj_exact_workspace": (_i32, [_i64, _i32, ctypes.POINTER(_sz)]),
    "psdproj_exact": (_i32, [_i64, _i32, _vp, _i64, _vp, _i64, _vp, _sz, _vp, _vp]),
    "psdproj_sdls_workspace": (_i32, [ctypes.POINTER(SdlsDesc), ctypes.POINTER(_sz)]),
    "psdproj_sdls_solve": (_i32, [ctypes.POINTER(SdlsDesc), _vp, _i64, _vp, _i64, _i64, _vp, _vp, _vp, _i64, _vp,
                                  _sz, ctypes.POINTER(SdlsInfo), _vp]),
    "psdproj_server_create": (_i32, [_sz, _i32, ctypes.POINTER(_vp)]),
    "psdproj_submit": (_i32, [_vp, ctypes.POINTER(Desc), _vp, _i64, _vp, _i64, ctypes.POINTER(_u64)]),
    "psdproj_poll": (_i32, [_vp, _u64, ctypes.POINTER(Result)]),
    "psdproj_wait": (_i32, [_vp, _u64, ctypes.POINTER(Result), _dbl]),
    "psdproj_server_times": (_i32, [_vp, _u64, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]),
    "psdproj_server_destroy": (None, [_vp]),
    "psdproj_philox_words": (_i32, [_u64, _u32, _u64, _i64, _vp, _vp]),
    "psdproj_gaussian": (_i32, [_u64, _u32, _u64, _i64, _vp, _vp]),
    "psdproj_srht_matrix": (_i32, [_u64, _i64, _i32, _vp, _vp]),
    "psdproj_profile_enable": (_i32, [_i32]),
    "psdproj_profile_select": (_i32, [ctypes.c_uint64]),
    "psdproj_profile_reset": (_i32, []),
    "psdproj_profile_read": (_i32, [_i32, ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]),
    "psdproj_kernel_kinds": (_i32, []),
    "psdproj_kernel_name": (ctypes.c_char_p, [_i32]),
    "psdproj_status_str": (ctypes.c_char_p, [_i32]),
    "psdproj_abi_version": (_i32, []),
}
EXPORTED = tuple(_SIGS)
for _name, (_res, _args) in _SIGS.items():
    try:
        _f = getattr(lib, _name)
    except AttributeError as _e:
        raise ImportError(f"{LIB_PATH} does not export {_name}: it is stale, rebuild it with "
                          "`python paper_2410_19208_amd/build.py`") from _e
    _f.restype = _res
    _f.argtypes = _args


def psdproj_profile_enable(enable: bool = True) -> None:
    _check(lib.psdproj_profile_enable(1 if enable else 0), "psdproj_profile_enable")


def psdproj_profile_select(kinds) -> None:
    """Time only the given kernel kinds (an iterable of kind numbers), or every kind (None)."""
    mask = (1 << 64) - 1 if kinds is None else sum(1 << int(k) for k in kinds)
    _check(lib.psdproj_profile_select(ctypes.c_uint64(mask)), "psdproj_profile_select")


def psdproj_profile_reset() -> None:
    _check(lib.psdproj_profile_reset(), "psdproj_profile_reset")


def psdproj_profile_read(kind: int):
    """(total device milliseconds, launches) of one kernel kind since the last reset."""
    t = _dbl()
    c = _i64()
    _check(lib.psdproj_profile_read(kind, ctypes.byref(t), ctypes.byref(c)), "psdproj_profile_read")
    return t.value, c.value


def psdproj_kernel_kinds() -> int:
    return lib.psdproj_kernel_kinds()


def psdproj_kernel_name(kind: int) -> str:
    return lib.psdproj_kernel_name(kind).decode()


def psdproj_srht_matrix(seed, n, r, out_dev, stream=0) -> None:
    _check(lib.psdproj_srht_matrix(seed, n, r, out_dev, stream), "psdproj_srht_matrix")


def psdproj_status_str(status: int) -> str:
    return lib.psdproj_status_str(int(status)).decode()


def psdproj_abi_version() -> int:
    return lib.psdproj_abi_version()


def _check(st: int, where: str) -> None:
    if st != OK:
        raise PsdprojError(st, where)


def psdproj_plan(n, k, p, q=0, variant=PLAIN, precision=FP32, seed=0, alpha=0.0, alpha_iters=10, flags=0):
    """Returns (plan handle, workspace bytes).  Raises PsdprojError on a bad descriptor."""
    d = Desc(n, k, p, q, variant, precision, seed, alpha, alpha_iters, flags)
    h = _vp()
    ws = _sz()
    _check(lib.psdproj_plan(ctypes.byref(d), ctypes.byref(h), ctypes.byref(ws)), "psdproj_plan")
    return h.value, ws.value


def psdproj_plan_destroy(plan) -> None:
    lib.psdproj_plan_destroy(plan)


def psdproj_plan_layout(plan) -> Layout:
    out = Layout()
    _check(lib.psdproj_plan_layout(plan, ctypes.byref(out)), "psdproj_plan_layout")
    return out


def psdproj_run(plan, A, lda, P, ldp, workspace, result_dev, stream=0) -> None:
    """All pointers are device addresses (ints); stream is a hipStream_t handle (int)."""
    _check(lib.psdproj_run(plan, A, lda, P, ldp, workspace, result_dev, stream), "psdproj_run")


def psdproj_run_csr(plan, row_ptr, col_idx, vals, nnz, P, ldp, workspace, result_dev, stream=0) -> None:
    """One projection of a sparse A (CSR, both triangles) planned with FLAG_CSR."""
    _check(lib.psdproj_run_csr(plan, row_ptr, col_idx, vals, nnz, P, ldp, workspace, result_dev, stream),
           "psdproj_run_csr")


def psdproj_run_static(plan, A, lda, P, ldp, result_dev, stream=0) -> None:
    """psdproj_run with the library's static per-device scratch array as its workspace."""
    _check(lib.psdproj_run_static(plan, A, lda, P, ldp, result_dev, stream), "psdproj_run_static")


def psdproj_static_scratch_bytes(plan):
    """(bytes the plan needs, bytes the static scratch array holds)."""
    need, cap = _sz(), _sz()
    _check(lib.psdproj_static_scratch_bytes(plan, ctypes.byref(need), ctypes.byref(cap)),
           "psdproj_static_scratch_bytes")
    return need.value, cap.value


def psdproj_batch_workspace(plans) -> int:
    arr = (_vp * len(plans))(*plans)
    out = _sz()
    _check(lib.psdproj_batch_workspace(len(plans), arr, ctypes.byref(out)), "psdproj_batch_workspace")
    return out.value


def psdproj_batch(plans, A, lda, P, ldp, workspace, workspace_bytes, results_dev, stream=0) -> None:
    m = len(plans)
    _check(lib.psdproj_batch(m, (_vp * m)(*plans), (_vp * m)(*A), (_i64 * m)(*lda), (_vp * m)(*P),
                             (_i64 * m)(*ldp), workspace, workspace_bytes, results_dev, stream), "psdproj_batch")


def psdproj_graph_create(plans, A, lda, P, ldp, workspace, workspace_bytes, results_dev):
    """Capture the batch (arguments as psdproj_batch) into a replayable HIP graph handle."""
    m = len(plans)
    h = _vp()
    _check(lib.psdproj_graph_create(m, (_vp * m)(*plans), (_vp * m)(*A), (_i64 * m)(*lda), (_vp * m)(*P),
                                    (_i64 * m)(*ldp), workspace, workspace_bytes, results_dev, ctypes.byref(h)),
           "psdproj_graph_create")
    return h.value


def psdproj_graph_launch(graph, stream=0) -> None:
    _check(lib.psdproj_graph_launch(graph, stream), "psdproj_graph_launch")


def psdproj_graph_destroy(graph) -> None:
    lib.psdproj_graph_destroy(graph)


def psdproj_graph_stats():
    """(sequences captured, replays) of the run/batch/server graph cache."""
    c, r = _i64(), _i64()
    _check(lib.psdproj_graph_stats(ctypes.byref(c), ctypes.byref(r)), "psdproj_graph_stats")
    return c.value, r.value


def psdproj_tile_override(precision, split) -> None:
    """Plans created afterwards with `precision` use pass split-K `split` (0: the tuned table)."""
    _check(lib.psdproj_tile_override(int(precision), int(split)), "psdproj_tile_override")


def psdproj_exact_workspace(n, precision) -> int:
    out = _sz()
    _check(lib.psdproj_exact_workspace(n, precision, ctypes.byref(out)), "psdproj_exact_workspace")
    return out.value


def psdproj_exact(n, precision, A, lda, P, ldp, workspace, workspace_bytes, result_dev, stream=0) -> None:
    """The exact projection (Thm 1) of the n x n matrix at A into P."""
    _check(lib.psdproj_exact(n, precision, A, lda, P, ldp, workspace, workspace_bytes, result_dev, stream),
           "psdproj_exact")


def sdls_desc(n, m, k=0, p=0, q=0, scal=0, precision=FP64, alpha_iters=10, max_iters=100, rho=1.0, beta=0.5,
              eps=1e-10, seed=0) -> SdlsDesc:
    return SdlsDesc(n, m, k, p, q, scal, precision, alpha_iters, max_iters, 0, rho, beta, eps, seed)


def psdproj_sdls_workspace(desc: SdlsDesc) -> int:
    out = _sz()
    _check(lib.psdproj_sdls_workspace(ctypes.byref(desc), ctypes.byref(out)), "psdproj_sdls_workspace")
    return out.value


def psdproj_sdls_solve(desc: SdlsDesc, C, ldc, A, lda, a_stride, b_dev, y_dev, X, ldx, workspace, workspace_bytes,
                       stream=0) -> SdlsInfo:
    """Alg. 6 on device buffers (pointers); returns the host info record."""
    info = SdlsInfo()
    _check(lib.psdproj_sdls_solve(ctypes.byref(desc), C, ldc, A, lda, a_stride, b_dev, y_dev, X, ldx, workspace,
                                  workspace_bytes, ctypes.byref(info), stream), "psdproj_sdls_solve")
    return info


def psdproj_server_create(hbm_budget_bytes, max_inflight):
    h = _vp()
    _check(lib.psdproj_server_create(hbm_budget_bytes, max_inflight, ctypes.byref(h)), "psdproj_server_create")
    return h.value


def psdproj_submit(server, A, lda, P, ldp, n, k, p, q=0, variant=PLAIN, precision=BF16X3, seed=0, alpha=0.0,
                   alpha_iters=10) -> int:
    d = Desc(n, k, p, q, variant, precision, seed, alpha, alpha_iters, 0)
    t = _u64()
    _check(lib.psdproj_submit(server, ctypes.byref(d), A, lda, P, ldp, ctypes.byref(t)), "psdproj_submit")
    return t.value


def psdproj_poll(server, ticket):
    """Result, or None while the request is still in flight."""
    out = Result()
    st = lib.psdproj_poll(server, ticket, ctypes.byref(out))
    if st == E_PENDING:
        return None
    _check(st, "psdproj_poll")
    return out


def psdproj_wait(server, ticket, timeout_s=60.0) -> Result:
    out = Result()
    _check(lib.psdproj_wait(server, ticket, ctypes.byref(out), timeout_s), "psdproj_wait")
    return out


def psdproj_server_times(server, ticket):
    a, b, c = _dbl(), _dbl(), _dbl()
    _check(lib.psdproj_server_times(server, ticket, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "psdproj_server_times")
    return a.value, b.value, c.value


def psdproj_server_destroy(server) -> None:
    lib.psdproj_server_destroy(server)


def psdproj_philox_words(seed, stream_id, c0, count, out_dev, stream=0) -> None:
    _check(lib.psdproj_philox_words(seed, stream_id, c0, count, out_dev, stream), "psdproj_philox_words")


def psdproj_gaussian(seed, stream_id, start, count, out_dev, stream=0) -> None:
    _check(lib.psdproj_gaussian(seed, stream_id, start, count, out_dev, stream), "psdproj_gaussian")
