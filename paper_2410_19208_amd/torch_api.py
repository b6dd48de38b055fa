"""PyTorch plumbing around the C ABI: device buffers, streams and result read-back.

Nothing here computes any step of the projection; it allocates the workspace and result
buffers as torch tensors and passes their addresses to libpsdproj.
"""
from __future__ import annotations

import ctypes

import torch

from . import (BF16X3, FLAG_CSR, FLAG_SRHT, FP32, FP64, PLAIN, SCALED, Layout, Result, psdproj_batch, psdproj_batch_workspace,
               psdproj_exact, psdproj_exact_workspace, psdproj_run_csr, psdproj_sdls_solve, psdproj_sdls_workspace, sdls_desc,
               psdproj_plan, psdproj_plan_destroy, psdproj_plan_layout, psdproj_poll, psdproj_run,
               psdproj_server_create, psdproj_server_destroy, psdproj_server_times, psdproj_submit, psdproj_wait)

__all__ = ["Projector", "SparseProjector", "BatchProjector", "Server", "SdlsSolver", "ExactProjector", "stream_handle", "read_results", "PRECISIONS",
           "VARIANTS", "storage_dtype"]

PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
VARIANTS = {"plain": PLAIN, "scaled": SCALED}


def storage_dtype(precision: int) -> torch.dtype:
    return torch.float64 if precision == FP64 else torch.float32


def stream_handle(stream: torch.cuda.Stream | None = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def read_results(buf: torch.Tensor, count: int = 1) -> list[Result]:
    """Copy `count` device-written psdproj_result records to the host (synchronising)."""
    raw = bytes(buf[: count * ctypes.sizeof(Result)].cpu().numpy().tobytes())
    return [Result.from_buffer_copy(raw, i * ctypes.sizeof(Result)) for i in range(count)]


class Projector:
    """One plan with its own workspace and result buffers on `device`."""

    def __init__(self, n, k, p, q=0, variant="plain", precision="bf16x3", seed=0, alpha=0.0,
                 alpha_iters=10, device="cuda", sketch="gaussian"):
        self.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.n = int(n)
        flags = {"gaussian": 0, "srht": FLAG_SRHT}[sketch]
        self.plan, self.ws_bytes = psdproj_plan(n, k, p, q, self.variant, self.precision, seed, alpha, alpha_iters,
                                                flags)
        self.layout: Layout = psdproj_plan_layout(self.plan)
        self.device = torch.device(device)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.result_buf = torch.zeros(ctypes.sizeof(Result), dtype=torch.uint8, device=self.device)
        self.dtype = storage_dtype(self.precision)

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan and psdproj_plan_destroy is not None:   # module globals may be gone at exit
            psdproj_plan_destroy(plan)
            self.plan = None

    def __call__(self, A: torch.Tensor, P: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if A.dtype != self.dtype or A.device != self.device or A.shape != (self.n, self.n):
            raise ValueError(f"A must be a {self.n}x{self.n} {self.dtype} tensor on {self.device}")
        if A.stride(1) != 1:
            raise ValueError("A must be row-contiguous")
        if P is None:
            P = torch.empty_like(A)
        psdproj_run(self.plan, A.data_ptr(), A.stride(0), P.data_ptr(), P.stride(0), self.workspace.data_ptr(),
                    self.result_buf.data_ptr(), stream_handle(stream))
        return P

    def result(self) -> Result:
        return read_results(self.result_buf, 1)[0]

    # --- intermediates, for inspection after the stream has passed the run
    def _panel(self, offset: int, cols: int) -> torch.Tensor:
        L = self.layout
        dt = torch.float64 if L.panel_elem_bytes == 8 else torch.float32
        nbytes = cols * L.panel_ld * L.panel_elem_bytes
        flat = self.workspace[offset: offset + nbytes].view(dt)
        return flat.view(cols, L.panel_ld)[:, : self.n].t()

    def q_panel(self) -> torch.Tensor:
        return self._panel(self.layout.q_panel, self.layout.r)

    def omega(self) -> torch.Tensor:
        """Omega is only resident until the first orthonormalisation overwrites the panel."""
        return self._panel(self.layout.omega, self.layout.r)

    def y_panel(self) -> torch.Tensor:
        return self._panel(self.layout.y_panel, self.layout.r)

    def gram(self) -> torch.Tensor:
        L = self.layout
        flat = self.workspace[L.gram: L.gram + L.r_pad * L.r_pad * 8].view(torch.float64)
        return flat.view(L.r_pad, L.r_pad)[: L.r, : L.r].t()

    def compressed(self) -> torch.Tensor:
        L = self.layout
        flat = self.workspace[L.compressed: L.compressed + L.r_pad * L.r_pad * 8].view(torch.float64)
        return flat.view(L.r_pad, L.r_pad)[: L.r, : L.r].t()

    def evals(self) -> torch.Tensor:
        L = self.layout
        return self.workspace[L.evals: L.evals + L.r * 8].view(torch.float64)

    def factor(self, r_plus: int) -> torch.Tensor:
        """W (n x r_plus) with P = W W^T (row-major, row stride r_pad)."""
        L = self.layout
        dt = torch.float64 if L.panel_elem_bytes == 8 else torch.float32
        rows = L.panel_ld
        flat = self.workspace[L.factor: L.factor + rows * L.r_pad * L.panel_elem_bytes].view(dt)
        return flat.view(rows, L.r_pad)[: self.n, :r_plus]


class BatchProjector:
    """A list of plans run through one psdproj_batch call."""

    def __init__(self, specs, device="cuda"):
        self.device = torch.device(device)
        self.projectors = []
        self.plans = []
        for s in specs:
            s = dict(s)
            v = s.pop("variant", "plain")
            pr = s.pop("precision", "bf16x3")
            vv = VARIANTS[v] if isinstance(v, str) else int(v)
            pp = PRECISIONS[pr] if isinstance(pr, str) else int(pr)
            plan, _ = psdproj_plan(s["n"], s["k"], s["p"], s.get("q", 0), vv, pp, s.get("seed", 0),
                                   s.get("alpha", 0.0), s.get("alpha_iters", 10))
            self.plans.append(plan)
            self.projectors.append((s["n"], storage_dtype(pp)))
        self.ws_bytes = psdproj_batch_workspace(self.plans)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.result_buf = torch.zeros(len(self.plans) * ctypes.sizeof(Result), dtype=torch.uint8, device=self.device)

    def __del__(self):
        if psdproj_plan_destroy is None:   # interpreter shutdown: the library goes with the process
            return
        for p in getattr(self, "plans", []):
            psdproj_plan_destroy(p)
        self.plans = []

    def __call__(self, As, Ps=None, stream=None):
        if Ps is None:
            Ps = [torch.empty_like(a) for a in As]
        psdproj_batch(self.plans, [a.data_ptr() for a in As], [a.stride(0) for a in As],
                      [p.data_ptr() for p in Ps], [p.stride(0) for p in Ps], self.workspace.data_ptr(),
                      self.ws_bytes, self.result_buf.data_ptr(), stream_handle(stream))
        return Ps

    def results(self):
        return read_results(self.result_buf, len(self.plans))


class Server:
    """The continuous-batching request server (psdproj_server_*).

    submit() takes a device tensor A (and optionally the output P), synchronises the current
    stream so that A is complete before the server's own streams read it, and returns a
    ticket; wait()/poll() return the device-written result record.  The tensors are kept
    alive until their ticket is collected.
    """

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 64, device="cuda"):
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.handle = psdproj_server_create(int(hbm_budget_bytes), int(max_inflight))
        self._keep = {}

    def submit(self, A: torch.Tensor, k: int, p: int, q: int = 0, variant="plain", precision="bf16x3", seed=0,
               alpha=0.0, alpha_iters=10, P: torch.Tensor | None = None):
        vv = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        pp = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        n = A.shape[0]
        if A.dtype != storage_dtype(pp) or A.device != self.device or A.shape != (n, n) or A.stride(1) != 1:
            raise ValueError(f"A must be a row-contiguous {n}x{n} {storage_dtype(pp)} tensor on {self.device}")
        if P is None:
            P = torch.empty_like(A)
        torch.cuda.current_stream(self.device).synchronize()
        t = psdproj_submit(self.handle, A.data_ptr(), A.stride(0), P.data_ptr(), P.stride(0), n, k, p, q, vv, pp,
                           seed, alpha, alpha_iters)
        self._keep[t] = (A, P)
        return t, P

    def poll(self, ticket):
        r = psdproj_poll(self.handle, ticket)
        if r is not None:
            self._keep.pop(ticket, None)
        return r

    def wait(self, ticket, timeout_s: float = -1.0):
        r = psdproj_wait(self.handle, ticket, timeout_s)
        self._keep.pop(ticket, None)
        return r

    def times(self, ticket):
        """(submit, admit, finish) in seconds since the server was created."""
        return psdproj_server_times(self.handle, ticket)

    def close(self):
        if getattr(self, "handle", None) and psdproj_server_destroy is not None:
            psdproj_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        self.close()


class SdlsSolver:
    """Alg. 6 (dual gradient descent for the SDLS problem) through psdproj_sdls_solve.

    scal: -1 exact projection, 0 Alg. 2, 1 Alg. 3 (alpha by Alg. 5).  C (n x n), A (m x n x n) and
    b (m) are device tensors (C and A in the precision's storage dtype, b float64); solve(y0)
    returns (y, X, info) with X the last projection."""

    def __init__(self, n, m, k=0, p=0, q=0, scal=0, precision="fp64", alpha_iters=10, max_iters=100, rho=1.0,
                 beta=0.5, eps=1e-10, seed=0, device="cuda"):
        pr = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.desc = sdls_desc(n, m, k, p, q, scal, pr, alpha_iters, max_iters, rho, beta, eps, seed)
        self.n, self.m = int(n), int(m)
        self.dtype = storage_dtype(pr)
        self.device = torch.device(device)
        self.ws_bytes = psdproj_sdls_workspace(self.desc)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def solve(self, C, A, b, y0, X=None, stream=None):
        n, m = self.n, self.m
        if C.shape != (n, n) or A.shape != (m, n, n) or C.dtype != self.dtype or A.dtype != self.dtype:
            raise ValueError("C must be n x n and A m x n x n in the storage dtype")
        if not (C.is_contiguous() and A.is_contiguous()):
            raise ValueError("C and A must be contiguous")
        y = y0.to(device=self.device, dtype=torch.float64).clone()
        bb = b.to(device=self.device, dtype=torch.float64).contiguous()
        if X is None:
            X = torch.empty((n, n), dtype=self.dtype, device=self.device)
        info = psdproj_sdls_solve(self.desc, C.data_ptr(), C.stride(0), A.data_ptr(), A.stride(1), A.stride(0),
                                  bb.data_ptr(), y.data_ptr(), X.data_ptr(), X.stride(0), self.workspace.data_ptr(),
                                  self.ws_bytes, stream_handle(stream))
        return y, X, info


class ExactProjector:
    """The exact projection (Thm 1) through psdproj_exact, with its own workspace."""

    def __init__(self, n, precision="fp64", device="cuda"):
        self.n = int(n)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.dtype = storage_dtype(self.precision)
        self.device = torch.device(device)
        self.ws_bytes = psdproj_exact_workspace(self.n, self.precision)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.result_buf = torch.zeros(ctypes.sizeof(Result), dtype=torch.uint8, device=self.device)

    def __call__(self, A, P=None, stream=None):
        if A.dtype != self.dtype or A.shape != (self.n, self.n) or A.stride(1) != 1:
            raise ValueError(f"A must be a row-contiguous {self.n}x{self.n} {self.dtype} tensor")
        if P is None:
            P = torch.empty_like(A)
        psdproj_exact(self.n, self.precision, A.data_ptr(), A.stride(0), P.data_ptr(), P.stride(0),
                      self.workspace.data_ptr(), self.ws_bytes, self.result_buf.data_ptr(), stream_handle(stream))
        return P

    def result(self) -> Result:
        return read_results(self.result_buf, 1)[0]


class SparseProjector:
    """One plan for a sparse symmetric A (CSR, both triangles) run through psdproj_run_csr."""

    def __init__(self, n, k, p, q=0, variant="plain", precision="fp32", seed=0, alpha=0.0, alpha_iters=10,
                 device="cuda"):
        self.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.n = int(n)
        self.plan, self.ws_bytes = psdproj_plan(n, k, p, q, self.variant, self.precision, seed, alpha, alpha_iters,
                                                FLAG_CSR)
        self.device = torch.device(device)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.result_buf = torch.zeros(ctypes.sizeof(Result), dtype=torch.uint8, device=self.device)
        self.dtype = storage_dtype(self.precision)

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan and psdproj_plan_destroy is not None:
            psdproj_plan_destroy(plan)
            self.plan = None

    def __call__(self, row_ptr, col_idx, vals, P=None, stream=None):
        if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32 or vals.dtype != self.dtype:
            raise ValueError("row_ptr, col_idx int32 and vals in the storage dtype")
        if row_ptr.numel() != self.n + 1 or col_idx.numel() != vals.numel():
            raise ValueError("CSR arrays of the wrong size")
        if P is None:
            P = torch.empty((self.n, self.n), dtype=self.dtype, device=self.device)
        psdproj_run_csr(self.plan, row_ptr.data_ptr(), col_idx.data_ptr(), vals.data_ptr(), vals.numel(),
                        P.data_ptr(), P.stride(0), self.workspace.data_ptr(), self.result_buf.data_ptr(),
                        stream_handle(stream))
        return P

    def result(self) -> Result:
        return read_results(self.result_buf, 1)[0]
