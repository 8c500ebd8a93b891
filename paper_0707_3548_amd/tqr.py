"""ctypes binding of ``libtqr.so`` (include/tqr.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of the computation runs in the library's kernels.  The
library must be built (``python -m paper_0707_3548_amd.build``); importing
this module on a machine without it raises at the first call, never falls
back to anything else.

Matrices are column-major: a torch tensor ``X`` of shape (m, n) whose
``X.stride() == (1, ld)`` with ``ld >= m`` (``fortran(x)`` makes one).
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtqr.so")

MODE_PERSISTENT, MODE_SERIAL = 0, 1
POLICY_PAPER, POLICY_LOOKAHEAD, POLICY_COLUMN = 0, 1, 2
TQR_EDEVICE, TQR_EABORTED, TQR_ESCRATCH = -1000, -1001, -1002
PRECISION_FP64, PRECISION_FP32_UPDATES, PRECISION_BF16_UPDATES = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 128 << 20  # TQR_NOALLOC_SCRATCH_BYTES


class TqrError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("workgroups", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("policy", ctypes.c_int32),
        ("trace", ctypes.c_void_p),
        ("abort_flag", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("timeout_ticks", ctypes.c_int64),
        ("event_begin", ctypes.c_void_p),
        ("event_end", ctypes.c_void_p),
        ("precision", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class BatchProblem(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("lda", ctypes.c_int64),
        ("A", ctypes.c_void_p),
        ("T", ctypes.c_void_p),
        ("tile_b", ctypes.c_int32),
        ("inner_ib", ctypes.c_int32),
        ("work_offset", ctypes.c_int64),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_0707_3548_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i64, i32, vp, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p
        L.tqr_t_elems.argtypes = [i64, i64, i32, i32]
        L.tqr_t_elems.restype = i64
        L.tqr_workspace_bytes.argtypes = [i64, i64, i64, i32, i32]
        L.tqr_workspace_bytes.restype = i64
        L.tqr_factor.argtypes = [i64, i64, dp, i64, i32, i32, dp, vp, i64, vp]
        L.tqr_factor.restype = i32
        L.tqr_factor_ex.argtypes = [i64, i64, dp, i64, i32, i32, dp, vp, i64, vp, ctypes.POINTER(Options)]
        L.tqr_factor_ex.restype = i32
        L.tqr_factor_noalloc.argtypes = [i64, i64, dp, i64, i32, i32, dp, vp]
        L.tqr_factor_noalloc.restype = i32
        for f in ("tqr_apply_qt", "tqr_apply_q"):
            getattr(L, f).argtypes = [i64, i64, i64, dp, i64, dp, i32, i32, dp, i64, vp, i64, vp]
            getattr(L, f).restype = i32
        L.tqr_form_q.argtypes = [i64, i64, dp, i64, dp, i32, i32, dp, i64, vp, i64, vp]
        L.tqr_form_q.restype = i32
        L.tqr_solve_ls.argtypes = [i64, i64, i64, dp, i64, dp, i64, i32, i32, dp, vp, i64, vp, vp]
        L.tqr_solve_ls.restype = i32
        L.tqr_solve_ls_ex.argtypes = [i64, i64, i64, dp, i64, dp, i64, i32, i32, dp, vp, i64, vp, vp, ctypes.POINTER(Options)]
        L.tqr_solve_ls_ex.restype = i32
        L.tqr_ls_mixed_workspace_bytes.argtypes = [i64, i64, i64, i32]
        L.tqr_ls_mixed_workspace_bytes.restype = i64
        L.tqr_solve_ls_mixed.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64, i32, i32, dp, vp, i64, vp, vp, vp,
                                         ctypes.POINTER(Options)]
        L.tqr_solve_ls_mixed.restype = i32
        L.tqr_batch_plan.argtypes = [i64, ctypes.POINTER(BatchProblem)]
        L.tqr_batch_plan.restype = i64
        L.tqr_factor_batched.argtypes = [i64, vp, vp, i64, vp, ctypes.c_int32, ctypes.c_int32, vp]
        L.tqr_factor_batched.restype = i32
        L.tqr_last_error_string.argtypes = []
        L.tqr_last_error_string.restype = ctypes.c_char_p
        L.tqr_graph_tasks.argtypes = [i64, i64, i32]
        L.tqr_graph_tasks.restype = i64
        L.tqr_graph_task.argtypes = [i64, i64, i32, i64, ctypes.POINTER(ctypes.c_int32)]
        L.tqr_graph_task.restype = i32
        L.tqr_graph_indegree.argtypes = [i64, i64, i32, i64]
        L.tqr_graph_indegree.restype = i32
        L.tqr_graph_successors.argtypes = [i64, i64, i32, i64, ctypes.POINTER(ctypes.c_int64), i32]
        L.tqr_graph_successors.restype = i32
        _lib = L
    return _lib


def _check(fn: str, rc: int) -> None:
    if rc != 0:
        msg = lib().tqr_last_error_string()
        raise TqrError(fn, rc, msg.decode() if msg else "")


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def fortran(x: torch.Tensor) -> torch.Tensor:
    """A column-major copy of a 2-D tensor (shape kept)."""
    return x.t().contiguous().t()


def _ld(X: torch.Tensor) -> int:
    if X.dim() != 2 or X.dtype != torch.float64 or not X.is_cuda:
        raise ValueError("expected a 2-D float64 CUDA tensor")
    if X.shape[0] > 1 and X.stride(0) != 1:
        raise ValueError("expected a column-major tensor (use tqr.fortran)")
    return max(1, X.stride(1) if X.shape[1] > 1 else X.shape[0])


def t_elems(m: int, n: int, tile_b: int, inner_ib: int) -> int:
    return int(lib().tqr_t_elems(m, n, tile_b, inner_ib))


def workspace_bytes(m: int, n: int, nrhs: int, tile_b: int, inner_ib: int) -> int:
    return int(lib().tqr_workspace_bytes(m, n, nrhs, tile_b, inner_ib))


class Workspace:
    """Device buffers sized for a problem shape, reusable across calls."""

    def __init__(self, m: int, n: int, nrhs: int, tile_b: int, inner_ib: int, device="cuda"):
        self.m, self.n, self.nrhs, self.tile_b, self.inner_ib = m, n, nrhs, tile_b, inner_ib
        nb = workspace_bytes(m, n, nrhs, tile_b, inner_ib)
        te = t_elems(m, n, tile_b, inner_ib)
        if nb < 0 or te < 0:
            raise ValueError("unsupported sizes or tiling")
        self.work = torch.empty(max(nb, 256), dtype=torch.uint8, device=device)
        self.T = torch.zeros(max(te, 1), dtype=torch.float64, device=device)


def factor(A: torch.Tensor, tile_b: int, inner_ib: int, ws: Workspace | None = None, *, workgroups: int = 0,
           mode: int = MODE_PERSISTENT, policy: int = POLICY_COLUMN, trace: torch.Tensor | None = None,
           status: torch.Tensor | None = None, abort_flag=None, timeout_ticks: int = 0,
           events=None, precision: int = PRECISION_FP64):
    """In-place tiled QR of the column-major A; returns (A, T).  ``events`` is
    an optional pair of raw hipEvent_t handles recorded around the scheduler
    launch (see HipEvents); ``precision`` PRECISION_FP32_UPDATES runs the
    trailing updates on the FP32 matrix cores."""
    m, n = A.shape
    lda = _ld(A)
    if ws is None:
        ws = Workspace(m, n, 0, tile_b, inner_ib, A.device)
    opt = Options(ctypes.sizeof(Options), workgroups, mode, policy,
                  trace.data_ptr() if trace is not None else None,
                  abort_flag, status.data_ptr() if status is not None else None, timeout_ticks,
                  events[0] if events else None, events[1] if events else None, precision, 0)
    rc = lib().tqr_factor_ex(m, n, A.data_ptr(), lda, tile_b, inner_ib, ws.T.data_ptr(), ws.work.data_ptr(),
                             ws.work.numel(), _stream(), ctypes.byref(opt))
    _check("tqr_factor", rc)
    return A, ws.T


def factor_plain(A: torch.Tensor, tile_b: int, inner_ib: int, ws: Workspace | None = None):
    """In-place tiled QR through the plain boundary call tqr_factor (no
    options: one persistent launch with the library's default policy);
    returns (A, T)."""
    m, n = A.shape
    lda = _ld(A)
    if ws is None:
        ws = Workspace(m, n, 0, tile_b, inner_ib, A.device)
    rc = lib().tqr_factor(m, n, A.data_ptr(), lda, tile_b, inner_ib, ws.T.data_ptr(), ws.work.data_ptr(),
                          ws.work.numel(), _stream())
    _check("tqr_factor", rc)
    return A, ws.T


def factor_noalloc(A: torch.Tensor, T: torch.Tensor, tile_b: int, inner_ib: int):
    """In-place tiled QR through tqr_factor_noalloc: the caller passes A and
    a T of ``t_elems`` doubles; the workspace is the library's fixed scratch
    (no device allocation in the call)."""
    m, n = A.shape
    lda = _ld(A)
    if T.dtype != torch.float64 or not T.is_cuda or T.numel() < max(t_elems(m, n, tile_b, inner_ib), 0):
        raise ValueError("T must be a float64 CUDA tensor of at least t_elems(m, n, tile_b, inner_ib) elements")
    rc = lib().tqr_factor_noalloc(m, n, A.data_ptr(), lda, tile_b, inner_ib, T.data_ptr(), _stream())
    _check("tqr_factor_noalloc", rc)
    return A, T


def _apply(fn: str, A, T, B, tile_b, inner_ib, ws: Workspace | None):
    m, n = A.shape
    nrhs = B.shape[1]
    if ws is None:
        ws = Workspace(m, n, nrhs, tile_b, inner_ib, A.device)
    rc = getattr(lib(), fn)(m, n, nrhs, A.data_ptr(), _ld(A), T.data_ptr(), tile_b, inner_ib, B.data_ptr(), _ld(B),
                            ws.work.data_ptr(), ws.work.numel(), _stream())
    _check(fn, rc)
    return B


def apply_qt(A, T, B, tile_b, inner_ib, ws=None):
    """B <- Q^T B in place (B column-major m x nrhs)."""
    return _apply("tqr_apply_qt", A, T, B, tile_b, inner_ib, ws)


def apply_q(A, T, B, tile_b, inner_ib, ws=None):
    """B <- Q B in place."""
    return _apply("tqr_apply_q", A, T, B, tile_b, inner_ib, ws)


def form_q(A, T, tile_b, inner_ib, Q: torch.Tensor | None = None, ws: Workspace | None = None):
    """The explicit thin Q (m x n, column-major) of a factorisation from
    ``factor``; written into ``Q`` if given, else into a new tensor."""
    m, n = A.shape
    if Q is None:
        Q = torch.empty((n, m), dtype=torch.float64, device=A.device).t()
    if ws is None:
        ws = Workspace(m, n, n, tile_b, inner_ib, A.device)
    rc = lib().tqr_form_q(m, n, A.data_ptr(), _ld(A), T.data_ptr(), tile_b, inner_ib, Q.data_ptr(), _ld(Q),
                          ws.work.data_ptr(), ws.work.numel(), _stream())
    _check("tqr_form_q", rc)
    return Q


def solve_ls(A, B, tile_b, inner_ib, ws: Workspace | None = None, *, workgroups: int = 0,
             status: torch.Tensor | None = None, info: torch.Tensor | None = None, policy: int = POLICY_COLUMN):
    """min ||A X - B||: A overwritten by its factors, X in B[0:n].  Returns
    (B, info tensor on the device).  ``workgroups`` > 0 caps the persistent
    workers of every phase; ``policy`` picks the priority policy
    (tqr_solve_ls_ex)."""
    m, n = A.shape
    nrhs = B.shape[1]
    if ws is None:
        ws = Workspace(m, n, nrhs, tile_b, inner_ib, A.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    if workgroups > 0 or status is not None or policy != POLICY_COLUMN:
        opt = Options(ctypes.sizeof(Options), workgroups, MODE_PERSISTENT, policy, None, None,
                      status.data_ptr() if status is not None else None, 0, None, None)
        rc = lib().tqr_solve_ls_ex(m, n, nrhs, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), tile_b, inner_ib,
                                   ws.T.data_ptr(), ws.work.data_ptr(), ws.work.numel(), info.data_ptr(), _stream(),
                                   ctypes.byref(opt))
        _check("tqr_solve_ls_ex", rc)
    else:
        rc = lib().tqr_solve_ls(m, n, nrhs, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), tile_b, inner_ib,
                                ws.T.data_ptr(), ws.work.data_ptr(), ws.work.numel(), info.data_ptr(), _stream())
        _check("tqr_solve_ls", rc)
    return B, info


# ---- mixed-precision least squares -------------------------------------------------

REFINE_CONVERGED, REFINE_STAGNATED, REFINE_MAX_ITERATIONS, REFINE_BREAKDOWN = 1, 2, 3, 4
REFINE_ETA_TOL = 1e-15

def refine_stats(stats: torch.Tensor):
    """Host copy of a device tqr_refine_stats array (see solve_ls_mixed): a
    list of dicts with iterations, stop and eta per right-hand side."""
    import numpy as np
    raw = stats.cpu().numpy().view(np.dtype([("iterations", "<i4"), ("stop", "<i4"), ("eta", "<f8")]))
    return [{"iterations": int(r["iterations"]), "stop": int(r["stop"]), "eta": float(r["eta"])} for r in raw]


def solve_ls_mixed(A: torch.Tensor, B: torch.Tensor, tile_b: int, iterations: int = 20, *,
                   precision: int = PRECISION_FP32_UPDATES, workgroups: int = 0, work: torch.Tensor | None = None,
                   X: torch.Tensor | None = None, info: torch.Tensor | None = None, events=None,
                   policy: int = POLICY_COLUMN, status: torch.Tensor | None = None):
    """min ||A X - B|| with the factor's trailing updates in FP32 and FP64
    CGLS on A R^{-1} (tqr_solve_ls_mixed), at most ``iterations`` iterations
    per right-hand side.  A and B are column-major and left unchanged;
    returns (X, T, info, stats) with ``stats`` the device tqr_refine_stats
    array (decode with refine_stats)."""
    m, n = A.shape
    nrhs = B.shape[1]
    nb = int(lib().tqr_ls_mixed_workspace_bytes(m, n, nrhs, tile_b))
    if nb < 0:
        raise ValueError("unsupported sizes or tile_b")
    if work is None or work.numel() < nb:
        work = torch.empty(nb, dtype=torch.uint8, device=A.device)
    if X is None:
        X = torch.empty((nrhs, max(n, 1)), dtype=torch.float64, device=A.device).t()[:n]
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    stats = torch.zeros(2 * nrhs, dtype=torch.float64, device=A.device)
    T = torch.zeros(max(t_elems(m, n, tile_b, 16), 1), dtype=torch.float64, device=A.device)
    opt = Options(ctypes.sizeof(Options), workgroups, MODE_PERSISTENT, policy, None, None,
                  status.data_ptr() if status is not None else None, 0,
                  events[0] if events else None, events[1] if events else None, precision, 0)
    rc = lib().tqr_solve_ls_mixed(m, n, nrhs, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), X.data_ptr(),
                                  max(1, X.stride(1) if nrhs > 1 else n), tile_b, iterations, T.data_ptr(),
                                  work.data_ptr(), work.numel(), info.data_ptr(), stats.data_ptr(), _stream(),
                                  ctypes.byref(opt))
    _check("tqr_solve_ls_mixed", rc)
    return X, T, info, stats


# ---- batched factorisation ------------------------------------------------------

class Batch:
    """Many independent problems factorised in one launch (tqr_factor_batched).

    ``shapes`` is a list of (m, n) with m >= n; ``tile_bs`` the tile size of
    each problem and ``inner_ibs`` its inner block (default 16; see
    autotune.tiling_for); ``precision`` PRECISION_FP64 or
    PRECISION_FP32_UPDATES for the whole batch.  The matrices live
    column-major, back to back, in one device buffer ``A``; ``matrix(i)`` is
    problem i's view.  Problems are launched largest first (by the standard
    flop count), which the result does not depend on."""

    def __init__(self, shapes, tile_bs, inner_ibs=None, device="cuda", precision: int = PRECISION_FP64):
        self.shapes = [(int(m), int(n)) for m, n in shapes]
        self.tile_bs = [int(b) for b in tile_bs]
        self.inner_ibs = [16] * len(self.shapes) if inner_ibs is None else [int(ib) for ib in inner_ibs]
        self.precision = int(precision)
        if len(self.tile_bs) != len(self.shapes) or len(self.inner_ibs) != len(self.shapes):
            raise ValueError("one tile size and inner block per problem")
        count = len(self.shapes)
        a_off, t_off, a, t = [], [], 0, 0
        for (m, n), b, ib in zip(self.shapes, self.tile_bs, self.inner_ibs):
            a_off.append(a)
            t_off.append(t)
            a += m * n
            t += max(t_elems(m, n, b, ib), 0)
        self.A = torch.zeros(max(a, 1), dtype=torch.float64, device=device)
        self.T = torch.zeros(max(t, 1), dtype=torch.float64, device=device)
        self.a_off, self.t_off = a_off, t_off
        order = sorted(range(count), key=lambda i: -(self.shapes[i][1] ** 2 * (self.shapes[i][0] - self.shapes[i][1] / 3.0)))
        probs = (BatchProblem * max(count, 1))()
        base_a, base_t = self.A.data_ptr(), self.T.data_ptr()
        for slot, i in enumerate(order):
            m, n = self.shapes[i]
            probs[slot] = BatchProblem(m, n, max(1, m), base_a + 8 * a_off[i], base_t + 8 * t_off[i], self.tile_bs[i],
                                       self.inner_ibs[i], 0)
        nb = int(lib().tqr_batch_plan(count, probs))
        if nb < 0:
            _check("tqr_batch_plan", nb)
        self.work = torch.empty(nb, dtype=torch.uint8, device=device)
        raw = bytes(ctypes.string_at(ctypes.addressof(probs), ctypes.sizeof(BatchProblem) * count))
        self.desc = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device) if count else torch.empty(
            0, dtype=torch.uint8, device=device)
        self.count = count
        self.status = torch.zeros(1, dtype=torch.int32, device=device)

    def load(self, mats) -> None:
        """Copies host matrices (one per problem, shapes as given) in."""
        import numpy as np
        flat = np.concatenate([np.asarray(M, dtype=np.float64).ravel(order="F") for M in mats]) if mats else np.zeros(0)
        if flat.size:
            self.A[:flat.size].copy_(torch.from_numpy(flat))

    def matrix(self, i: int) -> torch.Tensor:
        """Problem i as an (m, n) column-major view of the shared buffer."""
        m, n = self.shapes[i]
        return self.A[self.a_off[i]:self.a_off[i] + m * n].view(n, m).t()

    def t_slots(self, i: int) -> torch.Tensor:
        m, n = self.shapes[i]
        return self.T[self.t_off[i]:self.t_off[i] + t_elems(m, n, self.tile_bs[i], self.inner_ibs[i])]

    def factor(self, workgroups: int = 0) -> None:
        rc = lib().tqr_factor_batched(self.count, ctypes.c_void_p(self.desc.data_ptr() if self.count else 0),
                                      ctypes.c_void_p(self.work.data_ptr()), self.work.numel(),
                                      ctypes.c_void_p(self.status.data_ptr()), int(workgroups), self.precision,
                                      _stream())
        _check("tqr_factor_batched", rc)


# ---- task-graph introspection (host only) ------------------------------------

def graph_tasks(p: int, q: int, tile_b: int) -> int:
    return int(lib().tqr_graph_tasks(p, q, tile_b))


def graph_task(p: int, q: int, tile_b: int, t: int):
    out = (ctypes.c_int32 * 5)()
    if lib().tqr_graph_task(p, q, tile_b, t, out) != 0:
        raise IndexError(t)
    return tuple(out)


def graph_indegree(p: int, q: int, tile_b: int, t: int) -> int:
    return int(lib().tqr_graph_indegree(p, q, tile_b, t))


def graph_successors(p: int, q: int, tile_b: int, t: int):
    buf = (ctypes.c_int64 * 4096)()
    ns = lib().tqr_graph_successors(p, q, tile_b, t, buf, 4096)
    if ns < 0:
        raise IndexError(t)
    return [buf[i] for i in range(ns)]


# ---- raw HIP events on the caller's stream (timing of the scheduler launch) --

class HipEvents:
    """hipEvent_t handles from the HIP runtime already loaded by torch, so the
    events can be recorded by the library on torch's stream."""

    def __init__(self):
        import glob
        self.rt = None
        for name in ("libamdhip64.so.7", "libamdhip64.so"):
            try:
                self.rt = ctypes.CDLL(name, mode=ctypes.RTLD_GLOBAL)
                break
            except OSError:
                continue
        if self.rt is None:
            cands = glob.glob(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so*"))
            self.rt = ctypes.CDLL(cands[0], mode=ctypes.RTLD_GLOBAL)
        self.rt.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.rt.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.rt.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        ev = ctypes.c_void_p()
        if self.rt.hipEventCreate(ctypes.byref(ev)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return ev.value

    def elapsed_ms(self, a, b) -> float:
        self.rt.hipEventSynchronize(ctypes.c_void_p(b))
        out = ctypes.c_float()
        if self.rt.hipEventElapsedTime(ctypes.byref(out), ctypes.c_void_p(a), ctypes.c_void_p(b)) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(out.value)

    def destroy(self, ev):
        self.rt.hipEventDestroy(ctypes.c_void_p(ev))
