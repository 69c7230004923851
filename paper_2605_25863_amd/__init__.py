"""linac-mi355x: exact Gaussian elimination over F_p on AMD MI355X (gfx950).

A thin ctypes binding of the C-ABI library ``liblinac_mi355x.so`` (declared in
include/linac.h).  Every step of the elimination runs in the library's HIP
kernels; this module only marshals arguments.  PyTorch provides device memory
and the current stream.

User-level calls follow the paper (Sec. 2.3 "Basic Usage", Sec. 5.1-5.2):

* ``row_reduce(matrix, field_characteristic)`` -- the RREF in the original
  shape, zero rows at the bottom (``cuda_row_reduce`` in the paper);
* ``rref(A, p)`` -- (R, rank, pivots) on device tensors;
* ``solve(A, B, p)`` -- (X, rank, pivots, consistent): the particular
  solution of A X = B with free variables zero;
* ``solve_batched(systems)`` -- many independent systems in one launch;
* ``drop_bottom_zero_rows`` and ``pivot_columns_from_row_reduced_echelon_form``
  -- the helpers of Sec. 2.3 and Sec. 5.1.

Inputs may be numpy arrays (copied to ``cuda:0`` and results copied back) or
torch int32 CUDA tensors (residues below 2^31 have the same bits as uint32).
There is no CPU fallback: without the built library or a GPU these calls
raise.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "LinacError", "library_path", "row_reduce", "rref", "solve", "solve_batched",
    "drop_bottom_zero_rows", "pivot_columns_from_row_reduced_echelon_form", "HipTimer",
    "PATH_AUTO", "PATH_PLAIN", "PATH_BLOCKED_INT8", "PATH_BLOCKED_FP64", "check_prime",
    "load_tuning", "TUNING_FILE", "LaunchTimes", "rref_workspace_bytes",
]

PATH_AUTO, PATH_PLAIN, PATH_BLOCKED_INT8, PATH_BLOCKED_FP64 = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liblinac_mi355x.so")
TUNING_FILE = os.path.join(_HERE, "tuning_gfx950.json")
_lib = None


class LinacError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _load()
        msg = lib.linac_status_string(status).decode()
        if status == 7:
            msg += f" (hip error {lib.linac_last_hip_error()})"
        super().__init__(f"{where}: {msg}")
        self.status = status


class _Opts(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int), ("panel_width", ctypes.c_int),
                ("validate", ctypes.c_int), ("verbose", ctypes.c_int),
                ("ev_begin", ctypes.c_void_p), ("ev_end", ctypes.c_void_p),
                ("dominant_launches", ctypes.POINTER(ctypes.c_int64)),
                ("launch_events", ctypes.POINTER(ctypes.c_void_p)),
                ("launch_kinds", ctypes.POINTER(ctypes.c_int32)),
                ("launch_cap", ctypes.c_int32),
                ("launch_used", ctypes.POINTER(ctypes.c_int32))]


KERNEL_KINDS = {1: "step", 2: "leaf_product", 3: "trail_product", 4: "batched", 5: "select",
                6: "operands"}


class _System(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("X", ctypes.c_void_p),
                ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("lda", ctypes.c_int32), ("ldb", ctypes.c_int32), ("ldx", ctypes.c_int32),
                ("p", ctypes.c_uint32), ("rank", ctypes.c_void_p), ("pivots", ctypes.c_void_p),
                ("consistent", ctypes.c_void_p)]


def library_path() -> str:
    return _LIBPATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise RuntimeError(f"{_LIBPATH} is not built; run `python -m paper_2605_25863_amd.build`")
    lib = ctypes.CDLL(_LIBPATH)
    vp, i64, u32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    optp = ctypes.POINTER(_Opts)
    szp = ctypes.POINTER(ctypes.c_size_t)
    lib.linac_plan.argtypes = [i64, i64, optp, ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_int)]
    lib.linac_rref_workspace.argtypes = [i64, i64, optp, szp]
    lib.linac_rref.argtypes = [vp, i64, i64, i64, u32, vp, vp, vp, sz, optp, vp]
    lib.linac_solve_workspace.argtypes = [i64, i64, i64, optp, szp]
    lib.linac_solve.argtypes = [vp, i64, i64, i64, vp, i64, i64, u32, vp, i64, vp, vp, vp, vp, sz,
                                optp, vp]
    lib.linac_solve_batched_workspace.argtypes = [ctypes.POINTER(_System), ctypes.c_int32, optp,
                                                  szp]
    lib.linac_solve_batched.argtypes = [ctypes.POINTER(_System), ctypes.c_int32, vp, sz, optp, vp]
    lib.linac_load_tuning.argtypes = [ctypes.c_char_p]
    lib.linac_check_prime.argtypes = [u32]
    lib.linac_status_string.restype = ctypes.c_char_p
    lib.linac_status_string.argtypes = [ctypes.c_int]
    for name in ("linac_plan", "linac_rref_workspace", "linac_rref", "linac_solve_workspace", "linac_solve",
                 "linac_solve_batched_workspace", "linac_solve_batched", "linac_load_tuning",
                 "linac_check_prime", "linac_version", "linac_last_hip_error"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    if os.path.exists(TUNING_FILE):
        with open(TUNING_FILE) as f:
            _check(lib.linac_load_tuning(f.read().encode()), "linac_load_tuning")
    return lib


def _check(status: int, where: str):
    if status != 0:
        raise LinacError(status, where)


def load_tuning(json_text):
    """Install a tuning table (JSON text, see include/linac.h); None restores the
    built-in defaults.  Tables only change speed, never results."""
    lib = _load()
    _check(lib.linac_load_tuning(None if json_text is None else json_text.encode()),
           "linac_load_tuning")


def restore_tuning():
    """Back to the table loaded at import: the shipped tuning file if there is
    one, else the built-in defaults."""
    if os.path.exists(TUNING_FILE):
        with open(TUNING_FILE) as f:
            load_tuning(f.read())
    else:
        load_tuning(None)


def check_prime(p: int) -> int:
    """Status of the library's host-side modulus check (0 = usable prime)."""
    return int(_load().linac_check_prime(int(p)))


def _opts(path=PATH_AUTO, panel_width=0, validate=False, verbose=False, events=None,
          launches=None, per_launch=None):
    o = _Opts()
    o.path, o.panel_width = int(path), int(panel_width)
    o.validate, o.verbose = int(bool(validate)), int(bool(verbose))
    if events is not None:
        o.ev_begin, o.ev_end = events.begin, events.end
    if launches is not None:
        o.dominant_launches = ctypes.pointer(launches)
    if per_launch is not None:
        o.launch_events = per_launch.events
        o.launch_kinds = per_launch.kinds
        o.launch_cap = per_launch.cap
        o.launch_used = ctypes.pointer(per_launch.used)
    return o


class LaunchTimes:
    """Events for the library's per-launch timing hook: after a call,
    by_kind() returns {kind: (launches, total_ms)}."""

    def __init__(self, cap: int):
        self._hip = ctypes.CDLL("libamdhip64.so")
        self.cap = int(cap)
        self.events = (ctypes.c_void_p * (2 * self.cap))()
        for i in range(2 * self.cap):
            ev = ctypes.c_void_p()
            assert self._hip.hipEventCreate(ctypes.byref(ev)) == 0
            self.events[i] = ev.value
        self.kinds = (ctypes.c_int32 * self.cap)()
        self.used = ctypes.c_int32(0)

    def by_kind(self):
        self._hip.hipEventSynchronize(ctypes.c_void_p(self.events[2 * self.used.value - 1]))
        out = {}
        ms = ctypes.c_float()
        for i in range(self.used.value):
            assert self._hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self.events[2 * i]),
                                                 ctypes.c_void_p(self.events[2 * i + 1])) == 0
            name = KERNEL_KINDS.get(self.kinds[i], str(self.kinds[i]))
            n, t = out.get(name, (0, 0.0))
            out[name] = (n + 1, t + ms.value)
        return out

    def __del__(self):
        try:
            for i in range(2 * self.cap):
                self._hip.hipEventDestroy(ctypes.c_void_p(self.events[i]))
        except Exception:
            pass


# ---------------------------------------------------------------------------
# torch plumbing (device memory and streams only)
# ---------------------------------------------------------------------------

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("linac_mi355x needs a ROCm GPU; none is visible")
    return torch


def _stream(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _to_dev(torch, M, device):
    """(tensor int32 on device, was_numpy)."""
    if isinstance(M, np.ndarray):
        arr = np.ascontiguousarray(M)
        if arr.size and int(arr.max()) >= (1 << 31):
            raise ValueError("entries must be residues below 2^31")
        t = torch.from_numpy(arr.astype(np.int64).astype(np.int32)).to(device)
        return t, True
    if not M.is_cuda:
        raise ValueError("torch inputs must be CUDA tensors")
    if M.dtype != torch.int32:
        raise ValueError("torch inputs must be int32 residues")
    return M.contiguous(), False


def _workspace(torch, nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


class HipTimer:
    """A pair of HIP events (created through the HIP runtime) for the library's
    ev_begin / ev_end hooks; elapsed_ms() synchronises on the end event."""

    def __init__(self):
        self._hip = ctypes.CDLL("libamdhip64.so")
        self.begin = ctypes.c_void_p()
        self.end = ctypes.c_void_p()
        assert self._hip.hipEventCreate(ctypes.byref(self.begin)) == 0
        assert self._hip.hipEventCreate(ctypes.byref(self.end)) == 0
        self.begin, self.end = self.begin.value, self.end.value

    def record_begin(self, stream):
        assert self._hip.hipEventRecord(ctypes.c_void_p(self.begin), stream) == 0

    def record_end(self, stream):
        assert self._hip.hipEventRecord(ctypes.c_void_p(self.end), stream) == 0

    def elapsed_ms(self) -> float:
        assert self._hip.hipEventSynchronize(ctypes.c_void_p(self.end)) == 0
        ms = ctypes.c_float()
        assert self._hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self.begin),
                                             ctypes.c_void_p(self.end)) == 0
        return float(ms.value)

    def __del__(self):
        try:
            self._hip.hipEventDestroy(ctypes.c_void_p(self.begin))
            self._hip.hipEventDestroy(ctypes.c_void_p(self.end))
        except Exception:
            pass


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def rref(A, p: int, *, inplace: bool = False, path: int = PATH_AUTO, validate: bool = False,
         verbose: bool = False, stream=None, events: HipTimer | None = None, launches=None,
         panel_width: int = 0, per_launch: "LaunchTimes | None" = None, workspace=None):
    """RREF of A over F_p.  Returns (R, rank, pivots) as device tensors (R int32
    m x n, rank int32[1], pivots int32[min(m, n)], ascending, -1 padded)."""
    torch = _torch()
    lib = _load()
    dev = torch.device("cuda", torch.cuda.current_device())
    At, _ = _to_dev(torch, A, dev)
    if not inplace and not isinstance(A, np.ndarray):
        At = At.clone()
    m, n = At.shape
    rank = torch.zeros(1, dtype=torch.int32, device=dev)
    pivots = torch.empty(min(m, n), dtype=torch.int32, device=dev)
    o = _opts(path, panel_width, validate, verbose, events, launches, per_launch)
    need = ctypes.c_size_t()
    _check(lib.linac_rref_workspace(m, n, ctypes.byref(o), ctypes.byref(need)), "rref_workspace")
    ws = workspace if workspace is not None else _workspace(torch, need.value, dev)
    _check(lib.linac_rref(_ptr(At), m, n, max(n, 1), int(p), _ptr(rank), _ptr(pivots), _ptr(ws),
                          ws.numel(), ctypes.byref(o), _stream(torch, stream)), "linac_rref")
    return At, rank, pivots


def row_reduce(matrix, field_characteristic: int = 0, verbose: bool = False, **kw):
    """RREF of ``matrix`` mod ``field_characteristic`` (the paper's
    cuda_row_reduce, Sec. 2.3).  Same container type out as in."""
    if field_characteristic == 0:
        raise NotImplementedError("floating-point row reduction is outside this library; "
                                  "pass a prime field_characteristic")
    torch = _torch()
    R, rank, piv = rref(matrix, field_characteristic, verbose=verbose, **kw)
    if isinstance(matrix, np.ndarray):
        torch.cuda.synchronize()
        return R.cpu().numpy().astype(matrix.dtype if matrix.dtype != np.int32 else np.int32)
    return R


def solve(A, B, p: int, *, path: int = PATH_AUTO, validate: bool = False, verbose: bool = False,
          stream=None, events: HipTimer | None = None, launches=None, out=None, workspace=None,
          panel_width: int = 0, per_launch: "LaunchTimes | None" = None):
    """Solve A X = B over F_p (Sec. 5.2).  Returns (X, rank, pivots, consistent).

    numpy in -> numpy out (rank as int); torch in -> device tensors out.
    ``out`` may supply preallocated (X, rank, pivots, consistent) tensors and
    ``workspace`` a preallocated uint8 tensor, so repeated calls allocate
    nothing.
    """
    torch = _torch()
    lib = _load()
    dev = torch.device("cuda", torch.cuda.current_device())
    At, was_np = _to_dev(torch, A, dev)
    Bt, _ = _to_dev(torch, B, dev)
    m, n = At.shape
    k = Bt.shape[1]
    if Bt.shape[0] != m:
        raise ValueError("A and B must have the same number of rows")
    if out is None:
        X = torch.empty((n, k), dtype=torch.int32, device=dev)
        rank = torch.zeros(1, dtype=torch.int32, device=dev)
        pivots = torch.empty(min(m, n), dtype=torch.int32, device=dev)
        cons = torch.empty(k, dtype=torch.uint8, device=dev)
    else:
        X, rank, pivots, cons = out
    o = _opts(path, panel_width, validate, verbose, events, launches, per_launch)
    need = ctypes.c_size_t()
    _check(lib.linac_solve_workspace(m, n, k, ctypes.byref(o), ctypes.byref(need)),
           "solve_workspace")
    ws = workspace if workspace is not None else _workspace(torch, need.value, dev)
    _check(lib.linac_solve(_ptr(At), m, n, max(n, 1), _ptr(Bt), k, max(k, 1), int(p), _ptr(X),
                           max(k, 1), _ptr(rank), _ptr(pivots), _ptr(cons), _ptr(ws),
                           ws.numel(), ctypes.byref(o), _stream(torch, stream)), "linac_solve")
    if was_np:
        torch.cuda.synchronize()
        return (X.cpu().numpy().astype(np.uint32), int(rank.item()),
                pivots.cpu().numpy()[: int(rank.item())].astype(np.int64),
                cons.cpu().numpy().astype(np.uint8))
    return X, rank, pivots, cons


def plan(m: int, n: int, path: int = PATH_AUTO, panel_width: int = 0):
    """(path, panel width) a call on an m x n system takes: AUTO resolved by
    size and the tuning table; panel 0 on the plain path (linac_plan)."""
    lib = _load()
    o = _opts(path, panel_width)
    pth, pw = ctypes.c_int(), ctypes.c_int()
    _check(lib.linac_plan(m, n, ctypes.byref(o), ctypes.byref(pth), ctypes.byref(pw)), "plan")
    return int(pth.value), int(pw.value)


def rref_workspace_bytes(m: int, n: int, path: int = PATH_AUTO, panel_width: int = 0) -> int:
    lib = _load()
    o = _opts(path, panel_width)
    need = ctypes.c_size_t()
    _check(lib.linac_rref_workspace(m, n, ctypes.byref(o), ctypes.byref(need)), "rref_workspace")
    return int(need.value)


def solve_workspace_bytes(m: int, n: int, k: int, path: int = PATH_AUTO,
                          panel_width: int = 0) -> int:
    lib = _load()
    o = _opts(path, panel_width)
    need = ctypes.c_size_t()
    _check(lib.linac_solve_workspace(m, n, k, ctypes.byref(o), ctypes.byref(need)),
           "solve_workspace")
    return int(need.value)


def solve_batched(systems, *, path: int = PATH_AUTO, verbose: bool = False, stream=None,
                  events: HipTimer | None = None, launches=None, prepared=None, per_launch=None,
                  validate: bool = False):
    """Solve many independent systems in one launch.

    ``systems``: list of dicts {A, B, p} (numpy or device int32 tensors).
    Returns a list of (X, rank, pivots, consistent) like ``solve``.
    ``prepared`` (from ``prepare_batched``) reuses device buffers and the
    workspace so the call allocates nothing.
    """
    torch = _torch()
    prep = prepared if prepared is not None else prepare_batched(systems)
    lib = _load()
    o = _opts(path, 0, validate, verbose, events, launches, per_launch)
    _check(lib.linac_solve_batched(prep["desc"], len(prep["items"]), _ptr(prep["ws"]),
                                   prep["ws"].numel(), ctypes.byref(o), _stream(torch, stream)),
           "linac_solve_batched")
    if prepared is not None:
        return prep
    torch.cuda.synchronize()
    out = []
    for it in prep["items"]:
        r = int(it["rank"].item())
        k = it["X"].shape[1]
        out.append((it["X"].cpu().numpy().astype(np.uint32), r,
                    it["pivots"].cpu().numpy()[:r].astype(np.int64),
                    it["cons"].cpu().numpy()[:k].astype(np.uint8)))
    return out


def prepare_batched(systems, path: int = PATH_AUTO):
    """Device copies, output buffers, descriptors and workspace for a batch."""
    torch = _torch()
    lib = _load()
    dev = torch.device("cuda", torch.cuda.current_device())
    items = []
    desc = (_System * max(len(systems), 1))()
    for i, s in enumerate(systems):
        At, _ = _to_dev(torch, s["A"], dev)
        Bt, _ = _to_dev(torch, s["B"], dev)
        m, n = At.shape
        k = Bt.shape[1]
        it = dict(A=At, B=Bt, X=torch.zeros((n, k), dtype=torch.int32, device=dev),
                  rank=torch.zeros(1, dtype=torch.int32, device=dev),
                  pivots=torch.empty(max(min(m, n), 1), dtype=torch.int32, device=dev),
                  cons=torch.empty(max(k, 1), dtype=torch.uint8, device=dev), p=int(s["p"]))
        items.append(it)
        d = desc[i]
        d.A, d.B, d.X = _ptr(At), _ptr(Bt), _ptr(it["X"])
        d.m, d.n, d.k = m, n, k
        d.lda, d.ldb, d.ldx = max(n, 1), max(k, 1), max(k, 1)
        d.p = int(s["p"])
        d.rank, d.pivots, d.consistent = _ptr(it["rank"]), _ptr(it["pivots"]), _ptr(it["cons"])
    o = _opts(path)
    need = ctypes.c_size_t()
    _check(lib.linac_solve_batched_workspace(desc, len(systems), ctypes.byref(o),
                                             ctypes.byref(need)), "solve_batched_workspace")
    ws = _workspace(torch, need.value, dev)
    return dict(items=items, desc=desc, ws=ws)


def drop_bottom_zero_rows(R):
    """R without its trailing all-zero rows (Sec. 2.3 footnote)."""
    keep = R.shape[0]
    while keep and not bool((R[keep - 1] != 0).any()):
        keep -= 1
    return R[:keep]


def pivot_columns_from_row_reduced_echelon_form(R):
    """Column of the leading 1 in each non-zero row of an RREF (Sec. 5.1)."""
    out = []
    for row in R:
        nz = np.nonzero(np.asarray(row.cpu() if hasattr(row, "cpu") else row))[0]
        if len(nz):
            out.append(int(nz[0]))
    return out
