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
* ``rref_batched(matrices, p)`` -- the RREF of many matrices in one call,
  reduced concurrently on the library's stream lanes;
* ``load_matrix(bases, lindices, p)`` -- the matrix of a monomial ansatz at
  sampling points (``cuda_load_matrix``, Sec. 3.3);
* ``canonical_kernel(R, rank, pivots, p)``, ``column_basis`` and
  ``rank_factorization(A, p)`` -- the null-space basis and the rank
  factorisation A = C R read off the RREF (Sec. 5.1);
* ``rref_u64`` / ``solve_u64`` -- the same for 64-bit primes below 2^63
  (uint64 residues, Sec. 3.2 "Number types"), and ``lup(A, p)`` -- the LUP
  factorisation P A = L U with a fixed pivot rule (future work of Sec. 6);
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
    "load_tuning", "TUNING_FILE", "LaunchTimes", "rref_workspace_bytes", "load_matrix",
    "canonical_kernel", "column_basis", "rank_factorization", "rref_batched", "rref_u64",
    "solve_u64", "lup", "solve_noalloc",
    "NOALLOC_SCRATCH_BYTES",
]

NOALLOC_SCRATCH_BYTES = 64 << 20  # LINAC_NOALLOC_SCRATCH_BYTES in include/linac.h

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
                6: "operands", 7: "leaf_fused"}


class _Matrix(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("p", ctypes.c_uint32), ("rank", ctypes.c_void_p),
                ("pivots", ctypes.c_void_p)]


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
    # torch ships its own HIP runtime under the same soname as the system one
    # the library links; whichever loads first serves the whole process.  Load
    # torch's first, so that both see the devices through one runtime (with the
    # system runtime first, the library's calls found no device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
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
    lib.linac_solve_noalloc.argtypes = [vp, i64, i64, i64, vp, i64, i64, u32, vp, i64, vp, vp, vp,
                                        optp, vp]
    lib.linac_rref_batched_workspace.argtypes = [ctypes.POINTER(_Matrix), ctypes.c_int32, optp, szp]
    lib.linac_rref_batched.argtypes = [ctypes.POINTER(_Matrix), ctypes.c_int32, vp, sz, optp, vp]
    u64 = ctypes.c_uint64
    lib.linac_rref_u64_workspace.argtypes = [i64, i64, szp]
    lib.linac_rref_u64.argtypes = [vp, i64, i64, i64, u64, vp, vp, vp, sz, optp, vp]
    lib.linac_solve_u64_workspace.argtypes = [i64, i64, i64, szp]
    lib.linac_solve_u64.argtypes = [vp, i64, i64, i64, vp, i64, i64, u64, vp, i64, vp, vp, vp, vp,
                                    sz, optp, vp]
    lib.linac_lup_workspace.argtypes = [i64, i64, ctypes.c_int, szp]
    lib.linac_lup.argtypes = [vp, i64, i64, i64, u32, vp, vp, vp, vp, sz, optp, vp]
    lib.linac_lup_u64.argtypes = [vp, i64, i64, i64, u64, vp, vp, vp, vp, sz, optp, vp]
    lib.linac_check_prime_u64.argtypes = [u64]
    lib.linac_load_matrix.argtypes = [vp, i64, i64, i64, vp, i64, i64, i64, u32, vp, i64, vp]
    lib.linac_nullspace.argtypes = [vp, i64, i64, i64, vp, vp, u32, vp, i64, i64, vp, vp]
    lib.linac_column_basis.argtypes = [vp, i64, i64, i64, vp, vp, vp, i64, i64, vp]
    lib.linac_load_tuning.argtypes = [ctypes.c_char_p]
    lib.linac_check_prime.argtypes = [u32]
    lib.linac_status_string.restype = ctypes.c_char_p
    lib.linac_status_string.argtypes = [ctypes.c_int]
    for name in ("linac_plan", "linac_rref_workspace", "linac_rref", "linac_solve_workspace", "linac_solve",
                 "linac_solve_batched_workspace", "linac_solve_batched", "linac_load_tuning",
                 "linac_check_prime", "linac_version", "linac_last_hip_error",
                 "linac_load_matrix", "linac_nullspace", "linac_column_basis",
                 "linac_rref_batched_workspace", "linac_rref_batched",
                 "linac_rref_u64_workspace", "linac_rref_u64", "linac_solve_u64_workspace",
                 "linac_solve_u64", "linac_lup_workspace", "linac_lup", "linac_lup_u64",
                 "linac_check_prime_u64",
                 "linac_solve_noalloc"):
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


def solve_noalloc(A, B, p: int, *, path: int = PATH_AUTO, verbose: bool = False, stream=None,
                  out=None, panel_width: int = 0):
    """``solve`` through linac_solve_noalloc: the library's fixed scratch
    array instead of a workspace (for callers that cannot allocate).  With
    ``out`` = preallocated (X, rank, pivots, consistent) tensors and device
    inputs the call allocates nothing.  Calls that overlap on one GPU race."""
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
    o = _opts(path, panel_width, False, verbose)
    _check(lib.linac_solve_noalloc(_ptr(At), m, n, max(n, 1), _ptr(Bt), k, max(k, 1), int(p),
                                   _ptr(X), max(k, 1), _ptr(rank), _ptr(pivots), _ptr(cons),
                                   ctypes.byref(o), _stream(torch, stream)), "linac_solve_noalloc")
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


def rref_batched(matrices, p, *, inplace: bool = False, path: int = PATH_AUTO,
                 panel_width: int = 0, validate: bool = False, verbose: bool = False,
                 stream=None, events: HipTimer | None = None, workspace=None, outs=None):
    """RREF of every matrix in ``matrices`` (numpy arrays or int32 CUDA
    tensors) in one linac_rref_batched call; ``p`` is one prime or one per
    matrix.  Returns a list of (R, rank, pivots) device tensors like ``rref``
    (numpy in -> numpy R and int rank / pivots out).  With ``inplace`` device
    inputs are overwritten; ``workspace`` may be a preallocated uint8 tensor
    and ``outs`` preallocated (rank, pivots) pairs."""
    torch = _torch()
    lib = _load()
    dev = torch.device("cuda", torch.cuda.current_device())
    count = len(matrices)
    ps = list(p) if isinstance(p, (list, tuple)) else [int(p)] * count
    desc = (_Matrix * max(count, 1))()
    items = []
    any_np = False
    for i, M in enumerate(matrices):
        At, was_np = _to_dev(torch, M, dev)
        any_np |= was_np
        if not inplace and not was_np:
            At = At.clone()
        m, n = At.shape
        if outs is not None:
            rank, piv = outs[i]
        else:
            rank = torch.zeros(1, dtype=torch.int32, device=dev)
            piv = torch.empty(min(m, n), dtype=torch.int32, device=dev)
        items.append((At, rank, piv))
        d = desc[i]
        d.A, d.m, d.n, d.lda, d.p = _ptr(At), m, n, max(n, 1), int(ps[i])
        d.rank, d.pivots = _ptr(rank), _ptr(piv)
    o = _opts(path, panel_width, validate, verbose, events)
    if workspace is None:
        need = ctypes.c_size_t()
        _check(lib.linac_rref_batched_workspace(desc, count, ctypes.byref(o), ctypes.byref(need)),
               "rref_batched_workspace")
        workspace = _workspace(torch, need.value, dev)
    _check(lib.linac_rref_batched(desc, count, _ptr(workspace), workspace.numel(), ctypes.byref(o),
                                  _stream(torch, stream)), "linac_rref_batched")
    if any_np:
        torch.cuda.synchronize()
        out = []
        for (At, rank, piv), M in zip(items, matrices):
            r = int(rank.item())
            out.append((At.cpu().numpy().astype(np.uint32), r,
                        piv.cpu().numpy()[:r].astype(np.int64)))
        return out
    return items


def rref_batched_workspace_bytes(shapes, path: int = PATH_AUTO, panel_width: int = 0) -> int:
    """Workspace of linac_rref_batched for matrices of these (m, n) shapes."""
    lib = _load()
    desc = (_Matrix * max(len(shapes), 1))()
    for i, (m, n) in enumerate(shapes):
        desc[i].m, desc[i].n, desc[i].lda = m, n, max(n, 1)
    o = _opts(path, panel_width)
    need = ctypes.c_size_t()
    _check(lib.linac_rref_batched_workspace(desc, len(shapes), ctypes.byref(o), ctypes.byref(need)),
           "rref_batched_workspace")
    return int(need.value)


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


def _to_dev_index(torch, L, device):
    if isinstance(L, np.ndarray):
        arr = np.ascontiguousarray(L)
        if arr.size and (int(arr.max()) >= (1 << 31) or int(arr.min()) < -(1 << 31)):
            raise ValueError("indices must fit int32")
        return torch.from_numpy(arr.astype(np.int32)).to(device), True
    if not L.is_cuda or L.dtype != torch.int32:
        raise ValueError("torch lindices must be an int32 CUDA tensor")
    return L.contiguous(), False


def load_matrix(bases, lindices, p: int, *, stream=None, out=None):
    """A[r, c] = prod_t bases[r, lindices[c, t]] mod p (the paper's
    cuda_load_matrix, Sec. 3.3): one row per sampling point, one column per
    monomial.  numpy in -> numpy out; torch int32 CUDA tensors -> device
    tensor.  ``out`` may supply the nrows x ncols int32 result tensor."""
    torch = _torch()
    lib = _load()
    dev = torch.device("cuda", torch.cuda.current_device())
    Bt, was_np = _to_dev(torch, bases, dev)
    Lt, _ = _to_dev_index(torch, lindices, dev)
    nrows, nb = Bt.shape
    ncols, d = Lt.shape
    A = out if out is not None else torch.empty((nrows, ncols), dtype=torch.int32, device=dev)
    _check(lib.linac_load_matrix(_ptr(Bt), nrows, nb, max(nb, 1), _ptr(Lt), ncols, d, max(d, 1),
                                 int(p), _ptr(A), max(ncols, 1), _stream(torch, stream)),
           "linac_load_matrix")
    if was_np:
        torch.cuda.synchronize()
        return A.cpu().numpy().astype(np.uint32)
    return A


def canonical_kernel(R, rank, pivots, p: int, *, kcols=None, stream=None, with_free=False):
    """Null-space basis K (n x kcols device tensor, kcols = n by default) of the
    RREF R (device int32, as ``rref`` returns it, with its device rank and
    pivots): columns f < n - r hold the canonical basis (free variables -I),
    later columns are zero (linac_nullspace, Sec. 5.1).  With ``with_free``
    also returns the free columns (int32[n], -1 padded)."""
    torch = _torch()
    lib = _load()
    m, n = R.shape
    kc = n if kcols is None else int(kcols)
    K = torch.empty((n, kc), dtype=torch.int32, device=R.device)
    free = torch.empty(max(n, 1), dtype=torch.int32, device=R.device) if with_free else None
    _check(lib.linac_nullspace(_ptr(R), m, n, max(n, 1), _ptr(rank), _ptr(pivots), int(p), _ptr(K),
                               kc, max(kc, 1), _ptr(free), _stream(torch, stream)),
           "linac_nullspace")
    return (K, free) if with_free else K


def column_basis(A, rank, pivots, *, ccols=None, stream=None):
    """C = A[:, J] (m x ccols device tensor, ccols = min(m, n) by default,
    columns from the rank on zero) for the pivot columns J of A's RREF
    (linac_column_basis, Sec. 5.1)."""
    torch = _torch()
    lib = _load()
    m, n = A.shape
    cc = min(m, n) if ccols is None else int(ccols)
    C = torch.empty((m, cc), dtype=torch.int32, device=A.device)
    _check(lib.linac_column_basis(_ptr(A), m, n, max(n, 1), _ptr(rank), _ptr(pivots), _ptr(C), cc,
                                  max(cc, 1), _stream(torch, stream)), "linac_column_basis")
    return C


def rank_factorization(A, p: int, **kw):
    """(C, R, K, rank): A = C R with C = A[:, J] (m x r) and R the r non-zero
    rows of the RREF (r x n), and K (n x (n - r)) with A K = 0 (Sec. 5.1).
    numpy in -> numpy out; a torch int32 CUDA tensor -> device tensors (the
    rank is read back once to trim the shapes)."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device())
    At, was_np = _to_dev(torch, A, dev)
    R, rank, piv = rref(At, p, **kw)
    C = column_basis(At, rank, piv)
    K = canonical_kernel(R, rank, piv, p)
    r = int(rank.item())
    n = At.shape[1]
    C, R, K = C[:, :r], R[:r], K[:, : n - r]
    if was_np:
        return (C.cpu().numpy().astype(np.uint32), R.cpu().numpy().astype(np.uint32),
                K.cpu().numpy().astype(np.uint32), r)
    return C, R, K, r



def _to_dev64(torch, M, device):
    """(int64 tensor on device, was_numpy): 64-bit residues below 2^63 have the
    same bits as int64."""
    if isinstance(M, np.ndarray):
        arr = np.ascontiguousarray(M)
        if arr.size and int(arr.max()) >= (1 << 63):
            raise ValueError("entries must be residues below 2^63")
        return torch.from_numpy(arr.astype(np.uint64).view(np.int64)).to(device), True
    if not M.is_cuda or M.dtype != torch.int64:
        raise ValueError("torch inputs of the 64-bit calls must be int64 CUDA tensors")
    return M.contiguous(), False


def _u64_out(t):
    return t.cpu().numpy().view(np.uint64)


def rref_u64(A, p: int, *, inplace: bool = False, validate: bool = False, stream=None):
    """RREF over F_p for a prime p < 2^63 (linac_rref_u64).  numpy uint64 in ->
    (R uint64, rank, pivots) numpy out; int64 CUDA tensors -> device tensors."""
    torch = _torch()
    lib = _load()
    dev = torch.device("cuda", torch.cuda.current_device())
    At, was_np = _to_dev64(torch, A, dev)
    if not inplace and not was_np:
        At = At.clone()
    m, n = At.shape
    rank = torch.zeros(1, dtype=torch.int32, device=dev)
    piv = torch.empty(min(m, n), dtype=torch.int32, device=dev)
    need = ctypes.c_size_t()
    _check(lib.linac_rref_u64_workspace(m, n, ctypes.byref(need)), "rref_u64_workspace")
    ws = _workspace(torch, need.value, dev)
    o = _opts(validate=validate)
    _check(lib.linac_rref_u64(_ptr(At), m, n, max(n, 1), int(p), _ptr(rank), _ptr(piv), _ptr(ws),
                              ws.numel(), ctypes.byref(o), _stream(torch, stream)), "linac_rref_u64")
    if was_np:
        torch.cuda.synchronize()
        r = int(rank.item())
        return _u64_out(At), r, piv.cpu().numpy()[:r].astype(np.int64)
    return At, rank, piv


def solve_u64(A, B, p: int, *, validate: bool = False, stream=None):
    """Solve A X = B over F_p for a prime p < 2^63 (linac_solve_u64).  numpy
    in -> (X uint64, rank, pivots, consistent) numpy out."""
    torch = _torch()
    lib = _load()
    dev = torch.device("cuda", torch.cuda.current_device())
    At, was_np = _to_dev64(torch, A, dev)
    Bt, _ = _to_dev64(torch, B, dev)
    m, n = At.shape
    k = Bt.shape[1]
    X = torch.empty((n, k), dtype=torch.int64, device=dev)
    rank = torch.zeros(1, dtype=torch.int32, device=dev)
    piv = torch.empty(min(m, n), dtype=torch.int32, device=dev)
    cons = torch.empty(k, dtype=torch.uint8, device=dev)
    need = ctypes.c_size_t()
    _check(lib.linac_solve_u64_workspace(m, n, k, ctypes.byref(need)), "solve_u64_workspace")
    ws = _workspace(torch, need.value, dev)
    o = _opts(validate=validate)
    _check(lib.linac_solve_u64(_ptr(At), m, n, max(n, 1), _ptr(Bt), k, max(k, 1), int(p), _ptr(X),
                               max(k, 1), _ptr(rank), _ptr(piv), _ptr(cons), _ptr(ws), ws.numel(),
                               ctypes.byref(o), _stream(torch, stream)), "linac_solve_u64")
    if was_np:
        torch.cuda.synchronize()
        r = int(rank.item())
        return (_u64_out(X), r, piv.cpu().numpy()[:r].astype(np.int64),
                cons.cpu().numpy().astype(np.uint8))
    return X, rank, piv, cons


def lup(A, p: int, *, wide: bool | None = None, inplace: bool = False, validate: bool = False,
        stream=None):
    """P A = L U (linac_lup / linac_lup_u64): returns (LU, perm, rank, pivots)
    with LU the packed factors in P order (see include/linac.h).  ``wide``
    selects the 64-bit call (default: when p >= 2^31 or the input is uint64 /
    int64).  numpy in -> numpy out (LU uint32 or uint64)."""
    torch = _torch()
    lib = _load()
    dev = torch.device("cuda", torch.cuda.current_device())
    if wide is None:
        wide = p >= (1 << 31) or (isinstance(A, np.ndarray) and A.dtype in (np.uint64, np.int64)) \
            or (not isinstance(A, np.ndarray) and A.dtype == torch.int64)
    At, was_np = (_to_dev64 if wide else _to_dev)(torch, A, dev)
    if not inplace and not was_np:
        At = At.clone()
    m, n = At.shape
    perm = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    rank = torch.zeros(1, dtype=torch.int32, device=dev)
    piv = torch.empty(min(m, n), dtype=torch.int32, device=dev)
    need = ctypes.c_size_t()
    _check(lib.linac_lup_workspace(m, n, int(wide), ctypes.byref(need)), "lup_workspace")
    ws = _workspace(torch, need.value, dev)
    o = _opts(validate=validate)
    fn = lib.linac_lup_u64 if wide else lib.linac_lup
    _check(fn(_ptr(At), m, n, max(n, 1), int(p), _ptr(perm), _ptr(rank), _ptr(piv), _ptr(ws),
              ws.numel(), ctypes.byref(o), _stream(torch, stream)), "linac_lup")
    if was_np:
        torch.cuda.synchronize()
        r = int(rank.item())
        LU = _u64_out(At) if wide else At.cpu().numpy().astype(np.uint32)
        return LU, perm.cpu().numpy()[:m].astype(np.int64), r, piv.cpu().numpy()[:r].astype(np.int64)
    return At, perm, rank, piv
