"""Python binding of libsp2.so, the gfx950 SP2 density-matrix purification
library (C ABI in include/sp2.h).

The binding only marshals arguments: every step of the purification runs in
the library's HIP kernels. PyTorch supplies device memory and the HIP stream.
There is no CPU fallback: if libsp2.so is missing or no GPU is visible the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsp2.so")
# Square-kernel choices per size, written by autotune.py on an MI355X.
TABLE_PATH = os.path.join(HERE, "kernel_table_mi355x.json")

# sp2_status
OK, INVALID_ARG, OUT_OF_MEMORY, HIP_ERROR, NOT_CONVERGED, DIVERGED, BAD_STATE = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "HIP_ERROR",
                4: "NOT_CONVERGED", 5: "DIVERGED", 6: "BAD_STATE"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
BRANCHES = {"nearest": 0, "literal": 1}
NORMS = {"fro": 0, "mixed": 1, "spectral": 2}
LAUNCHES = {"auto": 0, "sequence": 1, "persistent": 2}
MIXED_BLOCK = 32
MAX_ITER_LIMIT = 200

# Exported entry points and their ctypes signatures (mirrors include/sp2.h).
_c = ctypes
SIGNATURES = {
    "sp2_default_options": (None, [_c.c_void_p]),
    "sp2_create": (_c.c_int, [_c.POINTER(_c.c_void_p), _c.c_int, _c.c_void_p]),
    "sp2_destroy": (_c.c_int, [_c.c_void_p]),
    "sp2_init_dense": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int64,
                                  _c.c_double, _c.c_double, _c.c_int64, _c.c_void_p]),
    "sp2_run": (_c.c_int, [_c.c_void_p]),
    "sp2_get_density": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int32]),
    "sp2_get_info": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_int32),
                                _c.POINTER(_c.c_int32), _c.POINTER(_c.c_double)]),
    "sp2_get_history": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.POINTER(_c.c_int32),
                                   _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                   _c.c_void_p, _c.c_void_p]),
    "sp2_get_kernel_times": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.POINTER(_c.c_int32),
                                        _c.c_void_p]),
    "sp2_get_mixed_history": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32,
                                         _c.POINTER(_c.c_int32), _c.c_void_p]),
    "sp2_get_norm_times": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.POINTER(_c.c_int32),
                                      _c.c_void_p]),
    "sp2_get_norm_history": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32,
                                        _c.POINTER(_c.c_int32), _c.c_void_p,
                                        _c.c_void_p]),
    "sp2_init_bsr": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int32, _c.c_int64,
                                _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_double,
                                _c.c_double, _c.c_int64, _c.c_void_p]),
    "sp2_get_bsr_nnzb": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_int64)]),
    "sp2_get_bsr": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                               _c.c_int32]),
    "sp2_get_bsr_stats": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.POINTER(_c.c_int32),
                                     _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "sp2_batch_init": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                  _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                  _c.c_void_p]),
    "sp2_batch_run": (_c.c_int, [_c.c_void_p]),
    "sp2_batch_get": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_int64,
                                 _c.c_int32, _c.POINTER(_c.c_int32),
                                 _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    "sp2_batch_get_history": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32,
                                         _c.POINTER(_c.c_int32), _c.c_void_p,
                                         _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                         _c.c_void_p]),
    "sp2_get_config": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.POINTER(_c.c_int32)]),
    "sp2_acc_schedule": (_c.c_int, [_c.c_double] * 6 + [_c.c_int32, _c.c_int32,
                                                      _c.POINTER(_c.c_int32),
                                                      _c.POINTER(_c.c_int32),
                                                      _c.c_void_p, _c.c_void_p]),
    "sp2_set_homo_lumo": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                     _c.c_void_p, _c.c_void_p, _c.c_int32]),
    "sp2_set_mcweeny": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p]),
    "sp2_batch_get_run_time": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_double),
                                          _c.POINTER(_c.c_int32)]),
    "sp2_set_kernel_table": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p,
                                        _c.c_void_p]),
    "sp2_kernel_config_count": (_c.c_int32, []),
    "sp2_kernel_config_info": (_c.c_int, [_c.c_int32] + [_c.POINTER(_c.c_int32)] * 5),
    "sp2_kernel_config_name": (_c.c_char_p, [_c.c_int32]),
    "sp2_run_dense_noalloc": (_c.c_int, [_c.c_int, _c.c_void_p, _c.c_void_p, _c.c_int64,
                                         _c.c_int64, _c.c_double, _c.c_double,
                                         _c.c_int64, _c.c_void_p, _c.c_void_p,
                                         _c.c_int64, _c.c_int32, _c.c_int32,
                                         _c.c_void_p, _c.POINTER(_c.c_int32),
                                         _c.POINTER(_c.c_int32)]),
    "sp2_status_string": (_c.c_char_p, [_c.c_int]),
    "sp2_last_error": (_c.c_char_p, [_c.c_void_p]),
}


class Options(ctypes.Structure):
    """sp2_options."""
    _fields_ = [("precision", ctypes.c_int32), ("branch", ctypes.c_int32),
                ("trunc_tau", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("kernel_config", ctypes.c_int32), ("tail_split", ctypes.c_int32),
                ("kernel_timing", ctypes.c_int32), ("norm", ctypes.c_int32),
                ("launch", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libsp2.so and declares every signature; raises if it is absent.

    torch is imported first: its bundled HIP runtime then answers
    libsp2.so's dependency on libamdhip64.so.7 (same SONAME), so the library
    and torch share one HIP runtime, and with it device pointers and
    streams. Loading libsp2.so first would map the system runtime and torch
    would later map a second one."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (see above)
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SP2Error(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}"
                         + (f" ({detail})" if detail else ""))


@dataclass
class Result:
    """Outcome of one run."""
    D: object                 # torch.Tensor (n, n) on the device
    status: int
    n: int                    # index of the returned iterate X~_n
    n_squares: int
    run_ms: float
    v: list = field(default_factory=list)
    t1: list = field(default_factory=list)
    t2: list = field(default_factory=list)
    p: list = field(default_factory=list)
    r: list = field(default_factory=list)
    m: list = field(default_factory=list)    # history of the mixed or spectral norm

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Context:
    """An sp2_ctx bound to one device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the SP2 library has no CPU path")
        self._lib = load_library()
        self.device = device
        with torch.cuda.device(device):
            self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = self._lib.sp2_create(ctypes.byref(h), device,
                                  ctypes.c_void_p(_stream_handle(self._stream)))
        if st != OK:
            raise SP2Error(st, "sp2_create")
        self._h = h
        self._n = 0
        self._prec = "fp64"
        if os.path.exists(TABLE_PATH):
            self.load_kernel_table(TABLE_PATH)

    def set_kernel_table(self, entries):
        """entries: list of (precision name, n_max, 1-based config id); the
        first entry matching an instance's precision with n <= n_max picks
        its square-kernel configuration."""
        cnt = len(entries)
        prec = (ctypes.c_int32 * max(1, cnt))(*[PRECISIONS[e[0]] for e in entries])
        nmax = (ctypes.c_int64 * max(1, cnt))(*[int(e[1]) for e in entries])
        cid = (ctypes.c_int32 * max(1, cnt))(*[int(e[2]) for e in entries])
        self._check(self._lib.sp2_set_kernel_table(self._h, cnt, prec, nmax, cid),
                    "sp2_set_kernel_table")

    def load_kernel_table(self, path: str | None = None):
        """Installs the autotuned table (JSON written by autotune.py)."""
        import json
        path = path or TABLE_PATH
        with open(path) as fh:
            data = json.load(fh)
        ids = {c["name"]: c["id"] for c in kernel_configs()}
        entries = []
        for e in data["entries"]:
            if e["name"] in ids:
                entries.append((e["precision"], e["n_max"], ids[e["name"]]))
        self.set_kernel_table(entries)
        return entries

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sp2_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _err(self) -> str:
        s = self._lib.sp2_last_error(self._h)
        return s.decode() if s else ""

    def _check(self, st: int, where: str, ok=(OK,)):
        if st not in ok:
            raise SP2Error(st, where, self._err())
        return st

    # -- C ABI wrappers (same names as the library, minus the prefix) -----
    def init_dense(self, F, lambda_min: float, lambda_max: float, n_occ: int,
                   precision: str = "fp64", branch: str = "nearest",
                   trunc_tau: float = 0.0, max_iter: int = 100,
                   kernel_config: int = 0, tail_split: int = 0,
                   kernel_timing: bool = False, norm: str = "fro",
                   launch: str = "auto"):
        import torch
        if not (isinstance(F, torch.Tensor) and F.is_cuda and F.dtype == torch.float64):
            raise TypeError("F must be a float64 CUDA tensor")
        if F.dim() != 2 or F.shape[0] != F.shape[1] or F.stride(1) != 1:
            raise ValueError("F must be square with unit column stride")
        opt = Options(PRECISIONS[precision], BRANCHES[branch], float(trunc_tau),
                      int(max_iter), int(kernel_config), int(tail_split),
                      1 if kernel_timing else 0, NORMS[norm], LAUNCHES[launch])
        self._F = F   # keep alive until run() returns
        st = self._lib.sp2_init_dense(self._h, ctypes.c_void_p(F.data_ptr()),
                                      F.shape[0], F.stride(0), float(lambda_min),
                                      float(lambda_max), int(n_occ),
                                      ctypes.byref(opt))
        self._check(st, "sp2_init_dense")
        self._n = F.shape[0]
        self._prec = precision

    def run(self) -> int:
        st = self._lib.sp2_run(self._h)
        return self._check(st, "sp2_run", ok=(OK, NOT_CONVERGED, DIVERGED))

    def get_density(self, out=None, as_fp64: bool = True):
        import torch
        n = self._n
        if out is None:
            dt = torch.float64 if (as_fp64 or self._prec == "fp64") else torch.float32
            out = torch.empty((n, n), dtype=dt, device=f"cuda:{self.device}")
        st = self._lib.sp2_get_density(self._h, ctypes.c_void_p(out.data_ptr()),
                                       out.stride(0), 1 if as_fp64 else 0)
        self._check(st, "sp2_get_density")
        return out

    def get_info(self):
        n = ctypes.c_int32()
        sq = ctypes.c_int32()
        ms = ctypes.c_double()
        self._check(self._lib.sp2_get_info(self._h, ctypes.byref(n), ctypes.byref(sq),
                                           ctypes.byref(ms)), "sp2_get_info")
        return n.value, sq.value, ms.value

    def set_homo_lumo(self, homo_out, homo_in, lumo_in, lumo_out,
                      accelerate: bool = True):
        """Switches the instances of the last init to SP2-ACC (Alg. 3/4):
        scalars for a dense or block-sparse context, sequences (one entry per
        instance) for a batch."""
        vals = [homo_out, homo_in, lumo_in, lumo_out]
        if all(isinstance(v, (int, float)) for v in vals):
            vals = [[v] for v in vals]
        cnt = len(vals[0])
        if any(len(v) != cnt for v in vals):
            raise ValueError("bound sequences differ in length")
        arrs = [_arr(ctypes.c_double, [float(x) for x in v]) for v in vals]
        self._check(self._lib.sp2_set_homo_lumo(self._h, cnt, *arrs,
                                                1 if accelerate else 0),
                    "sp2_set_homo_lumo")

    def set_mcweeny(self, mu, xi=None):
        """Switches the instances of the last init to McWeeny (xi None) or
        McW-ACC with gap estimate xi (sec. 3): scalars for a dense context,
        sequences (one entry per instance) for a batch."""
        if isinstance(mu, (int, float)):
            mu = [mu]
            xi = None if xi is None else [xi]
        mus = _arr(ctypes.c_double, [float(x) for x in mu])
        xis = None if xi is None else _arr(ctypes.c_double, [float(x) for x in xi])
        if xi is not None and len(xi) != len(mu):
            raise ValueError("mu and xi differ in length")
        self._check(self._lib.sp2_set_mcweeny(self._h, len(mu), mus, xis),
                    "sp2_set_mcweeny")

    def get_mixed_history(self, index: int = 0):
        """m[k] = mixed norm of X~_k - X~_k^2 of the last run (norm="mixed")."""
        import numpy as np
        ln = ctypes.c_int32()
        m = np.full(MAX_ITER_LIMIT + 1, np.nan)
        self._check(self._lib.sp2_get_mixed_history(self._h, index, m.size,
                                                    ctypes.byref(ln),
                                                    ctypes.c_void_p(m.ctypes.data)),
                    "sp2_get_mixed_history")
        return m[:ln.value].tolist()

    def get_norm_history(self, index: int = 0, krylov: bool = False):
        """e[k] = ||X~_k - X~_k^2|| in the norm the stop read (norm="mixed"
        or "spectral") of the last run; with krylov=True also the Lanczos
        steps behind each e[k]."""
        import numpy as np
        ln = ctypes.c_int32()
        e = np.full(MAX_ITER_LIMIT + 1, np.nan)
        ks = np.zeros(MAX_ITER_LIMIT + 1, dtype=np.int32)
        self._check(self._lib.sp2_get_norm_history(self._h, index, e.size,
                                                   ctypes.byref(ln),
                                                   ctypes.c_void_p(e.ctypes.data),
                                                   ctypes.c_void_p(ks.ctypes.data)),
                    "sp2_get_norm_history")
        if krylov:
            return e[:ln.value].tolist(), ks[:ln.value].astype(int).tolist()
        return e[:ln.value].tolist()

    def get_config(self, index: int = 0):
        """(id, name) of the square-kernel configuration instance `index`
        uses; (0, None) where no square is computed."""
        cid = ctypes.c_int32()
        self._check(self._lib.sp2_get_config(self._h, index, ctypes.byref(cid)),
                    "sp2_get_config")
        if cid.value == 0:
            return 0, None
        return cid.value, self._lib.sp2_kernel_config_name(cid.value).decode()

    def get_kernel_times(self):
        """Square-kernel durations (ms) of the last run with kernel_timing."""
        import numpy as np
        ln = ctypes.c_int32()
        buf = np.zeros(MAX_ITER_LIMIT + 1, dtype=np.float32)
        self._check(self._lib.sp2_get_kernel_times(self._h, buf.size, ctypes.byref(ln),
                                                   ctypes.c_void_p(buf.ctypes.data)),
                    "sp2_get_kernel_times")
        return buf[:ln.value].astype(float).tolist()

    def get_norm_times(self):
        """Spectral-norm launch durations (ms) of the last run with
        kernel_timing and norm="spectral"."""
        import numpy as np
        ln = ctypes.c_int32()
        buf = np.zeros(MAX_ITER_LIMIT + 1, dtype=np.float32)
        self._check(self._lib.sp2_get_norm_times(self._h, buf.size, ctypes.byref(ln),
                                                 ctypes.c_void_p(buf.ctypes.data)),
                    "sp2_get_norm_times")
        return buf[:ln.value].astype(float).tolist()

    def get_history(self, cap: int = MAX_ITER_LIMIT + 2):
        import numpy as np
        ln = ctypes.c_int32()
        v = np.full(cap, np.nan)
        t1 = np.full(cap, np.nan)
        t2 = np.full(cap, np.nan)
        r = np.full(cap, np.nan)
        p = np.full(cap, -1, dtype=np.int8)
        ptr = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
        self._check(self._lib.sp2_get_history(self._h, cap, ctypes.byref(ln), ptr(v),
                                              ptr(t1), ptr(t2), ptr(p), ptr(r)),
                    "sp2_get_history")
        m = ln.value
        return dict(v=v[:m].tolist(), r=r[:m].tolist(), t1=t1[:m + 1].tolist(),
                    t2=t2[:m + 1].tolist(), p=p[:m + 1].astype(int).tolist())


class BsrContext(Context):
    """A context running the block-sparse (32 x 32 blocks, FP32) path."""

    def init_bsr(self, n: int, row_ptr, col_idx, blocks, lambda_min: float,
                 lambda_max: float, n_occ: int, trunc_tau: float = 0.0,
                 branch: str = "nearest", max_iter: int = 100,
                 kernel_timing: bool = False, norm: str = "fro"):
        """row_ptr/col_idx: int32 CUDA tensors; blocks: float64 CUDA tensor of
        shape (nnzb, 32, 32)."""
        import torch
        if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32:
            raise TypeError("row_ptr and col_idx must be int32")
        if blocks.dtype != torch.float64 or not blocks.is_contiguous():
            raise TypeError("blocks must be a contiguous float64 tensor")
        if not (row_ptr.is_cuda and col_idx.is_cuda and blocks.is_cuda):
            raise TypeError("arrays must be CUDA tensors")
        opt = Options(PRECISIONS["fp32"], BRANCHES[branch], float(trunc_tau),
                      int(max_iter), 0, 0, 1 if kernel_timing else 0, NORMS[norm], 0)
        self._keep = (row_ptr, col_idx, blocks)
        st = self._lib.sp2_init_bsr(self._h, int(n), 32, int(col_idx.numel()),
                                    ctypes.c_void_p(row_ptr.data_ptr()),
                                    ctypes.c_void_p(col_idx.data_ptr()),
                                    ctypes.c_void_p(blocks.data_ptr()),
                                    float(lambda_min), float(lambda_max), int(n_occ),
                                    ctypes.byref(opt))
        self._check(st, "sp2_init_bsr")
        self._n = int(n)
        self._prec = "fp32"

    def get_bsr(self, as_fp64: bool = True):
        """(row_ptr, col_idx, blocks) of the returned iterate's nonzero blocks."""
        import torch
        nnzb = ctypes.c_int64()
        self._check(self._lib.sp2_get_bsr_nnzb(self._h, ctypes.byref(nnzb)),
                    "sp2_get_bsr_nnzb")
        nb = (self._n + 31) // 32
        dev = f"cuda:{self.device}"
        rp = torch.empty(nb + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(max(1, nnzb.value), dtype=torch.int32, device=dev)
        bl = torch.empty((max(1, nnzb.value), 32, 32),
                         dtype=torch.float64 if as_fp64 else torch.float32, device=dev)
        self._check(self._lib.sp2_get_bsr(self._h, ctypes.c_void_p(rp.data_ptr()),
                                          ctypes.c_void_p(ci.data_ptr()),
                                          ctypes.c_void_p(bl.data_ptr()),
                                          1 if as_fp64 else 0), "sp2_get_bsr")
        return rp, ci[:nnzb.value], bl[:nnzb.value]

    def get_bsr_stats(self):
        """Per step: stored blocks, nonzero input blocks, block products."""
        import numpy as np
        cap = MAX_ITER_LIMIT + 1
        ln = ctypes.c_int32()
        a, b, c = (np.zeros(cap, dtype=np.int64) for _ in range(3))
        ptr = lambda x: ctypes.c_void_p(x.ctypes.data)  # noqa: E731
        self._check(self._lib.sp2_get_bsr_stats(self._h, cap, ctypes.byref(ln), ptr(a),
                                                ptr(b), ptr(c)), "sp2_get_bsr_stats")
        m = ln.value
        return dict(stored=a[:m].tolist(), nonzero=b[:m].tolist(), products=c[:m].tolist())


def _arr(ctype, vals):
    return (ctype * len(vals))(*vals)


class BatchContext(Context):
    """A context running many independent instances per launch sequence."""

    def batch_init(self, Fs, lambda_min, lambda_max, n_occ, precision: str = "fp64",
                   branch: str = "nearest", trunc_tau: float = 0.0,
                   max_iter: int = 100, kernel_config: int = 0, tail_split: int = 0,
                   kernel_timing: bool = False, norm: str = "fro", launch: str = "auto"):
        import torch
        for F in Fs:
            if not (isinstance(F, torch.Tensor) and F.is_cuda and F.dtype == torch.float64):
                raise TypeError("every F must be a float64 CUDA tensor")
            if F.dim() != 2 or F.shape[0] != F.shape[1] or F.stride(1) != 1:
                raise ValueError("every F must be square with unit column stride")
        cnt = len(Fs)
        opt = Options(PRECISIONS[precision], BRANCHES[branch], float(trunc_tau),
                      int(max_iter), int(kernel_config), int(tail_split),
                      1 if kernel_timing else 0, NORMS[norm], LAUNCHES[launch])
        self._Fs = list(Fs)   # keep alive until batch_run() returns
        ptrs = _arr(ctypes.c_void_p, [F.data_ptr() for F in Fs])
        ns = _arr(ctypes.c_int64, [F.shape[0] for F in Fs])
        lds = _arr(ctypes.c_int64, [F.stride(0) for F in Fs])
        lo = _arr(ctypes.c_double, [float(x) for x in lambda_min])
        hi = _arr(ctypes.c_double, [float(x) for x in lambda_max])
        no = _arr(ctypes.c_int64, [int(x) for x in n_occ])
        st = self._lib.sp2_batch_init(self._h, cnt, ptrs, ns, lds, lo, hi, no,
                                      ctypes.byref(opt))
        self._check(st, "sp2_batch_init")
        self._ns = [F.shape[0] for F in Fs]
        self._prec = precision

    def batch_run(self) -> int:
        return self._check(self._lib.sp2_batch_run(self._h), "sp2_batch_run")

    def batch_get(self, idx: int, as_fp64: bool = True, with_density: bool = True):
        import torch
        n = self._ns[idx]
        out = None
        if with_density:
            dt = torch.float64 if (as_fp64 or self._prec == "fp64") else torch.float32
            out = torch.empty((n, n), dtype=dt, device=f"cuda:{self.device}")
        it, sq, stt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.sp2_batch_get(
            self._h, idx, ctypes.c_void_p(out.data_ptr() if out is not None else 0),
            n, 1 if as_fp64 else 0, ctypes.byref(it), ctypes.byref(sq),
            ctypes.byref(stt)), "sp2_batch_get")
        return out, stt.value, it.value, sq.value

    def batch_history(self, idx: int, cap: int = MAX_ITER_LIMIT + 2):
        import numpy as np
        ln = ctypes.c_int32()
        v, t1, t2, r = (np.full(cap, np.nan) for _ in range(4))
        p = np.full(cap, -1, dtype=np.int8)
        ptr = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
        self._check(self._lib.sp2_batch_get_history(
            self._h, idx, cap, ctypes.byref(ln), ptr(v), ptr(t1), ptr(t2), ptr(p),
            ptr(r)), "sp2_batch_get_history")
        m = ln.value
        return dict(v=v[:m].tolist(), r=r[:m].tolist(), t1=t1[:m + 1].tolist(),
                    t2=t2[:m + 1].tolist(), p=p[:m + 1].astype(int).tolist())

    def batch_run_time(self):
        ms, steps = ctypes.c_double(), ctypes.c_int32()
        self._check(self._lib.sp2_batch_get_run_time(self._h, ctypes.byref(ms),
                                                     ctypes.byref(steps)),
                    "sp2_batch_get_run_time")
        return ms.value, steps.value


def run_batch(Fs, lambda_min, lambda_max, n_occ, ctx: BatchContext | None = None,
              as_fp64: bool = True, homo_lumo=None, accelerate: bool = True,
              mcweeny=None, **opts):
    """SP2 on many independent matrices at once; returns (results, run_ms).
    homo_lumo = four sequences (homo_out, homo_in, lumo_in, lumo_out) with one
    entry per matrix selects SP2-ACC (Alg. 3/4)."""
    own = ctx is None
    if own:
        ctx = BatchContext(Fs[0].device.index or 0)
    try:
        ctx.batch_init(Fs, lambda_min, lambda_max, n_occ, **opts)
        if homo_lumo is not None:
            ctx.set_homo_lumo(*homo_lumo, accelerate=accelerate)
        if mcweeny is not None:
            ctx.set_mcweeny(*mcweeny)
        ctx.batch_run()
        ms, _ = ctx.batch_run_time()
        out = []
        for b in range(len(Fs)):
            D, st, n, sq = ctx.batch_get(b, as_fp64=as_fp64)
            m = ctx.get_norm_history(b) if opts.get("norm", "fro") != "fro" else []
            out.append(Result(D=D, status=st, n=n, n_squares=sq, run_ms=ms, m=m,
                              **ctx.batch_history(b)))
        return out, ms
    finally:
        if own:
            ctx.close()


def run_dense(F, lambda_min: float, lambda_max: float, n_occ: int,
              precision: str = "fp64", branch: str = "nearest",
              trunc_tau: float = 0.0, max_iter: int = 100,
              kernel_config: int = 0, tail_split: int = 0,
              as_fp64: bool = True, ctx: Context | None = None,
              homo_lumo=None, accelerate: bool = True, norm: str = "fro",
              mcweeny=None, launch: str = "auto") -> Result:
    """SP2 (Alg. 2) on the GPU from F to the converged density matrix; with
    homo_lumo = (homo_out, homo_in, lumo_in, lumo_out), SP2-ACC (Alg. 3/4);
    with mcweeny = (mu, xi or None), McWeeny / McW-ACC (sec. 3)."""
    own = ctx is None
    if own:
        ctx = Context(F.device.index or 0)
    try:
        ctx.init_dense(F, lambda_min, lambda_max, n_occ, precision, branch,
                       trunc_tau, max_iter, kernel_config, tail_split, norm=norm,
                       launch=launch)
        if homo_lumo is not None:
            ctx.set_homo_lumo(*homo_lumo, accelerate=accelerate)
        if mcweeny is not None:
            ctx.set_mcweeny(*mcweeny)
        st = ctx.run()
        D = ctx.get_density(as_fp64=as_fp64)
        n, sq, ms = ctx.get_info()
        h = ctx.get_history()
        m = ctx.get_norm_history() if norm != "fro" else []
        return Result(D=D, status=st, n=n, n_squares=sq, run_ms=ms, m=m, **h)
    finally:
        if own:
            ctx.close()


def status_string(st: int) -> str:
    return load_library().sp2_status_string(st).decode()


def acc_schedule(lambda_min, lambda_max, homo_out, homo_in, lumo_in, lumo_out,
                 accelerate: bool = True):
    """The library's Alg. 3 schedule (host computation, no device): dict with
    n_min, n_max and the lists p, alpha of steps 1..n_max."""
    lib = load_library()
    cap = MAX_ITER_LIMIT
    p = (ctypes.c_int8 * cap)()
    a = (ctypes.c_double * cap)()
    lo, hi = ctypes.c_int32(), ctypes.c_int32()
    st = lib.sp2_acc_schedule(float(lambda_min), float(lambda_max), float(homo_out),
                              float(homo_in), float(lumo_in), float(lumo_out),
                              1 if accelerate else 0, cap, ctypes.byref(lo),
                              ctypes.byref(hi), ctypes.cast(p, ctypes.c_void_p),
                              ctypes.cast(a, ctypes.c_void_p))
    if st != OK:
        raise SP2Error(st, "sp2_acc_schedule: bounds not finite, out of order or "
                           "overlapping")
    n = hi.value
    return dict(n_min=lo.value, n_max=n, p=list(p[:n]), alpha=list(a[:n]))


def kernel_configs():
    """All compiled square-kernel configurations: list of dicts with the
    1-based id, precision name, macro tile, waves and K slice."""
    lib = load_library()
    names = {v: k for k, v in PRECISIONS.items()}
    out = []
    for i in range(1, lib.sp2_kernel_config_count() + 1):
        vals = [ctypes.c_int32() for _ in range(5)]
        st = lib.sp2_kernel_config_info(i, *[ctypes.byref(v) for v in vals])
        if st != OK:
            raise SP2Error(st, "sp2_kernel_config_info")
        prec, tile, wm, wn, bk = (v.value for v in vals)
        out.append(dict(id=i, name=lib.sp2_kernel_config_name(i).decode(),
                        precision=names[prec], tile=tile, waves_m=wm,
                        waves_n=wn, k_slice=bk))
    return out
