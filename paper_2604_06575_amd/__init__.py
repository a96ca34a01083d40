"""Python binding of the polyhip C ABI (``include/polyhip.h``).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of every operation runs in the library's HIP kernels.
There is no CPU fallback: if ``libpolyhip.so`` is missing or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

__all__ = [
    "Batch", "PolyError", "PolyEval", "PolyEvalBackward", "PolyEvalDense", "Plan", "eval_dense_backward", "batch_from_numpy", "batch_to_numpy", "mul", "simplify", "jacobian",
    "eval", "grad", "hess", "eval_backward", "eval_dense", "mtimes", "mpower", "msum", "mprod", "concat", "subs",
    "affine_normal",
    "library_path", "lib",
    "POLY_FP64", "POLY_SPLIT_BF16",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpolyhip.so")
_lib = None

POLY_FP64 = 0
POLY_SPLIT_BF16 = 1

EXPORTS = [
    "poly_strerror", "poly_read_status", "poly_tune_set", "poly_tune_get",
    "poly_timing_enable", "poly_timing_read",
    "poly_simplify_workspace", "poly_simplify",
    "poly_mul_workspace", "poly_mul",
    "poly_jacobian_workspace", "poly_jacobian",
    "poly_eval_workspace", "poly_eval",
    "poly_grad_workspace", "poly_grad",
    "poly_hess_workspace", "poly_hess",
    "poly_eval_backward_workspace", "poly_eval_backward",
    "poly_eval_backward2_workspace", "poly_eval_backward2",
    "poly_eval_dense_workspace", "poly_eval_dense",
    "poly_affine_normal_workspace", "poly_affine_normal",
    "poly_affine_normal_stochastic_workspace", "poly_affine_normal_stochastic",
    "poly_mtimes_workspace", "poly_mtimes",
    "poly_concat",
    "poly_simplify_noalloc",
    "poly_plan_workspace", "poly_plan_create", "poly_plan_launch", "poly_plan_destroy",
    "poly_eval_dense_backward_workspace", "poly_eval_dense_backward",
]


class PolyError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().poly_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: status {code} ({msg})")


class PolyCSR(ctypes.Structure):
    _fields_ = [
        ("nvars", ctypes.c_int32),
        ("max_exp", ctypes.c_int32),
        ("npolys", ctypes.c_int64),
        ("capacity", ctypes.c_int64),
        ("row_ptr_host", ctypes.c_void_p),
        ("row_ptr", ctypes.c_void_p),
        ("exps", ctypes.c_void_p),
        ("coefs", ctypes.c_void_p),
    ]


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libpolyhip.so (built in-tree by ``paper_2604_06575_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"HIP library not built: {_LIB_PATH} is missing "
                           "(run `python -m paper_2604_06575_amd.build`)")
    L = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    d = ctypes.c_double
    pcsr = ctypes.POINTER(PolyCSR)
    psz = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "poly_strerror": ([i32], ctypes.c_char_p),
        "poly_read_status": ([P, P], i32),
        "poly_tune_set": ([ctypes.c_char_p, i64], i32),
        "poly_tune_get": ([ctypes.c_char_p, ctypes.POINTER(i64)], i32),
        "poly_timing_enable": ([i32], i32),
        "poly_timing_read": ([i32, ctypes.POINTER(d), ctypes.POINTER(i64)], i32),
        "poly_simplify_workspace": ([pcsr, psz], i32),
        "poly_simplify": ([pcsr, pcsr, d, P, ctypes.c_size_t, P], i32),
        "poly_mul_workspace": ([pcsr, pcsr, psz, ctypes.POINTER(i64)], i32),
        "poly_mul": ([pcsr, pcsr, pcsr, d, P, ctypes.c_size_t, P], i32),
        "poly_jacobian_workspace": ([pcsr, psz], i32),
        "poly_jacobian": ([pcsr, pcsr, P, ctypes.c_size_t, P], i32),
        "poly_eval_workspace": ([pcsr, i64, i32, i32, psz], i32),
        "poly_eval": ([pcsr, P, i64, P, i32, i32, P, ctypes.c_size_t, P], i32),
        "poly_grad_workspace": ([pcsr, i64, i32, i32, psz], i32),
        "poly_grad": ([pcsr, P, i64, P, i32, i32, P, ctypes.c_size_t, P], i32),
        "poly_hess_workspace": ([pcsr, i64, i32, i32, psz], i32),
        "poly_hess": ([pcsr, P, i64, P, i32, i32, P, ctypes.c_size_t, P], i32),
        "poly_eval_backward_workspace": ([pcsr, i64, i32, i32, psz], i32),
        "poly_eval_backward": ([pcsr, P, i64, P, P, P, i32, i32, P, ctypes.c_size_t, P], i32),
        "poly_eval_backward2_workspace": ([pcsr, i64, psz], i32),
        "poly_eval_backward2": ([pcsr, P, i64, P, P, P, P, P, P, P, ctypes.c_size_t, P], i32),
        "poly_eval_dense_workspace": ([i32, i64, i64, i64, i32, i32, psz], i32),
        "poly_affine_normal_workspace": ([pcsr, i64, psz], i32),
        "poly_mtimes_workspace": ([pcsr, pcsr, i64, i64, i64, psz, ctypes.POINTER(i64)], i32),
        "poly_mtimes": ([pcsr, pcsr, i64, i64, i64, pcsr, d, P, ctypes.c_size_t, P], i32),
        "poly_affine_normal": ([pcsr, P, i64, d, P, P, P, ctypes.c_size_t, P], i32),
        "poly_affine_normal_stochastic_workspace": ([pcsr, i64, psz], i32),
        "poly_affine_normal_stochastic": ([pcsr, P, i64, P, i32, i32, d, d, i32, P, P, P, P, ctypes.c_size_t, P],
                                          i32),
        "poly_concat": ([ctypes.POINTER(pcsr), i32, pcsr, P], i32),
        "poly_simplify_noalloc": ([pcsr, pcsr, d, P, P], i32),
        "poly_plan_workspace": ([pcsr, i64, psz], i32),
        "poly_plan_create": ([pcsr, d, P, i64, pcsr, pcsr, P, P, ctypes.c_size_t, P, ctypes.POINTER(P)], i32),
        "poly_plan_launch": ([P, P], i32),
        "poly_plan_destroy": ([P], i32),
        "poly_eval_dense_backward_workspace": ([i32, i64, i64, i64, i32, i32, psz], i32),
        "poly_eval_dense_backward": ([i32, i64, P, i32, i64, P, i64, P, P, P, P, i32, i32, P, ctypes.c_size_t, P],
                                     i32),
        "poly_eval_dense": ([i32, i64, P, i32, i64, P, i64, P, P, i32, i32, P, ctypes.c_size_t, P], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    _load_tuning(L)
    return L


TUNING_DIR = os.path.join(_HERE, "tuning")


def _load_tuning(L):
    """Apply the autotuner's cache (``tuning/<arch>.json`` or the file named
    by POLYHIP_TUNE_FILE) to the library's launch parameters."""
    import json
    path = os.environ.get("POLYHIP_TUNE_FILE") or os.path.join(TUNING_DIR, "gfx950.json")
    if not os.path.exists(path):
        return
    with open(path) as f:
        data = json.load(f)
    for name, value in data.get("tunables", {}).items():
        _check(L.poly_tune_set(name.encode(), int(value)), f"poly_tune_set({name})")


def tune_set(name: str, value: int):
    _check(lib().poly_tune_set(name.encode(), int(value)), f"poly_tune_set({name})")


def tune_get(name: str) -> int:
    v = ctypes.c_int64()
    _check(lib().poly_tune_get(name.encode(), ctypes.byref(v)), f"poly_tune_get({name})")
    return int(v.value)


TIMING_MUL, TIMING_DENSE, TIMING_TERMS, TIMING_AFFINE = 0, 1, 2, 3


def timing_enable(on: bool = True):
    """Start (clearing earlier records) or stop recording HIP events around
    the dominant kernel of each entry point (see poly_timing_enable)."""
    _check(lib().poly_timing_enable(1 if on else 0), "poly_timing_enable")


def timing_read(slot: int) -> tuple[float, int]:
    """(summed kernel milliseconds, launches) recorded in `slot`."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib().poly_timing_read(int(slot), ctypes.byref(ms), ctypes.byref(cnt)), "poly_timing_read")
    return float(ms.value), int(cnt.value)


def _check(code: int, where: str):
    if code != 0:
        raise PolyError(code, where)


def _check_device(name: str, t: torch.Tensor, device=None):
    """Every tensor handed to the library is read or written by HIP kernels
    through its raw pointer: it must live on a GPU (the same one as the rest
    of the call) and be contiguous, or the kernels would read a host address
    or the wrong layout."""
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor, got device {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the other operands on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return None if t is None or t.numel() == 0 else ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# --------------------------------------------------------------------- batches

@dataclass
class Batch:
    """A CSR batch of polynomials on the GPU.

    ``row_ptr`` (int64 [P+1]) lives on the device and ``row_ptr_host``
    (numpy int64 [P+1]) is its host copy; ``exps`` is uint8 [T, n] and
    ``coefs`` float64 [T], both on the device.  ``max_exp`` bounds every
    stored exponent."""
    n: int
    max_exp: int
    row_ptr: torch.Tensor
    row_ptr_host: np.ndarray
    exps: torch.Tensor
    coefs: torch.Tensor

    @property
    def npolys(self) -> int:
        return int(self.row_ptr_host.shape[0] - 1)

    @property
    def nterms(self) -> int:
        return int(self.row_ptr_host[-1])

    def csr(self) -> PolyCSR:
        # the library trusts these sizes and dereferences these pointers on the
        # device: check dtypes, sizes, device and layout first
        if (self.exps.dtype != torch.uint8 or self.coefs.dtype != torch.float64 or
                self.row_ptr.dtype != torch.int64 or self.row_ptr.numel() != self.row_ptr_host.shape[0] or
                self.coefs.dim() != 1 or self.exps.numel() < self.coefs.shape[0] * self.n):
            raise ValueError("inconsistent batch tensors (uint8 exps [cap, n], float64 coefs [cap], "
                             "int64 row_ptr [P+1])")
        _check_device("row_ptr", self.row_ptr)
        _check_device("exps", self.exps, self.row_ptr.device)
        _check_device("coefs", self.coefs, self.row_ptr.device)
        c = PolyCSR()
        c.nvars = self.n
        c.max_exp = self.max_exp
        c.npolys = self.npolys
        c.capacity = int(self.coefs.shape[0])
        self._rph = np.ascontiguousarray(self.row_ptr_host, dtype=np.int64)
        c.row_ptr_host = self._rph.ctypes.data_as(ctypes.c_void_p)
        c.row_ptr = ctypes.c_void_p(self.row_ptr.data_ptr())
        c.exps = _ptr(self.exps)
        c.coefs = _ptr(self.coefs)
        return c

    def with_coefs(self, coefs: torch.Tensor) -> "Batch":
        return Batch(self.n, self.max_exp, self.row_ptr, self.row_ptr_host, self.exps, coefs)


def batch_from_numpy(row_ptr, exps, coefs, n: int | None = None, max_exp: int | None = None,
                     device="cuda") -> Batch:
    exps = np.ascontiguousarray(np.asarray(exps, dtype=np.uint8))
    n = n if n is not None else exps.shape[1]
    exps = exps.reshape(-1, n)
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    me = int(exps.max()) if (max_exp is None and exps.size) else (max_exp or 0)
    return Batch(n, me, torch.from_numpy(rp).to(device), rp,
                 torch.from_numpy(exps).to(device),
                 torch.from_numpy(np.ascontiguousarray(np.asarray(coefs, dtype=np.float64))).to(device))


def batch_to_numpy(b: Batch):
    T = b.nterms
    return (b.row_ptr_host.copy(), b.exps[:T].cpu().numpy().reshape(-1, b.n), b.coefs[:T].cpu().numpy())


def _empty_out(n: int, P: int, cap: int, max_exp: int, device) -> Batch:
    return Batch(n, max_exp, torch.zeros(P + 1, dtype=torch.int64, device=device), np.zeros(P + 1, np.int64),
                 torch.empty((max(cap, 1), n), dtype=torch.uint8, device=device),
                 torch.empty(max(cap, 1), dtype=torch.float64, device=device))


def _finish(out: Batch, ws: torch.Tensor, where: str, trim: bool) -> Batch:
    """Read back the device row pointer (one sync) and the device status."""
    st = lib().poly_read_status(ctypes.c_void_p(ws.data_ptr()), _stream())
    _check(st, where)
    out.row_ptr_host = out.row_ptr.cpu().numpy()
    if trim:
        T = out.nterms
        out.exps = out.exps[:T]
        out.coefs = out.coefs[:T]
    return out


# ------------------------------------------------------------------ operations

def simplify_workspace(b: Batch) -> int:
    ws_bytes = ctypes.c_size_t()
    cin = b.csr()
    _check(lib().poly_simplify_workspace(ctypes.byref(cin), ctypes.byref(ws_bytes)), "poly_simplify_workspace")
    return int(ws_bytes.value)


def simplify(b: Batch, tol: float = 0.0, trim: bool = True, ws: torch.Tensor | None = None,
             out: Batch | None = None, finish: bool = True) -> Batch:
    """simplify(p, zeroprec) for every entry of the batch.  With finish=False
    nothing is read back (the call only enqueues kernels, e.g. under graph
    capture); the output row pointer stays on the device."""
    L = lib()
    cin = b.csr()
    need = simplify_workspace(b)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, b.coefs.device)
    if out is None:
        out = _empty_out(b.n, b.npolys, b.nterms, b.max_exp, b.coefs.device)
    cout = out.csr()
    _check(L.poly_simplify(ctypes.byref(cin), ctypes.byref(cout), float(tol), ctypes.c_void_p(ws.data_ptr()),
                           ws.numel(), _stream()), "poly_simplify")
    if not finish:
        return out
    return _finish(out, ws, "poly_simplify", trim)


NOALLOC_SCRATCH_BYTES = 64 << 20   # POLY_NOALLOC_SCRATCH_BYTES


def simplify_noalloc(b: Batch, out: Batch, status: torch.Tensor, tol: float = 0.0) -> Batch:
    """simplify into a caller-provided output with the library's fixed device
    scratch as workspace (poly_simplify_noalloc): nothing is allocated and
    nothing is read back.  `status` (int32 [1] on the device) receives the
    device-detected status; out.row_ptr holds the output row pointer on the
    device (out.row_ptr_host is not updated)."""
    if status.dtype != torch.int32 or status.numel() < 1:
        raise ValueError("status must be an int32 tensor of at least one element")
    _check_device("status", status, b.coefs.device)
    cin, cout = b.csr(), out.csr()
    _check(lib().poly_simplify_noalloc(ctypes.byref(cin), ctypes.byref(cout), float(tol),
                                       ctypes.c_void_p(status.data_ptr()), _stream()), "poly_simplify_noalloc")
    return out


class Plan:
    """The captured pipeline simplify -> jacobian -> gradient values of a
    polynomial matrix (poly_plan_create).  ``launch()`` replays the graph on
    the current stream; outputs: ``simplified`` and ``jac`` (row pointers on
    the device; ``finish()`` reads them back) and ``G`` [P, N, n]."""

    def __init__(self, b: Batch, X: torch.Tensor, tol: float = 0.0, stream=None):
        L = lib()
        self._b, self._X = b, X.contiguous()
        _check_points(self._X, b.n, b.coefs.device)
        dev = b.coefs.device
        N, n, P, T = self._X.shape[0], b.n, b.npolys, b.nterms
        cin = b.csr()
        self._cin = cin
        ws_bytes = ctypes.c_size_t()
        _check(L.poly_plan_workspace(ctypes.byref(cin), N, ctypes.byref(ws_bytes)), "poly_plan_workspace")
        self.ws = _workspace(ws_bytes.value, dev)
        self.simplified = _empty_out(n, P, T, b.max_exp, dev)
        self.jac = _empty_out(n, P * n, T * min(n, 8), b.max_exp, dev)
        self.G = torch.empty((P, N, n), dtype=torch.float64, device=dev)
        self._csimp, self._cjac = self.simplified.csr(), self.jac.csr()
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(L.poly_plan_create(ctypes.byref(cin), float(tol), _ptr(self._X), N, ctypes.byref(self._csimp),
                                  ctypes.byref(self._cjac), _ptr(self.G), ctypes.c_void_p(self.ws.data_ptr()),
                                  self.ws.numel(), _stream(self._stream), ctypes.byref(h)), "poly_plan_create")
        self._h = h

    def launch(self, stream=None):
        _check(lib().poly_plan_launch(self._h, _stream(stream)), "poly_plan_launch")

    def finish(self):
        """Device status and the output row pointers on the host (one sync)."""
        _check(lib().poly_read_status(ctypes.c_void_p(self.ws.data_ptr()), _stream()), "poly_plan")
        self.simplified.row_ptr_host = self.simplified.row_ptr.cpu().numpy()
        self.jac.row_ptr_host = self.jac.row_ptr.cpu().numpy()
        return self

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().poly_plan_destroy(self._h), "poly_plan_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mul_workspace(a: Batch, b: Batch) -> tuple[int, int]:
    L = lib()
    ca, cb = a.csr(), b.csr()
    ws_bytes = ctypes.c_size_t()
    raw = ctypes.c_int64()
    _check(L.poly_mul_workspace(ctypes.byref(ca), ctypes.byref(cb), ctypes.byref(ws_bytes), ctypes.byref(raw)),
           "poly_mul_workspace")
    return int(ws_bytes.value), int(raw.value)


def mul(a: Batch, b: Batch, tol: float = 0.0, trim: bool = True, ws: torch.Tensor | None = None,
        out: Batch | None = None, finish: bool = True) -> Batch:
    """Entrywise simplify(a_p .* b_p)."""
    L = lib()
    ca, cb = a.csr(), b.csr()
    ws_bytes, raw = mul_workspace(a, b)
    if ws is None or ws.numel() < ws_bytes:
        ws = _workspace(ws_bytes, a.coefs.device)
    if out is None:
        out = _empty_out(a.n, a.npolys, raw, a.max_exp + b.max_exp, a.coefs.device)
    cout = out.csr()
    _check(L.poly_mul(ctypes.byref(ca), ctypes.byref(cb), ctypes.byref(cout), float(tol),
                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()), "poly_mul")
    if not finish:
        return out
    return _finish(out, ws, "poly_mul", trim)


def mtimes_workspace(a: Batch, b: Batch, I: int, K: int, J: int) -> tuple[int, int]:
    ws_bytes = ctypes.c_size_t()
    raw = ctypes.c_int64()
    _check(lib().poly_mtimes_workspace(ctypes.byref(a.csr()), ctypes.byref(b.csr()), I, K, J,
                                       ctypes.byref(ws_bytes), ctypes.byref(raw)), "poly_mtimes_workspace")
    return int(ws_bytes.value), int(raw.value)


def mtimes(a: Batch, b: Batch, I: int, K: int, J: int, tol: float = 0.0, trim: bool = True,
           ws: torch.Tensor | None = None, out: Batch | None = None, finish: bool = True) -> Batch:
    """Matrix product of polynomial matrices: a is I x K, b is K x J, both
    with entries in row-major order; returns the I x J product."""
    L = lib()
    ws_bytes, raw = mtimes_workspace(a, b, I, K, J)
    if ws is None or ws.numel() < ws_bytes:
        ws = _workspace(ws_bytes, a.coefs.device)
    if out is None:
        out = _empty_out(a.n, I * J, raw, a.max_exp + b.max_exp, a.coefs.device)
    _check(L.poly_mtimes(ctypes.byref(a.csr()), ctypes.byref(b.csr()), I, K, J, ctypes.byref(out.csr()),
                         float(tol), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()), "poly_mtimes")
    if not finish:
        return out
    return _finish(out, ws, "poly_mtimes", trim)


def mpower(a: Batch, I: int, p: int, tol: float = 0.0) -> Batch:
    """a^p for a square I x I polynomial matrix (p >= 1): p - 1 products
    a * (a * (... a)), each one library call."""
    if p < 1:
        raise ValueError("mpower needs p >= 1")
    r = a
    for _ in range(p - 1):
        r = mtimes(a, r, I, I, I, tol)
    return r


def _selector(n: int, rows: int, cols: int, hot, device) -> Batch:
    """rows x cols matrix (row-major) of constant polynomials: 1 where
    hot(i, j), the structural zero elsewhere."""
    flags = np.array([bool(hot(i, j)) for i in range(rows) for j in range(cols)], dtype=bool)
    rp = np.zeros(rows * cols + 1, np.int64)
    np.cumsum(flags, out=rp[1:])
    k = int(rp[-1])
    return batch_from_numpy(rp, np.zeros((k, n), np.uint8), np.ones(k), n=n, max_exp=0, device=device)


def msum(a: Batch, R: int, C: int, dim: int, tol: float = 0.0) -> Batch:
    """sum(A, dim) of an R x C polynomial matrix (entries row-major): dim 1
    gives 1 x C, dim 2 gives R x 1.  Each entry is simplify of the reduced
    entries' terms concatenated in index order: the product with a vector of
    constant ones (one mtimes call; products by 1 are exact)."""
    dev = a.coefs.device
    if dim == 1:
        return mtimes(_selector(a.n, 1, R, lambda i, j: True, dev), a, 1, R, C, tol)
    if dim == 2:
        return mtimes(a, _selector(a.n, C, 1, lambda i, j: True, dev), R, C, 1, tol)
    raise ValueError("dim must be 1 or 2")


def mprod(a: Batch, R: int, C: int, dim: int, tol: float = 0.0) -> Batch:
    """prod(A, dim) of an R x C polynomial matrix: the left fold of times over
    the simplified entries along dim, ((A_1 .* A_2) .* A_3) ...  Each line
    along dim is picked out (and simplified) by a product with a 0/1
    selector, and each fold step is one batched times call.  An empty
    dimension gives the constant 1."""
    if dim not in (1, 2):
        raise ValueError("dim must be 1 or 2")
    dev = a.coefs.device
    length, count = (C, R) if dim == 2 else (R, C)
    if length == 0 or count == 0:
        return batch_from_numpy(np.arange(count + 1, dtype=np.int64), np.zeros((count, a.n), np.uint8),
                                np.ones(count), n=a.n, max_exp=0, device=dev)

    def line(k):
        if dim == 2:
            return mtimes(a, _selector(a.n, C, 1, lambda i, j: i == k, dev), R, C, 1, tol)
        return mtimes(_selector(a.n, 1, R, lambda i, j: j == k, dev), a, 1, R, C, tol)

    acc = line(0)
    for k in range(1, length):
        acc = mul(acc, line(k), tol)
    return acc


def concat(batches, max_exp: int | None = None) -> Batch:
    """The entries of several batches (same n) in order, as one batch."""
    if not batches:
        raise ValueError("concat needs at least one batch")
    n = batches[0].n
    me = max(b.max_exp for b in batches) if max_exp is None else max_exp
    P = sum(b.npolys for b in batches)
    T = sum(b.nterms for b in batches)
    dev = batches[0].coefs.device
    out = _empty_out(n, P, T, me, dev)
    csrs = [b.csr() for b in batches]
    arr = (ctypes.POINTER(PolyCSR) * len(csrs))(*[ctypes.pointer(c) for c in csrs])
    _check(lib().poly_concat(arr, len(csrs), ctypes.byref(out.csr()), _stream()), "poly_concat")
    rp = np.zeros(P + 1, np.int64)
    o = 0
    for b in batches:
        rp[o:o + b.npolys + 1] = b.row_ptr_host[:b.npolys + 1] + rp[o]
        o += b.npolys
    out.row_ptr_host = rp
    return out


def subs(p: Batch, q: Batch, tol: float = 0.0) -> Batch:
    """Substitution p(q_1, ..., q_n) (Section 3.4): p is one polynomial in n
    variables, q a batch of n polynomials in m variables.  Powers q_i^k are
    left folds of times, a term's product runs over i = 1..n (acc times the
    simplified q_i^(e_i)), and the result is simplify of the terms' products,
    each scaled by its coefficient, in term order.  Every step is a library
    call: batched times for the powers and products, one concatenation for
    the power table, products with 0/1 selectors (mtimes) to gather each
    term's factor, and a product with the coefficient row for the sum."""
    if p.npolys != 1 or q.npolys != p.n:
        raise ValueError("subs takes one polynomial in n variables and a batch of n substitutes")
    n, m = p.n, q.n
    dev = q.coefs.device
    _, E, C = batch_to_numpy(p)
    T = E.shape[0]
    kmax = int(E.max()) if E.size else 0
    qe = q.max_exp
    # Declared exponent bounds follow what the products can reach, not the sum
    # of the factors' declarations: q_i^k stays within k * max_exp(q), a
    # term's partial product over variables 1..i within (its degree) *
    # max_exp(q).  (The device still checks every exponent against them.)
    pows = [q]
    for k in range(2, kmax + 1):
        pk = mul(pows[-1], q, tol)
        pk.max_exp = min(pk.max_exp, k * qe)
        pows.append(pk)
    one = batch_from_numpy([0, 1], np.zeros((1, m), np.uint8), np.ones(1), n=m, max_exp=0, device=dev)
    table = concat([one] + pows, max_exp=min(255, max(kmax, 1) * qe))
    L = table.npolys
    slot = lambda i, k: 0 if k == 0 else 1 + (k - 1) * n + i  # noqa: E731
    acc = batch_from_numpy(np.arange(T + 1, dtype=np.int64), np.zeros((T, m), np.uint8), np.ones(T), n=m,
                           max_exp=0, device=dev)
    partial_deg = np.cumsum(E.astype(np.int64), axis=1) if T else np.zeros((0, n), np.int64)
    for i in range(n):
        pick = _selector(m, T, L, lambda t, j: j == slot(i, int(E[t, i])), dev)
        factor = mtimes(pick, table, T, L, 1, tol)
        factor.max_exp = min(factor.max_exp, int(E[:, i].max()) * qe if T else 0)
        acc = mul(acc, factor, tol)
        acc.max_exp = min(acc.max_exp, int(partial_deg[:, i].max()) * qe if T else 0)
    crow = batch_from_numpy(np.arange(T + 1, dtype=np.int64), np.zeros((T, m), np.uint8), C, n=m, max_exp=0,
                            device=dev)
    return mtimes(crow, acc, 1, T, 1, tol)


def jacobian(b: Batch, trim: bool = True) -> Batch:
    """Symbolic Jacobian: entry p*n + j = diff(b_p, x_{j+1})."""
    L = lib()
    cin = b.csr()
    ws_bytes = ctypes.c_size_t()
    _check(L.poly_jacobian_workspace(ctypes.byref(cin), ctypes.byref(ws_bytes)), "poly_jacobian_workspace")
    ws = _workspace(ws_bytes.value, b.coefs.device)
    cap = b.nterms * b.n
    out = _empty_out(b.n, b.npolys * b.n, cap, b.max_exp, b.coefs.device)
    cout = out.csr()
    _check(L.poly_jacobian(ctypes.byref(cin), ctypes.byref(cout), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                           _stream()), "poly_jacobian")
    return _finish(out, ws, "poly_jacobian", trim)


def _check_points(X: torch.Tensor, n: int, device=None):
    # the kernels index X as [N, n] float64: reject anything else before a launch
    if X.dtype != torch.float64 or X.dim() != 2 or X.shape[1] != n:
        raise ValueError(f"points must be float64 [N, {n}], got {X.dtype} {tuple(X.shape)}")
    _check_device("points", X, device)


def _eval_like(fname: str, b: Batch, X: torch.Tensor, shape, check: bool, prec: int = POLY_FP64,
               nslices: int = 5):
    L = lib()
    X = X.contiguous()
    cin = b.csr()
    _check_points(X, b.n, b.coefs.device)
    N = X.shape[0]
    ws_bytes = ctypes.c_size_t()
    _check(getattr(L, fname + "_workspace")(ctypes.byref(cin), N, int(prec), int(nslices), ctypes.byref(ws_bytes)),
           fname + "_workspace")
    ws = _workspace(ws_bytes.value, b.coefs.device)
    Y = torch.empty(shape, dtype=torch.float64, device=b.coefs.device)
    _check(getattr(L, fname)(ctypes.byref(cin), _ptr(X), N, _ptr(Y), int(prec), int(nslices),
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()), fname)
    if check:
        _check(L.poly_read_status(ctypes.c_void_p(ws.data_ptr()), _stream()), fname)
    return Y


def eval(b: Batch, X: torch.Tensor, check: bool = False, prec: int = POLY_FP64, nslices: int = 5) -> torch.Tensor:
    """Y[p, pt] = f_p(x_pt).  prec=POLY_SPLIT_BF16 needs a shared monomial set
    (every polynomial the same exponent rows in the same order)."""
    return _eval_like("poly_eval", b, X, (b.npolys, X.shape[0]), check, prec, nslices)


def grad(b: Batch, X: torch.Tensor, check: bool = False, prec: int = POLY_FP64, nslices: int = 5) -> torch.Tensor:
    """G[p, pt, j] = d f_p / d x_j at x_pt."""
    return _eval_like("poly_grad", b, X, (b.npolys, X.shape[0], b.n), check, prec, nslices)


def hess(b: Batch, X: torch.Tensor, check: bool = False, prec: int = POLY_FP64, nslices: int = 5) -> torch.Tensor:
    """H[p, pt, j, k] = d^2 f_p / dx_j dx_k at x_pt."""
    return _eval_like("poly_hess", b, X, (b.npolys, X.shape[0], b.n, b.n), check, prec, nslices)


def eval_backward(b: Batch, X: torch.Tensor, gY: torch.Tensor, want_dX: bool = True, want_dC: bool = True,
                  check: bool = False, prec: int = POLY_FP64, nslices: int = 5):
    """Reverse mode of eval: (dX [N, n], dC [T]).  prec=POLY_SPLIT_BF16 takes a
    batch that is one shared monomial set (equal exponent rows in every
    polynomial) through the dense reverse mode on ``nslices`` BF16 digits
    (check=True reads back the shared-rows check)."""
    L = lib()
    X = X.contiguous()
    gY = gY.contiguous()
    cin = b.csr()
    _check_points(X, b.n, b.coefs.device)
    N = X.shape[0]
    if gY.dtype != torch.float64 or tuple(gY.shape) != (b.npolys, N):
        raise ValueError(f"gY must be float64 [{b.npolys}, {N}], got {gY.dtype} {tuple(gY.shape)}")
    _check_device("gY", gY, b.coefs.device)
    ws_bytes = ctypes.c_size_t()
    _check(L.poly_eval_backward_workspace(ctypes.byref(cin), N, prec, nslices, ctypes.byref(ws_bytes)),
           "poly_eval_backward_workspace")
    ws = _workspace(ws_bytes.value, b.coefs.device)
    dX = torch.empty((N, b.n), dtype=torch.float64, device=b.coefs.device) if want_dX else None
    dC = torch.empty(b.nterms, dtype=torch.float64, device=b.coefs.device) if want_dC else None
    _check(L.poly_eval_backward(ctypes.byref(cin), _ptr(X), N, _ptr(gY), _ptr(dX), _ptr(dC), prec, nslices,
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()), "poly_eval_backward")
    if check:
        _check(L.poly_read_status(ctypes.c_void_p(ws.data_ptr()), _stream()), "poly_eval_backward")
    return dX, dC


def eval_backward2(b: Batch, X: torch.Tensor, gY: torch.Tensor, u: torch.Tensor | None, w: torch.Tensor | None,
                   want_gY: bool = True, want_X: bool = True, want_C: bool = True, check: bool = False):
    """Reverse mode of eval_backward for cotangents u [N, n] (of dX) and
    w [T] (of dC), either may be None: (ggY [P, N], ggX [N, n], ggC [T])."""
    L = lib()
    X = X.contiguous()
    gY = gY.contiguous()
    cin = b.csr()
    dev = b.coefs.device
    _check_points(X, b.n, dev)
    N = X.shape[0]
    if gY.dtype != torch.float64 or tuple(gY.shape) != (b.npolys, N):
        raise ValueError(f"gY must be float64 [{b.npolys}, {N}], got {gY.dtype} {tuple(gY.shape)}")
    _check_device("gY", gY, dev)
    if u is not None:
        u = u.contiguous()
        if u.dtype != torch.float64 or tuple(u.shape) != (N, b.n):
            raise ValueError(f"u must be float64 [{N}, {b.n}], got {u.dtype} {tuple(u.shape)}")
        _check_device("u", u, dev)
    if w is not None:
        w = w.contiguous()
        if w.dtype != torch.float64 or w.dim() != 1 or w.shape[0] != b.nterms:
            raise ValueError(f"w must be float64 [{b.nterms}], got {w.dtype} {tuple(w.shape)}")
        _check_device("w", w, dev)
    ws_bytes = ctypes.c_size_t()
    _check(L.poly_eval_backward2_workspace(ctypes.byref(cin), N, ctypes.byref(ws_bytes)),
           "poly_eval_backward2_workspace")
    ws = _workspace(ws_bytes.value, dev)
    ggY = torch.empty((b.npolys, N), dtype=torch.float64, device=dev) if want_gY else None
    ggX = torch.empty((N, b.n), dtype=torch.float64, device=dev) if want_X else None
    ggC = torch.empty(b.nterms, dtype=torch.float64, device=dev) if want_C else None
    _check(L.poly_eval_backward2(ctypes.byref(cin), _ptr(X), N, _ptr(gY), _ptr(u), _ptr(w), _ptr(ggY), _ptr(ggX),
                                 _ptr(ggC), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()),
           "poly_eval_backward2")
    if check:
        _check(L.poly_read_status(ctypes.c_void_p(ws.data_ptr()), _stream()), "poly_eval_backward2")
    return ggY, ggX, ggC


def affine_normal(b: Batch, X: torch.Tensor, reg: float = 1e-6, check: bool = False, ws: torch.Tensor | None = None,
                  info: bool = False):
    """Affine-normal directions of one polynomial at the rows of X:
    (D [N, n], |grad f| [N]), plus with info=True a dict of the route's work
    per point in the units of Section 5's example output: the Hessian as n
    Hessian-vector products (hv_evals) and the n - 1 tangent third-derivative
    directions (third_evals)."""
    L = lib()
    X = X.contiguous()
    cin = b.csr()
    _check_points(X, b.n, b.coefs.device)
    N = X.shape[0]
    ws_bytes = ctypes.c_size_t()
    _check(L.poly_affine_normal_workspace(ctypes.byref(cin), N, ctypes.byref(ws_bytes)),
           "poly_affine_normal_workspace")
    if ws is None or ws.numel() < ws_bytes.value:
        ws = _workspace(ws_bytes.value, b.coefs.device)
    D = torch.empty((N, b.n), dtype=torch.float64, device=b.coefs.device)
    gn = torch.empty(N, dtype=torch.float64, device=b.coefs.device)
    _check(L.poly_affine_normal(ctypes.byref(cin), _ptr(X), N, float(reg), _ptr(D), _ptr(gn),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()), "poly_affine_normal")
    if check:
        _check(L.poly_read_status(ctypes.c_void_p(ws.data_ptr()), _stream()), "poly_affine_normal")
    if info:
        return D, gn, {"method": "mf-exact", "hv_evals": b.n, "third_evals": b.n - 1}
    return D, gn


def affine_normal_stochastic(b: Batch, X: torch.Tensor, Z: torch.Tensor, reg: float = 1e-6, tol: float = 1e-4,
                             maxit: int = 40, check: bool = False, ws: torch.Tensor | None = None):
    """Affine-normal directions by the stochastic log-det route: probes Z
    [q, n] (shared by the points) or [N, q, n] (per point), conjugate-gradient
    solves with relative tolerance tol and at most maxit steps.  Returns
    (D [N, n], |grad f| [N], Hessian-vector products per point [N] int32)."""
    L = lib()
    X = X.contiguous()
    Z = Z.contiguous()
    cin = b.csr()
    _check_points(X, b.n, b.coefs.device)
    N = X.shape[0]
    if Z.dtype != torch.float64 or Z.device != b.coefs.device or Z.dim() not in (2, 3) or Z.shape[-1] != b.n:
        raise ValueError("Z must be float64 [q, n] or [N, q, n] on the batch's device")
    per_point = 1 if Z.dim() == 3 else 0
    if per_point and Z.shape[0] != N:
        raise ValueError("per-point probes need Z.shape[0] == N")
    q = int(Z.shape[-2])
    ws_bytes = ctypes.c_size_t()
    _check(L.poly_affine_normal_stochastic_workspace(ctypes.byref(cin), N, ctypes.byref(ws_bytes)),
           "poly_affine_normal_stochastic_workspace")
    if ws is None or ws.numel() < ws_bytes.value:
        ws = _workspace(ws_bytes.value, b.coefs.device)
    D = torch.empty((N, b.n), dtype=torch.float64, device=b.coefs.device)
    gn = torch.empty(N, dtype=torch.float64, device=b.coefs.device)
    hv = torch.empty(N, dtype=torch.int32, device=b.coefs.device)
    _check(L.poly_affine_normal_stochastic(ctypes.byref(cin), _ptr(X), N, _ptr(Z), q, per_point, float(reg),
                                           float(tol), int(maxit), _ptr(D), _ptr(gn), _ptr(hv),
                                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()),
           "poly_affine_normal_stochastic")
    if check:
        _check(L.poly_read_status(ctypes.c_void_p(ws.data_ptr()), _stream()), "poly_affine_normal_stochastic")
    return D, gn, hv


def affine_normal_workspace(b: Batch, N: int) -> int:
    ws_bytes = ctypes.c_size_t()
    _check(lib().poly_affine_normal_workspace(ctypes.byref(b.csr()), N, ctypes.byref(ws_bytes)),
           "poly_affine_normal_workspace")
    return int(ws_bytes.value)


def eval_dense_workspace(n: int, K: int, P: int, N: int, prec: int = POLY_FP64, nslices: int = 5) -> int:
    ws_bytes = ctypes.c_size_t()
    _check(lib().poly_eval_dense_workspace(n, K, P, N, prec, nslices, ctypes.byref(ws_bytes)),
           "poly_eval_dense_workspace")
    return int(ws_bytes.value)


def eval_dense(basis: torch.Tensor, C: torch.Tensor, X: torch.Tensor, prec: int = POLY_FP64, nslices: int = 5,
               max_exp: int | None = None, ws: torch.Tensor | None = None, Y: torch.Tensor | None = None):
    """Y = C V for P polynomials over one shared monomial set."""
    L = lib()
    basis = basis.contiguous()
    C = C.contiguous()
    X = X.contiguous()
    K, n = basis.shape
    P = C.shape[0]
    N = X.shape[0]
    if basis.dtype != torch.uint8:
        raise ValueError("basis must be uint8 [K, n]")
    if C.dim() != 2 or C.shape[1] != K or C.dtype != torch.float64:
        raise ValueError(f"C must be float64 [P, {K}]")
    _check_device("C", C)
    _check_device("basis", basis, C.device)
    _check_points(X, n, C.device)
    need = eval_dense_workspace(n, K, P, N, prec, nslices)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, C.device)
    if Y is None:
        Y = torch.empty((P, N), dtype=torch.float64, device=C.device)
    elif Y.dtype != torch.float64 or not Y.is_contiguous() or tuple(Y.shape) != (P, N):
        raise ValueError(f"Y must be contiguous float64 [{P}, {N}]")
    _check_device("Y", Y, C.device)
    me = int(max_exp) if max_exp is not None else 255
    _check(L.poly_eval_dense(n, K, _ptr(basis), me, P, _ptr(C), N, _ptr(X), _ptr(Y), prec, nslices,
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()), "poly_eval_dense")
    return Y


def eval_dense_backward(basis: torch.Tensor, C: torch.Tensor, X: torch.Tensor, gY: torch.Tensor,
                        want_dC: bool = True, want_dX: bool = True, max_exp: int | None = None,
                        prec: int = POLY_FP64, nslices: int = 5):
    """Reverse mode of eval_dense: (dC [P, K], dX [N, n]) on FP64 MFMA or, with
    prec=POLY_SPLIT_BF16, on ``nslices`` BF16 digits per operand (the forward
    split scheme: dC contracts over points, W = C^T gY for dX over the
    polynomials)."""
    L = lib()
    basis, C, X, gY = basis.contiguous(), C.contiguous(), X.contiguous(), gY.contiguous()
    K, n = basis.shape
    P, N = C.shape[0], X.shape[0]
    if basis.dtype != torch.uint8 or C.dtype != torch.float64 or C.dim() != 2 or C.shape[1] != K:
        raise ValueError(f"basis must be uint8 [K, n] and C float64 [P, {K}]")
    _check_device("C", C)
    _check_device("basis", basis, C.device)
    _check_points(X, n, C.device)
    if gY.dtype != torch.float64 or tuple(gY.shape) != (P, N):
        raise ValueError(f"gY must be float64 [{P}, {N}]")
    _check_device("gY", gY, C.device)
    ws_bytes = ctypes.c_size_t()
    _check(L.poly_eval_dense_backward_workspace(n, K, P, N, prec, nslices, ctypes.byref(ws_bytes)),
           "poly_eval_dense_backward_workspace")
    ws = _workspace(ws_bytes.value, C.device)
    dC = torch.empty((P, K), dtype=torch.float64, device=C.device) if want_dC else None
    dX = torch.empty((N, n), dtype=torch.float64, device=C.device) if want_dX else None
    me = int(max_exp) if max_exp is not None else 255
    _check(L.poly_eval_dense_backward(n, K, _ptr(basis), me, P, _ptr(C), N, _ptr(X), _ptr(gY), _ptr(dC), _ptr(dX),
                                      prec, nslices, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()),
           "poly_eval_dense_backward")
    return dC, dX


# -------------------------------------------------------------------- autograd


class PolyEvalDense(torch.autograd.Function):
    """Y = C V for P polynomials over one shared monomial set, differentiable
    in (C, X): the forward is eval_dense (FP64 or split BF16), the backward
    eval_dense_backward at the same precision and digit count."""

    @staticmethod
    def forward(ctx, C, X, basis, prec: int = POLY_FP64, nslices: int = 5):
        ctx.save_for_backward(C, X, basis)
        ctx.prec, ctx.nslices = prec, nslices
        return eval_dense(basis, C.detach(), X.detach(), prec=prec, nslices=nslices)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gY):
        C, X, basis = ctx.saved_tensors
        dC, dX = eval_dense_backward(basis, C.detach(), X.detach(), gY.detach(),
                                     want_dC=ctx.needs_input_grad[0], want_dX=ctx.needs_input_grad[1],
                                     prec=ctx.prec, nslices=ctx.nslices)
        return dC, dX, None, None, None

class PolyEval(torch.autograd.Function):
    """Y = eval(f, X) as a differentiable function of (coefs, X).

    The backward pass is the library's reverse-mode kernel
    (``poly_eval_backward``, dC from the monomial values, dX from the
    derivatives streamed term by term), itself differentiable through
    :class:`PolyEvalBackward`, so double backward (Hessian-vector products,
    Hessians) runs in the library's second-order kernel."""

    @staticmethod
    def forward(ctx, coefs, X, structure: Batch):
        b = structure.with_coefs(coefs.detach().contiguous())
        ctx.structure = structure
        ctx.save_for_backward(coefs, X)
        return eval(b, X.detach())

    @staticmethod
    def backward(ctx, gY):
        coefs, X = ctx.saved_tensors
        dC, dX = PolyEvalBackward.apply(coefs, X, gY, ctx.structure, ctx.needs_input_grad[0],
                                        ctx.needs_input_grad[1])
        return dC, dX, None


class PolyEvalBackward(torch.autograd.Function):
    """(dC, dX) = reverse mode of eval at cotangent gY, differentiable in
    (coefs, X, gY): its backward is ``poly_eval_backward2``."""

    @staticmethod
    def forward(ctx, coefs, X, gY, structure: Batch, want_dC: bool = True, want_dX: bool = True):
        b = structure.with_coefs(coefs.detach().contiguous())
        ctx.structure = structure
        ctx.save_for_backward(coefs, X, gY)
        dX, dC = eval_backward(b, X.detach(), gY.detach().contiguous(), want_dX=want_dX, want_dC=want_dC)
        return dC, dX

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g_dC, g_dX):
        coefs, X, gY = ctx.saved_tensors
        b = ctx.structure.with_coefs(coefs.detach().contiguous())
        u = None if g_dX is None else g_dX.detach()
        w = None if g_dC is None else g_dC.detach()
        need_c, need_x, need_g = ctx.needs_input_grad[0], ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        if u is None and w is None:
            return None, None, None, None, None, None
        ggY, ggX, ggC = eval_backward2(b, X.detach(), gY.detach(), u, w, want_gY=need_g, want_X=need_x,
                                       want_C=need_c and u is not None)
        if need_c and u is None:
            ggC = torch.zeros_like(coefs)
        return ggC, ggX, ggY, None, None, None
