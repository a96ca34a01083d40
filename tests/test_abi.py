"""CPU-side checks of the boundary: the shared library loads and exports
every symbol the header declares; host argument checks reject bad input
without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "polyhip.h")).read()
    return sorted(set(re.findall(r"\b(poly_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2604_06575_amd as ph
    if not os.path.exists(ph.library_path()):
        pytest.skip("library not built")
    L = ctypes.CDLL(ph.library_path())
    syms = header_symbols()
    assert len(syms) == 38
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(ph.EXPORTS) == syms


def test_only_declared_entry_points_have_c_linkage():
    """Every unmangled symbol the library defines is an entry point the
    header declares: internal helpers keep internal linkage."""
    import shutil
    import subprocess
    import paper_2604_06575_amd as ph
    if not os.path.exists(ph.library_path()) or not shutil.which("nm"):
        pytest.skip("library not built or nm missing")
    out = subprocess.run(["nm", "-D", "--defined-only", ph.library_path()], capture_output=True, text=True).stdout
    names = {line.split()[-1] for line in out.splitlines() if line.strip()}
    plain = {n for n in names if not n.startswith("_Z") and not n.startswith("__hip_cuid")}
    assert plain == set(header_symbols())


def test_strerror_and_host_argument_checks():
    import paper_2604_06575_amd as ph
    if not os.path.exists(ph.library_path()):
        pytest.skip("library not built")
    L = ph.lib()
    for code in range(0, 9):
        assert L.poly_strerror(code)
    # host checks: null / inconsistent CSR are rejected before any launch
    c = ph.PolyCSR()
    c.nvars = 0
    size = ctypes.c_size_t()
    assert L.poly_simplify_workspace(ctypes.byref(c), ctypes.byref(size)) == 1
    rp = np.array([0, 3, 2], np.int64)        # decreasing row pointer
    c.nvars = 2
    c.max_exp = 3
    c.npolys = 2
    c.capacity = 3
    c.row_ptr_host = rp.ctypes.data_as(ctypes.c_void_p)
    c.row_ptr = ctypes.c_void_p(1)
    c.exps = ctypes.c_void_p(1)
    c.coefs = ctypes.c_void_p(1)
    assert L.poly_simplify_workspace(ctypes.byref(c), ctypes.byref(size)) == 1
    rp2 = np.array([0, 2, 3], np.int64)
    c.row_ptr_host = rp2.ctypes.data_as(ctypes.c_void_p)
    assert L.poly_simplify_workspace(ctypes.byref(c), ctypes.byref(size)) == 0
    assert size.value > 0
    # key overflow: 40 variables * 3 bits > 64
    c.nvars = 40
    raw = ctypes.c_int64()
    assert L.poly_mul_workspace(ctypes.byref(c), ctypes.byref(c), ctypes.byref(size), ctypes.byref(raw)) == 0
    assert raw.value == 2 * 2 + 1 * 1
    # dense workspace sizes
    assert L.poly_eval_dense_workspace(30, 1000, 10, 10, 1, 9, ctypes.byref(size)) == 1   # nslices out of range
    assert L.poly_eval_dense_workspace(30, 1000, 10, 10, 1, 5, ctypes.byref(size)) == 0
    # dense reverse mode: split dC takes 3..5 digits and its digit planes of gY
    assert L.poly_eval_dense_backward_workspace(30, 1000, 10, 100, 1, 6, ctypes.byref(size)) == 1
    assert L.poly_eval_dense_backward_workspace(30, 1000, 10, 100, 2, 5, ctypes.byref(size)) == 1   # no such prec
    assert L.poly_eval_dense_backward_workspace(30, 1000, 10, 100, 0, 9, ctypes.byref(size)) == 0   # FP64: unused
    fp64 = size.value
    assert L.poly_eval_dense_backward_workspace(30, 1000, 10, 100, 1, 4, ctypes.byref(size)) == 0
    assert size.value >= fp64 + 2 * 4 * 32 * 128
    # affine normal: one polynomial, 2 <= n <= 255
    c.nvars = 2
    c.npolys = 2
    assert L.poly_affine_normal_workspace(ctypes.byref(c), 10, ctypes.byref(size)) == 1   # two polynomials
    one = np.array([0, 3], np.int64)
    c.npolys = 1
    c.row_ptr_host = one.ctypes.data_as(ctypes.c_void_p)
    assert L.poly_affine_normal_workspace(ctypes.byref(c), 10, ctypes.byref(size)) == 0
    assert size.value > 0
    c.nvars = 1
    assert L.poly_affine_normal_workspace(ctypes.byref(c), 10, ctypes.byref(size)) == 1   # no tangent space
    c.nvars = 255   # past the LDS-resident size the matrix works in the Hessian's workspace slot
    assert L.poly_affine_normal_workspace(ctypes.byref(c), 10, ctypes.byref(size)) == 0
    assert size.value >= 10 * 255 * 255 * 8
    # stochastic route: matrix-free, the workspace holds only the factor lists
    assert L.poly_affine_normal_stochastic_workspace(ctypes.byref(c), 10, ctypes.byref(size)) == 0
    assert 0 < size.value < 4096
    c.nvars = 1
    assert L.poly_affine_normal_stochastic_workspace(ctypes.byref(c), 10, ctypes.byref(size)) == 1
    c.nvars = 4
    X = np.zeros(40)
    Z = np.zeros(8)
    D = np.zeros(40)
    g = np.zeros(10)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    for q, per_point, tol, maxit in ((0, 0, 1e-4, 10), (2, 2, 1e-4, 10), (2, 0, -1.0, 10), (2, 0, 1e-4, -1),
                                     (1 << 20, 0, 1e-4, 1 << 12)):
        assert L.poly_affine_normal_stochastic(ctypes.byref(c), p(X), 10, p(Z), q, per_point, 1e-6, tol, maxit,
                                               p(D), p(g), None, None, 0, None) == 1


def test_noalloc_rejects_work_beyond_its_scratch():
    """The allocation-free simplify refuses, on the host and before touching a
    device, an input whose workspace exceeds its fixed scratch, and checks
    its arguments like poly_simplify."""
    import paper_2604_06575_amd as ph
    if not os.path.exists(ph.library_path()):
        pytest.skip("library not built")
    L = ph.lib()
    assert L.poly_strerror(8).decode().startswith("work exceeds the fixed scratch")
    size = ctypes.c_size_t()
    c = ph.PolyCSR()
    c.nvars = 4
    c.max_exp = 6
    c.npolys = 1
    big = np.array([0, 4_000_000], np.int64)
    c.capacity = int(big[-1])
    c.row_ptr_host = big.ctypes.data_as(ctypes.c_void_p)
    c.row_ptr = ctypes.c_void_p(1)
    c.exps = ctypes.c_void_p(1)
    c.coefs = ctypes.c_void_p(1)
    assert L.poly_simplify_workspace(ctypes.byref(c), ctypes.byref(size)) == 0
    assert size.value > ph.NOALLOC_SCRATCH_BYTES
    assert L.poly_simplify_noalloc(ctypes.byref(c), ctypes.byref(c), 0.0, None, None) == 8
    # many small entries: the per-entry path, 24 bytes per term and 16 per entry
    many = np.arange(0, 3_000_001, 3, dtype=np.int64)
    c.npolys = many.shape[0] - 1
    c.capacity = int(many[-1])
    c.row_ptr_host = many.ctypes.data_as(ctypes.c_void_p)
    assert L.poly_simplify_workspace(ctypes.byref(c), ctypes.byref(size)) == 0
    assert size.value > ph.NOALLOC_SCRATCH_BYTES
    assert L.poly_simplify_noalloc(ctypes.byref(c), ctypes.byref(c), 0.0, None, None) == 8
    c.nvars = 0   # argument errors come first, as for poly_simplify
    assert L.poly_simplify_noalloc(ctypes.byref(c), ctypes.byref(c), 0.0, None, None) == 1


def test_concat_host_checks():
    import paper_2604_06575_amd as ph
    if not os.path.exists(ph.library_path()):
        pytest.skip("library not built")
    L = ph.lib()
    rp = np.array([0, 2], np.int64)
    a = ph.PolyCSR()
    a.nvars, a.max_exp, a.npolys, a.capacity = 2, 3, 1, 2
    a.row_ptr_host = rp.ctypes.data_as(ctypes.c_void_p)
    a.row_ptr = a.exps = a.coefs = ctypes.c_void_p(1)
    out = ph.PolyCSR()
    out.nvars, out.max_exp, out.npolys, out.capacity = 2, 3, 2, 4
    out.row_ptr = out.exps = out.coefs = ctypes.c_void_p(1)
    ins = (ctypes.POINTER(ph.PolyCSR) * 2)(ctypes.pointer(a), ctypes.pointer(a))
    out.npolys = 3
    assert L.poly_concat(ins, 2, ctypes.byref(out), None) == 1     # entry count mismatch
    out.npolys, out.capacity = 2, 3
    assert L.poly_concat(ins, 2, ctypes.byref(out), None) == 4     # capacity below the 4 terms
    out.capacity, out.max_exp = 4, 2
    assert L.poly_concat(ins, 2, ctypes.byref(out), None) == 1     # max_exp below an input's
    assert L.poly_concat(ins, -1, ctypes.byref(out), None) == 1


def test_tunables_roundtrip():
    import paper_2604_06575_amd as ph
    if not os.path.exists(ph.library_path()):
        pytest.skip("library not built")
    old = ph.tune_get("mul_bucket_terms")
    ph.tune_set("mul_bucket_terms", 8192)
    assert ph.tune_get("mul_bucket_terms") == 8192
    ph.tune_set("mul_bucket_terms", old)
    old = ph.tune_get("simplify_wide_min")
    ph.tune_set("simplify_wide_min", 1)
    assert ph.tune_get("simplify_wide_min") == 1
    ph.tune_set("simplify_wide_min", old)
    with pytest.raises(ph.PolyError):
        ph.tune_set("simplify_wide_min", 0)
    with pytest.raises(ph.PolyError):
        ph.tune_set("no_such_knob", 1)
    with pytest.raises(ph.PolyError):
        ph.tune_set("seg_blocks_per_cu", 0)
    old = ph.tune_get("dense_f64_rows")
    for bad in (96, 63, 256):
        with pytest.raises(ph.PolyError):
            ph.tune_set("dense_f64_rows", bad)
    ph.tune_set("dense_f64_rows", 128)
    assert ph.tune_get("dense_f64_rows") == 128
    ph.tune_set("dense_f64_rows", old)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2604_06575_amd as ph
    monkeypatch.setattr(ph, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ph, "_lib", None)
    with pytest.raises(RuntimeError):
        ph.lib()


def test_timing_hooks_host_checks():
    """poly_timing_read rejects bad slots and null outputs without a GPU."""
    import ctypes
    import paper_2604_06575_amd as ph
    L = ph.lib()
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    assert L.poly_timing_read(4, ctypes.byref(ms), ctypes.byref(cnt)) == 1
    assert L.poly_timing_read(-1, ctypes.byref(ms), ctypes.byref(cnt)) == 1
    assert L.poly_timing_read(0, None, ctypes.byref(cnt)) == 1
    # nothing recorded yet: zero launches, no device access
    assert L.poly_timing_read(0, ctypes.byref(ms), ctypes.byref(cnt)) == 0
    assert cnt.value == 0 and ms.value == 0.0


def test_binding_rejects_bad_shapes():
    """The binding checks tensor shapes and dtypes before any launch (the
    library trusts the sizes it is given)."""
    import torch
    import paper_2604_06575_amd as ph
    if not os.path.exists(ph.library_path()):
        pytest.skip("library not built")
    b = ph.Batch(2, 2, torch.zeros(2, dtype=torch.int64), np.array([0, 1]), torch.zeros((1, 2), dtype=torch.uint8),
                 torch.zeros(1, dtype=torch.float64))
    with pytest.raises(ValueError):
        ph.eval(b, torch.zeros((3, 5), dtype=torch.float64))
    with pytest.raises(ValueError):
        ph.eval(b, torch.zeros((3, 2), dtype=torch.float32))
    bad = ph.Batch(2, 2, torch.zeros(2, dtype=torch.int64), np.array([0, 1]), torch.zeros((1, 1), dtype=torch.uint8),
                   torch.zeros(1, dtype=torch.float64))
    with pytest.raises(ValueError):
        bad.csr()
    with pytest.raises(ValueError):
        ph.mpower(b, 1, 0)
    with pytest.raises(ValueError):
        ph.subs(b, b)
    # CPU tensors and strided views are rejected before their pointers reach a kernel
    with pytest.raises(ValueError, match="GPU tensor"):
        b.csr()
    with pytest.raises(ValueError):
        ph.eval_backward(b, torch.zeros((3, 2), dtype=torch.float64), torch.zeros((1, 3), dtype=torch.float64))
    strided = ph.Batch(2, 2, torch.zeros(2, dtype=torch.int64), np.array([0, 1]),
                       torch.zeros((2, 2), dtype=torch.uint8), torch.zeros(4, dtype=torch.float64)[::2])
    assert not strided.coefs.is_contiguous()
    with pytest.raises(ValueError):
        strided.csr()
    with pytest.raises(ValueError):
        ph.eval_dense(torch.zeros((4, 2), dtype=torch.uint8), torch.zeros((3, 4), dtype=torch.float64),
                      torch.zeros((5, 2), dtype=torch.float64))
    with pytest.raises(ValueError, match="GPU tensor"):
        ph._check_points(torch.zeros((5, 2), dtype=torch.float64), 2)
