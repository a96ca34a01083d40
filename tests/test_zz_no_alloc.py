"""The allocation-free simplify (poly_simplify_noalloc) against poly_simplify.

Both are called through the C ABI on the same inputs and must agree bit for
bit (row pointers, exponent rows, coefficients) and report the same device
status.  Two calls in a row share the library's fixed scratch: a batch that
takes the device-wide path (an entry above the wide threshold), then a smaller
batch of small entries that takes the per-entry path, so the second call
starts from the scratch the first one left behind; a third batch in 40
variables takes the sort over key words.  A third call declares an
exponent bound below a stored exponent and must report POLY_ERR_EXPONENT."""
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_06575_amd as ph
    ph.lib()
    return ph


def _batch(ph, wl, max_exp=None):
    return ph.batch_from_numpy(wl.row_ptr, wl.exps, wl.coefs, n=wl.n,
                               max_exp=wl.max_exp if max_exp is None else max_exp)


def _both(ph, b, tol=0.0):
    ref = ph.simplify(b, tol=tol, trim=False)
    T = b.nterms
    out = ph._empty_out(b.n, b.npolys, T, b.max_exp, b.coefs.device)
    out.exps.fill_(0xAB)
    out.coefs.fill_(float("nan"))
    status = torch.full((1,), -1, dtype=torch.int32, device=b.coefs.device)
    ph.simplify_noalloc(b, out, status, tol=tol)
    torch.cuda.synchronize()
    return ref, out, int(status.item())


def _assert_same(ref, out):
    rp = out.row_ptr.cpu().numpy()
    assert np.array_equal(rp, ref.row_ptr_host)
    U = int(rp[-1])
    assert np.array_equal(out.exps[:U].cpu().numpy(), ref.exps[:U].cpu().numpy())
    a = out.coefs[:U].cpu().numpy()
    b = ref.coefs[:U].cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_noalloc_matches_simplify_on_two_calls(ph):
    wide_min = ph.tune_get("simplify_wide_min")
    big = W.batch_matrix(seed=W.SEED_BASE + 71, entries=48, tmin=10, tmax=20000, npts=0)
    assert int(np.diff(big.row_ptr).max()) >= wide_min, "first call must take the device-wide path"
    small = W.batch_matrix(seed=W.SEED_BASE + 72, entries=300, tmin=1, tmax=600, npts=0)
    assert small.row_ptr[-1] < big.row_ptr[-1]
    assert int(np.diff(small.row_ptr).max()) < wide_min, "second call must take the per-entry path"
    # then 40 variables of 3-bit fields (120 bits): the sort over key words
    words = W.batch_matrix(seed=W.SEED_BASE + 74, entries=30, n=40, tmin=5, tmax=3000, npts=0)
    for name, wl, tol in (("wide", big, 0.0), ("per-entry", small, 0.5), ("key words", words, 0.0)):
        say(f"noalloc {name}: {wl.row_ptr.shape[0] - 1} entries, {int(wl.row_ptr[-1])} terms, tol {tol}")
        ref, out, st = _both(ph, _batch(ph, wl), tol)
        assert st == 0
        _assert_same(ref, out)


def test_noalloc_reports_device_status(ph):
    wl = W.batch_matrix(seed=W.SEED_BASE + 73, entries=20, tmin=5, tmax=300, npts=0)
    assert int(wl.exps.max()) > 2
    say(f"noalloc status: {int(wl.row_ptr[-1])} terms, declared max_exp 2")
    b = _batch(ph, wl, max_exp=2)   # a stored exponent exceeds the declaration
    out = ph._empty_out(b.n, b.npolys, b.nterms, b.max_exp, b.coefs.device)
    status = torch.zeros(1, dtype=torch.int32, device=b.coefs.device)
    ph.simplify_noalloc(b, out, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 5   # POLY_ERR_EXPONENT
    # the next call clears the status it starts from
    good = _batch(ph, wl)
    ref, out2, st = _both(ph, good)
    assert st == 0
    _assert_same(ref, out2)
