"""Captured pipeline plans (poly_plan_*): simplify -> jacobian -> gradient
values of a polynomial matrix recorded into one HIP graph and replayed.

Every replay is checked against the eager entry points on the same inputs,
bit for bit (simplified terms, Jacobian terms, gradient values), with eager
work and synchronisations between replays, and the input coefficients
changed between replays (the plan reads its inputs at replay time).  The
simplified matrix is also held to the oracle.  Both simplify paths (one
workgroup per entry, device-wide sort over one key word or several) are
captured."""
import sys

import numpy as np
import pytest
import torch

import oracle
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
    old = ph.tune_get("simplify_wide_min")
    yield ph
    ph.tune_set("simplify_wide_min", old)


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


@pytest.mark.parametrize("path", ["per-entry", "device-wide", "key words"])
def test_plan_replays_match_eager(ph, path):
    ph.tune_set("simplify_wide_min", 1 << 62 if path == "per-entry" else 1)
    # 40 variables of degree <= 6: 120 bits of exponent fields, sorted over key words
    n = 40 if path == "key words" else 20
    wl = W.batch_matrix(seed=W.SEED_BASE + 60, entries=64, n=n, tmin=5, tmax=2000, npts=1024 if n == 40 else 4096)
    b = ph.batch_from_numpy(wl.row_ptr, wl.exps, wl.coefs, n=wl.n, max_exp=wl.max_exp)
    X = torch.from_numpy(wl.X).cuda()
    side = torch.cuda.Stream()
    say(f"plan ({path} simplify): 64 entries, n={n}, {b.nterms} terms, {X.shape[0]} points")
    with torch.cuda.stream(side):
        plan = ph.Plan(b, X)
    rng = W.rng_for(61)
    try:
        for rep in range(3):
            if rep:   # new coefficients, written before the replay
                b.coefs.copy_(torch.from_numpy(rng.standard_normal(b.nterms)).cuda())
            torch.cuda.synchronize()
            with torch.cuda.stream(side):
                plan.launch()
            side.synchronize()
            plan.finish()
            # eager pipeline on the same inputs
            s = ph.simplify(b)
            J = ph.jacobian(s)
            G = ph.grad(s, X)
            torch.cuda.synchronize()
            srp, sE, sC = ph.batch_to_numpy(plan.simplified)
            erp, eE, eC = ph.batch_to_numpy(s)
            assert np.array_equal(srp, erp) and np.array_equal(sE, eE) and np.array_equal(bits(sC), bits(eC))
            jrp, jE, jC = ph.batch_to_numpy(plan.jac)
            frp, fE, fC = ph.batch_to_numpy(J)
            assert np.array_equal(jrp, frp) and np.array_equal(jE, fE) and np.array_equal(bits(jC), bits(fC))
            assert np.array_equal(bits(plan.G.cpu().numpy()), bits(G.cpu().numpy()))
            if rep == 2:
                orp, oE, oC = oracle.simplify_batch(wl.row_ptr, wl.exps, b.coefs.cpu().numpy())
                assert np.array_equal(srp, orp) and np.array_equal(sE, oE) and np.array_equal(bits(sC), bits(oC))
            say(f"  replay {rep}: {int(srp[-1])} simplified terms, {int(jrp[-1])} Jacobian terms, bitwise")
    finally:
        plan.close()


def test_plan_rejects_null_stream_and_small_outputs(ph):
    import ctypes
    wl = W.batch_matrix(seed=W.SEED_BASE + 62, entries=4, tmin=5, tmax=50, npts=64)
    b = ph.batch_from_numpy(wl.row_ptr, wl.exps, wl.coefs, n=wl.n, max_exp=wl.max_exp)
    X = torch.from_numpy(wl.X).cuda()
    L = ph.lib()
    cin = b.csr()
    simp = ph._empty_out(b.n, b.npolys, b.nterms, b.max_exp, "cuda")
    jac = ph._empty_out(b.n, b.npolys * b.n, b.nterms * 8, b.max_exp, "cuda")
    G = torch.empty((b.npolys, 64, b.n), dtype=torch.float64, device="cuda")
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    cs, cj = simp.csr(), jac.csr()
    args = lambda st: (ctypes.byref(cin), 0.0, ph._ptr(X), 64, ctypes.byref(cs), ctypes.byref(cj),  # noqa: E731
                       ph._ptr(G), ctypes.c_void_p(ws.data_ptr()), ws.numel(), st, ctypes.byref(h))
    assert L.poly_plan_create(*args(None)) == 1                  # the null stream
    small = ph._empty_out(b.n, b.npolys * b.n, b.nterms, b.max_exp, "cuda")
    cj = small.csr()
    side = torch.cuda.Stream()
    assert L.poly_plan_create(*args(ctypes.c_void_p(side.cuda_stream))) == 1   # Jacobian capacity too small
    assert L.poly_plan_destroy(None) == 0
