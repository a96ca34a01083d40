"""The times+simplify and simplify launch sequences captured into a HIP graph
(torch.cuda.CUDAGraph on ROCm) and replayed: every replay, with eager work
and synchronisations between replays, reproduces the eager result bit for
bit.  The sequences clear their counters with kernels, never memsets."""
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


def _snapshot(out):
    T = int(out.row_ptr[-1].item())
    return (out.row_ptr.cpu().numpy().copy(), out.exps[:T].cpu().numpy().copy(),
            out.coefs[:T].cpu().numpy().copy())


def test_mul_graph_replay(ph):
    wl = W.plain_large(seed=W.SEED_BASE + 60, terms=900, n=8, d=6)
    a = ph.batch_from_numpy([0, 900], wl.a_exps, wl.a_coefs, n=8, max_exp=6)
    b = ph.batch_from_numpy([0, 900], wl.b_exps, wl.b_coefs, n=8, max_exp=6)
    ws_bytes, raw = ph.mul_workspace(a, b)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = ph._empty_out(8, 1, raw, 12, "cuda")
    say("eager")
    ref = ph.batch_to_numpy(ph.mul(a, b))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ph.mul(a, b, ws=ws, out=out, finish=False)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("capture")
    with torch.cuda.graph(g, stream=s):
        ph.mul(a, b, ws=ws, out=out, finish=False)
    for rep in range(3):
        out.coefs.fill_(-1.0)
        out.row_ptr.fill_(0)
        torch.cuda.synchronize()
        say(f"replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        rp, E, C = _snapshot(out)
        assert np.array_equal(rp, ref[0]) and np.array_equal(E, ref[1])
        assert C.view(np.uint64).tolist() == ref[2].view(np.uint64).tolist()
        _ = ph.mul(a, b)   # eager work between replays


def test_simplify_graph_replay(ph):
    wl = W.batch_matrix(seed=W.SEED_BASE + 61, entries=300, tmin=10, tmax=9000, npts=0)
    b = ph.batch_from_numpy(wl.row_ptr, wl.exps, wl.coefs, n=wl.n, max_exp=wl.max_exp)
    ref = ph.batch_to_numpy(ph.simplify(b))
    out = ph._empty_out(wl.n, 300, int(wl.row_ptr[-1]), wl.max_exp, "cuda")
    ws = torch.empty(ph.simplify_workspace(b), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ph.simplify(b, ws=ws, out=out, finish=False)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ph.simplify(b, ws=ws, out=out, finish=False)
    for rep in range(3):
        out.coefs.fill_(7.0)
        torch.cuda.synchronize()
        say(f"simplify replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        rp, E, C = _snapshot(out)
        assert np.array_equal(rp, ref[0]) and np.array_equal(E, ref[1])
        assert C.view(np.uint64).tolist() == ref[2].view(np.uint64).tolist()
        _ = ph.simplify(b)
