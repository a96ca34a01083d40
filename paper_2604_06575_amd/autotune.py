"""Autotuner for the library's launch parameters (run on the GPU).

Sweeps each tunable on a workload shaped like the one it governs, keeps the
fastest value, and writes ``tuning/gfx950.json``; the binding applies that
file when it loads the library.

    python -m paper_2604_06575_amd.autotune [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import paper_2604_06575_amd as ph  # noqa: E402
import workloads as W  # noqa: E402


def _time(fn, reps=5, warmup=2):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def sweep(name, values, fn, log):
    best, best_t = None, float("inf")
    rows = []
    for v in values:
        ph.tune_set(name, v)
        t = _time(fn)
        rows.append({"value": v, "ms": t})
        print(f"{name}={v}: {t:.3f} ms", flush=True)
        if t < best_t:
            best, best_t = v, t
    ph.tune_set(name, best)
    log[name] = {"best": best, "sweep": rows}
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning", "gfx950.json"))
    args = ap.parse_args()
    ph.lib()
    log = {}
    # times + simplify: raw terms per bucket workgroup
    wl = W.plain_large()
    a = ph.batch_from_numpy([0, 5000], wl.a_exps, wl.a_coefs, n=10, max_exp=8)
    b = ph.batch_from_numpy([0, 5000], wl.b_exps, wl.b_coefs, n=10, max_exp=8)
    ws_bytes, raw = ph.mul_workspace(a, b)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = ph._empty_out(10, 1, raw, 16, "cuda")
    sweep("mul_bucket_terms", [4096, 8192, 12288, 16384, 24576, 32768, 65536],
          lambda: ph.mul(a, b, ws=ws, out=out, finish=False), log)
    # batched simplify: persistent workgroups per CU
    bm = W.batch_matrix(npts=0)
    bb = ph.batch_from_numpy(bm.row_ptr, bm.exps, bm.coefs, n=bm.n, max_exp=bm.max_exp)
    sws = torch.empty(ph.simplify_workspace(bb), dtype=torch.uint8, device="cuda")
    sout = ph._empty_out(bm.n, 4096, int(bm.row_ptr[-1]), bm.max_exp, "cuda")
    sweep("seg_blocks_per_cu", [1, 2, 3, 4, 6],
          lambda: ph.simplify(bb, ws=sws, out=sout, finish=False), log)
    # sparse evaluation: point-tile workgroups per CU
    q = W.quartic(n=40, terms=30000, npts=8192)
    qb = ph.batch_from_numpy([0, 30000], q.exps, q.coefs, n=40, max_exp=4)
    X = torch.from_numpy(q.X).cuda()
    sweep("eval_blocks_per_cu", [2, 4, 8, 16, 32], lambda: ph.eval(qb, X), log)
    res = {"arch": "gfx950", "tool": "paper_2604_06575_amd.autotune", "date": time.strftime("%Y-%m-%d"),
           "tunables": {k: v["best"] for k, v in log.items()}, "sweeps": log}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res["tunables"]))


if __name__ == "__main__":
    main()
