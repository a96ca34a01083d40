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

import numpy as np
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
    # times + simplify of batches (bucket path): raw terms per bucket workgroup
    pairs = [W.plain_large(seed=W.SEED_BASE + 70 + k, terms=1200, n=8, d=8) for k in range(8)]
    rp = np.arange(9, dtype=np.int64) * 1200
    a = ph.batch_from_numpy(rp, np.concatenate([w.a_exps for w in pairs]), np.concatenate([w.a_coefs for w in pairs]),
                            n=8, max_exp=8)
    b = ph.batch_from_numpy(rp, np.concatenate([w.b_exps for w in pairs]), np.concatenate([w.b_coefs for w in pairs]),
                            n=8, max_exp=8)
    ws_bytes, raw = ph.mul_workspace(a, b)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = ph._empty_out(8, 8, raw, 16, "cuda")
    sweep("mul_bucket_terms", [8192, 16384, 32768, 65536],
          lambda: ph.mul(a, b, ws=ws, out=out, finish=False), log)
    del ws, out
    # one pair: the raw size from which the radix-sort path beats the bucket path
    rows, threshold = [], None
    for terms in (100, 150, 200, 300, 700, 1500, 3000):
        w = W.plain_large(seed=W.SEED_BASE + 80, terms=terms, n=8, d=8)
        a1 = ph.batch_from_numpy([0, terms], w.a_exps, w.a_coefs, n=8, max_exp=8)
        b1 = ph.batch_from_numpy([0, terms], w.b_exps, w.b_coefs, n=8, max_exp=8)
        ph.tune_set("mul_sort_min_raw", 0)
        t_sort = _time(lambda: ph.mul(a1, b1))
        ph.tune_set("mul_sort_min_raw", 1 << 62)
        t_bucket = _time(lambda: ph.mul(a1, b1))
        rows.append({"raw": terms * terms, "sort_ms": t_sort, "bucket_ms": t_bucket})
        print(f"one pair raw={terms * terms}: sort {t_sort:.3f} ms, bucket {t_bucket:.3f} ms", flush=True)
        if threshold is None and t_sort < t_bucket:
            threshold = terms * terms
    threshold = threshold if threshold is not None else 1 << 62
    ph.tune_set("mul_sort_min_raw", threshold)
    log["mul_sort_min_raw"] = {"best": threshold, "sweep": rows}
    # global radix sorts: widest digit (fewer, wider passes against larger
    # per-tile histograms), on the headline one-pair product
    big = W.plain_large()
    a2 = ph.batch_from_numpy([0, big.a_exps.shape[0]], big.a_exps, big.a_coefs, n=big.n, max_exp=big.max_exp)
    b2 = ph.batch_from_numpy([0, big.b_exps.shape[0]], big.b_exps, big.b_coefs, n=big.n, max_exp=big.max_exp)
    ph.tune_set("mul_sort_min_raw", 0)
    # one workspace for every width (the widest needs the most), values
    # interleaved over two rounds and the faster round kept, so allocation
    # and clock drift do not pick the winner
    ph.tune_set("sort_digit_bits", 11)
    ws2_bytes, raw2 = ph.mul_workspace(a2, b2)
    ws2 = torch.empty(ws2_bytes, dtype=torch.uint8, device="cuda")
    out2 = ph._empty_out(big.n, 1, raw2, 2 * big.max_exp, "cuda")
    widths = (6, 7, 8, 9, 10, 11)
    best_of = {b: float("inf") for b in widths}
    for _ in range(2):
        for bits in widths:
            ph.tune_set("sort_digit_bits", bits)
            t = _time(lambda: ph.mul(a2, b2, ws=ws2, out=out2, finish=False), reps=20, warmup=3)
            best_of[bits] = min(best_of[bits], t)
    rows = [{"value": b, "ms": best_of[b]} for b in widths]
    for r in rows:
        print(f"sort_digit_bits={r['value']}: {r['ms']:.3f} ms", flush=True)
    best_bits = min(widths, key=lambda b: best_of[b])
    del ws2, out2
    ph.tune_set("sort_digit_bits", best_bits)
    ph.tune_set("mul_sort_min_raw", threshold)
    log["sort_digit_bits"] = {"best": best_bits, "sweep": rows}
    # batched simplify: the largest-entry size from which the device-wide sort
    # beats one workgroup per entry (16 entries of that size)
    rows, threshold = [], None
    for size in (1024, 2048, 4096, 8192, 16384, 32768):
        polys = [W.random_poly(W.rng_for(W.SEED_BASE + 90 + k), 6, 4, size) for k in range(16)]
        rp, E, C = W.csr_from_list(polys, 6)
        sb = ph.batch_from_numpy(rp, E, C, n=6, max_exp=4)
        ph.tune_set("simplify_wide_min", 1)
        t_wide = _time(lambda: ph.simplify(sb))
        ph.tune_set("simplify_wide_min", 1 << 62)
        t_seg = _time(lambda: ph.simplify(sb))
        rows.append({"entry_terms": size, "wide_ms": t_wide, "per_entry_ms": t_seg})
        print(f"simplify 16 x {size}: device-wide {t_wide:.3f} ms, per entry {t_seg:.3f} ms", flush=True)
        if threshold is None and t_wide < t_seg:
            threshold = size
    threshold = threshold if threshold is not None else 1 << 62
    ph.tune_set("simplify_wide_min", threshold)
    log["simplify_wide_min"] = {"best": threshold, "sweep": rows}
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
    # gradients: derivatives streamed from the source terms (n up to the
    # value) or through the formed Jacobian, on a 20-variable matrix
    gm = W.batch_matrix(entries=256, npts=4096)
    gb = ph.simplify(ph.batch_from_numpy(gm.row_ptr, gm.exps, gm.coefs, n=gm.n, max_exp=gm.max_exp))
    GX = torch.from_numpy(gm.X).cuda()
    sweep("deriv_fused_max_n", [0, 255], lambda: ph.grad(gb, GX), log)
    # dense FP64 contraction: rows of C per workgroup, on a sixteenth of the
    # 4,096 x 46,376 x 65,536 shape (the full degree-4 basis in 30 variables)
    dw = W.dense_shared(P=1024, N=16384)
    dbasis, dC, dX = (torch.from_numpy(x).cuda() for x in (dw.basis, dw.C, dw.X))
    dY = torch.empty((dC.shape[0], dX.shape[0]), dtype=torch.float64, device="cuda")
    sweep("dense_f64_rows", [64, 128], lambda: ph.eval_dense(dbasis, dC, dX, Y=dY), log)
    del dbasis, dC, dX, dY
    res = {"arch": "gfx950", "tool": "paper_2604_06575_amd.autotune", "date": time.strftime("%Y-%m-%d"),
           "tunables": {k: v["best"] for k, v in log.items()}, "sweeps": log}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res["tunables"]))


if __name__ == "__main__":
    main()
