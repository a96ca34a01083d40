"""Benchmark of the hot path on one MI355X.

Default workload (the expand + simplify metric): p and q in n=10 variables,
degree <= 8, 5,000 distinct terms each, N(0,1) coefficients, exponents packed
at 5 bits per variable -- 25,000,000 raw product terms per step.  A step is
one poly_mul call (pack, raw product generation, stable radix sort of
(key, raw index) pairs, in-order run sums with zero drop, scan, unpack); inputs are resident in HBM before the timed region and the
output/workspace buffers are allocated once.  `value` is raw product terms
merged per second.  The roofline object describes the dominant kernel (one
radix pass), timed live with HIP events the library records around each of
its launches; its `traffic` comes from the committed rocprofv3 counter
summary when that summary was taken on the current kernel sources.

It also measures the evaluation metric: 4,096 polynomials over the full
degree <= 4 monomial set in n=30 variables (46,376 monomials) at 65,536
points, in plain FP64 (FP64 MFMA) and split BF16 (BF16 MFMA, FP32
accumulation, FP64 recombination), each with its error against an FP64
reference on sampled outputs; the sparse derivative paths, the
affine-normal direction of a sparse quartic at a batch of points, the
square of a 3 x 3 polynomial matrix, the paper's heavy-simplify family
simplify(p_d^3), its affine-normal scaling family up to n = 240, and the
stochastic affine-normal route on its crossover family (speed preset,
against the exact route) and accuracy preset (angle over probe seeds).

Prints one JSON line.  --gpus N with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic bytes per raw product term for expand + simplify: the raw term
# written once and read once as a 64-bit key and a 32-bit payload
BYTES_PER_RAW_TERM = 24


def sort_plan(n, max_exp_a, max_exp_b, raw, bits=8):
    """The radix-sort path's pass structure for one pair (the library's own
    rule): mixed-radix keys in [0, r^n) with r = max_exp_a + max_exp_b + 1,
    as few passes of at most `bits` bits (the sort_digit_bits tunable) as
    that range needs, and -- when the
    digits left after the first pass and the raw index fit one 64-bit word --
    packed 8-byte elements from the first pass on.  Returns (passes, digit
    bits, packed, average algorithmic bytes per raw term per scatter launch):
    a pass reads and writes every element once, 12 B each way unpacked, 8 B
    packed; the first pass generates its elements from the operands (reads
    nothing per raw term) and writes 8 B packed or 12 B unpacked."""
    r = max_exp_a + max_exp_b + 1
    key_bits = (r ** n - 1).bit_length()
    passes = -(-key_bits // bits)
    db = max(-(-key_bits // passes) if passes else 4, 4)
    raw_bits = (raw - 1).bit_length() if raw > 1 else 0
    packed = passes >= 2 and key_bits - db + raw_bits <= 64
    if not passes:
        return 0, db, packed, 0.0
    per_term = (8 + 16 * (passes - 1)) / passes if packed else (12 + 24 * (passes - 1)) / passes
    return passes, db, packed, per_term


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--terms", type=int, default=5000, help="terms per operand")
    ap.add_argument("--no-eval", action="store_true", help="skip the evaluation measurement")
    ap.add_argument("--eval-steps", type=int, default=3)
    ap.add_argument("--eval-points", type=int, default=65536)
    ap.add_argument("--eval-polys", type=int, default=4096)
    ap.add_argument("--nslices", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-terms", type=int, default=5000, help="q terms in the CPU baseline sample")
    ap.add_argument("--no-batch", action="store_true", help="skip the polynomial-matrix workload")
    ap.add_argument("--no-latency", action="store_true", help="skip the small-call latency workload")
    ap.add_argument("--no-deriv", action="store_true", help="skip the quartic derivative workload")
    ap.add_argument("--no-affine", action="store_true", help="skip the affine-normal workload")
    ap.add_argument("--no-mtimes", action="store_true", help="skip the polynomial-matrix product workload")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's simplify(p_d^3) family")
    ap.add_argument("--no-affine-scaling", action="store_true", help="skip the affine-normal scaling family")
    ap.add_argument("--no-affine-stochastic", action="store_true",
                    help="skip the stochastic affine-normal route (crossover family and accuracy preset)")
    ap.add_argument("--affine-n", type=int, default=64)
    ap.add_argument("--affine-points", type=int, default=4096)
    ap.add_argument("--graph", action="store_true", help="also time the times+simplify step as a captured HIP graph")
    ap.add_argument("--tune", action="append", default=[], metavar="NAME=VALUE",
                    help="set a library tunable before measuring (repeatable)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def time_events(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3 / steps, wall / steps


def bench_mul(args):
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    wl = W.plain_large(terms=args.terms)
    rp = [0, args.terms]
    a = ph.batch_from_numpy(rp, wl.a_exps, wl.a_coefs, n=wl.n, max_exp=wl.max_exp)
    b = ph.batch_from_numpy(rp, wl.b_exps, wl.b_coefs, n=wl.n, max_exp=wl.max_exp)
    ws_bytes, raw = ph.mul_workspace(a, b)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = ph._empty_out(wl.n, 1, raw, 2 * wl.max_exp, "cuda")
    step = lambda: ph.mul(a, b, ws=ws, out=out, finish=False)  # noqa: E731
    # correctness of the timed configuration: status word and term count
    ph.mul(a, b, ws=ws, out=out, finish=True, trim=False)
    uniq = int(out.row_ptr_host[-1])
    t_ev, t_wall = time_events(step, args.steps, args.warmup)
    # the dominant kernel's own duration: HIP events recorded by the library
    # on its launch stream around every bucket-kernel launch of K more steps
    k_ms, k_n = kernel_ms(ph.TIMING_MUL, step, args.steps)
    sort_path = raw >= ph.tune_get("mul_sort_min_raw")
    plan = sort_plan(wl.n, wl.max_exp, wl.max_exp, raw, ph.tune_get("sort_digit_bits")) if sort_path else None
    return dict(raw=raw, unique=uniq, t=t_ev, t_wall=t_wall, ws_bytes=ws_bytes, wl=wl, k_ms=k_ms, k_n=k_n,
                sort_path=sort_path, plan=plan)


def kernel_ms(slot, fn, steps):
    """Average duration (ms) of the dominant kernel in `slot` over `steps`
    calls of fn, from the library's event hooks."""
    import torch
    import paper_2604_06575_amd as ph
    torch.cuda.synchronize()
    ph.timing_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms, n = ph.timing_read(slot)
    ph.timing_enable(False)
    return (ms / n if n else float("nan")), n


KERNEL_SOURCES = ["paper_2604_06575_amd/csrc/mulsort.hip", "paper_2604_06575_amd/csrc/mulsort.h",
                  "paper_2604_06575_amd/csrc/internal.h"]
TRAFFIC_FILE = "profiles/k_gs_scatter_times_n10_5000x5000_traffic.txt"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per bucket-kernel launch from the committed rocprofv3
    counter summary, or None if it is missing or was taken on other sources."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def dense_reference(basis, C, Xs):
    """Y = C V and |C| |V| at a few points in plain NumPy FP64, V[k, pt] the
    product of x_i ** e_ki: the error yardstick for the dense timings."""
    V = np.prod(Xs[None, :, :] ** basis.astype(np.float64)[:, None, :], axis=2)
    return C @ V, np.abs(C) @ np.abs(V)


def bench_eval(args):
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    P, N = args.eval_polys, args.eval_points
    wl = W.dense_shared(P=P, N=N)
    K = wl.basis.shape[0]
    basis = torch.from_numpy(wl.basis).cuda()
    C = torch.from_numpy(wl.C).cuda()
    X = torch.from_numpy(wl.X).cuda()
    Y = torch.empty((P, N), dtype=torch.float64, device="cuda")
    res = {}
    # FP64 reference values on a sample of outputs (NumPy, CPU): 8 points x all polys
    rng = np.random.default_rng(7)
    pts = np.sort(rng.choice(N, size=8, replace=False))
    Yref, Aref = dense_reference(wl.basis, wl.C, wl.X[pts])
    for name, prec, S in (("fp64", ph.POLY_FP64, 0), ("split_bf16", ph.POLY_SPLIT_BF16, args.nslices)):
        need = ph.eval_dense_workspace(wl.n, K, P, N, prec, S if S else 5)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        fn = lambda: ph.eval_dense(basis, C, X, prec=prec, nslices=S if S else 5, ws=ws, Y=Y)  # noqa: E731
        t_ev, _ = time_events(fn, args.eval_steps, 1)
        k_ms, _ = kernel_ms(ph.TIMING_DENSE, fn, args.eval_steps)
        Ys = Y[:, torch.from_numpy(pts).cuda()].cpu().numpy()
        err = np.abs(Ys - Yref)
        flops = 2.0 * P * K * N
        if prec == ph.POLY_FP64:
            mfma_flops, peak = flops, FP64_PEAK_TFLOPS
        else:
            pairs = S * (S + 1) // 2
            mfma_flops, peak = flops * pairs, BF16_PEAK_TFLOPS
        res[name] = {
            "point_evals_per_s": P * N / t_ev,
            "ms": t_ev * 1e3,
            "nslices": S if S else None,
            "max_cond_scaled_err": float((err / Aref).max()),
            "median_rel_err": float(np.median(err / np.maximum(np.abs(Yref), 1e-300))),
            "max_rel_err": float((err / np.maximum(np.abs(Yref), 1e-300)).max()),
            "fp64_equiv_tflops": flops / t_ev / 1e12,
            "mfma_tflops": mfma_flops / t_ev / 1e12,
            "mfma_peak_tflops": peak,
            "mfma_frac": mfma_flops / t_ev / 1e12 / peak,
            "kernel_ms": k_ms,
            "kernel_mfma_frac": mfma_flops / (k_ms / 1e3) / 1e12 / peak,
            "error_sample": "8 points x all polynomials vs a NumPy FP64 reference (C V)",
        }
        if prec == ph.POLY_FP64:
            Y64 = Y.clone()
        else:
            # the split result over every output against the FP64 GPU path,
            # condition-scaled by sum_k |c_k v_k| (an FP64 contraction of |C|
            # with the monomials at |x|) and componentwise
            A = ph.eval_dense(basis, C.abs(), X.abs(), prec=ph.POLY_FP64)
            d = (Y - Y64).abs()
            rel = d / Y64.abs().clamp_min(1e-300)
            res[name]["all_outputs_vs_fp64_gpu"] = {
                "outputs": int(Y.numel()),
                "max_cond_scaled_err": float((d / A).max().item()),
                "max_rel_err": float(rel.max().item()),
                "median_rel_err": float(rel.flatten()[::97].median().item()),
                "frac_rel_err_above_1e-10": float((rel > 1e-10).double().mean().item()),
                "note": "median over every 97th output; max and fraction over all outputs",
            }
            del A, d, rel, Y64
        del ws
    # reverse mode (FP64 MFMA): dC = gY V^T and dX through W = C^T gY
    gY = torch.randn((P, N), dtype=torch.float64, device="cuda")
    fn_b = lambda: ph.eval_dense_backward(basis, C, X, gY)  # noqa: E731
    t_b, _ = time_events(fn_b, 1, 1)
    k_ms_b, _ = kernel_ms(ph.TIMING_DENSE, lambda: ph.eval_dense_backward(basis, C, X, gY, want_dX=False), 1)
    t_dx, _ = time_events(lambda: ph.eval_dense_backward(basis, C, X, gY, want_dC=False), 1, 1)
    flops = 2.0 * P * K * N
    res["backward_fp64"] = {"ms": t_b * 1e3, "dC_kernel_ms": k_ms_b, "dX_ms": t_dx * 1e3,
                            "dC_mfma_frac": flops / (k_ms_b / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                            "dX_mfma_frac": flops / t_dx / 1e12 / FP64_PEAK_TFLOPS,
                            "flops_note": "dC = gY V^T and W = C^T gY are 2 P K N flops each"}
    # split reverse mode (BF16 digits per 128-point block for dC, per
    # 128-polynomial block for W = C^T gY), against the FP64 kernels over
    # every output, condition-scaled by the same sums over absolute values
    S = args.nslices
    fn_s = lambda: ph.eval_dense_backward(basis, C, X, gY, want_dX=False,  # noqa: E731
                                          prec=ph.POLY_SPLIT_BF16, nslices=S)
    t_s, _ = time_events(fn_s, 1, 1)
    k_ms_s, _ = kernel_ms(ph.TIMING_DENSE, fn_s, 1)
    pairs = S * (S + 1) // 2
    dCs = fn_s()[0]
    d = (dCs - ph.eval_dense_backward(basis, C, X, gY, want_dX=False)[0]).abs()
    del dCs
    A = ph.eval_dense_backward(basis, C, X.abs(), gY.abs(), want_dX=False)[0]
    cond = d / A
    del A
    res["backward_split_dC"] = {
        "nslices": S, "ms": t_s * 1e3, "kernel_ms": k_ms_s,
        "kernel_mfma_frac": flops * pairs / (k_ms_s / 1e3) / 1e12 / BF16_PEAK_TFLOPS,
        "fp64_equiv_speedup_vs_fp64_kernel": k_ms_b / k_ms_s,
        "max_cond_scaled_err_vs_fp64_gpu": float(cond.max().item()),
        "frac_cond_scaled_err_above_1e-10": float((cond > 1e-10).double().mean().item()),
        "note": "every output; sum_pt |gY v_k| from the FP64 kernel on |gY|, |x| (|C| does not enter dC)",
    }
    del d, cond
    fn_x = lambda: ph.eval_dense_backward(basis, C, X, gY, want_dC=False,  # noqa: E731
                                          prec=ph.POLY_SPLIT_BF16, nslices=S)
    t_sx, _ = time_events(fn_x, 1, 1)
    dx = (fn_x()[1] - ph.eval_dense_backward(basis, C, X, gY, want_dC=False)[1]).abs()
    ax = ph.eval_dense_backward(basis, C.abs(), X.abs(), gY.abs(), want_dC=False)[1]
    condx = dx / ax
    res["backward_split_dX"] = {
        "nslices": S, "ms": t_sx * 1e3, "speedup_vs_fp64": t_dx / t_sx,
        "mfma_frac": flops * pairs / t_sx / 1e12 / BF16_PEAK_TFLOPS,
        "max_cond_scaled_err_vs_fp64_gpu": float(condx.max().item()),
        "frac_cond_scaled_err_above_1e-10": float((condx > 1e-10).double().mean().item()),
        "note": "W = C^T gY on BF16 MFMA per chunk of 4,096 points, then W contracted with the monomial "
                "derivatives in FP64; mfma_frac over the whole call (digit planes, W round trip and the "
                "derivative pass included)",
    }
    del dx, ax, condx, gY
    res["workload"] = {"polys": P, "monomials": K, "points": N, "n": wl.n, "degree": 4}
    return res


def bench_batch(args):
    """64x64 polynomial matrix, n=20: one persistent simplify launch, the
    64x64x20 Jacobian, and its evaluation at 4,096 points."""
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    wl = W.batch_matrix()
    b = ph.batch_from_numpy(wl.row_ptr, wl.exps, wl.coefs, n=wl.n, max_exp=wl.max_exp)
    X = torch.from_numpy(wl.X).cuda()
    s = ph.simplify(b)
    J = ph.jacobian(s)
    t_simp, _ = time_events(lambda: ph.simplify(b, trim=False), 3, 1)
    t_jac, _ = time_events(lambda: ph.jacobian(s, trim=False), 3, 1)
    t_eval, _ = time_events(lambda: ph.eval(J, X), 2, 1)
    t_grad, _ = time_events(lambda: ph.grad(s, X), 2, 1)
    T_in, T_s, T_j = int(wl.row_ptr[-1]), s.nterms, J.nterms
    term_points = T_j * X.shape[0]
    # algorithmic work: simplify reads every input term and writes every kept
    # one ((n + 8) B each); evaluating a term of degree d at a point is d
    # multiplications and one FMA
    simp_bytes = (T_in + T_s) * (wl.n + 8)
    jd = J.exps[:T_j].sum(1, dtype=torch.int64)
    eval_flops = float((jd + 2).sum().item()) * X.shape[0]
    # the kernel reads a term's factors from the LDS point tile in chunks of
    # four (padding chunks point at a row of ones): 4 ceil(d / 4) 8-byte reads
    # per term and point
    lds_bytes = float((4 * ((jd + 3) // 4)).sum().item()) * 8.0 * X.shape[0]
    return {"entries": 4096, "raw_terms": T_in, "simplified_terms": T_s, "jacobian_terms": T_j, "points": X.shape[0],
            "simplify_ms": t_simp * 1e3, "simplify_terms_per_s": T_in / t_simp,
            "simplify_gbps": simp_bytes / t_simp / 1e9, "simplify_hbm_frac": simp_bytes / t_simp / 8e12,
            "jacobian_ms": t_jac * 1e3, "jacobian_terms_per_s": T_j / t_jac,
            "jacobian_eval_ms": t_eval * 1e3, "jacobian_eval_term_points_per_s": term_points / t_eval,
            "jacobian_eval_fp64_tflops": eval_flops / t_eval / 1e12,
            "jacobian_eval_fp64_frac": eval_flops / t_eval / 78.6e12,
            "jacobian_eval_lds_tbps": lds_bytes / t_eval / 1e12,
            "grad_fused_ms": t_grad * 1e3, **bench_plan(b, X),
            "note": "simplify/jacobian times include the host readback of the output row pointer"}


def bench_plan(b, X):
    """simplify -> jacobian -> gradient values of the batch: eager calls (with
    their host read-backs of output sizes) against the same pipeline captured
    once as a plan (one HIP graph, sizes kept on the device) and replayed."""
    import torch
    import paper_2604_06575_amd as ph

    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan = ph.Plan(b, X)
        try:
            t_plan, _ = time_events(plan.launch, 3, 1)
            t_eager, _ = time_events(lambda: ph.grad(ph.simplify(b), X), 3, 1)
        finally:
            side.synchronize()
            plan.close()
    return {"pipeline_eager_ms": t_eager * 1e3, "pipeline_graph_ms": t_plan * 1e3}


def bench_latency(args):
    """Latency of single small calls (n=4, two polynomials of 200 terms,
    degree <= 6, integer coefficients; 1,024 points): times + simplify of the
    pair, simplify of one operand, evaluation of the product at the points;
    microseconds per call over back-to-back calls with the workspace and
    output allocated once, and the output size read back (mul, simplify)."""
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    wl = W.plain_small()
    rp = [0, wl.a_exps.shape[0]]
    a = ph.batch_from_numpy(rp, wl.a_exps, wl.a_coefs, n=wl.n, max_exp=wl.max_exp)
    b = ph.batch_from_numpy(rp, wl.b_exps, wl.b_coefs, n=wl.n, max_exp=wl.max_exp)
    X = torch.from_numpy(wl.X).cuda()
    ws_bytes, raw = ph.mul_workspace(a, b)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = ph._empty_out(wl.n, 1, raw, 2 * wl.max_exp, "cuda")
    p = ph.mul(a, b)
    t_mul, _ = time_events(lambda: ph.mul(a, b, ws=ws, out=out), 50, 5)
    t_simp, _ = time_events(lambda: ph.simplify(a), 50, 5)
    t_eval, _ = time_events(lambda: ph.eval(p, X), 50, 5)
    return {"n": wl.n, "terms": [int(rp[1]), int(rp[1])], "raw_terms": int(raw), "product_terms": p.nterms,
            "points": int(X.shape[0]), "mul_us": t_mul * 1e6, "simplify_us": t_simp * 1e6,
            "eval_us": t_eval * 1e6}


def bench_deriv(args):
    """Random quartic, n=100, 100,000 terms, 8,192 points: value, gradient
    through the reverse-mode kernel (unit cotangent), Hessian."""
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    wl = W.quartic()
    b = ph.batch_from_numpy([0, wl.exps.shape[0]], wl.exps, wl.coefs, n=wl.n, max_exp=4)
    X = torch.from_numpy(wl.X).cuda()
    gY = torch.ones((1, X.shape[0]), dtype=torch.float64, device="cuda")
    t_eval, _ = time_events(lambda: ph.eval(b, X), 3, 1)
    t_bwd, _ = time_events(lambda: ph.eval_backward(b, X, gY), 2, 1)
    t_hess, _ = time_events(lambda: ph.hess(b, X), 1, 1)
    N = X.shape[0]
    # algorithmic FP64 flops per point: a term of degree d costs d
    # multiplications and one FMA; its first derivatives are supp terms of
    # degree d - 1, its Hessian entries (j <= k) c2 terms of degree d - 2
    E = wl.exps.astype(np.int64)
    d = E.sum(1)
    supp = (E > 0).sum(1)
    c2 = supp * (supp - 1) // 2 + (E >= 2).sum(1)
    f_eval = float((d + 2).sum()) * N
    f_grad = float((supp * (d + 1)).sum()) * N
    f_hess = float((c2 * d).sum()) * N
    return {"terms": wl.exps.shape[0], "n": wl.n, "points": N,
            "eval_ms": t_eval * 1e3, "backward_dx_dc_ms": t_bwd * 1e3, "hessian_ms": t_hess * 1e3,
            "eval_fp64_tflops": f_eval / t_eval / 1e12, "hessian_fp64_tflops": f_hess / t_hess / 1e12,
            "hessian_write_gbps": 8.0 * N * wl.n * wl.n / t_hess / 1e9,
            "flops_note": f"per call: eval {f_eval:.3g}, gradient {f_grad:.3g} (inside the reverse mode), "
                          f"Hessian {f_hess:.3g} FP64 flops; FP64 vector peak 78.6 TFLOP/s",
            "dtype": {"f": "f64", "grad": "f64", "hessian": "f64 (100x100 per point, both triangles)"}}


def bench_affine(args):
    """Affine-normal directions (exact log-det route) of a sparse quartic in
    n=64 variables (support 3, 4n monomials, plus sum x_i^2) at 4,096 points:
    gradient and Hessian paths, then one workgroup per point."""
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    wl = W.sparse_quartic(n=args.affine_n, npts=args.affine_points)
    n, N = wl.n, wl.X.shape[0]
    b = ph.batch_from_numpy([0, wl.exps.shape[0]], wl.exps, wl.coefs, n=n, max_exp=4)
    X = torch.from_numpy(wl.X).cuda()
    ws = torch.empty(ph.affine_normal_workspace(b, N), dtype=torch.uint8, device="cuda")
    step = lambda: ph.affine_normal(b, X, reg=1e-8, ws=ws)  # noqa: E731
    D, _ = ph.affine_normal(b, X, reg=1e-8, ws=ws, check=True)
    finite = bool(torch.isfinite(D).all().item())
    t, _ = time_events(step, 5, 2)
    k_ms, k_n = kernel_ms(ph.TIMING_AFFINE, step, 5)
    m = n - 1
    # per point: Gauss-Jordan inverse of the (n-1)^2 tangent block (2 m^3),
    # two rank-two frame updates and three matrix-vector products (~18 n^2)
    flops = N * (2.0 * m ** 3 + 18.0 * n * n)
    return {"n": n, "terms": int(wl.exps.shape[0]), "points": N, "ms": t * 1e3,
            "points_per_s": N / t, "kernel_ms": k_ms, "kernel_launches_timed": k_n,
            "kernel_fp64_tflops": flops / (k_ms / 1e3) / 1e12, "fp64_vector_peak_tflops": 78.6,
            "kernel_fp64_frac": flops / (k_ms / 1e3) / 1e12 / 78.6,
            "flops_note": "2 (n-1)^3 + 18 n^2 FP64 flops per point (tangent-block inverse, frame updates)",
            "all_finite": finite, "regularization": 1e-8}


def bench_affine_scaling(args):
    """The paper's exact log-det scaling family (sparse quartics of support 3
    with 4n monomials) at n = 20, 40, 80, 160 and 240, 256 points each: the
    work matrix sits in registers (n <= 65), LDS (n <= 128) or the
    workspace (larger n)."""
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    res = {}
    for n in (20, 40, 80, 160, 240):
        wl = W.sparse_quartic(seed=W.SEED_BASE + 300 + n, n=n, npts=256)
        N = wl.X.shape[0]
        b = ph.batch_from_numpy([0, wl.exps.shape[0]], wl.exps, wl.coefs, n=n, max_exp=4)
        X = torch.from_numpy(wl.X).cuda()
        ws = torch.empty(ph.affine_normal_workspace(b, N), dtype=torch.uint8, device="cuda")
        step = lambda: ph.affine_normal(b, X, reg=1e-8, ws=ws)  # noqa: E731
        D, _ = ph.affine_normal(b, X, reg=1e-8, ws=ws, check=True)
        t, _ = time_events(step, 3, 1)
        k_ms, _ = kernel_ms(ph.TIMING_AFFINE, step, 3)
        res[f"n{n}"] = {"points": N, "ms": t * 1e3, "points_per_s": N / t, "kernel_ms": k_ms,
                        "all_finite": bool(torch.isfinite(D).all().item())}
        del ws
    return res


def _angles_deg(A, B):
    import torch
    c = (A * B).sum(1) / (A.norm(dim=1) * B.norm(dim=1))
    return torch.rad2deg(torch.arccos(c.clamp(-1.0, 1.0)))


def bench_affine_stochastic(args):
    """The stochastic log-det route (Section 5, MF-logDet-Stochastic).
    Crossover family of the paper's Section 6.6: support-2 sparse quartics
    with m = 3n monomials at n = 80, 120, 180 and 240, 256 points per call
    in [-0.25, 0.25]^n (where the tangent blocks are positive definite),
    the speed preset (one Rademacher probe, reg 5e-4, tol 2e-2, 6 steps)
    against the exact route (reg 1e-8) on the same points: time per call,
    speedup t_exact / t_stochastic, and the angle between the two
    directions.  Accuracy preset of the paper's accuracy tables (64
    Rademacher probes, tol 1e-4, 80 steps, reg 1e-8) on a sparse quartic in 6
    variables with 17 monomials at 4,096 points, over 10 probe seeds: angle
    to the exact direction (mean and standard deviation over points and
    seeds)."""
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    cross = {}
    for n in (80, 120, 180, 240):
        wl = W.sparse_quartic(seed=W.SEED_BASE + 400 + n, n=n, npts=256, support=2)
        N = wl.X.shape[0]
        b = ph.batch_from_numpy([0, wl.exps.shape[0]], wl.exps, wl.coefs, n=n, max_exp=4)
        X = torch.from_numpy(wl.X * 0.25).cuda()   # the locally convex regime: tangent blocks positive definite
        Z = torch.from_numpy(W.rng_for(W.SEED_BASE + 401 + n).choice([-1.0, 1.0], size=(1, n))).cuda()
        wse = torch.empty(ph.affine_normal_workspace(b, N), dtype=torch.uint8, device="cuda")
        exact = lambda: ph.affine_normal(b, X, reg=1e-8, ws=wse)  # noqa: E731
        stoch = lambda: ph.affine_normal_stochastic(b, X, Z, reg=5e-4, tol=2e-2, maxit=6)  # noqa: E731
        De, _ = ph.affine_normal(b, X, reg=1e-8, ws=wse, check=True)
        Ds, _, hv = ph.affine_normal_stochastic(b, X, Z, reg=5e-4, tol=2e-2, maxit=6, check=True)
        te, _ = time_events(exact, 3, 1)
        ts, _ = time_events(stoch, 5, 2)
        ks, _ = kernel_ms(ph.TIMING_AFFINE, stoch, 5)
        ang = _angles_deg(Ds, De)
        cross[f"n{n}"] = {"terms": int(wl.exps.shape[0]), "points": N, "exact_ms": te * 1e3,
                          "stochastic_ms": ts * 1e3, "stochastic_kernel_ms": ks, "speedup": te / ts,
                          "angle_deg_mean": float(ang.mean()), "angle_deg_max": float(ang.max()),
                          "hv_evals_mean": float(hv.double().mean())}
        del wse
    wl = W.sparse_quartic(seed=W.SEED_BASE + 450, n=6, npts=4096, m=11)
    b = ph.batch_from_numpy([0, wl.exps.shape[0]], wl.exps, wl.coefs, n=6, max_exp=4)
    X = torch.from_numpy(wl.X * 0.5).cuda()
    De, _ = ph.affine_normal(b, X, reg=1e-8, check=True)
    angs, times = [], []
    for seed in range(10):
        Z = torch.from_numpy(W.rng_for(W.SEED_BASE + 460 + seed).choice([-1.0, 1.0], size=(64, 6))).cuda()
        Ds, _, _ = ph.affine_normal_stochastic(b, X, Z, reg=1e-8, tol=1e-4, maxit=80, check=True)
        angs.append(_angles_deg(Ds, De))
        t, _ = time_events(lambda: ph.affine_normal_stochastic(b, X, Z, reg=1e-8, tol=1e-4, maxit=80), 3, 1)
        times.append(t)
    a = torch.cat(angs)
    acc = {"n": 6, "terms": int(wl.exps.shape[0]), "points": int(X.shape[0]), "probes": 64, "seeds": 10,
           "ms_per_call": 1e3 * sum(times) / len(times), "points_per_s": X.shape[0] * len(times) / sum(times),
           "angle_deg_mean": float(a.mean()), "angle_deg_std": float(a.std())}
    return {"crossover_speed_preset": cross, "accuracy_preset": acc}


def bench_mtimes(args):
    """A^2 for a 3 x 3 polynomial matrix whose entries are random degree-4
    polynomials in n=8 with 300 distinct monomials (N(0,1) coefficients):
    27 entry products, 2,430,000 raw terms."""
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    rng = W.rng_for(W.SEED_BASE + 95)
    n, d, terms, I = 8, 4, 300, 3
    ents = [W.random_poly(rng, n, d, terms, integer=False, distinct=True) for _ in range(I * I)]
    rp, E, C = W.csr_from_list(ents, n)
    a = ph.batch_from_numpy(rp, E, C, n=n, max_exp=d)
    ws_bytes, raw = ph.mtimes_workspace(a, a, I, I, I)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = ph._empty_out(n, I * I, raw, 2 * d, "cuda")
    step = lambda: ph.mtimes(a, a, I, I, I, ws=ws, out=out, finish=False)  # noqa: E731
    ph.mtimes(a, a, I, I, I, ws=ws, out=out, finish=True, trim=False)
    merged = int(out.row_ptr_host[-1])
    t, _ = time_events(step, 10, 2)
    return {"matrix": f"{I}x{I}", "n": n, "terms_per_entry": terms, "raw_terms": raw, "merged_terms_out": merged,
            "ms": t * 1e3, "raw_terms_per_s": raw / t}


def bench_paper_family(args):
    """simplify(p_d^3) for p_d = the sum of all monomials of degree <= d in
    five variables with coefficients 1 (the heavy-simplify family of
    Section 6.3, d = 2, 3, 4: 21, 56, 126 base monomials), as the two
    products p_d * p_d and (p_d^2) * p_d; the host reads the size of p_d^2
    back between them."""
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    res = {}
    for d in (2, 3, 4):
        e, c = W.all_ones_family(5, d)
        T = e.shape[0]
        p = ph.batch_from_numpy([0, T], e, c, n=5, max_exp=d)
        box = {}

        def step():
            box["r"] = ph.mul(ph.mul(p, p), p)

        t, wall = time_events(step, 20, 3)
        res[f"d{d}"] = {"base_terms": T, "terms_out": int(box["r"].row_ptr_host[-1]),
                        "raw_terms": T * T + int(ph.mul(p, p).row_ptr_host[-1]) * T,
                        "ms": t * 1e3, "wall_ms": wall * 1e3}
    torch.cuda.synchronize()
    return res


def bench_graph(args, m):
    """The times+simplify step captured once into a HIP graph and replayed."""
    import torch
    import paper_2604_06575_amd as ph
    import workloads as W

    wl = W.plain_large(terms=args.terms)
    rp = [0, args.terms]
    a = ph.batch_from_numpy(rp, wl.a_exps, wl.a_coefs, n=wl.n, max_exp=wl.max_exp)
    b = ph.batch_from_numpy(rp, wl.b_exps, wl.b_coefs, n=wl.n, max_exp=wl.max_exp)
    ws_bytes, raw = ph.mul_workspace(a, b)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    out = ph._empty_out(wl.n, 1, raw, 2 * wl.max_exp, "cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ph.mul(a, b, ws=ws, out=out, finish=False)   # warm-up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ph.mul(a, b, ws=ws, out=out, finish=False)
    t, _ = time_events(g.replay, args.steps, 1)
    return {"ms_per_step": t * 1e3, "merged_terms_per_s": raw / t}


def copy_probe():
    """A plain device copy of known size (256 MiB, three times): the
    reference against which the HBM byte counters are scaled."""
    import torch
    n = 256 * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3}))


def host_description():
    """Logical CPUs visible to this process and the CPU model (Linux)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return ncpu, model


def cpu_baseline(args):
    """The oracle's times+simplify on the host: single-threaded as it stands
    (`value`), and a threaded leg that runs it on term chunks of p in parallel
    (the C oracle releases the GIL) and simplifies the concatenated partial
    results once more (`threaded`)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    import workloads as W
    wl = W.plain_large(terms=args.terms)
    nb = min(args.cpu_terms, args.terms)
    ncpu, model = host_description()
    t0 = time.perf_counter()
    e, _ = oracle.mul(wl.a_exps, wl.a_coefs, wl.b_exps[:nb], wl.b_coefs[:nb])
    dt = time.perf_counter() - t0
    raw = args.terms * nb
    threads = max(1, min(ncpu, 16))
    chunks = [c for c in np.array_split(np.arange(args.terms), threads) if c.size]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=len(chunks)) as ex:
        parts = list(ex.map(lambda c: oracle.mul(wl.a_exps[c[0]:c[-1] + 1], wl.a_coefs[c[0]:c[-1] + 1],
                                                 wl.b_exps[:nb], wl.b_coefs[:nb]), chunks))
    et, _ = oracle.simplify(np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))
    dt_mt = time.perf_counter() - t0
    return {"value": raw / dt, "unit": "raw terms merged/s", "cores": 1, "kind": "oracle",
            "merged_terms_out_per_s": e.shape[0] / dt,
            "sample": f"times+simplify of p ({args.terms} terms) by the first {nb} terms of q: "
                      f"{raw} raw terms -> {e.shape[0]} merged, {dt:.1f} s single-threaded C oracle",
            "host": {"logical_cpus": ncpu, "cpu_model": model},
            "threaded": {"value": raw / dt_mt, "unit": "raw terms merged/s", "cores": len(chunks),
                         "sample": f"the same product as {len(chunks)} oracle calls on term chunks of p in "
                                   f"parallel threads, then one oracle simplify of their {sum(p[0].shape[0] for p in parts)} "
                                   f"concatenated terms -> {et.shape[0]} merged: {dt_mt:.1f} s"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.copy_probe:
        copy_probe()
        return
    if args.tune:
        import paper_2604_06575_amd as ph
        ph.lib()
        for kv in args.tune:
            name, value = kv.split("=", 1)
            ph.tune_set(name, int(value))
    m = bench_mul(args)
    value = m["raw"] / m["t"]
    # algorithmic bytes of the dominant kernel's average launch / its average duration
    if m["sort_path"]:
        passes, db, packed, per_term = m["plan"]
        alg_bytes = per_term * m["raw"]
        alg_note = (f"average per launch over the {passes} radix passes of {db}-bit digits: every element read "
                    f"once and written once, except that the first pass generates its elements from the operands "
                    f"(no per-term read); (key 8 B, raw index 4 B) pairs"
                    + (", packed into one 8-byte word from the first pass on (first pass writes 8 B, the others "
                       f"read and write 8 B) = {per_term:.2f} B x raw terms" if packed else
                       f" (first pass writes 12 B, the others read and write 12 B) = {per_term:.2f} B x raw terms"))
    else:
        alg_bytes = BYTES_PER_RAW_TERM * m["raw"]
        alg_note = "per launch: every raw product term as a 64-bit key and a 32-bit payload, written and read once"
    achieved = alg_bytes / (m["k_ms"] / 1e3) / 1e9
    line = {
        "metric": "merged terms/s (expand+simplify); point-evals/s split-MFMA vs FP64 at 1e-10",
        "value": value,
        "unit": "raw terms merged/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["t"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"times+simplify, n=10, degree<=8, {args.terms}x{args.terms} terms, "
                               f"N(0,1) coefficients, 5-bit fields",
                   "raw_terms": m["raw"], "merged_terms_out": m["unique"]},
        "merged_terms_out_per_s": m["unique"] / m["t"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if m["sort_path"] else None,
                     "kernel": "k_gs_scatter" if m["sort_path"] else "k_mul_buckets_lds",
                     "kernel_ms": m["k_ms"], "kernel_launches_timed": m["k_n"],
                     "algorithmic_bytes": alg_bytes,
                     "algorithmic_bytes_note": alg_note},
        "wall_ms_per_step": m["t_wall"] * 1e3,
    }
    if args.graph:
        line["graph"] = bench_graph(args, m)
    if not args.no_eval:
        line["eval"] = bench_eval(args)
    if not args.no_latency:
        line["latency_small"] = bench_latency(args)
    if not args.no_batch:
        line["batch_matrix"] = bench_batch(args)
    if not args.no_deriv:
        line["quartic_derivatives"] = bench_deriv(args)
    if not args.no_affine:
        line["affine_normal"] = bench_affine(args)
    if not args.no_mtimes:
        line["mtimes"] = bench_mtimes(args)
    if not args.no_paper:
        line["paper_family"] = bench_paper_family(args)
    if not args.no_affine and not args.no_affine_scaling:
        line["affine_scaling"] = bench_affine_scaling(args)
    if not args.no_affine and not args.no_affine_stochastic:
        line["affine_stochastic"] = bench_affine_stochastic(args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
