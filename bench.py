#!/usr/bin/env python
"""Benchmark of frPCA / frPCAt on one MI355X.

Default workload: the 1,000,000 x 200,000 power-law CSR matrix (40 distinct nonzeros per row,
Zipf(1.1) columns, lognormal(0,1) values), k = 100, s = 20, q = 5 passes, inputs resident in
HBM. One step = one frpca_run (Gaussian draw, all passes, LU and eigSVD bases, final
Rayleigh-Ritz, sign convention). Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0       # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 matrix
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix
SEED = 20181015
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_spmm_zipf_lognormal.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="zipf_lognormal")
    p.add_argument("--passes", type=int, default=0, help="override q")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true", help="skip the odd/even, BF16 and backward timings")
    p.add_argument("--gram-f32", action="store_true",
                   help="time the variant whose eigSVD Gram runs on the FP32 matrix cores (profiling runs)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a 1 GiB elementwise read+write kernel 5 times (scales the HBM byte counters)")
    return p.parse_args()


def copy_calibration():
    """A plain streaming kernel of known traffic: out = 2 * in over 1 GiB of FP32, five times.
    Its FETCH_SIZE / WRITE_SIZE counters per dispatch give the factor from counter units to bytes."""
    import torch

    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n, "dispatches": 5}}), flush=True)


def spmm_source_hash():
    import hashlib

    with open(os.path.join(ROOT, "paper_1810_06825_amd", "csrc", "k_spmm.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def slice_rows(A, m_s):
    from synth import Csr

    nz = int(A.row_ptr[m_s])
    return Csr(m_s, A.n, A.row_ptr[:m_s + 1].copy(), A.col[:nz].copy(), A.val[:nz].copy(),
               {"workload": A.meta.get("workload", "") + f"[:{m_s}]"})


def spmm_bytes(A, l, trans):
    """Compulsory bytes of one product: nonzero indices + values, 32-bit pointers, the
    input panel read once and the output panel written once (l columns of FP32)."""
    nseg, nin = (A.n, A.m) if trans else (A.m, A.n)
    return A.nnz * 8 + (nseg + 1) * 4 + nin * l * 4 + nseg * l * 4


def timed_runs(mat, k, q, s, steps, warmup, torch):
    U = torch.empty((mat.m, k), dtype=torch.float32, device=mat.device)
    S = torch.empty((k,), dtype=torch.float32, device=mat.device)
    V = torch.empty((mat.n, k), dtype=torch.float32, device=mat.device)
    for _ in range(warmup):
        mat.run(k, q, s, SEED, out=(U, S, V))
    torch.cuda.synchronize()
    mat.reset_timers()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        mat.run(k, q, s, SEED, out=(U, S, V))
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, (U, S, V)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the row-partitioned multi-GPU scheme is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1810_06825_amd import FrPCA
    from synth import WORKLOADS

    gen, kw, k, s, q = WORKLOADS[args.workload]
    if args.passes:
        q = args.passes
    l = k + s
    t0 = time.time()
    A = gen(**kw)
    log(f"generated {args.workload} {A.m}x{A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")
    # the timed handle records no per-class events (the production configuration); a second
    # handle with opts.timing gives the per-class breakdown of the same runs
    mat = FrPCA.from_csr(A, device="cuda:0", gram_f32=args.gram_f32)
    create_ms = mat.info()["create_ms"]
    log(f"create (validation + column-major mirror) {create_ms:.1f} ms")

    ms, (U, S, V) = timed_runs(mat, k, q, s, args.steps, args.warmup, torch)
    log(f"frpca_run q={q}: {ms:.3f} ms/step")
    matt = FrPCA.from_csr(A, device="cuda:0", timing=True, gram_f32=args.gram_f32)
    ms_timers, _ = timed_runs(matt, k, q, s, args.steps, args.warmup, torch)
    info = matt.info()
    log(f"with per-class events: {ms_timers:.3f} ms/step")
    per = {}
    for name in info["t_ms"]:
        c = info["t_count"][name]
        if c:
            per[name] = {"ms_total_per_step": info["t_ms"][name] / args.steps, "launches_per_step": c / args.steps,
                         "ms_per_launch": info["t_ms"][name] / c}
    log("per-class:", json.dumps({kk: round(v["ms_total_per_step"], 3) for kk, v in per.items()}))

    # dominant kernel and its roofline (algorithmic bytes / measured launch duration)
    dom = max(per, key=lambda n: per[n]["ms_total_per_step"])
    a6 = A.m >= A.n
    fwd_bytes = spmm_bytes(A, l, trans=not a6)
    back_bytes = spmm_bytes(A, l, trans=a6)
    if a6 and info["hot_cols"] > 0:
        # the back product runs as three kernels: the row-blocked hot part (index/value pairs,
        # segment pointers, Y read once, one partial row per (row block, hot column) written),
        # the tail columns (their pairs, pointers, gathered rows at most all of Y, rows out),
        # and the fixed-order combine; the "spmm_back" class is the first
        nseg = info["row_blocks"] * info["hot_cols"]
        back_bytes = info["hot_nnz"] * 8 + (nseg + 1) * 4 + A.m * l * 4 + nseg * l * 4
    roof = None
    if dom in ("spmm_fwd", "spmm_back"):
        b = fwd_bytes if dom == "spmm_fwd" else back_bytes
        ach = b / (per[dom]["ms_per_launch"] * 1e-3) / 1e9
        traffic = None
        if os.path.exists(PROFILE_TRAFFIC):
            # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter runs, valid only for
            # the SpMM source they were taken on
            with open(PROFILE_TRAFFIC) as f:
                tr = json.load(f)
            if (tr.get("kernel_source_sha256") == spmm_source_hash() and dom in tr.get("per_launch", {})
                    and tr.get("workload", "").startswith(args.workload + " ")):
                traffic = tr["per_launch"][dom]["hbm_bytes"]
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBPS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": b}
    spmm_report = {}
    for name, b in (("spmm_fwd", fwd_bytes), ("spmm_back", back_bytes)):
        if name in per:
            t = per[name]["ms_per_launch"] * 1e-3
            nseg = A.m if (name == "spmm_fwd") == a6 else A.n   # segments = rows of A for the CSR side
            gathered = A.nnz * (8 + l * 4) + nseg * l * 4
            spmm_report[name] = {"ms_per_launch": round(per[name]["ms_per_launch"], 4),
                                 "algorithmic_GBps": round(b / t / 1e9, 1),
                                 "per_nnz_gather_GBps": round(gathered / t / 1e9, 1)}
    if "spmm_combine" in per:
        c = per["spmm_combine"]
        tail = per.get("spmm_back_tail", {"ms_per_launch": 0.0})
        spmm_report["spmm_back"]["tail_ms_per_launch"] = round(tail["ms_per_launch"], 4)
        spmm_report["spmm_back"]["combine_ms_per_launch"] = round(c["ms_per_launch"], 4)
        spmm_report["spmm_back"]["hot_cols"] = info["hot_cols"]
        spmm_report["spmm_back"]["hot_nnz"] = info["hot_nnz"]
        spmm_report["spmm_back"]["row_blocks"] = info["row_blocks"]
        # the whole transpose product against its compulsory bytes (index/value pairs, CSC
        # pointers, Y read once, X written once)
        whole = per["spmm_back"]["ms_per_launch"] + tail["ms_per_launch"] + c["ms_per_launch"]
        spmm_report["spmm_back"]["product_ms"] = round(whole, 4)
        spmm_report["spmm_back"]["product_compulsory_GBps"] = round(spmm_bytes(A, l, trans=True) / (whole * 1e-3) / 1e9, 1)
    gram = None
    if "gram" in per:
        # two Gram launches per run (the short-side panel of the one inner eigSVD basis and the
        # long-side panel Z of the final step), each with its reduction. Algorithmic flops: the
        # l (l + 1) / 2 distinct entries of the symmetric product, 2 per row each. Executed: the
        # upper 16 x 16 tiles of l padded to an even tile count, as issued on the matrix cores.
        rows_total = min(A.m, A.n) + max(A.m, A.n)
        nt = -(-l // 16)
        nt += nt & 1
        t_g = per["gram"]["ms_total_per_step"] * 1e-3
        alg = rows_total * l * (l + 1) / t_g / 1e12
        exe = 2.0 * rows_total * (nt * (nt + 1) // 2) * 256 / t_g / 1e12
        peak = PEAK_FP32_MFMA_TFLOPS if args.gram_f32 else PEAK_FP64_TFLOPS
        gram = {"mfma": "fp32" if args.gram_f32 else "fp64", "ms_per_run": round(t_g * 1e3, 4),
                "algorithmic_tflops": round(alg, 2), "executed_tflops": round(exe, 2), "peak_tflops": peak,
                "frac_algorithmic": round(alg / peak, 4), "frac_executed": round(exe / peak, 4)}

    extras = {}
    if not args.no_extras:
        for qq in sorted({4, 6, q} - {q}):
            m2, _ = timed_runs(mat, k, qq, s, max(3, args.steps // 2), 1, torch)
            extras[f"ms_q{qq}"] = round(m2, 3)
            log(f"q={qq}: {m2:.3f} ms")
        # differentiated form: loss = sum(sigma) + ||U W||^2 (W: k x 8, seeded). A backward uses
        # the factors of its handle's last run: both handles run q once more first. Its time
        # comes from the handle without per-class events, the breakdown from the other.
        U, S, V = mat.run(k, q, s, SEED)
        matt.run(k, q, s, SEED)
        W = torch.from_numpy(np.random.default_rng(7).standard_normal((k, 8)).astype(np.float32)).cuda()
        dU = 2.0 * (U @ W) @ W.T
        dS = torch.ones_like(S)
        nb = max(3, args.steps // 2)
        for _ in range(2):
            mat.backward(U, S, V, dU, dS, None)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(nb):
            mat.backward(U, S, V, dU, dS, None)
        e1.record()
        torch.cuda.synchronize()
        bms = e0.elapsed_time(e1) / nb
        matt.reset_timers()
        for _ in range(nb):
            matt.backward(U, S, V, dU, dS, None)
        torch.cuda.synchronize()
        binf = matt.info()
        extras["backward_per_class_ms"] = {kk: round(binf["t_ms"][kk] / nb, 4) for kk in binf["t_ms"]
                                           if binf["t_count"][kk]}
        extras["ms_backward"] = round(bms, 3)
        extras["fwd_bwd_over_fwd"] = round((ms + bms) / ms, 3)
        log(f"backward {bms:.3f} ms, (fwd+bwd)/fwd = {(ms + bms) / ms:.3f}")
        mat_b = FrPCA.from_csr(A, device="cuda:0", panel_bf16=True)
        mb, (Ub, Sb, Vb) = timed_runs(mat_b, k, q, s, max(3, args.steps // 2), 1, torch)
        Sf = S.double().cpu().numpy()
        extras["ms_bf16_panel"] = round(mb, 3)
        extras["bf16_sigma_rel_diff_vs_fp32"] = float(np.max(np.abs(Sb.double().cpu().numpy() - Sf) / Sf))
        log(f"BF16 panels: {mb:.3f} ms, sigma rel diff vs FP32 {extras['bf16_sigma_rel_diff_vs_fp32']:.2e}")
        mat_b.close()
        # eigSVD's Gram on the FP32 matrix cores (16-row FP32 sums added in FP64): time and
        # singular-value difference against the default FP64-MFMA Gram
        ng = max(3, args.steps // 2)
        mat_g = FrPCA.from_csr(A, device="cuda:0", gram_f32=True)
        mg, (_, Sg32, _) = timed_runs(mat_g, k, q, s, ng, 1, torch)
        mat_g.close()
        mat_g = FrPCA.from_csr(A, device="cuda:0", gram_f32=True, timing=True)
        timed_runs(mat_g, k, q, s, ng, 1, torch)
        ginf = mat_g.info()
        extras["ms_gram_f32"] = round(mg, 3)
        extras["gram_f32_gram_ms"] = round(ginf["t_ms"]["gram"] / ng, 4)
        extras["gram_f32_sigma_rel_diff_vs_fp64_gram"] = float(
            np.max(np.abs(Sg32.double().cpu().numpy() - Sf) / Sf))
        log(f"FP32-MFMA Gram: {mg:.3f} ms (Gram {extras['gram_f32_gram_ms']:.3f} ms), sigma rel diff vs FP64 Gram "
            f"{extras['gram_f32_sigma_rel_diff_vs_fp64_gram']:.2e}")
        mat_g.close()
        # centred PCA (A - 1 mu^T, never formed): cost of the rank-1 terms
        mat_c = FrPCA.from_csr(A, device="cuda:0", center=True)
        mc, _ = timed_runs(mat_c, k, q, s, max(3, args.steps // 2), 1, torch)
        mat_c.close()
        mat_c = FrPCA.from_csr(A, device="cuda:0", center=True, timing=True)
        timed_runs(mat_c, k, q, s, max(3, args.steps // 2), 1, torch)
        cinf = mat_c.info()
        extras["ms_centered"] = round(mc, 3)
        extras["centered_terms_ms"] = round(cinf["t_ms"]["center"] / max(3, args.steps // 2), 4)
        log(f"centred: {mc:.3f} ms (rank-1 terms {extras['centered_terms_ms']:.3f} ms)")
        mat_c.close()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from threadpoolctl import threadpool_info

        m_s = max(A.m // 4, min(A.m, A.n + 1))
        As = slice_rows(A, m_s)
        t1 = time.perf_counter()
        Uo, So, Vo, _ = oracle.frpca(As, k, q, s, SEED)
        tcpu = time.perf_counter() - t1
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        scale = A.nnz / As.nnz
        # GPU on the same sample: error of the FP32 path against the FP64 oracle
        ms_s = FrPCA.from_csr(As, device="cuda:0")
        Ug, Sg, Vg = (t.double().cpu().numpy() for t in ms_s.run(k, q, s, SEED))
        ms_s.close()
        sig_err = float(np.max(np.abs(Sg - So) / So))
        Qo = np.linalg.qr(Vo)[0]
        sin_v = float(np.linalg.norm(Vg - Qo @ (Qo.T @ Vg), 2))
        ms_s = FrPCA.from_csr(As, device="cuda:0", gram_f32=True)
        Sg32 = ms_s.run(k, q, s, SEED)[1].double().cpu().numpy()
        ms_s.close()
        sig_err32 = float(np.max(np.abs(Sg32 - So) / So))
        cpu = {"value": round(tcpu * scale, 2), "unit": "s", "cores": int(cores), "kind": "oracle",
               "sample": f"first {m_s} of {A.m} rows ({As.nnz} nnz), same k/s/q/seed; {tcpu:.1f} s measured, "
                         f"scaled by nnz ratio {scale:.2f}",
               "gpu_vs_oracle_on_sample": {"sigma_rel_err": sig_err, "sin_theta_V": sin_v,
                                           "sigma_rel_err_gram_f32": sig_err32}}
        log(f"oracle on sample: {tcpu:.1f} s -> {tcpu * scale:.1f} s scaled; GPU sigma err {sig_err:.2e} "
            f"(FP32-MFMA Gram {sig_err32:.2e})")

    out = {
        "metric": "frPCA wall time (s) + SpMM HBM GB/s at k=100; fwd+bwd time vs fwd at stated error",
        "value": round(ms * 1e-3, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} {A.m}x{A.n} CSR, {A.nnz} nnz", "m": A.m, "n": A.n,
                   "nnz": A.nnz, "k": k, "s": s, "passes": q, "seed": SEED,
                   "gram": "fp32-mfma" if args.gram_f32 else "fp64-mfma"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "spmm": spmm_report,
        "gram": gram,
        "create_ms": round(create_ms, 2),
        "per_class_ms": {kk: round(v["ms_total_per_step"], 4) for kk, v in per.items()},
        "ms_per_step_with_class_events": round(ms_timers, 4),
        **extras,
    }
    print(json.dumps(out), flush=True)
    matt.close()
    mat.close()


if __name__ == "__main__":
    main()
