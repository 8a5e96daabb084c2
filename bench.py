#!/usr/bin/env python
"""Benchmark of frPCA / frPCAt on one MI355X.

Default workload: the Aminer-shaped CSR matrix (12,869,521 x 323,899, 20 distinct nonzeros per
row, Zipf(1.0) columns, tf-idf values; the stand-in for the 12.87M x 324K matrix of Table 4),
k = 100, s = 20, q = 5 passes, inputs resident in HBM. One step = one frpca_run (Gaussian draw,
all passes, LU and eigSVD bases, final Rayleigh-Ritz, sign convention). Beside it: q = 3 and 7
on the same matrix, the BF16-panel and FP32-Gram variants, the 1M x 200K power-law workload,
the differentiated workload (500K x 100K, k = 50, q = 4) with its forward + backward time
through the autograd function, the basic randomized algorithm (Alg. 1 / Alg. 4 with QR) against
the fast one on the paper's Table 2 and Table 4 structures, eigSVDs (Alg. 3) against both on its
Table 3 structure, and the FP64 CPU oracle on the whole headline job. Prints one
JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
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
METRIC = "frPCA wall time (s) + SpMM HBM GB/s at k=100; fwd+bwd time vs fwd at stated error"
# other pass counts timed beside the headline one, per workload
PASS_SWEEP = {"aminer_tfidf": (3, 7), "zipf_lognormal": (4, 6), "planted_blocks": (3, 7), "zipf_normal": (2, 6)}
SPMM_SOURCES = ("k_spmm.hip", "k_bcsc.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


EXTRAS = ("peaks", "passes", "variants", "basic", "zipf", "planted", "differentiated", "eigsvds")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="aminer_tfidf")
    p.add_argument("--passes", type=int, default=0, help="override q")
    p.add_argument("--cpu-baseline", choices=("full", "none"), default="full",
                   help="full: time the FP64 oracle on the whole headline job (minutes of host CPU)")
    p.add_argument("--no-cpu-baseline", action="store_true", help="same as --cpu-baseline none")
    p.add_argument("--no-extras", action="store_true",
                   help="only the headline timing (profiling runs): no pass sweep, variants or other workloads")
    p.add_argument("--extra", action="append", choices=EXTRAS, default=None,
                   help="run only the named extras (repeatable; default: all of them unless --no-extras)")
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


def measured_copy_peak(torch) -> dict:
    """Bytes moved per second by a device-to-device copy of 2 GiB (read + write), best of 10:
    the practical streaming rate of this GPU's HBM beside the nominal 8 TB/s."""
    n = 1 << 29
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    gbps = 2 * 4 * n / (best * 1e-3) / 1e9
    return {"GBps": round(gbps, 1), "frac_of_nominal": round(gbps / PEAK_HBM_GBPS, 4),
            "kernel": "torch copy_ of 2 GiB FP32 (2 GiB read + 2 GiB written), best of 10"}


def measured_gather_peak(torch, short_rows: int, long_rows: int) -> dict:
    """Random 512-byte row gathers in the sparse products' lane shape (frpca_gather_probe) from
    panels of the workload's two sides (128 FP32 columns), best of 3: the ceiling of the
    products' access pattern beside the streaming copy rate."""
    from paper_1810_06825_amd import FrPCA, binding
    from synth import random_sparse

    tiny = FrPCA.from_csr(random_sparse(64, 64, 0.2, seed=1), device="cuda:0")
    out = torch.zeros(64, dtype=torch.float32, device="cuda:0")
    rec = {"kernel": "frpca_gather_probe: random rows of 128 FP32 (512 B), float4 per lane, two rows per "
                     "wave instruction, 8 row pairs in flight per wave; best of 3"}
    for name, rows in (("short_side_panel", short_rows), ("long_side_panel", long_rows)):
        P = torch.zeros((rows, 128), dtype=torch.float32, device="cuda:0")
        gathers = 100_000_000
        binding.frpca_gather_probe(tiny.h, P, rows, 128, gathers // 10, 7, out)
        best, nr = float("inf"), 0
        for it in range(3):
            ms, nr = binding.frpca_gather_probe(tiny.h, P, rows, 128, gathers, 11 + it, out)
            best = min(best, ms)
        gbps = nr * 512 / (best * 1e-3) / 1e9
        rec[name] = {"rows": rows, "panel_MB": round(rows * 512 / 1e6, 1), "rows_read": nr,
                     "GBps": round(gbps, 1), "frac_of_nominal": round(gbps / PEAK_HBM_GBPS, 4)}
        del P
        torch.cuda.empty_cache()
    tiny.close()
    return rec


def spmm_source_hash():
    h = hashlib.sha256()
    for f in SPMM_SOURCES:
        with open(os.path.join(ROOT, "paper_1810_06825_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_spmm_{workload}.json")


def slice_rows(A, m_s):
    from synth import Csr

    nz = int(A.row_ptr[m_s])
    return Csr(m_s, A.n, A.row_ptr[:m_s + 1].copy(), A.col[:nz].copy(), A.val[:nz].copy(),
               {"workload": A.meta.get("workload", "") + f"[:{m_s}]"})


def spmm_bytes(A, l, trans):
    """Compulsory bytes of one product: nonzero indices + values, 32-bit pointers of the
    segments, the input panel read once and the output panel written once (l columns of FP32)."""
    nseg, nin = (A.n, A.m) if trans else (A.m, A.n)
    return A.nnz * 8 + (nseg + 1) * 4 + nin * l * 4 + nseg * l * 4


def class_bytes(A, l, info) -> dict:
    """Algorithmic bytes per launch of each sparse-product kernel class.

    spmm_fwd: the forward product (A Q for m >= n). spmm_back: the back product, or with
    frequent ("hot") columns its row-blocked part: their index/value pairs, the segment
    pointers, Y read once and one partial row per (row block, hot column) written.
    spmm_back_tail: the other columns: their pairs and pointers, Y read once (it touches
    nearly every row), their rows of X written."""
    a6 = A.m >= A.n
    out = {"spmm_fwd": spmm_bytes(A, l, trans=not a6), "spmm_back": spmm_bytes(A, l, trans=a6)}
    if a6 and info["hot_cols"] > 0:
        nseg = info["row_blocks"] * info["hot_cols"]
        out["spmm_back"] = info["hot_nnz"] * 8 + (nseg + 1) * 4 + A.m * l * 4 + nseg * l * 4
        tail_cols = A.n - info["hot_cols"]
        out["spmm_back_tail"] = ((A.nnz - info["hot_nnz"]) * 8 + (tail_cols + 1) * 4 + A.m * l * 4
                                 + tail_cols * l * 4)
    return out


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


def per_class(info, steps) -> dict:
    per = {}
    for name in info["t_ms"]:
        c = info["t_count"][name]
        if c:
            per[name] = {"ms_total_per_step": info["t_ms"][name] / steps, "launches_per_step": c / steps,
                         "ms_per_launch": info["t_ms"][name] / c}
    return per


def sin_theta(Ref, X):
    import numpy as np

    Q = np.linalg.qr(X)[0]
    Qr = np.linalg.qr(Ref)[0]
    return float(np.linalg.norm(Q - Qr @ (Qr.T @ Q), 2))


def free(torch, *objs):
    for o in objs:
        if hasattr(o, "close"):
            o.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def headline(args, A, k, q, s, torch, np):
    """Time frpca_run on A; per-class breakdown, roofline of the dominant kernel, Gram figures."""
    from paper_1810_06825_amd import FrPCA

    l = k + s
    mat = FrPCA.from_csr(A, device="cuda:0", gram_f32=args.gram_f32)
    create_ms = mat.info()["create_ms"]
    log(f"create (validation + column-major mirror + row-blocked order) {create_ms:.1f} ms")
    ms, (U, S, V) = timed_runs(mat, k, q, s, args.steps, args.warmup, torch)
    log(f"frpca_run q={q}: {ms:.3f} ms/step")
    # a second handle records per-class HIP events on the library's stream
    matt = FrPCA.from_csr(A, device="cuda:0", timing=True, gram_f32=args.gram_f32)
    ms_timers, _ = timed_runs(matt, k, q, s, args.steps, args.warmup, torch)
    info = matt.info()
    per = per_class(info, args.steps)
    log(f"with per-class events: {ms_timers:.3f} ms/step;",
        json.dumps({kk: round(v["ms_total_per_step"], 3) for kk, v in per.items()}))
    cb = class_bytes(A, l, info)
    spmm_report = {}
    for name, b in cb.items():
        if name in per:
            t = per[name]["ms_per_launch"] * 1e-3
            spmm_report[name] = {"ms_per_launch": round(per[name]["ms_per_launch"], 4),
                                 "algorithmic_bytes": b, "algorithmic_GBps": round(b / t / 1e9, 1),
                                 "frac_of_hbm_peak": round(b / t / 1e9 / PEAK_HBM_GBPS, 4)}
    if A.m >= A.n and "spmm_combine" in per:
        whole = sum(per.get(c, {"ms_per_launch": 0.0})["ms_per_launch"]
                    for c in ("spmm_back", "spmm_back_tail", "spmm_combine"))
        spmm_report["back_product"] = {
            "ms": round(whole, 4), "hot_cols": info["hot_cols"], "hot_nnz": info["hot_nnz"],
            "row_blocks": info["row_blocks"],
            "compulsory_GBps": round(spmm_bytes(A, l, trans=True) / (whole * 1e-3) / 1e9, 1)}
    # dominant sparse-product kernel class and its roofline: algorithmic bytes per launch over
    # the launch's average duration from the events above
    sp = [c for c in per if c in cb]
    dom = max(sp, key=lambda c: per[c]["ms_total_per_step"])
    ach = cb[dom] / (per[dom]["ms_per_launch"] * 1e-3) / 1e9
    traffic = None
    tf = traffic_file(args.workload)
    if os.path.exists(tf):
        # FETCH_SIZE / WRITE_SIZE bytes per launch, valid only for the kernel sources and the
        # workload the counters were taken on
        with open(tf) as f:
            tr = json.load(f)
        if tr.get("kernel_source_sha256") == spmm_source_hash() and dom in tr.get("per_launch", {}):
            traffic = tr["per_launch"][dom]["fetch_write_bytes"]
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBPS, 4), "traffic": traffic, "algorithmic_bytes_per_launch": cb[dom]}
    gram = None
    if "gram" in per:
        # two Gram launches per run (the short-side panel of the last inner eigSVD basis and the
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
    matt.close()
    res = {"ms": ms, "create_ms": create_ms, "per": per, "roofline": roof, "spmm": spmm_report, "gram": gram,
           "ms_timers": ms_timers, "factors": (U, S, V)}
    return mat, res


def variants(A, k, q, s, steps, torch, np, S_ref):
    """BF16 panels (every inner pass pair, all but the last one, or the long-side panel of all
    but the last one), the FP32-MFMA Gram, the final products on FP64 MFMA, the
    one-sweep pass pairs with atomic adds and the centred run on the headline matrix: time and
    singular-value difference against the default FP32 path."""
    from paper_1810_06825_amd import FrPCA

    out = {}
    Sf = S_ref.double().cpu().numpy()
    n = max(3, steps // 2)
    for name, kw in (("bf16_panel", {"panel_bf16": 1}), ("bf16_mixed", {"panel_bf16": 2}),
                     ("bf16_long", {"panel_bf16": 4}), ("gram_f32", {"gram_f32": True}),
                     ("final_f64", {"final_f64": True}), ("fused_pass", {"fused_pass": True}),
                     ("centered", {"center": True})):
        m2 = FrPCA.from_csr(A, device="cuda:0", **kw)
        t, (_, S2, _) = timed_runs(m2, k, q, s, n, 1, torch)
        m2.close()
        m2 = FrPCA.from_csr(A, device="cuda:0", timing=True, **kw)
        timed_runs(m2, k, q, s, n, 1, torch)
        inf = m2.info()
        m2.close()
        rec = {"ms": round(t, 3)}
        if name != "centered":   # the centred run computes another matrix's spectrum
            rec["sigma_rel_diff_vs_fp32"] = float(np.max(np.abs(S2.double().cpu().numpy() - Sf) / Sf))
            rec["S"] = S2.double().cpu().numpy()
        if name == "gram_f32":
            rec["gram_ms"] = round(inf["t_ms"]["gram"] / n, 4)
        if name == "fused_pass":
            rec["pass_pairs_ms"] = round(inf["t_ms"]["spmm_fwd"] / n, 4)
        if name == "centered":
            rec["rank1_terms_ms"] = round(inf["t_ms"]["center"] / n, 4)
        log(f"variant {name}: {t:.3f} ms", {kk: v for kk, v in rec.items() if kk != "S"})
        out[name] = rec
        torch.cuda.empty_cache()
    return out


def secondary_zipf(args, torch, np):
    """The 1,000,000 x 200,000 power-law workload (Zipf 1.1 columns, 40 per row, lognormal
    values), k = 100, s = 20, q = 5 (also 4 and 6)."""
    from paper_1810_06825_amd import FrPCA
    from synth import WORKLOADS

    gen, kw, k, s, q = WORKLOADS["zipf_lognormal"]
    A = gen(**kw)
    l = k + s
    mat = FrPCA.from_csr(A, device="cuda:0")
    ms, (_, S0, _) = timed_runs(mat, k, q, s, args.steps, args.warmup, torch)
    S0 = S0.double().cpu().numpy()
    rec = {"workload": f"zipf_lognormal {A.m}x{A.n} CSR, {A.nnz} nnz", "k": k, "s": s, "ms_q5": round(ms, 3)}
    for qq in (4, 6):
        t, _ = timed_runs(mat, k, qq, s, max(3, args.steps // 2), 1, torch)
        rec[f"ms_q{qq}"] = round(t, 3)
    mat.close()
    # the precision and fusion variants on this matrix: time and sigma difference against FP32
    rec["variants"] = {}
    for name, vkw in (("bf16_panel", {"panel_bf16": 1}), ("bf16_mixed", {"panel_bf16": 2}),
                      ("bf16_long", {"panel_bf16": 4}), ("fused_pass", {"fused_pass": True})):
        mv = FrPCA.from_csr(A, device="cuda:0", **vkw)
        t, (_, Sv, _) = timed_runs(mv, k, q, s, max(3, args.steps // 2), 1, torch)
        mv.close()
        Sv = Sv.double().cpu().numpy()
        rec["variants"][name] = {"ms": round(t, 3), "sigma_rel_diff_vs_fp32": float(np.max(np.abs(Sv - S0) / S0))}
    matt = FrPCA.from_csr(A, device="cuda:0", timing=True)
    timed_runs(matt, k, q, s, max(3, args.steps // 2), 1, torch)
    info = matt.info()
    per = per_class(info, max(3, args.steps // 2))
    matt.close()
    cb = class_bytes(A, l, info)
    rec["spmm_GBps"] = {c: round(cb[c] / (per[c]["ms_per_launch"] * 1e-3) / 1e9, 1) for c in cb if c in per}
    rec["per_class_ms"] = {kk: round(v["ms_total_per_step"], 4) for kk, v in per.items()}
    log("zipf_lognormal:", json.dumps(rec))
    free(torch)
    return rec


def planted_cfg(args, torch, np):
    """The planted-spectrum workload: 200,000 x 50,000 (50M nnz, 250 per row), exact
    sigma_i = 10^(-3 i / 200) on 200 disjoint blocks, k = 100, s = 20. The default path at
    q = 2, 3, 5, 7 and, at q = 5, the precision variants (BF16 panels, FP32-MFMA Gram, FP64
    final products), each with its sigma error against the exact spectrum and its difference
    from the default path."""
    from paper_1810_06825_amd import FrPCA
    from synth import WORKLOADS

    gen, kw, k, s, q0 = WORKLOADS["planted_blocks"]
    A = gen(**kw)
    exact = np.asarray(A.meta["sigma"], dtype=np.float64)[:k]

    def errs(S):
        S = S.double().cpu().numpy()
        r = np.abs(S - exact) / exact
        return S, {"sigma_rel_err_top10": float(r[:10].max()), "sigma_rel_err_top100": float(r.max())}

    rec = {"workload": f"planted_blocks {A.m}x{A.n} CSR, {A.nnz} nnz", "k": k, "s": s, "passes": {}}
    n = max(3, args.steps // 2)
    mat = FrPCA.from_csr(A, device="cuda:0")
    S5 = None
    for q in (2, 3, 5, 7):
        t, (_, S, _) = timed_runs(mat, k, q, s, n, 1, torch)
        Sq, e = errs(S)
        rec["passes"][f"q{q}"] = {"ms": round(t, 3), **e}
        if q == 5:
            S5 = Sq
    mat.close()
    rec["variants_q5"] = {}
    for name, vkw in (("bf16_panel", {"panel_bf16": 1}), ("bf16_mixed", {"panel_bf16": 2}),
                      ("bf16_long", {"panel_bf16": 4}), ("gram_f32", {"gram_f32": True}),
                      ("final_f64", {"final_f64": True})):
        mv = FrPCA.from_csr(A, device="cuda:0", **vkw)
        t, (_, S, _) = timed_runs(mv, k, 5, s, n, 1, torch)
        mv.close()
        Sv, e = errs(S)
        rec["variants_q5"][name] = {"ms": round(t, 3), **e,
                                    "sigma_rel_diff_vs_default": float(np.max(np.abs(Sv - S5) / S5))}
    log("planted_blocks:", json.dumps(rec))
    free(torch)
    return rec


def differentiated(args, torch, np):
    """The differentiated workload: 500,000 x 100,000, 30 per row, Zipf 1.1, N(0,1) values,
    k = 50, s = 10, q = 4, loss = sum(sigma) + ||U W||^2 (W 50 x 8, seed 7). Forward alone
    (frpca_run) against forward + loss + backward through the autograd function, with the
    forward's error against the FP64 oracle and the gradient's against its closed form (the
    second loss term is invariant, so dL/dA = sum_i u_i v_i^T at the stored nonzeros)."""
    import oracle
    from paper_1810_06825_amd import FrPCA, frpca_autograd
    from synth import WORKLOADS

    gen, kw, k, s, q = WORKLOADS["zipf_normal"]
    A = gen(**kw)
    mat = FrPCA.from_csr(A, device="cuda:0")
    nrep = max(3, args.steps)
    ms_f, (U, S, V) = timed_runs(mat, k, q, s, nrep, 2, torch)
    vals = torch.from_numpy(A.val).to("cuda:0")
    W = torch.from_numpy(np.random.default_rng(7).standard_normal((k, 8)).astype(np.float32)).to("cuda:0")

    def step():
        v = vals.detach().requires_grad_(True)
        U_, S_, V_ = frpca_autograd(v, mat, k, q, s, SEED)
        loss = S_.sum() + ((U_ @ W) ** 2).sum()
        loss.backward()
        return U_, S_, V_, v.grad

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(nrep):
        Ua, Sa, Va, g = step()
    e1.record()
    torch.cuda.synchronize()
    ms_fb = e0.elapsed_time(e1) / nrep
    # backward alone, by kernel class, on a handle with events
    matt = FrPCA.from_csr(A, device="cuda:0", timing=True)
    matt.run(k, q, s, SEED)
    dU = 2.0 * (Ua @ W) @ W.T
    matt.reset_timers()
    for _ in range(nrep):
        matt.backward(dU, torch.ones_like(Sa), None)
    torch.cuda.synchronize()
    binf = matt.info()
    matt.close()
    Ug, Sg, Vg, gg = (t.detach().double().cpu().numpy() for t in (Ua, Sa, Va, g))
    mat.close()
    log("differentiated: oracle forward (FP64, CPU)")
    Uo, So, Vo, _ = oracle.frpca(A, k + 1, q, s - 1, SEED)
    sig_err = float(np.max(np.abs(Sg - So[:k]) / So[:k]))
    sin_v = sin_theta(Vo[:, :k], Vg)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    ref = np.empty(A.nnz)
    for e0_ in range(0, A.nnz, 1 << 21):
        e1_ = min(A.nnz, e0_ + (1 << 21))
        ref[e0_:e1_] = np.einsum("ij,ij->i", Ug[rows[e0_:e1_]], Vg[A.col[e0_:e1_]])
    grad_err = float(np.abs(gg - ref).max() / np.abs(ref).max())
    rec = {"workload": f"zipf_normal {A.m}x{A.n} CSR, {A.nnz} nnz", "k": k, "s": s, "passes": q,
           "loss": "sum(sigma) + ||U W||^2, W 50x8 N(0,1) seed 7",
           "ms_forward": round(ms_f, 3), "ms_forward_backward": round(ms_fb, 3),
           "fwd_bwd_over_fwd": round(ms_fb / ms_f, 3),
           "backward_per_class_ms": {kk: round(binf["t_ms"][kk] / nrep, 4) for kk in binf["t_ms"]
                                     if binf["t_count"][kk]},
           "error": {"sigma_rel_err_vs_oracle": sig_err, "sin_theta_V_vs_oracle": sin_v,
                     "grad_rel_err_vs_closed_form": grad_err}}
    log("differentiated:", json.dumps(rec))
    free(torch)
    return rec


def time_call(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        out = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, out


def basic_vs_fast(torch, np, head_mat=None, head_A=None):
    """The paper's speedup of the fast algorithm over the basic one (Sp1), measured on this GPU.

    Table 2 structure: the ratings stand-in for Matrix 2 (90,230 x 45,115, 24 per row), k = 100,
    s = 5, Alg. 1 with p = floor((q - 1) / 2) power steps against Alg. 6 with q = 2, 4, 6, 9, 11
    passes. Table 4 structure on the headline matrix: Alg. 1 with p = 5 against Alg. 6 with
    q = 12 (k = 100, s = 5). Each line gives both times, Sp1 and the relative difference of
    the singular values (zero in exact arithmetic for even q by Theorems 1 and 2 when the
    basic algorithm is Alg. 4; Alg. 1 sketches the other side)."""
    from paper_1810_06825_amd import FrPCA
    from synth import ratings_zipf

    A = ratings_zipf()
    k, s = 100, 5
    mat = FrPCA.from_csr(A, device="cuda:0")
    rows = []
    for q in (2, 4, 6, 9, 11):
        p = (q - 1) // 2
        tb, (_, Sb, _) = time_call(lambda: mat.run_basic(k, p, s, SEED, 1), 5, torch)
        tf, (_, Sf, _) = time_call(lambda: mat.run(k, q, s, SEED), 5, torch)
        t4, (_, S4, _) = time_call(lambda: mat.run_basic(k, p, s, SEED, 4), 5, torch)
        Sb, Sf, S4 = (x.double().cpu().numpy() for x in (Sb, Sf, S4))
        rows.append({"q": q, "p": p, "ms_alg1": round(tb, 3), "ms_alg4": round(t4, 3), "ms_alg6": round(tf, 3),
                     "sp1_alg1_over_alg6": round(tb / tf, 2), "sp1_alg4_over_alg6": round(t4 / tf, 2),
                     "sigma_rel_diff_alg4_vs_alg6": float(np.max(np.abs(S4 - Sf) / Sf))})
        log(f"basic vs fast q={q}:", rows[-1])
    mat.close()
    out = {"workload": f"ratings_zipf {A.m}x{A.n} CSR, {A.nnz} nnz", "k": k, "s": s, "table2": rows}
    if head_mat is not None:
        tb, _ = time_call(lambda: head_mat.run_basic(k, 5, s, SEED, 1), 2, torch)
        tf, _ = time_call(lambda: head_mat.run(k, 12, s, SEED), 2, torch)
        out["table4"] = {"workload": f"{head_A.meta.get('workload')} {head_A.m}x{head_A.n}", "k": k, "s": s,
                         "ms_alg1_p5": round(tb, 3), "ms_alg6_q12": round(tf, 3), "sp1": round(tb / tf, 2)}
        log("basic vs fast, headline matrix:", out["table4"])
    free(torch)
    return out


def eigsvds_vs_fast(torch, np):
    """Table 3 structure (the paper's Matrix 7: a 647,989 x 107,966 slice of the Aminer matrix
    with a few nonzeros per row): eigSVDs (Alg. 3, k = 100, block of 128, converged to
    ||B w - theta w|| <= 1e-6 theta_max) against Alg. 6 (q = 11) and Alg. 1 (p = 5), s = 5 for
    the randomized ones as in the paper; times, eigSVDs' iterations and the singular-value
    differences between the three."""
    from paper_1810_06825_amd import FrPCA
    from synth import aminer_tfidf

    A = aminer_tfidf(m=647_989, n=107_966, t=4, seed=1007)
    mat = FrPCA.from_csr(A, device="cuda:0")
    k = 100
    te, (_, Se, _, it) = time_call(lambda: mat.eigsvds(k, 28, SEED), 2, torch)
    tf, (_, Sf, _) = time_call(lambda: mat.run(k, 11, 5, SEED), 3, torch)
    tb, (_, Sb, _) = time_call(lambda: mat.run_basic(k, 5, 5, SEED, 1), 3, torch)
    _, Se, Ve, _ = mat.eigsvds(k, 28, SEED)
    _, Sf, Vf = mat.run(k, 11, 5, SEED)
    Se, Sf, Sb = (x.double().cpu().numpy() for x in (Se, Sf, Sb))
    Ve, Vf = Ve.double().cpu().numpy(), Vf.double().cpu().numpy()
    mat.close()
    free(torch)
    # how well each result solves A^T A v = sigma^2 v (FP64 on the host, relative to sigma_1^2)
    Asp = A.to_scipy()

    def resid(S, V):
        R = Asp.T @ (Asp @ V) - V * S ** 2
        return float(np.max(np.linalg.norm(R, axis=0)) / S[0] ** 2)

    out = {"workload": f"aminer_tfidf {A.m}x{A.n} CSR, {A.nnz} nnz (seed 1007)", "k": k,
           "ms_eigsvds": round(te, 3), "eigsvds_iterations": it, "ms_alg6_q11": round(tf, 3),
           "ms_alg1_p5": round(tb, 3), "sigma_rel_diff_alg6_vs_eigsvds": float(np.max(np.abs(Sf - Se) / Se)),
           "sigma_rel_diff_alg1_vs_eigsvds": float(np.max(np.abs(Sb - Se) / Se)),
           "max_residual_eigsvds": resid(Se, Ve), "max_residual_alg6_q11": resid(Sf, Vf)}
    log("eigSVDs vs fast:", out)
    return out


def cpu_baseline_full(A, k, q, s, factors, np):
    """The FP64 oracle on the whole headline job, timed on the host, and the GPU's error
    against it (singular values, and the subspace of V)."""
    import oracle
    from threadpoolctl import threadpool_info

    t0 = time.time()
    Uo, So, Vo, _ = oracle.frpca(A, k + 1, q, s - 1, SEED,
                                 log=lambda msg: log(f"  oracle {msg} ({time.time() - t0:.0f} s)"))
    tcpu = time.time() - t0
    cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    _, S, V = factors
    Sg = S.double().cpu().numpy()
    Vg = V.double().cpu().numpy()
    sig_err = float(np.max(np.abs(Sg - So[:k]) / So[:k]))
    sin_v = sin_theta(Vo[:, :k], Vg)
    try:
        import psutil

        mem_gb = round(psutil.virtual_memory().total / 2 ** 30, 1)
    except Exception:
        mem_gb = None
    log(f"oracle on the whole job: {tcpu:.1f} s; GPU sigma err {sig_err:.2e}, sin theta V {sin_v:.2e}")
    return ({"value": round(tcpu, 2), "unit": "s", "cores": int(cores), "kind": "oracle",
             "sample": (f"the whole job: {A.m}x{A.n}, {A.nnz} nnz, k={k}, s={s}, q={q}, seed {SEED}, one run "
                        f"(FP64 numpy/scipy; dense steps on {cores} BLAS threads, scipy's sparse products on one "
                        f"thread; host memory {mem_gb} GiB)"),
             "gpu_vs_oracle": {"sigma_rel_err": sig_err, "sin_theta_V": sin_v}}, So[:k])


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the row-partitioned multi-GPU scheme is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.no_cpu_baseline:
        args.cpu_baseline = "none"
    import numpy as np
    import torch

    from synth import WORKLOADS

    gen, kw, k, s, q = WORKLOADS[args.workload]
    if args.passes:
        q = args.passes
    def want(name):
        return not args.no_extras and (args.extra is None or name in args.extra)

    copy_peak = measured_copy_peak(torch) if want("peaks") else None
    if copy_peak:
        log("device copy:", copy_peak)
    t0 = time.time()
    A = gen(**kw)
    log(f"generated {args.workload} {A.m}x{A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")
    gather_peak = measured_gather_peak(torch, min(A.m, A.n), max(A.m, A.n)) if want("peaks") else None
    if gather_peak:
        log("random row gathers:", gather_peak)
    mat, h = headline(args, A, k, q, s, torch, np)
    ms = h["ms"]
    extras = {}
    var = {}
    basic = None
    if want("passes"):
        for qq in PASS_SWEEP.get(args.workload, ()):
            t, _ = timed_runs(mat, k, qq, s, max(3, args.steps // 2), 1, torch)
            extras[f"ms_q{qq}"] = round(t, 3)
            log(f"q={qq}: {t:.3f} ms")
    if want("variants"):
        var = variants(A, k, q, s, args.steps, torch, np, h["factors"][1])
    if want("basic"):
        basic = basic_vs_fast(torch, np, mat, A)
    U, S, V = (t.detach() for t in h["factors"])
    S_host, V_host = S.cpu(), V.cpu()
    mat.close()
    del U, S, V, h["factors"]
    free(torch)
    secondary = diff = eigs = planted = None
    if want("zipf"):
        secondary = secondary_zipf(args, torch, np)
    if want("planted"):
        planted = planted_cfg(args, torch, np)
    if want("differentiated"):
        diff = differentiated(args, torch, np)
    if want("eigsvds"):
        eigs = eigsvds_vs_fast(torch, np)
    cpu = None
    So = None
    if args.cpu_baseline == "full":
        cpu, So = cpu_baseline_full(A, k, q, s, (None, S_host, V_host), np)
    for name, rec in var.items():
        S2 = rec.pop("S", None)
        if S2 is not None and So is not None:
            rec["sigma_rel_err_vs_oracle"] = float(np.max(np.abs(S2 - So) / So))

    out = {
        "metric": METRIC,
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
        "roofline": h["roofline"],
        "cpu_baseline": cpu,
        "spmm": h["spmm"],
        "gram": h["gram"],
        "hbm_copy_measured": copy_peak,
        "row_gather_measured": gather_peak,
        "create_ms": round(h["create_ms"], 2),
        "per_class_ms": {kk: round(v["ms_total_per_step"], 4) for kk, v in h["per"].items()},
        "ms_per_step_with_class_events": round(h["ms_timers"], 4),
        **extras,
        "variants": var or None,
        "zipf_lognormal": secondary,
        "planted_blocks": planted,
        "differentiated": diff,
        "basic_vs_fast": basic,
        "eigsvds_vs_fast": eigs,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
