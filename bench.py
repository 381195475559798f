#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload: the 1700 x 350 grid with three parameter fields (n = 1,785,000), k = 200
BFGS pairs of the seeded synthetic quadratic (seed 1), bfloat16 storage of S, Y
and probe blocks.  One step is one pass of the whole path:
  1. out = B_k V for a block of 220 probe columns          (bfgs_apply_Hinv)
  2. single-pass randomized SVD of B_k - B_0, rank 200, oversampling 20
                                                           (bfgs_rsvd, Alg. 3)
  3. posterior variance diag(V Lambda V^T + B_0)           (bfgs_posterior_diag)
Inputs are resident in HBM before the timed region.  `value` is B_k V columns
per second from HIP events around step 1; `rsvd_ms` is the mean wall time of
step 2; `ms_per_step` is the whole step.

Prints one JSON line on stdout; progress goes to stderr.
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

HBM_PEAK = 8.0e12          # bytes/s
BF16_PEAK = 2.5e15         # dense MFMA flop/s
FP32_PEAK = 157.3e12
FP64_PEAK = 78.6e12        # vector and matrix
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_models(n, k, c, rank, wb, vb, ob):
    """Algorithmic bytes and flops per launch of each kernel group: GEMM1 reads S, Y
    (2 n k words), the block and h0; GEMM2 reads S, Y, the block (B_k V only: the h0 V
    term) and h0, and writes the output; the rSVD groups are listed with their inputs
    and outputs read and written once.  The TSQR passes count the usual Householder
    flops for n >> c: 2 n c^2 to factor and 4 n c^2 to form the thin Q explicitly
    (4/3 c^2 (3n - c) in full)."""
    pass_bytes = 2 * n * k * wb
    return {
        "apply_gemm1": dict(bound="hbm", bytes=pass_bytes + n * c * vb + 4 * n, flops=2 * n * 2 * k * c),
        "apply_gemm2": dict(bound="hbm", bytes=pass_bytes + n * c * vb + n * c * ob + 4 * n,
                            flops=2 * n * 2 * k * c),
        "hdiff_gemm1": dict(bound="hbm", bytes=pass_bytes + n * c * vb + 4 * n, flops=2 * n * 2 * k * c),
        "hdiff_gemm2": dict(bound="hbm", bytes=pass_bytes + n * c * ob + 4 * n, flops=2 * n * 2 * k * c),
        "tsqr_leaf_fwd": dict(bound="alu", bytes=n * c * ob + n * c * 8, flops=2 * n * c * c),
        "tsqr_leaf_bwd": dict(bound="alu", bytes=n * c * 8 + n * c * ob, flops=4 * n * c * c),
        "proj_QtX": dict(bound="hbm", bytes=n * c * (ob + vb), flops=2 * n * c * c),
        "basis_diag": dict(bound="hbm", bytes=n * c * ob + 2 * n * rank * ob + 8 * n, flops=2 * n * c * rank),
        "probes": dict(bound="hbm", bytes=n * c * vb, flops=0),
    }


def roofline_entry(name, model, avg_s, traffic):
    if model["bound"] == "hbm":
        achieved = model["bytes"] / avg_s / 1e9
        peak = HBM_PEAK / 1e9
        unit = "GB/s"
    else:
        achieved = model["flops"] / avg_s / 1e12
        peak = FP64_PEAK / 1e12
        unit = "TFLOP/s"
    return {"kernel": name, "bound": model["bound"], "achieved": round(achieved, 3), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 4), "traffic": traffic,
            "avg_ms": round(avg_s * 1e3, 4)}


def load_traffic(kernel, digest):
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except Exception:
        return None
    entry = t.get(kernel)
    if not entry or entry.get("source_digest") != digest:
        return None
    return entry.get("hbm_bytes_per_launch")


def cpu_baseline(H, V, out, wq_prob_n, storage, ncols, budget_s=15.0):
    """Oracle (eq. (3) recursion, float64 C/OpenMP) on a bounded sample of the same
    workload: whole chunks of `threads` probe columns until about `budget_s` seconds
    of oracle time (or all columns).  Also returns the relative error of the GPU's
    H_k V on those columns against the oracle (both from the stored values)."""
    import numpy as np
    from oracle import recursion
    threads = len(os.sched_getaffinity(0))
    k = H.k
    n = wq_prob_n
    S = np.empty((k, n))
    Y = np.empty((k, n))
    for j in range(k):
        s, y = H.get_pair(j)          # exact upcast of the stored values
        S[j] = s.double().cpu().numpy()
        Y[j] = y.double().cpu().numpy()
    h0 = H.get_h0().double().cpu().numpy()
    chunk = max(1, min(threads, ncols))
    done, spent = 0, 0.0
    num = den = 0.0
    elem_max = 0.0
    while done < ncols and (done == 0 or spent < budget_s):
        cols = list(range(done, min(ncols, done + chunk)))
        Vs = V[cols].double().cpu().numpy()
        t0 = time.perf_counter()
        ref = recursion.apply_hk(h0, S, Y, Vs, nthreads=threads)
        spent += time.perf_counter() - t0
        got = out[cols].double().cpu().numpy()
        num += float(((got - ref) ** 2).sum())
        den += float((ref ** 2).sum())
        elem_max = max(elem_max, float((np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)).max()))
        done += len(cols)
        log(f"[bench] oracle: {done} columns in {spent:.1f} s")
    used = min(threads, recursion.max_threads(), chunk)
    rel = (num / den) ** 0.5 if den > 0 else None
    return {"value": round(done / spent, 4), "unit": "columns/s", "cores": used, "kind": "oracle",
            "sample": f"{done} of the {ncols} probe columns of the same workload (n={n}, k={k}), "
                      f"float64 eq. (3) recursion over the stored pairs, {spent:.1f} s"}, \
        {"apply_rel_F": rel, "apply_elem_max": elem_max}, (S, Y, h0)


def oracle_rsvd_errors(S, Y, h0, storage, seed, rank, p, Sig, dg):
    """The rSVD of the timed step against the float64 oracle (Alg. 3 on the same
    stored pairs and probes): max |Sigma - Sigma_ref| / |Sigma_ref,0| and the
    posterior variance's relative Frobenius and element-wise errors."""
    import numpy as np
    from oracle import rsvd as orsvd, probes as oprobes
    t0 = time.perf_counter()
    n = h0.shape[0]
    X = oprobes.round_to(oprobes.normal_block(n, rank + p, seed), storage)
    ref = orsvd.rsvd(h0, S, Y, X, rank)
    del X
    dref = orsvd.posterior_diag(h0, ref["U"], ref["Sigma"])
    sig = Sig.cpu().numpy()
    d = dg.double().cpu().numpy()
    # the spectra compared as sets (sorted by signed value): near-ties in |lambda| of
    # opposite sign may be ordered either way
    out = {"sigma_rel_err": float(np.abs(np.sort(sig) - np.sort(ref["Sigma"])).max() / abs(ref["Sigma"][0])),
           "diag_rel_F": float(np.linalg.norm(d - dref) / np.linalg.norm(dref)),
           "diag_elem_max": float(np.abs(d - dref).max() / np.abs(dref).max()),
           "oracle_rsvd_s": round(time.perf_counter() - t0, 1)}
    log(f"[bench] oracle rSVD: {out}")
    return out


def fp32_library_apply(S, Y, V, ref, apply_ms_bf16):
    """A float32-arithmetic baseline of the same apply from the vendor library: the
    compact form's two tall products in float32 GEMMs (hipBLASLt through torch, no
    reduced-precision modes), the small solve in float64 with the inverse of R formed
    once outside the timed region (as the library keeps it from push time).  Timed on
    the same stored pairs and probes; its result is compared with the float32 form of
    this library (float64 arithmetic)."""
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    St, Yt, Vt = S.float(), Y.float(), V.float()          # (k, n), (k, n), (c, n)
    k = St.shape[0]
    gamma = float((St[0].double() @ Yt[0].double()) / (Yt[0].double() @ Yt[0].double()))
    gamma = float(torch.tensor(gamma, dtype=torch.float32))
    Sd, Yd = St.double(), Yt.double()
    SY = Sd @ Yd.T
    R = torch.triu(SY)
    Rinv = torch.linalg.solve_triangular(R, torch.eye(k, dtype=torch.float64, device=R.device), upper=True)
    M = torch.diag(torch.diagonal(SY)) + gamma * (Yd @ Yd.T)
    del Sd, Yd

    def apply():
        Zs = (St @ Vt.T).double()                        # (k, c)
        Zy = gamma * (Yt @ Vt.T).double()
        P = Rinv @ Zs
        T = Rinv.T @ (M @ P - Zy)
        # out^T = gamma (V - Y^T P)^T + (S^T T)^T, as (c, n)
        o = torch.addmm(Vt, P.float().T, Yt, beta=1.0, alpha=-1.0)
        o.mul_(gamma)
        o.addmm_(T.float().T, St)
        return o

    o = apply()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        o = apply()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    err = float(torch.linalg.vector_norm((o - ref).double()) / torch.linalg.vector_norm(ref.double()))
    elem = float(((o - ref).abs().amax(dim=1) / ref.abs().amax(dim=1)).max())
    del o
    torch.cuda.empty_cache()
    return {"apply_ms": round(ms, 4), "speedup_bf16_over_fp32_arith": round(ms / apply_ms_bf16, 3),
            "rel_F_vs_float32_form": err, "elem_max_vs_float32_form": elem}


def fp32_path(P, S, Y, n, k, V, out, rank, p, seed, Sig, dg, ncols, apply_ms_bf16):
    """The plain float32 form on the same pairs and probe values: its apply time (the
    speedup baseline of the bfloat16 form) and the bfloat16 results against it."""
    import torch
    Hf = P.Bfgs(n, k, None, "f32")
    for s_, y_ in zip(S, Y):
        Hf.push_pair(s_.float(), y_.float())
    Vf = V.float()                          # the bfloat16 probe values, exact in float32
    of = torch.empty((ncols, n), dtype=torch.float32, device="cuda")
    Hf.apply_Hinv(Vf, of)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        Hf.apply_Hinv(Vf, of)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    Uf = torch.empty((rank, n), dtype=torch.float32, device="cuda")
    Sf = torch.empty(rank, dtype=torch.float64, device="cuda")
    Hf.rsvd(rank, p, seed, Uf, Sf)
    df = Hf.posterior_diag()
    torch.cuda.synchronize()
    status = Hf.get_status()
    Hf.close()

    def rel(a, b):
        return float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))
    lib = fp32_library_apply(S, Y, V, of, apply_ms_bf16)
    res = {"apply_ms": round(ms, 4), "columns_per_s": round(ncols / (ms / 1e3), 2),
           "arithmetic": "float32 storage, float64 matrix-core arithmetic",
           "speedup_bf16_over_fp32": round(ms / apply_ms_bf16, 3),
           "fp32_arithmetic_library": lib,
           "bf16_apply_rel_F_vs_fp32": rel(out, of),
           "bf16_sigma_rel_err_vs_fp32": float((torch.sort(Sig).values - torch.sort(Sf).values).abs().max()
                                               / Sf[0].abs()),
           "bf16_diag_rel_F_vs_fp32": rel(dg, df), "device_status": status}
    log(f"[bench] fp32 path: {res}")
    return res


def bench_batch(args):
    """64-problem batch: plain float32 per-problem launches on one stream; the float32
    batch (persistent work-queue passes, the same arithmetic as the per-problem
    launches); the bfloat16 batch (forked streams, autotuned, replayed from one
    captured hipGraph)."""
    import torch
    import paper_2009_12663_amd as P
    from workloads import quadratic as wq

    shapes = wq.batch_shapes()
    p = 10
    t0 = time.perf_counter()
    pairs = []
    for sh in shapes:
        prob = wq.make_grid(sh["nx"], sh["nz"], sh["seed"], device="cuda")
        S, Y, _ = wq.cg_pairs(prob, sh["k"], rel_tol=1e-13)
        pairs.append((S.float(), Y.float()))
    ns = [sh["n"] for sh in shapes]
    ks = [S.shape[0] for S, _ in pairs]
    cs = [k + p for k in ks]
    log(f"[bench-batch] 64 problems, sum n = {sum(ns)}, k {min(ks)}..{max(ks)}, pairs in {time.perf_counter() - t0:.1f}s")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # plain float32, one problem after another on one stream
    plain = []
    for (S, Y), n, k in zip(pairs, ns, ks):
        H = P.Bfgs(n, k, None, "f32")
        for s, y in zip(S, Y):
            H.push_pair(s, y)
        plain.append(H)
    Vp = [H.generate_probes(2 + i, c) for i, (H, c) in enumerate(zip(plain, cs))]
    outp = [torch.empty(v.shape, dtype=torch.float32, device="cuda") for v in Vp]
    Up = [torch.empty((k, n), dtype=torch.float32, device="cuda") for k, n in zip(ks, ns)]
    Sp = [torch.empty(k, dtype=torch.float64, device="cuda") for k in ks]

    def plain_apply():
        for H, v, o in zip(plain, Vp, outp):
            H.apply_Hinv(v, o)

    def plain_rsvd():
        for i, (H, k, u, sg) in enumerate(zip(plain, ks, Up, Sp)):
            H.rsvd(k, p, 7 + i, u, sg)

    t_plain_apply = timed(plain_apply, args.steps)
    t_plain_rsvd = timed(plain_rsvd, 1)
    log(f"[bench-batch] plain f32: apply {t_plain_apply:.2f} ms, rsvd {t_plain_rsvd:.2f} ms")
    for H in plain:
        H.close()
    del plain, Vp, outp, Up, Sp

    # float32 batch: the persistent passes take (problem, tile) items from a work queue
    B32 = P.BfgsBatch(ns, ks, None, "f32")
    B32.push_pairs([S for S, _ in pairs], [Y for _, Y in pairs])
    V32 = [B32.problems[i].generate_probes(2 + i, c) for i, c in enumerate(cs)]
    out32 = [torch.empty(v.shape, dtype=torch.float32, device="cuda") for v in V32]
    t_p32 = timed(lambda: B32.apply_Hinv(V32, out32), args.steps)
    B32.autotune(V32)
    t_p32_tuned = timed(lambda: B32.apply_Hinv(V32, out32), args.steps)
    log(f"[bench-batch] f32 persistent batch: apply {t_p32:.2f} ms, after tuning the grid {t_p32_tuned:.2f} ms")
    B32.close()
    del V32, out32

    B = P.BfgsBatch(ns, ks, None, "bf16")
    for (S, Y), H in zip(pairs, B.problems):
        for s, y in zip(S, Y):
            H.push_pair(s, y)
    del pairs
    V = [B.problems[i].generate_probes(2 + i, c) for i, c in enumerate(cs)]
    out = [torch.empty(v.shape, dtype=torch.float32, device="cuda") for v in V]
    U = [torch.empty((k, n), dtype=torch.float32, device="cuda") for k, n in zip(ks, ns)]
    Sg = [torch.empty(k, dtype=torch.float64, device="cuda") for k in ks]
    B.autotune(V, ks, p)
    t_batch_apply = timed(lambda: B.apply_Hinv(V, out), args.steps)
    t_batch_rsvd = timed(lambda: B.rsvd(ks, p, 7, U, Sg), 1)
    B.graph_build(V, out, ks, p, 7, U, Sg)
    t_graph = timed(B.graph_launch, max(1, args.steps // 2))
    B.close()
    cols = sum(cs)
    res = {
        "metric": "batched B_k V columns/s + rSVD wall time, 64 problems (n 5e4..1e6, k 20..150)",
        "value": round(cols / (t_batch_apply / 1e3), 2), "unit": "columns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(t_graph, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "64-problem batch, rank k + 10", "sum_n": sum(ns), "sum_cols": cols},
        "batch_apply_ms": round(t_batch_apply, 4), "batch_rsvd_ms": round(t_batch_rsvd, 4),
        "graph_apply_plus_rsvd_ms": round(t_graph, 4),
        "plain_f32_apply_ms": round(t_plain_apply, 4), "plain_f32_rsvd_ms": round(t_plain_rsvd, 4),
        "f32_persistent_apply_ms": round(min(t_p32, t_p32_tuned), 4),
        "speedup_f32_persistent_over_plain_f32": round(t_plain_apply / min(t_p32, t_p32_tuned), 3),
        "speedup_apply": round(t_plain_apply / t_batch_apply, 3),
        "speedup_apply_plus_rsvd": round((t_plain_apply + t_plain_rsvd) / t_graph, 3),
    }
    print(json.dumps(res), flush=True)


def bench_streamed(args):
    """Out-of-core history: the 1700 x 350 x 3 grid with k = 50 float32 pairs kept in
    pinned host memory (bfgs_create_streamed, row slices of --slice-rows), against the
    same pairs in device memory.  Reports the apply time of 220 columns, the bytes the
    two passes stage over the host link and the rate they reach."""
    import torch
    import paper_2009_12663_amd as P
    from workloads import quadratic as wq

    k, c = 50, args.ncols
    prob = wq.make_problem("grid3", device="cuda")
    S, Y, _ = wq.cg_pairs(prob, k)
    n = prob.n
    k = S.shape[0]
    del prob

    def build(slice_rows):
        H = P.Bfgs(n, k, None, "f32", slice_rows=slice_rows)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_, y_ in zip(S, Y):
            H.push_pair(s_.float(), y_.float())
        torch.cuda.synchronize()
        return H, (time.perf_counter() - t0) * 1e3

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    Hs, push_ms = build(args.slice_rows)
    Hd, push_dev_ms = build(None)
    V = Hd.generate_probes(seed=2, ncols=c)
    out_s = torch.empty((c, n), dtype=torch.float32, device="cuda")
    out_d = torch.empty_like(out_s)
    t_s = timed(lambda: Hs.apply_Hinv(V, out_s), max(1, args.steps // 4))
    t_d = timed(lambda: Hd.apply_Hinv(V, out_d), args.steps)
    diff = float(((out_s - out_d).abs().amax(dim=1) / out_d.abs().amax(dim=1)).max())
    staged = 2 * 2 * n * k * 4
    res = {"metric": "streamed B_k V: host-link rate of the staged pair slices", "value": round(staged / t_s / 1e6, 2),
           "unit": "GB/s", "n_gpus": 1, "steps": max(1, args.steps // 4), "higher_is_better": True,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"grid3: n={n}, k={k} float32 pairs in pinned host memory, {c} columns",
                      "slice_rows": args.slice_rows},
           "streamed_apply_ms": round(t_s, 3), "device_resident_apply_ms": round(t_d, 3),
           "staged_bytes_per_apply": staged, "push_all_ms": round(push_ms, 1),
           "push_all_device_resident_ms": round(push_dev_ms, 1), "max_col_rel_diff_vs_device": diff,
           "status": [Hs.get_status(), Hd.get_status()]}
    Hs.close()
    Hd.close()
    print(json.dumps(res), flush=True)


def bench_sweep(args):
    """The 1700 x 350 x 3 grid (k = 200) with bfloat16 and float32 storage side by side:
    apply columns/s and HBM fraction over probe widths c, the bfloat16 path's relative
    error against the float32 path on the same probe values, rSVD time of both (rank
    200 + 20) with the bfloat16 Sigma and posterior variance against float32, and the
    measured stream ceilings (device copy and fill) next to the 8 TB/s peak."""
    import torch
    import paper_2009_12663_amd as P
    from workloads import quadratic as wq

    cfg = wq.CONFIGS["grid3"]
    k, rank, p = cfg["k"], cfg["rank"], cfg["oversample"]
    prob = wq.make_problem("grid3", device="cuda")
    S, Y, _ = wq.cg_pairs(prob, k)
    n = prob.n
    hs = {}
    for st in ("bf16", "f32"):
        H = P.Bfgs(n, k, None, st)
        for s_, y_ in zip(S, Y):
            H.push_pair(s_.float(), y_.float())
        hs[st] = H
    del S, Y
    torch.cuda.synchronize()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def rel(a, b):
        return float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))

    widths = [1, 8, 32, 64, 128, 220, 256]
    sweep = []
    for c in widths:
        v32 = hs["f32"].generate_probes(seed=2, ncols=c)
        vb = v32.to(torch.bfloat16)
        vf = vb.float()                                   # the same probe values for both paths
        row = {"c": c}
        outs = {}
        for st, v in (("bf16", vb), ("f32", vf)):
            out = torch.empty((c, n), dtype=torch.float32, device="cuda")
            ms = timed(lambda: hs[st].apply_Hinv(v, out), max(3, args.steps))
            wbytes = 2 if st == "bf16" else 4
            bytes_ = 2 * 2 * n * k * wbytes + n * c * (2 * wbytes + 4) + 8 * n
            row[st] = {"ms": round(ms, 4), "columns_per_s": round(c / (ms / 1e3), 1),
                       "hbm_frac": round(bytes_ / (ms / 1e3) / HBM_PEAK, 4)}
            outs[st] = out
        row["bf16_rel_err_vs_f32"] = rel(outs["bf16"], outs["f32"])
        row["speedup_bf16_over_f32"] = round(row["f32"]["ms"] / row["bf16"]["ms"], 3)
        log(f"[sweep] c={c}: bf16 {row['bf16']['ms']:.3f} ms, f32 {row['f32']['ms']:.3f} ms, "
            f"rel err {row['bf16_rel_err_vs_f32']:.2e}")
        sweep.append(row)
        del outs
    rs = {}
    for st in ("bf16", "f32"):
        U = torch.empty((rank, n), dtype=torch.float32, device="cuda")
        sg = torch.empty(rank, dtype=torch.float64, device="cuda")
        dg = torch.empty(n, dtype=torch.float32, device="cuda")
        ms = timed(lambda: hs[st].rsvd(rank, p, cfg["seed"], U, sg), 2)
        hs[st].posterior_diag(dg)
        torch.cuda.synchronize()
        rs[st] = {"ms": round(ms, 3), "sigma": sg.clone(), "diag": dg.clone()}
        log(f"[sweep] rsvd {st}: {ms:.2f} ms")
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    t_copy = timed(lambda: dst.copy_(src), 5)
    t_fill = timed(lambda: dst.fill_(1.5), 5)
    res = {
        "metric": "B_k V columns/s over probe widths, bfloat16 vs float32 storage (1700 x 350 x 3, k = 200)",
        "config": {"workload": "grid3 sweep", "n": n, "k": k, "rank": rank, "oversample": p},
        "sweep": sweep,
        "rsvd_ms": {st: rs[st]["ms"] for st in rs},
        "rsvd_speedup_bf16_over_f32": round(rs["f32"]["ms"] / rs["bf16"]["ms"], 3),
        "bf16_sigma_rel_err_vs_f32": rel(rs["bf16"]["sigma"], rs["f32"]["sigma"]),
        "bf16_diag_rel_err_vs_f32": rel(rs["bf16"]["diag"], rs["f32"]["diag"]),
        "stream_ceiling_GBps": {"copy_read_plus_write": round(2 * nbytes / (t_copy / 1e3) / 1e9, 1),
                                "fill_write": round(nbytes / (t_fill / 1e3) / 1e9, 1),
                                "peak": HBM_PEAK / 1e9},
    }
    for H in hs.values():
        H.close()
    print(json.dumps(res), flush=True)


def bench_learned(args):
    """Learned diagonal B_0: train the network on the posterior variances of 32 runs
    of the 600 x 200 x 3 grid (k = 100, rank 100 + 20), then compare it with gamma I
    on 4 held-out 1700 x 350 x 3 problems (k = 200): iterations of the exact-line-search
    BFGS (= preconditioned CG) to a relative gradient of 1e-6, the secant residual of the
    library's H_k, and on the first problem the rSVD against the float64 oracle."""
    import numpy as np
    import torch
    import paper_2009_12663_amd as P
    from paper_2009_12663_amd import learned
    from workloads import quadratic as wq

    def iters(gn, tol=1e-6):
        g = np.asarray(gn) / gn[0]
        hit = np.nonzero(g <= tol)[0]
        return int(hit[0]) if hit.size else None

    t0 = time.perf_counter()
    Xs, Ts = [], []
    for seed in range(32):
        prob = wq.make_grid(600, 200, seed, device="cuda")
        S, Y, _ = wq.cg_pairs(prob, 100)
        Ts.append(learned.posterior_log_diag(S, Y, 100, 20, seed))
        Xs.append(learned.features(torch.log(prob.D), prob.b.abs(), 600, 200, prob.sigma / 5.0))
        del S, Y, prob
    X, T = torch.cat(Xs), torch.cat(Ts)
    del Xs, Ts
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"[bench-learned] {X.shape[0]} training samples in {t_data:.1f} s")
    t0 = time.perf_counter()
    steps = 3000
    net, losses = learned.train(X, T, steps=steps, batch=65536, lr=3e-3, seed=0, log_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"[bench-learned] trained {steps} Adam steps in {t_train:.1f} s, loss {losses[0][1]:.4g} -> {losses[-1][1]:.4g}")
    del X, T

    evals = []
    rsvd_err = None
    for seed in (100, 101, 102, 103):
        prob = wq.make_grid(1700, 350, seed, device="cuda")
        h0 = learned.predict_h0(net, torch.log(prob.D), prob.b.abs(), 1700, 350, prob.sigma / 5.0)
        _, _, gn_g = wq.cg_pairs(prob, 1000, rel_tol=1e-7)
        S, Y, gn_l = wq.cg_pairs(prob, 1000, precond=h0.double(), rel_tol=1e-7)
        _, _, gn_j = wq.cg_pairs(prob, 1000, precond=1.0 / prob.diag(), rel_tol=1e-7)
        k = min(200, S.shape[0])
        S, Y = S[:k], Y[:k]
        H = P.Bfgs(prob.n, k, h0, "f32")
        for s_, y_ in zip(S, Y):
            H.push_pair(s_.float(), y_.float())
        idx = list(range(max(0, k - 8), k))
        HY = H.apply_Hinv(Y[idx].float()).double()
        Sq = S[idx].float().double()
        secant = float((torch.linalg.vector_norm(HY - Sq, dim=1) / torch.linalg.vector_norm(Sq, dim=1)).max())
        row = {"seed": seed, "iters_gamma_I": iters(gn_g), "iters_learned": iters(gn_l), "iters_jacobi": iters(gn_j),
               "secant_residual_max": secant}
        # the same counts from the library's own driver (device BFGS with exact line
        # search on the device grid operator), with the smoothed, median-damped
        # Jacobi diagonal of the paper's recipe beside them
        op = P.GridOp(prob.nx, prob.nz, prob.nparam, prob.D, prob.sigma, wq.SMOOTH_HALF, prob.coupling)
        h0_sm, _, lam = P.precond_diag(prob.diag(), prob.nx, prob.nz, prob.nparam, 5.0, 20, 1.0)

        def lib_iters(h0v, memory=0, damping=1.0, max_iter=200):
            Hm = P.Bfgs(prob.n, memory if memory else max_iter, h0v, "f32")
            _, gn = P.minimize_quadratic(Hm, op, prob.b, max_iter, 1e-6, memory=memory, damping=damping)
            Hm.close()
            return len(gn) - 1 if gn[-1] <= 1e-6 * gn[0] else None

        row.update({"lib_iters_gamma_I": lib_iters(None), "lib_iters_learned": lib_iters(h0.float()),
                    "lib_iters_smoothed_jacobi": lib_iters(h0_sm), "smoothed_jacobi_lambda": lam})
        # the paper's L-BFGS (m = 5) against full-memory BFGS, with the learned B_0: with
        # exact line searches on a quadratic the two coincide in exact arithmetic, so the
        # comparison also runs with every step halved (an inexact line search)
        row.update({"lib_iters_lbfgs5_learned": lib_iters(h0.float(), memory=5),
                    "lib_iters_bfgs_learned_half_steps": lib_iters(h0.float(), damping=0.5, max_iter=400),
                    "lib_iters_lbfgs5_learned_half_steps": lib_iters(h0.float(), memory=5, damping=0.5, max_iter=400)})
        op.close()
        if seed == 100 and not args.no_cpu_baseline:
            # rSVD of the learned-H0 history against the float64 oracle (same stored values)
            from oracle import rsvd as orsvd, probes as oprobes
            rank = min(k, 200)
            U, Sig = H.rsvd(rank, 20, 5)
            Sq_all = S.float().double().cpu().numpy()
            Yq_all = Y.float().double().cpu().numpy()
            hq = h0.double().cpu().numpy()
            Xp = oprobes.round_to(oprobes.normal_block(prob.n, rank + 20, 5), "f32")
            ref = orsvd.rsvd(hq, Sq_all, Yq_all, Xp, rank)
            rsvd_err = float(np.abs(np.sort(Sig.cpu().numpy()) - np.sort(ref["Sigma"])).max() / abs(ref["Sigma"][0]))
            row["rsvd_sigma_rel_err_vs_oracle"] = rsvd_err
        H.close()
        evals.append(row)
        log(f"[bench-learned] {row}")
        del S, Y, prob
    it_g = [e["iters_gamma_I"] for e in evals]
    it_l = [e["iters_learned"] for e in evals]
    res = {
        "metric": "learned diagonal B_0 vs gamma I: BFGS iterations to |g|/|g0| <= 1e-6 on held-out problems",
        "value": round(float(np.mean(it_l)), 2), "unit": "iterations", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": round(t_train * 1e3 / steps, 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 weights, f32 accumulation", "data": "synthetic",
        "config": {"workload": "train: 32 x (600 x 200 x 3 grid, k 100, rank 100 + 20); evaluate: 4 x (1700 x 350 x 3, "
                               "k 200), seeds 100-103"},
        "mean_iters_gamma_I": round(float(np.mean(it_g)), 2),
        "library_driver_mean_iters": {key: round(float(np.mean([e[key] for e in evals if e[key] is not None])), 2)
                                      for key in ("lib_iters_gamma_I", "lib_iters_learned",
                                                  "lib_iters_smoothed_jacobi", "lib_iters_lbfgs5_learned",
                                                  "lib_iters_bfgs_learned_half_steps",
                                                  "lib_iters_lbfgs5_learned_half_steps")
                                      if any(e[key] is not None for e in evals)},
        "iteration_ratio_gamma_over_learned": round(float(np.mean(it_g)) / float(np.mean(it_l)), 3),
        "training_seconds": round(t_train, 2), "data_seconds": round(t_data, 2),
        "loss_first_last": [losses[0][1], losses[-1][1]], "evaluations": evals,
    }
    net.close()
    print(json.dumps(res), flush=True)


# ---------------------------------------------------------------------------
# rocprofv3 summaries (CSV output of --kernel-trace --stats and of --pmc runs)
# ---------------------------------------------------------------------------
KERNEL_GROUPS = [
    ("gemm1_mfma", "apply_gemm1"), ("gemm1_f64mfma", "apply_gemm1"), ("reduce_z", "apply_reduce"),
    ("reduce_partials", "apply_reduce"), ("small_solve", "apply_solve"), ("pack_small", "apply_pack"),
    ("gemm2_mfma", "apply_gemm2"), ("gemm2_f64mfma", "apply_gemm2"), ("scale_by_h0", "apply_gemm2"),
    ("probes_kernel", "probes"), ("leaf_forward_q", "tsqr_leaf_fwd"),
    ("tree_forward_q", "tsqr_tree"), ("tree_backward", "tsqr_tree"), ("set_identity", "tsqr_tree"),
    ("leaf_backward", "tsqr_leaf_bwd"), ("tri_mul", "tsqr_tree"),
    ("qtx_mfma", "proj_QtX"), ("qtx_bf16", "proj_QtX"), ("sum_chunks", "proj_QtX"), ("omega_solve", "omega_lu"),
    ("sym_tridiag", "sym_eig"), ("householder_accum", "sym_eig"), ("dc_leaves", "sym_eig"),
    ("dc_merge_gemm", "sym_eig"), ("dc_merge", "sym_eig"), ("order_sign", "sym_eig"), ("basis_mfma", "basis_diag"),
    ("basis_bf16", "basis_diag"), ("split_us", "basis_diag"),
    ("posterior_diag_kernel", "basis_diag"), ("store_pair_kernel", "push_pair"), ("gram_partial_kernel", "push_pair"),
    ("gram_finish_kernel", "push_pair"), ("rinv_update_kernel", "push_pair"), ("scatter_pair_layouts", "push_pair"),
    ("fill_h0_kernel", "push_pair"), ("upcast_kernel", "push_pair"),
]


# Groups with a kernel that runs once per launch while others run less often.
GROUP_ANCHORS = {"push_pair": "store_pair_kernel"}


def group_launches(group, calls_by_kernel):
    """Launches of a group in a trace: the anchor kernel's calls, else the fewest calls
    of any of its kernels (each launch runs every kernel of the group at least once)."""
    anchor = GROUP_ANCHORS.get(group)
    for k, cn in calls_by_kernel:
        if anchor and anchor in k:
            return cn
    return min(cn for _, cn in calls_by_kernel)


def group_of(kernel_name):
    if "gemm2_mfma<" in kernel_name and ", true>" in kernel_name:
        return "hdiff_gemm2"            # the difference form inside the rSVD
    for key, grp in KERNEL_GROUPS:
        if key in kernel_name:
            return grp
    return None


def short_name(kernel_name):
    k = kernel_name.replace("(anonymous namespace)::", "")
    return k.split("(")[0].replace("void ", "")


def summarize_profiles(d, out_dir, digest, cmd_prefix):
    """Turns the CSVs of one profiling session (kt = kernel trace, fetch/write =
    FETCH_SIZE/WRITE_SIZE of the bench, cfetch/cwrite = the same counters over a plain
    1 GiB device copy) into profiles/*.md and profiles/traffic.json."""
    import csv
    import glob

    def rows(pattern):
        files = glob.glob(os.path.join(d, pattern))
        return list(csv.DictReader(open(files[0]))) if files else []

    os.makedirs(out_dir, exist_ok=True)
    stats = rows("kt_*kernel_stats.csv")
    lines = ["# Kernel times: 1700 x 350 x 3 grid, n = 1,785,000, k = 200, bfloat16, 220 columns, rSVD 200 + 20", "",
             "Command (from the repository root, on one MI355X):", "",
             f"    {cmd_prefix} --kernel-trace --stats -d <dir> -o kt --output-format csv -- "
             "python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-fp32-path", "",
             "| kernel | group | calls | total ms | avg ms |", "|---|---|---|---|---|"]
    groups = {}
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:40]:
        g = group_of(r["Name"])
        if g is None and float(r["TotalDurationNs"]) < 2e6:
            continue
        lines.append(f"| {short_name(r['Name'])[:70]} | {g or '(input generation, torch)'} | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e6:.4f} |")
    for r in stats:
        g = group_of(r["Name"])
        if g is not None:
            groups.setdefault(g, []).append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"])))
    # a group launch runs each of its kernels at least once: launches = fewest calls
    lines += ["", "Per group (the library's profiling groups; `ms per launch` is what bench.py's "
              "HIP-event timing of the same group measures):", "",
              "| group | kernels | launches | ms per launch |", "|---|---|---|---|"]
    for g, v in sorted(groups.items(), key=lambda kv: -sum(t for _, _, t in kv[1])):
        launches = group_launches(g, [(k, cn) for k, cn, _ in v])
        lines.append(f"| {g} | {len(v)} | {launches} | {sum(t for _, _, t in v) / launches / 1e6:.4f} |")
    open(os.path.join(out_dir, "kernels_grid3_bf16.md"), "w").write("\n".join(lines) + "\n")

    def counter_values(pattern, counter):
        acc = {}
        for r in rows(pattern):
            if r.get("Counter_Name") != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc

    def counter_means(pattern, counter):
        return {k: sum(v) / len(v) for k, v in counter_values(pattern, counter).items()}

    fetch_all = counter_values("fetch_*counter_collection.csv", "FETCH_SIZE")
    write_all = counter_values("write_*counter_collection.csv", "WRITE_SIZE")
    fetch = {k: sum(v) / len(v) for k, v in fetch_all.items()}
    write = {k: sum(v) / len(v) for k, v in write_all.items()}
    cf = counter_means("cfetch_*counter_collection.csv", "FETCH_SIZE")
    cw = counter_means("cwrite_*counter_collection.csv", "WRITE_SIZE")
    copy_f = max([v for k, v in cf.items() if "copyBuffer" in k] or [0.0])
    copy_w = max([v for k, v in cw.items() if "copyBuffer" in k] or [0.0])
    gib_kib = float(1 << 20)
    f_scale = gib_kib / copy_f if copy_f else None
    w_scale = gib_kib / copy_w if copy_w else None
    lines = ["# HBM traffic per dispatch: 1700 x 350 x 3 grid, n = 1,785,000, k = 200, bfloat16", "",
             "Commands (from the repository root, one counter per run):", "",
             f"    {cmd_prefix} --pmc FETCH_SIZE -d <dir> -o fetch --output-format csv -- "
             "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp32-path",
             f"    {cmd_prefix} --pmc WRITE_SIZE -d <dir> -o write --output-format csv -- "
             "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp32-path",
             f"    {cmd_prefix} --pmc FETCH_SIZE -d <dir> -o cfetch --output-format csv -- "
             "python3 bench.py --calibrate-copy 1024",
             f"    {cmd_prefix} --pmc WRITE_SIZE -d <dir> -o cwrite --output-format csv -- "
             "python3 bench.py --calibrate-copy 1024", "",
             f"Calibration: a 1 GiB device copy reads FETCH_SIZE = {copy_f:.0f} KiB and WRITE_SIZE = "
             f"{copy_w:.0f} KiB per dispatch, so the counters are scaled by {f_scale:.3f} (fetch) and "
             f"{w_scale:.3f} (write) to bytes moved.", "",
             "| kernel | group | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) |", "|---|---|---|---|---|"]
    per_group = {}
    for k in sorted(set(fetch) | set(write), key=lambda k: -(fetch.get(k, 0) + write.get(k, 0))):
        g = group_of(k)
        if g is None:
            continue
        fb = fetch.get(k, 0.0) * 1024 * (f_scale or 0)
        wb = write.get(k, 0.0) * 1024 * (w_scale or 0)
        lines.append(f"| {short_name(k)[:70]} | {g} | {fetch.get(k, 0):.0f} | {write.get(k, 0):.0f} | {fb + wb:.4g} |")
        calls = max(len(fetch_all.get(k, [])), len(write_all.get(k, [])), 1)
        per_group.setdefault(g, []).append((k, calls, (fb + wb) * calls))
    # bytes per group launch: all dispatches of the group's kernels over the number of launches
    traffic = {}
    lines += ["", "Per group launch (sum over the group's kernels):", "",
              "| group | launches | HBM bytes per launch |", "|---|---|---|"]
    for g, v in sorted(per_group.items(), key=lambda kv: -sum(b for _, _, b in kv[1])):
        launches = group_launches(g, [(k, cn) for k, cn, _ in v])
        per_launch = sum(b for _, _, b in v) / launches
        lines.append(f"| {g} | {launches} | {per_launch:.4g} |")
        traffic[g] = {"hbm_bytes_per_launch": per_launch, "source_digest": digest,
                      "fetch_scale": f_scale, "write_scale": w_scale}
    open(os.path.join(out_dir, "hbm_traffic_grid3_bf16.md"), "w").write("\n".join(lines) + "\n")
    json.dump(traffic, open(os.path.join(out_dir, "traffic.json"), "w"), indent=1)

    # matrix-core use: MFMA operation counts (x 512 = flops) and busy cycles per dispatch,
    # next to the kernel-trace duration of the same kernel
    mops = {c: counter_means("mfma_*counter_collection.csv", c)
            for c in ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_VALU_MFMA_BUSY_CYCLES",
                      "GRBM_GUI_ACTIVE")}
    if mops["GRBM_GUI_ACTIVE"]:
        avg_ns = {r["Name"]: float(r["AverageNs"]) for r in stats}
        simds = 256 * 4
        lines = ["# Matrix-core use per dispatch: 1700 x 350 x 3 grid, n = 1,785,000, k = 200, bfloat16", "",
                 "Command (from the repository root; one pass, 3 SQ and 1 GRBM counters):", "",
                 f"    {cmd_prefix} --pmc SQ_INSTS_VALU_MFMA_MOPS_BF16 SQ_INSTS_VALU_MFMA_MOPS_F64 "
                 "SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE -d <dir> -o mfma --output-format csv -- "
                 "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp32-path", "",
                 "flops = MOPS x 512; TFLOP/s uses the kernel-trace average duration of the same kernel; "
                 "busy = SQ_VALU_MFMA_BUSY_CYCLES / (that duration x 2.4 GHz x 1024 SIMDs), the share of "
                 "the matrix cores' cycles they were busy (GRBM_GUI_ACTIVE, collected in the same pass, "
                 "includes the profiler's dispatch window and is not used). Peaks: bfloat16 dense "
                 "2.5 PFLOP/s, float64 matrix 78.6 TFLOP/s.", "",
                 "| kernel | group | bf16 GFLOP | f64 GFLOP | avg ms | bf16 TFLOP/s (% of 2500) | "
                 "f64 TFLOP/s (% of 78.6) | MFMA busy % |", "|---|---|---|---|---|---|---|---|"]
        names = set(mops["SQ_INSTS_VALU_MFMA_MOPS_BF16"]) | set(mops["SQ_INSTS_VALU_MFMA_MOPS_F64"])
        for k in sorted(names, key=lambda k: -(mops["SQ_INSTS_VALU_MFMA_MOPS_BF16"].get(k, 0)
                                              + 64 * mops["SQ_INSTS_VALU_MFMA_MOPS_F64"].get(k, 0))):
            fb = mops["SQ_INSTS_VALU_MFMA_MOPS_BF16"].get(k, 0.0) * 512
            fd = mops["SQ_INSTS_VALU_MFMA_MOPS_F64"].get(k, 0.0) * 512
            if fb + fd == 0:
                continue
            ms = avg_ns.get(k, 0.0) / 1e6
            cyc = avg_ns.get(k, 0.0) * 2.4
            busy = 100 * mops["SQ_VALU_MFMA_BUSY_CYCLES"].get(k, 0.0) / (cyc * simds) if cyc else 0.0
            tb = fb / ms / 1e9 if ms else 0.0
            td = fd / ms / 1e9 if ms else 0.0
            lines.append(f"| {short_name(k)[:60]} | {group_of(k) or '-'} | {fb / 1e9:.2f} | {fd / 1e9:.2f} | {ms:.4f} | "
                         f"{tb:.1f} ({100 * tb / 2500:.1f} %) | {td:.2f} ({100 * td / 78.6:.1f} %) | {busy:.1f} |")
        open(os.path.join(out_dir, "mfma_grid3_bf16.md"), "w").write("\n".join(lines) + "\n")
    # address translation: the per-CU translation cache's requests, hits and misses
    tl = {c: counter_means("utcl1_*counter_collection.csv", c)
          for c in ("TCP_UTCL1_REQUEST_sum", "TCP_UTCL1_TRANSLATION_HIT_sum", "TCP_UTCL1_TRANSLATION_MISS_sum",
                    "TCP_UTCL1_THRASHING_STALL_sum")}
    if tl["TCP_UTCL1_REQUEST_sum"]:
        lines = ["# Address translation per dispatch: 1700 x 350 x 3 grid, n = 1,785,000, k = 200, bfloat16", "",
                 "Command (from the repository root; one pass, 4 TCP counters):", "",
                 f"    {cmd_prefix} --pmc TCP_UTCL1_TRANSLATION_MISS_sum TCP_UTCL1_TRANSLATION_HIT_sum "
                 "TCP_UTCL1_REQUEST_sum TCP_UTCL1_THRASHING_STALL_sum -d <dir> -o utcl1 --output-format csv -- "
                 "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp32-path", "",
                 "miss % = misses / (hits + misses) of the per-CU translation cache (UTCL1), summed over "
                 "the CUs; library kernels with at least 10^6 requests.", "",
                 "| kernel | group | requests | miss % | thrashing stalls |", "|---|---|---|---|---|"]
        req = tl["TCP_UTCL1_REQUEST_sum"]
        for k in sorted(req, key=lambda k: -req[k]):
            if group_of(k) is None or req[k] < 1e6:
                continue
            hit = tl["TCP_UTCL1_TRANSLATION_HIT_sum"].get(k, 0.0)
            miss = tl["TCP_UTCL1_TRANSLATION_MISS_sum"].get(k, 0.0)
            lines.append(f"| {short_name(k)[:60]} | {group_of(k)} | {req[k]:.3e} | "
                         f"{100 * miss / max(hit + miss, 1.0):.2f} | "
                         f"{tl['TCP_UTCL1_THRASHING_STALL_sum'].get(k, 0.0):.3e} |")
        open(os.path.join(out_dir, "translation_grid3_bf16.md"), "w").write("\n".join(lines) + "\n")
    log(f"[bench] wrote profile summaries for {len(per_group)} kernel groups to {out_dir}")


def csrc_digest():
    csrc = sorted(os.path.join("paper_2009_12663_amd", "csrc", f)
                  for f in os.listdir(os.path.join(ROOT, "paper_2009_12663_amd", "csrc")))
    return source_digest(csrc)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--storage", default="bf16", choices=["bf16", "f32", "f64"])
    ap.add_argument("--ncols", type=int, default=220)
    ap.add_argument("--config", default="grid3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slice-rows", type=int, default=1 << 18, help="row slice of --config streamed")
    ap.add_argument("--no-fp32-path", action="store_true",
                    help="skip the float32-storage comparison run after the timed region")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (counter calibration)")
    ap.add_argument("--summarize", default="", metavar="DIR",
                    help="only summarise the rocprofv3 CSVs in DIR into profiles/ (no GPU needed)")
    args = ap.parse_args()

    if args.summarize:
        summarize_profiles(args.summarize, os.path.join(ROOT, "profiles"), csrc_digest(), "rocprofv3")
        return

    if args.calibrate_copy:
        import torch
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.calibrate_copy} MiB x3")
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the path's row sharding over several GPUs is "
              "designed but not implemented. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.config == "batch":
        bench_batch(args)
        return
    if args.config == "learned":
        bench_learned(args)
        return
    if args.config == "sweep":
        bench_sweep(args)
        return
    if args.config == "streamed":
        bench_streamed(args)
        return

    import torch
    import paper_2009_12663_amd as P
    from workloads import quadratic as wq

    cfg = wq.CONFIGS[args.config]
    k, rank, p = cfg["k"], cfg["rank"], cfg["oversample"]
    c_rsvd = rank + p
    t0 = time.perf_counter()
    prob = wq.make_problem(args.config, device="cuda")
    S, Y, gn = wq.cg_pairs(prob, k)
    torch.cuda.synchronize()
    n = prob.n
    log(f"[bench] {args.config}: n={n} k={S.shape[0]} pairs generated in {time.perf_counter() - t0:.1f}s")

    H = P.Bfgs(n, k, None, args.storage)
    for s, y in zip(S, Y):
        H.push_pair(s.float() if args.storage != "f64" else s, y.float() if args.storage != "f64" else y)
    if args.storage != "bf16" or args.no_fp32_path:
        del S, Y
    V = H.generate_probes(seed=2, ncols=args.ncols)
    out = torch.empty((args.ncols, n), dtype=H.rdt, device="cuda")
    U = torch.empty((rank, n), dtype=H.rdt, device="cuda")
    Sig = torch.empty(rank, dtype=torch.float64, device="cuda")
    dg = torch.empty(n, dtype=H.rdt, device="cuda")
    seed = cfg["seed"]

    def step():
        H.apply_Hinv(V, out)
        H.rsvd(rank, p, seed, U, Sig)
        H.posterior_diag(dg)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    if H.get_status() != 0:
        raise RuntimeError("device status after warmup is not OK")

    H.L.bfgs_profile(H.h, 1)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        e = evs[i]
        e[0].record()
        H.apply_Hinv(V, out)
        e[1].record()
        H.rsvd(rank, p, seed, U, Sig)
        e[2].record()
        H.posterior_diag(dg)
        e[3].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    import ctypes
    buf = ctypes.create_string_buffer(1 << 16)
    H.L.bfgs_profile_report(H.h, buf, len(buf))
    H.L.bfgs_profile(H.h, 0)
    prof = json.loads(buf.value.decode())
    status = H.get_status()
    apply_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    rsvd_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    diag_ms = sum(e[2].elapsed_time(e[3]) for e in evs) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    log(f"[bench] {args.steps} steps: apply {apply_ms:.3f} ms, rsvd {rsvd_ms:.3f} ms, step {ms_per_step:.3f} ms")

    wb = {"bf16": 2, "f32": 4, "f64": 8}[args.storage]
    ob = 8 if args.storage == "f64" else 4
    models = kernel_models(n, k, args.ncols, rank, wb, wb, ob)
    models_rsvd = kernel_models(n, k, c_rsvd, rank, wb, wb, ob)
    digest = csrc_digest()
    entries = []
    for name, (cnt, tot_ms) in prof.items():
        model = models.get(name)
        if name.startswith("tsqr") or name.startswith("hdiff") or name in ("proj_QtX", "basis_diag", "probes"):
            model = models_rsvd.get(name)
        if model is None:
            continue
        entries.append((tot_ms, name, cnt, model))
    entries.sort(reverse=True)
    dom = entries[0] if entries else None
    roof = None
    if dom:
        tot_ms, name, cnt, model = dom
        roof = roofline_entry(name, model, tot_ms / cnt / 1e3, load_traffic(name, digest))
    roof_apply = []
    for name in ("apply_gemm1", "apply_gemm2"):
        if name in prof:
            cnt, tot_ms = prof[name]
            roof_apply.append(roofline_entry(name, models[name], tot_ms / cnt / 1e3, load_traffic(name, digest)))
    # the other modelled groups of the rSVD step, each against its own bound
    roof_rsvd = []
    for name in ("tsqr_leaf_bwd", "proj_QtX", "basis_diag", "hdiff_gemm1", "hdiff_gemm2"):
        if name in prof and name in models_rsvd and not (dom and dom[1] == name):
            cnt, tot_ms = prof[name]
            roof_rsvd.append(roofline_entry(name, models_rsvd[name], tot_ms / cnt / 1e3, load_traffic(name, digest)))

    result = {
        "metric": "H_k V columns/s + rSVD wall time at n=1.785M, k=200; rel err vs FP64 oracle",
        "value": round(args.ncols / (apply_ms / 1e3), 2),
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg.get('nx', '')}x{cfg.get('nz', '')}x3 grid quadratic, "
                               f"n={n}, k={k} exact-line-search BFGS pairs, {args.ncols} probe columns, "
                               f"rSVD rank {rank} + {p}", "n": n, "k": k, "ncols": args.ncols,
                   "rank": rank, "oversample": p, "storage": args.storage, "parallelism": "single GPU"},
        "apply_ms": round(apply_ms, 4),
        "rsvd_ms": round(rsvd_ms, 4),
        "posterior_diag_ms": round(diag_ms, 4),
        "device_status": status,
        "roofline": roof,
        "roofline_apply": roof_apply,
        "roofline_rsvd": roof_rsvd,
        "kernels_ms_per_step": {name: round(v[1] / args.steps, 4) for name, v in prof.items()},
        "source_digest": digest,
    }
    if args.storage == "bf16" and not args.no_fp32_path:
        result["fp32_path"] = fp32_path(P, S, Y, n, k, V, out, rank, p, seed, Sig, dg, args.ncols, apply_ms)
        del S, Y
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"], errs, (So, Yo, h0o) = cpu_baseline(H, V, out, n, args.storage, args.ncols)
        errs.update(oracle_rsvd_errors(So, Yo, h0o, args.storage, seed, rank, p, Sig, dg))
        errs["sample"] = result["cpu_baseline"]["sample"] + "; rSVD: all of Sigma and the posterior variance"
        result["rel_err_vs_oracle"] = errs
        del So, Yo
        log(f"[bench] cpu baseline: {result['cpu_baseline']['value']} columns/s "
            f"({result['cpu_baseline']['cores']} threads)")
    else:
        result["cpu_baseline"] = None
    H.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
