#!/usr/bin/env python3
"""Benchmark: adaptive randomized hybrid butterfly construction (Alg. 2) on one
MI355X, headline workload at n = m = 65536.

A step is one whole construction (every row of the hot path: random blocks,
black-box products, partial-factor products, batched pivoted QR, centre-block
least squares, apply plan) of the segment-kernel operator exp(i k r)/r between
two parallel unit segments at 8 points per wavelength, leaf 64, p = 2,
r0 = 4.  Each step uses a fresh seed (a new construction request); inputs
(point coordinates) are resident in HBM before the timed region.  K steps are
timed back to back (closed loop); the line reports factorizations/s, p50/p99
latency, the relative error of the last factorization against the FP64
oracle on sampled rows (16 Gaussian test columns, Sec. 6 error measure), the
roofline of the dominant kernel measured with HIP events on each of its
launches (over --roofline-steps further constructions of the same workload on
one stream: the timed loop runs each construction's two sides side by side,
so its black-box launches share the device and each one's events would span
the other's work), and the FP64 oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# per-request constructions run their two sides on two streams (bf_opts
# BF_OPT_ONE_STREAM off; the request engine with several slots keeps one
# stream per request, with one slot the two sides)
TWO_SIDES = True
METRIC = "factorizations/s + p50/p99 latency at n=64K, rel err ≤1e-6 vs FP64 oracle"
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 2.4 GHz x 64 flops/clock
# (16 lanes, a packed dual FMA per lane) = 157.3 TFLOP/s.  The vector ALUs
# issue one wave64 instruction per SIMD every 4 clocks: 256 x 4 x 16 lanes x
# 2.4 GHz = 39.3e12 lane-instructions/s, each worth 4 FP32 flops at the peak
# rating.  The black-box products are bound by that issue rate: the vector
# ALUs evaluate the kernel entries while the complex multiply-adds run in
# split form on the BF16 matrix cores beside them.  Their roofline therefore
# counts the vector-ALU work of the entry evaluations (lane-instructions per
# entry, measured by rocprofv3 SQ_INSTS_VALU on this kernel) in FP32 flop
# equivalents against this peak; the complex-MAC flop rate is reported beside.
PEAK_FP32_TFLOPS = 157.3
VALU_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9
PEAK_HBM_GBS = 8000.0
# MI355X dense BF16 matrix-core peak (no sparsity): the black-box kernel's
# complex multiply-adds run there, so its roofline fraction is its algorithmic
# MAC flops (8 per complex multiply-add of A(:, seg) X(seg, :)) over this peak.
PEAK_BF16_MFMA_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--roofline-steps", type=int, default=2,
                    help="one-stream constructions after the timed loop whose kernels give the "
                         "roofline and the per-phase times (each kernel alone on the device)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--ppw", type=float, default=8.0)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--tol", type=float, default=2e-7)
    ap.add_argument("--rows", type=int, default=128, help="sampled rows of the error check")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the n=262144 FIO butterfly's apply roofline in the default line")
    ap.add_argument("--slots", type=int, default=4,
                    help="device slots of the Poisson streams and the mixed stream")
    ap.add_argument("--served-slots", type=int, default=2,
                    help="device slots of the served closed loop at the headline size (2 "
                         "measured 4%% more constructions per second than 4 on one box)")
    ap.add_argument("--stream", type=int, default=64,
                    help="requests of each Poisson stream at the headline size, run at 0.5x, "
                         "1x and 2x the measured capacity (0 = skip)")
    ap.add_argument("--one-stream", action="store_true",
                    help="run each per-request construction's two sides on one stream and "
                         "thread (bf_opts BF_OPT_ONE_STREAM; the request engine always does)")
    ap.add_argument("--max-constructs-line", type=int, default=1, choices=[0, 1],
                    help="also run the Poisson streams with at most 2 constructions at once "
                         "(bf_server_opts.max_constructs; keys 0.5x_max2, ...)")
    ap.add_argument("--mix", type=int, default=256,
                    help="requests of the mixed serving stream (0 = skip); run served and "
                         "through the per-request path")
    ap.add_argument("--mix-rate", type=float, default=160.0,
                    help="Poisson arrival rate (requests/s) of the mixed stream")
    ap.add_argument("--apply-burst", type=int, default=0,
                    help="only submit this many 1-column applies at once against one "
                         "factorization of the headline operator, with and without continuous "
                         "batching (--batch-cols), and print one JSON line")
    ap.add_argument("--solve-rounds", type=int, default=0, choices=(0, 1),
                    help="served runs: cross-request solve rounds in the request engine")
    ap.add_argument("--batch-cols", type=int, default=64,
                    help="continuous batching of the mixed stream's applies (columns per "
                         "merged product; 0 = off)")
    ap.add_argument("--exact-scaling", default="",
                    help="only recover exact random butterflies (Sec. 6.1) through the "
                         "butterfly black box: comma-separated entries L or L:r:leaf "
                         "(default r = 8, leaf 8); one JSON line per entry")
    ap.add_argument("--em3d", default="",
                    help="only construct the 3D semi-sphere operator (Sec. 6.3, p = 4, "
                         "r0 = 64): comma-separated entries n:L; one JSON line per n and "
                         "tolerance")
    ap.add_argument("--em3d-tols", default="1e-2,1e-3,1e-4",
                    help="tolerances of --em3d")
    ap.add_argument("--variants", default="",
                    help="only compare the hybrid (l_m = L/2), column-wise (l_m = 0) and "
                         "row-wise (l_m = L) constructions of the segment-kernel operator at "
                         "these comma-separated n (leaf 64, tol 1e-6); one JSON line each")
    ap.add_argument("--precision-form", type=int, default=0, metavar="N",
                    help="only run the precision comparison on the 1D Fourier integral "
                         "operator of size N (e.g. 262144; leaf 16, tol 1e-6): matrix-free construction with the split-BF16 and FP64 black "
                         "boxes, recompression with the butterfly as black box (FP32 and "
                         "split-BF16 applies) and apply rates; one JSON line each")
    ap.add_argument("--compose", type=int, default=0, metavar="N",
                    help="only run the category (ii) recompression at size N (e.g. 65536): "
                         "B1 ~ A(X0,X1) and B2 ~ A(X1,X2) built matrix-free on the GPU (three "
                         "segments y = 0, 1, 2, 8 points per wavelength, leaf 64, tol 1e-6), "
                         "the composition B1 B2 recompressed with Alg. 2, error against FP64 "
                         "A01 (A12 Omega) on sampled rows; one JSON line")
    ap.add_argument("--save-tune", default="",
                    help="after the run, write the autotuner's table (with the timed candidates) "
                         "to this file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy three times (reference "
                         "dispatch for calibrating rocprofv3 byte counters) and exit")
    return ap.parse_args()


def exact_scaling(cases, tol=1e-5):
    """Sec. 6.1 workload at growing L: random exact butterflies (all ranks r)
    recovered with the butterfly as the black box; time of the construction
    (second of two), ranks, factor entries and device bytes, error against
    the source factors on 16 Gaussian columns."""
    import torch

    import paper_2002_03400_amd as bf
    import workloads as wl
    torch.cuda.init()
    for L, r, leaf in cases:
        n = leaf << L
        kU, kV, data = wl.exact_butterfly_canonical(L, r, seed=L, leaf=leaf)
        src = bf.import_factors(n, n, leaf, kU, kV, data)
        del data
        op = bf.from_factors(src)
        Om = torch.from_numpy(wl.test_columns(n, 16, 1001).astype(np.complex64)).cuda()
        ref = src.apply(Om)
        for rep in range(2):
            bf.profile_start()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F = bf.construct(op, tol, leaf, seed=3 + rep)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            prof = bf.profile_stop()
            print(f"exact L={L} r={r} leaf={leaf}: construction {rep} took {dt:.2f} s",
                  file=sys.stderr, flush=True)
            gU, gV = F.ranks()
            st = F.stats()
            err = float((F.apply(Om) - ref).norm() / ref.norm())
            if rep == 1:
                print(json.dumps({
                    "workload": "exact random butterfly (Sec. 6.1), butterfly black box",
                    "L": L, "n": n, "r": r, "leaf": leaf, "tol": tol, "seconds": dt,
                    "rel_err": err, "ranks": sorted({int(x) for x in np.unique(gU)} |
                                                    {int(x) for x in np.unique(gV)}),
                    "factor_entries": st.factor_entries, "device_bytes": st.device_bytes,
                    "phase_ms": {k: v["ms"] for k, v in prof.items()}}), flush=True)
            F.close()
        op.close()
        src.close()
        torch.cuda.empty_cache()


def em3d(cases, tols):
    """Sec. 6.3 workload: exp(i k r)/r between two adjacent unit semi-spheres
    (synthetic equal-area point sets, ten points per wavelength), built from
    the matrix-free black box with p = 4, r0 = 64 and leaves of about n / 2^L
    points.  Error: ||A W - F W|| / ||A W|| on 16 Gaussian columns W with A
    the black-box product (complex64, FP32-accurate entries).  One untimed
    construction at n = 8192 first loads every kernel."""
    import torch

    import paper_2002_03400_amd as bf
    import workloads as wl
    torch.cuda.init()
    gw = wl.hemisphere_pair(8192, seed=1)
    opw = bf.helmholtz3d(gw.targets, gw.sources, gw.k)
    bf.construct(opw, min(tols), 93, p=4, r0=64, seed=1).close()
    opw.close()
    for n, L in cases:
        leaf = -(-n // (1 << L))
        g = wl.hemisphere_pair(n, seed=1)
        op = bf.helmholtz3d(g.targets, g.sources, g.k)
        Om = torch.from_numpy(wl.test_columns(n, 16, 1001).astype(np.complex64)).cuda()
        ref = op.matvec(Om)
        for tol in tols:
            bf.profile_start()
            torch.cuda.synchronize()
            t0 = time.perf_counter()

            def progress(phase, level, n=n, tol=tol, t0=t0):
                print(f"em3d n={n} tol={tol:g}: {phase} {level} done at "
                      f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
            F = bf.construct(op, tol, leaf, p=4, r0=64, seed=1, progress=progress)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            prof = bf.profile_stop()
            gU, gV = F.ranks()
            st = F.stats()
            err = float((F.apply(Om) - ref).norm() / ref.norm())
            print(json.dumps({
                "workload": "two adjacent unit semi-spheres (Sec. 6.3), matrix-free black box",
                "n": n, "L": F.L, "leaf": leaf, "tol": tol, "k": g.k, "seconds": dt,
                "rel_err": err, "max_rank": int(max(gU.max(), gV.max())),
                "factor_entries": st.factor_entries, "device_bytes": st.device_bytes,
                "phase_ms": {k: v["ms"] for k, v in prof.items()}}), flush=True)
            F.close()
        op.close()
        torch.cuda.empty_cache()


def precision_form(n, leaf=16, tol=1e-6):
    """Precision form: A_jk = exp(2 pi i (x_j xi_k + c(x_j)|xi_k|)) (the 1D
    Fourier integral operator), leaf 16, tol 1e-6.  (1) Matrix-free
    construction with the split-BF16 black box and with the FP64 one;
    (2) recompression of the first result with the butterfly itself as the
    black box, its applies in FP32 and in split-BF16; (3) apply rates of that
    butterfly at 1, 16 and 64 right-hand sides.  Errors ||A W - F W|| / ||A W||
    on 16 Gaussian columns W, A W from the FP64-accumulating black box.  Times
    are the second of two runs (the first loads the kernels)."""
    import torch

    import paper_2002_03400_amd as bf
    import workloads as wl
    torch.cuda.init()
    op = bf.fio(n)
    Om = torch.from_numpy(wl.test_columns(n, 16, 1001).astype(np.complex64)).cuda()
    op.set_precision("fp64")
    ref = op.matvec(Om)

    def rel(F):
        return float((F.apply(Om) - ref).norm() / ref.norm())

    def timed(o, seed):
        bf.construct(o, tol, leaf, seed=seed).close()
        bf.profile_start()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = bf.construct(o, tol, leaf, seed=seed)
        torch.cuda.synchronize()
        return F, time.perf_counter() - t0, bf.profile_stop()

    keep = None
    for prec in ("bf16x3", "fp64"):
        op.set_precision(prec)
        F, dt, prof = timed(op, 5)
        st = F.stats()
        print(json.dumps({
            "workload": "1D Fourier integral operator, matrix-free black box",
            "n": n, "L": F.L, "leaf": leaf, "tol": tol, "black_box": prec, "seconds": dt,
            "rel_err": rel(F), "max_rank": st.max_rank, "factor_entries": st.factor_entries,
            "device_bytes": st.device_bytes,
            "phase_ms": {k: v["ms"] for k, v in prof.items()}}), flush=True)
        if prec == "bf16x3":
            keep = F
        else:
            F.close()
    op.set_precision("bf16x3")
    opb = bf.from_factors(keep)
    for aprec in ("fp32", "bf16x3"):
        keep.set_precision(aprec)
        G, dt, prof = timed(opb, 7)
        st = G.stats()
        ap = prof.get("apply", {"ms": 0.0, "flops": 0.0})
        print(json.dumps({
            "workload": "recompression of the FIO butterfly, the butterfly as black box",
            "n": n, "leaf": leaf, "tol": tol, "apply_precision": aprec, "seconds": dt,
            "rel_err": rel(G), "max_rank": st.max_rank, "factor_entries": st.factor_entries,
            "apply_ms": ap["ms"], "apply_TFLOP_per_s": ap["flops"] / max(ap["ms"], 1e-9) / 1e9,
            "phase_ms": {k: v["ms"] for k, v in prof.items()}}), flush=True)
        G.close()
    fe = keep.stats().factor_entries
    for aprec in ("fp32", "bf16x3"):
        keep.set_precision(aprec)
        out = {}
        for s in (1, 16, 64):
            X = torch.randn(n, s, dtype=torch.complex64, device="cuda")
            keep.apply(X)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                keep.apply(X)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 5
            gbs = 8.0 * fe / dt / 1e9
            out[f"s={s}"] = {"ms": 1e3 * dt, "factor_GB_per_s": gbs, "frac_hbm": gbs / 8000.0,
                             "TFLOP_per_s": 8.0 * fe * s / dt / 1e12}
        print(json.dumps({"workload": "applies of the FIO butterfly", "n": n,
                          "precision": aprec, "factor_bytes": 8 * fe, "applies": out}), flush=True)
    keep.close()
    op.close()


def variants(sizes, leaf=64, tol=1e-6):
    """Sec. 3.3 / Sec. 4: the same algorithm building the column-wise and
    row-wise factorizations instead of the hybrid one; time (second of two
    runs), black-box columns, error on 16 Gaussian columns against the
    black-box product, phases."""
    import torch

    import paper_2002_03400_amd as bf
    import workloads as wl
    torch.cuda.init()
    for n in sizes:
        g = wl.segment_pair(n, ppw=8.0)
        op = bf.segkernel(g.targets, g.sources, g.k)
        Om = torch.from_numpy(wl.test_columns(n, 16, 1001).astype(np.complex64)).cuda()
        ref = op.matvec(Om)
        for center in ("hybrid", "column", "row"):
            for rep in range(2):
                bf.profile_start()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F = bf.construct(op, tol, leaf, seed=1, center=center)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                prof = bf.profile_stop()
                print(f"variants n={n} {center}: construction {rep} took {dt:.2f} s",
                      file=sys.stderr, flush=True)
                if rep == 1:
                    st = F.stats()
                    err = float((F.apply(Om) - ref).norm() / ref.norm())
                    print(json.dumps({
                        "workload": "segment pair (Sec. 6.2 geometry), factorization variants",
                        "n": n, "leaf": leaf, "tol": tol, "center": center, "L": st.L,
                        "lm": st.lm, "seconds": dt, "rel_err": err, "max_rank": st.max_rank,
                        "matvec_cols": st.matvec_cols, "rmatvec_cols": st.rmatvec_cols,
                        "factor_entries": st.factor_entries,
                        "phase_ms": {k: v["ms"] for k, v in prof.items()}}), flush=True)
                F.close()
        op.close()


def apply_burst(args):
    """K one-column applies against one factorization of the headline operator
    (n = 65536), queued behind its construction: the time from the
    construction's completion until the last apply finished (server clock),
    and each apply's wait after that point, without and with continuous
    batching in the request engine."""
    import torch

    import paper_2002_03400_amd as bf
    import workloads as wl
    torch.cuda.init()
    g = wl.segment_pair(args.n, ppw=args.ppw)
    op = bf.segkernel(g.targets, g.sources, g.k)
    out = {"workload": f"{args.apply_burst} one-column applies queued behind a construction, "
                       f"segment kernel n={args.n}"}
    xs = [torch.randn(args.n, 1, dtype=torch.complex64, device="cuda")
          for _ in range(args.apply_burst)]
    torch.cuda.synchronize()
    for bc in (0, args.batch_cols):
        for rep in range(2):      # the first round warms the kernels up
            S = bf.Server(slots=args.slots, batch_cols=bc)
            tf = S.submit_construct(op, args.tol, args.leaf, seed=3)
            ts = [S.submit_apply(tf, x) for x in xs]
            done = S.wait(tf)["finish_ns"]
            infos = [S.wait(t) for t in ts]
            S.close()
        drain = (max(i["finish_ns"] for i in infos) - done) * 1e-9
        lat = [(i["finish_ns"] - max(done, i["arrival_ns"])) * 1e-9 for i in infos]
        out[f"batch_cols={bc}"] = {
            "drain_ms": 1e3 * drain, "applies_per_s": args.apply_burst / max(drain, 1e-9),
            "p50_ms": 1e3 * pct(lat, 50), "p99_ms": 1e3 * pct(lat, 99),
            "mean_batch": sum(i["batch"] for i in infos) / len(infos)}
    print(json.dumps(out), flush=True)


def _kernel_rows_times(args):
    """Rows [r0, r1) of the FP64 kernel matrix times X (process-pool worker)."""
    from oracle import operators as ops
    t, src, k, r0, r1, X = args
    return ops.segment_kernel_entries(t, src, k, rows=slice(r0, r1)) @ X


def compose(n, leaf=64, tol=1e-6, rows=128, workers=12):
    """Category (ii) of Sec. 1 at size n: two butterflies B1 ~ A(X0, X1) and
    B2 ~ A(X1, X2) built on the GPU from the matrix-free black box, their
    composition recompressed into one butterfly by Alg. 2 with the two
    butterflies' applies as the black box.  Errors on 16 Gaussian columns:
    against the FP64 product A01 (A12 Omega) of the oracle's kernel entries on
    `rows` sampled rows (A12 Omega in full, row blocks over a process pool),
    and against the composition B1 (B2 Omega) on every row."""
    import multiprocessing as mp

    import torch

    import paper_2002_03400_amd as bf
    import workloads as wl
    from oracle import operators as ops
    torch.cuda.init()
    g01, g12 = wl.segment_triple(n, ppw=8.0)
    o1 = bf.segkernel(g01.targets, g01.sources, g01.k)
    o2 = bf.segkernel(g12.targets, g12.sources, g12.k)
    bf.construct(o1, tol, leaf, seed=20).close()            # kernels loaded, tuner classes timed
    times = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B1 = bf.construct(o1, tol, leaf, seed=21)
    torch.cuda.synchronize()
    times["B1_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    B2 = bf.construct(o2, tol, leaf, seed=22)
    torch.cuda.synchronize()
    times["B2_s"] = time.perf_counter() - t0
    prod = bf.compose(bf.from_factors(B1), bf.from_factors(B2))
    F = bf.construct(prod, tol, leaf, seed=30)               # untimed: first recompression
    F.close()
    bf.profile_start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = bf.construct(prod, tol, leaf, seed=23)
    torch.cuda.synchronize()
    times["recompress_s"] = time.perf_counter() - t0
    prof = bf.profile_stop()
    st = F.stats()
    Om = wl.test_columns(n, 16, 1001)
    Omd = torch.from_numpy(Om.astype(np.complex64)).cuda()
    FO = F.apply(Omd)
    BB = B1.apply(B2.apply(Omd))
    err_bb = float((FO - BB).norm() / BB.norm())
    # FP64 reference: A12 Omega in full, then sampled rows of A01
    t0 = time.perf_counter()
    step = max(1, (1 << 22) // n)
    jobs = [(g12.targets, g12.sources, g12.k, r0, min(n, r0 + step), Om)
            for r0 in range(0, n, step)]
    # fresh interpreters: the workers never touch the GPU this process holds
    with mp.get_context("spawn").Pool(workers) as pool:
        A12Om = np.concatenate(pool.map(_kernel_rows_times, jobs), axis=0)
    sel = np.sort(np.random.default_rng(0).choice(n, min(rows, n), replace=False))
    ref = ops.segment_kernel_entries(g01.targets, g01.sources, g01.k, rows=sel) @ A12Om
    ref_s = time.perf_counter() - t0
    got = FO.cpu().numpy()[sel]
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    b1s, b2s = B1.stats(), B2.stats()
    print(json.dumps({
        "workload": (f"category (ii) recompression: B1 B2, three unit segments y=0,1,2, "
                     f"n={n}, 8 points/wavelength, leaf {leaf}, tol {tol:g}"),
        "n": n, "leaf": leaf, "tol": tol, "L": st.L, "max_rank": st.max_rank,
        "B1_max_rank": b1s.max_rank, "B2_max_rank": b2s.max_rank, **times,
        "matvec_cols": st.matvec_cols, "rmatvec_cols": st.rmatvec_cols,
        "rel_err_vs_fp64": err, "rows_checked": int(len(sel)),
        "rel_err_vs_B1B2": err_bb, "fp64_reference_s": ref_s,
        "phase_ms": {k: v["ms"] for k, v in prof.items()}}), flush=True)
    F.close()
    B1.close()
    B2.close()


def copy_calibration():
    """Three dispatches of a plain 1 GiB device-to-device copy (torch copy_)."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_dispatch": a.numel() * 4}), flush=True)


def profile_value(name, key):
    """A figure from a committed rocprofv3 summary under profiles/, if it was
    taken on the current black-box kernel source (else None)."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2002_03400_amd", "csrc", "matfree.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line)
    if vals.get("source_sha256 paper_2002_03400_amd/csrc/matfree.hip", "").strip() != sha:
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per launch of the black-box kernel (byte counters)."""
    return profile_value("matfree_segkernel_n65536_hbm_bytes.md", "traffic_bytes_per_launch")


def measured_valu_per_entry():
    """Vector-ALU lane-instructions per kernel entry of the black-box kernel."""
    return profile_value("matfree_segkernel_n65536_valu_mfma.md", "valu_instr_per_entry")


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f, c = math.floor(k), math.ceil(k)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def error_rows(geom, nrows):
    """FP64 oracle reference of the error check: sampled rows of A times 16
    Gaussian test columns (Sec. 6 error measure), computed once per operator."""
    import workloads as wl
    from oracle import operators as ops
    n = geom.sources.shape[0]
    Om = wl.test_columns(n, 16, 1001)
    rows = np.sort(np.random.default_rng(0).choice(n, min(nrows, n), replace=False))
    ref = ops.segment_kernel_entries(geom.targets, geom.sources, geom.k, rows=rows) @ Om
    return Om, rows, ref


def sampled_err(F_gpu, chk):
    """Relative error of a GPU factorization on the oracle's sampled rows."""
    import torch
    Om, rows, ref = chk
    got = F_gpu.apply(torch.from_numpy(Om.astype(np.complex64)).cuda()).cpu().numpy()[rows]
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(geom, args, passes):
    """The FP64 oracle on the host: (a) its construction time at the benchmark
    size estimated from a timed slice of its black-box product (the dominant
    cost of Alg. 2: every adaptive pass and every sweep level evaluates all
    m*n kernel entries once), (b) a whole oracle construction (Alg. 2 end to
    end) timed at n = 1024, leaf 32, tol 1e-6 for scale."""
    import workloads as wl
    from oracle import butterfly as obf
    from oracle import operators as ops

    n = args.n
    # (a) the oracle's matvec on row slices of one pass (s = 40 columns)
    op = ops.SegmentKernelOp(geom.targets, geom.sources, geom.k)
    X = wl.test_columns(n, 40, 7)
    slice_rows = 512
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < args.cpu_seconds and done < n:
        r0 = done
        r1 = min(n, r0 + slice_rows)
        _ = ops.segment_kernel_entries(op.t, op.s, op.k, rows=slice(r0, r1)) @ X
        done = r1
    t = time.perf_counter() - t0
    per_pass = t * n / done
    est = per_pass * passes
    # (b) a complete oracle construction at n = 1024
    g1 = wl.segment_pair(1024, ppw=args.ppw)
    op1 = ops.SegmentKernelOp(g1.targets, g1.sources, g1.k)
    t0 = time.perf_counter()
    obf.construct(op1, 1e-6, 32, seed=1)
    c1_s = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas = 1
    return {
        "value": 1.0 / est, "unit": "factorizations/s", "cores": int(blas),
        "kind": "oracle",
        "sample": (f"oracle FP64 black-box product of {done} of {n} rows of one pass "
                   f"(s=40 columns) in {t:.1f}s, x{n / done:.0f} rows x {passes} passes "
                   f"(the construction's adaptive iterations + sweep levels); "
                   f"elementwise numpy single-threaded, BLAS {blas} threads; "
                   f"host cores {os.cpu_count()}"),
        "est_seconds_per_factorization": est,
        "cpu_model": cpu_model(),
        "oracle_construction_n1024_s": c1_s,
    }


def apply_roofline(bf, F, n, reps=20, sizes=(1, 4, 16, 64)):
    """bf_apply of the given factors (default arithmetic) at `sizes` right-hand
    sides: algorithmic bytes (8 per factor entry + 8 per input and output
    value) over the device time of an apply, against the HBM peak.  The device
    time is one pair of HIP events on the apply's stream around `reps`
    back-to-back applies, queued while a spin kernel holds the stream so that
    the host's launch cost does not leave the device idle between them (events
    around every launch would add a few microseconds each, the launches being
    only a few microseconds long); the sum of per-launch event times is
    reported beside it, and the host wall time per apply launched directly and
    as one captured HIP graph."""
    import torch
    out = {}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # spin-kernel cycles per millisecond on this device
    torch.cuda._sleep(1000)
    e0.record()
    torch.cuda._sleep(20_000_000)
    e1.record()
    torch.cuda.synchronize()
    cyc_per_ms = 20_000_000 / max(e0.elapsed_time(e1), 1e-3)
    for s in sizes:
        X = torch.randn(n, s, dtype=torch.complex64, device="cuda")
        Y = F.apply(X)
        F.apply(X, out=Y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.apply(X, out=Y)
        torch.cuda.synchronize()
        host_ms = (time.perf_counter() - t0) * 1e3
        torch.cuda._sleep(int(cyc_per_ms * (2.0 * reps * host_ms + 2.0)))
        e0.record()
        for _ in range(reps):
            F.apply(X, out=Y)
        e1.record()
        torch.cuda.synchronize()
        kms = e0.elapsed_time(e1) / reps
        bf.profile_start()
        t0 = time.perf_counter()
        for _ in range(reps):
            F.apply(X, out=Y)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        ap = bf.profile_stop()["apply"]
        gbs = ap["bytes"] / reps / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
        # the same applies as one captured HIP graph each (bf_set_apply_graph_cols)
        F.set_graph_cols(64)
        F.apply(X, out=Y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            F.apply(X, out=Y)
        torch.cuda.synchronize()
        gwall = (time.perf_counter() - t0) / reps
        F.set_graph_cols(0)
        out[f"s={s}"] = {"kernel_ms": kms, "launch_event_sum_ms": ap["ms"] / reps,
                         "wall_ms": wall * 1e3, "graph_wall_ms": gwall * 1e3,
                         "bytes": ap["bytes"] / reps, "GB_per_s": gbs,
                         "frac_hbm": gbs / PEAK_HBM_GBS,
                         "TFLOP_per_s": ap["flops"] / reps / (kms * 1e-3) / 1e12 if kms > 0 else 0.0,
                         "launches": ap["launches"] // reps}
    return out


def c5_apply(bf, n=262144, leaf=16, tol=1e-6):
    """The precision-form workload's butterfly (1D Fourier integral operator,
    n = 262144, leaf 16, tol 1e-6, built matrix-free with the split-BF16 black
    box) and its apply roofline at 1, 4 and 16 right-hand sides."""
    import torch
    op = bf.fio(n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = bf.construct(op, tol, leaf, seed=5)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = F.stats()
    out = {"workload": f"1D Fourier integral operator butterfly, n={n}, leaf {leaf}, tol {tol:g}",
           "construct_s": dt, "L": st.L, "max_rank": st.max_rank,
           "factor_GB": 8.0 * st.factor_entries / 1e9,
           "apply": apply_roofline(bf, F, n, reps=10, sizes=(1, 4, 16))}
    F.close()
    op.close()
    return out


def run_served(bf, reqs, slots, leaf, keep_all=False, batch_cols=0, rounds=False,
               max_constructs=0):
    """Replay a request stream in real time through the request engine.
    Returns (server, wall seconds, [latency s of constructions], [latency s of
    applies], [borrowed factors of every construction] if keep_all else [])."""
    import torch

    import workloads as wl
    S = bf.Server(slots=slots, batch_cols=batch_cols, solve_rounds=rounds,
                  max_constructs=max_constructs)
    ops_ = {}
    tickets = {}
    start = time.perf_counter()
    for i, r in enumerate(reqs):
        now = time.perf_counter() - start
        if r.t > now:
            time.sleep(r.t - now)
        if r.kind == "construct":
            key = (r.n, r.ppw)
            if key not in ops_:
                g = wl.segment_pair(r.n, ppw=r.ppw)
                ops_[key] = bf.segkernel(g.targets, g.sources, g.k)
            op = ops_[key]
            tickets[i] = S.submit_construct(op, r.tol, leaf, seed=r.seed)
        else:
            n = reqs[r.target].n
            X = torch.randn(n, r.nrhs, dtype=torch.complex64, device="cuda")
            tickets[i] = S.submit_apply(tickets[r.target], X)
    lat_c, lat_a = [], []
    merged = 0
    for i, r in enumerate(reqs):
        info = S.wait(tickets[i])
        (lat_c if r.kind == "construct" else lat_a).append(
            (info["finish_ns"] - info["arrival_ns"]) * 1e-9)
        merged += r.kind != "construct" and info["batch"] > 1
    S.merged_applies = merged
    wall = time.perf_counter() - start
    kept = []
    if keep_all:
        kept = [S.factors(tickets[i]) for i, r in enumerate(reqs) if r.kind == "construct"]
    return S, wall, lat_c, lat_a, kept


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the build targets a single MI355X)", file=sys.stderr)
        sys.exit(2)
    if run_mode(args):
        if args.save_tune:
            import paper_2002_03400_amd as bf
            bf.autotune_save(args.save_tune)
        return
    headline(args)


def run_mode(args):
    """The measurement modes other than the headline line; True if one ran."""
    if args.copy_calibration:
        copy_calibration()
        return True
    if args.apply_burst:
        apply_burst(args)
        return True
    if args.variants:
        variants([int(x) for x in args.variants.split(",")])
        return True
    if args.precision_form:
        precision_form(args.precision_form)
        return True
    if args.compose:
        compose(args.compose)
        return True
    if args.em3d:
        em3d([tuple(int(x) for x in e.split(":")) for e in args.em3d.split(",")],
             [float(t) for t in args.em3d_tols.split(",")])
        return True
    if args.exact_scaling:
        cases = []
        for e in args.exact_scaling.split(","):
            f = [int(x) for x in e.split(":")]
            cases.append((f[0], f[1], f[2]) if len(f) == 3 else (f[0], 8, 8))
        exact_scaling(cases)
        return True
    return False


def headline(args):
    import torch

    import paper_2002_03400_amd as bf
    import workloads as wl

    torch.cuda.init()
    geom = wl.segment_pair(args.n, ppw=args.ppw)
    op = bf.segkernel(geom.targets, geom.sources, geom.k)
    global TWO_SIDES
    TWO_SIDES = not args.one_stream
    for w in range(args.warmup):
        bf.construct(op, args.tol, args.leaf, seed=10_000 + w, two_sides=TWO_SIDES).close()
    torch.cuda.synchronize()

    lat = []
    last = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ta = time.perf_counter()
        F = bf.construct(op, args.tol, args.leaf, seed=3 + k, two_sides=TWO_SIDES)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ta)
        if last is not None:
            last.close()
        last = F
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total = t1 - t0
    info = last.stats()
    # kernel roofline and phase split: further constructions of the same
    # workload on one stream, each kernel timed by its own HIP events with no
    # other kernel sharing the device (the two sides of the timed loop run
    # their black-box launches side by side, which stretches each launch)
    bf.profile_start()
    torch.cuda.synchronize()
    for k in range(args.roofline_steps):
        bf.construct(op, args.tol, args.leaf, seed=3 + args.steps + k, two_sides=False).close()
    torch.cuda.synchronize()
    prof = bf.profile_stop()
    passes = info.v_iters + info.u_iters + info.L

    per_request_fs = args.steps / total
    chk = error_rows(geom, args.rows)
    rel_err = sampled_err(last, chk)

    # served closed loop: all K requests submitted at once, `slots` in flight;
    # every served factorization is checked against the oracle rows
    import workloads as wl
    reqs = [wl.Request(0.0, "construct", args.n, args.ppw, args.tol, 3 + k) for k in range(args.steps)]
    S, wall, lat_c, _, kept = run_served(bf, reqs, args.served_slots, args.leaf, keep_all=True,
                                         rounds=bool(args.solve_rounds))
    served_fs = args.steps / wall
    served_errs = [sampled_err(Fk, chk) for Fk in kept]
    S.close()
    streams = None
    if args.stream > 0:
        cap = max(served_fs, per_request_fs)
        streams = {}
        # the same streams again with at most 2 constructions at once
        # (bf_server_opts.max_constructs): latency against throughput
        for cap_c, suffix in ((0, ""), (2, "_max2")):
            if cap_c and (args.max_constructs_line == 0 or cap_c >= args.slots):
                continue
            for mult in (0.5, 1.0, 2.0):
                reqs = wl.poisson_stream(args.stream, mult * cap, n=args.n, ppw=args.ppw,
                                         tol=args.tol)
                S, wall_s, lat_s, _, _ = run_served(bf, reqs, args.slots, args.leaf,
                                                    rounds=bool(args.solve_rounds),
                                                    max_constructs=cap_c)
                S.close()
                streams[f"{mult:g}x{suffix}"] = {
                    "requests": args.stream, "rate_per_s": mult * cap, "wall_s": wall_s,
                    "max_constructs": cap_c,
                    "p50_ms": 1e3 * pct(lat_s, 50), "p99_ms": 1e3 * pct(lat_s, 99),
                    "completed_per_s": args.stream / wall_s}
    mix = None
    if args.mix > 0:
        reqs = wl.mixed_stream(args.mix, rate=args.mix_rate)
        mix = {"requests": args.mix, "rate_per_s": args.mix_rate,
               "constructions": sum(r.kind == "construct" for r in reqs),
               "applies": sum(r.kind != "construct" for r in reqs)}
        # served: `slots` device slots with continuous batching of applies;
        # per-request path: one slot, every request its own launches (its two
        # sides on two streams, as in the closed loop)
        for name, slots, bc in (("served", args.slots, args.batch_cols), ("per_request", 1, 0)):
            S, wall_m, lat_mc, lat_ma, _ = run_served(bf, reqs, slots, args.leaf, batch_cols=bc,
                                                      rounds=bool(args.solve_rounds) and slots > 1)
            S.close()
            mix[name] = {"slots": slots, "batch_cols": bc, "wall_s": wall_m,
                         "solve_rounds": bool(args.solve_rounds) and slots > 1,
                         "factorizations_per_s": len(lat_mc) / wall_m,
                         "construct_p50_ms": 1e3 * pct(lat_mc, 50),
                         "construct_p99_ms": 1e3 * pct(lat_mc, 99),
                         "apply_p50_ms": 1e3 * pct(lat_ma, 50),
                         "apply_p99_ms": 1e3 * pct(lat_ma, 99),
                         "merged_applies": S.merged_applies}

    cpu = None if args.no_cpu_baseline else cpu_baseline_leg(geom, args, passes)
    apply_rl = apply_roofline(bf, last, args.n)
    c5 = None if args.no_c5 else c5_apply(bf)

    mf = prof["matfree"]
    # algorithmic work of the black-box launches: 8 flops per complex
    # multiply-add of every sampled column with every kernel entry of its
    # segment (counted by the library per launch), over their event time
    mac_tflops = mf["flops"] / (mf["ms"] * 1e-3) / 1e12 if mf["ms"] > 0 else 0.0
    # every launch of this workload (sample widths <= 80, one column chunk)
    # evaluates each of the m*n kernel entries once
    evals_per_s = mf["launches"] * float(args.n) * args.n / max(1e-30, mf["ms"] * 1e-3)
    vpe = measured_valu_per_entry()
    out = {
        "metric": METRIC,
        "value": max(per_request_fs, served_fs),
        "unit": "factorizations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "p50_ms": 1e3 * pct(lat, 50),
        "p99_ms": 1e3 * pct(lat, 99),
        "per_request_fs": per_request_fs,
        "served_fs": served_fs,
        "served_p50_ms": 1e3 * pct(lat_c, 50),
        "served_p99_ms": 1e3 * pct(lat_c, 99),
        "slots": args.served_slots,
        "stream_slots": args.slots,
        "two_sides": TWO_SIDES,
        "solve_rounds": bool(args.solve_rounds),
        "poisson_streams": streams,
        "mixed_stream": mix,
        "rel_err": rel_err,
        "served_rel_err_max": max(served_errs) if served_errs else None,
        "served_checked": len(served_errs),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (bf16x3 MFMA, f64 accumulate) + f64 solves",
        "data": "synthetic",
        "config": {
            "workload": (f"segment-kernel exp(ikr)/r, two parallel unit segments at distance 1, "
                         f"n=m={args.n}, {args.ppw:g} points/wavelength, leaf {args.leaf}, "
                         f"tol {args.tol:g}, p=2, r0=4, closed-loop stream of constructions"),
            "n": args.n, "leaf": args.leaf, "tol": args.tol, "ppw": args.ppw,
            "L": info.L, "max_rank": info.max_rank,
            "matvec_cols": info.matvec_cols, "rmatvec_cols": info.rmatvec_cols,
            "factor_MB": info.factor_entries * 16 / 1e6,
        },
        "roofline": {
            "kernel": "matfree_bf16_kernel<SegEntry> (black-box products, split-BF16 MFMA)",
            "bound": "mfma",
            "achieved": mac_tflops,
            "peak": PEAK_BF16_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": mac_tflops / PEAK_BF16_MFMA_TFLOPS,
            "work": ("algorithmic complex multiply-adds of the black-box products, 8 flops each, "
                     "per launch over the launch's HIP-event time; peak = MI355X dense BF16 "
                     "matrix-core rate"),
            "flops_per_launch": mf["flops"] / max(1, mf["launches"]),
            "entry_evals_per_s": evals_per_s,
            "valu_instr_per_entry": vpe,
            "valu_issue_frac": evals_per_s * vpe / VALU_LANE_INSTR_PER_S if vpe else None,
            "mfma_busy_frac": profile_value("matfree_segkernel_n65536_valu_mfma.md",
                                            "mfma_busy_frac"),
            "traffic": measured_traffic(),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1)",
            "algorithmic_bytes_per_launch": mf["bytes"] / max(1, mf["launches"]),
            "avg_launch_ms": mf["ms"] / max(1, mf["launches"]),
            "launches": mf["launches"],
        },
        "phase_ms_per_step": {k: v["ms"] / max(1, args.roofline_steps) for k, v in prof.items()},
        "roofline_steps": args.roofline_steps,
        "apply_roofline": apply_rl,
        "apply_roofline_c5": c5,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if args.save_tune:
        bf.autotune_save(args.save_tune)


if __name__ == "__main__":
    main()
