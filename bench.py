#!/usr/bin/env python3
"""Benchmark of the w-product hot path on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input:
  * w-product forward + backward of A, B in R^{512x512x256} (N(0,1)), L = 4,
    with the split-precision (bf16x3) face-products: forward lifting of A and B
    with the hi/lo epilogue, the face-product, the inverse lifting, then
    W^{-T} of the cotangent, the two transposed face-products and two W^T
    passes (9 kernels);
  * w-svd, k = 20, L = 3, of a 256x256x192 hyperspectral-like tensor
    (lifting, Jacobi, rank-k rebuild, inverse lifting, FP64 orthogonality check).
`value` is the effective w-product forward+backward rate, 3 * 2*n1*n2*n3*p
flops divided by the w-product part of the step (HIP events on the stream
the kernels run on).  FP32 and plain BF16 forward+backward are timed beside it
outside the timed steps.  Prints one JSON line.

With --sp-w-svd it instead compares w-svd and sp-w-svd (Sec. IV-B) on a
256x192x96 hyperspectral-like cube at L = 5; --pinv-deblur times the
pseudo-inverse deblurring of Sec. IV-C; --schemes the lifting with chosen
predict / update stencils; --table1 the p x p x p w-products of Table 1;
--configs the other workloads.  Each prints its own JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--sp-w-svd | --pinv-deblur | --schemes | --table1 | --configs]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

P, N1, N2, N3, LEV = 256, 512, 512, 512, 4
SVD_P, SVD_N, SVD_L, SVD_K = 192, 256, 3, 20
# Table 3 shape (Sec. IV-B): 256x192x96 hyperspectral cubes, L = 5.
T3_N1, T3_N2, T3_P, T3_L, T3_RANKS = 256, 192, 96, 5, (2, 8, 32, 64)
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFS = 2500.0          # dense BF16 MFMA
N_CUS = 256                 # MI355X compute units
FP32_PEAK_TFS = 157.3
# FP32 vector arithmetic without packed (two-wide) instructions, which this
# build does not emit: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
FP32_VALU_UNPACKED_TFS = 78.6
FP64_VALU_PEAK_TFS = 78.6


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing leg (used by profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--sp-w-svd", action="store_true",
                    help="instead of the step: w-svd against sp-w-svd on 256x192x96, L=5")
    ap.add_argument("--table1", action="store_true",
                    help="instead of the step: w-product of p x p x p tensors, p = 2 .. 1024 "
                         "(the shapes of the paper's Table 1), L = log2 p")
    ap.add_argument("--pinv-deblur", action="store_true",
                    help="instead of the step: pseudo-inverse deblurring (Sec. IV-C) of "
                         "PaviaU-, Salinas- and Botswana-shaped hyperspectral-like cubes, FP64")
    ap.add_argument("--schemes", action="store_true",
                    help="instead of the step: lifting with chosen predict / update stencils "
                         "(lazy, interpolating, CDF 5/3) on 512x512x256 FP32, passes and "
                         "bf16x3 w-product")
    ap.add_argument("--configs", action="store_true",
                    help="instead of the step: the other workloads (FP64 small case, config-3 "
                         "PSNR, 1024x1024x128 precision modes, 50-step deblurring solve)")
    return ap.parse_args()


class Marks:
    """Records one event after each library call of a step, on the current stream."""

    def __init__(self, torch):
        self.torch = torch
        self.rows = []  # per step: list of (name, start_event, end_event)
        self.cur = None
        self.last = None

    def begin(self):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record()
        self.cur = []
        self.last = ev

    def __call__(self, name):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record()
        self.cur.append((name, self.last, ev))
        self.last = ev

    def end(self):
        self.rows.append(self.cur)

    def per_kernel_ms(self):
        """Mean duration of each named call over all recorded steps (ms, summed per step)."""
        tot = {}
        cnt = {}
        for row in self.rows:
            seen = {}
            for name, a, b in row:
                seen[name] = seen.get(name, 0.0) + a.elapsed_time(b)
                cnt[name] = cnt.get(name, 0) + 1
            for k, v in seen.items():
                tot[k] = tot.get(k, 0.0) + v
        n = len(self.rows)
        return {k: v / n for k, v in tot.items()}, {k: cnt[k] // n for k in cnt}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus %d is not supported "
                          "(the w-product shards over whole 2^L-slice blocks with no exchange, "
                          "see the design notes)" % args.gpus}))
        sys.exit(2)

    import torch
    import paper_2601_08228_amd as wp
    from paper_2601_08228_amd import synth, _lib
    from paper_2601_08228_amd.autograd import forward_kernels, backward_kernels

    _lib.load()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.sp_w_svd:
        sparse_report(torch, wp, synth, dev, args)
        return
    if args.configs:
        configs_report(torch, wp, synth, dev, args)
        return
    if args.table1:
        table1_report(torch, wp, dev, args)
        return
    if args.pinv_deblur:
        deblur_report(torch, wp, synth, dev, args)
        return
    if args.schemes:
        schemes_report(torch, wp, synth, dev, args)
        return

    a = synth.normal_device((P, N1, N2), 21, dev)
    b = synth.normal_device((P, N2, N3), 22, dev)
    g = synth.normal_device((P, N1, N3), 102, dev)
    x_hsi = torch.tensor(synth.hsi_like(SVD_N, SVD_N, SVD_P, seed=3), dtype=torch.float32,
                         device=dev)
    svd_ws = torch.empty(wp.w_svd_workspace(SVD_N, SVD_N, SVD_P, SVD_L, SVD_K), dtype=torch.uint8,
                         device=dev)

    marks = Marks(torch)

    def wprod_step(gemm, mark):
        c, saved = forward_kernels(a, b, LEV, gemm, mark)
        da, db = backward_kernels(saved, g, LEV, gemm, mark=mark)
        return c, da, db

    jac_events = []  # per timed step: (begin, end) events around the Jacobi stage

    def step():
        marks.begin()
        out = wprod_step("bf16x3", marks)
        j0 = torch.cuda.Event(enable_timing=True)
        j1 = torch.cuda.Event(enable_timing=True)
        res = wp.w_svd_timed(x_hsi, SVD_L, SVD_K, j0, j1, workspace=svd_ws)
        jac_events.append((j0, j1))
        marks("w_svd")
        marks.end()
        return out, res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    marks.rows.clear()
    jac_events.clear()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    kern_ms, kern_cnt = marks.per_kernel_ms()
    wprod_ms = sum(v for k, v in kern_ms.items() if k != "w_svd")
    flops = 2.0 * N1 * N2 * N3 * P
    value = 3.0 * flops / (wprod_ms * 1e-3) / 1e12
    info = res.info.cpu().numpy()
    orth = res.orth_err.cpu().numpy()
    c_x3, da_x3, db_x3 = out

    # ---- comparisons outside the timed steps: FP32 and plain BF16 fwd+bwd ----
    def time_mode(gemm, reps=5):
        wprod_step(gemm, lambda n: None)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            o = wprod_step(gemm, lambda n: None)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, o

    fp32_ms, (c32, da32, db32) = time_mode("native")
    bf16_ms, (c16, _, _) = time_mode("bf16")

    def rel(x, y):
        return float(torch.linalg.vector_norm((x - y).double()) / torch.linalg.vector_norm(y.double()))

    rel_x3_fp32 = max(rel(c_x3, c32), rel(da_x3, da32), rel(db_x3, db32))
    rel_bf16_fp32 = rel(c16, c32)

    if args.copy_calibration:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        torch.cuda.synchronize()

    # ---- roofline of every kernel of the step --------------------------------
    tensor_b = P * N1 * N2 * 4            # one 512x512x256 FP32 tensor
    bytes_per = {
        "lift_fwd_split": tensor_b + tensor_b,          # read FP32, write bf16 hi + lo
        "lift_inv": 2 * tensor_b,
        "lift_inv_adj_split": 2 * tensor_b,
        "lift_fwd_adj": 2 * tensor_b,
    }
    rows = {}
    for name, ms in kern_ms.items():
        launches = kern_cnt[name]
        per_launch_ms = ms / launches
        if name in bytes_per:
            ach = bytes_per[name] / (per_launch_ms * 1e-3) / 1e9
            rows[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                          "launches_per_step": launches, "ms_per_launch": round(per_launch_ms, 4),
                          "algorithmic_bytes_per_launch": bytes_per[name]}
        elif name.startswith("face"):
            # Both ceilings: three BF16 products per effective product on the
            # matrix cores, and the bytes a launch must move (hi + lo parts of
            # both operands read, the FP32 product written).  On this shape the
            # bytes take longer at the HBM peak than the flops at the MFMA
            # peak, so HBM is the binding bound.
            peak = BF16_PEAK_TFS / 3.0
            face_bytes = 4 * P * N1 * N2 + 4 * P * N2 * N3 + 4 * P * N1 * N3
            t_flops = flops / (peak * 1e12)
            t_bytes = face_bytes / (HBM_PEAK_GBS * 1e9)
            ach_f = flops / (per_launch_ms * 1e-3) / 1e12
            ach_b = face_bytes / (per_launch_ms * 1e-3) / 1e9
            mfma = {"achieved": round(ach_f, 2), "peak": round(peak, 1), "unit": "TFLOP/s",
                    "frac": round(ach_f / peak, 4), "algorithmic_flops_per_launch": flops}
            hbm = {"achieved": round(ach_b, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(ach_b / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": face_bytes}
            if t_bytes >= t_flops:
                rows[name] = dict(bound="hbm", **hbm, mfma=mfma)
            else:
                rows[name] = dict(bound="mfma", **mfma, hbm=hbm)
            rows[name].update(launches_per_step=launches, ms_per_launch=round(per_launch_ms, 4))
    # The Jacobi kernel dominates the step.  Algorithmic work per pair visit of
    # a one-sided Jacobi sweep: 6 mr flops for the two norms and the inner
    # product, 6 mr for rotating the two columns of W and 6 nc for rotating
    # the two columns of V, so (12 mr + 6 nc) nc (nc - 1) / 2 flops per
    # slice-sweep, times the sweeps each slice ran.  The kernel forms no V
    # (the second factor is recovered afterwards) and runs nc_pad pair rounds
    # per sweep (one more than the tournament needs): 12 mr flops per executed
    # pair, reported beside.  Duration: the events w_svd_timed records around
    # the Jacobi stage, on the stream the kernel runs on.
    sweeps_total = int(np.abs(info).sum())
    mr, nc = SVD_N, SVD_N
    nc_pad = nc + (nc & 1)
    jac_flops = (12.0 * mr + 6.0 * nc) * (nc * (nc - 1) / 2) * sweeps_total
    jac_exec_flops = 12.0 * mr * (nc_pad // 2) * nc_pad * sweeps_total
    jac_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in jac_events]))
    jac_ach = jac_flops / (jac_ms * 1e-3) / 1e12
    jac_exec = jac_exec_flops / (jac_ms * 1e-3) / 1e12
    rows["w_svd"] = {"bound": "alu", "achieved": round(jac_ach, 2), "peak": FP32_PEAK_TFS,
                     "unit": "TFLOP/s", "frac": round(jac_ach / FP32_PEAK_TFS, 4),
                     "launches_per_step": 1, "ms_per_launch": round(jac_ms, 4),
                     "w_svd_call_ms": round(kern_ms["w_svd"], 4),
                     "algorithmic_flops_per_launch": jac_flops,
                     "slice_sweeps": sweeps_total,
                     "executed": {"achieved": round(jac_exec, 2),
                                  "frac": round(jac_exec / FP32_PEAK_TFS, 4),
                                  "flops_per_launch": jac_exec_flops},
                     "unpacked_fp32_ceiling": {"peak": FP32_VALU_UNPACKED_TFS,
                                               "frac": round(jac_ach / FP32_VALU_UNPACKED_TFS, 4),
                                               "executed_frac": round(
                                                   jac_exec / FP32_VALU_UNPACKED_TFS, 4)},
                     "note": "jacobi_reg_kernel: (12 mr + 6 nc) nc (nc-1)/2 flops per "
                             "slice-sweep x sweeps run; FP32 lane partials and FP32 cross-lane "
                             "sums, FP64 rotation parameters, FP32 rotations; duration from "
                             "events around the Jacobi stage of each w_svd call"}
    traffic = measured_traffic()
    for name, row in rows.items():
        row["traffic"] = traffic.get(name)
    dom_name = max(rows, key=lambda k: kern_ms[k])
    roof = dict(rows[dom_name])
    roof["kernel"] = "jacobi_reg_kernel<float,4,16> (w_svd)" if dom_name == "w_svd" else dom_name

    # ---- CPU baseline: the oracle on a bounded sample of the same workload ----
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(torch, a, b, g, {"bf16x3": (c_x3, da_x3, db_x3),
                                            "fp32": (c32, da32, db32)}, x_hsi, res)

    line = {
        "metric": "w-product fwd+bwd effective TFLOP/s (bf16x3 face-products, 512x512x256, L=4)",
        "value": round(value, 2),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3",
        "data": "synthetic",
        "config": {
            "workload": "w-product fwd+bwd, A,B 512x512x256 N(0,1), L=4, bf16x3 "
                        "+ w-svd k=20 of a 256x256x192 hyperspectral-like tensor, L=3",
            "w_product": {"n1": N1, "n2": N2, "n3": N3, "p": P, "L": LEV, "gemm": "bf16x3"},
            "w_svd": {"n1": SVD_N, "n2": SVD_N, "p": SVD_P, "L": SVD_L, "k": SVD_K},
        },
        "parts_ms": {"w_product_fwd_bwd": round(wprod_ms, 4), "w_svd": round(kern_ms["w_svd"], 4)},
        "kernel_ms_per_step": {k: round(v, 4) for k, v in kern_ms.items()},
        "fp32_fwd_bwd_ms": round(fp32_ms, 4),
        "bf16_fwd_bwd_ms": round(bf16_ms, 4),
        "bf16x3_fwd_bwd_ms": round(wprod_ms, 4),
        "bf16x3_speedup_vs_fp32": round(fp32_ms / wprod_ms, 3),
        "rel_diff_bf16x3_vs_fp32": rel_x3_fp32,
        "rel_diff_bf16_vs_fp32": rel_bf16_fp32,
        "w_svd_sweeps": [int(info.min()), int(info.max())],
        "w_svd_orth_err": [float(orth[0]), float(orth[1])],
        "roofline": roof,
        "roofline_kernels": rows,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def sparse_report(torch, wp, synth, dev, args):
    """w-svd against sp-w-svd (Sec. IV-B) on the Table 3 cube shape, one JSON line.

    256x192x96 hyperspectral-like FP32 tensor, L = 5 (m = 3: sp-w-svd decomposes
    the 6 slices of s_5 and d_5, w-svd all 96), ranks 2, 8, 32, 64.  Each call
    is timed with HIP events on the current stream (mean of `--steps` calls
    after `--warmup`); the FP64 oracle of both is timed on the host for context.
    """
    import oracle
    x = torch.tensor(synth.hsi_like(T3_N1, T3_N2, T3_P, seed=31), dtype=torch.float32,
                     device=dev)
    x_h = x.double().cpu().numpy()
    reps = max(args.steps, 1)

    def time_call(fn):
        for _ in range(max(args.warmup, 1)):
            r = fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, r

    def rel(x_, ref):
        return float(np.linalg.norm((x_ - ref).ravel()) / np.linalg.norm(ref.ravel()))

    rows, cpu_ms = {}, {}
    for rk in T3_RANKS:
        full_ms, rf = time_call(lambda: wp.w_svd(x, T3_L, rk))
        sp_ms, rs = time_call(lambda: wp.w_svd_sparse(x, T3_L, rk))
        t0 = time.perf_counter()
        _, _, _, ak_full = oracle.w_svd(x_h, T3_L, rk)
        t1 = time.perf_counter()
        _, _, _, ak_sp = oracle.w_svd_sparse(x_h, T3_L, rk)
        t2 = time.perf_counter()
        ak_f = rf.ak.double().cpu().numpy()
        ak_s = rs.ak.double().cpu().numpy()
        rows[str(rk)] = {
            "w_svd_ms": round(full_ms, 4), "sp_w_svd_ms": round(sp_ms, 4),
            "sp_speedup_vs_w_svd": round(full_ms / sp_ms, 3),
            "w_svd_sweeps_max": int(rf.info.max().item()),
            "sp_w_svd_sweeps_max": int(rs.info.max().item()),
            "converged": bool(rf.info.min().item() > 0 and rs.info.min().item() > 0),
            "psnr_w_svd_db": round(float(oracle.psnr(x_h, ak_f)), 3),
            "psnr_sp_w_svd_db": round(float(oracle.psnr(x_h, ak_s)), 3),
            "rel_err_vs_oracle": {"w_svd_Ak": rel(ak_f, ak_full), "sp_w_svd_Ak": rel(ak_s, ak_sp)},
        }
        cpu_ms[str(rk)] = {"w_svd": round((t1 - t0) * 1e3, 1), "sp_w_svd": round((t2 - t1) * 1e3, 1)}
    _, rs32 = time_call(lambda: wp.w_svd_sparse(x, T3_L, 32))
    sp_flops = jacobi_flops(rs32.info.cpu().numpy(), T3_N1, T3_N2)
    sp_ms = rows["32"]["sp_w_svd_ms"]
    # Block Jacobi geometry of the call: blocks of 16 columns (8 beyond 1024
    # rows), an even block count, one workgroup per block pair and slice.
    sp_mr, sp_nc = max(T3_N1, T3_N2), min(T3_N1, T3_N2)
    sp_b = 16 if sp_mr <= 1024 else 8
    sp_nbp = -(-sp_nc // sp_b)
    sp_nbp += sp_nbp % 2
    sp_wgs = (sp_nbp // 2) * 2 * (T3_P >> T3_L)
    # The paper's Table 3 at the ranks measured here: t-svd, w-svd and sp-w-svd
    # seconds for its three images (Coffee, Sugar-Salt-Flour, Yatsuhashi).
    paper_t3 = {"2": ([5.0527, 5.1041, 5.0454], [0.8583, 0.8642, 0.8646], [0.0548, 0.0631, 0.0641]),
                "8": ([5.1427, 5.1191, 5.1430], [0.8808, 0.8871, 0.8898], [0.0783, 0.0730, 0.0795]),
                "32": ([5.1278, 5.1361, 5.1695], [0.9026, 0.8968, 0.8980], [0.0674, 0.0802, 0.0796]),
                "64": ([5.1108, 5.1562, 5.1286], [0.8961, 0.9006, 0.9035], [0.0802, 0.0732, 0.0753])}
    paper_table3 = {
        "note": "the paper's own CPU timings (s) on three 256x192x96 NIR images (" + PAPER_HOST +
                "); context only, the t-svd is not built here",
        "by_rank": {rk: {"t_svd_s": t, "w_svd_s": w, "sp_w_svd_s": sp,
                         "w_svd_speedup_vs_t_svd": [round(a / b, 2) for a, b in zip(t, w)],
                         "sp_w_svd_speedup_vs_t_svd": [round(a / b, 2) for a, b in zip(t, sp)]}
                    for rk, (t, w, sp) in paper_t3.items()}}
    line = {
        "metric": "sp-w-svd and w-svd time (FP32, 256x192x96 hyperspectral-like, L=5)",
        "value": rows["32"]["sp_w_svd_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sp-w-svd vs w-svd, 256x192x96 hyperspectral-like tensor "
                               "(12 components, noise 0.01), L=5, ranks 2/8/32/64; value at rank 32",
                   "n1": T3_N1, "n2": T3_N2, "p": T3_P, "L": T3_L},
        "ranks": rows,
        "paper_table3": paper_table3,
        "roofline": {"bound": "alu", "achieved": round(sp_flops / sp_ms / 1e9, 2),
                     "peak": FP32_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": round(sp_flops / sp_ms / 1e9 / FP32_PEAK_TFS, 4), "traffic": None,
                     "kernel": "bj_round_kernel<float, 16, 8> (block Jacobi, 6 slices)",
                     "algorithmic_flops_per_call": sp_flops,
                     "workgroups_per_launch": sp_wgs,
                     "frac_of_occupied_cus": round(sp_flops / sp_ms / 1e9 / FP32_PEAK_TFS
                                                   * N_CUS / min(N_CUS, sp_wgs), 4),
                     "note": "12*mr flops per pair visit times the sweeps of each slice; "
                             "duration = whole sp-w-svd call at rank 32; the 6 slices give "
                             "the block Jacobi one workgroup per block pair, so a launch "
                             "occupies workgroups_per_launch of the 256 CUs and the call is "
                             "bound by its chain of dependent sub-rounds"},
        "cpu_baseline": {
            "value": cpu_ms["32"]["sp_w_svd"], "unit": "ms", "cores": host_threads(),
            "kind": "oracle",
            "sample": "FP64 NumPy oracle of the same calls on the whole tensor (ms per call, "
                      "by rank)",
            "ms": cpu_ms},
    }
    print(json.dumps(line), flush=True)


# Sec. IV-C deblurring problems, Table 4 shapes and levels:
# (name, n1, n2, p, L, the paper's w-product and sp-w-product times in s).
DEBLUR_CASES = [("PaviaU", 610, 340, 102, 1, 9.8508, 9.7492),
                ("Salinas", 512, 217, 204, 2, 10.9848, 6.5197),
                ("Botswana", 1476, 256, 144, 4, 40.5728, 7.3428)]
# The same table's t-product times (s) and the PSNRs it reports (t-product, w-product).
PAPER_TABLE4_T = {"PaviaU": (23.6328, 21.1510, 26.7206), "Salinas": (31.4715, 17.6921, 23.6444),
                  "Botswana": (204.7620, 34.4265, 36.7636)}
DEBLUR_B = 10


def deblur_report(torch, wp, synth, dev, args):
    """Pseudo-inverse deblurring X = A_V^+ *_w B *_w (A_H^T)^+ (Sec. IV-C), FP64.

    Per case: a hyperspectral-like cube X of the image's shape, the linear
    blur (b = 10) stacked over the bands, B = A_V *_w X *_w A_H^T built on the
    GPU outside the timed region; then the whole deblurring (two w_pinv, two
    w_product calls) timed with HIP events, full and sparse (sp-w-product),
    with a per-call breakdown.  Checked on sampled coarse coefficient slices
    against a direct solve with the blur matrices.  The FP64 oracle of the
    PaviaU sparse deblurring is timed on the host for context.
    """
    import oracle
    from paper_2601_08228_amd import deblur
    reps = max(args.steps, 1)

    def ev_ms(fn):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, r

    def rel(x_, ref):
        return float(np.linalg.norm((x_ - ref).ravel()) / np.linalg.norm(ref.ravel()))

    def psnr(x_, ref):
        return float(10.0 * np.log10(np.max(ref) ** 2 / np.mean((x_ - ref) ** 2)))

    cases = {}
    cpu = None
    for name, n1, n2, p, L, paper_w, paper_sp in DEBLUR_CASES:
        tv = synth.toeplitz_blur(n1, DEBLUR_B)
        th = synth.toeplitz_blur(n2, DEBLUR_B)
        av = torch.from_numpy(synth.stack_slices(tv, p)).to(dev)
        ah = torch.from_numpy(synth.stack_slices(th, p)).to(dev)
        x_true = synth.hsi_like(n1, n2, p, seed=41)
        xt = torch.from_numpy(x_true).to(dev)
        bt = wp.w_product(wp.w_product(av, xt, L), ah, L, trans_b=True)
        torch.cuda.synchronize()
        row = {"n1": n1, "n2": n2, "p": p, "L": L}
        for sparse in (False, True):
            key = "sp_w_product" if sparse else "w_product"
            ms, (x, (iv, ih)) = ev_ms(lambda: deblur.pinv_deblur(bt, av, ah, L, sparse=sparse))
            # Breakdown of one call.
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            ev[0].record()
            pv, _ = wp.w_pinv(av, L, sparse=sparse)
            ev[1].record()
            ph, _ = wp.w_pinv(ah, L, sparse=sparse)
            ev[2].record()
            t = wp.w_product(pv, bt, L)
            ev[3].record()
            wp.w_product(t, ph, L, trans_b=True)
            ev[4].record()
            torch.cuda.synchronize()
            xs = x.cpu().numpy()
            xhat = oracle.lift_fwd(xs, L)
            bhat = oracle.lift_fwd(bt.cpu().numpy(), L)
            errs = []
            for c in (0, (p >> L) // 2, (p >> L) - 1):
                want = np.linalg.solve(tv, np.linalg.solve(th, bhat[c].T).T)
                errs.append(rel(xhat[c], want))
            jf = jacobi_flops(iv.cpu().numpy(), n1, n1) + jacobi_flops(ih.cpu().numpy(), n2, n2)
            row[key] = {
                "ms": round(ms, 3),
                "jacobi_flops": jf,
                "jacobi_TFLOPs_over_call": round(jf / ms / 1e9, 3),
                "pinv_av_ms": round(ev[0].elapsed_time(ev[1]), 3),
                "pinv_ah_ms": round(ev[1].elapsed_time(ev[2]), 3),
                "w_products_ms": round(ev[2].elapsed_time(ev[4]), 3),
                "jacobi_sweeps_max": int(max(iv.max().item(), ih.max().item())),
                "converged": bool(min(iv.min().item(), ih.min().item()) > 0),
                "psnr_db": round(psnr(xs, x_true), 3),
                "coarse_rel_err_vs_solve_max": max(errs),
                "paper_s": paper_sp if sparse else paper_w,
            }
        row["psnr_blurred_db"] = round(psnr(bt.cpu().numpy(), x_true), 3)
        cases[name] = row
        if name == "PaviaU" and not args.no_cpu_baseline:
            av_h, ah_h, bt_h = av.cpu().numpy(), ah.cpu().numpy(), bt.cpu().numpy()
            t0 = time.perf_counter()
            x_o = oracle.pinv_deblur(bt_h, av_h, ah_h, L, sparse=True)
            cpu = {"ms": round((time.perf_counter() - t0) * 1e3, 1),
                   "rel_err_gpu_vs_oracle": rel(x.cpu().numpy(), x_o)}
        del av, ah, xt, bt
        torch.cuda.empty_cache()
    line = {
        "metric": "pseudo-inverse deblurring time (FP64, sp-w-product, Salinas-shaped cube)",
        "value": cases["Salinas"]["sp_w_product"]["ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pseudo-inverse deblurring X = A_V^+ *_w B *_w (A_H^T)^+ of "
                               "hyperspectral-like cubes (12 components, noise 0.01) blurred by "
                               "the linear Toeplitz blur b = 10 stacked over the bands; "
                               "PaviaU 610x340x102 L=1, Salinas 512x217x204 L=2 and "
                               "Botswana 1476x256x144 L=4 shapes; "
                               "value: Salinas, sp-w-product",
                   "blur_b": DEBLUR_B},
        "cases": cases,
        "paper_table4": {
            "note": "the paper's own CPU timings on the real images (" + PAPER_HOST + "); "
                    "context only, the t-product is not built here",
            "cases": {name: {"t_product_s": PAPER_TABLE4_T[name][0], "w_product_s": pw,
                             "sp_w_product_s": ps,
                             "sp_w_product_speedup_vs_t_product": round(PAPER_TABLE4_T[name][0] / ps, 2),
                             "psnr_t_db": PAPER_TABLE4_T[name][1],
                             "psnr_w_db": PAPER_TABLE4_T[name][2]}
                      for name, _, _, _, _, pw, ps in DEBLUR_CASES}},
    }
    sal = cases["Salinas"]["sp_w_product"]
    line["roofline"] = {
        "bound": "alu", "achieved": sal["jacobi_TFLOPs_over_call"], "peak": FP64_VALU_PEAK_TFS,
        "unit": "TFLOP/s", "frac": round(sal["jacobi_TFLOPs_over_call"] / FP64_VALU_PEAK_TFS, 4),
        "traffic": None, "kernel": "bj_round_kernel<double, 16, 16> (block Jacobi)",
        "algorithmic_flops_per_call": sal["jacobi_flops"],
        "note": "12*mr flops per pair visit times the sweeps of each rotating slice of both "
                "blurs; duration = whole Salinas sp-w-product deblurring call"}
    if cpu is not None:
        line["cpu_baseline"] = {
            "value": cpu["ms"], "unit": "ms", "cores": host_threads(), "kind": "oracle",
            "sample": "FP64 NumPy oracle of the PaviaU sparse deblurring, whole cube, one call",
            "rel_err_gpu_vs_oracle": cpu["rel_err_gpu_vs_oracle"]}
    print(json.dumps(line), flush=True)


def schemes_report(torch, wp, synth, dev, args):
    """Lifting with chosen predict / update stencils (Sec. II-A; Remark 3.1).

    On the w-product operands of the step (512x512x256 FP32 N(0,1), L = 4):
    each pass of the lazy, interpolating (Example 2.1) and CDF 5/3 stencils
    against the lazy kernels, as ms and HBM GB/s (read once, written once),
    and the bf16x3 w-product under each scheme.  Passes are checked against
    the FP64 oracle on 2048 sampled tubes; the oracle's forward pass is timed
    on the host on a tensor of the same shape.
    """
    import oracle
    from paper_2601_08228_amd import schemes as sch
    reps = max(args.steps, 1)
    x = synth.normal_device((P, N1, N2), 21, dev)
    y = synth.normal_device((P, N2, N3), 22, dev)
    nbytes = 2 * x.numel() * 4

    def ev_ms(fn):
        for _ in range(max(args.warmup, 1)):
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

    named = {"lazy": sch.lazy(LEV), "interpolating": sch.interpolating(LEV),
             "cdf53": sch.cdf53(LEV)}
    rng = np.random.default_rng(5)
    cols = rng.choice(N1 * N2, size=2048, replace=False)
    xs = x.reshape(P, -1)[:, torch.as_tensor(cols, device=dev)].double().cpu().numpy()
    rows = {}
    lazy_kernels = {"forward": wp.w_transform, "inverse": wp.w_itransform,
                    "adj": wp.w_transform_adj, "iadj": wp.w_itransform_adj}
    rows["lazy_kernels"] = {k: {"ms": round(ev_ms(lambda: f(x, LEV)), 4)}
                            for k, f in lazy_kernels.items()}
    for k in rows["lazy_kernels"].values():
        k["GBps"] = round(nbytes / k["ms"] / 1e6, 1)
    fwd_ms = {}
    for name, taps in named.items():
        r = {}
        for kind in ("forward", "inverse", "adj", "iadj"):
            ms = ev_ms(lambda: wp.w_transform_scheme(x, LEV, taps, kind))
            out = wp.w_transform_scheme(x, LEV, taps, kind)
            got = out.reshape(P, -1)[:, torch.as_tensor(cols, device=dev)].double().cpu().numpy()
            ref = {"forward": oracle.lift_fwd_scheme, "inverse": oracle.lift_inv_scheme,
                   "adj": oracle.lift_fwd_scheme_adj,
                   "iadj": oracle.lift_inv_scheme_adj}[kind](xs, LEV, taps)
            err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            r[kind] = {"ms": round(ms, 4), "GBps": round(nbytes / ms / 1e6, 1),
                       "hbm_frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 3),
                       "rel_err_sampled_tubes": err}
            if kind == "forward":
                fwd_ms[name] = ms
        pm = ev_ms(lambda: wp.w_product_scheme(x, y, LEV, taps, gemm="bf16x3"))
        r["w_product_bf16x3_ms"] = round(pm, 4)
        r["w_product_bf16x3_TFLOPs"] = round(2.0 * N1 * N2 * N3 * P / pm / 1e9, 1)
        rows[name] = r
    lazy_prod = ev_ms(lambda: wp.w_product(x, y, LEV, gemm="bf16x3"))
    rows["lazy_kernels"]["w_product_bf16x3_ms"] = round(lazy_prod, 4)
    cpu = None
    if not args.no_cpu_baseline:
        # Host oracle on a sample (forward CDF 5/3 pass).
        sample = synth.normal((P, N1, N2), 23)
        t0 = time.perf_counter()
        oracle.lift_fwd_scheme(sample, LEV, named["cdf53"])
        cpu_s = time.perf_counter() - t0
        cpu = {"value": round(2 * sample.size * 4 / cpu_s / 1e9, 3), "unit": "GB/s",
               "cores": host_threads(), "kind": "oracle",
               "sample": "FP64 NumPy oracle CDF 5/3 forward pass on a 256x512x512 tensor "
                         "(FP32-equivalent bytes, %.2f s)" % cpu_s}
    ms = fwd_ms["cdf53"]
    line = {
        "metric": "lifting-scheme pass HBM throughput (CDF 5/3 forward, FP32, 512x512x256, L=4)",
        "value": round(nbytes / ms / 1e6, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lifting passes with chosen predict / update stencils (lazy, "
                               "interpolating, CDF 5/3) on a 512x512x256 N(0,1) FP32 tensor, "
                               "L=4, and the bf16x3 w-product 512x512x512 per slice x 256 under "
                               "each scheme; value: CDF 5/3 forward pass",
                   "p": P, "n1": N1, "n2": N2, "L": LEV},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / ms / 1e6, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 3), "traffic": None,
                     "kernel": "lift_scheme_kernel<float, kForward>",
                     "algorithmic_bytes": nbytes},
        "schemes": rows,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


# The paper's Table 1 w-product times (seconds, CPU, mean of 10 runs), p = 2^1 .. 2^10.
PAPER_TABLE1_W_S = [1.576734e-04, 1.577830e-04, 3.587484e-04, 4.789996e-04, 1.763617e-03,
                    8.662295e-03, 5.306451e-02, 3.919755e-01, 3.161437e+00, 7.749125e+01]
# The same table's t-product times (seconds), for the paper's own t / w ratio.
PAPER_TABLE1_T_S = [2.240753e-04, 3.964186e-04, 4.737735e-04, 6.299186e-04, 2.113118e-03,
                    1.014814e-02, 7.131300e-02, 5.213821e-01, 4.842443e+00, 1.574944e+02]
# Where the paper's timings were taken (Sec. III): context only.
PAPER_HOST = "the paper's setup: Python 3.11 on an Intel Core i9-12900K (16 cores), CPU only"


def table1_report(torch, wp, dev, args):
    """w-product of A, B in R^{p x p x p}, U[0,1) entries, p = 2^1 .. 2^10, L = log2 p
    (the worst case the paper names for Table 1), FP32 and bf16x3 face-products.
    Each call (one library call: both liftings, the face-products, the inverse) is
    timed with HIP events, mean of `--steps` calls after one warm-up.  Both
    results are checked against the FP64 oracle: the whole product for
    p <= 256, 16 sampled tubes (row i of A, column j of B) above.
    """
    import oracle

    def sampled_err(a, b, c, e):
        rng = np.random.default_rng(e)
        got, ref = [], []
        for i, j in zip(rng.integers(0, a.shape[1], 16), rng.integers(0, b.shape[2], 16)):
            arow = a[:, i:i + 1, :].double().cpu().numpy()
            bcol = b[:, :, j:j + 1].double().cpu().numpy()
            ref.append(oracle.w_product(arow, bcol, e)[:, 0, 0])
            got.append(c[:, i, j].double().cpu().numpy())
        got, ref = np.array(got), np.array(ref)
        return float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))

    rows = []
    for e in range(1, 11):
        p = 1 << e
        g = torch.Generator(device=dev)
        g.manual_seed(1000 + e)
        a = torch.rand((p, p, p), generator=g, device=dev)
        b = torch.rand((p, p, p), generator=g, device=dev)
        row = {"p": p, "L": e, "paper_cpu_w_product_s": PAPER_TABLE1_W_S[e - 1],
               "paper_cpu_t_product_s": PAPER_TABLE1_T_S[e - 1],
               "paper_t_over_w": round(PAPER_TABLE1_T_S[e - 1] / PAPER_TABLE1_W_S[e - 1], 2)}
        ref = None
        if p <= 256:
            t0 = time.perf_counter()
            ref = oracle.w_product(a.double().cpu().numpy(), b.double().cpu().numpy(), e)
            row["oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
        for gemm in ("native", "bf16x3"):
            ws = torch.empty(max(wp.w_product_workspace(p, p, p, p, e, torch.float32, gemm), 1),
                             dtype=torch.uint8, device=dev)
            c = torch.empty_like(a)
            wp.w_product(a, b, e, gemm=gemm, out=c, workspace=ws)
            torch.cuda.synchronize()
            reps = max(args.steps, 1)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                wp.w_product(a, b, e, gemm=gemm, out=c, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            key = "fp32" if gemm == "native" else "bf16x3"
            row[key + "_ms"] = round(ms, 5)
            row[key + "_effective_tflops"] = round(2.0 * p ** 4 / (ms * 1e-3) / 1e12, 4)
            if gemm == "native":
                row["speedup_vs_paper_cpu"] = round(PAPER_TABLE1_W_S[e - 1] / (ms * 1e-3), 1)
            if ref is not None:
                got = c.double().cpu().numpy()
                row[key + "_rel_err_vs_oracle"] = float(np.linalg.norm((got - ref).ravel())
                                                        / np.linalg.norm(ref.ravel()))
            else:
                row[key + "_rel_err_vs_oracle_sampled"] = sampled_err(a, b, c, e)
            del ws, c
        rows.append(row)
        del a, b
        torch.cuda.empty_cache()
    top = rows[-1]
    eff = 2.0 * 1024 ** 4 / (top["bf16x3_ms"] * 1e-3) / 1e12
    line = {
        "metric": "w-product time of p x p x p tensors (the shapes of Table 1), L = log2 p",
        "value": top["bf16x3_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": max(args.steps, 1),
        "higher_is_better": False,
        "vs_baseline": None,
        "data": "synthetic U[0,1)",
        "config": {"workload": "w-product A *_w B, A, B p x p x p, p = 2..1024, L = log2 p, "
                               "FP32 and bf16x3 face-products"},
        "rows": rows,
        "roofline": {"bound": "mfma", "achieved": round(eff, 1), "peak": round(BF16_PEAK_TFS / 3, 1),
                     "unit": "TFLOP/s", "frac": round(eff / (BF16_PEAK_TFS / 3), 4),
                     "traffic": None,
                     "kernel": "face_bf16_direct (bf16x3), p = 1024: whole w_product call",
                     "note": "effective 2 p^4 flops per call; peak = BF16 dense MFMA / 3 products"},
        "cpu_baseline": {"value": rows[7]["oracle_ms"], "unit": "ms", "cores": host_threads(),
                         "kind": "oracle",
                         "sample": "FP64 NumPy oracle of the p = 256 product (one call); "
                                   "value is for p = 256, not the p = 1024 of `value`"},
        "note": "paper_cpu_w_product_s / paper_cpu_t_product_s are the paper's own CPU timings "
                "of the w-product and the t-product (Table 1; " + PAPER_HOST + "), context only; "
                "the t-product is not built here",
    }
    print(json.dumps(line), flush=True)


def configs_report(torch, wp, synth, dev, args):
    """The workloads beside the step, one JSON line (GPU timed with HIP events).

    * FP64 32x24x16 . 24x20x16, L=2: w-product and full-rank w-svd latency and
      errors; the oracle timed as the median of 20 calls, on all host threads
      and on one.
    * 256x256x192 hyperspectral-like tensor, L=3, k=20: PSNR of A_20 from the GPU
      and from the oracle.
    * 1024x1024x128 U(-1,1), L=3: w-product per face-product mode, against the
      whole FP64 oracle product.
    * Deblurring 256x256x128, L=3: 50 gradient steps through the adjoint (FP32
      and bf16x3 face-products), against the oracle trajectory.
    """
    import statistics
    import oracle
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # threadpoolctl missing: no one-thread figure
        threadpool_limits = None

    def ev_ms(fn, reps):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return statistics.median(times)

    def host_ms(fn, reps):
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            times.append((time.perf_counter() - t0) * 1e3)
        return statistics.median(times)

    def rel(x_, ref):
        return float(np.linalg.norm((np.asarray(x_, np.float64) - ref).ravel())
                     / np.linalg.norm(ref.ravel()))

    out = {}
    # FP64 small case
    a = synth.normal((16, 32, 24), seed=1)
    b = synth.normal((16, 24, 20), seed=2)
    ta = torch.tensor(a, device=dev)
    tb = torch.tensor(b, device=dev)
    c = wp.w_product(ta, tb, 2)
    res = wp.w_svd(ta, 2, 24)
    torch.cuda.synchronize()
    c_ref = oracle.w_product(a, b, 2)
    _, sh_ref, _, _ = oracle.w_svd(a, 2, 24)
    row = {
        "w_product_ms": round(ev_ms(lambda: wp.w_product(ta, tb, 2), 50), 4),
        "w_svd_ms": round(ev_ms(lambda: wp.w_svd(ta, 2, 24), 20), 4),
        "rel_err_C": rel(c.cpu().numpy(), c_ref),
        "rel_err_A_vs_U_S_Vt": rel(res.ak.cpu().numpy(), a),
        "rel_err_shat": rel(res.shat.cpu().numpy(), sh_ref),
        "orth_err": [float(v) for v in res.orth_err.cpu()],
        "oracle_w_product_ms": round(host_ms(lambda: oracle.w_product(a, b, 2), 20), 3),
        "oracle_w_svd_ms": round(host_ms(lambda: oracle.w_svd(a, 2, 24), 20), 3),
        "oracle_threads": host_threads(),
    }
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            row["oracle_w_product_ms_1_thread"] = round(host_ms(lambda: oracle.w_product(a, b, 2), 20), 3)
            row["oracle_w_svd_ms_1_thread"] = round(host_ms(lambda: oracle.w_svd(a, 2, 24), 20), 3)
    out["fp64_32x24x16_L2"] = row

    # config-3 PSNR
    x = synth.hsi_like(SVD_N, SVD_N, SVD_P, seed=3)
    x32 = x.astype(np.float32)
    res = wp.w_svd(torch.tensor(x32, device=dev), SVD_L, SVD_K)
    ak = res.ak.double().cpu().numpy()
    _, _, _, ak_ref = oracle.w_svd(x32.astype(np.float64), SVD_L, SVD_K)
    out["w_svd_256x256x192_L3_k20"] = {
        "psnr_gpu_db": round(float(oracle.psnr(x32, ak)), 4),
        "psnr_oracle_db": round(float(oracle.psnr(x32, ak_ref)), 4),
        "rel_err_Ak": rel(ak, ak_ref),
    }

    # precision modes at 1024x1024x128
    a = synth.uniform_device((128, 1024, 1024), 41, dev)
    b = synth.uniform_device((128, 1024, 1024), 42, dev)
    t0 = time.perf_counter()
    c_ref = oracle.w_product(a.double().cpu().numpy(), b.double().cpu().numpy(), 3)
    oracle_s = time.perf_counter() - t0
    flops = 2.0 * 1024 ** 3 * 128
    modes = {}
    for gemm in ("native", "bf16x3", "bf16"):
        ws = torch.empty(wp.w_product_workspace(1024, 1024, 1024, 128, 3, torch.float32, gemm),
                         dtype=torch.uint8, device=dev)
        cc = torch.empty((128, 1024, 1024), dtype=torch.float32, device=dev)
        ms = ev_ms(lambda: wp.w_product(a, b, 3, gemm=gemm, out=cc, workspace=ws), 10)
        modes["fp32" if gemm == "native" else gemm] = {
            "ms": round(ms, 4), "effective_tflops": round(flops / (ms * 1e-3) / 1e12, 2),
            "rel_err_vs_oracle": rel(cc.cpu().numpy(), c_ref)}
        del ws, cc
    out["w_product_1024x1024x128_L3"] = {"modes": modes, "oracle_s": round(oracle_s, 2)}
    del a, b, c_ref
    torch.cuda.empty_cache()

    # deblurring solve
    from paper_2601_08228_amd import deblur
    n, p, L, steps = 256, 128, 3, 50
    g = synth.gaussian_band(n)
    k = synth.stack_slices(g, p).astype(np.float32)
    xt = synth.hsi_like(n, n, p, seed=5)
    noise = synth.normal((p, n, n), seed=105, scale=0.01)
    y = (oracle.w_product(k, xt, L) + noise).astype(np.float32)
    eta = 1.0 / (2.0 * np.linalg.norm(g, 2) ** 2)
    t0 = time.perf_counter()
    x_ref, loss_ref = oracle.deblur_gd(k, y, L, steps, eta)
    oracle_s = time.perf_counter() - t0
    tk = torch.tensor(k, device=dev)
    ty = torch.tensor(y, device=dev)
    solves = {}
    for gemm in ("native", "bf16x3"):
        deblur.solve(tk, ty, L, 2, eta, gemm=gemm)  # warm-up
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        xs, losses = deblur.solve(tk, ty, L, steps, eta, gemm=gemm)
        e1.record()
        torch.cuda.synchronize()
        solver = deblur.GraphedSolver(tk, ty, L, eta, gemm=gemm)
        torch.cuda.synchronize()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record()
        xg = solver.run(steps)
        g1.record()
        torch.cuda.synchronize()
        solves["fp32" if gemm == "native" else gemm] = {
            "ms_per_step": round(e0.elapsed_time(e1) / steps, 4),
            "graphed_ms_per_step": round(g0.elapsed_time(g1) / steps, 4),
            "graphed_equals_eager": bool(torch.equal(xg, xs)),
            "loss_first": losses[0], "loss_last": losses[-1],
            "loss_rel_err_vs_oracle_max": max(abs(l1 - l2) / l2 for l1, l2 in zip(losses, loss_ref)),
            "rel_err_X50_vs_oracle": rel(xs.cpu().numpy(), x_ref)}
        del solver
    out["deblur_256x256x128_L3_50_steps"] = {"solves": solves, "oracle_s": round(oracle_s, 2),
                                             "eta": eta}
    line = {
        "metric": "workloads beside the step: FP64 small-case latency, w-svd PSNR, precision "
                  "modes at 1024x1024x128, 50-step deblurring",
        "n_gpus": 1,
        "data": "synthetic",
        "config": {"workload": "see keys"},
        "results": out,
    }
    print(json.dumps(line), flush=True)


def jacobi_flops(info, mr, nc):
    """Algorithmic flops of one-sided Jacobi: 12 * mr per pair visit (three dot
    products and the rotation), nc (nc - 1) / 2 pairs per sweep, summed over
    the slices that rotated (a slice that converged in its first sweep without
    a rotation, such as an all-zero slice, is not counted)."""
    sw = np.abs(np.asarray(info, dtype=np.int64))
    return float(12.0 * mr * (nc * (nc - 1) / 2) * sw[sw > 1].sum())


def host_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:  # threadpoolctl missing: report the visible cores
        return int(os.cpu_count())


def host_info():
    """CPU model, visible cores and the BLAS NumPy calls (for the oracle timings)."""
    info = {"cpu_count": os.cpu_count(), "cpu_model": None, "blas": None}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    info["cpu_model"] = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cfg = np.show_config(mode="dicts")
        blas = cfg.get("Build Dependencies", {}).get("blas", {})
        info["blas"] = "%s %s" % (blas.get("name", "?"), blas.get("version", ""))
    except Exception:  # older NumPy without the dict form
        pass
    return info


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary.

    FETCH_SIZE and WRITE_SIZE were taken in two runs of this benchmark and
    scaled by the counters of a plain copy; a kernel's figure is used only while
    its source file still has the hash recorded with it, otherwise None.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic_bench_step.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f)
    out = {}
    for name, k in rec.get("kernels", {}).items():
        src = os.path.join(ROOT, k["source"])
        if os.path.exists(src):
            with open(src, "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() == k["source_sha256"]:
                    out[name] = k["traffic_bytes"]
    return out


def cpu_baseline(torch, a, b, g, gpu_out, x_hsi, svd_res):
    """The FP64 oracle on the step's work, timed on the host cores.

    w-product forward + backward of the whole 512x512x256 pair (the metric's
    unit), then the w-svd of the same hyperspectral-like tensor.
    """
    import oracle
    rows = N1
    a_s = a[:, :rows, :].double().cpu().numpy()
    b_h = b.double().cpu().numpy()
    g_s = g[:, :rows, :].double().cpu().numpy()
    t0 = time.perf_counter()
    c_ref = oracle.w_product(a_s, b_h, LEV)
    da_ref, db_ref = oracle.w_product_vjp(a_s, b_h, g_s, LEV)
    t1 = time.perf_counter()
    sample_flops = 3.0 * 2.0 * rows * N2 * N3 * P
    x_h = x_hsi.double().cpu().numpy()
    t2 = time.perf_counter()
    _, sh_ref, _, ak_ref = oracle.w_svd(x_h, SVD_L, SVD_K)
    t3 = time.perf_counter()
    threads = host_threads()

    def rel(x, ref):
        return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))

    return {
        "value": round(sample_flops / (t1 - t0) / 1e12, 6),
        "unit": "TFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": "FP64 NumPy oracle: the step's whole w-product fwd+bwd (512x512x256 pair, "
                  "L=4) in %.1f s; w-svd of the 256x256x192 tensor in %.1f s"
                  % (t1 - t0, t3 - t2),
        "seconds": round(t1 - t0, 3),
        "w_svd_seconds": round(t3 - t2, 3),
        "host": host_info(),
        "rel_err_gpu_vs_oracle": dict(
            [(name + "_" + mode, rel(t.double().cpu().numpy(), ref))
             for mode, outs in gpu_out.items()
             for name, t, ref in zip(("C", "dA", "dB"), outs, (c_ref, da_ref, db_ref))]
            + [("w_svd_shat", rel(svd_res.shat.double().cpu().numpy(), sh_ref)),
               ("w_svd_Ak", rel(svd_res.ak.double().cpu().numpy(), ak_ref))]),
    }


if __name__ == "__main__":
    main()
