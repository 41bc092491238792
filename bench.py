#!/usr/bin/env python3
"""Benchmark: ADMM LP decoding of the (3,6)-regular n=2640 code on one MI355X.

One step decodes one batch: 4096 frames at each of Eb/N0 = 1.5, 2.0, 2.5, 3.0 dB
(16384 frames, BPSK over AWGN, all-zero codeword, mu = 3, rho = 1.9, t_max =
1000, eps = 1e-5) in a single call of the library's batched form.  LLRs are
generated once and are resident in HBM before the timed region.

Printed: one JSON line with the decoded throughput (coded Mbit/s), the
roofline of the dominant kernel, the oracle's CPU baseline on a bounded
sample, and the plain (one frame per launch sequence) and streamed (state in
HBM) forms for comparison.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1]
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

METRIC = "decoded Mbit/s + HBM GB/s % at n=2640, batched vs plain; serving p99 latency"
HBM_PEAK_GBS = 8000.0
# Non-packed FP32 VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_PEAK_GOPS = 256 * 64 * 2.4
FRAMES_PER_SNR = 4096


def algorithmic_bytes_per_frame_iter(H) -> int:
    """HBM bytes one ADMM iteration of one frame must move when the replicas z and
    scaled duals u live in HBM: read and write z, u (16 B per edge) and read gamma."""
    return 16 * H.nnz + 4 * H.n


def algorithmic_ops_per_frame_iter(H) -> int:
    """FP32 operations of one iteration in the branch-free formulation the kernels
    implement (each add/mul/fma/min/max/med3/compare-select counts one):
      per edge   9  (w = z-u; q, v; dual; two residual terms)
      per check  13 d + 2 S_d + 2 M_d + 9  (projection: clip/sum, parity, sorting
                 network of S_d comparators, f_r^T zhat, thresholds, breakpoints,
                 bitonic merge of M_d comparators, prefix averages, final clip)
      per variable  d_v + 3  (slot sum, gamma/mu, scale, clip)"""
    S = {2: 1, 3: 3, 4: 5, 5: 9, 6: 12, 7: 16, 8: 19}
    M = {2: 1, 3: 4, 4: 4, 5: 12, 6: 12, 7: 12, 8: 12}
    cd = H.check_degrees()
    vd = H.var_degrees()
    ops = 9 * H.nnz
    ops += int(sum(13 * d + 2 * S[int(d)] + 2 * M[int(d)] + 9 for d in cd))
    ops += int(np.sum(vd + 3))
    return ops


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="auto", choices=["auto", "resident", "persistent_global", "streamed"])
    ap.add_argument("--cpu-frames", type=int, default=512, help="oracle sample size (frames)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the plain and streamed comparisons")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py decodes on one GPU only: frames are independent, so a multi-GPU run is frame "
              "sharding with no exchange on the hot path; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": a.numel() * 4, "launches": 3}))
        return

    import paper_1204_0556_amd as lp
    import workloads as W

    modes = {"auto": lp.MODE_AUTO, "resident": lp.MODE_RESIDENT,
             "persistent_global": lp.MODE_PERSISTENT_GLOBAL, "streamed": lp.MODE_STREAMED}
    P = W.PAPER_PARAMS
    H = W.gallager36(2640)
    llr_h = np.concatenate([W.awgn_batch(H, FRAMES_PER_SNR, s) for s in W.HEADLINE_SNRS])
    F = llr_h.shape[0]
    dev = torch.device("cuda:0")
    llr = torch.from_numpy(llr_h).to(dev)
    code = lp.Code(H)
    out = (torch.empty((F, H.n), dtype=torch.float32, device=dev),
           torch.empty(F, dtype=torch.int32, device=dev), torch.empty(F, dtype=torch.uint8, device=dev))
    mode = modes[args.form]
    stream = torch.cuda.current_stream()

    def step():
        lp.decode(code, llr, out=out, mode=mode, **P)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = max(gpu_ms, wall * 1e3 / args.steps)

    x, it, fl = (t.cpu().numpy() for t in out)
    iters = it.astype(np.int64)
    value = F * H.n / (ms_per_step / 1e3) / 1e6
    rank = W.gf2_rank(H)
    k_info = H.n - rank
    B = algorithmic_bytes_per_frame_iter(H)
    ops = algorithmic_ops_per_frame_iter(H)
    frame_iters = int(iters.sum())
    kernel_s = gpu_ms / 1e3
    form = "resident" if args.form in ("auto", "resident") and code.info["resident_capable"] else args.form
    if form == "auto":
        form = "persistent_global"
    fer = {}
    for b, s in enumerate(W.HEADLINE_SNRS):
        sl = slice(b * FRAMES_PER_SNR, (b + 1) * FRAMES_PER_SNR)
        errs = int(np.sum((x[sl] >= 0.5).any(axis=1)))
        fer[str(s)] = {"frame_errors": errs, "fer": errs / FRAMES_PER_SNR,
                       "mean_iters": float(iters[sl].mean())}

    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "ADMM LP decoding (Alg. 1 + over-relaxation), (3,6)-regular LDPC n=2640 m=1320 "
                        "(Gallager, seed-fixed), BPSK/AWGN Eb/N0 1.5/2.0/2.5/3.0 dB x 4096 frames, "
                        "mu=3 rho=1.9 max_iter=1000 tol=1e-5, one batched call",
            "frames": F, "n": H.n, "nnz": H.nnz, "form": form,
            "threads_per_frame": code.info["threads_per_frame"],
        },
        "info_mbit_s": round(F * k_info / (ms_per_step / 1e3) / 1e6, 2),
        "mean_iterations": round(float(iters.mean()), 2),
        "frame_iterations_per_s": round(frame_iters / (ms_per_step / 1e3), 1),
        "fer": fer,
        "hbm_equivalent_gbs": round(B * frame_iters / (ms_per_step / 1e3) / 1e9, 1),
    }
    if form == "resident":
        achieved = ops * frame_iters / kernel_s / 1e9
        res["roofline"] = {"bound": "alu", "achieved": round(achieved / 1e3, 3), "peak": round(VALU_PEAK_GOPS / 1e3, 2),
                           "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_GOPS, 4), "traffic": None,
                           "kernel": "k_decode (resident)", "ops_per_frame_iter": ops,
                           "kernel_ms": round(gpu_ms, 3), "launches_per_step": 1}
    else:
        achieved = B * frame_iters / kernel_s / 1e9
        res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                           "kernel": f"k_decode ({form})", "bytes_per_frame_iter": B,
                           "kernel_ms": round(gpu_ms, 3)}

    if not args.no_extra:
        # streamed form over the same batch: state in HBM, one launch per iteration
        lp.decode(code, llr, out=out, mode=lp.MODE_STREAMED, **P)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lp.decode(code, llr, out=out, mode=lp.MODE_STREAMED, **P)
        e1.record(stream)
        torch.cuda.synchronize()
        sms = e0.elapsed_time(e1)
        sit = out[1].cpu().numpy().astype(np.int64)
        sfi = int(sit.sum())
        sach = B * sfi / (sms / 1e3) / 1e9
        res["streamed"] = {"mbit_s": round(F * H.n / (sms / 1e3) / 1e6, 2), "ms": round(sms, 3),
                           "launches": int(sit.max()), "hbm_achieved_gbs": round(sach, 1),
                           "hbm_frac": round(sach / HBM_PEAK_GBS, 4), "bytes_per_frame_iter": B}
        # plain: one frame per launch sequence (streamed form, batch of one), sampled
        sample = np.concatenate([b * FRAMES_PER_SNR + np.arange(8) for b in range(len(W.HEADLINE_SNRS))])
        one = [(torch.empty((1, H.n), dtype=torch.float32, device=dev),
                torch.empty(1, dtype=torch.int32, device=dev), torch.empty(1, dtype=torch.uint8, device=dev))
               for _ in sample]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, f in enumerate(sample):
            lp.decode(code, llr[f:f + 1], out=one[k], mode=lp.MODE_STREAMED, **P)
        torch.cuda.synchronize()
        pt = time.perf_counter() - t0
        pit = np.array([o[1].item() for o in one])
        res["plain"] = {"mbit_s": round(len(sample) * H.n / pt / 1e6, 3), "frames": int(len(sample)),
                        "form": "streamed, batch of 1", "mean_iterations": round(float(pit.mean()), 1),
                        "batched_over_plain": round(value / (len(sample) * H.n / pt / 1e6), 1)}

    if not args.no_cpu:
        import oracle
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        per = max(1, args.cpu_frames // len(W.HEADLINE_SNRS))
        sample = np.concatenate([b * FRAMES_PER_SNR + np.arange(per) for b in range(len(W.HEADLINE_SNRS))])
        t0 = time.perf_counter()
        ref = oracle.decode(H, llr_h[sample], nthreads=cores, **P)
        ct = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(len(sample) * H.n / ct / 1e6, 3), "unit": "Mbit/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{len(sample)} frames ({per} per Eb/N0, same LLRs), FP64 C oracle, "
                                         f"{ct:.1f} s, mean iterations {ref.iters.mean():.1f}"}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
