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


KERNEL_SOURCES = ("paper_1204_0556_amd/csrc/lpdec_kernels.hip", "paper_1204_0556_amd/csrc/lpdec_internal.h")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(name: str, field: str = "traffic_bytes_per_launch"):
    """HBM bytes per launch of the decoder kernel from the committed counter summary
    profiles/<name>.md (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration),
    or None when the summary is missing or was taken from other kernel sources."""
    path = os.path.join(ROOT, "profiles", name + ".md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("    ") and ":" in line:
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return int(fields[field])
    except (KeyError, ValueError):
        return None


def run_serving(lp, W, seconds: float, seed: int = 0, budget_bytes: int = 512 << 20):
    """Replay a seeded Poisson trace in real time through the continuous-batching
    server: mean 50k frames/s, 1..256 frames per request, codes n in
    {96, 576, 2640, 8064, 16384}, Eb/N0 ~ U[1.5, 3.5] dB per request."""
    import threading

    Hs = [W.gallager36(96), W.irregular_half(576), W.gallager36(2640), W.irregular_half(8064),
          W.gallager36(16384)]
    codes = [lp.Code(H) for H in Hs]
    trace = W.serving_trace(Hs, duration_s=seconds, frames_per_s=50_000.0, max_frames=256, seed=seed)
    srv = lp.Server(codes, budget_bytes=budget_bytes, max_batch_frames=4096, max_inflight=4)
    # warm the kernels (module load, first-launch costs) outside the measurement
    for c, H in enumerate(Hs):
        srv.wait(srv.submit(c, W.awgn_batch(H, 2, 3.0, tag="warm")), timeout=120.0)
    base = srv.stats()
    tickets = []
    t0 = time.perf_counter()

    def submitter():
        for r in trace:
            dt = r.arrival_s - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets.append(srv.submit(r.code, r.llr))

    th = threading.Thread(target=submitter)
    th.start()
    lat = []
    k = 0
    while k < len(trace):
        if k < len(tickets):
            lat.append(srv.wait(tickets[k], timeout=300.0)[3])
            k += 1
        else:
            time.sleep(0.0005)
    th.join()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = np.array(lat)
    bits = sum(r.frames * Hs[r.code].n for r in trace)
    return {
        "requests": len(trace), "frames": int(sum(r.frames for r in trace)), "trace_seconds": seconds,
        "offered_mbit_s": round(bits / seconds / 1e6, 1), "delivered_mbit_s": round(bits / wall / 1e6, 1),
        "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "max_latency_ms": round(float(lat.max()) * 1e3, 3),
        "peak_admitted_bytes": int(st["peak_bytes"]), "budget_bytes": budget_bytes,
        "launches": int(st["launches"] - base["launches"]),
    }


def workload_serving(args, lp, W):
    sv = run_serving(lp, W, args.serving_seconds if args.serving_seconds > 0 else 3.0)
    return {
        "metric": METRIC, "value": sv["p99_latency_ms"], "unit": "ms (p99 latency)", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": sv["trace_seconds"] * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals, mean 50k frames/s, 1-256 frames per request, "
                               "codes n in {96,576,2640,8064,16384} rate 1/2, Eb/N0 U[1.5,3.5] dB, "
                               "HBM-admitted, codes resident, FP32"},
        "serving": sv,
    }


def workload_uneven(args, lp, W, torch):
    """16384 frames drawn from six irregular rate-1/2 codes in one persistent launch."""
    codes_h = [W.irregular_half(n) for n in W.IRREGULAR_LENGTHS]
    batch = W.mixed_batch(codes_h, 16384, 1.5, 3.0, tag="uneven")
    flat, off = batch.flat_llr()
    codes = [lp.Code(H) for H in codes_h]
    dev_llr = torch.from_numpy(flat).cuda()
    P = W.PAPER_PARAMS

    def step():
        return lp.decode_multi(codes, batch.code_of_frame, off, dev_llr, off, flat.size, **P)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        x, it, fl = step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    it = it.cpu().numpy().astype(np.int64)
    bits = int(sum(codes_h[c].n for c in batch.code_of_frame))
    ops = sum(algorithmic_ops_per_frame_iter(codes_h[c]) * int(it[f]) for f, c in enumerate(batch.code_of_frame))
    achieved = ops / (ms / 1e3) / 1e9
    byt = sum(algorithmic_bytes_per_frame_iter(codes_h[c]) * int(it[f]) for f, c in enumerate(batch.code_of_frame))
    return {
        "metric": METRIC, "value": round(bits / (ms / 1e3) / 1e6, 2), "unit": "Mbit/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched uneven: 16384 frames from 6 irregular rate-1/2 codes n in "
                               "{576,1152,2304,4608,6912,8064} (variable degrees {2,3,6}, check degrees "
                               "{6,7,8}), Eb/N0 U[1.5,3] dB per frame, one persistent launch", "frames": 16384},
        "mean_iterations": round(float(it.mean()), 2),
        "hbm_equivalent_gbs": round(byt / (ms / 1e3) / 1e9, 1),
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e3, 3), "peak": round(VALU_PEAK_GOPS / 1e3, 2),
                     "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_GOPS, 4), "traffic": None,
                     "kernel": "k_decode (persistent-global, degrees 2..8)"},
    }


def workload_precision(args, lp, W, torch):
    """FP16 versus FP32 message storage (streamed form) on the two n = 16384 codes."""
    import oracle
    out = {}
    P = W.PAPER_PARAMS
    for name, H in (("(3,6) n=16384", W.gallager36(16384)), ("(4,8) n=16384", W.gallager48(16384))):
        llr_h = W.awgn_batch(H, 8192, 2.5, tag="precision")
        llr = torch.from_numpy(llr_h).cuda()
        code = lp.Code(H)
        res = {}
        for sname, st in (("fp32", lp.STORAGE_FP32), ("fp16", lp.STORAGE_FP16)):
            x, it, fl = lp.decode(code, llr, mode=lp.MODE_STREAMED, storage=st, **P)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, it, fl = lp.decode(code, llr, mode=lp.MODE_STREAMED, storage=st, **P)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            it_h = it.cpu().numpy().astype(np.int64)
            B = (16 if st == lp.STORAGE_FP32 else 8) * H.nnz + 4 * H.n
            res[sname] = {"mbit_s": round(8192 * H.n / dt / 1e6, 1), "ms": round(dt * 1e3, 2),
                          "mean_iterations": round(float(it_h.mean()), 2),
                          "hbm_gbs": round(B * int(it_h.sum()) / dt / 1e9, 1),
                          "hbm_frac": round(B * int(it_h.sum()) / dt / 1e9 / HBM_PEAK_GBS, 4),
                          "frame_errors": int(((x >= 0.5).any(dim=1)).sum().item()),
                          "hard": (x >= 0.5).cpu().numpy()}
        agree = float(np.mean(np.all(res["fp16"]["hard"] == res["fp32"]["hard"], axis=1)))
        for v in res.values():
            v.pop("hard")
        # error against the FP64 oracle after K iterations (stopping disabled), sampled frames
        K, S = 50, 16
        ref = oracle.decode(H, llr_h[:S], max_iter=K, tol=0.0, state=True)
        errs = {}
        for sname, st in (("fp32", lp.STORAGE_FP32), ("fp16", lp.STORAGE_FP16)):
            x, _, _, z, u = lp.decode_state(code, llr[:S].contiguous(), mode=lp.MODE_STREAMED, storage=st,
                                            tol=0.0, max_iter=K, mu=P["mu"], rho=P["rho"])
            torch.cuda.synchronize()
            errs[sname] = {"max_abs_x": float(np.abs(x.cpu().numpy() - ref.x).max()),
                           "max_abs_lambda": float(P["mu"] * np.abs(u.cpu().numpy() - ref.u).max())}
        out[name] = {"throughput": res, "hard_decision_agreement_fp16_vs_fp32": agree,
                     f"error_vs_oracle_after_{K}_iterations_{S}_frames": errs}
    v = out["(3,6) n=16384"]["throughput"]["fp16"]["mbit_s"]
    return {
        "metric": METRIC, "value": v, "unit": "Mbit/s (FP16 storage, (3,6) n=16384)", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": out["(3,6) n=16384"]["throughput"]["fp16"]["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16 storage / f32 compute", "data": "synthetic",
        "config": {"workload": "precision: (3,6) and (4,8) regular n=16384, 8192 frames at 2.5 dB, streamed "
                               "form, FP16 vs FP32 message/dual storage"},
        "precision": out,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="auto", choices=["auto", "resident", "persistent_global", "streamed"])
    ap.add_argument("--cpu-frames", type=int, default=4096, help="oracle sample size (frames)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the plain and streamed comparisons")
    ap.add_argument("--workload", default="headline", choices=["headline", "uneven", "precision", "serving"])
    ap.add_argument("--serving-seconds", type=float, default=1.0,
                    help="length of the serving trace folded into the headline line (0: skip)")
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

    if args.workload == "serving":
        print(json.dumps(workload_serving(args, lp, W)))
        return
    if args.workload == "uneven":
        print(json.dumps(workload_uneven(args, lp, W, torch)))
        return
    if args.workload == "precision":
        print(json.dumps(workload_precision(args, lp, W, torch)))
        return

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
                           "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_GOPS, 4),
                           "traffic": profiled_traffic("k_decode_resident_n2640_headline"),
                           "kernel": "k_decode (resident)", "ops_per_frame_iter": ops,
                           "kernel_ms": round(gpu_ms, 3), "launches_per_step": 1}
    else:
        achieved = B * frame_iters / kernel_s / 1e9
        res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": profiled_traffic(f"k_decode_{form}_n2640_headline"),
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
                           "algorithmic_bytes": B * sfi,
                           "traffic_bytes": profiled_traffic("k_decode_streamed_n2640_headline",
                                                             "traffic_bytes_per_decode"),
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

    if args.serving_seconds > 0 and not args.no_extra:
        res["serving"] = run_serving(lp, W, args.serving_seconds)

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
