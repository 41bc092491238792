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
CODE313_SNRS = (3.0, 3.5, 4.0, 4.5)
FORM_NAMES = {1: "resident", 2: "streamed", 3: "persistent-global"}


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
    S = {2: 1, 3: 3, 4: 5, 5: 9, 6: 12, 7: 16, 8: 19, 9: 28, 10: 32, 11: 38, 12: 42, 13: 48, 14: 53, 15: 59,
         16: 63}
    M = {2: 1, 3: 4, 4: 4, 5: 12, 6: 12, 7: 12, 8: 12}
    M.update({d: 32 for d in range(9, 17)})
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
    """A figure of the committed counter summary profiles/<name>.md -- by default the
    HBM bytes per launch of the decoder kernel (FETCH_SIZE and WRITE_SIZE scaled by
    the copy calibration) -- or None when the summary is missing or was taken from
    other kernel sources."""
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


def run_serving(lp, W, seconds: float, seed: int = 0, budget_bytes: int = 2 << 30):
    """Replay a seeded Poisson trace in real time through the continuous-batching
    server: mean 50k frames/s, 1..256 frames per request, codes n in
    {96, 576, 2640, 8064, 16384}, Eb/N0 ~ U[1.5, 3.5] dB per request.  The budget
    bounds all of the server's device memory (the launch slots' scratch, sized for
    the n = 16384 code's full persistent grid, and the LLR arena)."""
    import threading

    Hs = [W.gallager36(96), W.irregular_half(576), W.gallager36(2640), W.irregular_half(8064),
          W.gallager36(16384)]
    codes = [lp.Code(H) for H in Hs]
    trace = W.serving_trace(Hs, duration_s=seconds, frames_per_s=50_000.0, max_frames=256, seed=seed)
    srv = lp.Server(codes, budget_bytes=budget_bytes, max_batch_frames=4096, max_inflight=8)
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
    by_code = {}
    for c, H in enumerate(Hs):
        lc = np.array([lat[i] for i, r in enumerate(trace) if r.code == c])
        if lc.size:
            by_code[str(H.n)] = {"requests": int(lc.size), "p50_ms": round(float(np.percentile(lc, 50)) * 1e3, 2),
                                 "p99_ms": round(float(np.percentile(lc, 99)) * 1e3, 2)}
    return {
        "requests": len(trace), "frames": int(sum(r.frames for r in trace)), "trace_seconds": seconds,
        "offered_mbit_s": round(bits / seconds / 1e6, 1), "delivered_mbit_s": round(bits / wall / 1e6, 1),
        "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "max_latency_ms": round(float(lat.max()) * 1e3, 3),
        "peak_admitted_bytes": int(st["peak_bytes"]), "budget_bytes": budget_bytes,
        "workspace_bytes": int(st["workspace_bytes"]), "peak_device_bytes": int(st["peak_device_bytes"]),
        "peak_concurrent_launches": int(st["peak_concurrent_launches"]),
        "launches": int(st["launches"] - base["launches"]), "latency_by_code_n": by_code,
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
    # the fused launch's form, workgroups per CU and frame order, picked by the
    # library's multi-code autotuner on this batch
    (mode, bpc, order), tune_ms = lp.autotune_multi(codes, batch.code_of_frame, off, dev_llr,
                                                    max_blocks_per_cu=2, **W.PAPER_PARAMS)
    resident = mode == lp.MODE_RESIDENT
    P = dict(W.PAPER_PARAMS, mode=mode)

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
        "autotune": {"mode": {lp.MODE_RESIDENT: "resident", lp.MODE_PERSISTENT_GLOBAL: "persistent_global"}[mode],
                     "blocks_per_cu": bpc, "order": "larger codes first" if order == 1 else "submission order",
                     "candidates_ms": {f"{'resident' if m == lp.MODE_RESIDENT else 'persistent_global'}/"
                                       f"{'larger-first' if o == 1 else 'submission'}/{b}": round(v, 3)
                                       for (m, o, b), v in tune_ms.items()}},
        # every code of the batch fits the register-resident form (check degrees
        # 6..8): the state stays on chip, so the roof is VALU issue
        "roofline": ({"bound": "alu", "achieved": round(achieved / 1e3, 3), "peak": VALU_PEAK_GOPS / 1e3,
                      "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_GOPS, 4), "traffic": None,
                      "kernel": "k_decode (resident, check degrees 6..8)"} if resident else
                     {"bound": "hbm", "achieved": round(byt / (ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(byt / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                      "kernel": "k_decode (persistent-global, degrees 2..8)"}),
    }


def workload_precision(args, lp, W, torch):
    """FP16 versus FP32 message storage on the two n = 16384 codes, 8192 frames at
    2.5 dB each, in the streamed form (state in HBM; keys fp32 / fp16, with their HBM
    fraction) and the persistent-global form (keys *_persistent_global; FP16 holds a
    wave's chunks in registers as packed FP16 pairs).  With the CPU leg, the oracle
    decodes a sample of the same frames: its decode rate, the GPU's hard-decision
    agreement with it, and the error of x and lambda after a fixed number of
    iterations."""
    out = {}
    P = W.PAPER_PARAMS
    stream = torch.cuda.current_stream()
    forms = (("", lp.MODE_STREAMED), ("_persistent_global", lp.MODE_PERSISTENT_GLOBAL))
    for name, H in (("(3,6) n=16384", W.gallager36(16384)), ("(4,8) n=16384", W.gallager48(16384))):
        llr_h = W.awgn_batch(H, 8192, 2.5, tag="precision")
        llr = torch.from_numpy(llr_h).cuda()
        code = lp.Code(H)
        res, hard, xs = {}, {}, {}
        for sname, st in (("fp32", lp.STORAGE_FP32), ("fp16", lp.STORAGE_FP16)):
            for suffix, mode in forms:
                key = sname + suffix
                lp.decode(code, llr, mode=mode, storage=st, **P)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                x, it, fl = lp.decode(code, llr, mode=mode, storage=st, **P)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                it_h = it.cpu().numpy().astype(np.int64)
                ops = algorithmic_ops_per_frame_iter(H) * int(it_h.sum())
                r = {"mbit_s": round(8192 * H.n / (ms / 1e3) / 1e6, 1), "ms": round(ms, 2),
                     "mean_iterations": round(float(it_h.mean()), 2),
                     "frame_errors": int(((x >= 0.5).any(dim=1)).sum().item()),
                     "kernel_vgprs": code.launch_info(mode=mode, storage=st)["vgprs"],
                     # the same algorithmic op count as the headline's VALU roofline (the
                     # accumulator exchange's fixed-point conversions are not counted)
                     "alu_tops": round(ops / (ms / 1e3) / 1e12, 2),
                     "alu_frac": round(ops / (ms / 1e3) / 1e9 / VALU_PEAK_GOPS, 4)}
                if mode == lp.MODE_STREAMED:
                    B = (16 if st == lp.STORAGE_FP32 else 8) * H.nnz + 4 * H.n
                    r.update({"bytes_per_frame_iter": B,
                              "hbm_gbs": round(B * int(it_h.sum()) / (ms / 1e3) / 1e9, 1),
                              "hbm_frac": round(B * int(it_h.sum()) / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)})
                res[key] = r
                hard[key] = (x >= 0.5).cpu().numpy()
                xs[key] = x.cpu().numpy()
        best = {s: min(res[s]["ms"], res[s + "_persistent_global"]["ms"]) for s in ("fp32", "fp16")}
        out[name] = {"throughput": res,
                     "fp16_over_fp32_speed": round(res["fp32"]["ms"] / res["fp16"]["ms"], 3),
                     "fp16_over_fp32_speed_best_forms": round(best["fp32"] / best["fp16"], 3),
                     "fp16_forms_bitwise_equal": bool(np.array_equal(xs["fp16"], xs["fp16_persistent_global"])),
                     "fp32_forms_bitwise_equal": bool(np.array_equal(xs["fp32"], xs["fp32_persistent_global"])),
                     "hard_decision_agreement_fp16_vs_fp32":
                         float(np.mean(np.all(hard["fp16"] == hard["fp32"], axis=1)))}
        if not args.no_cpu:
            # CPU leg: the oracle on the first frames of the batch (its rate and the GPU's
            # agreement with it), and the error after K iterations with stopping disabled
            import oracle
            S = 256
            t0 = time.perf_counter()
            ref = oracle.decode(H, llr_h[:S], **P)
            ct = time.perf_counter() - t0
            amb = np.any(np.abs(ref.x - 0.5) < 1e-3, axis=1)
            agree = {s: float(np.all(hard[s][:S] == (ref.x >= 0.5), axis=1)[~amb].mean()) for s in hard}
            K, S2 = 50, 16
            ref = oracle.decode(H, llr_h[:S2], max_iter=K, tol=0.0, state=True)
            errs = {}
            for sname, st in (("fp32", lp.STORAGE_FP32), ("fp16", lp.STORAGE_FP16)):
                x, _, _, z, u = lp.decode_state(code, llr[:S2].contiguous(), mode=lp.MODE_STREAMED, storage=st,
                                                tol=0.0, max_iter=K, mu=P["mu"], rho=P["rho"])
                torch.cuda.synchronize()
                errs[sname] = {"max_abs_x": float(np.abs(x.cpu().numpy() - ref.x).max()),
                               "max_abs_lambda": float(P["mu"] * np.abs(u.cpu().numpy() - ref.u).max())}
            out[name]["cpu_baseline"] = {
                "value": round(S * H.n / ct / 1e6, 3), "unit": "Mbit/s", "cores": oracle.host_threads(),
                "kind": "oracle", "sample": f"first {S} frames, FP64 C oracle, {ct:.1f} s",
                "hard_decision_agreement_with_oracle": agree, "non_ambiguous_frames": int((~amb).sum()),
                f"error_vs_oracle_after_{K}_iterations_{S2}_frames": errs}
    top = out["(3,6) n=16384"]["throughput"]["fp16_persistent_global"]
    return {
        "metric": METRIC, "value": top["mbit_s"],
        "unit": "Mbit/s (FP16 storage, persistent-global form, (3,6) n=16384)", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": top["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16 storage / f32 compute", "data": "synthetic",
        "config": {"workload": "precision: (3,6) and (4,8) regular n=16384, 8192 frames at 2.5 dB, streamed and "
                               "persistent-global forms, FP16 vs FP32 message/dual storage"},
        "precision": out,
    }


def large_streamed_llr(W, H):
    """The 32768-frame streamed batch: the headline's 16384 frames and a second seeded
    block of 4096 frames at each Eb/N0 (a 2.8 GB working set that only HBM holds)."""
    return np.concatenate([W.awgn_batch(H, FRAMES_PER_SNR, s) for s in W.HEADLINE_SNRS] +
                          [W.awgn_batch(H, FRAMES_PER_SNR, s, block=1) for s in W.HEADLINE_SNRS])


def workload_streamed_large(args, lp, W, torch):
    """The streamed (HBM-resident) form alone on the 32768-frame batch, warm-up + steps
    decodes, against the 8 TB/s roof (used to profile that form by itself)."""
    H = W.gallager36(2640)
    code = lp.Code(H)
    llr = torch.from_numpy(large_streamed_llr(W, H)).cuda()
    P = dict(W.PAPER_PARAMS, mode=lp.MODE_STREAMED)
    (x, it, fl), ms = _timed(torch, lambda: lp.decode(code, llr, **P), steps=args.steps, warmup=args.warmup)
    fi = int(it.cpu().numpy().astype(np.int64).sum())
    B = algorithmic_bytes_per_frame_iter(H)
    ach = B * fi / (ms / 1e3) / 1e9
    return {
        "metric": METRIC, "value": round(int(llr.shape[0]) * H.n / (ms / 1e3) / 1e6, 2), "unit": "Mbit/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "streamed form: (3,6) n=2640, 32768 frames (two seeded blocks of 4096 at each of "
                               "1.5/2.0/2.5/3.0 dB), state in HBM, one launch per iteration", "frames": int(llr.shape[0])},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "target_frac": 0.60,
                     "traffic": profiled_traffic("k_decode_streamed_n2640_large", "traffic_bytes_per_decode"),
                     "algorithmic_bytes": B * fi, "kernel": "k_decode (streamed)"},
    }


def _cpu_model() -> str:
    """The first processor's identification in /proc/cpuinfo (vendor, model name,
    family/model/stepping, clock, cache) and the machine's processor count."""
    keys = ("vendor_id", "model name", "cpu family", "model", "stepping", "cpu MHz", "cache size")
    got, nproc = {}, 0
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                continue
            k, v = (t.strip() for t in line.split(":", 1))
            if k == "processor":
                nproc += 1
            elif k in keys and k not in got:
                got[k] = v
    except OSError:
        return "unknown"
    return "; ".join(f"{k}: {got[k]}" for k in keys if k in got) + f"; processors: {nproc}"


def measured_copy_gbs(torch, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Achievable HBM bandwidth: a plain device-to-device copy of nbytes (read +
    write counted), timed with HIP events on the current stream."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms / 1e3) / 1e9


def _timed(torch, fn, steps=1, warmup=1):
    """Run fn warmup + steps times; return (last result, mean ms of the timed runs)
    from HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    out = None
    for _ in range(steps):
        out = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1) / steps


def _iteration_stats(it, err):
    it = np.asarray(it, np.int64)
    err = np.asarray(err, bool)
    return {"all": round(float(it.mean()), 2),
            "correct": round(float(it[~err].mean()), 2) if (~err).any() else None,
            "erroneous": round(float(it[err].mean()), 2) if err.any() else None}


def _clopper_pearson(k, n, a=0.05):
    from scipy.stats import beta
    lo = 0.0 if k == 0 else float(beta.ppf(a / 2, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(1 - a / 2, k + 1, n - k))
    return [lo, hi]


def workload_bsc(args, lp, W, torch):
    """The random-code BSC study of Sec. 5.1: 100 random (3,6)-regular n = 1002 codes
    (parallel edges removed, length-4 cycles kept), BSC crossover p in BSC_CROSSOVERS,
    `--bsc-frames` frames per code and crossover, all codes in one batched launch per
    crossover.  Reports WER, BER, the ML lower bound of Sec. 5.1 and the iteration
    counts (all / correct / erroneous decodes), as in the ensemble figures."""
    codes_h = W.bsc_ensemble()
    codes = [lp.Code(H) for H in codes_h]
    n = codes_h[0].n
    F = args.bsc_frames
    P = W.PAPER_PARAMS
    cof = np.repeat(np.arange(len(codes_h), dtype=np.int32), F)
    off = np.arange(cof.size, dtype=np.int64) * n
    out, total_ms, total_bits, ops = {}, 0.0, 0, 0
    for p in W.BSC_CROSSOVERS:
        llr_h = np.concatenate([W.bsc_batch(H, F, p, tag="bsc-bench") for H in codes_h]).reshape(-1)
        llr = torch.from_numpy(llr_h).cuda()
        (x, it, fl), ms = _timed(torch, lambda: lp.decode_multi(codes, cof, off, llr, off, llr.numel(), **P),
                                 steps=args.steps, warmup=args.warmup)
        be, ch, cs, oc = lp.evaluate_multi(codes, cof, off, llr, x, off)
        torch.cuda.synchronize()
        be, oc, it_h = be.cpu().numpy(), oc.cpu().numpy(), it.cpu().numpy()
        werr = (oc & lp.EVAL_WORD_ERROR) != 0
        k = int(werr.sum())
        frames = int(cof.size)
        total_ms += ms
        total_bits += frames * n
        ops += algorithmic_ops_per_frame_iter(codes_h[0]) * int(it_h.astype(np.int64).sum())
        out[str(p)] = {
            "frames": frames, "word_errors": k, "wer": k / frames, "wer_ci95": _clopper_pearson(k, frames),
            "ber": float(be.sum()) / (frames * n),
            "ml_lower_bound_errors": int(((oc & lp.EVAL_ML_ERROR) != 0).sum()),
            "ml_lower_bound_wer": float(((oc & lp.EVAL_ML_ERROR) != 0).mean()),
            "iterations": _iteration_stats(it_h, werr),
            "certified": int(((fl.cpu().numpy() & lp.FLAG_CERTIFIED) != 0).sum()),
            "ms": round(ms, 3), "mbit_s": round(frames * n / (ms / 1e3) / 1e6, 1),
        }
    achieved = ops / (total_ms / 1e3) / 1e9
    return {
        "metric": METRIC, "value": round(total_bits / (total_ms / 1e3) / 1e6, 2), "unit": "Mbit/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(total_ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"BSC ensemble: {len(codes_h)} random (3,6)-regular n={n} codes (parallel edges "
                               f"removed), crossover p in {list(W.BSC_CROSSOVERS)}, {F} frames per code and p, "
                               "all-zero codeword, mu=3 rho=1.9 max_iter=1000 tol=1e-5, one batched launch per p"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e3, 3), "peak": round(VALU_PEAK_GOPS / 1e3, 2),
                     "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_GOPS, 4), "traffic": None,
                     "kernel": "k_decode (resident, multi-code)"},
        "bsc": out,
    }


def workload_code313(args, lp, W, torch):
    """The (3,13) code class of Sec. 5 (stand-in for the [1057,813] code: 243 checks of
    degree 13, one of 12): `--sweep-frames` frames at each Eb/N0 in CODE313_SNRS (noise for
    the code's rate 813/1057), the paper's parameters, decoded in one batch by the default
    form (resident: one chunk per wave, its state in registers) and, for comparison, the
    persistent-global and streamed forms.  Reports throughput, WER per Eb/N0 and the VALU
    roofline of the default form."""
    H = W.code313(1057)
    rate = 1.0 - H.m / H.n
    F = args.sweep_frames
    P = W.PAPER_PARAMS
    llr_h = np.concatenate([W.awgn_batch(H, F, s, tag="code313-bench", rate=rate) for s in CODE313_SNRS])
    llr = torch.from_numpy(llr_h).cuda()
    code = lp.Code(H)
    li = code.launch_info()
    (x, it, fl), ms = _timed(torch, lambda: lp.decode(code, llr, **P), steps=args.steps, warmup=args.warmup)
    torch.cuda.synchronize()
    x_h, it_h, fl_h = x.cpu().numpy(), it.cpu().numpy(), fl.cpu().numpy()
    others = {}
    for name, m in (("persistent_global", lp.MODE_PERSISTENT_GLOBAL), ("streamed", lp.MODE_STREAMED)):
        (xo, ito, flo), mso = _timed(torch, lambda: lp.decode(code, llr, mode=m, **P),
                                     steps=args.steps, warmup=args.warmup)
        torch.cuda.synchronize()
        same = bool(np.array_equal(x_h, xo.cpu().numpy()) and np.array_equal(it_h, ito.cpu().numpy())
                    and np.array_equal(fl_h, flo.cpu().numpy()))
        others[name] = {"ms": round(mso, 3), "mbit_s": round(llr_h.shape[0] * H.n / (mso / 1e3) / 1e6, 2),
                        "bitwise_equal_to_default_form": same}
    werr = (x_h >= 0.5).any(axis=1)
    per_snr = {}
    for b, snr in enumerate(CODE313_SNRS):
        sl = slice(b * F, (b + 1) * F)
        k = int(werr[sl].sum())
        per_snr[str(snr)] = {"frames": F, "word_errors": k, "wer": k / F, "wer_ci95": _clopper_pearson(k, F),
                             "iterations": _iteration_stats(it_h[sl], werr[sl]),
                             "certified": int(((fl_h[sl] & lp.FLAG_CERTIFIED) != 0).sum())}
    frames = llr_h.shape[0]
    ops = algorithmic_ops_per_frame_iter(H) * int(it_h.astype(np.int64).sum())
    achieved = ops / (ms / 1e3) / 1e9
    return {
        "metric": METRIC, "value": round(frames * H.n / (ms / 1e3) / 1e6, 2), "unit": "Mbit/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"(3,13) code class: variable degree 3, n={H.n}, m={H.m} (243 checks of degree 13, "
                               f"one of 12, rate {rate:.4f}), {F} frames at each Eb/N0 in {list(CODE313_SNRS)} dB, "
                               "all-zero codeword over BPSK/AWGN, mu=3 rho=1.9 max_iter=1000 tol=1e-5, one batch"},
        "launch": li,
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e3, 3), "peak": round(VALU_PEAK_GOPS / 1e3, 2),
                     "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_GOPS, 4), "traffic": None,
                     "kernel": "k_decode (%s, check degrees 2..16)" % FORM_NAMES.get(li["mode"], "?")},
        "other_forms": others,
        "per_ebn0": per_snr,
    }


def workload_sweep(args, lp, W, torch):
    """Parameter sensitivity of Sec. 5.2 on the (3,6) n = 2640 code: WER and decode time
    against the stopping tolerance (2.2 dB, mu in {1,5,7}, rho = 1), against mu
    (1.9/2.2/2.5 dB, eps = 1e-5, rho = 1), and against the over-relaxation rho
    (2.8 dB, mu in {1,3,5,7})."""
    H = W.gallager36(2640)
    code = lp.Code(H)
    F = args.sweep_frames
    llrs = {}

    def llr_at(snr):
        if snr not in llrs:
            llrs[snr] = torch.from_numpy(W.awgn_batch(H, F, snr, tag="sweep")).cuda()
        return llrs[snr]

    def point(snr, **kw):
        prm = dict(W.PAPER_PARAMS)
        prm.update(kw)
        (x, it, fl), ms = _timed(torch, lambda: lp.decode(code, llr_at(snr), **prm), steps=1, warmup=1)
        err = (x >= 0.5).any(dim=1).cpu().numpy()
        it_h = it.cpu().numpy()
        return {"wer": float(err.mean()), "word_errors": int(err.sum()), "ms": round(ms, 3),
                "mean_iterations": round(float(it_h.mean()), 2), "us_per_frame": round(ms * 1e3 / F, 3)}

    total_ms, points = 0.0, 0
    eps = {}
    for mu in (1.0, 5.0, 7.0):
        for b in (4, 7, 10, 13, 17, 20):
            r = point(2.2, mu=mu, rho=1.0, tol=2.0 ** -b)
            eps[f"mu={mu:g},-log2(eps)={b}"] = r
            total_ms += r["ms"]
            points += 1
    mus = {}
    for snr in (1.9, 2.2, 2.5):
        for mu in (0.5, 1.0, 2.0, 3.0, 5.0, 7.0, 10.0):
            r = point(snr, mu=mu, rho=1.0, tol=1e-5)
            mus[f"{snr}dB,mu={mu:g}"] = r
            total_ms += r["ms"]
            points += 1
    rhos, speedup = {}, {}
    for mu in (1.0, 3.0, 5.0, 7.0):
        for rho in (1.0, 1.3, 1.6, 1.9):
            r = point(2.8, mu=mu, rho=rho, tol=1e-5)
            rhos[f"mu={mu:g},rho={rho:g}"] = r
            total_ms += r["ms"]
            points += 1
        a, b = rhos[f"mu={mu:g},rho=1"], rhos[f"mu={mu:g},rho=1.9"]
        speedup[f"mu={mu:g}"] = {"time": round(a["ms"] / b["ms"], 3),
                                 "iterations": round(a["mean_iterations"] / b["mean_iterations"], 3)}
    bits = points * F * H.n
    return {
        "metric": METRIC, "value": round(bits / (total_ms / 1e3) / 1e6, 2), "unit": "Mbit/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(total_ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"parameter sweeps: (3,6) n=2640, {F} frames per point, {points} points "
                               "(eps at 2.2 dB, mu at 1.9/2.2/2.5 dB, rho at 2.8 dB), t_max=1000"},
        "sweep": {"tolerance": eps, "mu": mus, "over_relaxation": rhos,
                  "rho_1_over_rho_1.9": speedup},
    }


def workload_dual(args, lp, W, torch):
    """Dual subgradient ascent (Appendix A) against ADMM on the (3,6) n = 2640 code:
    the same frames, t_max = 1000, three step sizes, three Eb/N0."""
    H = W.gallager36(2640)
    code = lp.Code(H)
    F = args.sweep_frames
    out, total_ms, bits = {}, 0.0, 0
    for snr in (2.5, 3.0, 3.5):
        llr = torch.from_numpy(W.awgn_batch(H, F, snr, tag="dual-bench")).cuda()
        (x, it, fl), ms = _timed(torch, lambda: lp.decode(code, llr, **W.PAPER_PARAMS))
        err = (x >= 0.5).any(dim=1).cpu().numpy()
        row = {"admm": {"wer": float(err.mean()), "iterations": _iteration_stats(it.cpu().numpy(), err),
                        "ms": round(ms, 3)}}
        for mu in (0.1, 0.25, 0.5):
            (x, it, fl), ms = _timed(torch, lambda: lp.decode_dual(code, llr, mu=mu, max_iter=1000))
            err = (x >= 0.5).any(dim=1).cpu().numpy()
            conv = (fl.cpu().numpy() & lp.FLAG_CONVERGED) != 0
            row[f"dual_mu={mu:g}"] = {"wer": float(err.mean()), "converged": float(conv.mean()),
                                      "iterations": _iteration_stats(it.cpu().numpy(), err), "ms": round(ms, 3)}
            total_ms += ms
            bits += F * H.n
        out[f"{snr}dB"] = row
    return {
        "metric": METRIC, "value": round(bits / (total_ms / 1e3) / 1e6, 2), "unit": "Mbit/s (dual subgradient)",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(total_ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i32 (f64 decisions)", "data": "synthetic",
        "config": {"workload": f"dual subgradient ascent vs ADMM: (3,6) n=2640, {F} frames at 2.5/3.0/3.5 dB, "
                               "step mu in {0.1,0.25,0.5}, t_max=1000"},
        "dual": out,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="auto", choices=["auto", "resident", "persistent_global", "streamed"])
    ap.add_argument("--cpu-frames", type=int, default=16384,
                    help="oracle sample size in frames (default: the whole batch, about 30 s on 16 cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the plain and streamed comparisons and the per-Eb/N0 blocks decoded alone")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "uneven", "precision", "serving", "bsc", "sweep", "dual", "streamed_large",
                             "code313"])
    ap.add_argument("--bsc-frames", type=int, default=128, help="frames per code and crossover (bsc workload)")
    ap.add_argument("--sweep-frames", type=int, default=4096, help="frames per point (sweep and dual workloads)")
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
    if args.workload == "bsc":
        print(json.dumps(workload_bsc(args, lp, W, torch)))
        return
    if args.workload == "sweep":
        print(json.dumps(workload_sweep(args, lp, W, torch)))
        return
    if args.workload == "dual":
        print(json.dumps(workload_dual(args, lp, W, torch)))
        return
    if args.workload == "streamed_large":
        print(json.dumps(workload_streamed_large(args, lp, W, torch)))
        return
    if args.workload == "code313":
        print(json.dumps(workload_code313(args, lp, W, torch)))
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
    # per-SNR error rates and the ML lower bound of Sec. 5.1 (evaluation kernel)
    _, _, _, ml_oc = lp.evaluate(code, llr, out[0])
    ml_oc = ml_oc.cpu().numpy()
    fer = {}
    for b, s in enumerate(W.HEADLINE_SNRS):
        sl = slice(b * FRAMES_PER_SNR, (b + 1) * FRAMES_PER_SNR)
        errs = int(np.sum((x[sl] >= 0.5).any(axis=1)))
        fer[str(s)] = {"frame_errors": errs, "fer": errs / FRAMES_PER_SNR,
                       "fer_ci95": _clopper_pearson(errs, FRAMES_PER_SNR),
                       "ml_lower_bound_errors": int(((ml_oc[sl] & lp.EVAL_ML_ERROR) != 0).sum()),
                       "mean_iters": float(iters[sl].mean())}
        if not args.no_extra:
            # the block decoded alone (same form), for per-SNR throughput
            blk = llr[sl].contiguous()
            (_, bit, _), bms = _timed(torch, lambda: lp.decode(code, blk, mode=mode, **P), steps=2, warmup=1)
            bfi = int(bit.cpu().numpy().astype(np.int64).sum())
            fer[str(s)].update({"alone_mbit_s": round(FRAMES_PER_SNR * H.n / (bms / 1e3) / 1e6, 1),
                                "alone_info_mbit_s": round(FRAMES_PER_SNR * k_info / (bms / 1e3) / 1e6, 1),
                                "alone_mean_iters": round(bfi / FRAMES_PER_SNR, 2)})

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
    }
    if form == "resident":
        achieved = ops * frame_iters / kernel_s / 1e9
        prof = "k_decode_resident_n2640_headline"
        valu = profiled_traffic(prof, "valu_insts_per_launch")
        busy = profiled_traffic(prof, "valu_busy_x10000")  # SQ_ACTIVE_INST_VALU share, in 1e-4
        res["roofline"] = {"bound": "alu", "achieved": round(achieved / 1e3, 3), "peak": round(VALU_PEAK_GOPS / 1e3, 2),
                           "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_GOPS, 4),
                           "traffic": profiled_traffic(prof),
                           "kernel": "k_decode_pair (resident, two frames per workgroup)",
                           "ops_per_frame_iter": ops, "kernel_ms": round(gpu_ms, 3), "launches_per_step": 1,
                           # analytic lane operations of the step as wave instructions (64 lanes),
                           # beside the VALU wave instructions the counters saw in one launch
                           "algorithmic_wave_ops": int(ops * frame_iters // 64),
                           "valu_insts_per_launch": valu,
                           "valu_insts_over_algorithmic": (round(valu / (ops * frame_iters / 64), 4)
                                                           if valu else None),
                           "valu_busy_frac": busy / 1e4 if busy is not None else None}
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
        copy_gbs = measured_copy_gbs(torch)
        # the HBM-resident form against the HBM roof (z, u and gamma move through HBM
        # every iteration: B = 16 E + 4 n bytes per frame-iteration)
        res["roofline_streamed"] = {
            "bound": "hbm", "achieved": round(sach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(sach / HBM_PEAK_GBS, 4), "target_frac": 0.60,
            "traffic": profiled_traffic("k_decode_streamed_n2640_headline", "traffic_bytes_per_decode"),
            "algorithmic_bytes": B * sfi, "bytes_per_frame_iter": B, "kernel": "k_decode (streamed)",
            "ms": round(sms, 3), "mbit_s": round(F * H.n / (sms / 1e3) / 1e6, 2), "launches": int(sit.max()),
            "copy_ceiling_gbs": round(copy_gbs, 1), "frac_of_copy": round(sach / copy_gbs, 4)}
        # the headline batch's state (16384 x 63 KB) is of the order of the 256 MB
        # last-level cache; twice the frames (a second seeded block) move a 4.5 GB
        # working set that only HBM holds
        llr2 = torch.from_numpy(large_streamed_llr(W, H)).to(dev)
        lp.decode(code, llr2, mode=lp.MODE_STREAMED, **P)
        torch.cuda.synchronize()
        e0.record(stream)
        x2, it2, _ = lp.decode(code, llr2, mode=lp.MODE_STREAMED, **P)
        e1.record(stream)
        torch.cuda.synchronize()
        lms = e0.elapsed_time(e1)
        lfi = int(it2.cpu().numpy().astype(np.int64).sum())
        lach = B * lfi / (lms / 1e3) / 1e9
        res["roofline_streamed_large"] = {
            "bound": "hbm", "achieved": round(lach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(lach / HBM_PEAK_GBS, 4), "target_frac": 0.60,
            "traffic": profiled_traffic("k_decode_streamed_n2640_large", "traffic_bytes_per_decode"),
            "frames": int(llr2.shape[0]), "working_set_bytes": int(llr2.shape[0]) * (8 * H.nnz + 8 * H.n),
            "ms": round(lms, 3), "frac_of_copy": round(lach / copy_gbs, 4)}
        del llr2, x2, it2
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
        # one frame per launch without per-iteration launches: the resident form on a
        # batch of one (a single workgroup decodes the frame to completion)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, f in enumerate(sample):
            lp.decode(code, llr[f:f + 1], out=one[k], mode=lp.MODE_RESIDENT, **P)
        torch.cuda.synchronize()
        rt = time.perf_counter() - t0
        res["plain_resident"] = {"mbit_s": round(len(sample) * H.n / rt / 1e6, 3), "frames": int(len(sample)),
                                 "form": "resident, batch of 1",
                                 "batched_over_plain": round(value / (len(sample) * H.n / rt / 1e6), 1)}

    if args.serving_seconds > 0 and not args.no_extra:
        res["serving"] = run_serving(lp, W, args.serving_seconds)

    if not args.no_cpu:
        # the FP64 oracle on the same LLRs, all host cores (at most 16): its decode rate
        # is the CPU baseline, and its results give the batch's parity figures
        import oracle
        cores = oracle.host_threads()
        per = max(1, min(args.cpu_frames, F) // len(W.HEADLINE_SNRS))
        sample = np.concatenate([b * FRAMES_PER_SNR + np.arange(per) for b in range(len(W.HEADLINE_SNRS))])
        t0 = time.perf_counter()
        ref = oracle.decode(H, llr_h[sample], nthreads=cores, **P)
        ct = time.perf_counter() - t0
        # one thread on a smaller sample (the first frames of each Eb/N0 block, ~4 s)
        per1 = 16
        sample1 = np.concatenate([b * FRAMES_PER_SNR + np.arange(per1) for b in range(len(W.HEADLINE_SNRS))])
        t0 = time.perf_counter()
        oracle.decode(H, llr_h[sample1], nthreads=1, **P)
        ct1 = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(len(sample) * H.n / ct / 1e6, 3), "unit": "Mbit/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{len(sample)} frames ({per} per Eb/N0, same LLRs), FP64 C oracle, "
                                         f"{ct:.1f} s, mean iterations {ref.iters.mean():.1f}",
                               "single_thread": {"value": round(len(sample1) * H.n / ct1 / 1e6, 4),
                                                 "frames": int(len(sample1)), "seconds": round(ct1, 2)},
                               "cpu_model": _cpu_model()}
        # GPU against oracle on those frames (reading R13: a frame whose oracle x has an
        # entry within 1e-3 of 1/2 is ambiguous; its hard decision is not compared)
        xs, its, fls = x[sample], iters[sample], fl[sample]
        amb = np.any(np.abs(ref.x - 0.5) < 1e-3, axis=1)
        same = np.all((xs >= 0.5) == (ref.x >= 0.5), axis=1)
        dit = np.abs(its - ref.iters)
        res["parity"] = {"frames": int(len(sample)), "ambiguous": int(amb.sum()),
                         "hard_decision_mismatches": int((~same & ~amb).sum()),
                         "hard_decision_agreement": round(float(same[~amb].mean()), 6),
                         "iterations_within_2": round(float((dit <= 2).mean()), 6),
                         "iterations_max_diff": int(dit.max()),
                         "flags_agreement": round(float(((fls & 0x0F) == (ref.flags & 0x0F))[~amb].mean()), 6)}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
