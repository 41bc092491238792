"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances
* Projection: both sides project the same FP32 input; the kernel works in FP32.
  Its beta is a prefix average of <= 8 breakpoints of magnitude <= 1 + |v|, so
  the error is a few FP32 ulps of (1 + max|v|): 2e-6 (1 + max|v|).
* Messages after K iterations with stopping disabled: 1e-4 absolute (x, z and
  u = lambda/mu).  ADMM's fixed-point map is non-expansive, so FP32 rounding
  grows at most about linearly in K; 1e-4 covers K <= 200 on these codes.
* Hard decisions: identical on every frame whose oracle x has no entry within
  1e-3 of 1/2 (ambiguous frames are counted but not compared).
* Iteration counts: the FP32 residual sums may cross eps^2 E one iteration
  earlier or later than the FP64 ones: |delta| <= 2.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_parity, parity_summary, ref_slice

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

lp = None


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global lp
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1204_0556_amd as m
    lp = m
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _proj_inputs(d, count, seed):
    rng = np.random.default_rng([d, seed])
    parts = [rng.uniform(-0.5, 1.5, (count, d)), rng.normal(0.5, 1.0, (count, d)),
             rng.choice([-0.2, 0.0, 0.3, 0.7, 1.0, 1.2], size=(count, d)), rng.normal(0.0, 4.0, (count, d))]
    # near-even clipped sums
    near = rng.uniform(0, 1, (count, d))
    tgt = 2 * np.maximum(1, np.round(near.sum(1) / 2))
    near = near + ((tgt - near.sum(1)) / d)[:, None] + rng.normal(0, 1e-6, (count, d))
    parts.append(near)
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("d", list(range(2, 17)))
def test_projection_matches_oracle(d):
    v = _proj_inputs(d, 2000, 1)
    print(f"projection d={d} count={len(v)}", flush=True)
    z = host(lp.project(dev(v)))
    zo = oracle.project(v.astype(np.float64))
    tol = 2e-6 * (1.0 + np.abs(v).max(axis=1))
    err = np.abs(z - zo).max(axis=1)
    assert np.all(err <= tol), (err.max(), v[np.argmax(err - tol)])


def _fixed_k(H, llr, K, mode):
    x, it, fl, z, u = lp.decode_state(lp.Code(H), dev(llr), tol=0.0, max_iter=K, mode=mode)
    return host(x), host(it), host(fl), host(z), host(u)


@pytest.mark.parametrize("mode", ["resident", "persistent_global", "streamed"])
@pytest.mark.parametrize("K", [1, 10, 50, 200])
def test_messages_after_k_iterations(K, mode):
    m = {"resident": lp.MODE_RESIDENT, "persistent_global": lp.MODE_PERSISTENT_GLOBAL,
         "streamed": lp.MODE_STREAMED}[mode]
    for n, frames in ((96, 64), (2640, 8)):
        H = W.gallager36(n)
        llr = W.awgn_batch(H, frames, 2.0, tag="fixedk")
        print(f"fixed-K n={n} K={K} mode={mode}", flush=True)
        x, it, fl, z, u = _fixed_k(H, llr, K, m)
        ref = oracle.decode(H, llr, mu=3.0, rho=1.9, max_iter=K, tol=0.0, state=True)
        assert np.all(it == K)
        assert np.abs(x - ref.x).max() < 1e-4
        assert np.abs(z - ref.z).max() < 1e-4
        assert np.abs(u - ref.u).max() < 1e-4


@pytest.mark.parametrize("n", [2640, 4608, 8064])
def test_forms_agree_bitwise(n):
    # n = 4608 and 8064 run the resident form with three and four chunks per wave
    # (16 waves, metadata and gamma/mu read from memory each iteration)
    H = W.gallager36(n)
    llr = W.awgn_batch(H, 32, 2.0, tag="forms")
    code = lp.Code(H)
    assert code.info["resident_capable"]
    print(f"forms n={n}: {code.launch_info(mode=lp.MODE_RESIDENT)}", flush=True)
    outs = []
    for m in (lp.MODE_RESIDENT, lp.MODE_PERSISTENT_GLOBAL, lp.MODE_STREAMED):
        x, it, fl = lp.decode(code, dev(llr), mode=m, max_iter=300)
        outs.append((host(x), host(it), host(fl)))
    for o in outs[1:]:
        assert np.array_equal(o[1], outs[0][1])
        assert np.array_equal(o[2], outs[0][2])
        assert np.abs(o[0] - outs[0][0]).max() == 0.0


def test_streamed_variants_many_frames_per_workgroup():
    # 3072 frames at low SNR: every workgroup walks many frames, finished and
    # unfinished ones interleave, and the staged variant's copy of the next frame
    # overlaps the current one.  All streamed variants equal the resident form.
    H = W.gallager36(2640)
    llr = np.concatenate([W.awgn_batch(H, 1536, s, tag="variants") for s in (1.5, 2.5)])
    code = lp.Code(H)
    kw = dict(max_iter=120)
    x0, it0, fl0 = (host(t) for t in lp.decode(code, dev(llr), mode=lp.MODE_RESIDENT, **kw))
    for var in (2, 1, 0):
        code.set_tuning(lp.MODE_STREAMED, 0, var)
        print(f"streamed variant {var}: {llr.shape[0]} frames", flush=True)
        assert code.launch_info(mode=lp.MODE_STREAMED)["variant"] == var
        x, it, fl = (host(t) for t in lp.decode(code, dev(llr), mode=lp.MODE_STREAMED, **kw))
        assert np.array_equal(it, it0) and np.array_equal(fl, fl0)
        assert np.abs(x - x0).max() == 0.0


def _compare_decodes(H, llr, x, it, fl, ref, max_iter):
    ambiguous = np.any(np.abs(ref.x - 0.5) < 1e-3, axis=1)
    hard, href = (x >= 0.5), (ref.x >= 0.5)
    same = np.all(hard == href, axis=1)
    assert np.all(same | ambiguous), np.nonzero(~(same | ambiguous))[0]
    dit = np.abs(it.astype(int) - ref.iters)
    assert np.mean(dit <= 2) >= 0.99, np.sort(dit)[-10:]
    # flags: converged / certified agree except at the iteration-count margin
    agree = (fl & 0x0F) == (ref.flags & 0x0F)
    assert np.mean(agree) >= 0.99
    return ambiguous


def test_small_code_end_to_end():
    """(3,6) n=96, 1000 frames at 3 dB, T = 200 (the small FP64 reference workload)."""
    H = W.gallager36(96)
    llr = W.awgn_batch(H, 1000, 3.0)
    x, it, fl = lp.decode(lp.Code(H), dev(llr), mu=3.0, rho=1.9, max_iter=200, tol=1e-5)
    ref = oracle.decode(H, llr, mu=3.0, rho=1.9, max_iter=200, tol=1e-5)
    _compare_decodes(H, llr, host(x), host(it), host(fl), ref, 200)
    fer_gpu = np.mean(host(x).__ge__(0.5).any(axis=1))
    fer_cpu = np.mean(ref.hard.any(axis=1))
    assert abs(fer_gpu - fer_cpu) <= 0.005
    # the GPU FER lies inside the oracle's 95 % Clopper-Pearson interval
    from scipy.stats import beta
    k, N = int(round(fer_cpu * len(llr))), len(llr)
    lo = beta.ppf(0.025, k, N - k + 1) if k > 0 else 0.0
    hi = beta.ppf(0.975, k + 1, N - k) if k < N else 1.0
    assert lo <= fer_gpu <= hi, (fer_gpu, lo, hi)


def _fer_ci(k, N):
    from scipy.stats import beta
    lo = beta.ppf(0.025, k, N - k + 1) if k > 0 else 0.0
    hi = beta.ppf(0.975, k + 1, N - k) if k < N else 1.0
    return lo, hi


def test_headline_batch_full_size():
    """n=2640 (3,6) at the four Eb/N0 points, 4096 frames each, decoded in one call in
    the benchmark's launch configuration; every frame is checked against the oracle
    (Alg. 1 with over-relaxation, FP64), which runs on all host cores (about 30 s)."""
    H = W.gallager36(2640)
    llr = np.concatenate([W.awgn_batch(H, 4096, s) for s in W.HEADLINE_SNRS])
    print(f"headline batch frames={len(llr)}", flush=True)
    x, it, fl = lp.decode(lp.Code(H), dev(llr))
    x, it, fl = host(x), host(it), host(fl)
    print(f"oracle on {len(llr)} frames, {oracle.host_threads()} threads", flush=True)
    ref = oracle.decode(H, llr)
    for b, snr in enumerate(W.HEADLINE_SNRS):
        blk = slice(b * 4096, (b + 1) * 4096)
        sm = parity_summary(x[blk], it[blk], fl[blk], ref_slice(ref, blk))
        assert_parity(sm, f"headline {snr} dB")
        # the GPU FER lies inside the 95 % Clopper-Pearson interval of the oracle's FER
        k = int(ref.hard[blk].any(axis=1).sum())
        lo, hi = _fer_ci(k, 4096)
        fer = float((x[blk] >= 0.5).any(axis=1).mean())
        assert lo <= fer <= hi, (snr, fer, lo, hi)
    assert_parity(parity_summary(x, it, fl, ref), "headline all")
    # every frame: flags consistent with x (certificate recomputed on the host)
    hard = (x >= 0.5).astype(np.int64)
    Hd = H.to_scipy()
    syn = (Hd @ hard.T) % 2
    codeword = ~np.any(syn, axis=0)
    assert np.array_equal(codeword, (fl & 0x04) != 0)
    integral = np.max(np.minimum(x, 1 - x), axis=1) <= 1e-3
    assert np.array_equal(integral, (fl & 0x02) != 0)
    assert np.all(it[(fl & 0x01) == 0] == 1000)


def test_invalid_frames_are_flagged():
    H = W.gallager36(96)
    llr = W.awgn_batch(H, 6, 3.0, tag="nan")
    llr[1, 3] = np.nan
    llr[4, 0] = -np.inf
    for m in (lp.MODE_RESIDENT, lp.MODE_PERSISTENT_GLOBAL, lp.MODE_STREAMED):
        x, it, fl = lp.decode(lp.Code(H), dev(llr), mode=m)
        x, it, fl = host(x), host(it), host(fl)
        for f in (1, 4):
            assert fl[f] == lp.FLAG_INVALID and it[f] == 0 and np.all(x[f] == 0.5)
        for f in (0, 2, 3, 5):
            assert fl[f] & lp.FLAG_CONVERGED


@pytest.mark.parametrize("n", [2640, 8064])
def test_warm_start_resume_is_exact(n):
    H = W.gallager36(n)
    llr = W.awgn_batch(H, 4, 1.5, tag="warm")
    code = lp.Code(H)
    for m in (lp.MODE_RESIDENT, lp.MODE_STREAMED):
        a = lp.decode_state(code, dev(llr), tol=0.0, max_iter=30, mode=m)
        b = lp.decode_state(code, dev(llr), tol=0.0, max_iter=12, mode=m)
        c = lp.decode_state(code, dev(llr), z=b[3], u=b[4], state_in=True, tol=0.0, max_iter=18, mode=m)
        assert np.array_equal(host(a[3]), host(c[3])) and np.array_equal(host(a[4]), host(c[4]))
        assert np.array_equal(host(a[0]), host(c[0]))


@pytest.mark.parametrize("n,mode,storage", [(2640, "pglobal", 0), (16384, "pglobal", 0), (16384, "streamed", 0),
                                            (16384, "streamed", 1)])
def test_warm_start_resume_is_exact_in_every_form(n, mode, storage):
    # 12 + 18 iterations from the exported state equal 30 in one go, bitwise: the
    # persistent-global form with LDS float slots (n = 2640) and with LDS fixed-point
    # accumulators (n = 16384), the streamed form with FP32 and FP16 state storage
    # (FP16 values export to FP32 exactly and load back exactly)
    H = W.gallager36(n)
    llr = W.awgn_batch(H, 3, 1.5, tag="warm-forms")
    code = lp.Code(H)
    m = {"pglobal": lp.MODE_PERSISTENT_GLOBAL, "streamed": lp.MODE_STREAMED}[mode]
    kw = dict(tol=0.0, mode=m, storage=storage)
    print(f"warm start n={n} {mode} storage={storage}", flush=True)
    a = lp.decode_state(code, dev(llr), max_iter=30, **kw)
    b = lp.decode_state(code, dev(llr), max_iter=12, **kw)
    c = lp.decode_state(code, dev(llr), z=b[3], u=b[4], state_in=True, max_iter=18, **kw)
    assert np.array_equal(host(a[3]), host(c[3])) and np.array_equal(host(a[4]), host(c[4]))
    assert np.array_equal(host(a[0]), host(c[0]))
    assert np.all(host(c[1]) == 18)


def test_edge_batches():
    H = W.gallager36(96)
    code = lp.Code(H)
    llr = W.awgn_batch(H, 1, 3.0, tag="one")
    x, it, fl = lp.decode(code, dev(llr))
    ref = oracle.decode(H, llr)
    assert np.array_equal(host(x) >= 0.5, ref.x >= 0.5)
    empty = torch.empty((0, H.n), dtype=torch.float32, device="cuda")
    x, it, fl = lp.decode(code, empty)
    assert x.shape == (0, H.n)
