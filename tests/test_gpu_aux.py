"""GPU parity of the BSC workload, the dual subgradient decoder (Appendix A) and
the ML lower-bound bookkeeping (Sec. 5.1), through the C ABI, against the FP64
oracle.

Tolerances
* BSC messages after K iterations (stopping disabled): 1e-4 absolute, as for
  AWGN.  Two-valued LLRs make many entries of a check's input tie exactly;
  the projection is unique, so tie order does not matter.
* Dual decoding: bit-exact (x, iterations, flags).  Every multiplier is mu
  times an integer count, the z-update compares counts, and the x decision is
  the same FP64 expression on both sides.
* Evaluation: bit errors and outcome bits exact, except that the ML-error bit
  is not compared when |cost_hat - cost_sent| <= 1e-9 (1 + |cost_sent|): both
  sides sum in FP64 but in different orders.  Costs agree to 1e-12 relative.
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

lp = pytest.importorskip("paper_1204_0556_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ---------------------------------------------------------------- BSC (ADMM)
@pytest.mark.parametrize("mode", ["resident", "persistent_global", "streamed"])
def test_bsc_messages_after_k_iterations(mode):
    m = {"resident": lp.MODE_RESIDENT, "persistent_global": lp.MODE_PERSISTENT_GLOBAL,
         "streamed": lp.MODE_STREAMED}[mode]
    H = W.bsc_ensemble()[0]
    llr = W.bsc_batch(H, 32, 0.06, tag="bsc-k")
    code = lp.Code(H)
    for K in (1, 10, 50):
        print(f"bsc messages mode={mode} K={K}", flush=True)
        x, it, fl, z, u = lp.decode_state(code, dev(llr), tol=0.0, max_iter=K, mode=m)
        ref = oracle.decode(H, llr, tol=0.0, max_iter=K, state=True)
        assert np.abs(host(x) - ref.x).max() <= 1e-4
        assert np.abs(host(z) - ref.z).max() <= 1e-4
        assert np.abs(host(u) - ref.u).max() <= 1e-4
        assert np.all(host(it) == K)


def test_bsc_ensemble_batch_against_oracle():
    codes = W.bsc_ensemble()[:12]
    lcodes = [lp.Code(H) for H in codes]
    per = 16
    llr_parts, cof = [], []
    for c, H in enumerate(codes):
        llr_parts.append(W.bsc_batch(H, per, 0.05, tag="bsc-e2e"))
        cof += [c] * per
    llr = np.concatenate([a.reshape(-1) for a in llr_parts])
    off = np.arange(len(cof), dtype=np.int64) * 1002
    print(f"bsc ensemble batch frames={len(cof)}", flush=True)
    x, it, fl = lp.decode_multi(lcodes, np.array(cof), off, dev(llr), off, llr.size, **W.PAPER_PARAMS)
    x, it, fl = host(x).reshape(-1, 1002), host(it), host(fl)
    amb = 0
    for c, H in enumerate(codes):
        sl = slice(c * per, (c + 1) * per)
        ref = oracle.decode(H, llr_parts[c], **W.PAPER_PARAMS)
        for f in range(per):
            if np.any(np.abs(ref.x[f] - 0.5) < 1e-3):
                amb += 1
                continue
            assert np.array_equal(x[sl][f] >= 0.5, ref.x[f] >= 0.5), (c, f)
            assert abs(int(it[sl][f]) - int(ref.iters[f])) <= 2, (c, f, it[sl][f], ref.iters[f])
            assert (fl[sl][f] & 0x0e) == (ref.flags[f] & 0x0e), (c, f)
    assert amb <= 4


# ---------------------------------------------------------- dual subgradient
def _dual_cases():
    yield "gallager96", W.gallager36(96), W.awgn_batch(W.gallager36(96), 48, 3.0, tag="dual"), 1.0
    H = W.bsc_ensemble()[3]
    yield "bsc1002", H, W.bsc_batch(H, 48, 0.03, tag="dual"), 0.5
    H = W.gallager36(2640)
    yield "gallager2640", H, W.awgn_batch(H, 16, 4.0, tag="dual"), 0.25
    H = W.irregular_half(576)
    yield "irregular576", H, W.awgn_batch(H, 32, 4.0, tag="dual"), 0.5
    H = W.gallager36(16384)
    yield "gallager16384", H, W.awgn_batch(H, 4, 4.5, tag="dual"), 0.5


@pytest.mark.parametrize("case", [c[0] for c in _dual_cases()])
def test_dual_decoder_bit_exact(case):
    name, H, llr, mu = next(c for c in _dual_cases() if c[0] == case)
    T = 300
    print(f"dual case={name} frames={llr.shape[0]} mu={mu}", flush=True)
    x, it, fl = lp.decode_dual(lp.Code(H), dev(llr), mu=mu, max_iter=T)
    ref = oracle.dual_decode(H, llr, mu=mu, max_iter=T)
    assert np.array_equal(host(x), ref.x.astype(np.float32))
    assert np.array_equal(host(it), ref.iters)
    assert np.array_equal(host(fl), ref.flags)
    # both outcomes occur on these inputs
    assert (ref.flags & 1).any()


def test_dual_invalid_and_empty():
    H = W.gallager36(96)
    llr = W.awgn_batch(H, 4, 3.0, tag="dual-bad")
    llr[2, 7] = np.nan
    x, it, fl = lp.decode_dual(lp.Code(H), dev(llr), mu=1.0, max_iter=50)
    ref = oracle.dual_decode(H, llr, mu=1.0, max_iter=50)
    assert host(fl)[2] == 0x80 and host(it)[2] == 0 and np.all(host(x)[2] == 0.5)
    assert np.array_equal(host(fl), ref.flags)
    with pytest.raises(lp.LpdecError):
        lp.decode_dual(lp.Code(H), dev(llr), mu=0.0, max_iter=50)


# ------------------------------------------------------------ ML lower bound
def _check_eval(got, ref):
    be, ch, cs, oc = (host(t) for t in got)
    assert np.array_equal(be, ref["bit_errors"])
    assert np.allclose(ch, ref["cost_hat"], rtol=1e-12, atol=1e-9)
    assert np.allclose(cs, ref["cost_sent"], rtol=1e-12, atol=1e-9)
    near = np.abs(ref["cost_hat"] - ref["cost_sent"]) <= 1e-9 * (1 + np.abs(ref["cost_sent"]))
    mask = np.where(near, 0x03, 0x07).astype(np.uint8)
    assert np.array_equal(oc & mask, ref["outcome"] & mask)


def test_evaluate_against_oracle():
    H = W.gallager36(2640)
    llr = np.concatenate([W.awgn_batch(H, 64, s, tag="eval") for s in (1.25, 1.5, 2.0)])
    code = lp.Code(H)
    x, it, fl = lp.decode(code, dev(llr), max_iter=300)
    xh = host(x)
    got = lp.evaluate(code, dev(llr), x)
    ref = oracle.evaluate(H, llr, xh.astype(np.float64))
    _check_eval(got, ref)
    # the codeword bit agrees with the decoder's own flag
    oc = host(got[3])
    assert np.array_equal((oc & 0x02) != 0, (host(fl) & 0x04) != 0)
    # a non-zero transmitted word: flip the roles of a decoded codeword
    sent = (xh >= 0.5).astype(np.uint8)
    got2 = lp.evaluate(code, dev(llr), x, sent=dev(sent))
    ref2 = oracle.evaluate(H, llr, xh.astype(np.float64), sent=sent)
    _check_eval(got2, ref2)
    assert np.all(host(got2[0]) == 0)


def test_evaluate_multi_matches_single():
    codes = [W.bsc_ensemble()[k] for k in range(4)] + [W.irregular_half(576)]
    lcodes = [lp.Code(H) for H in codes]
    rng = np.random.default_rng(3)
    cof = rng.integers(len(codes), size=40).astype(np.int32)
    lens = np.array([codes[c].n for c in cof], np.int64)
    off = np.zeros_like(lens)
    np.cumsum(lens[:-1], out=off[1:])
    llr = np.concatenate([W.bsc_llr(codes[c].n, 1, 0.08, rng)[0] for c in cof])
    x = (rng.random(llr.size) < 0.1).astype(np.float32)
    got = lp.evaluate_multi(lcodes, cof, off, dev(llr), dev(x), off)
    be, ch, cs, oc = (host(t) for t in got)
    for f, c in enumerate(cof):
        sl = slice(off[f], off[f] + codes[c].n)
        ref = oracle.evaluate(codes[c], llr[sl][None, :], x[sl][None, :].astype(np.float64))
        assert be[f] == ref["bit_errors"][0] and oc[f] == ref["outcome"][0]
        assert abs(ch[f] - ref["cost_hat"][0]) <= 1e-9
