"""Check degree 13: the (3,13) code class of Sec. 5 ([1057,813], stand-in code).

Checks above degree 8 run in the persistent-global and streamed forms, and in the
resident form when the code needs one chunk per wave, with the projection of
Algorithm 2 on 9..16 coordinates.  The decoder's state after a fixed number of
iterations matches the oracle, the forms give bitwise the same decodes, and the
forms that do not take such codes refuse them.
"""
import numpy as np
import pytest

import oracle
import workloads as W

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


FORMS = {"resident": 1, "persistent_global": 3, "streamed": 2}
LARGE_FORMS = {"persistent_global": 3, "streamed": 2}


def _llr(H, frames, snr, tag):
    # noise for Eb/N0 at the code's rate (H has full rank: 1 - m/n = 813/1057 for n = 1057)
    return W.awgn_batch(H, frames, snr, tag=tag, rate=1.0 - H.m / H.n)


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("K", [1, 10, 60])
def test_code313_state_after_k_iterations(K, form):
    H = W.code313(1057)
    llr = _llr(H, 12, 3.0, "313-fixedk")
    print(f"(3,13) n=1057 K={K} form={form}", flush=True)
    x, it, fl, z, u = lp.decode_state(lp.Code(H), dev(llr), tol=0.0, max_iter=K, mode=FORMS[form])
    ref = oracle.decode(H, llr, mu=3.0, rho=1.9, max_iter=K, tol=0.0, state=True)
    assert np.all(host(it) == K)
    assert np.abs(host(x) - ref.x).max() < 1e-4
    assert np.abs(host(z) - ref.z).max() < 1e-4
    assert np.abs(host(u) - ref.u).max() < 1e-4


def test_code313_decodes_match_oracle_and_agree_across_forms():
    H = W.code313(1057)
    # 3.0 dB: about a tenth of the frames end as pseudocodewords or at the iteration limit
    llr = np.concatenate([_llr(H, 150, s, "313-full") for s in (3.0, 3.5)])
    code = lp.Code(H)
    li = code.launch_info()
    print(f"(3,13) n=1057 AUTO: {li}", flush=True)
    assert li["mode"] == lp.MODE_RESIDENT and code.info["resident_capable"]
    outs = {}
    for name, m in FORMS.items():
        x, it, fl = lp.decode(code, dev(llr), mode=m, **W.PAPER_PARAMS)
        outs[name] = (host(x), host(it), host(fl))
    a = outs["resident"]
    for b in (outs["persistent_global"], outs["streamed"]):
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        assert np.abs(a[0] - b[0]).max() == 0.0
    ref = oracle.decode(H, llr, **W.PAPER_PARAMS)
    x, it, fl = a
    ambiguous = np.any(np.abs(ref.x - 0.5) < 1e-3, axis=1)
    same = np.all((x >= 0.5) == (ref.x >= 0.5), axis=1)
    assert np.all(same | ambiguous), np.nonzero(~(same | ambiguous))[0]
    assert np.mean(np.abs(it.astype(int) - ref.iters) <= 2) >= 0.99
    assert np.mean((fl & 0x0F) == (ref.flags & 0x0F)) >= 0.99


def test_code313_large_accumulator_exchange():
    # n = 16380 (13 | n): 4 (E + n) bytes exceed the LDS, the exchange runs on
    # fixed-point accumulators; 60 chunks on 16 waves take the 1024-thread build
    H = W.code313(16380)
    llr = _llr(H, 4, 3.0, "313-large")
    code = lp.Code(H)
    assert not code.info["resident_capable"]  # four chunks per wave
    with pytest.raises(lp.LpdecError):
        lp.decode(code, dev(llr), mode=lp.MODE_RESIDENT)
    K = 12
    ref = oracle.decode(H, llr, mu=3.0, rho=1.9, max_iter=K, tol=0.0, state=True)
    outs = []
    for name, m in LARGE_FORMS.items():
        print(f"(3,13) n=16380 K={K} form={name}: {code.launch_info(mode=m)}", flush=True)
        x, it, fl, z, u = lp.decode_state(code, dev(llr), tol=0.0, max_iter=K, mode=m)
        x, z, u = host(x), host(z), host(u)
        assert np.abs(x - ref.x).max() < 1e-4
        assert np.abs(z - ref.z).max() < 1e-4 and np.abs(u - ref.u).max() < 1e-4
        outs.append((x, z, u))
    for p, q in zip(outs[0], outs[1]):
        assert np.abs(p - q).max() == 0.0


def test_code313_fp16_storage():
    H = W.code313(1057)
    llr = _llr(H, 200, 3.0, "313-fp16")
    code = lp.Code(H)
    x32, _, fl32 = lp.decode(code, dev(llr), mode=lp.MODE_STREAMED, **W.PAPER_PARAMS)
    x16, _, _ = lp.decode(code, dev(llr), mode=lp.MODE_STREAMED, storage=lp.STORAGE_FP16, **W.PAPER_PARAMS)
    h32, h16 = host(x32) >= 0.5, host(x16) >= 0.5
    # frames whose FP32 decode is certified (the LP optimum is that codeword): FP16
    # storage reaches the same word; word-error counts stay close
    cert = (host(fl32) & 0x08) != 0
    agree = np.all(h32 == h16, axis=1)
    print(f"fp16 (3,13): certified {cert.sum()}, agree on them {agree[cert].mean():.3f}, "
          f"word errors fp32 {h32.any(1).sum()} fp16 {h16.any(1).sum()}", flush=True)
    assert cert.sum() >= 150
    assert agree[cert].mean() >= 0.99
    assert abs(int(h32.any(1).sum()) - int(h16.any(1).sum())) <= 10


def test_code313_mixed_with_degree6_code():
    # a multi-code batch holding a degree-13 and a degree-6 code runs the 2..16
    # build for both; each frame's result equals its single-code decode
    H13, H6 = W.code313(1057), W.gallager36(2640)
    l13 = _llr(H13, 40, 3.0, "313-mix")
    l6 = W.awgn_batch(H6, 40, 2.0, tag="313-mix")
    c13, c6 = lp.Code(H13), lp.Code(H6)
    kw = dict(max_iter=200)
    singles = [tuple(host(t) for t in lp.decode(c, dev(l), mode=lp.MODE_PERSISTENT_GLOBAL, **kw))
               for c, l in ((c13, l13), (c6, l6))]
    order = np.arange(80)
    cof = (order % 2).astype(np.int32)  # interleaved frames: code 0, 1, 0, 1, ...
    frames = [l13[i // 2] if c == 0 else l6[i // 2] for i, c in zip(order, cof)]
    lens = np.array([f.size for f in frames], np.int64)
    off = np.zeros(80, np.int64)
    np.cumsum(lens[:-1], out=off[1:])
    flat = np.concatenate(frames).astype(np.float32)
    print("(3,13) + (3,6) multi-code batch, 80 frames", flush=True)
    x, it, fl = lp.decode_multi([c13, c6], cof, off, dev(flat), off, flat.size, **kw)
    x, it, fl = host(x), host(it), host(fl)
    for i in range(80):
        c, k = cof[i], i // 2
        xs, its, fls = singles[c]
        assert it[i] == its[k] and fl[i] == fls[k]
        assert np.array_equal(x[off[i]:off[i] + lens[i]], xs[k])


def test_code313_dual_is_refused():
    H = W.code313(1057)
    code = lp.Code(H)
    llr = dev(_llr(H, 4, 3.0, "313-refuse"))
    with pytest.raises(lp.LpdecError) as e:
        lp.decode_dual(code, llr)
    assert "degree" in str(e.value)
