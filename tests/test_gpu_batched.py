"""GPU: batched uneven decoding (several codes, one persistent launch), large codes
whose slot exchange lives in global memory, and FP16 message storage.

"Same alone and in the mix" is checked bitwise: a frame's arithmetic depends only
on its code's layout plan, never on which workgroup or launch decodes it.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_parity, parity_summary

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


def _mixed(frames, seed=0, lengths=W.IRREGULAR_LENGTHS, lo=1.5, hi=3.0):
    codes = [W.irregular_half(n) for n in lengths]
    batch = W.mixed_batch(codes, frames, lo, hi, seed=seed)
    flat, off = batch.flat_llr()
    return codes, batch, flat, off


def test_multi_code_frames_match_single_code_decodes_bitwise():
    codes, batch, flat, off = _mixed(192)
    handles = [lp.Code(H) for H in codes]
    print(f"multi-code batch frames={batch.frames}", flush=True)
    x, it, fl = lp.decode_multi(handles, batch.code_of_frame, off, dev(flat), off, flat.size)
    x, it, fl = host(x), host(it), host(fl)
    for c, H in enumerate(codes):
        idx = np.nonzero(batch.code_of_frame == c)[0]
        if idx.size == 0:
            continue
        llr = np.stack([batch.llr[f] for f in idx])
        xs, its, fls = lp.decode(handles[c], dev(llr))
        xs, its, fls = host(xs), host(its), host(fls)
        for k, f in enumerate(idx):
            assert np.array_equal(x[off[f]:off[f] + H.n], xs[k])
            assert it[f] == its[k] and fl[f] == fls[k]


def test_multi_code_degree6_mid_size_matches_single_code_decodes_bitwise():
    """(3,6) codes of n = 576, 2640 and 8064 in one launch: the fused launch runs the
    resident kernel with four chunks per wave (sized for n = 8064), so the smaller codes'
    frames go through a different kernel than when decoded alone (one or two chunks per
    wave, or two frames per workgroup); the results are bitwise the same."""
    codes = [W.gallager36(n) for n in (576, 2640, 8064)]
    batch = W.mixed_batch(codes, 96, 1.5, 3.0, seed=4)
    flat, off = batch.flat_llr()
    handles = [lp.Code(H) for H in codes]
    x, it, fl = lp.decode_multi(handles, batch.code_of_frame, off, dev(flat), off, flat.size)
    x, it, fl = host(x), host(it), host(fl)
    for c, H in enumerate(codes):
        idx = np.nonzero(batch.code_of_frame == c)[0]
        if idx.size == 0:
            continue
        llr = np.stack([batch.llr[f] for f in idx])
        xs, its, fls = lp.decode(handles[c], dev(llr))
        xs, its, fls = host(xs), host(its), host(fls)
        for k, f in enumerate(idx):
            assert np.array_equal(x[off[f]:off[f] + H.n], xs[k]), (H.n, f)
            assert it[f] == its[k] and fl[f] == fls[k]


def test_multi_code_against_oracle():
    codes, batch, flat, off = _mixed(96, seed=1)
    handles = [lp.Code(H) for H in codes]
    x, it, fl = lp.decode_multi(handles, batch.code_of_frame, off, dev(flat), off, flat.size)
    x, it, fl = host(x), host(it), host(fl)
    for c, H in enumerate(codes):
        idx = np.nonzero(batch.code_of_frame == c)[0]
        if idx.size == 0:
            continue
        llr = np.stack([batch.llr[f] for f in idx])
        ref = oracle.decode(H, llr)
        for k, f in enumerate(idx):
            xg = x[off[f]:off[f] + H.n]
            ambiguous = np.any(np.abs(ref.x[k] - 0.5) < 1e-3)
            assert ambiguous or np.array_equal(xg >= 0.5, ref.x[k] >= 0.5)
            assert abs(int(it[f]) - int(ref.iters[k])) <= 2 or ambiguous


def test_multi_code_rejects_bad_offsets():
    codes, batch, flat, off = _mixed(4, seed=2, lengths=(576,))
    handles = [lp.Code(H) for H in codes]
    bad = off.copy()
    bad[-1] = flat.size  # frame would read past the end
    with pytest.raises(lp.LpdecError) as e:
        lp.decode_multi(handles, batch.code_of_frame, bad, dev(flat), off, flat.size)
    assert e.value.status == -1 and "outside llr_len" in str(e.value)


@pytest.mark.parametrize("which", ["36", "48"])
def test_large_codes_global_slots(which):
    """n = 16384: the slot exchange exceeds LDS and goes through global scratch."""
    H = W.gallager36(16384) if which == "36" else W.gallager48(16384)
    llr = W.awgn_batch(H, 8, 2.5, tag="large")
    code = lp.Code(H)
    assert not code.info["resident_capable"]
    print(f"large code {which} n={H.n} nnz={H.nnz}", flush=True)
    for m in (lp.MODE_PERSISTENT_GLOBAL, lp.MODE_STREAMED):
        x, it, fl, z, u = lp.decode_state(code, dev(llr), mode=m, tol=0.0, max_iter=20)
        ref = oracle.decode(H, llr, max_iter=20, tol=0.0, state=True)
        assert np.abs(host(x) - ref.x).max() < 1e-4
        assert np.abs(host(z) - ref.z).max() < 1e-4 and np.abs(host(u) - ref.u).max() < 1e-4
    x, it, fl = lp.decode(code, dev(llr))
    ref = oracle.decode(H, llr)
    assert np.array_equal(host(x) >= 0.5, ref.x >= 0.5)


def test_fp16_storage_error_is_bounded():
    """FP16 z/u storage with FP32 compute (streamed form) against FP32 storage and the
    oracle after a fixed number of iterations.  FP16 keeps 11 significant bits; one
    rounding per stored value and iteration gives |dz| <= 2^-11 per step."""
    H = W.gallager36(2640)
    llr = W.awgn_batch(H, 16, 2.5, tag="fp16")
    code = lp.Code(H)
    K = 20
    ref = oracle.decode(H, llr, max_iter=K, tol=0.0, state=True)
    x16, _, _, z16, u16 = lp.decode_state(code, dev(llr), mode=lp.MODE_STREAMED, storage=lp.STORAGE_FP16,
                                          tol=0.0, max_iter=K)
    x16, z16, u16 = host(x16), host(z16), host(u16)
    ex, ez, eu = np.abs(x16 - ref.x).max(), np.abs(z16 - ref.z).max(), np.abs(u16 - ref.u).max()
    print(f"fp16 storage K={K}: max|dx|={ex:.2e} max|dz|={ez:.2e} max|dlambda|={3 * eu:.2e}", flush=True)
    assert ex < 2e-2 and ez < 2e-2 and eu < 5e-2
    # full decodes: hard decisions agree with FP32 storage on nearly every frame
    llr = W.awgn_batch(H, 256, 2.5, tag="fp16b")
    x32, it32, _ = lp.decode(code, dev(llr), mode=lp.MODE_STREAMED)
    x16, it16, fl16 = lp.decode(code, dev(llr), mode=lp.MODE_STREAMED, storage=lp.STORAGE_FP16)
    agree = np.all((host(x32) >= 0.5) == (host(x16) >= 0.5), axis=1)
    assert agree.mean() >= 0.99


def test_largest_codes_use_global_slots():
    # (3,6) n = 21840 has nnz = 65520, just under the 16-bit index limit; 8 n bytes
    # of accumulators exceed the LDS, so the slot exchange lives in global memory.
    H = W.gallager_regular(21840, 3, 6, seed=3)
    assert H.nnz == 65520
    llr = W.awgn_batch(H, 3, 2.5, tag="largest")
    code = lp.Code(H)
    ref = oracle.decode(H, llr, max_iter=15, tol=0.0, state=True)
    outs = []
    for m in (lp.MODE_PERSISTENT_GLOBAL, lp.MODE_STREAMED):
        print(f"largest code n={H.n} mode={m}", flush=True)
        x, it, fl, z, u = lp.decode_state(code, dev(llr), mode=m, max_iter=15, tol=0.0)
        x, z, u = host(x), host(z), host(u)
        assert np.abs(x - ref.x).max() <= 1e-4
        assert np.abs(z - ref.z).max() <= 1e-4 and np.abs(u - ref.u).max() <= 1e-4
        outs.append((x, z, u))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


_UNEVEN = {}


def _uneven_full():
    """The full 16384-frame uneven batch decoded once, in the launch the benchmark
    times (one decode_multi call over the six codes)."""
    if not _UNEVEN:
        codes_h = [W.irregular_half(n) for n in W.IRREGULAR_LENGTHS]
        batch = W.mixed_batch(codes_h, 16384, 1.5, 3.0, tag="uneven")
        flat, off = batch.flat_llr()
        handles = [lp.Code(H) for H in codes_h]
        print(f"uneven full batch frames={batch.frames}", flush=True)
        x, it, fl = lp.decode_multi(handles, batch.code_of_frame, off, dev(flat), off, flat.size,
                                    **W.PAPER_PARAMS)
        _UNEVEN.update(codes=codes_h, batch=batch, off=off, x=host(x), it=host(it), fl=host(fl))
    return _UNEVEN


@pytest.mark.parametrize("n", W.IRREGULAR_LENGTHS)
def test_uneven_batch_full_size(n):
    """1024 frames of each code of the full uneven batch against the oracle (all host
    cores), and every frame's flags against a host recomputation of the certificate."""
    u = _uneven_full()
    c = W.IRREGULAR_LENGTHS.index(n)
    H, batch, off = u["codes"][c], u["batch"], u["off"]
    idx = np.nonzero(batch.code_of_frame == c)[0]
    pick = idx[:1024]
    llr = np.stack([batch.llr[f] for f in pick])
    print(f"oracle on {len(pick)} frames of n={n}", flush=True)
    ref = oracle.decode(H, llr, **W.PAPER_PARAMS)
    xs = np.stack([u["x"][off[f]:off[f] + H.n] for f in pick])
    assert_parity(parity_summary(xs, u["it"][pick], u["fl"][pick], ref), f"uneven n={n}")
    Hd = H.to_scipy()
    xa = np.stack([u["x"][off[f]:off[f] + H.n] for f in idx])
    codeword = ~np.any((Hd @ (xa >= 0.5).astype(np.int64).T) % 2, axis=0)
    integral = np.max(np.minimum(xa, 1 - xa), axis=1) <= 1e-3
    assert np.array_equal(codeword, (u["fl"][idx] & 0x04) != 0)
    assert np.array_equal(integral, (u["fl"][idx] & 0x02) != 0)


_PRECISION = {}


def _precision_full(which):
    """The 8192-frame n = 16384 batch of the precision study in the launches the
    benchmark times, FP32 and FP16 storage, decoded once: the streamed form, and the
    persistent-global form (which must give bitwise the same result on every frame)."""
    if which not in _PRECISION:
        H = W.gallager36(16384) if which == "36" else W.gallager48(16384)
        llr_h = W.awgn_batch(H, 8192, 2.5, tag="precision")
        code = lp.Code(H)
        print(f"precision batch ({which}) frames=8192", flush=True)
        out, out_pg = {}, {}
        for st in (lp.STORAGE_FP32, lp.STORAGE_FP16):
            x, it, fl = lp.decode(code, dev(llr_h), mode=lp.MODE_STREAMED, storage=st, **W.PAPER_PARAMS)
            out[st] = (host(x), host(it), host(fl))
            x, it, fl = lp.decode(code, dev(llr_h), mode=lp.MODE_PERSISTENT_GLOBAL, storage=st, **W.PAPER_PARAMS)
            out_pg[st] = (host(x), host(it), host(fl))
        _PRECISION[which] = (H, llr_h, out, out_pg)
    return _PRECISION[which]


@pytest.mark.parametrize("which", ["36", "48"])
def test_precision_batch_forms_agree_on_every_frame(which):
    """Both storages: the persistent-global form (every chunk held in registers where
    the registers allow it) equals the streamed form bitwise on all 8192 frames."""
    _, _, out, out_pg = _precision_full(which)
    for st in (lp.STORAGE_FP32, lp.STORAGE_FP16):
        for a, b in zip(out[st], out_pg[st]):
            assert np.array_equal(a, b), (which, st)


@pytest.mark.parametrize("which,part", [("36", 0), ("48", 0), ("48", 1)])
def test_precision_batch_full_size(which, part):
    """Every frame of the precision batches in FP32 storage against the oracle (the
    (4,8) batch in two halves, to keep each test's oracle run short), and FP16 hard
    decisions against FP32 on every frame."""
    H, llr_h, out, _ = _precision_full(which)
    sl = slice(0, 8192) if which == "36" else slice(part * 4096, (part + 1) * 4096)
    print(f"oracle on frames {sl.start}..{sl.stop} of ({which})", flush=True)
    ref = oracle.decode(H, llr_h[sl], **W.PAPER_PARAMS)
    x32, it32, fl32 = (a[sl] for a in out[lp.STORAGE_FP32])
    assert_parity(parity_summary(x32, it32, fl32, ref), f"precision ({which}) fp32 frames {sl.start}..{sl.stop}")
    x16 = out[lp.STORAGE_FP16][0][sl]
    ambiguous = np.any(np.abs(ref.x - 0.5) < 1e-3, axis=1)
    agree16 = np.all((x16 >= 0.5) == (ref.x >= 0.5), axis=1)[~ambiguous].mean()
    agree = np.all((x32 >= 0.5) == (x16 >= 0.5), axis=1)
    print(f"fp16 hard-decision agreement: with fp32 {agree.mean():.5f}, with the oracle {agree16:.5f}", flush=True)
    assert agree.mean() >= 0.999
