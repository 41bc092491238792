"""GPU: the resident form with two frames per workgroup (variant 1) against the
one-frame resident kernel (variant 0) and the oracle.

Two frames share a workgroup of 12 waves, each physical wave hosting at most one
virtual wave (a wave of the code's plan) of each frame; the frames start, stop and
are replaced independently.  Every result must equal the one-frame kernel's
bitwise: x, iteration counts, flags, exported state, warm starts.  Codes: n = 2640
(21 chunks), 2304 (18), 2112 (17, the last one holding 32 checks) and 3072 (24
chunks, which the default leaves at one frame per workgroup).
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


def _batch(H, frames, tag):
    # Eb/N0 from 1.0 to 3.5 dB interleaved: neighbouring frames stop at very
    # different iterations, so the two frames of a workgroup fall out of step
    snrs = (1.0, 3.5, 1.75, 2.5, 3.0, 1.5)
    per = [W.awgn_batch(H, (frames + len(snrs) - 1) // len(snrs), s, tag=tag) for s in snrs]
    llr = np.stack([per[f % len(snrs)][f // len(snrs)] for f in range(frames)]).astype(np.float32)
    llr[frames // 3, 5] = np.nan  # one invalid frame
    return llr


def _both(code, fn):
    out = []
    for var in (0, 1):
        code.set_tuning(lp.MODE_RESIDENT, 0, var)
        assert code.launch_info(mode=lp.MODE_RESIDENT)["variant"] == var
        out.append([host(t) for t in fn()])
    code.set_tuning(lp.MODE_RESIDENT, 0, -1)
    return out


@pytest.mark.parametrize("n", [2640, 2304, 2112, 3072])
def test_two_frames_per_workgroup_equal_one(n):
    H = W.gallager36(n)
    code = lp.Code(H)
    li = code.launch_info(mode=lp.MODE_RESIDENT)
    assert li["variant"] == (0 if n == 3072 else 1)  # default: pairing only where it evens out the SIMDs
    llr = dev(_batch(H, 301, "pair"))
    print(f"pair n={n} frames=301", flush=True)
    a, b = _both(code, lambda: lp.decode(code, llr, mode=lp.MODE_RESIDENT))
    assert a[2][301 // 3] == lp.FLAG_INVALID and a[1][301 // 3] == 0
    assert len(np.unique(a[1])) > 10  # the frames really stop at different iterations
    for r, g in zip(a, b):
        assert np.array_equal(r, g)
    # frames at the iteration limit
    a, b = _both(code, lambda: lp.decode(code, llr, mode=lp.MODE_RESIDENT, max_iter=37))
    assert np.any(a[1] == 37)
    for r, g in zip(a, b):
        assert np.array_equal(r, g)


def test_two_frames_state_export_and_warm_start():
    H = W.gallager36(2112)
    code = lp.Code(H)
    llr = dev(_batch(H, 45, "pair-state"))
    print("pair state export", flush=True)
    a, b = _both(code, lambda: lp.decode_state(code, llr, mode=lp.MODE_RESIDENT, max_iter=60))
    for r, g in zip(a, b):
        assert np.array_equal(r, g)
    z0, u0 = dev(a[3]), dev(a[4])
    print("pair warm start", flush=True)
    a, b = _both(code, lambda: lp.decode_state(code, llr, z=z0.clone(), u=u0.clone(), state_in=True,
                                               mode=lp.MODE_RESIDENT, max_iter=25))
    for r, g in zip(a, b):
        assert np.array_equal(r, g)


@pytest.mark.parametrize("n", [2640, 2112])
def test_two_frames_messages_against_oracle(n):
    H = W.gallager36(n)
    code = lp.Code(H)
    assert code.launch_info(mode=lp.MODE_RESIDENT)["variant"] == 1
    llr = W.awgn_batch(H, 7, 2.0, tag="pair-oracle")
    print(f"pair oracle n={n}", flush=True)
    K = 20
    x, it, fl, z, u = lp.decode_state(code, dev(llr), mode=lp.MODE_RESIDENT, tol=0.0, max_iter=K)
    ref = oracle.decode(H, llr, max_iter=K, tol=0.0, state=True)
    assert np.all(host(it) == K)
    assert np.abs(host(x) - ref.x).max() < 1e-4
    assert np.abs(host(z) - ref.z).max() < 1e-4
    assert np.abs(host(u) - ref.u).max() < 1e-4


def test_two_frames_one_frame_batch_and_tuning():
    H = W.gallager36(2640)
    code = lp.Code(H)
    llr = _batch(H, 64, "pair-tune")
    print("pair single frame", flush=True)
    one = [host(t) for t in lp.decode(code, dev(llr[:1]), mode=lp.MODE_RESIDENT)]  # the second slot idles
    ref = [host(t) for t in lp.decode(code, dev(llr), mode=lp.MODE_RESIDENT)]
    for r, g in zip(ref, one):
        assert np.array_equal(r[:1], g)
    print("pair tuning", flush=True)
    for bpc in (1, 2):
        code.set_tuning(lp.MODE_RESIDENT, bpc, 1)
        got = [host(t) for t in lp.decode(code, dev(llr), mode=lp.MODE_RESIDENT)]
        for r, g in zip(ref, got):
            assert np.array_equal(r, g)
    code.set_tuning(lp.MODE_RESIDENT, 0, -1)
    (bpc, var), times = code.autotune(dev(llr), max_blocks_per_cu=2, mode=lp.MODE_RESIDENT)
    assert var in (0, 1) and set(times) == {(v, b) for v in (0, 1) for b in (1, 2)}
    got = [host(t) for t in lp.decode(code, dev(llr), mode=lp.MODE_RESIDENT)]
    for r, g in zip(ref, got):
        assert np.array_equal(r, g)
