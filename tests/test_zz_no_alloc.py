"""lpdec_decode_noalloc: the allocation-free decode entry point.

Its scratch is a static device array shared by every call on a GPU; results
must be bitwise those of lpdec_decode (the same kernels; a frame's result does
not depend on the grid, which the array may cut).  Each case makes two calls in
a row, the second with fewer frames, so the second call runs on whatever the
first left in the array.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

lp = pytest.importorskip("paper_1204_0556_amd")


def _llr(H, frames, tag):
    snrs = (1.5, 2.0, 2.5, 3.0)
    per = [(frames + k) // len(snrs) for k in range(len(snrs))]
    a = np.concatenate([W.awgn_batch(H, c, s, tag=tag) for c, s in zip(per, snrs)])
    return torch.from_numpy(a).cuda()


def _out(B, n):
    return (torch.full((B, n), -1.0, dtype=torch.float32, device="cuda"),
            torch.full((B,), -1, dtype=torch.int32, device="cuda"),
            torch.full((B,), 0xEE, dtype=torch.uint8, device="cuda"))


def _both(code, llr, **kw):
    ref = lp.decode(code, llr, **kw)
    got = lp.decode_noalloc(code, llr, _out(llr.shape[0], code.n), **kw)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in got]


def _same(ref, got, what):
    for name, a, b in zip(("x", "iters", "flags"), ref, got):
        assert np.array_equal(a, b), f"{what}: {name} differs ({np.sum(a != b)} entries)"


# (code, first batch, second batch, max_iter, expected mode): the headline code
# in the resident form (the first batch is large enough for two frames per
# workgroup), an irregular code with degree 6..8 checks (resident, gamma/mu staged
# in the array), and a code too large for registers (persistent-global: state,
# previous x and gamma/mu per workgroup in the array, grid cut to fit); and the
# (3,13) code class: one chunk per wave (resident) and n = 16380 (persistent-global,
# fixed-point accumulators, checks of degree 13)
CASES = {
    "n2640_resident": (lambda: W.gallager36(2640), 600, 40, 300, lp.MODE_RESIDENT),
    "n8064_irregular": (lambda: W.irregular_half(8064), 300, 20, 200, lp.MODE_RESIDENT),
    "n16384_persistent_global": (lambda: W.gallager36(16384), 300, 16, 60, lp.MODE_PERSISTENT_GLOBAL),
    "n1057_degree13_resident": (lambda: W.code313(1057), 600, 40, 300, lp.MODE_RESIDENT),
    "n16380_degree13_persistent_global": (lambda: W.code313(16380), 200, 12, 40, lp.MODE_PERSISTENT_GLOBAL),
}


@pytest.mark.parametrize("case", list(CASES))
def test_noalloc_matches_decode_on_two_calls(case):
    make, b1, b2, max_iter, mode = CASES[case]
    H = make()
    code = lp.Code(H)
    assert code.launch_info()["mode"] == mode
    kw = dict(W.PAPER_PARAMS, max_iter=max_iter)
    print(f"case {case}: n={H.n} batches {b1} then {b2}", flush=True)
    llr1 = _llr(H, b1, "noalloc1")
    ref, got = _both(code, llr1, **kw)
    _same(ref, got, f"{case} first call ({b1} frames)")
    assert np.all(got[1] >= 1)
    llr2 = _llr(H, b2, "noalloc2")
    ref, got = _both(code, llr2, **kw)
    _same(ref, got, f"{case} second call ({b2} frames)")


def test_noalloc_after_other_codes_and_with_invalid_frames():
    # the array keeps the last call's contents: a call after calls of other codes
    # (and a frame with a non-finite LLR) must still match
    Ha, Hb = W.gallager36(2640), W.gallager36(16384)
    ca, cb = lp.Code(Ha), lp.Code(Hb)
    kw = dict(W.PAPER_PARAMS, max_iter=100)
    la = _llr(Ha, 64, "noalloc3")
    la[5, 7] = float("nan")
    first = lp.decode_noalloc(ca, la, _out(64, Ha.n), **kw)
    torch.cuda.synchronize()
    first = [t.cpu().numpy() for t in first]
    lp.decode_noalloc(cb, _llr(Hb, 32, "noalloc4"), _out(32, Hb.n), **kw)
    ref, again = _both(ca, la, **kw)
    _same(ref, again, "after other codes")
    _same(first, again, "repeated call")
    assert again[2][5] == lp.FLAG_INVALID


def test_noalloc_rejects_the_streamed_form_and_fp16_storage():
    H = W.gallager36(2640)
    code = lp.Code(H)
    llr = _llr(H, 8, "noalloc5")
    for kw in (dict(mode=lp.MODE_STREAMED), dict(storage=lp.STORAGE_FP16)):
        with pytest.raises(lp.LpdecError) as e:
            lp.decode_noalloc(code, llr, _out(8, H.n), **kw)
        assert e.value.status == -4, kw
    # empty batch: a no-op
    lp.decode_noalloc(code, llr[:0], _out(0, H.n))
