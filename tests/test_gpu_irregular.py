"""GPU: the irregular rate-1/2 codes (variable degrees {2,3,6}, check degrees 6..8) in
the register-resident form, which holds up to eight degree-8 chunks per wave and
reads the edge metadata and variable tables from memory.

Messages after a fixed number of iterations are compared with the oracle, and the
resident, persistent-global and streamed forms with each other bitwise (every form
of a code uses the same chunk-to-wave plan, so the arithmetic is the same).
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


@pytest.mark.parametrize("n", W.IRREGULAR_LENGTHS)
def test_resident_messages_after_k_iterations(n):
    H = W.irregular_half(n)
    code = lp.Code(H)
    assert code.info["resident_capable"]
    assert code.launch_info(mode=lp.MODE_RESIDENT)["mode"] == lp.MODE_RESIDENT
    frames = 6 if n > 4000 else 12
    llr = W.awgn_batch(H, frames, 2.0, tag="irr-fixedk")
    for K in (1, 25):
        print(f"irregular n={n} K={K} frames={frames}", flush=True)
        x, it, fl, z, u = lp.decode_state(code, dev(llr), mode=lp.MODE_RESIDENT, tol=0.0, max_iter=K)
        ref = oracle.decode(H, llr, max_iter=K, tol=0.0, state=True)
        assert np.all(host(it) == K)
        assert np.abs(host(x) - ref.x).max() < 1e-4
        assert np.abs(host(z) - ref.z).max() < 1e-4
        assert np.abs(host(u) - ref.u).max() < 1e-4


@pytest.mark.parametrize("n", [576, 4608, 8064])
def test_forms_agree_bitwise_irregular(n):
    H = W.irregular_half(n)
    code = lp.Code(H)
    llr = W.awgn_batch(H, 24, 1.75, tag="irr-forms")
    llr[5, 7] = np.nan  # one invalid frame among them
    outs = []
    for m in (lp.MODE_RESIDENT, lp.MODE_PERSISTENT_GLOBAL, lp.MODE_STREAMED):
        print(f"irregular forms n={n} mode={m}", flush=True)
        x, it, fl = lp.decode(code, dev(llr), mode=m, max_iter=150)
        outs.append((host(x), host(it), host(fl)))
    assert outs[0][2][5] == lp.FLAG_INVALID and outs[0][1][5] == 0
    for o in outs[1:]:
        assert np.array_equal(o[1], outs[0][1])
        assert np.array_equal(o[2], outs[0][2])
        assert np.abs(o[0] - outs[0][0]).max() == 0.0


def test_resident_whole_decodes_against_oracle():
    H = W.irregular_half(2304)
    llr = np.concatenate([W.awgn_batch(H, 16, s, tag="irr-whole") for s in (1.5, 2.5)])
    print(f"irregular whole decodes frames={len(llr)}", flush=True)
    x, it, fl = lp.decode(lp.Code(H), dev(llr), mode=lp.MODE_RESIDENT)
    x, it, fl = host(x), host(it), host(fl)
    ref = oracle.decode(H, llr)
    ambiguous = np.any(np.abs(ref.x - 0.5) < 1e-3, axis=1)
    same = np.all((x >= 0.5) == (ref.x >= 0.5), axis=1)
    assert np.all(same | ambiguous)
    assert np.mean(np.abs(it.astype(int) - ref.iters) <= 2) >= 0.95


def test_degree6_code_in_a_degree_6_to_8_launch():
    """A (3,6) code batched with irregular codes runs in the degree-6..8 resident kernel
    (metadata from memory, mixed-degree variable tables); its frames still equal
    the degree-6 kernel's single-code decodes bitwise."""
    codes_h = [W.gallager36(2640), W.irregular_half(576), W.gallager36(96), W.irregular_half(2304)]
    handles = [lp.Code(H) for H in codes_h]
    batch = W.mixed_batch(codes_h, 160, 1.5, 3.0, tag="mix6-8", seed=3)
    flat, off = batch.flat_llr()
    print(f"mixed degree-6 / irregular batch frames={batch.frames}", flush=True)
    x, it, fl = lp.decode_multi(handles, batch.code_of_frame, off, dev(flat), off, flat.size, max_iter=300)
    x, it, fl = host(x), host(it), host(fl)
    for c, H in enumerate(codes_h):
        idx = np.nonzero(batch.code_of_frame == c)[0]
        if idx.size == 0:
            continue
        llr = np.stack([batch.llr[f] for f in idx])
        xs, its, fls = (host(t) for t in lp.decode(handles[c], dev(llr), max_iter=300))
        for k, f in enumerate(idx):
            assert np.array_equal(x[off[f]:off[f] + H.n], xs[k])
            assert it[f] == its[k] and fl[f] == fls[k]


def test_resident_warm_start_resume_is_exact():
    H = W.irregular_half(4608)
    code = lp.Code(H)
    llr = W.awgn_batch(H, 6, 1.5, tag="irr-warm")
    print(f"irregular warm start n={H.n}", flush=True)
    a = lp.decode_state(code, dev(llr), tol=0.0, max_iter=30, mode=lp.MODE_RESIDENT)
    b = lp.decode_state(code, dev(llr), tol=0.0, max_iter=12, mode=lp.MODE_RESIDENT)
    c = lp.decode_state(code, dev(llr), z=b[3], u=b[4], state_in=True, tol=0.0, max_iter=18,
                        mode=lp.MODE_RESIDENT)
    assert np.array_equal(host(a[3]), host(c[3])) and np.array_equal(host(a[4]), host(c[4]))
    assert np.array_equal(host(a[0]), host(c[0]))


def test_resident_tuning_and_autotune_keep_results():
    H = W.irregular_half(1152)
    code = lp.Code(H)
    llr = torch.from_numpy(np.concatenate([W.awgn_batch(H, 128, s, tag="irr-tune") for s in (1.5, 2.5)])).cuda()
    kw = dict(W.PAPER_PARAMS, max_iter=300, mode=lp.MODE_RESIDENT)
    ref = [host(t) for t in lp.decode(code, llr, **kw)]
    for bpc in (1, 2, 3):
        code.set_tuning(lp.MODE_RESIDENT, bpc, -1)
        assert code.launch_info(mode=lp.MODE_RESIDENT)["blocks_per_cu"] == bpc
        got = [host(t) for t in lp.decode(code, llr, **kw)]
        for r, g in zip(ref, got):
            assert np.array_equal(r, g), bpc
    (bpc, _), times = code.autotune(llr, max_blocks_per_cu=3, **kw)
    assert 1 <= bpc <= 3 and times
    got = [host(t) for t in lp.decode(code, llr, **kw)]
    for r, g in zip(ref, got):
        assert np.array_equal(r, g)
