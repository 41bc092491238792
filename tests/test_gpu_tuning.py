"""Launch tuning and the autotuner: the launch shape changes speed only, never
results (frames are independent and every in-frame sum has a fixed order)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

lp = pytest.importorskip("paper_1204_0556_amd")

FORMS = {"resident": 1, "streamed": 2, "persistent_global": 3}


def _decode(code, llr, mode, **kw):
    x, it, fl = lp.decode(code, llr, mode=mode, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy(), it.cpu().numpy(), fl.cpu().numpy()


@pytest.mark.parametrize("form", list(FORMS))
def test_launch_info(form):
    H = W.gallager36(2640)
    code = lp.Code(H)
    li = code.launch_info(mode=FORMS[form])
    assert li["mode"] == FORMS[form]
    assert li["threads"] % 64 == 0 and li["threads"] >= 64
    assert li["vgprs"] > 0 and li["blocks_per_cu"] >= 1 and li["resource_blocks_per_cu"] >= 1
    assert li["lds_bytes"] > 0


@pytest.mark.parametrize("form", list(FORMS))
def test_results_do_not_depend_on_the_launch_shape(form):
    H = W.gallager36(2640)
    code = lp.Code(H)
    llr = torch.from_numpy(np.concatenate([W.awgn_batch(H, 96, s, tag="tune") for s in (1.5, 2.5)])).cuda()
    kw = dict(W.PAPER_PARAMS, max_iter=300)
    ref = _decode(code, llr, FORMS[form], **kw)
    shapes = [(1, -1), (2, -1), (3, -1)]
    if form == "streamed":
        shapes += [(1, 0), (2, 0), (1, 1), (2, 1), (1, 2), (2, 2)]
    for bpc, var in shapes:
        code.set_tuning(FORMS[form], bpc, var)
        if form == "streamed" and var >= 0:
            assert code.launch_info(mode=FORMS[form])["variant"] == var
        got = _decode(code, llr, FORMS[form], **kw)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (form, bpc, var)
    code.set_tuning(FORMS[form], 0, -1)


def test_autotune_keeps_results_and_records_choice():
    H = W.gallager36(2640)
    code = lp.Code(H)
    llr = torch.from_numpy(W.awgn_batch(H, 512, 2.0, tag="tune")).cuda()
    kw = dict(W.PAPER_PARAMS, max_iter=200)
    ref = _decode(code, llr, lp.MODE_STREAMED, **kw)
    (bpc, var), times = code.autotune(llr, max_blocks_per_cu=2, mode=lp.MODE_STREAMED, **kw)
    assert 1 <= bpc <= 2 and var in (0, 1, 2)
    assert len(times) == 6 and all(t > 0 for t in times.values())
    assert times[(var, bpc)] == min(times.values())
    assert code.launch_info(mode=lp.MODE_STREAMED)["variant"] == var
    assert code.launch_info(mode=lp.MODE_STREAMED)["blocks_per_cu"] == bpc
    got = _decode(code, llr, lp.MODE_STREAMED, **kw)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_tuning_rejects_bad_values():
    code = lp.Code(W.gallager36(96))
    with pytest.raises(lp.LpdecError):
        code.set_tuning(lp.MODE_AUTO, 1, -1)
    with pytest.raises(lp.LpdecError):
        code.set_tuning(lp.MODE_RESIDENT, 33, -1)
    with pytest.raises(lp.LpdecError):
        code.set_tuning(lp.MODE_STREAMED, 1, lp.TUNE_VARIANTS)
    code.set_tuning(lp.MODE_STREAMED, 1, 3)  # a variant the form lacks falls back to the highest allowed
    assert code.launch_info(mode=lp.MODE_STREAMED)["variant"] == 2
    code.set_tuning(lp.MODE_STREAMED, 1, 2)  # n = 96: staging allowed, default already


def test_multi_autotune_keeps_results_and_records_choice():
    codes_h = [W.irregular_half(n) for n in (576, 2304, 8064)]
    batch = W.mixed_batch(codes_h, 512, 1.5, 3.0, tag="tune-multi")
    flat, off = batch.flat_llr()
    codes = [lp.Code(H) for H in codes_h]
    llr = torch.from_numpy(flat).cuda()
    kw = dict(W.PAPER_PARAMS, max_iter=200)

    def run(**extra):
        x, it, fl = lp.decode_multi(codes, batch.code_of_frame, off, llr, off, flat.size, **kw, **extra)
        torch.cuda.synchronize()
        return x.cpu().numpy(), it.cpu().numpy(), fl.cpu().numpy()

    ref = run()
    (mode, bpc, order), times = lp.autotune_multi(codes, batch.code_of_frame, off, llr, max_blocks_per_cu=2, **kw)
    print(f"multi-code tuning: mode {mode} blocks {bpc} order {order}; {times}", flush=True)
    assert mode in (lp.MODE_RESIDENT, lp.MODE_PERSISTENT_GLOBAL) and 1 <= bpc <= 2 and order in (0, 1)
    # every code fits the resident form: both forms, both orders, two grids were timed
    assert len(times) == 8 and all(v > 0 for v in times.values())
    for a, b in zip(ref, run(mode=mode)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("which", ["36", "48"])
def test_large_code_held_chunk_variants_agree_bitwise(which):
    """The n = 16384 codes: every held-chunk variant of the accumulator kernel (and
    k_decode's walk) in the persistent-global and streamed forms, FP32 and FP16
    storage, gives bitwise the result of the default launch."""
    H = W.gallager36(16384) if which == "36" else W.gallager48(16384)
    code = lp.Code(H)
    llr = torch.from_numpy(np.concatenate([W.awgn_batch(H, 24, s, tag="held") for s in (2.0, 2.5)])).cuda()
    kw = dict(W.PAPER_PARAMS, max_iter=40)
    for mode, storage in ((lp.MODE_PERSISTENT_GLOBAL, 0), (lp.MODE_STREAMED, 0), (lp.MODE_STREAMED, 1)):
        ref = _decode(code, llr, mode, storage=storage, **kw)
        # persistent-global FP32, degree 6: variant 3 holds every chunk with two of the
        # plan's waves per hardware wave (512 threads)
        variants = (0, 1, 2, 3) if (mode == lp.MODE_PERSISTENT_GLOBAL and which == "36") else (0, 1, 2)
        for var in variants:
            code.set_tuning(mode, 0, var)
            assert code.launch_info(mode=mode, storage=storage)["variant"] == var
            print(f"({which}) mode {mode} storage {storage} variant {var}", flush=True)
            if var == 3:
                assert code.launch_info(mode=mode, storage=storage)["threads"] == 512
            got = _decode(code, llr, mode, storage=storage, **kw)
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), (which, mode, storage, var)
        code.set_tuning(mode, 0, -1)


@pytest.mark.parametrize("which", ["36", "48"])
def test_fp16_persistent_global_equals_streamed(which):
    """FP16 storage in the persistent-global form (held chunks as packed FP16 pairs in
    registers, the rest in FP16 scratch) rounds exactly as the streamed form's FP16
    stores do: bitwise the same x, iterations and flags, for every held-chunk variant,
    from a zero start and from an exported state."""
    H = W.gallager36(16384) if which == "36" else W.gallager48(16384)
    code = lp.Code(H)
    llr = torch.from_numpy(np.concatenate([W.awgn_batch(H, 24, s, tag="half-pg") for s in (2.0, 2.5)])).cuda()
    kw = dict(W.PAPER_PARAMS, max_iter=60, storage=lp.STORAGE_FP16)
    ref = _decode(code, llr, lp.MODE_STREAMED, **kw)
    for var in (0, 1):
        code.set_tuning(lp.MODE_PERSISTENT_GLOBAL, 0, var)
        li = code.launch_info(mode=lp.MODE_PERSISTENT_GLOBAL, storage=lp.STORAGE_FP16)
        print(f"({which}) FP16 persistent-global variant {var}: {li}", flush=True)
        got = _decode(code, llr, lp.MODE_PERSISTENT_GLOBAL, **kw)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (which, var)
    code.set_tuning(lp.MODE_PERSISTENT_GLOBAL, 0, -1)
    # 12 + 18 iterations through the exported (FP16-valued) state equal 30 in one go
    sub = llr[:6].contiguous()
    kw = dict(tol=0.0, storage=lp.STORAGE_FP16, mode=lp.MODE_PERSISTENT_GLOBAL)
    a = lp.decode_state(code, sub, max_iter=30, **kw)
    b = lp.decode_state(code, sub, max_iter=12, **kw)
    c = lp.decode_state(code, sub, z=b[3], u=b[4], state_in=True, max_iter=18, **kw)
    s = lp.decode_state(code, sub, max_iter=30, tol=0.0, storage=lp.STORAGE_FP16, mode=lp.MODE_STREAMED)
    for k in (0, 3, 4):
        assert np.array_equal(a[k].cpu().numpy(), c[k].cpu().numpy())
        assert np.array_equal(a[k].cpu().numpy(), s[k].cpu().numpy())


def test_fp16_persistent_global_needs_an_accumulator_code():
    # n = 2640 exchanges through LDS float slots: no FP16 persistent-global kernel
    code = lp.Code(W.gallager36(2640))
    llr = torch.from_numpy(W.awgn_batch(W.gallager36(2640), 4, 2.5, tag="half-pg-no")).cuda()
    with pytest.raises(lp.LpdecError):
        lp.decode(code, llr, mode=lp.MODE_PERSISTENT_GLOBAL, storage=lp.STORAGE_FP16)
    with pytest.raises(lp.LpdecError):
        lp.decode(code, llr, mode=lp.MODE_RESIDENT, storage=lp.STORAGE_FP16)


@pytest.mark.parametrize("which", ["36", "48"])
def test_large_code_forms_agree_bitwise(which):
    """n = 16384, FP32: the persistent-global default ((3,6): every chunk held, two of
    the plan's waves per hardware wave; (4,8): one held chunk) and the streamed default
    give bitwise the same x, iterations and flags."""
    H = W.gallager36(16384) if which == "36" else W.gallager48(16384)
    code = lp.Code(H)
    llr = torch.from_numpy(np.concatenate([W.awgn_batch(H, 24, s, tag="forms-large") for s in (2.0, 2.5)])).cuda()
    kw = dict(W.PAPER_PARAMS, max_iter=80)
    pg = _decode(code, llr, lp.MODE_PERSISTENT_GLOBAL, **kw)
    st = _decode(code, llr, lp.MODE_STREAMED, **kw)
    print(f"({which}) forms: {code.launch_info(mode=lp.MODE_PERSISTENT_GLOBAL)}", flush=True)
    for a, b in zip(pg, st):
        assert np.array_equal(a, b), which
