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
        code.set_tuning(lp.MODE_STREAMED, 1, 3)
    code.set_tuning(lp.MODE_STREAMED, 1, 2)  # n = 96: staging allowed, default already
