"""The streamed form replayed from captured HIP graphs: every replay must give the
result of direct launches.  Each decode replays its cached graph many times (one
replay per block of 16 iterations); the decodes are repeated with other eager work
and synchronisations in between, with new buffers (a new capture), and with an
iteration limit that is not a multiple of the block."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

lp = pytest.importorskip("paper_1204_0556_amd")


def _run(code, llr, graph, **kw):
    code.set_graph(graph)
    x, it, fl = lp.decode(code, llr, mode=lp.MODE_STREAMED, **kw)
    torch.cuda.synchronize()
    code.set_graph(False)
    return x.cpu().numpy(), it.cpu().numpy(), fl.cpu().numpy()


def _state(code, llr, graph, **kw):
    code.set_graph(graph)
    out = lp.decode_state(code, llr, mode=lp.MODE_STREAMED, **kw)
    torch.cuda.synchronize()
    code.set_graph(False)
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_graph_replay_matches_direct_launches(variant):
    H = W.gallager36(2640)
    code = lp.Code(H)
    code.set_tuning(lp.MODE_STREAMED, 0, variant)
    llr = torch.from_numpy(np.concatenate([W.awgn_batch(H, 256, s, tag="graph") for s in (1.5, 2.5)])).cuda()
    kw = dict(W.PAPER_PARAMS, max_iter=150)
    ref = _run(code, llr, False, **kw)
    for rep in range(3):
        print(f"variant {variant} replay round {rep}", flush=True)
        got = _run(code, llr, True, **kw)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (variant, rep)
        # eager work between the decodes that replay the cached graph
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()
    # new buffers: a new capture
    llr2 = llr[:100].clone()
    ref2 = _run(code, llr2, False, **kw)
    got2 = _run(code, llr2, True, **kw)
    for a, b in zip(ref2, got2):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n,storage", [(2640, 1), (16384, 0), (16384, 1)])
def test_graph_replay_fixed_iterations_and_state(n, storage):
    # 37 iterations with stopping off (not a multiple of the 16-launch block): the
    # replays past the limit do nothing; the exported state equals direct launches
    H = W.gallager36(n)
    code = lp.Code(H)
    llr = torch.from_numpy(W.awgn_batch(H, 12, 2.0, tag="graph-k")).cuda()
    kw = dict(tol=0.0, max_iter=37, storage=storage)
    ref = _state(code, llr, False, **kw)
    got = _state(code, llr, True, **kw)
    assert np.all(got[1] == 37)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
