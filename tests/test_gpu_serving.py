"""GPU serving: continuous batching over a mix of resident codes.

Each request's result must be the same alone and in the mix.  The stated
tolerance is 1e-4 on x (FP32 messages); the design gives bitwise identity,
because a frame's arithmetic depends only on its code's layout plan, and that
is what is checked."""
import numpy as np
import pytest

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


def _codes():
    Hs = [W.gallager36(96), W.irregular_half(576), W.gallager36(2640), W.irregular_half(8064),
          W.gallager36(16384)]
    return Hs, [lp.Code(H) for H in Hs]


def _alone(code, llr):
    x, it, fl = lp.decode(code, torch.from_numpy(llr).cuda())
    torch.cuda.synchronize()
    return x.cpu().numpy(), it.cpu().numpy(), fl.cpu().numpy()


def test_results_same_alone_and_in_the_mix():
    Hs, codes = _codes()
    trace = W.serving_trace(Hs, duration_s=0.02, frames_per_s=50_000.0, max_frames=64, seed=3)
    print(f"serving mix: {len(trace)} requests, {sum(r.frames for r in trace)} frames", flush=True)
    srv = lp.Server(codes, budget_bytes=64 << 20, max_batch_frames=512, max_inflight=4)
    tickets = [srv.submit(r.code, r.llr) for r in trace]
    mixed = [srv.wait(t, timeout=60.0) for t in tickets]
    st = srv.stats()
    srv.close()
    print(f"stats: {st}", flush=True)
    assert st["completed"] == len(trace) and st["peak_device_bytes"] <= 64 << 20
    assert st["workspace_bytes"] > 0 and st["peak_device_bytes"] == st["workspace_bytes"] + st["peak_bytes"]
    # requests submitted together ran in launches that overlapped on the device
    assert st["peak_concurrent_launches"] > 1
    # each request alone, in a fresh server, and through the plain batch API
    for k in range(0, len(trace), max(1, len(trace) // 6)):
        r = trace[k]
        solo = lp.Server(codes, budget_bytes=64 << 20)
        xs, its, fls, _ = solo.wait(solo.submit(r.code, r.llr), timeout=60.0)
        solo.close()
        xm, itm, flm, _ = mixed[k]
        assert np.array_equal(xs, xm) and np.array_equal(its, itm) and np.array_equal(fls, flm)
        xa, ita, fla = _alone(codes[r.code], r.llr)
        assert np.abs(xa - xm).max() <= 1e-4
        assert np.array_equal(ita, itm) and np.array_equal(fla, flm)


def test_small_budget_queues_without_exceeding_it():
    Hs, codes = _codes()
    H = Hs[2]
    # resident codes only: the launch slots' scratch is a few KB; the LLR arena then
    # holds about forty n=2640 frames, so twelve requests of sixteen frames queue
    budget = 4 * H.n * 40 + (16 << 10)
    srv = lp.Server([codes[0], codes[2]], budget_bytes=budget, max_batch_frames=64, max_inflight=2)
    llr = W.awgn_batch(H, 16, 2.5, tag="budget")
    tickets = [srv.submit(1, llr) for _ in range(12)]
    outs = [srv.wait(t, timeout=60.0) for t in tickets]
    st = srv.stats()
    srv.close()
    print(f"stats: {st}", flush=True)
    assert st["completed"] == 12 and 0 < st["peak_bytes"] <= budget - st["workspace_bytes"]
    assert st["peak_device_bytes"] <= budget
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0])


def test_large_code_requests_stay_within_the_device_budget():
    """n = 16384 requests (persistent-global form: each workgroup holds about 0.5 MB of
    state) through a 96 MB budget: the server's device allocations, measured from the
    device's free memory, stay within the budget, the dispatcher allocates nothing
    while serving, and the results equal a plain decode of the same frames."""
    H = W.gallager36(16384)
    code = lp.Code(H)
    llr = W.awgn_batch(H, 64, 2.5, tag="budget-large")
    ref = _alone(code, llr)  # also loads the kernels before memory is measured
    budget = 96 << 20
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    srv = lp.Server([code], budget_bytes=budget, max_batch_frames=256, max_inflight=4)
    free1 = torch.cuda.mem_get_info()[0]
    tickets = [srv.submit(0, llr[8 * k:8 * (k + 1)]) for k in range(8)]
    outs = [srv.wait(t, timeout=120.0) for t in tickets]
    free2 = torch.cuda.mem_get_info()[0]
    st = srv.stats()
    srv.close()
    print(f"server device bytes {free0 - free1}, during serving {free1 - free2}; stats {st}", flush=True)
    assert free0 - free1 <= budget + (8 << 20)  # allocation granularity
    assert abs(free1 - free2) <= (2 << 20)
    assert st["peak_device_bytes"] <= budget and st["workspace_bytes"] > 0
    x = np.concatenate([o[0] for o in outs])
    it = np.concatenate([o[1] for o in outs])
    fl = np.concatenate([o[2] for o in outs])
    assert np.array_equal(x, ref[0]) and np.array_equal(it, ref[1]) and np.array_equal(fl, ref[2])
