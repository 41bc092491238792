"""GPU parity away from the default parameters (the sweeps of Sec. 5.2): penalty
mu, over-relaxation rho and stopping tolerance eps, against the FP64 oracle.

Tolerances as in the default-parameter parity tests: messages after K
iterations within 1e-4; end to end, hard decisions identical on non-ambiguous
frames and iteration counts within 2 (FP32 residuals may cross eps^2 E one
iteration apart from FP64 ones)."""
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


@pytest.mark.parametrize("mu,rho", [(1.0, 1.0), (7.0, 1.5), (0.5, 1.9), (10.0, 1.0)])
def test_messages_at_other_parameters(mu, rho):
    for n, frames, K in ((96, 32, 60), (2640, 6, 30)):
        H = W.gallager36(n)
        llr = W.awgn_batch(H, frames, 2.2, tag="params")
        print(f"params mu={mu} rho={rho} n={n} K={K}", flush=True)
        x, it, fl, z, u = lp.decode_state(lp.Code(H), dev(llr), mu=mu, rho=rho, tol=0.0, max_iter=K)
        ref = oracle.decode(H, llr, mu=mu, rho=rho, tol=0.0, max_iter=K, state=True)
        assert np.abs(host(x) - ref.x).max() <= 1e-4
        assert np.abs(host(z) - ref.z).max() <= 1e-4
        assert np.abs(host(u) - ref.u).max() <= 1e-4


@pytest.mark.parametrize("tol", [2.0 ** -7, 2.0 ** -13])
def test_end_to_end_at_other_tolerances(tol):
    H = W.gallager36(2640)
    llr = W.awgn_batch(H, 24, 2.2, tag="params-eps")
    kw = dict(mu=5.0, rho=1.0, tol=tol, max_iter=1000)
    x, it, fl = lp.decode(lp.Code(H), dev(llr), **kw)
    x, it = host(x), host(it)
    ref = oracle.decode(H, llr, **kw)
    for f in range(llr.shape[0]):
        if np.any(np.abs(ref.x[f] - 0.5) < 1e-3):
            continue
        assert np.array_equal(x[f] >= 0.5, ref.x[f] >= 0.5), f
        assert abs(int(it[f]) - int(ref.iters[f])) <= 2, (f, it[f], ref.iters[f])
