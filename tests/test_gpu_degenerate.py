"""GPU: degenerate inputs and codes against the oracle.

* gamma = 0 (a zero-cost LP: the iteration stays at the all-zero point and certifies it);
* saturated channels (|gamma| of 1e4) where every x clips at once;
* LLRs that are exactly zero on some bits (the x-update has no channel pull there);
* single-check codes of every degree 2..8 and of degrees 9, 12, 13 and 16 (the LP
  optimum is Algorithm 3's vertex);
* a code whose checks have degrees 2..8 together (the general-degree kernels), and one
  whose checks have degrees 2..16 (the build for checks above degree 8).
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

lp = None
FORMS = None


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global lp, FORMS
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1204_0556_amd as m
    lp = m
    FORMS = (m.MODE_RESIDENT, m.MODE_PERSISTENT_GLOBAL, m.MODE_STREAMED)
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _check_fixed_k(H, llr, K, modes):
    ref = oracle.decode(H, llr, max_iter=K, tol=0.0, state=True)
    code = lp.Code(H)
    for m in modes:
        x, it, fl, z, u = lp.decode_state(code, dev(llr), mode=m, tol=0.0, max_iter=K)
        assert np.abs(host(x) - ref.x).max() < 1e-4, m
        assert np.abs(host(z) - ref.z).max() < 1e-4, m
        assert np.abs(host(u) - ref.u).max() < 1e-4, m


def test_zero_cost_stays_at_the_all_zero_codeword():
    H = W.gallager36(96)
    llr = np.zeros((4, H.n), np.float32)
    for m in FORMS:
        x, it, fl = lp.decode(lp.Code(H), dev(llr), mode=m)
        x, it, fl = host(x), host(it), host(fl)
        assert np.all(x == 0.0) and np.all(it == 1) and np.all(fl == lp.FLAG_CERTIFIED | 0x07), m
    _check_fixed_k(H, llr, 5, FORMS)


def test_saturated_and_exactly_zero_llrs():
    H = W.gallager36(2640)
    rng = np.random.default_rng(3)
    big = (rng.choice([-1.0, 1.0], size=(4, H.n)) * 1e4).astype(np.float32)
    _check_fixed_k(H, big, 10, FORMS)
    llr = W.awgn_batch(H, 4, 2.0, tag="zeros")
    llr[:, rng.choice(H.n, 300, replace=False)] = 0.0
    _check_fixed_k(H, llr, 30, FORMS)
    x, it, fl = lp.decode(lp.Code(H), dev(llr))
    ref = oracle.decode(H, llr)
    ambiguous = np.any(np.abs(ref.x - 0.5) < 1e-3, axis=1)
    assert np.all(np.all((host(x) >= 0.5) == (ref.x >= 0.5), axis=1) | ambiguous)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7, 8, 9, 12, 13, 16])
def test_single_check_codes(d):
    H = W.single_check(d)
    rng = np.random.default_rng([d, 5])
    llr = rng.normal(0.5, 2.0, (64, d)).astype(np.float32)
    print(f"single check d={d}", flush=True)
    # resident builds: degree 6, and one chunk per wave above degree 8
    modes = FORMS if (d == 6 or d > 8) else (lp.MODE_PERSISTENT_GLOBAL, lp.MODE_STREAMED)
    _check_fixed_k(H, llr, 25, modes)
    x, it, fl = lp.decode(lp.Code(H), dev(llr), max_iter=5000, tol=1e-7)
    ref = oracle.decode(H, llr, max_iter=5000, tol=1e-7)
    assert np.abs(host(x) - ref.x).max() < 1e-3


def test_check_degrees_two_to_eight_in_one_code():
    rng = np.random.default_rng(17)
    m, n = 40, 60
    while True:  # random H with row degrees spread over 2..8 and no empty column
        degs = rng.integers(2, 9, size=m)
        rows = np.repeat(np.arange(m), degs)
        cols = np.concatenate([rng.choice(n, d, replace=False) for d in degs])
        vdeg = np.bincount(cols, minlength=n)
        if vdeg.min() >= 1 and np.unique(vdeg).size <= 8 and set(degs) == set(range(2, 9)):
            break
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(m + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    H = W.ParityCheckMatrix(m, n, row_ptr, cols.astype(np.int32), "degrees 2..8")
    llr = W.awgn_batch(H, 16, 2.0, tag="deg2to8")
    print(f"degrees 2..8 code m={m} n={n} nnz={H.nnz}", flush=True)
    _check_fixed_k(H, llr, 40, (lp.MODE_PERSISTENT_GLOBAL, lp.MODE_STREAMED))


def test_check_degrees_two_to_sixteen_in_one_code():
    rng = np.random.default_rng(23)
    m, n = 45, 120
    while True:  # random H with row degrees spread over 2..16 and no empty column
        degs = rng.integers(2, 17, size=m)
        rows = np.repeat(np.arange(m), degs)
        cols = np.concatenate([rng.choice(n, d, replace=False) for d in degs])
        vdeg = np.bincount(cols, minlength=n)
        if vdeg.min() >= 1 and np.unique(vdeg).size <= 8 and set(degs) == set(range(2, 17)):
            break
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(m + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    H = W.ParityCheckMatrix(m, n, row_ptr, cols.astype(np.int32), "degrees 2..16")
    llr = W.awgn_batch(H, 16, 2.0, tag="deg2to16")
    code = lp.Code(H)
    print(f"degrees 2..16 code m={m} n={n} nnz={H.nnz}: {code.launch_info()}", flush=True)
    assert code.info["resident_capable"]  # one chunk per degree, one wave each
    _check_fixed_k(H, llr, 40, FORMS)
    outs = [tuple(host(t) for t in lp.decode(code, dev(llr), mode=md, max_iter=300)) for md in FORMS]
    for o in outs[1:]:
        assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])
        assert np.abs(o[0] - outs[0][0]).max() == 0.0
