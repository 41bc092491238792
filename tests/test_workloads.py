"""The seeded input generators: code structure and channel statistics."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("n", [96, 2640, 16384])
def test_regular_36_codes(n):
    H = W.gallager36(n)
    assert H.m == n // 2 and H.nnz == 3 * n
    assert np.all(H.var_degrees() == 3) and np.all(H.check_degrees() == 6)
    assert len(H.four_cycle_pairs()) == 0
    for j in range(0, H.m, max(1, H.m // 50)):
        row = H.col_idx[H.row_ptr[j]:H.row_ptr[j + 1]]
        assert np.all(np.diff(row) > 0)


def test_regular_48_code():
    H = W.gallager48(16384)
    assert H.m == 8192 and H.nnz == 65536
    assert np.all(H.var_degrees() == 4) and np.all(H.check_degrees() == 8)
    assert len(H.four_cycle_pairs()) == 0


@pytest.mark.parametrize("n", W.IRREGULAR_LENGTHS)
def test_irregular_codes(n):
    H = W.irregular_half(n)
    assert H.m == n // 2 and H.nnz == 7 * n // 2
    vd = np.bincount(H.var_degrees(), minlength=7)
    assert vd[2] == n // 4 and vd[3] == n // 2 and vd[6] == n // 4
    cd = np.bincount(H.check_degrees(), minlength=9)
    assert cd[6] == cd[7] == cd[8] == H.m // 3
    assert len(H.four_cycle_pairs()) == 0


@pytest.mark.parametrize("n", [1057, 16380])
def test_code313(n):
    # n = 1057: the [1057,813] shape (m = 244 independent checks, 243 of degree 13
    # and one of degree 12); 13 | 16380 gives an exactly (3,13)-regular code
    H = W.code313(n)
    assert np.all(H.var_degrees() == 3) and H.nnz == 3 * n
    cd = np.bincount(H.check_degrees(), minlength=14)
    if n == 1057:
        assert H.m == 244 and cd[13] == 243 and cd[12] == 1
        assert n - W.gf2_rank(H) == 813
    else:
        assert H.m == 3 * n // 13 and cd[13] == H.m
    assert len(H.four_cycle_pairs()) == 0


def test_codes_are_deterministic():
    a, b = W.gallager_regular(96, 3, 6, seed=5), W.gallager_regular(96, 3, 6, seed=5)
    assert np.array_equal(a.col_idx, b.col_idx)


def test_gf2_rank():
    H = W.gallager36(96)
    r = W.gf2_rank(H)
    # Gallager blocks each cover every column once, so the dv row-block sums are
    # equal: rank <= m - (dv - 1).
    assert r <= H.m - 2
    Hd = H.dense().astype(np.int64)
    assert np.linalg.matrix_rank(Hd) >= r  # real rank bounds GF(2) rank


def test_awgn_llr_statistics():
    rng = W.rng_for("stat", 1)
    for snr in (1.5, 3.0):
        s2 = float(W.sigma2_for(snr))
        g = W.awgn_llr(4000, 50, snr, rng).astype(np.float64)
        assert abs(g.mean() - 2 / s2) < 0.02 * (2 / s2)
        assert abs(g.var() - 4 / s2) < 0.03 * (4 / s2)


def test_bsc_llr():
    g = W.bsc_llr(1000, 20, 0.05, W.rng_for("bsc"))
    mag = np.log(0.95 / 0.05)
    assert np.allclose(np.abs(g), mag, rtol=1e-6)
    assert abs(np.mean(g < 0) - 0.05) < 0.01


def test_serving_trace_rates():
    codes = [W.gallager36(96), W.gallager36(2640)]
    tr = W.serving_trace(codes, duration_s=2.0, frames_per_s=5000.0)
    frames = sum(r.frames for r in tr)
    assert 0.8 * 10000 < frames < 1.2 * 10000
    assert all(1 <= r.frames <= 256 for r in tr)
    assert all(np.diff([r.arrival_s for r in tr]) > 0)


def test_bsc_ensemble():
    codes = W.bsc_ensemble()
    assert len(codes) == W.BSC_ENSEMBLE_SIZE == 100
    names = set()
    for H in codes[:10]:
        assert (H.m, H.n, H.nnz) == (501, 1002, 3006)
        assert set(H.check_degrees()) == {6} and set(H.var_degrees()) == {3}
        # no parallel edges: every (check, variable) pair appears once
        pairs = set(zip(np.repeat(np.arange(H.m), 6).tolist(), H.col_idx.tolist()))
        assert len(pairs) == H.nnz
        names.add(H.name)
    assert len(names) == 10
    # length-4 cycles are allowed (the paper removed parallel edges only)
    assert sum(len(H.four_cycle_pairs()) for H in codes[:10]) > 0
    a = W.bsc_batch(codes[0], 3, 0.05)
    b = W.bsc_batch(codes[0], 3, 0.05)
    c = W.bsc_batch(codes[1], 3, 0.05)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert set(np.unique(a).tolist()) <= {np.float32(np.log(0.95 / 0.05)), np.float32(-np.log(0.95 / 0.05))}
