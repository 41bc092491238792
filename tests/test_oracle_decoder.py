"""Pins for the oracle's ADMM decoder (Algorithm 1 with over-relaxation).

The iteration itself has no closed form; these tests pin it by what the
mathematics fixes: each update solves its sub-problem of the augmented
Lagrangian (eq. augLag), the fixed point is the LP optimum of eq. feldmanLP
(solved here by a generic simplex in two formulations), an integral LP
optimum is the ML codeword (Sec. 1), a single-check code decodes to the
linear-maximisation vertex of Algorithm 3, and the iteration is resumable.
"""
import numpy as np
import pytest

import oracle
import pins
import workloads as W


def small_code(n, m, dv, seed):
    """Random sparse H with column weight dv and every row of degree >= 2."""
    rng = np.random.default_rng([n, m, dv, seed])
    while True:
        H = np.zeros((m, n), np.uint8)
        for i in range(n):
            H[rng.choice(m, dv, replace=False), i] = 1
        if H.sum(1).min() >= 2 and H.sum(1).max() <= 8:
            break
    rows, cols = np.nonzero(H)
    row_ptr = np.zeros(m + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    return W.ParityCheckMatrix(m, n, row_ptr, cols.astype(np.int32), f"small{n}x{m}")


def hamming74():
    Hd = np.array([[1, 1, 1, 0, 1, 0, 0], [1, 1, 0, 1, 0, 1, 0], [1, 0, 1, 1, 0, 0, 1]], np.uint8)
    rows, cols = np.nonzero(Hd)
    return W.ParityCheckMatrix(3, 7, np.array([0, 4, 8, 12], np.int32), cols.astype(np.int32), "hamming74")


def test_x_update_minimises_lagrangian_over_box():
    # One iteration from a random state: the returned x is argmin_x L_mu(x, z, lambda)
    # over [0,1]^N (Sec. 3.2), computed here coordinate-wise by a bounded minimiser.
    H = small_code(16, 8, 3, 0)
    rng = np.random.default_rng(1)
    mu = 3.0
    gamma = rng.normal(1.0, 2.0, (1, H.n)).astype(np.float32)
    z0 = rng.uniform(0, 1, (1, H.nnz))
    u0 = rng.normal(0, 0.5, (1, H.nnz))
    res = oracle.decode(H, gamma, mu=mu, rho=1.0, max_iter=1, tol=0.0, z0=z0, u0=u0)
    for i in range(H.n):
        edges = np.nonzero(H.col_idx == i)[0]
        want = pins.lagrangian_x_argmin(float(gamma[0, i]), z0[0, edges], mu * u0[0, edges], mu)
        assert abs(res.x[0, i] - want) < 1e-7


def test_z_update_minimises_lagrangian_over_parity_polytope():
    # With rho = 1 the new replica z_j minimises mu/2 ||P_j x - z||^2 - lambda_j^T z over
    # PP_d (Sec. 3.2).  Minimise that over the vertex weights with a generic solver.
    from scipy.optimize import minimize
    H = small_code(12, 6, 2, 3)
    rng = np.random.default_rng(2)
    mu = 3.0
    gamma = rng.normal(0.5, 2.0, (1, H.n)).astype(np.float32)
    z0 = rng.uniform(0, 1, (1, H.nnz))
    u0 = rng.normal(0, 0.5, (1, H.nnz))
    res = oracle.decode(H, gamma, mu=mu, rho=1.0, max_iter=1, tol=0.0, z0=z0, u0=u0, state=True)
    x = res.x[0]
    for j in range(H.m):
        e = np.arange(H.row_ptr[j], H.row_ptr[j + 1])
        Px = x[H.col_idx[e]]
        lam = mu * u0[0, e]
        V = pins.even_vertices(e.size)

        def obj(a):
            zz = a @ V
            return 0.5 * mu * np.sum((Px - zz) ** 2) - lam @ zz

        k = V.shape[0]
        sol = minimize(obj, np.full(k, 1.0 / k), method="SLSQP", bounds=[(0, 1)] * k,
                       constraints=[{"type": "eq", "fun": lambda a: a.sum() - 1.0}],
                       options={"ftol": 1e-14, "maxiter": 1000})
        assert np.max(np.abs(sol.x @ V - res.z[0, e])) < 1e-5
        # lambda-update of Algorithm 1: lambda + mu (P_j x - z_j)
        assert np.allclose(mu * res.u[0, e], lam + mu * (Px - res.z[0, e]), atol=1e-12)


@pytest.mark.parametrize("rho", [1.0, 1.9])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fixed_point_is_the_lp_optimum(rho, seed):
    H = small_code(18, 9, 3, seed) if seed else hamming74()
    rng = np.random.default_rng([seed, 7])
    gamma = rng.normal(1.0, 1.5, (3, H.n)).astype(np.float32)
    res = oracle.decode(H, gamma, mu=3.0, rho=rho, max_iter=20000, tol=1e-10)
    for f in range(gamma.shape[0]):
        g = gamma[f].astype(np.float64)
        lp1, _ = pins.feldman_lp(H.row_ptr, H.col_idx, H.n, g)
        lp2, _ = pins.yannakakis_lp(H.row_ptr, H.col_idx, H.n, g)
        assert abs(lp1 - lp2) < 1e-7 * (1 + abs(lp1))
        obj = g @ res.x[f]
        assert abs(obj - lp1) < 1e-6 * (1 + abs(lp1)), (f, obj, lp1, res.iters[f])


def test_bsc_fixed_point_objective_is_the_lp_optimum():
    # BSC costs take two values, so the LP optimum is often not unique (ties);
    # what is unique is its value (Sec. 2, footnote on the BSC).
    H = small_code(18, 9, 3, 8)
    rng = np.random.default_rng(21)
    gamma = W.bsc_llr(H.n, 6, 0.15, rng)
    res = oracle.decode(H, gamma, mu=3.0, rho=1.9, max_iter=20000, tol=1e-10)
    for f in range(gamma.shape[0]):
        g = gamma[f].astype(np.float64)
        lp, _ = pins.feldman_lp(H.row_ptr, H.col_idx, H.n, g)
        assert abs(g @ res.x[f] - lp) < 1e-6 * (1 + abs(lp)), (f, g @ res.x[f], lp)


def test_objective_gap_shrinks_with_iterations():
    # gamma^T xhat - gamma^T x* = O(M d mu / T) (Sec. 3.3): the gap at a fixed T falls
    # as T grows (tolerance 0 disables stopping).
    H = small_code(20, 10, 3, 4)
    rng = np.random.default_rng(9)
    gamma = rng.normal(0.6, 1.5, (1, H.n)).astype(np.float32)
    lp, _ = pins.feldman_lp(H.row_ptr, H.col_idx, H.n, gamma[0].astype(np.float64))
    gaps = []
    for T in (5, 50, 500, 5000):
        res = oracle.decode(H, gamma, mu=3.0, rho=1.0, max_iter=T, tol=0.0)
        gaps.append(abs(gamma[0].astype(np.float64) @ res.x[0] - lp))
    assert gaps[-1] < 1e-6
    assert gaps[-1] <= gaps[0]


def test_single_check_code_decodes_to_alg3_vertex():
    # For m = 1 the LP is max (-gamma)^T z over PP_d: a vertex, given by Algorithm 3,
    # which is also single-parity-check ML decoding.
    rng = np.random.default_rng(3)
    for d in (3, 4, 5, 6, 7, 8):
        H = W.single_check(d)
        gamma = rng.normal(0.8, 1.5, (8, d)).astype(np.float32)
        res = oracle.decode(H, gamma, mu=3.0, rho=1.9, max_iter=20000, tol=1e-9)
        for f in range(8):
            g = gamma[f].astype(np.float64)
            vert = oracle.max_linear(-g)
            ml, _, unique = pins.ml_decode(np.ones((1, d), np.uint8), g)
            assert np.array_equal(vert, ml.astype(float))
            if unique:
                assert np.max(np.abs(res.x[f] - vert)) < 1e-4
                assert res.flags[f] & oracle.FLAG_CERTIFIED


def test_certified_frames_are_ml_codewords():
    # An integral LP solution is the ML codeword (Sec. 1).  Exhaustive ML over all
    # 2^k codewords of a small code.
    H = small_code(20, 10, 3, 5)
    Hd = H.dense()
    rng = np.random.default_rng(4)
    gamma = W.awgn_llr(H.n, 200, 1.0, rng)
    res = oracle.decode(H, gamma, mu=3.0, rho=1.9, max_iter=2000, tol=1e-7)
    n_cert = 0
    for f in range(gamma.shape[0]):
        if res.flags[f] & oracle.FLAG_CERTIFIED:
            ml, _, unique = pins.ml_decode(Hd, gamma[f])
            if unique:
                n_cert += 1
                assert np.array_equal(res.hard[f], ml)
    assert n_cert > 50


def test_warm_start_resume_is_bitwise():
    H = W.gallager36(96)
    llr = W.awgn_batch(H, 8, 2.0, tag="warm")
    a = oracle.decode(H, llr, max_iter=30, tol=0.0, state=True)
    b1 = oracle.decode(H, llr, max_iter=12, tol=0.0, state=True)
    b2 = oracle.decode(H, llr, max_iter=18, tol=0.0, z0=b1.z, u0=b1.u, state=True)
    assert np.array_equal(a.z, b2.z) and np.array_equal(a.u, b2.u) and np.array_equal(a.x, b2.x)


def test_invalid_input_flagged():
    H = W.gallager36(96)
    llr = W.awgn_batch(H, 3, 3.0, tag="nan")
    llr[1, 5] = np.nan
    llr[2, 7] = np.inf
    res = oracle.decode(H, llr, max_iter=50)
    assert res.flags[0] & oracle.FLAG_CONVERGED
    for f in (1, 2):
        assert res.flags[f] == oracle.FLAG_INVALID and res.iters[f] == 0
        assert np.all(res.x[f] == 0.5)


def test_over_relaxation_speeds_up_convergence():
    # Sec. 5.2: rho = 1.9 roughly halves the decoding time relative to rho = 1.
    H = W.gallager36(2640)
    llr = W.awgn_batch(H, 32, 2.8, tag="rho")
    it1 = oracle.decode(H, llr, rho=1.0).iters.mean()
    it19 = oracle.decode(H, llr, rho=1.9).iters.mean()
    assert it19 < 0.75 * it1


def test_small_config_reference_run_against_exact_lp():
    """The (3,6) n=96 workload at 3 dB (T = 200): on a subset of frames, every frame
    certified by the oracle has the LP optimum as objective, and certified frames
    are exactly the frames whose LP optimum is integral and a codeword."""
    H = W.gallager36(96)
    llr = W.awgn_batch(H, 1000, 3.0)
    res = oracle.decode(H, llr, mu=3.0, rho=1.9, max_iter=200, tol=1e-5)
    assert res.iters.max() <= 200
    fer = np.mean(res.hard.sum(1) > 0)
    assert 0.0 < fer < 0.2
    for f in range(0, 1000, 25):
        g = llr[f].astype(np.float64)
        lp, xlp = pins.feldman_lp(H.row_ptr, H.col_idx, H.n, g)
        if res.flags[f] & oracle.FLAG_CONVERGED:
            assert abs(g @ res.x[f] - lp) < 1e-3 * (1 + abs(lp))
        if res.flags[f] & oracle.FLAG_CERTIFIED:
            assert np.array_equal(res.hard[f], (xlp > 0.5).astype(np.uint8))


def mixed_degree_code(seed):
    """n = 24, m = 12 with variable degrees 2, 3 and 6 (6, 12 and 6 columns) and
    every check degree in [2, 8]: nnz = 84, mean check degree 7."""
    rng = np.random.default_rng([24, 12, seed])
    degs = np.array([2] * 6 + [3] * 12 + [6] * 6)
    while True:
        Hd = np.zeros((12, 24), np.uint8)
        for i, d in enumerate(degs):
            Hd[rng.choice(12, d, replace=False), i] = 1
        if Hd.sum(1).min() >= 2 and Hd.sum(1).max() <= 8:
            break
    rows, cols = np.nonzero(Hd)
    row_ptr = np.zeros(13, np.int32)
    np.cumsum(np.bincount(rows, minlength=12), out=row_ptr[1:])
    return W.ParityCheckMatrix(12, 24, row_ptr, cols.astype(np.int32), f"mixed24 seed={seed}")


def test_x_update_with_mixed_variable_degrees():
    # each variable averages over its own |N_v(i)| replicas (Sec. 3.2): the returned x
    # is the coordinate-wise argmin of L_mu over the box for degrees 2, 3 and 6 alike
    H = mixed_degree_code(0)
    assert set(np.bincount(H.col_idx, minlength=H.n)) == {2, 3, 6}
    rng = np.random.default_rng(4)
    mu = 3.0
    gamma = rng.normal(0.8, 2.0, (1, H.n)).astype(np.float32)
    z0 = rng.uniform(0, 1, (1, H.nnz))
    u0 = rng.normal(0, 0.5, (1, H.nnz))
    res = oracle.decode(H, gamma, mu=mu, rho=1.0, max_iter=1, tol=0.0, z0=z0, u0=u0)
    for i in range(H.n):
        edges = np.nonzero(H.col_idx == i)[0]
        want = pins.lagrangian_x_argmin(float(gamma[0, i]), z0[0, edges], mu * u0[0, edges], mu)
        assert abs(res.x[0, i] - want) < 1e-7


@pytest.mark.parametrize("seed", [1, 2])
def test_fixed_point_is_the_lp_optimum_mixed_degrees(seed):
    # checks of degree up to 8 and variables of degree 2, 3 and 6: the over-relaxed
    # iteration still converges to the optimum of the LP relaxation
    H = mixed_degree_code(seed)
    rng = np.random.default_rng([seed, 11])
    gamma = rng.normal(1.0, 1.5, (3, H.n)).astype(np.float32)
    res = oracle.decode(H, gamma, mu=3.0, rho=1.9, max_iter=20000, tol=1e-10)
    for f in range(gamma.shape[0]):
        g = gamma[f].astype(np.float64)
        lp, _ = pins.feldman_lp(H.row_ptr, H.col_idx, H.n, g)
        assert abs(g @ res.x[f] - lp) < 1e-6 * (1 + abs(lp)), (f, g @ res.x[f], lp, res.iters[f])
