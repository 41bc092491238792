"""Pins for the oracle's dual subgradient ascent (Appendix A) and its ML
lower-bound bookkeeping (Sec. 5.1).

The dual iteration is pinned by a trace worked by hand from the appendix's
updates, by weak duality (a converged frame is primal feasible, hence an LP
optimum -- checked against a generic simplex of the LP decoding problem -- and,
being integral, the ML codeword -- checked by enumeration), and by the scale
invariance of the Heaviside and Algorithm 3 decisions.  The bookkeeping is
pinned by hand-worked Hamming-code frames and by exhaustive ML decoding.
"""
import os

import numpy as np
import pytest

import oracle
import pins
import workloads as W
from test_oracle_decoder import hamming74, small_code

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_worked_trace():
    H = W.single_check(3)
    gamma = np.array([[-1.0, 2.0, 2.0]], np.float32)
    rows = [l for l in open(os.path.join(GOLDEN, "dual_spc3_trace.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 7
    for line in rows:
        k, x, conv = [p.strip() for p in line.split("|")]
        r = oracle.dual_decode(H, gamma, mu=1.0, max_iter=int(k))
        assert np.array_equal(r.x[0], np.array(x.split(), float)), line
        assert bool(r.flags[0] & oracle.FLAG_CONVERGED) == (conv == "1"), line
        if conv == "1":
            assert r.iters[0] == 6 and r.flags[0] & oracle.FLAG_CERTIFIED


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_converged_frames_are_lp_optimal_ml_codewords(seed):
    H = small_code(16, 8, 3, 30 + seed) if seed else hamming74()
    Hd = H.dense()
    rng = np.random.default_rng([seed, 11])
    gamma = rng.normal(1.5, 1.0, (40, H.n)).astype(np.float32)
    r = oracle.dual_decode(H, gamma, mu=0.1, max_iter=4000)
    n_conv = 0
    for f in range(gamma.shape[0]):
        if not r.flags[f] & oracle.FLAG_CONVERGED:
            continue
        n_conv += r.iters[f] > 1  # frames that needed the multipliers, not just the hard decision
        g = gamma[f].astype(np.float64)
        assert r.flags[f] & oracle.FLAG_CERTIFIED
        lp, _ = pins.feldman_lp(H.row_ptr, H.col_idx, H.n, g)
        assert abs(g @ r.x[f] - lp) < 1e-7 * (1 + abs(lp))
        ml, cost, unique = pins.ml_decode(Hd, g)
        assert abs(cost - g @ r.x[f]) < 1e-7 * (1 + abs(cost))
        if unique:
            assert np.array_equal(r.x[f].astype(np.uint8), ml)
    assert n_conv >= 10


def test_step_scale_invariance():
    # theta(-gamma - mu S) and Algorithm 3 on mu K only see signs and order, so
    # (gamma, mu) and (2 gamma, 2 mu) run the same iteration.
    H = W.gallager36(96)
    gamma = W.awgn_batch(H, 6, 2.0, tag="dual")
    a = oracle.dual_decode(H, gamma, mu=0.75, max_iter=300)
    b = oracle.dual_decode(H, 2 * gamma, mu=1.5, max_iter=300)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.iters, b.iters) and np.array_equal(a.flags, b.flags)


def test_invalid_frame():
    H = W.gallager36(96)
    g = W.awgn_batch(H, 2, 2.0, tag="dual")
    g[1, 5] = np.inf
    r = oracle.dual_decode(H, g, mu=1.0, max_iter=20)
    assert r.flags[1] == oracle.FLAG_INVALID and r.iters[1] == 0 and np.all(r.x[1] == 0.5)
    assert r.flags[0] != oracle.FLAG_INVALID


def test_evaluate_hand_worked_hamming_frames():
    H = hamming74()
    # 0100110 is a codeword of this H (c5 = c1+c2+c3, c6 = c1+c2+c4, c7 = c1+c3+c4)
    cw = np.array([0, 1, 0, 0, 1, 1, 0], float)
    g_win = np.array([1, 1, 1, 1, -0.5, -0.75, 1], np.float32)  # cost 1 - 0.5 - 0.75 = -0.25 < 0
    g_lose = np.array([1, 1, 1, 1, -0.5, -0.25, 1], np.float32)  # cost +0.25
    g_tie = np.array([1, 1, 1, 1, -0.5, -0.5, 1], np.float32)  # cost 0: a tie is an ML success
    llr = np.stack([g_win, g_lose, g_tie, g_win, g_win])
    x = np.stack([cw, cw, cw, np.zeros(7), np.eye(7)[2] * 0.7])
    r = oracle.evaluate(H, llr, x)
    assert list(r["bit_errors"]) == [3, 3, 3, 0, 1]
    assert np.allclose(r["cost_hat"], [-0.25, 0.25, 0.0, 0.0, 1.0])
    assert np.all(r["cost_sent"] == 0.0)
    E, C, M = oracle.EVAL_WORD_ERROR, oracle.EVAL_CODEWORD, oracle.EVAL_ML_ERROR
    assert list(r["outcome"]) == [E | C | M, E | C, E | C, C, E]
    # the same frames against a non-zero transmitted codeword
    r2 = oracle.evaluate(H, llr[:1], cw[None, :], sent=cw[None, :].astype(np.uint8))
    assert r2["bit_errors"][0] == 0 and r2["outcome"][0] == C
    assert r2["cost_sent"][0] == pytest.approx(-0.25)


def test_ml_lower_bound_never_exceeds_ml_errors():
    # Every frame the estimator counts is one an exhaustive ML decoder also gets
    # wrong, so the estimated ML error rate is a lower bound.
    H = small_code(20, 10, 3, 5)
    Hd = H.dense()
    rng = np.random.default_rng(12)
    gamma = W.bsc_llr(H.n, 300, 0.12, rng)
    res = oracle.decode(H, gamma, mu=3.0, rho=1.9, max_iter=500, tol=1e-6)
    ev = oracle.evaluate(H, gamma, res.x)
    ml_err = 0
    witnessed = 0
    for f in range(gamma.shape[0]):
        ml, cost, unique = pins.ml_decode(Hd, gamma[f])
        wrong = cost < -1e-12  # some codeword beats the all-zero one
        ml_err += wrong
        if ev["outcome"][f] & oracle.EVAL_ML_ERROR:
            witnessed += 1
            assert wrong
    assert witnessed <= ml_err
    assert witnessed > 0 and ml_err > 0
