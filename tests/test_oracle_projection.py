"""Pins for the oracle's projection onto the parity polytope (Sec. 4).

Every check here is independent of Algorithm 2: brute force over the even-weight
vertices, the variational-inequality characterisation of a Euclidean projection,
LP membership, closed forms from symmetry, and the lemmas of Sec. 4.3-4.4 as
invariants.
"""
import os

import numpy as np
import pytest

import oracle
import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_inputs(d, count, seed):
    rng = np.random.default_rng([d, seed])
    out = []
    for k in range(count):
        kind = k % 6
        if kind == 0:
            v = rng.uniform(-0.5, 1.5, d)
        elif kind == 1:
            v = rng.normal(0.5, 0.6, d)
        elif kind == 2:  # heavy ties
            v = rng.choice([-0.2, 0.3, 0.3, 0.7, 1.2], size=d)
        elif kind == 3:  # clipped sum close to an even integer
            v = rng.uniform(0, 1, d)
            s = v.sum()
            target = 2 * max(1, round(s / 2))
            if target <= d:
                v = v + (target - s) / d + rng.normal(0, 1e-7, d)
        elif kind == 4:  # wide range, ADMM-like magnitudes
            v = rng.normal(0.0, 2.0, d)
        else:  # near the box
            v = rng.uniform(0, 1, d)
        out.append(v)
    return out


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7, 8, 10, 13, 16])
def test_projection_equals_brute_force_vertex_qp(d):
    for v in _random_inputs(d, 60, seed=1):
        z = oracle.project(v)
        zb = pins.project_brute(v)
        assert np.max(np.abs(z - zb)) < 1e-9, (v, z, zb)


@pytest.mark.parametrize("d", [3, 6, 8, 13])
def test_projection_variational_certificate(d):
    # z = Pi_C(v) iff z in C and <v - z, e - z> <= 0 for every vertex e of C.
    for v in _random_inputs(d, 30, seed=2):
        z = oracle.project(v)
        assert pins.in_parity_polytope(z)
        assert pins.vi_gap(v, z) <= 1e-10


def test_fig1_points():
    path = os.path.join(GOLDEN, "fig1_d5_points.txt")
    rows = [ln for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) >= 10
    for ln in rows:
        a, b = ln.split("|")
        v = np.array(a.split(), float)
        want = np.array(b.split(), float)
        assert np.allclose(oracle.project(v), want, atol=1e-12), ln


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7, 8, 13])
def test_axis_closed_form(d):
    # Pi(c 1) is on the axis by symmetry (Prop. member-permute); the axis meets
    # PP_d in [0, 1] for even d and in [0, (d-1)/d] for odd d.
    cap = 1.0 if d % 2 == 0 else (d - 1) / d
    for c in np.linspace(-1.0, 2.0, 31):
        z = oracle.project(np.full(d, c))
        assert np.allclose(z, np.clip(c, 0.0, cap), atol=1e-12)


@pytest.mark.parametrize("d", [3, 4, 6, 8])
def test_idempotent_on_polytope_points(d):
    rng = np.random.default_rng(d)
    V = pins.even_vertices(d)
    for e in V:
        assert np.allclose(oracle.project(e), e, atol=1e-13)
    for _ in range(50):
        k = rng.integers(1, min(6, len(V)) + 1)
        w = rng.dirichlet(np.ones(k))
        p = w @ V[rng.choice(len(V), k, replace=False)]
        assert np.allclose(oracle.project(p), p, atol=1e-12)
    # Corollary even_containment: a box point with an even integer sum is in PP_d.
    for _ in range(50):
        s = 2 * rng.integers(0, d // 2 + 1)
        p = rng.dirichlet(np.ones(d)) * s
        if np.all(p <= 1):
            assert np.allclose(oracle.project(p), p, atol=1e-12)


def test_equivariance():
    rng = np.random.default_rng(7)
    for d in (5, 6, 8):
        for v in _random_inputs(d, 20, seed=3):
            perm = rng.permutation(d)
            assert np.allclose(oracle.project(v[perm]), oracle.project(v)[perm], atol=1e-12)


@pytest.mark.parametrize("d", [4, 6, 7, 8])
def test_kkt_and_lemmas(d):
    for v in _random_inputs(d, 80, seed=4):
        z, r, beta, branch = oracle.project_info(v)
        order = np.argsort(-v, kind="stable")
        vs, zs = v[order], z[order]
        zhat = np.clip(vs, 0, 1)
        s = zhat.sum()
        # Lemma const_parity: ||Pi(v)||_1 lies between the even floor and even ceiling of ||zhat||_1.
        lo, hi = 2 * np.floor(s / 2), 2 * np.ceil(s / 2)
        assert lo - 1e-12 <= z.sum() <= hi + 1e-12
        assert r == lo
        # Prop. proj-permute: order preserved.
        assert np.all(np.diff(zs) <= 1e-12)
        if branch == oracle.BRANCH_SEARCH:
            f = np.where(np.arange(d) <= r, 1.0, -1.0)
            beta_max = 0.5 * (vs[r] - vs[r + 1]) if r <= d - 2 else vs[r]
            # Lemma optimality: z = Pi_[0,1](v - beta f_r), beta in [0, beta_max], f_r^T z = r.
            assert 0.0 <= beta <= beta_max + 1e-12
            assert np.allclose(zs, np.clip(vs - beta * f, 0, 1), atol=1e-12)
            assert abs(f @ zs - r) < 1e-9
            # Proposition of Sec. 4.4: beta_opt <= v_{r+1} and beta_opt < 1 - v_{r+2}.
            assert beta <= vs[r] + 1e-12
            if r <= d - 2:
                assert beta < 1 - vs[r + 1] + 1e-12
            # PQP feasibility: r <= 1^T z <= r + 2.
            assert r - 1e-9 <= zs.sum() <= r + 2 + 1e-9
        else:
            assert np.allclose(zs, zhat, atol=1e-15)


def test_nonexpansive():
    rng = np.random.default_rng(11)
    for d in (3, 6, 8):
        for _ in range(200):
            v = rng.normal(0.5, 1.0, d)
            w = v + rng.normal(0, rng.choice([1e-3, 0.1, 1.0]), d)
            dz = np.linalg.norm(oracle.project(v) - oracle.project(w))
            assert dz <= np.linalg.norm(v - w) + 1e-12


def test_hand_worked_examples():
    # v sorted, zhat sum 3.2 -> r = 2, f_2^T zhat = 2.4 > 2; on the first gap the
    # active set is {2,3,4,5} (1-based) and eq. find-beta gives beta = 0.1.
    z, r, beta, _ = oracle.project_info([1.5, 0.9, 0.9, 0.3, 0.1, -0.1])
    assert r == 2 and abs(beta - 0.1) < 1e-12
    assert np.allclose(z, [1.0, 0.8, 0.8, 0.4, 0.2, 0.0], atol=1e-12)
    # Empty active set at beta = 0 (zhat binary, odd weight): all six breakpoints
    # sit at beta = 1, after which 6 coordinates move, 3 - 6 (beta - 1) = 2.
    z, r, beta, _ = oracle.project_info([2, 2, 2, -1, -1, -1])
    assert r == 2 and abs(beta - 7 / 6) < 1e-12
    assert np.allclose(z, [5 / 6] * 3 + [1 / 6] * 3, atol=1e-12)
    # Unsorted input: same result permuted.
    z2 = oracle.project([-1, 2, -1, 2, -1, 2])
    assert np.allclose(z2, [1 / 6, 5 / 6] * 3, atol=1e-12)


def test_max_linear_alg3_against_vertex_enumeration():
    rng = np.random.default_rng(5)
    for d in range(2, 9):
        V = pins.even_vertices(d)
        for _ in range(100):
            c = rng.normal(0, 1, d)
            z = oracle.max_linear(c)
            assert any(np.array_equal(z, e) for e in V)
            assert abs(c @ z - np.max(V @ c)) < 1e-12


def test_planted_mistake_is_caught():
    """A projection with a sign error in f_r must fail the brute-force pin (this
    guards the pin itself; the mistake is planted in a copy on the CPU)."""
    v = np.array([1.5, 0.9, 0.9, 0.3, 0.1, -0.1])
    z_bad = np.clip(v - 0.1 * np.array([1, 1, 1, 1, -1, -1]), 0, 1)  # wrong f_r
    assert np.max(np.abs(z_bad - pins.project_brute(v))) > 1e-3
