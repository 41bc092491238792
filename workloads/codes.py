"""Seeded parity-check matrix construction (input generation only).

Nothing here performs LP decoding: this module only produces sparse
parity-check matrices H (as CSR over checks) for the synthetic workloads, so
that the FP64 oracle and the HIP library are fed identical codes.

* ``gallager_regular`` -- Gallager's construction of a (dv, dc)-regular code:
  dv stacked blocks, the first a band matrix with dc consecutive ones per row,
  the others random column permutations of it.  Column pairs that share two or
  more checks (length-4 cycles) are removed by re-drawing permutation entries.
* ``irregular`` -- a random socket matching for given variable / check degree
  distributions, with parallel edges and length-4 cycles repaired by swapping
  edge endpoints (degrees are preserved).
* ``random_regular`` -- a (dv, dc)-regular socket matching drawn whole and
  rejected while it has a parallel edge; length-4 cycles are kept.  This is how
  the paper describes its ensemble of n = 1002 codes (Sec. 5.1).

Row neighbourhoods are returned sorted, i_1 < i_2 < ... < i_d, which is the
ordering the paper uses for the selection matrices P_j (Sec. 2).
"""
from __future__ import annotations

import dataclasses
import zlib

import numpy as np
import scipy.sparse as sp


def _key(k) -> int:
    if isinstance(k, str):
        return zlib.crc32(k.encode())
    return int(k)


def rng_for(*keys) -> np.random.Generator:
    """A PCG64 generator keyed by a tuple of ints/strings (reproducible)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([_key(k) for k in keys])))


@dataclasses.dataclass(frozen=True)
class ParityCheckMatrix:
    """H as CSR over checks: row j holds col_idx[row_ptr[j]:row_ptr[j+1]] (sorted)."""

    m: int
    n: int
    row_ptr: np.ndarray  # int32 [m+1]
    col_idx: np.ndarray  # int32 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def check_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def var_degrees(self) -> np.ndarray:
        return np.bincount(self.col_idx, minlength=self.n)

    def to_scipy(self) -> sp.csr_matrix:
        data = np.ones(self.nnz, dtype=np.int32)
        return sp.csr_matrix((data, self.col_idx, self.row_ptr), shape=(self.m, self.n))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray().astype(np.uint8)

    def four_cycle_pairs(self) -> np.ndarray:
        """Column pairs (a<b) sharing >= 2 checks, i.e. length-4 cycles."""
        return _shared_pairs(self.to_scipy())


def _from_edges(m: int, n: int, rows: np.ndarray, cols: np.ndarray, name: str) -> ParityCheckMatrix:
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    np.cumsum(counts, out=row_ptr[1:])
    return ParityCheckMatrix(m, n, row_ptr, cols.astype(np.int32), name)


def _shared_pairs(H: sp.csr_matrix) -> np.ndarray:
    Hb = H.astype(np.int32)
    C = (Hb.T @ Hb).tocoo()
    mask = (C.row < C.col) & (C.data >= 2)
    return np.stack([C.row[mask], C.col[mask]], axis=1)


def gallager_regular(n: int, dv: int, dc: int, seed: int = 0, max_rounds: int = 20000) -> ParityCheckMatrix:
    """(dv, dc)-regular Gallager code of length n with no length-4 cycles."""
    if n % dc:
        raise ValueError("n must be a multiple of dc")
    mb = n // dc
    m = mb * dv
    for attempt in range(64):
        rng = rng_for("gallager", n, dv, dc, seed, attempt)
        perms = [np.arange(n)] + [rng.permutation(n) for _ in range(dv - 1)]
        for _ in range(max_rounds):
            # position of column c inside block b's permutation -> row (pos // dc)
            pos = [np.argsort(p) for p in perms]
            rows = np.concatenate([b * mb + pos[b] // dc for b in range(dv)])
            cols = np.tile(np.arange(n), dv)
            H = sp.csr_matrix((np.ones(rows.size, np.int32), (rows, cols)), shape=(m, n))
            bad = _shared_pairs(H)
            if bad.size == 0:
                return _from_edges(m, n, rows, cols, f"gallager({dv},{dc}) n={n} seed={seed}")
            touched = set()
            for a, b in bad[rng.permutation(len(bad))]:
                if a in touched or b in touched:
                    continue
                # blocks in which a and b share a row
                shared = [bb for bb in range(1, dv) if pos[bb][a] // dc == pos[bb][b] // dc]
                if not shared:
                    shared = list(range(1, dv))
                t = shared[rng.integers(len(shared))]
                victim = a if rng.integers(2) else b
                other = int(rng.integers(n))
                pa, po = pos[t][victim], pos[t][other]
                perms[t][pa], perms[t][po] = perms[t][po], perms[t][pa]
                pos[t][victim], pos[t][other] = po, pa
                touched.update((int(a), int(b), other))
    raise RuntimeError("could not build a 4-cycle-free Gallager code")


def irregular(n: int, var_dist: dict, chk_dist: dict, m: int | None = None, seed: int = 0,
              max_rounds: int = 20000) -> ParityCheckMatrix:
    """Random code with exact degree counts, no parallel edges, no length-4 cycles.

    var_dist / chk_dist map degree -> fraction of nodes; the counts must be integral.
    """
    vdeg = _degree_sequence(n, var_dist)
    E = int(vdeg.sum())
    if m is None:
        mean_c = sum(d * f for d, f in chk_dist.items())
        m = int(round(E / mean_c))
    cdeg = _degree_sequence(m, chk_dist)
    if int(cdeg.sum()) != E:
        raise ValueError("degree distributions give different edge counts")
    vs = np.repeat(np.arange(n), vdeg)
    cs0 = np.repeat(np.arange(m), cdeg)
    for attempt in range(64):
        rng = rng_for("irregular", n, m, seed, attempt)
        cs = cs0[rng.permutation(E)]
        for _ in range(max_rounds):
            key = vs.astype(np.int64) * m + cs
            uniq, first, counts = np.unique(key, return_index=True, return_counts=True)
            dup_edges = np.setdiff1d(np.arange(E), first)  # second+ copies of a (v,c) pair
            H = sp.csr_matrix((np.ones(uniq.size, np.int32), (uniq % m, uniq // m)), shape=(m, n))
            bad = _shared_pairs(H)
            if dup_edges.size == 0 and bad.size == 0:
                return _from_edges(m, n, cs.copy(), vs.copy(), f"irregular n={n} m={m} seed={seed}")
            victims = list(dup_edges)
            if bad.size:
                # for a cycle between columns a and b, move one edge of a
                start = np.searchsorted(vs, bad[:, 0])
                stop = np.searchsorted(vs, bad[:, 0], side="right")
                for (a, b), s0, s1 in zip(bad, start, stop):
                    victims.append(int(s0 + rng.integers(s1 - s0)))
            for e in victims:
                f = int(rng.integers(E))
                cs[e], cs[f] = cs[f], cs[e]
    raise RuntimeError("could not build a 4-cycle-free irregular code")


def random_regular(n: int, dv: int, dc: int, seed: int = 0, max_draws: int = 100000) -> ParityCheckMatrix:
    """Random (dv, dc)-regular code: a uniform socket matching, re-drawn whole until
    no variable meets the same check twice.  Length-4 cycles are allowed."""
    if (n * dv) % dc:
        raise ValueError("n * dv must be a multiple of dc")
    m = n * dv // dc
    E = n * dv
    vs = np.repeat(np.arange(n), dv)
    cs0 = np.repeat(np.arange(m), dc)
    rng = rng_for("random_regular", n, dv, dc, seed)
    for _ in range(max_draws):
        cs = cs0[rng.permutation(E)]
        # sockets of one variable are consecutive in vs: a parallel edge is a repeated
        # check among a variable's dv sockets
        per_var = np.sort(cs.reshape(n, dv), axis=1)
        if not np.any(per_var[:, 1:] == per_var[:, :-1]):
            return _from_edges(m, n, cs.copy(), vs.copy(), f"random({dv},{dc}) n={n} seed={seed}")
    raise RuntimeError("no parallel-edge-free draw")


def _degree_sequence(count: int, dist: dict) -> np.ndarray:
    degs = []
    for d in sorted(dist):
        k = dist[d] * count
        if abs(k - round(k)) > 1e-9:
            raise ValueError(f"degree {d}: fraction {dist[d]} of {count} nodes is not integral")
        degs.append(np.full(int(round(k)), d, dtype=np.int64))
    seq = np.concatenate(degs)
    if seq.size != count:
        raise ValueError("degree fractions do not sum to one")
    return seq


def single_check(d: int) -> ParityCheckMatrix:
    """The length-d single parity-check code (one check over all d bits)."""
    return ParityCheckMatrix(1, d, np.array([0, d], np.int32), np.arange(d, dtype=np.int32), f"spc{d}")


def gf2_rank(H: ParityCheckMatrix) -> int:
    """Rank of H over GF(2) (bit-packed Gaussian elimination)."""
    A = np.packbits(H.dense(), axis=1, bitorder="little").view(np.uint8)
    words = (A.shape[1] + 7) // 8
    A = np.pad(A, ((0, 0), (0, words * 8 - A.shape[1]))).view(np.uint64).copy()
    rank = 0
    rows = A.shape[0]
    for col in range(H.n):
        w, bit = divmod(col, 64)
        mask = np.uint64(1) << np.uint64(bit)
        hits = np.nonzero(A[rank:, w] & mask)[0]
        if hits.size == 0:
            continue
        p = rank + hits[0]
        if p != rank:
            A[[rank, p]] = A[[p, rank]]
        others = np.nonzero(A[:, w] & mask)[0]
        others = others[others != rank]
        A[others] ^= A[rank]
        rank += 1
        if rank == rows:
            break
    return rank
