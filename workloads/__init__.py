"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This package only generates inputs -- parity-check matrices and channel cost
vectors -- and holds none of the decoder's arithmetic.  The paper's own codes
(the Margulis [2640,1320] code, the [1057,813] MacKay code and its ensemble of
100 random n=1002 codes, Sec. 5) are not available here; random codes with the
same length, rate and degrees stand in for them.
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

from .channel import awgn_llr, bsc_llr, sigma2_for
from .codes import (ParityCheckMatrix, gallager_regular, gf2_rank, irregular, random_regular,
                    rng_for, single_check)

__all__ = [
    "ParityCheckMatrix", "gallager_regular", "irregular", "single_check", "gf2_rank", "rng_for",
    "awgn_llr", "bsc_llr", "sigma2_for", "PAPER_PARAMS", "gallager36", "gallager48",
    "irregular_half", "IRREGULAR_LENGTHS", "Batch", "awgn_batch", "mixed_batch",
    "HEADLINE_SNRS", "serving_trace", "SERVING_LENGTHS", "random_regular", "bsc_ensemble",
    "bsc_batch", "BSC_CROSSOVERS", "BSC_ENSEMBLE_SIZE", "code313",
]

# Decoder parameters used for every simulation of Sec. 5.1: eps = 1e-5, mu = 3,
# t_max = 1000, rho = 1.9.
PAPER_PARAMS = dict(mu=3.0, rho=1.9, max_iter=1000, tol=1e-5)

HEADLINE_SNRS = (1.5, 2.0, 2.5, 3.0)
# BSC crossover probabilities for the random-code ensemble (the paper plots its
# BSC results against crossover without printing the grid; this one spans the
# LP decoder's waterfall for (3,6) codes of length 1002).
BSC_CROSSOVERS = (0.03, 0.04, 0.05, 0.06, 0.07)
BSC_ENSEMBLE_SIZE = 100
IRREGULAR_LENGTHS = (576, 1152, 2304, 4608, 6912, 8064)
SERVING_LENGTHS = (96, 576, 2640, 8064, 16384)


@functools.lru_cache(maxsize=None)
def gallager36(n: int) -> ParityCheckMatrix:
    """(3,6)-regular code of length n (fixed seed per n): Gallager's construction when
    6 divides n, otherwise a random regular socket matching (e.g. n = 16384)."""
    if n % 6 == 0:
        return gallager_regular(n, 3, 6, seed=n)
    return irregular(n, {3: 1.0}, {6: 1.0}, m=n // 2, seed=n)


@functools.lru_cache(maxsize=None)
def gallager48(n: int) -> ParityCheckMatrix:
    """(4,8)-regular Gallager code of length n (fixed seed per n)."""
    return gallager_regular(n, 4, 8, seed=n)


@functools.lru_cache(maxsize=None)
def code313(n: int = 1057) -> ParityCheckMatrix:
    """Variable degree 3, check degree 13: the stand-in for the paper's [1057,813] code
    (n = 1057: 3 n = 3171 edges over m = 244 checks, so 243 checks of degree 13 and one
    of degree 12; H then has full rank, dimension 813).  For 13 | n every check has
    degree 13 (m = 3 n / 13)."""
    m = -(-3 * n // 13)
    short = 13 * m - 3 * n  # checks of degree 12
    chk = {13: (m - short) / m} if short == 0 else {12: short / m, 13: (m - short) / m}
    return irregular(n, {3: 1.0}, chk, m=m, seed=n)


@functools.lru_cache(maxsize=None)
def irregular_half(n: int) -> ParityCheckMatrix:
    """Rate-1/2 irregular code: variable degrees {2:1/4, 3:1/2, 6:1/4}, check degrees
    {6,7,8} one third each, m = n/2, nnz = 3.5 n."""
    return irregular(n, {2: 0.25, 3: 0.5, 6: 0.25}, {6: 1 / 3, 7: 1 / 3, 8: 1 / 3}, m=n // 2, seed=n)


@functools.lru_cache(maxsize=None)
def bsc_ensemble(n: int = 1002, count: int = BSC_ENSEMBLE_SIZE) -> tuple:
    """`count` random (3,6)-regular codes of length n without parallel edges (length-4
    cycles allowed), seeds 0..count-1: the stand-in for the paper's ensemble of 100
    random n = 1002 codes."""
    return tuple(random_regular(n, 3, 6, seed=s) for s in range(count))


@dataclasses.dataclass
class Batch:
    """Frames to decode.  llr[f] is frame f's FP32 gamma (length n of its code)."""

    codes: list            # list[ParityCheckMatrix]
    code_of_frame: np.ndarray  # int32 [frames]
    llr: list              # list of float32 arrays, one per frame (lengths differ across codes)
    ebn0_db: np.ndarray    # float64 [frames]

    @property
    def frames(self) -> int:
        return int(self.code_of_frame.size)

    def flat_llr(self):
        """(concatenated float32 llr, int64 offsets of each frame)."""
        lens = np.array([a.size for a in self.llr], dtype=np.int64)
        off = np.zeros(lens.size, dtype=np.int64)
        np.cumsum(lens[:-1], out=off[1:])
        return np.concatenate(self.llr).astype(np.float32), off


def awgn_batch(H: ParityCheckMatrix, frames: int, ebn0_db: float, tag: str = "awgn", block: int = 0,
               rate: float = 0.5) -> np.ndarray:
    """[frames, n] float32 gamma for one code at one Eb/N0 (seeded by code length, SNR and block);
    `rate` is the code rate the noise level is computed for (1/2 for the rate-1/2 codes)."""
    rng = rng_for(tag, H.n, H.m, int(round(ebn0_db * 1000)), block)
    return awgn_llr(H.n, frames, ebn0_db, rng, rate=rate)


def bsc_batch(H: ParityCheckMatrix, frames: int, p: float, tag: str = "bsc", block: int = 0) -> np.ndarray:
    """[frames, n] float32 gamma = +-log((1-p)/p) for the all-zero codeword over a BSC(p),
    seeded by the code (length, name), the crossover and a block index."""
    rng = rng_for(tag, H.n, H.m, H.name, int(round(p * 1e6)), block)
    return bsc_llr(H.n, frames, p, rng)


def mixed_batch(codes, frames: int, snr_lo: float, snr_hi: float, tag: str = "mixed", seed: int = 0) -> Batch:
    """Frames drawn uniformly over `codes`, each with Eb/N0 ~ U[snr_lo, snr_hi]."""
    rng = rng_for(tag, frames, len(codes), seed)
    which = rng.integers(len(codes), size=frames).astype(np.int32)
    snr = rng.uniform(snr_lo, snr_hi, size=frames)
    llr = []
    for f in range(frames):
        H = codes[which[f]]
        llr.append(awgn_llr(H.n, 1, snr[f], rng)[0])
    return Batch(list(codes), which, llr, snr)


@dataclasses.dataclass
class Request:
    arrival_s: float
    code: int          # index into the serving code list
    frames: int
    ebn0_db: float
    llr: np.ndarray    # float32 [frames, n]


def serving_trace(codes, duration_s: float, frames_per_s: float = 50_000.0, max_frames: int = 256,
                  snr_lo: float = 1.5, snr_hi: float = 3.5, seed: int = 0) -> list:
    """Poisson arrivals of decode requests: each request carries 1..max_frames frames
    (uniform) of one code (uniform over `codes`) at one Eb/N0 ~ U[snr_lo, snr_hi]."""
    rng = rng_for("serving", len(codes), seed)
    mean_frames = (1 + max_frames) / 2.0
    rate = frames_per_s / mean_frames  # requests per second
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        c = int(rng.integers(len(codes)))
        k = int(rng.integers(1, max_frames + 1))
        snr = float(rng.uniform(snr_lo, snr_hi))
        out.append(Request(t, c, k, snr, awgn_llr(codes[c].n, k, snr, rng)))
    return out
