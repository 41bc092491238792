"""Seeded channel outputs -> cost vectors gamma (input generation only).

The all-zero codeword is sent with BPSK (bit 0 -> +1).  For the binary-input
AWGN channel the negative log-likelihood ratio of Sec. 2,
gamma_i = log W(y_i|0) / W(y_i|1), is 2 y_i / sigma^2.  For the BSC with
crossover p it is +log((1-p)/p) for a received 0 and -log((1-p)/p) for a
received 1 (the footnote to Sec. 2).

Values are drawn in FP64 and rounded once to FP32; that FP32 array is what the
HIP library decodes and what the oracle promotes back to FP64.
"""
from __future__ import annotations

import numpy as np


def sigma2_for(ebn0_db, rate: float = 0.5):
    """Noise variance for Eb/N0 (dB) at code rate `rate` with unit-energy BPSK."""
    return 1.0 / (2.0 * rate * 10.0 ** (np.asarray(ebn0_db, dtype=np.float64) / 10.0))


def awgn_llr(n: int, frames: int, ebn0_db, rng: np.random.Generator, rate: float = 0.5) -> np.ndarray:
    """[frames, n] float32 gamma for the all-zero codeword over BPSK/AWGN.

    ebn0_db may be a scalar or one value per frame.
    """
    s2 = np.broadcast_to(sigma2_for(ebn0_db, rate), (frames,)).reshape(frames, 1)
    y = 1.0 + np.sqrt(s2) * rng.standard_normal((frames, n))
    return (2.0 * y / s2).astype(np.float32)


def bsc_llr(n: int, frames: int, p: float, rng: np.random.Generator) -> np.ndarray:
    """[frames, n] float32 gamma for the all-zero codeword over a BSC(p)."""
    flips = rng.random((frames, n)) < p
    mag = np.log((1.0 - p) / p)
    return np.where(flips, -mag, mag).astype(np.float32)
