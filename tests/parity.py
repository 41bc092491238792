"""Frame-by-frame comparison of GPU decodes with the oracle's, for the full-size
parity tests (the acceptance bar: hard decisions identical on at least 99.99 % of
the frames whose oracle solution is not ambiguous, iteration counts within 2 on at
least 99 % of all frames, certificate flags equal on at least 99.9 % of the
non-ambiguous frames)."""
import numpy as np

import oracle


def parity_summary(x, it, fl, ref):
    """Per-frame comparison of GPU decodes with the oracle's (R13: a frame whose oracle x
    has an entry within 1e-3 of 1/2 is ambiguous and its hard decision is not compared)."""
    ambiguous = np.any(np.abs(ref.x - 0.5) < 1e-3, axis=1)
    same = np.all((x >= 0.5) == (ref.x >= 0.5), axis=1)
    dit = np.abs(it.astype(np.int64) - ref.iters)
    flags_same = (fl & 0x0F) == (ref.flags & 0x0F)
    clear = ~ambiguous
    return {
        "frames": int(len(x)), "ambiguous": int(ambiguous.sum()),
        "hard_mismatch": int((~same & clear).sum()),
        "hard_agreement": float(same[clear].mean()) if clear.any() else 1.0,
        "iters_within_2": float((dit <= 2).mean()), "iters_max_diff": int(dit.max()),
        "flags_agreement": float(flags_same[clear].mean()) if clear.any() else 1.0,
    }


def assert_parity(summary, what):
    print(f"{what}: {summary}", flush=True)
    # hard decisions identical on >= 99.99 % of the non-ambiguous frames
    clear = summary["frames"] - summary["ambiguous"]
    assert summary["hard_mismatch"] <= int(1e-4 * clear), (what, summary)
    assert summary["iters_within_2"] >= 0.99, (what, summary)
    assert summary["flags_agreement"] >= 0.999, (what, summary)


def ref_slice(ref, sl):
    return oracle.Result(ref.x[sl], ref.iters[sl], ref.flags[sl])
