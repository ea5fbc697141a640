"""Row comparison of GPU results against the oracle (shared by GPU tests).

A row whose id list equals the oracle's is exact. A differing row is
explained when the FP64 keys of both lists agree element by element within
the tolerance (near-equal keys ordered differently by FP32 and FP64 sums).
Any other differing row is genuine: typically a near-tie decided differently
early in the search, after which Alg. 1 follows another, equally valid
trajectory. The bar counts exact + explained rows."""

import numpy as np

from oracle import core


def classify(base, q, gi, oi, metric="l2", tol=1e-5):
    """Returns (exact, explained, genuine) boolean masks over rows."""
    exact = (gi == oi).all(1)
    explained = np.zeros_like(exact)
    bad = np.nonzero(~exact)[0]
    if len(bad):
        kg = core.pair_keys(base, q[bad], gi[bad], metric)
        ko = core.pair_keys(base, q[bad], oi[bad], metric)
        same_pad = (np.isfinite(kg) == np.isfinite(ko)).all(1)
        fin = np.isfinite(ko) & np.isfinite(kg)
        rel = np.where(fin, np.abs(kg - ko) / np.maximum(np.abs(ko), 1e-30), 0.0)
        ok = same_pad & (rel <= tol).all(1)
        explained[bad[ok]] = True
    genuine = ~exact & ~explained
    return exact, explained, genuine
