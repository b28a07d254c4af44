"""Error measures used by the GPU parity tests."""
import numpy as np

# parent vectors for fields that can start at zero
PARENT = {1: (1, 4), 2: (1, 4), 3: (1, 4), 5: (5, 8), 6: (5, 8), 7: (5, 8), 8: (5, 9)}


def rel_l1(a: np.ndarray, b: np.ndarray, parent_fields=()):
    """Per-field sum|a-b| / sum|b| over interior cells; a field whose reference sum is
    below 1e-12 of its parent vector's, or listed in parent_fields (fields that
    started from exactly zero, measured shortly after), is normalised by the parent
    vector instead."""
    out = []
    for q in range(a.shape[0]):
        num = np.abs(a[q] - b[q]).sum()
        den = np.abs(b[q]).sum()
        if q in PARENT:
            lo, hi = PARENT[q]
            pden = np.sqrt((b[lo:hi] ** 2).sum(axis=0)).sum()
            if den < 1e-12 * pden or den == 0.0 or q in parent_fields:
                den = pden
        out.append(num / den if den > 0 else num)
    return np.array(out)


def linf(a, b):
    return np.abs(a - b).max(axis=1)
