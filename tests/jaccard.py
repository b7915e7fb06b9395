"""Closed-form weighted Jaccard similarity, the checker the estimator laws are tested against."""
import numpy as np


def weighted_jaccard(ia, wa, ib, wb) -> float:
    """Closed form J(x,y) = sum min / sum max (eq. 1) for two sparse rows."""
    a = dict(zip(np.asarray(ia).tolist(), np.asarray(wa).tolist()))
    b = dict(zip(np.asarray(ib).tolist(), np.asarray(wb).tolist()))
    keys = set(a) | set(b)
    num = sum(min(a.get(i, 0.0), b.get(i, 0.0)) for i in keys)
    den = sum(max(a.get(i, 0.0), b.get(i, 0.0)) for i in keys)
    return num / den
