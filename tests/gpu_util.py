"""Helpers shared by the GPU parity tests (not a test module)."""
import numpy as np

FIELDS = ("cell", "ox", "oy", "vx", "vy")


def bits(p):
    """int32 views of the five state arrays (exact comparison keys)."""
    out = []
    for f in FIELDS:
        a = np.ascontiguousarray(p[f])
        if a.dtype == np.float64:
            a = a.astype(np.float32)
        out.append(a.view(np.int32) if a.dtype != np.int32 else a)
    return out


def canonical(p):
    """Rows sorted lexicographically by all five fields (a multiset view)."""
    k = bits(p)
    order = np.lexsort(k[::-1])
    return np.stack([x[order] for x in k], axis=1)


def pairing(gpu, ref):
    """Index map pi with gpu[k] == ref[pi[k]] for identical multisets whose
    rows are unique.  Raises if the multisets differ."""
    kg, kr = bits(gpu), bits(ref)
    og = np.lexsort(kg[::-1])
    orr = np.lexsort(kr[::-1])
    A = np.stack([x[og] for x in kg], axis=1)
    B = np.stack([x[orr] for x in kr], axis=1)
    if A.shape != B.shape or not np.array_equal(A, B):
        raise AssertionError("particle multisets differ")
    pi = np.empty(og.size, np.int64)
    pi[og] = orr
    return pi


def gpu_state(pic, s):
    return pic.particles_numpy(s)


def live(p):
    m = p["cell"] >= 0
    return {k: v[m] for k, v in p.items()}
