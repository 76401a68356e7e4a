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


_M1, _M2 = np.uint64(0xBF58476D1CE4E5B9), np.uint64(0x94D049BB133111EB)


def _mix64(z):
    """splitmix64's finaliser (Steele, Lea and Flood, OOPSLA 2014), wrapping uint64."""
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def multiset_hash(p, chunk=1 << 23):
    """Order-free digest of the rows of the five state arrays: the wrapping
    uint64 sum and the wrapping sum of squares of a 64-bit hash of each row
    (cell code and the float32 bits of ox, oy, vx, vy; every NaN counted as
    one canonical NaN).  Equal multisets give equal digests; a row that
    differs in any bit changes them except with probability ~2^-64."""
    n = int(p["cell"].size)
    s1 = np.uint64(0)
    s2 = np.uint64(0)
    with np.errstate(over="ignore"):
        for a in range(0, n, chunk):
            cols = []
            for f in FIELDS:
                x = np.ascontiguousarray(p[f][a:a + chunk])
                if x.dtype != np.int32:
                    x = np.where(np.isnan(x), np.float32(np.nan), x).astype(np.float32).view(np.int32)
                cols.append(x.view(np.uint32).astype(np.uint64))
            h = _mix64(cols[0] | (cols[1] << np.uint64(32)))
            h = _mix64(h ^ (cols[2] | (cols[3] << np.uint64(32))))
            h = _mix64(h + cols[4] + np.uint64(0x9E3779B97F4A7C15))
            s1 = s1 + h.sum(dtype=np.uint64)
            s2 = s2 + (h * h).sum(dtype=np.uint64)
    return n, int(s1), int(s2)


def unet_params(seed, conv_shapes):
    """Seeded network parameters in the flat layout's order: He-normal
    weights and small random biases per convolution (float32), then the 1 x 1
    head's 16 weights and its bias."""
    r = np.random.default_rng(seed)
    ps = []
    for cin, cout in conv_shapes:
        ps.append((r.standard_normal((cout, 3, 3, cin)) * np.sqrt(2.0 / (9 * cin))).astype(np.float32))
        ps.append((r.standard_normal(cout) * 0.05).astype(np.float32))
    ps.append((r.standard_normal(16) * 0.25).astype(np.float32))
    ps.append(np.array([0.1], np.float32))
    return ps


# forward cases of the device network tests: (parameter seed, input seed,
# shape, periodic along W); the crops of the 1024 x 512 case are 192 x 192
UNET_FORWARD_CASES = [(11, 3, (2, 16, 24, 3), False), (11, 3, (1, 64, 48, 3), False),
                      (15, 8, (2, 16, 24, 3), True), (15, 8, (1, 32, 64, 3), True)]
UNET_STEPS = 8.0

