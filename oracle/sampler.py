"""Counter-based batch sampling (oracle).

Sec. 3.2.1 trains on randomly drawn active voxels only; the hyper-parameter
appendix draws 2^16 random samples per epoch.  The paper does not name a
generator.  This project draws batch indices with SplitMix64 (Steele, Lea and
Flood 2014, "Fast splittable pseudorandom number generators"), used as a
counter-based hash so that any (seed, stream, step, j) can be evaluated on its
own:

  out_c(s)  = the c-th output (c >= 1) of SplitMix64 seeded with s
            = mix(s + c * 0x9E3779B97F4A7C15)
  h(seed, stream, step, j) = out_{j+1}(out_{step+1}(out_{stream+1}(seed)))
  idx = floor(h * N / 2^64)            (128-bit multiply-shift)

where mix is SplitMix64's output function.  The HIP library implements the same
published definition independently.  Streams: 0 voxel regressor, 1 level-0
classifier, 2 level-1 classifier; steps count from 0.
"""
import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB

STREAM_REGRESSOR, STREAM_L0, STREAM_L1, STREAM_TILE = 0, 1, 2, 3


def mix_int(z):
    """SplitMix64 output function on a Python int (exact)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def splitmix64_int(seed, count):
    """First `count` outputs of SplitMix64 seeded with `seed` (pure Python)."""
    out, s = [], seed & MASK64
    for _ in range(count):
        s = (s + GOLDEN) & MASK64
        out.append(mix_int(s))
    return out


def hash_int(seed, stream, step, j):
    s1 = mix_int(seed + GOLDEN * (stream + 1))
    s2 = mix_int(s1 + GOLDEN * (step + 1))
    return mix_int(s2 + GOLDEN * (j + 1))


def _mix_np(z):
    z = z.astype(np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def hash_np(seed, stream, step, j):
    """Vectorised h(seed, stream, step, j) over an array j (uint64 wrap-around arithmetic)."""
    with np.errstate(over="ignore"):
        s1 = mix_int(seed + GOLDEN * (stream + 1))
        s2 = mix_int(s1 + GOLDEN * (step + 1))
        jj = np.asarray(j, dtype=np.uint64)
        return _mix_np(np.uint64(s2) + np.uint64(GOLDEN) * (jj + np.uint64(1)))


def mulhi_u64_u32(h, n):
    """floor(h * n / 2^64) for uint64 h and n < 2^32, without 128-bit types."""
    h = np.asarray(h, dtype=np.uint64)
    n = np.uint64(n)
    hi = h >> np.uint64(32)
    lo = h & np.uint64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        t = hi * n + ((lo * n) >> np.uint64(32))
    return (t >> np.uint64(32)).astype(np.int64)


def iid_indices(seed, stream, step, batch, n):
    """Batch of i.i.d. indices in [0, n) for one training step."""
    if not (0 < n < (1 << 32)):
        raise ValueError("population must be in (0, 2^32)")
    return mulhi_u64_u32(hash_np(seed, stream, step, np.arange(batch, dtype=np.uint64)), n)
