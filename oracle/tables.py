"""Seeded hash and sign tables of the TensorSketch operators (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 2.2 (Definitions of CountSketch and TensorSketch) asks for per-mode hash
maps h_s: [n_s] -> [J] with uniform marginals (3-wise independent) and
Rademacher sign maps v_s (4-wise independent).  Algorithm 1 (Sec. 3) defines
new operators S_k once per outer iteration.  The oracle draws every table entry
independently (stronger than k-wise independence) from SplitMix64
(Steele, Lea, Flood, OOPSLA 2014), written here from its published definition:

    state_{j+1} = state_j + 0x9E3779B97F4A7C15  (mod 2^64)
    out_j       = mix64(state_{j+1})
    mix64(z)    = z ^= z>>30; z *= 0xBF58476D1CE4E5B9;
                  z ^= z>>27; z *= 0x94D049BB133111EB; z ^= z>>31

Table derivation (a reading of the paper, which leaves the hash family open):
    key      = seed XOR ((t + 1) * 2^16 + s)          (sweep t, mode s)
    state_0  = mix64(key)
    h_s[i]   = floor(out_i * J / 2^64)                  i < n_s
    v_s[i]   = +1 if out_{n_s + i} < 2^63 else -1       i < n_s
The hash draws and the sign draws use disjoint outputs so the two tables are
independent of each other.
"""
import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    """SplitMix64 output function on a 64-bit integer."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_stream(state: int, count: int):
    """The first ``count`` outputs of SplitMix64 started from ``state``."""
    out = []
    s = state & MASK64
    for _ in range(count):
        s = (s + GAMMA) & MASK64
        out.append(mix64(s))
    return out


def mode_tables(seed: int, sweep: int, mode: int, n: int, J: int):
    """(h, v) for one mode: h int64 in [0, J), v int8 in {-1, +1}."""
    if J < 1 or n < 0:
        raise ValueError("need J >= 1 and n >= 0")
    key = (seed ^ ((sweep + 1) * 65536 + mode)) & MASK64
    draws = splitmix64_stream(mix64(key), 2 * n)
    h = np.array([(x * J) >> 64 for x in draws[:n]], dtype=np.int64)
    v = np.array([1 if (x >> 63) == 0 else -1 for x in draws[n:]], dtype=np.int8)
    return h, v


def sweep_tables(seed: int, sweep: int, n, J: int):
    """Lists (hs, vs) over all modes for one sweep (Algorithm 1, one while-pass)."""
    hs, vs = [], []
    for s, ns in enumerate(n):
        h, v = mode_tables(seed, sweep, s, int(ns), J)
        hs.append(h)
        vs.append(v)
    return hs, vs
