"""Sketch-size bound of Corollary 3 (Sec. 4).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For q sketched modes and s unknowns per slice (s = R[k] R[k+1]) Lemma 3 /
Theorems 4-5 / Corollary 3 take
    m = max{ 8 s^2 (2 + 3^q) / delta,  8 s (2 + 3^q) / (eps * delta) },
which makes the sketched proximal update a (1 + eps)-approximation of the
subproblem optimum with probability at least 1 - delta.  Lemma 2 (approximate
matrix product) needs m >= (2 + 3^q) / (eps0^2 delta0).
"""
import math


def cor3_sketch_size(s, q, eps, delta):
    return max(8.0 * s * s * (2 + 3 ** q) / delta, 8.0 * s * (2 + 3 ** q) / (eps * delta))


def lemma2_sketch_size(q, eps0, delta0):
    return (2 + 3 ** q) / (eps0 * eps0 * delta0)


def cor3_sketch_size_int(s, q, eps, delta):
    return int(math.ceil(cor3_sketch_size(s, q, eps, delta)))
