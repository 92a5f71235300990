"""Pins of the oracle's TensorSketch (data sketch and interface sketch), CPU only.

Each check ties the oracle to something outside itself: the worked example the
paper prints (Sec. 2.2), brute-force index definitions (Sec. 1.2, 2.1), the
FFT identities of Lemma 1 / Corollary 1 / Theorems 1-2 (Sec. 3) evaluated with
numpy.fft, exact integer arithmetic, and the approximate-matrix-product
statements of Lemma 2 (Sec. 4) over many seeds.
"""
import itertools
import json
import os

import numpy as np
import pytest

import synth
from oracle import sketch, tables
from tests.conftest import GOLDEN


def _tabs(n, J, seed=3, t=0):
    return tables.sweep_tables(seed, t, n, J)


def test_paper_worked_example():
    ex = json.load(open(os.path.join(GOLDEN, "paper_example_tensorsketch.json")))
    hs = [np.array(h) - 1 for h in ex["h_one_based"]]
    vs = [np.array(v) for v in ex["v"]]
    S = sketch.tensorsketch_matrix(hs, vs, ex["m"])
    assert np.array_equal(S, np.array(ex["S"], dtype=float))
    # Omega and the combined sign separately
    assert np.array_equal(np.abs(S), np.array(ex["Omega"], dtype=float))
    assert np.array_equal(S.sum(axis=0), np.array(ex["v_combined"], dtype=float))


def _brute_unfold(T, n, k):
    d = len(n)
    others = [s for s in range(d) if s != k]
    ncol = int(np.prod([n[s] for s in others]))
    out = np.zeros((n[k], ncol))
    for idx in itertools.product(*[range(x) for x in n]):
        j, stride = 0, 1
        for s in others:                  # j = sum_{s != k} i_s prod_{t<s, t!=k} n_t
            j += idx[s] * stride
            stride *= n[s]
        out[idx[k], j] = T[idx]
    return out


@pytest.mark.parametrize("n", [(3, 4, 2), (2, 3, 2, 3), (5, 2)])
def test_unfold_matches_definition(n):
    X = synth.rng(1).standard_normal(int(np.prod(n)))
    T = X.reshape(n, order="F")
    for k in range(len(n)):
        assert np.array_equal(sketch.unfold(X, list(n), k), _brute_unfold(T, n, k))


def test_linear_index_is_first_mode_fastest():
    n = (3, 4, 2)
    X = np.arange(24.0)
    T = X.reshape(n, order="F")
    for i0, i1, i2 in itertools.product(range(3), range(4), range(2)):
        assert T[i0, i1, i2] == i0 + 3 * i1 + 12 * i2


@pytest.mark.parametrize("n,J", [((3, 4, 2), 5), ((2, 3, 2, 3), 7), ((5, 2), 4), ((4, 3, 5), 1), ((6,), 3)])
def test_data_sketch_equals_explicit(n, J):
    n = list(n)
    X = synth.rng(2).standard_normal(int(np.prod(n)))
    hs, vs = _tabs(n, J)
    for k in range(len(n)):
        Y = sketch.data_sketch(X, n, k, hs, vs, J)
        Ye = sketch.data_sketch_explicit(X, n, k, hs, vs, J)
        assert Y.shape == (J, n[k])
        np.testing.assert_allclose(Y, Ye, rtol=1e-13, atol=1e-13)


def test_data_sketch_integer_inputs_exact_and_slabbed():
    n, J = [5, 4, 3, 6], 11
    X = synth.rng(4).integers(-8, 9, size=int(np.prod(n))).astype(float)
    hs, vs = _tabs(n, J, seed=9)
    for k in range(4):
        Ye = sketch.data_sketch_explicit(X, n, k, hs, vs, J)
        for slab in (1 << 24, 7, 1):       # slab boundaries must not matter
            assert np.array_equal(sketch.data_sketch(X, n, k, hs, vs, J, slab_entries=slab), Ye)


def test_data_sketch_one_hot():
    n, J = [4, 3, 5], 6
    hs, vs = _tabs(n, J, seed=5)
    for p in (0, 7, 59):
        X = np.zeros(60)
        X[p] = 1.0
        i = np.unravel_index(p, n, order="F")
        for k in range(3):
            Y = sketch.data_sketch(X, n, k, hs, vs, J)
            b = sum(int(hs[s][i[s]]) for s in range(3) if s != k) % J
            sg = np.prod([int(vs[s][i[s]]) for s in range(3) if s != k])
            expect = np.zeros((J, n[k]))
            expect[b, i[k]] = sg
            assert np.array_equal(Y, expect)


def test_lemma1_fourier_form_of_tensorsketch():
    # S = F^{-1} [ (F S_2) face-split (F S_1) ]   (Lemma 1, Sec. 3)
    n, J = [3, 4], 6
    hs, vs = _tabs(n, J, seed=8)
    S = sketch.tensorsketch_matrix(hs, vs, J)
    S1 = sketch.tensorsketch_matrix([hs[0]], [vs[0]], J)
    S2 = sketch.tensorsketch_matrix([hs[1]], [vs[1]], J)
    F = np.exp(-2j * np.pi * np.outer(np.arange(J), np.arange(J)) / J)
    A, B = F @ S2, F @ S1
    face = np.einsum("si,sj->sij", A, B).reshape(J, -1)      # row-wise kron
    S_f = np.linalg.solve(F, face)
    np.testing.assert_allclose(S_f.real, S, atol=1e-12)
    np.testing.assert_allclose(S_f.imag, 0, atol=1e-12)


def test_corollary1_rank_one_closed_form():
    # X = a_0 o a_1 o a_2 o a_3  =>  Y_k[:, i] = a_k[i] * IFFT( prod_{s!=k} FFT(S_s a_s) )
    n, J = [4, 5, 3, 6], 16
    g = synth.rng(6)
    a = [g.standard_normal(x) for x in n]
    X = a[0]
    for v in a[1:]:
        X = np.kron(v, X)
    hs, vs = _tabs(n, J, seed=10)
    for k in range(4):
        prod = np.ones(J, dtype=complex)
        for s in range(4):
            if s != k:
                cs = np.zeros(J)
                np.add.at(cs, hs[s], vs[s] * a[s])
                prod *= np.fft.fft(cs)
        base = np.fft.ifft(prod).real
        np.testing.assert_allclose(sketch.data_sketch(X, n, k, hs, vs, J), np.outer(base, a[k]),
                                   rtol=1e-11, atol=1e-11)


def _brute_tt_entry(cores, idx):
    v = np.ones((1, 1))
    for G, i in zip(cores, idx):
        v = v @ G[:, i, :]
    return v[0, 0]


def test_tt_products_and_interface_matrix():
    # [[G]] entry by entry (Sec. 2.1) vs left/right products, and
    # A_(k)^T = H_k G_k(2)^T with H_k = G_{>k}^T (x) G_{<k} (Sec. 3, definition of H_k under (lrtt_sub4))
    from oracle import solve
    n, R = [3, 4, 2, 3], [1, 2, 3, 2, 1]
    cores = synth.random_cores(n, R, 12)
    # product over reversed ranges varies the last tuple slot (= i_0) fastest
    X = np.array([_brute_tt_entry(cores, idx[::-1]) for idx in
                  itertools.product(*[range(x) for x in reversed(n)])])
    np.testing.assert_allclose(sketch.left_product(cores, 4).reshape(-1, order="F"), X, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sketch.right_product(cores, -1).reshape(-1, order="F"), X, rtol=1e-12, atol=1e-12)
    for k in range(4):
        H = sketch.interface_matrix(cores, k)
        np.testing.assert_allclose(H @ solve.core_unfold2(cores[k]).T, sketch.unfold(X, n, k).T,
                                   rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("n,R,J", [([3, 4, 2, 3], [1, 2, 3, 2, 1], 7), ([4, 3, 5], [1, 3, 2, 1], 16),
                                   ([5, 4], [1, 3, 1], 9)])
def test_interface_cyclic_equals_explicit(n, R, J):
    cores = synth.random_cores(n, R, 13)
    hs, vs = _tabs(n, J, seed=14)
    for k in range(len(n)):
        np.testing.assert_allclose(sketch.interface_cyclic(cores, k, hs, vs, J),
                                   sketch.interface_explicit(cores, n, k, hs, vs, J), rtol=1e-11, atol=1e-11)


def _interface_fft(cores, k, hs, vs, J):
    """Theorems 1-2 (Sec. 3): per-core CountSketch along mode 2, FFT along the
    bucket axis, slice-wise products per frequency, face-split, inverse FFT."""
    d = len(cores)
    C = []
    for i, G in enumerate(cores):
        c = np.zeros((G.shape[0], J, G.shape[2]))
        for j in range(G.shape[1]):
            c[:, hs[i][j], :] += vs[i][j] * G[:, j, :]
        C.append(np.fft.fft(c, axis=1))
    P = np.ones((J, 1, 1), dtype=complex)
    for i in range(k):
        P = np.einsum("sab,bsc->sac", P, C[i])
    Q = np.ones((J, 1, 1), dtype=complex)
    for i in range(d - 1, k, -1):
        Q = np.einsum("asb,sbc->sac", C[i], Q)
    rk, rk1 = P.shape[2], Q.shape[1]
    Z = np.einsum("sa,sb->sab", P[:, 0, :], Q[:, :, 0]).reshape(J, rk * rk1, order="F")
    out = np.fft.ifft(Z, axis=0)
    return out


def test_theorems12_fft_route_equals_cyclic():
    n, R, J = [6, 5, 7, 4], [1, 3, 4, 2, 1], 30
    cores = synth.random_cores(n, R, 15)
    hs, vs = _tabs(n, J, seed=16)
    for k in range(4):
        out = _interface_fft(cores, k, hs, vs, J)
        ref = sketch.interface_cyclic(cores, k, hs, vs, J)
        np.testing.assert_allclose(out.real, ref, rtol=1e-10, atol=1e-10)
        assert np.abs(out.imag).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_lemma2_unbiased_inner_products():
    # E[(SA)^T (SB)] = A^T B over the hash/sign draws (Lemma 2's premise)
    n, J, T = [6, 5], 8, 3000
    g = synth.rng(17)
    A = g.standard_normal((30, 3))
    B = g.standard_normal((30, 2))
    est = np.empty((T, 3, 2))
    for t in range(T):
        hs, vs = tables.sweep_tables(1000 + t, 0, n, J)
        S = sketch.tensorsketch_matrix(hs, vs, J)
        est[t] = (S @ A).T @ (S @ B)
    mean, sd = est.mean(0), est.std(0, ddof=1)
    z = np.abs(mean - A.T @ B) / (sd / np.sqrt(T))
    assert z.max() < 4.5, z


def test_lemma2_tail_bound():
    # m >= (2 + 3^q)/(eps0^2 delta0)  =>  Pr[||A^T S^T S B - A^T B||^2 <= eps0^2 ||A||^2 ||B||^2] >= 1 - delta0
    from oracle import bound
    n, eps0, delta0 = [5, 6], 0.5, 0.5
    J = int(np.ceil(bound.lemma2_sketch_size(2, eps0, delta0)))
    assert J == 88
    g = synth.rng(18)
    A = g.standard_normal((30, 4))
    B = g.standard_normal((30, 3))
    ok = 0
    T = 400
    for t in range(T):
        hs, vs = tables.sweep_tables(5000 + t, 0, n, J)
        S = sketch.tensorsketch_matrix(hs, vs, J)
        err = np.linalg.norm((S @ A).T @ (S @ B) - A.T @ B) ** 2
        ok += err <= eps0 ** 2 * np.linalg.norm(A) ** 2 * np.linalg.norm(B) ** 2
    assert ok / T >= 1 - delta0


def test_sparse_sketch_equals_dense_sketch_of_densified_tensor():
    # the O(nnz) definition (sum over stored entries, repeated ones adding)
    # against the dense sketch of the tensor they describe
    n, J = [7, 5, 6, 4], 23
    g = synth.rng(61)
    nnz = 300
    coords = np.stack([g.integers(0, ns, size=nnz) for ns in n], axis=1)
    coords[10] = coords[3]                       # a repeated coordinate
    vals = g.standard_normal(nnz)
    X = np.zeros(n, order="F")
    np.add.at(X, tuple(coords.T), vals)
    hs = [g.integers(0, J, size=ns) for ns in n]
    vs = [g.choice([-1, 1], size=ns) for ns in n]
    for k in range(4):
        got = sketch.data_sketch_sparse(coords, vals, n, k, hs, vs, J)
        want = sketch.data_sketch(X.reshape(-1, order="F"), n, k, hs, vs, J)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
