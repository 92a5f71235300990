"""Pins of the oracle's proximal update, QR and orthogonalisation (CPU only).

Anchors: the stacked least-squares form of Theorem 5's proof (Sec. 4) solved
by numpy.linalg.lstsq, the exact proximal subproblem (Sec. 3, (lrtt_sub_prox)) under
an injective unit-sign sketch (S^T S = I), limiting cases of lambda, and QR /
TT invariants.
"""
import numpy as np
import pytest

import synth
from oracle import sketch, solve, tables


def test_prox_update_equals_stacked_lstsq():
    g = synth.rng(21)
    for (r0, nk, r1, J, lam) in [(2, 5, 3, 40, 0.3), (1, 7, 4, 25, 1e-3), (3, 4, 1, 12, 2.0)]:
        s = r0 * r1
        SH = g.standard_normal((J, s))
        Y = g.standard_normal((J, nk))
        G = g.standard_normal((r0, nk, r1))
        np.testing.assert_allclose(solve.prox_update(SH, Y, G, lam), solve.prox_update_stacked(SH, Y, G, lam),
                                   rtol=1e-10, atol=1e-12)


def test_prox_limits():
    g = synth.rng(22)
    SH = g.standard_normal((30, 6))
    Y = g.standard_normal((30, 5))
    G = g.standard_normal((2, 5, 3))
    # lambda -> infinity leaves the core unchanged
    np.testing.assert_allclose(solve.prox_update(SH, Y, G, 1e12), G, rtol=1e-9, atol=1e-9)
    # lambda = 0 with full column rank is ordinary least squares SH Z = Y
    Z = np.linalg.lstsq(SH, Y, rcond=None)[0]
    np.testing.assert_allclose(solve.core_unfold2(solve.prox_update(SH, Y, G, 0.0)).T, Z, rtol=1e-10, atol=1e-12)


def test_core_unfold2_index_order():
    G = np.arange(2 * 3 * 4, dtype=float).reshape((2, 3, 4), order="F")
    U = solve.core_unfold2(G)
    for a in range(2):
        for i in range(3):
            for b in range(4):
                assert U[i, a + 2 * b] == G[a, i, b]
    np.testing.assert_array_equal(solve.core_fold2(U, 2, 4), G)


def injective_tables(n):
    """h_s(i) = i * prod_{t<s} n_t, v = +1, J = N: every S_{-k} is an injection
    with unit signs, so S^T S = I and the sketched problem is the exact one."""
    hs, vs, stride = [], [], 1
    for ns in n:
        hs.append(np.arange(ns, dtype=np.int64) * stride)
        vs.append(np.ones(ns, dtype=np.int8))
        stride *= ns
    return hs, vs, stride


def test_injective_sketch_gives_exact_prox_update():
    n, R, lam = [4, 3, 5], [1, 2, 3, 1], 0.05
    cores = synth.random_cores(n, R, 23)
    X = synth.rng(24).standard_normal(60)
    hs, vs, J = injective_tables(n)
    for k in range(3):
        SH = sketch.interface_cyclic(cores, k, hs, vs, J)
        Y = sketch.data_sketch(X, n, k, hs, vs, J)
        got = solve.prox_update(SH, Y, cores[k], lam)
        # exact subproblem (lrtt_sub_prox): min ||H Z - A_(k)^T||^2 + lam ||Z - G_(2)^T||^2 by dense lstsq
        H = sketch.interface_matrix(cores, k)
        s = H.shape[1]
        A = np.vstack([H, np.sqrt(lam) * np.eye(s)])
        B = np.vstack([sketch.unfold(X, n, k).T, np.sqrt(lam) * solve.core_unfold2(cores[k]).T])
        Z = np.linalg.lstsq(A, B, rcond=None)[0]
        np.testing.assert_allclose(solve.core_unfold2(got).T, Z, rtol=1e-9, atol=1e-11)


def test_qr_pos_properties():
    g = synth.rng(25)
    for m, r in [(20, 4), (7, 7), (50, 1)]:
        A = g.standard_normal((m, r))
        Q, R = solve.qr_pos(A)
        np.testing.assert_allclose(Q.T @ Q, np.eye(r), atol=1e-13)
        np.testing.assert_allclose(Q @ R, A, atol=1e-12)
        assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)


def test_qr_of_zero_is_leading_identity():
    Q, R = solve.qr_pos(np.zeros((6, 3)))
    np.testing.assert_array_equal(Q, np.eye(6)[:, :3])
    np.testing.assert_array_equal(R, np.zeros((3, 3)))


def test_orthogonalisation_preserves_tt_and_orthonormalises():
    from oracle import als
    n, R = [5, 4, 6, 3], [1, 3, 4, 2, 1]
    cores = synth.random_cores(n, R, 26)
    full = als.tt_full(cores)
    rc = solve.right_orthogonalize(cores)
    np.testing.assert_allclose(als.tt_full(rc), full, rtol=1e-11, atol=1e-11)
    for k in range(1, 4):
        r0, nk, r1 = rc[k].shape
        GR = rc[k].reshape(r0, nk * r1, order="F")
        np.testing.assert_allclose(GR @ GR.T, np.eye(r0), atol=1e-12)
    a, b = solve.left_orth_absorb(rc[0], rc[1])
    cc = [a, b] + rc[2:]
    np.testing.assert_allclose(als.tt_full(cc), full, rtol=1e-11, atol=1e-11)
    GL = a.reshape(-1, a.shape[2], order="F")
    np.testing.assert_allclose(GL.T @ GL, np.eye(a.shape[2]), atol=1e-12)


def test_sweep_gauge_makes_interface_orthonormal():
    # In the sweep, cores < k are left- and cores > k right-orthonormal when
    # core k is updated, so H_k^T H_k = I and E[(S H_k)^T (S H_k)] = I.
    from oracle import als
    n, R, J = [4, 5, 3, 4], [1, 2, 3, 2, 1], 64
    X, _ = synth.tt_tensor_host(n, R, 0.1, 27)
    cores = synth.random_cores(n, R, 28)
    rec = []
    als.sweep(X, n, cores, J, 1e-3, seed=1, t=0, record=rec)
    for r in rec:
        H = sketch.interface_matrix(r["cores_in"], r["k"])
        np.testing.assert_allclose(H.T @ H, np.eye(H.shape[1]), atol=1e-11)


def test_round_bf16_pins():
    from oracle import solve
    # exact BF16 values are kept; 1 + 2^-8 is a tie between 1 and 1 + 2^-7
    # and goes to the even mantissa (1); 1 + 3 * 2^-8 ties up to 1 + 2^-6
    x = np.array([1.0, -2.5, 0.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, 3.0e38])
    want = np.array([1.0, -2.5, 0.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, 2.9980e38])
    got = solve.round_bf16(x)
    np.testing.assert_array_equal(got[:6], want[:6])
    assert abs(got[6] - 3.0e38) <= 2.0 ** -8 * 3.0e38
    # against torch's float32 -> bfloat16 conversion (round to nearest even)
    import torch
    g = np.random.default_rng(5).standard_normal(4000) * 10.0 ** np.random.default_rng(6).integers(-20, 20, 4000)
    ref = torch.from_numpy(g.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(solve.round_bf16(g), ref)
    # relative error at most 2^-9 of the FP32 value
    assert np.all(np.abs(solve.round_bf16(g) - g.astype(np.float32)) <= 2.0 ** -8 * np.abs(g.astype(np.float32)))
