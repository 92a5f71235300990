"""Pins of the oracle's full sweep (Algorithm 1, Sec. 3) and of Theorem 5 /
Corollary 3 (Sec. 4), CPU only.

Anchors: exact recovery of a noise-free TT (the objective (lrtt) reaches 0 at
the generating cores), convergence to the noise floor, the injective-sketch
sweep equals exact proximal TT-ALS, Eckart-Young for d = 2, and the
(1 + eps) * OPT guarantee of Theorem 5 at a size where Corollary 3's m is
attainable.
"""
import numpy as np
import pytest

import synth
from oracle import als, bound, sketch, solve, tables
from tests.test_oracle_solve import injective_tables


def test_noise_free_tt_is_recovered():
    n, R, J = [10, 10, 10, 10], [1, 3, 3, 3, 1], 256
    X, _ = synth.tt_tensor_host(n, R, 0.0, 31)
    cores = synth.random_cores(n, R, 32)
    res = []
    for t in range(10):
        cores = als.sweep(X, n, cores, J, 1e-3, seed=5, t=t)
        res.append(als.rel_residual(X, cores))
    assert res[-1] < 1e-7, res
    assert res[-1] < res[0] * 1e-4


def test_noisy_tt_converges_to_noise_floor():
    n, R, J, noise = [10, 10, 10, 10], [1, 3, 3, 3, 1], 256, 1e-2
    X, _ = synth.tt_tensor_host(n, R, noise, 33)
    floor = noise * np.sqrt(X.size) / np.linalg.norm(X)
    cores = synth.random_cores(n, R, 34)
    for t in range(8):
        cores = als.sweep(X, n, cores, J, 1e-3, seed=6, t=t)
    r = als.rel_residual(X, cores)
    assert 0.5 * floor < r < 1.5 * floor, (r, floor)


def test_injective_sketch_sweep_is_exact_prox_als():
    # With S^T S = I every step is the exact proximal TT-ALS step (lrtt_sub_prox).
    n, R, lam = [4, 5, 3], [1, 2, 3, 1], 0.1
    X = synth.rng(35).standard_normal(60)
    cores0 = synth.random_cores(n, R, 36)
    hs, vs, J = injective_tables(n)
    got = als.sweep(X, n, cores0, J, lam, tabs=(hs, vs))
    # exact proximal ALS written with dense H_k and A_(k)
    cores = solve.right_orthogonalize(cores0)
    for k in range(3):
        H = sketch.interface_matrix(cores, k)
        s = H.shape[1]
        A = np.vstack([H, np.sqrt(lam) * np.eye(s)])
        B = np.vstack([sketch.unfold(X, n, k).T, np.sqrt(lam) * solve.core_unfold2(cores[k]).T])
        Z = np.linalg.lstsq(A, B, rcond=None)[0]
        cores[k] = solve.core_fold2(Z.T, cores[k].shape[0], cores[k].shape[2])
        if k < 2:
            cores[k], cores[k + 1] = solve.left_orth_absorb(cores[k], cores[k + 1])
    for a, b in zip(got, cores):
        np.testing.assert_allclose(a, b, rtol=1e-8, atol=1e-10)


def test_d2_exact_sketch_reaches_eckart_young():
    g = synth.rng(37)
    n0, n1, r = 9, 8, 3
    U, _ = np.linalg.qr(g.standard_normal((n0, n0)))
    V, _ = np.linalg.qr(g.standard_normal((n1, n1)))
    sv = np.array([10.0, 8.0, 6.0, 1.0, 0.5, 0.3, 0.2, 0.1])
    M = U[:, :8] @ np.diag(sv) @ V.T
    X = M.reshape(-1, order="F")
    best = np.sqrt((sv[r:] ** 2).sum()) / np.linalg.norm(sv)
    hs, vs, J = injective_tables([n0, n1])
    cores = synth.random_cores([n0, n1], [1, r, 1], 38)
    for t in range(40):
        cores = als.sweep(X, [n0, n1], cores, J, 1e-12, tabs=(hs, vs))
    assert abs(als.rel_residual(X, cores) - best) < 1e-8


def test_cor3_bound_values():
    # s = 1, q = 2, eps = 1, delta = 0.5 -> m = max{88/0.5, 88/0.5} = 176
    assert bound.cor3_sketch_size_int(1, 2, 1.0, 0.5) == 176
    # the s^2 branch dominates when s > 1/eps
    assert bound.cor3_sketch_size(10, 3, 0.5, 0.1) == max(8 * 100 * 29 / 0.1, 8 * 10 * 29 / 0.05)


def test_theorem5_one_plus_eps_opt():
    # d = 3, update of the middle core (q = 2 sketched modes), ranks 1 (s = 1):
    # Cor. 3's m = 176 at eps = 1, delta = 0.5.
    eps, delta = 1.0, 0.5
    J = bound.cor3_sketch_size_int(1, 2, eps, delta)
    n, R, lam, k = [6, 5, 7], [1, 1, 1, 1], 0.5, 1
    g = synth.rng(39)
    X = g.standard_normal(210)
    cores = solve.right_orthogonalize(synth.random_cores(n, R, 40))
    H = sketch.interface_matrix(cores, k)
    B = sketch.unfold(X, n, k).T
    C = solve.core_unfold2(cores[k]).T

    def f(Z):
        return 0.5 * np.linalg.norm(H @ Z - B) ** 2 + 0.5 * lam * np.linalg.norm(Z - C) ** 2

    A = np.vstack([H, np.sqrt(lam) * np.eye(1)])
    Zopt = np.linalg.lstsq(A, np.vstack([B, np.sqrt(lam) * C]), rcond=None)[0]
    opt = f(Zopt)
    ok, T = 0, 200
    for t in range(T):
        hs, vs = tables.sweep_tables(900 + t, 0, n, J)
        SH = sketch.interface_cyclic(cores, k, hs, vs, J)
        Y = sketch.data_sketch(X, n, k, hs, vs, J)
        Z = solve.core_unfold2(solve.prox_update(SH, Y, cores[k], lam)).T
        ok += f(Z) <= (1 + eps) * opt
    assert ok / T >= 1 - delta


def test_core_change_hand_cases():
    # The accuracy measure of Sec. 5 (first paragraph): the largest, over the
    # cores, of ||G_k^(t+1) - G_k^(t)||_F / ||G_k^(t+1)||_F.
    g = synth.rng(41)
    old = [g.standard_normal((1, 4, 2)), g.standard_normal((2, 5, 3)), g.standard_normal((3, 4, 1))]
    assert als.core_change(old, [c.copy() for c in old]) == 0.0
    # one core doubled: ||2G - G|| / ||2G|| = 1/2 (denominator is the NEW core)
    new = [c.copy() for c in old]
    new[1] = 2.0 * old[1]
    assert abs(als.core_change(old, new) - 0.5) < 1e-15
    # one core halved: ||G/2 - G|| / ||G/2|| = 1 (with the old core as the
    # denominator this would read 1/2)
    new = [c.copy() for c in old]
    new[2] = 0.5 * old[2]
    assert abs(als.core_change(old, new) - 1.0) < 1e-15
    # two cores changed: the measure is their maximum, not their sum
    new = [c.copy() for c in old]
    new[0] = 2.0 * old[0]           # 0.5
    new[2] = -old[2]                # ||-2G|| / ||G|| = 2
    assert abs(als.core_change(old, new) - 2.0) < 1e-15
    # a change of one entry by e in a core of unit norm gives e / ||new||
    unit = [np.zeros((1, 3, 1)), np.zeros((1, 3, 1))]
    unit[0][0, 0, 0] = 1.0
    unit[1][0, 1, 0] = 1.0
    moved = [c.copy() for c in unit]
    moved[1][0, 2, 0] = 0.75        # ||(0,0,.75)|| / ||(0,1,.75)|| = 0.75 / 1.25
    assert abs(als.core_change(unit, moved) - 0.6) < 1e-15


def test_run_histories_match_single_sweeps():
    # als.run = repeated Algorithm 1 passes with the tables of pass t, logging
    # after each pass the exact residual and the core change of that pass.
    n, R, J, lam, seed, T = [6, 5, 4, 5], [1, 2, 3, 2, 1], 64, 1e-3, 17, 3
    X, _ = synth.tt_tensor_host(n, R, 1e-2, 42)
    init = synth.random_cores(n, R, 43)
    cores, res, chg = als.run(X, n, init, J, lam, seed, T)
    assert len(res) == T and len(chg) == T
    cur = [c.copy() for c in init]
    for t in range(T):
        nxt = als.sweep(X, n, cur, J, lam, seed=seed, t=t)
        assert res[t] == als.rel_residual(X, nxt)
        assert chg[t] == als.core_change(cur, nxt)
        cur = nxt
    for a, b in zip(cores, cur):
        assert np.array_equal(a, b)
    # the first pass starts from unorthogonalised random cores, so every core
    # moves; the residual history is that of a converging run
    assert chg[0] > 0.1 and res[-1] < res[0]


def test_exact_sweep_equals_injective_sketch_and_stacked_lstsq():
    # (lrtt_sub_prox) three ways: explicit H_k (sweep_exact), an injective
    # sketch (S^T S = I, als.sweep), and the stacked least squares of the
    # proof of Theorem 5 per core
    n, R, lam = [4, 5, 3, 2], [1, 2, 3, 2, 1], 0.05
    X = synth.rng(44).standard_normal(120)
    cores0 = synth.random_cores(n, R, 45)
    got = als.sweep_exact(X, n, cores0, lam)
    hs, vs, J = injective_tables(n)
    inj = als.sweep(X, n, cores0, J, lam, tabs=(hs, vs))
    cores = solve.right_orthogonalize(cores0)
    for k in range(4):
        H = sketch.interface_matrix(cores, k)
        cores[k] = solve.prox_update_stacked(H, sketch.unfold(X, n, k).T, cores[k], lam)
        if k < 3:
            cores[k], cores[k + 1] = solve.left_orth_absorb(cores[k], cores[k + 1])
    for a, b, c in zip(got, inj, cores):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(a, c, rtol=1e-9, atol=1e-11)


def test_exact_rhs_by_brute_force():
    # (A_(k) H_k)(i_k, alpha + R_k beta) = sum over the other indices of
    # X(i) G_<k(i_<k, alpha) G_>k(beta, i_>k), entry by entry
    n, R = [3, 4, 2], [1, 2, 3, 1]
    X = synth.rng(46).standard_normal(24)
    cores = synth.random_cores(n, R, 47)
    T = X.reshape(n, order="F")
    for k in range(3):
        B = als.exact_rhs(X, n, cores, k)
        want = np.zeros_like(B)
        for idx in np.ndindex(*n):
            left = np.ones((1,))
            for i in range(k):
                left = left @ cores[i][:, idx[i], :]
            right = np.ones((1,))
            for i in range(2, k, -1):
                right = cores[i][:, idx[i], :] @ right
            for a in range(R[k]):
                for b in range(R[k + 1]):
                    want[idx[k], a + R[k] * b] += T[idx] * left[a] * right[b]
        np.testing.assert_allclose(B, want, rtol=1e-12, atol=1e-12)
