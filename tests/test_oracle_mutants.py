"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case patches one plausible error into an oracle function (a wrong shift
direction, a dropped sign, a dropped proximal term, a transposed operand, a
missing QR sign normalisation) and checks that the corresponding pin test
fails.  Nothing here touches the GPU path.
"""
import numpy as np
import pytest

from oracle import sketch, solve
from tests import test_oracle_als as T_als
from tests import test_oracle_sketch as T_sk
from tests import test_oracle_solve as T_so


def _fails(fn, *a):
    with pytest.raises(AssertionError):
        fn(*a)


def test_shift_direction_mutant(monkeypatch):
    monkeypatch.setattr(sketch, "_shift", lambda P, h: np.roll(P, -int(h), axis=0))
    _fails(T_sk.test_interface_cyclic_equals_explicit, [3, 4, 2, 3], [1, 2, 3, 2, 1], 7)


def test_tensorsketch_sign_mutant(monkeypatch):
    orig = sketch.tensorsketch_matrix

    def bad(hs, vs, J):          # sign of the first mode only
        return orig(hs, [vs[0]] + [np.ones_like(v) for v in vs[1:]], J)
    monkeypatch.setattr(sketch, "tensorsketch_matrix", bad)
    _fails(T_sk.test_paper_worked_example)


def test_tensorsketch_no_mod_mutant(monkeypatch):
    def bad(hs, vs, J):          # hash sum clipped instead of reduced mod J
        sizes = [len(h) for h in hs]
        S = np.zeros((J, int(np.prod(sizes))))
        for j in range(S.shape[1]):
            rem, b, sg = j, 0, 1
            for h, v, ns in zip(hs, vs, sizes):
                i = rem % ns
                rem //= ns
                b += int(h[i])
                sg *= int(v[i])
            S[min(b, J - 1), j] += sg
        return S
    monkeypatch.setattr(sketch, "tensorsketch_matrix", bad)
    _fails(T_sk.test_paper_worked_example)


def test_data_sketch_dropped_sign_mutant(monkeypatch):
    orig = sketch.data_sketch

    def bad(X, n, k, hs, vs, J, slab_entries=1 << 24):
        return orig(X, n, k, hs, [np.ones_like(v) for v in vs], J, slab_entries)
    monkeypatch.setattr(sketch, "data_sketch", bad)
    _fails(T_sk.test_data_sketch_equals_explicit, (3, 4, 2), 5)


def test_prox_dropped_term_mutant(monkeypatch):
    def bad(SH, Y, G_old, lam):
        r0, nk, r1 = G_old.shape
        M = SH.T @ SH + lam * np.eye(r0 * r1)
        Z = np.linalg.solve(M, SH.T @ Y)            # lambda * G_old missing
        return solve.core_fold2(Z.T, r0, r1)
    monkeypatch.setattr(solve, "prox_update", bad)
    _fails(T_so.test_prox_update_equals_stacked_lstsq)


def test_interface_kron_order_mutant(monkeypatch):
    def bad(cores, k):           # operands of the Kronecker product swapped
        return np.kron(sketch.left_product(cores, k), sketch.right_product(cores, k).T)
    monkeypatch.setattr(sketch, "interface_matrix", bad)
    _fails(T_sk.test_tt_products_and_interface_matrix)


def test_qr_sign_mutant(monkeypatch):
    monkeypatch.setattr(solve, "qr_pos", lambda A: np.linalg.qr(-np.asarray(A, float), mode="reduced"))
    _fails(T_so.test_qr_pos_properties)


def test_sweep_wrong_gauge_mutant(monkeypatch):
    # skipping the QR + absorb step leaves H_k without orthonormal columns
    monkeypatch.setattr(solve, "left_orth_absorb", lambda a, b: (a, b))
    _fails(T_so.test_sweep_gauge_makes_interface_orthonormal)


def test_core_change_old_denominator_mutant(monkeypatch):
    from oracle import als

    def bad(old, new):           # divides by the OLD core's norm
        return max(float(np.linalg.norm(b - a) / np.linalg.norm(a)) for a, b in zip(old, new))
    monkeypatch.setattr(als, "core_change", bad)
    _fails(T_als.test_core_change_hand_cases)


def test_core_change_sum_mutant(monkeypatch):
    from oracle import als

    def bad(old, new):           # sums the per-core changes
        return sum(float(np.linalg.norm(b - a) / np.linalg.norm(b)) for a, b in zip(old, new))
    monkeypatch.setattr(als, "core_change", bad)
    _fails(T_als.test_core_change_hand_cases)


def test_run_skips_table_redraw_mutant(monkeypatch):
    from oracle import als
    orig = als.sweep

    def bad(X, n, cores, J, lam, seed=0, t=0, **kw):   # the tables of pass 0 every pass
        return orig(X, n, cores, J, lam, seed=seed, t=0, **kw)
    monkeypatch.setattr(als, "sweep", bad)
    import oracle.als as mod

    def run_bad(X, n, cores, J, lam, seed, sweeps, interface="cyclic"):
        res, chg = [], []
        for t in range(sweeps):
            new = bad(X, n, cores, J, lam, seed=seed, t=t, interface=interface)
            chg.append(mod.core_change(cores, new))
            cores = new
            res.append(mod.rel_residual(X, cores))
        return cores, res, chg
    monkeypatch.setattr(als, "run", run_bad)
    monkeypatch.setattr(als, "sweep", orig)
    _fails(T_als.test_run_histories_match_single_sweeps)


def test_round_bf16_truncation_mutant(monkeypatch):
    def bad(A):                  # truncates instead of rounding to nearest even
        x = np.ascontiguousarray(np.asarray(A, dtype=np.float64).astype(np.float32))
        b = (x.view(np.uint32) >> np.uint32(16)) << np.uint32(16)
        return b.view(np.float32).astype(np.float64).reshape(np.shape(A))
    monkeypatch.setattr(solve, "round_bf16", bad)
    _fails(T_so.test_round_bf16_pins)


def test_exact_rhs_kron_order_mutant(monkeypatch):
    # the exact right-hand side pinned by brute force catches swapped
    # Kronecker operands in H_k
    def bad(cores, k):
        return np.kron(sketch.left_product(cores, k), sketch.right_product(cores, k).T)
    monkeypatch.setattr(sketch, "interface_matrix", bad)
    _fails(T_als.test_exact_rhs_by_brute_force)
