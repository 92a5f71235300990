"""GPU parity of every step of the hot path against the FP64 oracle.

All calls go through the C ABI (via the thin binding) on seeded synthetic
inputs; the oracle receives the same arrays and the same tables.  Tolerances:
  * hash/sign tables and integer-valued data sketches: bit-exact;
  * FP64 work type: 1e-10 relative (Frobenius);
  * FP32 work type: 1e-5 relative for sketches, derived bounds for solves;
  * full sweeps: relative residual within 1e-4 of the oracle's.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import als, sketch, solve, tables

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_08093_amd as m
    return m


DEV = "cuda"


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def colmax(a, b):
    """Element-wise error: the largest over columns of max |a - b| in the
    column divided by max |b| in that column (a zero reference column counts
    with its absolute error).  A wrong small entry under a large column norm
    shows here, not in the Frobenius ratio."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    a2 = a.reshape(a.shape[0], -1) if a.ndim > 1 else a[:, None]
    b2 = b.reshape(b.shape[0], -1) if b.ndim > 1 else b[:, None]
    den = np.abs(b2).max(axis=0)
    err = np.abs(a2 - b2).max(axis=0)
    return float(np.max(np.where(den > 0, err / np.where(den > 0, den, 1.0), err)))


def host_tables(plan):
    hs, vs = [], []
    for s in range(plan.d):
        h, v = plan.get_tables(s)
        hs.append(h)
        vs.append(v)
    return hs, vs


def to_dev_x(Xh, dtype):
    t = synth.to_dtype_host(Xh, dtype)
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(t)
    return t.to(DEV)


# ------------------------------------------------------------------ tables
@pytest.mark.parametrize("seed,n,J", [(0, [16, 16, 16, 16], 256), (12345, [200, 7, 33], 4000),
                                      (2 ** 63 + 5, [5, 64, 3, 2, 9], 3000), (7, [3, 4], 1)])
def test_tables_bit_exact(tts, seed, n, J):
    say("tables", seed, n, J)
    R = [1] + [1] * (len(n) - 1) + [1]
    plan = tts.Plan(n, R, J, 1e-3, seed=seed, x_dtype="f32", work_dtype="f32")
    for t in (0, 1, 7):
        plan.set_sweep(t)
        for s in range(len(n)):
            h, v = plan.get_tables(s)
            ho, vo = tables.mode_tables(seed, t, s, n[s], J)
            assert np.array_equal(h, ho) and np.array_equal(v, vo), (t, s)


def test_set_tables_roundtrip(tts):
    say("set_tables")
    n, J = [6, 5, 4], 8
    plan = tts.Plan(n, [1, 2, 2, 1], J, 1e-3)
    h = np.array([7, 0, 3, 3, 1, 5])
    v = np.array([1, -1, -1, 1, 1, -1])
    plan.set_tables(0, h, v)
    h2, v2 = plan.get_tables(0)
    assert np.array_equal(h2, h) and np.array_equal(v2, v)
    with pytest.raises(tts.TTError):
        plan.set_tables(0, np.full(6, 8), v)       # bucket out of range


# ------------------------------------------------------------------ data sketch
SKETCH_CASES = [
    # n, J, x dtype, work dtype
    ([16, 16, 16, 16], 256, "f64", "f64"),
    ([37, 5, 9, 4], 60, "f32", "f32"),
    ([200, 3, 2], 4000, "f32", "f32"),
    ([65, 130], 12, "f32", "f32"),
    ([7, 300, 5], 1000, "f32", "f32"),
    ([64, 8, 8, 8, 8], 3000, "bf16", "f32"),
    ([300, 4, 3], 128, "f32", "f32"),
    ([1030, 3, 2], 50, "f32", "f32"),          # n_0 > 1024: chunked k = 0 path
    ([1, 5, 4], 8, "f32", "f32"),
    ([5, 1, 4], 8, "f64", "f64"),
    # at least two fibres per key for every k >= 1: key-grouped path
    ([20, 30, 40, 10], 60, "f32", "f32"),
    ([64, 16, 16, 16], 64, "bf16", "f32"),
    ([16, 16, 16, 16], 32, "f64", "f64"),
    ([37, 12, 11, 13], 40, "f32", "f32"),      # n_0 not a multiple of 4: scalar loads
    ([8, 40, 50], 24, "f64", "f64"),           # lane groups of 4 fibres
    # one fibre fills the wave (double-buffered loads), with a ragged batch tail
    ([256, 20, 20, 10], 64, "f32", "f32"),
    ([300, 12, 10, 7], 30, "f32", "f32"),      # two vectors per lane
    # the largest sketch size and the largest n_0
    ([4096, 3, 2], 8192, "f32", "f32"),
]


@pytest.mark.parametrize("n,J,xd,wd", SKETCH_CASES)
def test_data_sketch_integer_exact(tts, n, J, xd, wd):
    say("sketch int", n, J, xd, wd)
    N = int(np.prod(n))
    Xh = synth.rng(1).integers(-4, 5, size=N).astype(np.float64)   # every partial sum exact in FP32
    plan = tts.Plan(n, [1] * (len(n) + 1), J, 1e-3, seed=3, x_dtype=xd, work_dtype=wd)
    hs, vs = host_tables(plan)
    X = to_dev_x(Xh, xd)
    for k in range(len(n)):
        Y = plan.sketch_tensor(X, k).cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        Yo = sketch.data_sketch(Xh, n, k, hs, vs, J)
        assert np.array_equal(Y, Yo), (k, np.abs(Y - Yo).max())


@pytest.mark.parametrize("n,J,xd,wd", SKETCH_CASES)
def test_data_sketch_float(tts, n, J, xd, wd):
    say("sketch float", n, J, xd, wd)
    N = int(np.prod(n))
    Xh = synth.rng(2).standard_normal(N)
    plan = tts.Plan(n, [1] * (len(n) + 1), J, 1e-3, seed=4, x_dtype=xd, work_dtype=wd)
    hs, vs = host_tables(plan)
    X = to_dev_x(Xh, xd)
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))   # the oracle reads the same stored values
    tol = 1e-12 if wd == "f64" else 1e-5
    for k in range(len(n)):
        Y = plan.sketch_tensor(X, k).cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        Yo = sketch.data_sketch(Xo, n, k, hs, vs, J)
        assert rel(Y, Yo) < tol, k
        # bucket sums are FP64 and rounded once to the work type
        assert colmax(Y, Yo) < tol, (k, colmax(Y, Yo))


# all d sketches of a sweep with the outer sketch of the k = 0 pass forced on
# (Y_0 and Y_1 derived from it): f64, bf16 with short fibres (lane groups
# folded), n_0 above the k = 0 chunk, n_0 = 1, n_1 = 1, scalar loads, two
# vectors per lane, J = 1, slabs longer than one piece
FUSED_CASES = [
    ([16, 16, 16, 16], 256, "f64", "f64"),
    ([37, 5, 9, 4], 60, "f32", "f32"),
    ([64, 8, 8, 8, 8], 3000, "bf16", "f32"),
    ([7, 300, 5], 1000, "f32", "f32"),
    ([1030, 3, 2], 50, "f32", "f32"),
    ([1, 5, 4], 8, "f32", "f32"),
    ([5, 1, 4], 8, "f64", "f64"),
    ([37, 12, 11, 13], 40, "f32", "f32"),
    ([300, 12, 10, 7], 30, "f32", "f32"),
    ([20, 30, 40, 10], 60, "f32", "f32"),
    ([12, 9, 7], 1, "f32", "f32"),
    ([90, 50, 4, 4, 4], 8, "f32", "f32"),     # slabs of 4500 values: two pieces per slab
    ([77, 61, 4, 4, 3], 8, "f32", "f32"),     # 4697 (odd): single values, two pieces
]


@pytest.mark.parametrize("inner", [None, False])
@pytest.mark.parametrize("n,J,xd,wd", FUSED_CASES)
def test_sketch_all_fused(tts, n, J, xd, wd, inner):
    say("sketch all fused", n, J, xd, wd, inner)
    N = int(np.prod(n))
    plan = tts.Plan(n, [1] * (len(n) + 1), J, 1e-3, seed=5, x_dtype=xd, work_dtype=wd, fuse=True, inner=inner)
    assert plan.sketch_sources()[:2] == [0, 0]
    hs, vs = host_tables(plan)
    # integer-valued: bit-exact
    Xi = synth.rng(6).integers(-4, 5, size=N).astype(np.float64)
    Ys = plan.sketch_tensor_all(to_dev_x(Xi, xd))
    for k in range(len(n)):
        Y = Ys[k].cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        Yo = sketch.data_sketch(Xi, n, k, hs, vs, J)
        assert np.array_equal(Y, Yo), (k, np.abs(Y - Yo).max())
    # Gaussian: 1e-5 (FP32 work) or 1e-12 (FP64 work), norm-wise and element-wise
    Xh = synth.rng(7).standard_normal(N)
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))
    Ys = plan.sketch_tensor_all(to_dev_x(Xh, xd))
    tol = 1e-12 if wd == "f64" else 1e-5
    for k in range(len(n)):
        Y = Ys[k].cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        Yo = sketch.data_sketch(Xo, n, k, hs, vs, J)
        assert rel(Y, Yo) < tol and colmax(Y, Yo) < tol, (k, rel(Y, Yo), colmax(Y, Yo))


# key-grouped sketches at k >= 2 with fibres that straddle 128-byte lines at
# every phase: FP32 in 4-value loads (n_0 = 72, 96) and single values
# (n_0 = 77, fibres on 4-byte boundaries), FP64 (n_0 = 40), BF16 (n_0 = 136);
# X also shifted off its allocation's alignment (16 bytes keeps the vector
# loads, 4 bytes makes them single values)
LINE_CASES = [([72, 6, 9, 7], 16, "f32", 0), ([72, 6, 9, 7], 16, "f32", 4), ([72, 6, 9, 7], 16, "f32", 1),
              ([96, 5, 6, 8], 12, "f32", 0), ([77, 5, 8, 6], 12, "f32", 0), ([40, 6, 8, 5], 12, "f64", 0),
              ([40, 6, 8, 5], 12, "f64", 2), ([136, 4, 6, 5], 8, "bf16", 0), ([136, 4, 6, 5], 8, "bf16", 8)]


@pytest.mark.parametrize("n,J,xd,shift", LINE_CASES)
def test_sketch_straddling_lines(tts, n, J, xd, shift):
    say("sketch straddling lines", n, J, xd, shift)
    N = int(np.prod(n))
    plan = tts.Plan(n, [1] * (len(n) + 1), J, 1e-3, seed=9, x_dtype=xd, work_dtype="f64" if xd == "f64" else "f32")
    assert all(plan.sketch_kernel(k) == "k_sketch_gs" for k in range(2, len(n)))
    hs, vs = host_tables(plan)
    for kind in ("integer", "gaussian"):
        Xh = (synth.rng(11).integers(-4, 5, size=N).astype(np.float64) if kind == "integer"
              else synth.rng(12).standard_normal(N))
        xt = to_dev_x(Xh, xd)
        buf = torch.empty(N + shift, dtype=xt.dtype, device=DEV)
        buf[shift:] = xt
        X = buf[shift:]
        Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))
        for k in range(2, len(n)):
            Y = plan.sketch_tensor(X, k).cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
            Yo = sketch.data_sketch(Xo, n, k, hs, vs, J)
            if kind == "integer":
                assert np.array_equal(Y, Yo), (k, np.abs(Y - Yo).max())
            else:
                tol = 1e-12 if xd == "f64" else 1e-5
                assert rel(Y, Yo) < tol and colmax(Y, Yo) < tol, (k, rel(Y, Yo), colmax(Y, Yo))


# every Y_k, k >= 2, from the inner sketch (one pass over X writes the sketch
# of every slab over modes 0 and 1): 4-value, 2-value (FP64), 8-value (BF16)
# and single-value loads; 1, 2, 4 and 16 vectors per lane; short rows several
# to a wave; d = 5; a mode of size 1; J = 1; X shifted off its alignment
INNER_CASES = [
    ([20, 30, 40, 10], 60, "f32", "f32", None, 0),
    ([20, 30, 40, 10], 60, "f32", "f32", True, 4),
    ([37, 12, 11, 13], 40, "f32", "f32", None, 0),
    ([300, 12, 10, 7], 30, "f32", "f32", False, 0),
    ([64, 8, 8, 8, 8], 300, "bf16", "f32", None, 0),
    ([40, 6, 8, 5], 12, "f64", "f64", None, 0),
    ([40, 6, 8, 5], 12, "f64", "f64", None, 1),
    ([1000, 3, 4, 5], 16, "f32", "f32", None, 0),
    ([1000, 3, 4, 5], 16, "bf16", "f32", None, 0),
    ([999, 2, 3, 4], 16, "f32", "f32", None, 0),
    ([12, 9, 7, 1], 1, "f32", "f32", None, 0),
    ([8, 7, 1, 5, 3], 4, "f64", "f64", True, 0),
    # with the outer sketch and FP32 work the k = 0 pass writes both
    # intermediates (aligned X): 4, 8 and 10 vectors of FP32 per thread, a
    # slab of 40000 values (the 200^4 workload's), of 40960 (the largest),
    # BF16, d = 5
    ([20, 30, 40, 10], 60, "f32", "f32", True, 0),
    ([200, 200, 3, 2], 64, "f32", "f32", True, 0),
    ([128, 320, 2, 3], 32, "f32", "f32", True, 0),
    ([128, 256, 2, 2], 16, "f32", "f32", True, 0),
    ([1000, 3, 4, 5], 16, "f32", "f32", True, 0),
    ([96, 40, 5, 3], 16, "bf16", "f32", True, 0),
    ([128, 256, 2, 2], 16, "bf16", "f32", True, 0),
    ([64, 8, 8, 8, 8], 300, "bf16", "f32", True, 0),
    ([12, 10, 3, 4, 5], 20, "f32", "f32", True, 0),
    # the inner sketch over modes 0..2 (mode 2 keeps its own pass): d = 5
    # FP32, BF16 and FP64, and d = 6
    ([12, 10, 8, 9, 7], 300, "f32", "f32", None, 0),
    ([16, 8, 8, 6, 5], 64, "bf16", "f32", True, 0),
    ([10, 6, 5, 7, 4], 24, "f64", "f64", None, 0),
    ([10, 6, 5, 4, 6, 5], 32, "f32", "f32", None, 0),
]


@pytest.mark.parametrize("n,J,xd,wd,fuse,shift", INNER_CASES)
def test_sketch_all_inner(tts, n, J, xd, wd, fuse, shift):
    say("sketch all inner", n, J, xd, wd, fuse, shift)
    N = int(np.prod(n))
    plan = tts.Plan(n, [1] * (len(n) + 1), J, 1e-3, seed=5, x_dtype=xd, work_dtype=wd, fuse=fuse, inner=True)
    src = plan.sketch_sources()
    d = len(n)
    # Y_m.. from the inner sketch over modes 0..m-1, written by the pass of
    # mode m (modes 2..m-1 keep their own passes) or, for m = 2 with FP32 work
    # and the outer sketch, by the k = 0 pass
    m = src[-1]
    if m == 0:
        assert src[1:] == [0] * (d - 1), src
    else:
        assert 2 <= m <= d - 2 and src[2:] == list(range(2, m + 1)) + [m] * (d - m - 1), src
    vec = 8 if xd == "bf16" else 4
    if m == 0 or (m == 2 and fuse and wd == "f32" and n[0] % vec == 0 and
                  n[0] * n[1] <= 1024 * (32 if xd == "bf16" else 40)):
        assert src == [0] * d, src
    hs, vs = host_tables(plan)

    def shifted(Xh):
        xt = to_dev_x(Xh, xd)
        buf = torch.empty(N + shift, dtype=xt.dtype, device=DEV)
        buf[shift:] = xt
        return buf[shift:]

    # integer-valued: bit-exact
    Xi = synth.rng(6).integers(-4, 5, size=N).astype(np.float64)
    Ys = plan.sketch_tensor_all(shifted(Xi))
    for k in range(len(n)):
        Y = Ys[k].cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        Yo = sketch.data_sketch(Xi, n, k, hs, vs, J)
        assert np.array_equal(Y, Yo), (k, np.abs(Y - Yo).max())
    # Gaussian: 1e-5 (FP32 work) or 1e-12 (FP64 work), norm-wise and element-wise
    Xh = synth.rng(7).standard_normal(N)
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))
    Ys = plan.sketch_tensor_all(shifted(Xh))
    tol = 1e-12 if wd == "f64" else 1e-5
    for k in range(len(n)):
        Y = Ys[k].cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        Yo = sketch.data_sketch(Xo, n, k, hs, vs, J)
        assert rel(Y, Yo) < tol and colmax(Y, Yo) < tol, (k, rel(Y, Yo), colmax(Y, Yo))


def test_sketch_inner_rule(tts):
    say("sketch inner rule")
    # |Z| = J n_2 n_3 = 2e5 values against N = 4e6: one pass serves Y_2 and Y_3
    assert tts.Plan([100, 100, 20, 20], [1, 1, 1, 1, 1], 500, 1e-3).sketch_sources()[2:] == [2, 2]
    assert tts.Plan([100, 100, 20, 20], [1, 1, 1, 1, 1], 500, 1e-3, inner=False).sketch_sources()[2:] == [2, 3]
    # |Z| as large as X: each mode keeps its own pass
    assert tts.Plan([16, 16, 16, 16], [1, 1, 1, 1, 1], 256, 1e-3).sketch_sources() == [0, 1, 2, 3]
    # d = 3 has no mode beyond 2; n_0 > 1024 is not taken
    assert tts.Plan([30, 40, 50], [1, 3, 3, 1], 64, 1e-3, inner=True).sketch_sources() == [0, 1, 2]
    assert tts.Plan([1030, 3, 2, 2], [1] * 5, 8, 1e-3, inner=True, fuse=False).sketch_sources() == [0, 1, 2, 3]
    # both intermediates from the k = 0 pass: FP32 work, n_0 a multiple of
    # 4 (FP32 X), slabs of at most 40960 values
    assert tts.Plan([200, 200, 3, 2], [1] * 5, 64, 1e-3, inner=True, fuse=True).sketch_sources() == [0, 0, 0, 0]
    assert tts.Plan([202, 200, 3, 2], [1] * 5, 64, 1e-3, inner=True, fuse=True).sketch_sources() == [0, 0, 2, 2]
    assert tts.Plan([128, 324, 2, 3], [1] * 5, 32, 1e-3, inner=True, fuse=True).sketch_sources() == [0, 0, 2, 2]
    assert tts.Plan([200, 200, 3, 2], [1] * 5, 64, 1e-3, inner=True, fuse=True, x_dtype="f64",
                    work_dtype="f64").sketch_sources() == [0, 0, 2, 2]
    # d = 5: the grouping with the fewest bytes; over modes 0..2 when the
    # sketch of modes 0, 1 would be larger (|Z| = J n_2 n_3 n_4 = 151200
    # values against J n_3 n_4 = 18900 and one more pass over X)
    assert tts.Plan([12, 10, 8, 9, 7], [1] * 6, 300, 1e-3, inner=True, fuse=False).sketch_sources() == [0, 1, 2, 3, 3]
    assert tts.Plan([40, 30, 3, 3, 2], [1] * 6, 50, 1e-3, inner=True, fuse=False).sketch_sources() == [0, 1, 2, 2, 2]
    # the 64^5 BF16 workload (J = 3000): a pass per mode k >= 2 by default
    # (2-byte entries: the inner pass is bound by its LDS atomics), modes
    # 0..2 on request
    assert tts.Plan([64] * 5, [1, 8, 8, 8, 8, 1], 3000, 1e-3, x_dtype="bf16").sketch_sources() == [0, 0, 2, 3, 4]
    assert tts.Plan([64] * 5, [1, 8, 8, 8, 8, 1], 3000, 1e-3, x_dtype="bf16",
                    inner=True).sketch_sources() == [0, 0, 2, 3, 3]
    # BF16 X: 4 vectors of 8 values per thread at most (32768-value slabs)
    assert tts.Plan([128, 256, 2, 2], [1] * 5, 16, 1e-3, inner=True, fuse=True,
                    x_dtype="bf16").sketch_sources() == [0, 0, 0, 0]
    assert tts.Plan([200, 200, 3, 2], [1] * 5, 64, 1e-3, inner=True, fuse=True,
                    x_dtype="bf16").sketch_sources() == [0, 0, 2, 2]


def test_sketch_fusion_rule(tts):
    say("sketch fusion rule")
    # O_0 = n_2 ... n_{d-1} = 3600 outer tuples >= 4 J: fused by default
    assert tts.Plan([100, 10, 60, 60], [1, 1, 1, 1, 1], 500, 1e-3).sketch_sources() == [0, 0, 2, 3]
    # few outer tuples per bucket: every mode takes its own pass
    assert tts.Plan([16, 16, 16, 16], [1, 1, 1, 1, 1], 256, 1e-3).sketch_sources() == [0, 1, 2, 3]
    assert tts.Plan([100, 10, 60, 60], [1, 1, 1, 1, 1], 500, 1e-3, fuse=False).sketch_sources() == [0, 1, 2, 3]
    assert tts.Plan([30, 40], [1, 3, 1], 64, 1e-3, fuse=True).sketch_sources() == [0, 1]   # d = 2: no outer modes


def test_paper_example_via_gpu_sketch(tts):
    # Sec. 2.2 worked example: m = 2, two modes of size 2; a third mode of
    # size 1 plays the unsketched index, one-hot inputs read off S's columns.
    say("paper example")
    import json, os
    from tests.conftest import GOLDEN
    ex = json.load(open(os.path.join(GOLDEN, "paper_example_tensorsketch.json")))
    n = [2, 2, 1]
    plan = tts.Plan(n, [1, 1, 1, 1], 2, 1e-3, x_dtype="f32", work_dtype="f32")
    for s in range(2):
        plan.set_tables(s, np.array(ex["h_one_based"][s]) - 1, np.array(ex["v"][s]))
    plan.set_tables(2, np.array([0]), np.array([1]))
    S = np.zeros((2, 4))
    for j in range(4):
        X = torch.zeros(4, dtype=torch.float32, device=DEV)
        X[j] = 1.0
        S[:, j] = plan.sketch_tensor(X, 2).cpu().numpy()
    assert np.array_equal(S, np.array(ex["S"], dtype=float))


# ------------------------------------------------------------------ interface sketch
IFACE_CASES = [
    ([16, 16, 16, 16], [1, 3, 3, 3, 1], 256, "f64"),
    ([20, 9, 13, 7], [1, 4, 5, 3, 1], 120, "f32"),
    ([12, 10, 11], [1, 6, 5, 1], 3000, "f32"),
    ([9, 8], [1, 7, 1], 4000, "f32"),
    ([6, 5, 4, 5, 6], [1, 3, 4, 4, 3, 1], 210, "f64"),
    ([30, 30, 30], [1, 16, 11, 1], 210, "f32"),   # s = 176
    ([40, 30, 20], [1, 3, 2, 1], 8000, "f32"),     # J = 8000: 128 KB of LDS per FFT
]


@pytest.mark.parametrize("n,R,J,wd", IFACE_CASES)
def test_interface_sketch(tts, n, R, J, wd):
    say("interface", n, R, J, wd)
    cores = synth.random_cores(n, R, 7)
    plan = tts.Plan(n, R, J, 1e-3, seed=8, x_dtype=wd, work_dtype=wd)
    hs, vs = host_tables(plan)
    dc = [tts.core_to_device(c) for c in cores]
    tol = 1e-10 if wd == "f64" else 1e-5
    for k in range(len(n)):
        SH = plan.sketch_interface(dc, k).cpu().numpy().astype(np.float64).reshape(J, -1, order="F")
        ref = sketch.interface_cyclic(cores, k, hs, vs, J)
        assert rel(SH, ref) < tol, (k, rel(SH, ref))
        assert colmax(SH, ref) < tol, (k, colmax(SH, ref))


# ------------------------------------------------------------------ prox solve
@pytest.mark.parametrize("r0,nk,r1,J,wd,gram", [(3, 16, 3, 256, "f64", "work"), (10, 200, 10, 4000, "f32", "work"),
                                                (12, 37, 12, 500, "f32", "work"), (1, 50, 8, 64, "f64", "work"),
                                                (8, 64, 8, 3000, "f32", "bf16"), (13, 9, 13, 300, "f64", "work"),
                                                # s = 180, the largest system: 8 right-hand sides per block
                                                (12, 20, 15, 500, "f64", "work")])
def test_prox_solve(tts, r0, nk, r1, J, wd, gram):
    say("prox", r0, nk, r1, J, wd, gram)
    g = synth.rng(9)
    n = [r0, nk, r1]             # a 3-core problem whose middle core has this shape
    R = [1, r0, r1, 1]
    lam = 1e-2
    plan = tts.Plan(n, R, J, lam, x_dtype=wd, work_dtype=wd, gram=gram)
    s = r0 * r1
    SH = g.standard_normal((J, s)) / np.sqrt(J)
    Y = g.standard_normal((J, nk)) / np.sqrt(J)
    G = g.standard_normal((r0, nk, r1))
    tdt = torch.float64 if wd == "f64" else torch.float32
    SHd = torch.from_numpy(SH.reshape(-1, order="F").copy()).to(DEV, tdt)
    Yd = torch.from_numpy(Y.reshape(-1, order="F").copy()).to(DEV, tdt)
    SHo = SHd.cpu().double().numpy().reshape(J, s, order="F")
    Yo = Yd.cpu().double().numpy().reshape(J, nk, order="F")
    Gd = tts.core_to_device(G)
    out = tts.core_to_host(plan.prox_solve(1, SHd, Yd, Gd), G.shape)
    plan.sync_status()
    if gram == "bf16":
        # the oracle sees the same BF16-rounded operands; the FP32 accumulation
        # and the solve are compared at a BF16-scaled bound
        bf = lambda A: torch.from_numpy(A).float().bfloat16().double().numpy()
        ref = solve.prox_update(bf(SHo), bf(Yo), G, lam)
        tol = 1e-4
    else:
        # FP32 operands are contracted on the FP64 MFMA (exact products, FP64
        # sums), so the FP32 work type is held to the same 1e-5 as any FP32
        # result and in practice matches to FP64 rounding
        ref = solve.prox_update(SHo, Yo, G, lam)
        tol = 1e-11 if wd == "f64" else 1e-5
    print("prox rel %.3e colmax %.3e" % (rel(out, ref), colmax(solve.core_unfold2(out), solve.core_unfold2(ref))))
    assert rel(out, ref) < tol, rel(out, ref)
    assert colmax(solve.core_unfold2(out), solve.core_unfold2(ref)) < 10 * tol
    # aliasing G_old == G_new is allowed
    plan.prox_solve(1, SHd, Yd, Gd, Gd)
    assert rel(tts.core_to_host(Gd, G.shape), out) < 1e-14


def test_prox_not_spd_reported(tts):
    say("not spd")
    n, R, J = [2, 5, 2], [1, 2, 2, 1], 16
    plan = tts.Plan(n, R, J, 0.0, x_dtype="f32", work_dtype="f32")
    SH = torch.zeros(J * 4, dtype=torch.float32, device=DEV)
    Y = torch.zeros(J * 5, dtype=torch.float32, device=DEV)
    G = torch.zeros(20, dtype=torch.float64, device=DEV)
    plan.prox_solve(1, SH, Y, G)
    with pytest.raises(tts.TTError) as ei:
        plan.sync_status()
    assert ei.value.status == 5
    plan.sync_status()   # cleared


# ------------------------------------------------------------------ QR / orthogonalisation
@pytest.mark.parametrize("n,R", [([16, 16, 16, 16], [1, 3, 3, 3, 1]), ([200, 20, 7], [1, 10, 7, 1]),
                                 ([5, 4, 6, 3], [1, 5, 12, 3, 1]), ([3, 50, 40], [1, 3, 16, 1]),
                                 # register QR with 4 and 8 rows per thread (1600 and 2400 rows)
                                 ([4, 400, 6], [1, 4, 6, 1]),
                                 # 16 columns with 4 rows per thread; 4800 rows (global-memory QR)
                                 ([11, 120, 16], [1, 11, 16, 1]), ([2, 300, 16], [1, 2, 16, 1])])
def test_orthogonalisation(tts, n, R):
    say("orth", n, R)
    cores = synth.random_cores(n, R, 10)
    plan = tts.Plan(n, R, 16, 1e-3, x_dtype="f64", work_dtype="f64")
    dc = [tts.core_to_device(c) for c in cores]
    plan.right_orthogonalize(dc)
    ref = solve.right_orthogonalize(cores)
    for a, b in zip(dc, ref):
        assert rel(tts.core_to_host(a, b.shape), b) < 1e-12
    for k in range(len(n) - 1):
        plan.left_orth_absorb(dc, k)
        ref[k], ref[k + 1] = solve.left_orth_absorb(ref[k], ref[k + 1])
        for a, b in zip(dc, ref):
            assert rel(tts.core_to_host(a, b.shape), b) < 1e-12


def test_qr_zero_core_convention(tts):
    say("qr zeros")
    n, R = [4, 5, 3], [1, 3, 2, 1]
    cores = synth.zero_cores(n, R)
    plan = tts.Plan(n, R, 16, 1e-3, x_dtype="f64", work_dtype="f64")
    dc = [tts.core_to_device(c) for c in cores]
    plan.right_orthogonalize(dc)
    ref = solve.right_orthogonalize(cores)
    for a, b in zip(dc, ref):
        assert np.array_equal(tts.core_to_host(a, b.shape), b)


# ------------------------------------------------------------------ residual
@pytest.mark.parametrize("n,R,xd,wd", [([16, 16, 16, 16], [1, 3, 3, 3, 1], "f64", "f64"),
                                       ([40, 30, 20], [1, 5, 4, 1], "f32", "f32"),
                                       ([300, 12], [1, 9, 1], "f32", "f32"),
                                       ([64, 8, 8, 8], [1, 8, 8, 8, 1], "bf16", "f32")])
def test_residual(tts, n, R, xd, wd):
    say("residual", n, R, xd)
    Xh, _ = synth.tt_tensor_host(n, R, 0.05, 11)
    cores = synth.random_cores(n, R, 12)
    plan = tts.Plan(n, R, 16, 1e-3, x_dtype=xd, work_dtype=wd)
    X = to_dev_x(Xh, xd)
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))
    got = plan.residual(X, [tts.core_to_device(c) for c in cores])
    ref = als.rel_residual(Xo, cores)
    tol = 1e-12 if wd == "f64" else 1e-5
    assert abs(got - ref) / ref < tol, (got, ref)
    # exact TT: residual at round-off
    X2 = to_dev_x(als.tt_full(cores), xd)
    got2 = plan.residual(X2, [tts.core_to_device(c) for c in cores])
    assert got2 < (1e-13 if wd == "f64" else (5e-3 if xd == "bf16" else 1e-6))


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_residual_nonfinite_reported(tts, bad):
    say("residual nonfinite", bad)
    n, R = [12, 10, 8], [1, 3, 2, 1]
    Xh, _ = synth.tt_tensor_host(n, R, 0.05, 13)
    Xh[57] = bad
    cores = synth.random_cores(n, R, 14)
    plan = tts.Plan(n, R, 16, 1e-3, x_dtype="f32", work_dtype="f32")
    with pytest.raises(tts.TTError) as ei:
        plan.residual(to_dev_x(Xh, "f32"), [tts.core_to_device(c) for c in cores])
    assert ei.value.status == 6
    # a finite input afterwards is fine
    Xh[57] = 0.0
    assert np.isfinite(plan.residual(to_dev_x(Xh, "f32"), [tts.core_to_device(c) for c in cores]))


# ------------------------------------------------------------------ full sweeps
def _run_sweeps(tts, n, R, J, lam, seed, sweeps, xd, wd, noise, init_seed=2, gram="work", fuse=None, serial=False,
                inner=None):
    Xh, _ = synth.tt_tensor_host(n, R, noise, 1)
    init = synth.random_cores(n, R, init_seed)
    plan = tts.Plan(n, R, J, lam, seed=seed, x_dtype=xd, work_dtype=wd, gram=gram, fuse=fuse, serial=serial,
                    inner=inner)
    X = to_dev_x(Xh, xd)
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))
    dc = [tts.core_to_device(c) for c in init]
    ref = [c.copy() for c in init]
    res, res_o = [], []
    for t in range(sweeps):
        res.append(plan.als_sweep(X, dc, residual=True))
        ref = als.sweep(Xo, n, ref, J, lam, seed=seed, t=t, gram="bf16" if gram == "bf16" else "fp64")
        res_o.append(als.rel_residual(Xo, ref))
    return plan, dc, ref, res, res_o, Xo


def test_sweeps_c1_fp64(tts):
    # 16^4 FP64, ranks 3, J = 256, lambda = 1e-3, noise 1e-3, 5 sweeps
    say("sweeps C1")
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, [16] * 4, [1, 3, 3, 3, 1], 256, 1e-3, 17, 5, "f64", "f64", 1e-3)
    print("gpu", res, "\noracle", res_o)
    for a, b in zip(res, res_o):
        assert abs(a - b) < 1e-10
    got = [tts.core_to_host(c, r.shape) for c, r in zip(dc, ref)]
    assert rel(als.tt_full(got), als.tt_full(ref)) < 1e-9
    assert plan.get_sweep() == 5


def test_sweeps_fp32(tts):
    say("sweeps fp32")
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, [30, 20, 25, 10], [1, 4, 5, 3, 1], 500, 1e-3, 5, 4, "f32", "f32", 1e-2)
    print("gpu", res, "\noracle", res_o)
    assert abs(res[-1] - res_o[-1]) < 1e-4


def test_sweeps_fp32_key_grouped(tts):
    # 60 x 50 x 40 x 30 with J = 120: every k >= 1 sketch uses the key-grouped path
    say("sweeps fp32 key-grouped")
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, [60, 50, 40, 30], [1, 4, 5, 3, 1], 120, 1e-3, 6, 3, "f32", "f32",
                                                1e-2)
    print("gpu", res, "\noracle", res_o)
    assert abs(res[-1] - res_o[-1]) < 1e-4


def test_injective_sweep_is_exact_prox_als(tts):
    # h_s(i) = i prod_{t<s} n_t, v = +1, J = N: S^T S = I for every k.
    say("injective sweep")
    n, R, lam = [4, 5, 3], [1, 2, 3, 1], 0.1
    J = 60
    Xh = synth.rng(35).standard_normal(60)
    init = synth.random_cores(n, R, 36)
    plan = tts.Plan(n, R, J, lam, x_dtype="f64", work_dtype="f64")
    stride = 1
    hs, vs = [], []
    for s, ns in enumerate(n):
        hs.append(np.arange(ns) * stride)
        vs.append(np.ones(ns, dtype=np.int8))
        plan.set_tables(s, hs[-1], vs[-1])
        stride *= ns
    dc = [tts.core_to_device(c) for c in init]
    plan.als_sweep(torch.from_numpy(Xh).to(DEV), dc)
    ref = als.sweep(Xh, n, init, J, lam, tabs=(hs, vs))
    for a, b in zip(dc, ref):
        assert rel(tts.core_to_host(a, b.shape), b) < 1e-10


def test_overlapped_sweep_matches_serial(tts):
    # the data sketches on the side stream give the same sweep as the serial schedule
    say("overlap vs serial")
    n, R, J = [40, 30, 20, 12], [1, 5, 6, 4, 1], 600
    Xh, _ = synth.tt_tensor_host(n, R, 1e-2, 3)
    init = synth.random_cores(n, R, 4)
    X = to_dev_x(Xh, "f32")
    out = []
    for serial in (False, True):
        plan = tts.Plan(n, R, J, 1e-3, seed=9, x_dtype="f32", work_dtype="f32", serial=serial)
        dc = [tts.core_to_device(c) for c in init]
        for _ in range(3):
            plan.als_sweep(X, dc)
        res = plan.residual(X, dc)
        out.append(([tts.core_to_host(c, c0.shape) for c, c0 in zip(dc, init)], res))
    (a, ra), (b, rb) = out
    # equal up to FP32 rounding: LDS atomics sum in a run-dependent order and
    # three sweeps amplify last-bit differences of Y
    assert abs(ra - rb) < 1e-5 * ra
    assert rel(als.tt_full(a), als.tt_full(b)) < 1e-4


def test_sweeps_bf16_mixed_form(tts):
    # the precision form: X stored BF16, Gram and right-hand side on BF16 MFMA
    # with FP32 accumulation, Cholesky and QR in FP64.  Two oracles read the
    # same BF16 values of X: one forms the normal equations from BF16 copies
    # of SH and Y as the form does (the bar), the other stays FP64 throughout
    # (the error of the form, stated)
    say("sweeps bf16 mixed")
    n, R, J, lam, seed, T = [64, 8, 8, 8], [1, 8, 8, 8, 1], 3000, 1e-3, 21, 3
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, n, R, J, lam, seed, T, "bf16", "f32", 1e-3, gram="bf16")
    got = [tts.core_to_host(c, r.shape) for c, r in zip(dc, ref)]
    d_res = [abs(a - b) for a, b in zip(res, res_o)]
    d_tt = rel(als.tt_full(got), als.tt_full(ref))
    ref64 = synth.random_cores(n, R, 2)
    res64 = []
    for t in range(T):
        ref64 = als.sweep(Xo, n, ref64, J, lam, seed=seed, t=t)
        res64.append(als.rel_residual(Xo, ref64))
    d64 = [abs(a - b) / b for a, b in zip(res, res64)]
    d_tt64 = rel(als.tt_full(got), als.tt_full(ref64))
    print("mixed bf16: gpu", res, "\nbf16-gram oracle", res_o, "\n|dres|", d_res, "TT rel diff %.3e" % d_tt,
          "\nfp64 oracle", res64, "\nrel dres", d64, "TT rel diff %.3e" % d_tt64)
    assert max(d_res) < 1e-4 and max(r / o for r, o in zip(d_res, res_o)) < 1e-2, d_res
    assert d_tt < 1e-3, d_tt
    # against pure FP64: the BF16 rounding of SH and Y (2^-9) moves each
    # solve, and the residual near the noise floor by up to ~10 %
    assert max(d64) < 0.2 and d_tt64 < 1e-2, (d64, d_tt64)


def test_sweeps_fp32_elementwise(tts):
    # plain FP32 sweeps against the oracle, entry by entry on the final TT
    say("sweeps fp32 elementwise")
    n, R, J = [20, 15, 12, 10], [1, 3, 4, 3, 1], 400
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, n, R, J, 1e-3, 22, 3, "f32", "f32", 1e-2)
    got = [tts.core_to_host(c, r.shape) for c, r in zip(dc, ref)]
    T, To = als.tt_full(got), als.tt_full(ref)
    print("fp32: |dres|", [abs(a - b) for a, b in zip(res, res_o)], "TT rel %.3e max %.3e" %
          (rel(T, To), np.abs(T - To).max() / np.abs(To).max()))
    assert max(abs(a - b) for a, b in zip(res, res_o)) < 1e-4
    assert np.abs(T - To).max() <= 1e-3 * np.abs(To).max()


def test_video_shaped_steps(tts):
    # the smooth video-shaped workload 240 x 320 x 3 x 100 (sum of 20
    # separable sinusoid products plus 1e-2 noise), TT ranks 12, J = 3000:
    # sampled columns of every data sketch, the interface sketch and one
    # proximal step of the middle core (s = 144) against the oracle
    say("video-shaped steps")
    n, R, J, lam = [240, 320, 3, 100], [1, 12, 12, 12, 1], 3000, 1e-3
    Xh = synth.sinusoid_tensor_host(n, 20, 1e-2, 5)
    X = to_dev_x(Xh, "f32")
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, "f32"))
    plan = tts.Plan(n, R, J, lam, seed=31, x_dtype="f32", work_dtype="f32")
    hs, vs = host_tables(plan)
    T = Xo.reshape(n[::-1])            # axes (i_3, i_2, i_1, i_0)
    g = synth.rng(32)
    for k in range(4):
        Y = plan.sketch_tensor(X, k).cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        for c in g.choice(n[k], 2, replace=False):
            sub = np.take(T, c, axis=3 - k)          # the sub-tensor with i_k = c
            others = [s for s in range(4) if s != k]
            # a trailing mode of size 1 plays the unsketched index of the sub-tensor
            want = sketch.data_sketch(np.ascontiguousarray(sub).reshape(-1), [n[s] for s in others] + [1], 3,
                                      [hs[s] for s in others] + [np.zeros(1, int)],
                                      [vs[s] for s in others] + [np.ones(1, int)], J)[:, 0]
            assert rel(Y[:, c], want) < 1e-5 and colmax(Y[:, c], want) < 1e-5, (k, c)
    cores = synth.random_cores(n, R, 33)
    dc = [tts.core_to_device(c) for c in cores]
    k = 1
    SH = plan.sketch_interface(dc, k)
    SHh = SH.cpu().numpy().astype(np.float64).reshape(J, -1, order="F")
    ref = sketch.interface_cyclic(cores, k, hs, vs, J)
    assert rel(SHh, ref) < 1e-5 and colmax(SHh, ref) < 1e-5, (rel(SHh, ref), colmax(SHh, ref))
    Yk = plan.sketch_tensor(X, k)
    Yh = Yk.cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
    out = tts.core_to_host(plan.prox_solve(k, SH, Yk, dc[k]), cores[k].shape)
    plan.sync_status()
    want = solve.prox_update(SHh, Yh, cores[k], lam)
    print("video prox rel %.3e colmax %.3e" % (rel(out, want), colmax(solve.core_unfold2(out), solve.core_unfold2(want))))
    assert rel(out, want) < 1e-5


@pytest.mark.parametrize("serial", [False, True])
def test_sweeps_inner_sketch(tts, serial):
    # sweeps whose Y_k, k >= 2, come from the inner sketch (with and without
    # the outer sketch for Y_1), in both schedules, against the oracle's passes
    say("sweeps inner serial=%s" % serial)
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, [16] * 4, [1, 3, 3, 3, 1], 256, 1e-3, 17, 4, "f64", "f64", 1e-3,
                                                fuse=True, serial=serial, inner=True)
    assert plan.sketch_sources() == [0, 0, 2, 2]
    assert max(abs(a - b) for a, b in zip(res, res_o)) < 1e-10
    got = [tts.core_to_host(c, r.shape) for c, r in zip(dc, ref)]
    assert rel(als.tt_full(got), als.tt_full(ref)) < 1e-9
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, [30, 20, 25, 10], [1, 4, 5, 3, 1], 500, 1e-3, 5, 3, "f32", "f32",
                                                1e-2, fuse=False, serial=serial, inner=True)
    assert plan.sketch_sources() == [0, 1, 2, 2]
    assert max(abs(a - b) for a, b in zip(res, res_o)) < 1e-4
    # modes 0..2 in the inner sketch, mode 2 its own pass
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, [12, 10, 8, 9, 7], [1, 3, 4, 4, 3, 1], 300, 1e-3, 8, 3, "f32",
                                                "f32", 1e-2, serial=serial, inner=True, fuse=False)
    assert plan.sketch_sources()[2:] == [2, 3, 3]
    assert max(abs(a - b) for a, b in zip(res, res_o)) < 1e-4
    # both intermediates from the k = 0 pass (one pass over X per sweep)
    for n, R in (([40, 20, 6, 5], [1, 4, 5, 3, 1]), ([40, 30, 3, 3, 2], [1, 3, 3, 3, 2, 1])):
        plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, n, R, 200, 1e-3, 8, 3, "f32", "f32", 1e-2, serial=serial,
                                                    inner=True, fuse=True)
        assert plan.sketch_sources() == [0] * len(n)
        assert max(abs(a - b) for a, b in zip(res, res_o)) < 1e-4
        got = [tts.core_to_host(c, r.shape) for c, r in zip(dc, ref)]
        assert rel(als.tt_full(got), als.tt_full(ref)) < 1e-3


@pytest.mark.parametrize("serial", [False, True])
def test_sweeps_fused_sketches(tts, serial):
    # sweeps whose Y_1 comes from the outer sketch of the k = 0 pass, in the
    # overlapped and the serial schedule, against the oracle's passes
    say("sweeps fused serial=%s" % serial)
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, [16] * 4, [1, 3, 3, 3, 1], 256, 1e-3, 17, 4, "f64", "f64", 1e-3,
                                                fuse=True, serial=serial)
    assert plan.sketch_sources()[1] == 0
    assert max(abs(a - b) for a, b in zip(res, res_o)) < 1e-10
    got = [tts.core_to_host(c, r.shape) for c, r in zip(dc, ref)]
    assert rel(als.tt_full(got), als.tt_full(ref)) < 1e-9
    plan, dc, ref, res, res_o, Xo = _run_sweeps(tts, [30, 20, 25, 10], [1, 4, 5, 3, 1], 500, 1e-3, 5, 3, "f32", "f32",
                                                1e-2, fuse=True, serial=serial)
    assert max(abs(a - b) for a, b in zip(res, res_o)) < 1e-4
