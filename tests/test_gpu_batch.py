"""GPU tests of the batched form: the one-launch-per-step data sketch against
the oracle, batched sweeps against single-problem sweeps with the same
tables, hipGraph replays against eager sweeps, and the autotuner."""
import numpy as np
import pytest

from oracle import als, sketch, tables

pytestmark = pytest.mark.gpu

PROBLEMS = [
    dict(n=[9, 12, 7], ranks=[1, 3, 4, 1], J=96, seed=101),
    dict(n=[20, 8, 11, 6], ranks=[1, 4, 5, 3, 1], J=128, seed=102),
    dict(n=[33, 5, 9, 7, 6], ranks=[1, 3, 4, 4, 2, 1], J=128, seed=103),
    dict(n=[64, 10, 12], ranks=[1, 5, 6, 1], J=120, seed=104),
    dict(n=[5, 30, 4, 9], ranks=[1, 2, 3, 2, 1], J=64, seed=105),
    dict(n=[17, 6, 5, 8, 4], ranks=[1, 2, 2, 3, 2, 1], J=128, seed=106),
]


# the slab-step kernels: rows in memory order, or slabs in key order
SLAB_KERNELS = ("k_bsketch_slab", "k_bsketch_ks")


def say(msg):
    print("[case] " + msg, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2309_08093_amd as tts
    return torch, tts


def make_inputs(torch, problems, integer=False, noise=1e-3):
    import synth
    Xs, Xh = [], []
    for i, p in enumerate(problems):
        N = int(np.prod(p["n"]))
        if integer:
            x = np.random.default_rng(500 + i).integers(-8, 9, size=N).astype(np.float64)
        else:
            x, _ = synth.tt_tensor_host(p["n"], p["ranks"], noise, 600 + i)
            x = x.astype(np.float32).astype(np.float64)
        Xh.append(x)
        Xs.append(torch.from_numpy(x.astype(np.float32)).cuda())
    return Xs, Xh


@pytest.mark.parametrize("integer", [True, False])
def test_batched_sketch_matches_oracle(env, integer):
    torch, tts = env
    say("batched sketch integer=%s" % integer)
    b = tts.Batch(PROBLEMS)
    Xs, Xh = make_inputs(torch, PROBLEMS, integer)
    for k in range(5):
        Ys = b.sketch_tensor(Xs, k)
        torch.cuda.synchronize()
        for i, p in enumerate(PROBLEMS):
            d = len(p["n"])
            if d <= k:
                assert Ys[i] is None
                continue
            hs, vs = zip(*[b.plan_tables(i, s) for s in range(d)])
            want = sketch.data_sketch(Xh[i], p["n"], k, hs, vs, p["J"])
            got = Ys[i].cpu().numpy().astype(np.float64).reshape(want.shape, order="F")
            if integer:
                np.testing.assert_array_equal(got, want)
            else:
                assert np.linalg.norm(got - want) <= 1e-5 * np.linalg.norm(want)


# batches whose longest mode-0 fibre takes 2 and 4 entries per lane; batches
# whose k >= 2 steps run on slabs shorter than a wave (a lane steps over
# several slabs per row), and whose largest slab table does not fit in LDS
# (those steps run on fibres)
WIDE = {
    "tiny slabs": [dict(n=[3, 2, 5, 4], ranks=[1, 2, 2, 2, 1], J=40, seed=116),
                   dict(n=[2, 2, 3, 5, 3], ranks=[1, 2, 2, 2, 2, 1], J=50, seed=117),
                   dict(n=[7, 9, 4], ranks=[1, 3, 2, 1], J=32, seed=118)],
    "large slabs": [dict(n=[130, 100, 3], ranks=[1, 3, 2, 1], J=64, seed=119),
                    dict(n=[10, 10, 4, 3], ranks=[1, 2, 3, 2, 1], J=48, seed=120)],
    "n0<=128": [dict(n=[100, 6, 7], ranks=[1, 4, 5, 1], J=90, seed=111),
                dict(n=[40, 5, 4, 3], ranks=[1, 3, 3, 2, 1], J=64, seed=112)],
    "n0<=256": [dict(n=[200, 5, 4, 3], ranks=[1, 4, 3, 2, 1], J=150, seed=113),
                dict(n=[129, 7, 6], ranks=[1, 3, 4, 1], J=128, seed=114),
                dict(n=[9, 10, 11], ranks=[1, 3, 3, 1], J=72, seed=115)],
}


@pytest.mark.parametrize("which", sorted(WIDE))
def test_batched_sketch_wide_fibres(env, which):
    torch, tts = env
    say("batched sketch, wide fibres %s" % which)
    probs = WIDE[which]
    b = tts.Batch(probs)
    Xs, Xh = make_inputs(torch, probs, integer=True)
    for k in range(max(len(p["n"]) for p in probs)):
        # slabs (key-sorted by default) for k >= 2 unless a participating
        # problem's slab table does not fit in LDS (n = [130, 100, 3] at k = 2)
        want_kernel = "k_bsketch_0" if k == 0 else \
            "k_bsketch_ks" if k >= 2 and (which, k) != ("large slabs", 2) else "k_bsketch_k"
        assert b.sketch_kernel(k) == want_kernel, (k, b.sketch_kernel(k))
        Ys = b.sketch_tensor(Xs, k)
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            d = len(p["n"])
            if d <= k:
                assert Ys[i] is None
                continue
            hs, vs = zip(*[b.plan_tables(i, s) for s in range(d)])
            want = sketch.data_sketch(Xh[i], p["n"], k, hs, vs, p["J"])
            got = Ys[i].cpu().numpy().astype(np.float64).reshape(want.shape, order="F")
            np.testing.assert_array_equal(got, want)


def test_sketch_path_rejects_steps_outside_the_batch(env):
    torch, tts = env
    say("batch sketch path arguments")
    b = tts.Batch(PROBLEMS)
    assert [b.sketch_kernel(k) for k in range(5)][:2] == ["k_bsketch_0", "k_bsketch_k"]
    for k in (-1, 5):
        with pytest.raises(tts.TTError):
            b.sketch_kernel(k)


def test_tables_are_the_plans_tables(env):
    torch, tts = env
    say("batch tables")
    b = tts.Batch(PROBLEMS)
    for i, p in enumerate(PROBLEMS):
        for s in range(len(p["n"])):
            h, v = b.plan_tables(i, s)
            ho, vo = tables.mode_tables(p["seed"], 0, s, p["n"][s], p["J"])
            np.testing.assert_array_equal(h, ho)
            np.testing.assert_array_equal(v, vo)


def _cores(torch, tts, problems, seed):
    import synth
    return [[tts.core_to_device(c, "cuda") for c in synth.random_cores(p["n"], p["ranks"], seed + i)]
            for i, p in enumerate(problems)]


def _tt(tts, cores, p):
    return als.tt_full([tts.core_to_host(c, (p["ranks"][k], p["n"][k], p["ranks"][k + 1]))
                        for k, c in enumerate(cores)])


def test_batched_sweep_matches_single_plans(env):
    torch, tts = env
    say("batched sweep vs single plans")
    Xs, Xh = make_inputs(torch, PROBLEMS)
    b = tts.Batch(PROBLEMS)
    cb = _cores(torch, tts, PROBLEMS, 40)
    for _ in range(2):
        b.sweep(Xs, cb)
    res_b = b.sweep(Xs, cb, residuals=True)
    for i, p in enumerate(PROBLEMS):
        plan = tts.Plan(p["n"], p["ranks"], p["J"], 1e-3, seed=p["seed"], serial=True)
        cs = _cores(torch, tts, [p], 40 + i)[0]
        for _ in range(2):
            plan.als_sweep(Xs[i], cs)
        r = plan.als_sweep(Xs[i], cs, residual=True)
        # same tables and steps; the two k = 0 kernels add bucket contributions
        # in different orders in FP32, which three sweeps carry into the cores
        assert abs(res_b[i] - r) <= 1e-4 * r + 1e-9
        Tb, Ts = _tt(tts, cb[i], p), _tt(tts, cs, p)
        assert np.linalg.norm(Tb - Ts) <= 1e-4 * np.linalg.norm(Ts)
        assert res_b[i] == pytest.approx(als.rel_residual(Xh[i], [tts.core_to_host(
            c, (p["ranks"][k], p["n"][k], p["ranks"][k + 1])) for k, c in enumerate(cb[i])]), rel=1e-4)


# the problems above plus an order-5 problem of rank 2 and one whose k = 1 QR
# (8 x 300 = 2400 rows) takes the per-problem QR launch instead of a batched
# register-QR class
ORACLE_PROBLEMS = PROBLEMS + [
    dict(n=[6, 5, 4, 5, 6], ranks=[1, 2, 2, 2, 2, 1], J=96, seed=107),
    dict(n=[10, 300, 6], ranks=[1, 8, 6, 1], J=128, seed=108),
]


def test_batched_sweeps_match_oracle(env):
    """Three batched sweeps (interface FFTs, chains, Gram, Cholesky,
    substitution, QR and absorb of every problem in shared launches) against
    the FP64 oracle's Algorithm 1 passes from the same starting cores, with
    the tables the oracle derives from each problem's seed and sweep index."""
    import synth
    torch, tts = env
    say("batched sweeps vs oracle")
    probs = ORACLE_PROBLEMS
    Xs, Xh = make_inputs(torch, probs)
    b = tts.Batch(probs)
    init = [synth.random_cores(p["n"], p["ranks"], 90 + i) for i, p in enumerate(probs)]
    cb = [[tts.core_to_device(c, "cuda") for c in cs] for cs in init]
    ref = [[c.copy() for c in cs] for cs in init]
    for t in range(3):
        res_b = b.sweep(Xs, cb, residuals=True)
        for i, p in enumerate(probs):
            ref[i] = als.sweep(Xh[i], p["n"], ref[i], p["J"], 1e-3, seed=p["seed"], t=t)
            r_o = als.rel_residual(Xh[i], ref[i])
            Tb, To = _tt(tts, cb[i], p), als.tt_full(ref[i])
            d_tt = np.linalg.norm(Tb - To) / np.linalg.norm(To)
            print("sweep %d problem %d: residual %.6e oracle %.6e, TT rel diff %.2e" % (t, i, res_b[i], r_o, d_tt))
            assert abs(res_b[i] - r_o) < 1e-4, (t, i, res_b[i], r_o)
            assert d_tt < 1e-4, (t, i, d_tt)


def test_graph_replays_match_eager_sweeps(env):
    """Every replay of the captured sweep is checked against the eager sweep of
    the same index, with eager work and synchronisations in between; the
    tables advance with the device sweep counter."""
    torch, tts = env
    say("graph replays")
    Xs, _ = make_inputs(torch, PROBLEMS)
    be = tts.Batch(PROBLEMS)
    ce = _cores(torch, tts, PROBLEMS, 70)
    bg = tts.Batch(PROBLEMS)
    bg.set_graph(True)
    cg = _cores(torch, tts, PROBLEMS, 70)
    for t in range(4):
        be.sweep(Xs, ce)
        bg.sweep(Xs, cg)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum().item()     # eager work between replays
        assert np.isfinite(junk)
        for i, p in enumerate(PROBLEMS):
            Te, Tg = _tt(tts, ce[i], p), _tt(tts, cg[i], p)
            assert np.linalg.norm(Te - Tg) <= 1e-4 * np.linalg.norm(Te), (t, i)
    for i, p in enumerate(PROBLEMS):
        h, v = bg.plan_tables(i, 1)
        ho, vo = tables.mode_tables(p["seed"], 4, 1, p["n"][1], p["J"])
        np.testing.assert_array_equal(h, ho)
        np.testing.assert_array_equal(v, vo)


def test_autotune_keeps_results(env):
    torch, tts = env
    say("autotune")
    Xs, _ = make_inputs(torch, PROBLEMS, integer=True)
    b = tts.Batch(PROBLEMS)
    before = [b.sketch_tensor(Xs, k) for k in range(5)]
    chosen = b.autotune(Xs, reps=2)
    assert chosen[0] == 0 and all(c > 0 for c in chosen[1:])
    after = [b.sketch_tensor(Xs, k) for k in range(5)]
    for k in range(5):
        for y0, y1 in zip(before[k], after[k]):
            if y0 is not None:
                assert torch.equal(y0, y1)


def _tuning_with(b, **kw):
    """The batch's tuning with kw applied; fibres_in_flight (8 or 16) maps to
    4 or 8 at k = 0 and on slab steps, whose kernels take those."""
    steps = b.get_tuning()
    for k, st in enumerate(steps):
        st.update(kw)
        if "fibres_in_flight" in kw and (k == 0 or b.sketch_kernel(k) in SLAB_KERNELS):
            st["fibres_in_flight"] = kw["fibres_in_flight"] // 2
    steps[0]["workgroups"] = 0
    return steps


@pytest.mark.parametrize("which", ["default", "n0<=256"])
def test_every_tuned_shape_gives_the_oracle_sketch(env, which):
    """Every (entries per lane, fibres in flight) shape the autotuner can pick
    computes the same sketches, integer-exact against the oracle."""
    torch, tts = env
    probs = PROBLEMS if which == "default" else WIDE[which]
    say("tuned shapes %s" % which)
    b = tts.Batch(probs)
    Xs, Xh = make_inputs(torch, probs, integer=True)
    njs = (2, 4) if max(p["n"][0] for p in probs) <= 128 else (4,)
    dmax = max(len(p["n"]) for p in probs)
    for nj in njs:
        for fib in (8, 16):
            b.set_tuning(_tuning_with(b, entries_per_lane=nj, fibres_in_flight=fib))
            for k in range(dmax):
                Ys = b.sketch_tensor(Xs, k)
                torch.cuda.synchronize()
                for i, p in enumerate(probs):
                    if len(p["n"]) <= k:
                        continue
                    hs, vs = zip(*[b.plan_tables(i, s) for s in range(len(p["n"]))])
                    want = sketch.data_sketch(Xh[i], p["n"], k, hs, vs, p["J"])
                    got = Ys[i].cpu().numpy().astype(np.float64).reshape(want.shape, order="F")
                    np.testing.assert_array_equal(got, want, err_msg="nj=%d fib=%d k=%d" % (nj, fib, k))


def test_set_tuning_rejects_bad_values(env):
    torch, tts = env
    say("set_tuning arguments")
    b = tts.Batch(WIDE["n0<=256"])          # n_0 = 200: two entries per lane cannot cover a fibre
    before = b.get_tuning()
    for bad in (dict(entries_per_lane=2), dict(entries_per_lane=3), dict(fibres_in_flight=12),
                dict(gram_kchunk=300), dict(gram_kchunk=16384), dict(workgroups=1 << 20)):
        steps = _tuning_with(b, **bad)
        with pytest.raises(tts.TTError) as ei:
            b.set_tuning(steps)
        assert ei.value.status == 1, bad          # TT_ERR_ARG
        assert b.get_tuning() == before, bad      # unchanged


def test_gram_kchunk_and_tuning_keep_sweeps(env):
    """Sweeps under another tuning (Gram K-chunk 1024, 4 entries per lane, 8
    fibres in flight, twice the workgroups) match the default tuning's: only
    the order of FP64 partial sums changes."""
    import synth
    torch, tts = env
    say("tuning keeps sweeps")
    Xs, _ = make_inputs(torch, PROBLEMS)
    ba, bb = tts.Batch(PROBLEMS), tts.Batch(PROBLEMS)
    steps = _tuning_with(bb, gram_kchunk=1024, entries_per_lane=4, fibres_in_flight=8)
    for k in range(1, len(steps)):
        steps[k]["workgroups"] = 2 * 256
    bb.set_tuning(steps)
    assert [st["gram_kchunk"] for st in bb.get_tuning()] == [1024] * len(steps)
    init = [synth.random_cores(p["n"], p["ranks"], 40 + i) for i, p in enumerate(PROBLEMS)]
    ca = [[tts.core_to_device(c) for c in cs] for cs in init]
    cb = [[tts.core_to_device(c) for c in cs] for cs in init]
    for t in range(3):
        ra = ba.sweep(Xs, ca, residuals=True)
        rb = bb.sweep(Xs, cb, residuals=True)
        np.testing.assert_allclose(rb, ra, rtol=1e-5)
    for i, p in enumerate(PROBLEMS):
        Ta = als.tt_full([tts.core_to_host(c, g.shape) for c, g in zip(ca[i], init[i])])
        Tb = als.tt_full([tts.core_to_host(c, g.shape) for c, g in zip(cb[i], init[i])])
        assert np.linalg.norm(Ta - Tb) <= 1e-5 * np.linalg.norm(Ta), i


def test_autotune_persists_its_choices(env, tmp_path):
    """A tuning written to the cache file is taken back by a new batch of
    the same problems, which then skips the timing."""
    torch, tts = env
    say("autotune cache")
    Xs, _ = make_inputs(torch, PROBLEMS, integer=True)
    cache = str(tmp_path / "tune.json")
    b1 = tts.Batch(PROBLEMS)
    w1 = b1.autotune(Xs, reps=1, cache=cache)
    assert not b1.tuned_from_cache
    b2 = tts.Batch(PROBLEMS)
    w2 = b2.autotune(Xs, reps=1, cache=cache)
    assert b2.tuned_from_cache and w2 == w1 and b2.get_tuning() == b1.get_tuning()
    for k, st in enumerate(b1.get_tuning()):
        slab = b1.sketch_kernel(k) in SLAB_KERNELS
        allowed = (4, 8) if k == 0 else (1, 2, 4, 8) if slab else (8, 16)
        assert st["gram_kchunk"] in (256, 512, 1024) and st["fibres_in_flight"] in allowed
    # another batch (other problems) does not match the stored keys
    b3 = tts.Batch(PROBLEMS[:3])
    b3.autotune(Xs[:3], reps=1, cache=cache)
    assert not b3.tuned_from_cache


# problems whose plans take Y_1 from the outer sketch of the k = 0 step
# (J n_0 n_1 <= N / 4: the outer sketch is small beside X), mixed with one
# that does not
FUSED = [dict(n=[8, 6, 10, 10, 12], ranks=[1, 3, 4, 4, 3, 1], J=64, seed=131),
         dict(n=[20, 10, 30, 40], ranks=[1, 4, 5, 4, 1], J=128, seed=132),
         dict(n=[10, 8, 600], ranks=[1, 4, 3, 1], J=96, seed=133),
         dict(n=[9, 12, 7], ranks=[1, 3, 4, 1], J=96, seed=134)]


def test_batched_outer_sketch_gives_the_oracle_sketches(env):
    """Step 0 writes the outer sketch of the large problems and step 1 takes
    their Y_1 from it (the other problems keep the fibre launch): every Y_k
    integer-exact against the oracle, step 1 also asked for alone."""
    torch, tts = env
    say("batched outer sketch")
    # the first three take Y_1 from the outer sketch (source of Y_1 = mode 0), the last does not
    srcs = [tts.Plan(p["n"], p["ranks"], p["J"], 1e-3).sketch_sources()[1] for p in FUSED]
    assert srcs == [0, 0, 0, 1], srcs
    b = tts.Batch(FUSED)
    Xs, Xh = make_inputs(torch, FUSED, integer=True)
    for order in ([1, 0, 2, 3, 4], [0, 1, 2, 3, 4]):
        for k in order:
            Ys = b.sketch_tensor(Xs, k)
            torch.cuda.synchronize()
            for i, p in enumerate(FUSED):
                if len(p["n"]) <= k:
                    continue
                hs, vs = zip(*[b.plan_tables(i, s) for s in range(len(p["n"]))])
                want = sketch.data_sketch(Xh[i], p["n"], k, hs, vs, p["J"])
                got = Ys[i].cpu().numpy().astype(np.float64).reshape(want.shape, order="F")
                np.testing.assert_array_equal(got, want, err_msg="k=%d problem %d" % (k, i))


def test_batched_sweeps_with_outer_sketch_match_oracle(env):
    import synth
    torch, tts = env
    say("batched sweeps with outer sketch vs oracle")
    Xs, Xh = make_inputs(torch, FUSED)
    b = tts.Batch(FUSED)
    init = [synth.random_cores(p["n"], p["ranks"], 140 + i) for i, p in enumerate(FUSED)]
    cb = [[tts.core_to_device(c) for c in cs] for cs in init]
    ref = [[c.copy() for c in cs] for cs in init]
    for t in range(3):
        res = b.sweep(Xs, cb, residuals=True)
        for i, p in enumerate(FUSED):
            ref[i] = als.sweep(Xh[i], p["n"], ref[i], p["J"], 1e-3, seed=p["seed"], t=t)
            ro = als.rel_residual(Xh[i], ref[i])
            Tb, To = _tt(tts, cb[i], p), als.tt_full(ref[i])
            d_tt = np.linalg.norm(Tb - To) / np.linalg.norm(To)
            print("sweep %d problem %d: residual %.6e oracle %.6e, TT rel diff %.2e" % (t, i, res[i], ro, d_tt))
            assert abs(res[i] - ro) < 1e-4 and d_tt < 1e-4, (t, i)


def test_graph_replays_with_outer_sketch(env):
    torch, tts = env
    say("graph replays with outer sketch")
    Xs, _ = make_inputs(torch, FUSED)
    be, bg = tts.Batch(FUSED), tts.Batch(FUSED)
    bg.set_graph(True)
    ce, cg = _cores(torch, tts, FUSED, 150), _cores(torch, tts, FUSED, 150)
    for t in range(3):
        be.sweep(Xs, ce)
        bg.sweep(Xs, cg)
        torch.cuda.synchronize()
        for i, p in enumerate(FUSED):
            Te, Tg = _tt(tts, ce[i], p), _tt(tts, cg[i], p)
            assert np.linalg.norm(Te - Tg) <= 1e-6 * np.linalg.norm(Te), (t, i)


# outer-sketch problems whose slabs take each load width of the k = 0 pass:
# n_0 n_1 = 63 (odd: single values), 42 (even: pairs), 48 (four-value vectors)
WIDTHS = [dict(n=[7, 9, 10, 10, 12], ranks=[1, 3, 4, 4, 3, 1], J=64, seed=161),
          dict(n=[6, 7, 12, 10, 9], ranks=[1, 3, 4, 4, 3, 1], J=64, seed=162),
          dict(n=[8, 6, 10, 10, 12], ranks=[1, 3, 4, 4, 3, 1], J=64, seed=163)]


# outer-sketch problems whose slabs are longer than one piece of the k = 0
# pass (n_0 n_1 = 4800 in 4-value loads, 4331 in single values)
LONG_OUTER = [dict(n=[80, 60, 8, 8, 8], ranks=[1, 3, 4, 4, 3, 1], J=64, seed=181),
              dict(n=[71, 61, 8, 8, 8], ranks=[1, 3, 4, 4, 3, 1], J=64, seed=182)]


@pytest.mark.parametrize("which", ["widths", "long slabs"])
@pytest.mark.parametrize("shift", [0, 1, 2])
def test_outer_sketch_every_load_width(env, which, shift):
    """Every Y_k integer-exact against the oracle for slabs of odd, even and
    multiple-of-four size and slabs longer than one piece, with X at an
    aligned address and at 1 and 2 values past one (narrower loads for the
    same problems)."""
    torch, tts = env
    probs = WIDTHS if which == "widths" else LONG_OUTER
    say("outer sketch load widths %s, X shifted by %d values" % (which, shift))
    srcs = [tts.Plan(p["n"], p["ranks"], p["J"], 1e-3).sketch_sources()[1] for p in probs]
    assert srcs == [0] * len(probs), srcs
    b = tts.Batch(probs)
    Xs0, Xh = make_inputs(torch, probs, integer=True)
    Xs = []
    for x in Xs0:   # the same values at an address shift * 4 bytes past a 256-byte boundary
        buf = torch.empty(x.numel() + shift, dtype=x.dtype, device=x.device)
        buf[shift:] = x
        Xs.append(buf[shift:])
    for k in (0, 1, 2, 3, 4):
        Ys = b.sketch_tensor(Xs, k)
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            hs, vs = zip(*[b.plan_tables(i, s) for s in range(len(p["n"]))])
            want = sketch.data_sketch(Xh[i], p["n"], k, hs, vs, p["J"])
            got = Ys[i].cpu().numpy().astype(np.float64).reshape(want.shape, order="F")
            np.testing.assert_array_equal(got, want, err_msg="k=%d problem %d shift %d" % (k, i, shift))


# slab steps with slabs longer than one piece of the key-sorted kernel
# (n_0 n_1 = 5000 > 4096 values) beside short ones
LONG_SLABS = [dict(n=[100, 50, 6, 5], ranks=[1, 3, 4, 3, 1], J=64, seed=171),
              dict(n=[9, 7, 8, 6, 5], ranks=[1, 2, 3, 3, 2, 1], J=96, seed=172)]


@pytest.mark.parametrize("which", ["default", "widths", "long slabs"])
@pytest.mark.parametrize("slabs", [1, 2])
def test_key_sorted_slab_steps_give_the_oracle_sketch(env, which, slabs):
    """The key-sorted slab kernel (slab steps with 1 or 2 slabs per group in
    flight) integer-exact against the oracle, for slabs of odd, even and
    multiple-of-four size with X shifted off 16-byte alignment, and for slabs
    longer than one piece."""
    torch, tts = env
    probs = {"default": PROBLEMS, "widths": WIDTHS, "long slabs": LONG_SLABS}[which]
    say("key-sorted slabs %s, %d per group" % (which, slabs))
    b = tts.Batch(probs)
    Xs0, Xh = make_inputs(torch, probs, integer=True)
    Xs = []
    for x in Xs0:   # one value past a 256-byte boundary for half of the problems
        shift = len(Xs) % 2
        buf = torch.empty(x.numel() + shift, dtype=x.dtype, device=x.device)
        buf[shift:] = x
        Xs.append(buf[shift:])
    steps = b.get_tuning()
    dmax = max(len(p["n"]) for p in probs)
    for k in range(2, dmax):
        assert b.sketch_kernel(k) in SLAB_KERNELS, k
        steps[k]["fibres_in_flight"] = slabs
    steps[0]["workgroups"] = 0
    b.set_tuning(steps)
    assert all(b.get_tuning()[k]["fibres_in_flight"] == slabs for k in range(2, dmax))
    assert all(b.sketch_kernel(k) == "k_bsketch_ks" for k in range(2, dmax))
    for k in range(dmax):
        Ys = b.sketch_tensor(Xs, k)
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            if len(p["n"]) <= k:
                continue
            hs, vs = zip(*[b.plan_tables(i, s) for s in range(len(p["n"]))])
            want = sketch.data_sketch(Xh[i], p["n"], k, hs, vs, p["J"])
            got = Ys[i].cpu().numpy().astype(np.float64).reshape(want.shape, order="F")
            np.testing.assert_array_equal(got, want, err_msg="k=%d problem %d" % (k, i))
