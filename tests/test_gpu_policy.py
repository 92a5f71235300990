"""GPU parity of the sketch-size policy kernels (forward, backpropagation,
Adam) against the FP64 oracle, and of the policy-driven run loop."""
import math
import time

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu

F, H, O = 8, 64, 2


def say(msg):
    print("[case] " + msg, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2309_08093_amd as tts
    from paper_2309_08093_amd import jpolicy
    return torch, tts, jpolicy


def rand_inputs(seed, B, scale=1.0):
    g = np.random.default_rng(seed)
    return (g.standard_normal((B, F)) * scale).astype(np.float32), g.standard_normal((B, O)).astype(np.float32)


@pytest.mark.parametrize("B", [1, 63, 64, 200, 1000])
def test_forward_matches_oracle(env, B):
    torch, tts, jpolicy = env
    say("forward B=%d" % B)
    pol = jpolicy.Policy(seed=B)
    X, _ = rand_inputs(B + 1, B)
    Y = pol.forward(X).cpu().numpy()
    theta = pol.params.cpu().numpy().astype(np.float64)
    Yo, _ = mlp.forward(theta, X.astype(np.float64), F, H, O)
    assert np.linalg.norm(Y - Yo) <= 1e-5 * np.linalg.norm(Yo)


@pytest.mark.parametrize("B", [1, 64, 130, 4096])
def test_gradient_matches_oracle(env, B):
    torch, tts, jpolicy = env
    say("loss_grad B=%d" % B)
    pol = jpolicy.Policy(seed=3 * B)
    X, T = rand_inputs(B + 7, B)
    loss, g = pol.loss_grad(X, T)
    theta = pol.params.cpu().numpy().astype(np.float64)
    Lo, go = mlp.loss_grad(theta, X.astype(np.float64), T.astype(np.float64), F, H, O)
    g = g.cpu().numpy()
    assert float(loss.item()) == pytest.approx(Lo, rel=1e-5)
    assert np.linalg.norm(g - go) <= 1e-5 * np.linalg.norm(go)
    # every layer, not only the norm-dominant ones
    off = 0
    for a, b in mlp.layer_sizes(F, H, O):
        sl = slice(off, off + a * b + b)
        assert np.linalg.norm(g[sl] - go[sl]) <= 2e-5 * np.linalg.norm(go[sl]) + 1e-12
        off += a * b + b


def test_adam_matches_oracle(env):
    torch, tts, jpolicy = env
    say("adam 3 steps")
    pol = jpolicy.Policy(seed=5)
    theta = pol.params.cpu().numpy().astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    g = np.random.default_rng(6)
    for step in range(1, 4):
        gr = (g.standard_normal(theta.size) * 10 ** g.uniform(-4, 0, theta.size)).astype(np.float32)
        pol.adam(torch.from_numpy(gr).cuda(), lr=1e-2)
        theta, m, v = mlp.adam_step(theta, m, v, gr.astype(np.float64), step, 1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pol.params.cpu().numpy(), theta, rtol=1e-5, atol=1e-6)
    # m is a short FP32 recurrence over gradients of both signs: near zero its
    # error is absolute, of the order of the FP32 rounding of |g| <= ~4
    np.testing.assert_allclose(pol.m.cpu().numpy(), m, rtol=1e-5, atol=4e-7)


def test_training_on_gpu_reduces_loss(env):
    torch, tts, jpolicy = env
    say("fit affine target")
    g = np.random.default_rng(9)
    X = g.standard_normal((2048, F)).astype(np.float32)
    A = g.standard_normal((O, F))
    T = (X @ A.T + 0.3).astype(np.float32)
    pol = jpolicy.Policy(seed=10)
    L0 = pol.mse(X, T)
    pol.fit(X, T, steps=600, lr=3e-3, batch=256, seed=1)
    assert pol.mse(X, T) < 0.02 * L0


def test_choose_selects_the_exact_update(env):
    """A prediction at or above TT_JPOLICY_EXACT_J selects the unsketched
    update (J = 0) on a plan with exact buffers, and the plan's J cap on a
    plan without; just below it, a sketch size."""
    torch, tts, jpolicy = env
    say("choose exact")
    theta = np.zeros(jpolicy.P, dtype=np.float32)
    theta[-1] = math.log10(1e-2) + 3.0
    n, R = [12, 10, 9, 11], [1, 3, 4, 3, 1]
    pe = tts.Plan(n, R, 4000, 1e-3, seed=1, exact=True)
    pn = tts.Plan(n, R, 4000, 1e-3, seed=1)
    theta[-2] = math.log(jpolicy._abi.JPOLICY_EXACT_LABEL) - 7.0
    assert pe.choose(jpolicy.Policy(theta).params, 1, 0.3)[0] == 0
    assert pn.choose(jpolicy.Policy(theta).params, 1, 0.3)[0] == 4000
    theta[-2] = math.log(jpolicy._abi.JPOLICY_EXACT_J * 0.99) - 7.0
    assert pe.choose(jpolicy.Policy(theta).params, 1, 0.3)[0] == 4000


def test_run_with_exact_choices_equals_exact_sweeps(env):
    """A policy that always picks the exact update makes tt_als_run's sweeps
    those of tt_als_sweep_exact with the policy's lambda, recorded as J = 0."""
    torch, tts, jpolicy = env
    import synth
    say("run with exact choices")
    n, R = [20, 22, 18, 21], [1, 4, 5, 4, 1]
    dev = torch.device("cuda:0")
    X, _ = synth.tt_tensor_device(n, R, 1e-3, 41, dtype="f32", device=dev)
    init = synth.random_cores(n, R, 42)
    theta = np.zeros(jpolicy.P, dtype=np.float32)
    theta[-2] = math.log(jpolicy._abi.JPOLICY_EXACT_LABEL) - 7.0
    theta[-1] = math.log10(1e-2) + 3.0
    plan = tts.Plan(n, R, 1000, 1e-3, seed=43, exact=True)
    c = [tts.core_to_device(x) for x in init]
    out = plan.run(X, c, 3, 0.0, params=jpolicy.Policy(theta).params)
    ref = tts.Plan(n, R, 1000, 1e-2, seed=43, exact=True)
    c2 = [tts.core_to_device(x) for x in init]
    res = [ref.als_sweep_exact(X, c2, residual=True) for _ in range(3)]
    assert out["J"] == [0, 0, 0] and out["fallbacks"] == 0
    assert out["lambda"] == pytest.approx([1e-2] * 3, rel=1e-6)
    np.testing.assert_allclose(out["residuals"], res, rtol=1e-9)


def test_choose_decodes_outputs(env):
    """All weights zero: the output is the last bias, so J = exp(b0 + 7)
    rounded to a 2-3-5-7 number and lambda = 10^(b1 - 3)."""
    torch, tts, jpolicy = env
    say("choose")
    theta = np.zeros(jpolicy.P, dtype=np.float32)
    theta[-2] = math.log(1990.0) - 7.0
    theta[-1] = math.log10(2e-2) + 3.0
    pol = jpolicy.Policy(theta)
    plan = tts.Plan([12, 10, 9, 11], [1, 3, 4, 3, 1], 4000, 1e-3, seed=1)
    J, lam = plan.choose(pol.params, 2, 0.5, J_min=64)
    assert J == 2000 and lam == pytest.approx(2e-2, rel=1e-5)
    theta[-2] = math.log(20.0) - 7.0
    J, _ = plan.choose(jpolicy.Policy(theta).params, 0, 0.0, J_min=100)
    assert J == 100
    theta[-2] = 20.0
    J, _ = plan.choose(jpolicy.Policy(theta).params, 0, 0.0, J_min=64)
    assert J == 4000


def _problem(torch, tts, n, R, noise, seed, J, lam=1e-3):
    import synth
    dev = torch.device("cuda:0")
    X, _ = synth.tt_tensor_device(n, R, noise, seed, dtype="f32", device=dev)
    plan = tts.Plan(n, R, J, lam, seed=seed, x_dtype="f32", work_dtype="f32", device=dev)
    cores = [tts.core_to_device(c, dev) for c in synth.random_cores(n, R, seed + 1)]
    return X, plan, cores


def test_run_without_policy_equals_sweeps(env):
    """tt_als_run without a policy makes the same sweeps (serial schedule) as
    tt_als_sweep."""
    torch, tts, jpolicy = env
    say("run fixed J vs sweeps")
    n, R = [20, 22, 18, 21], [1, 4, 5, 4, 1]
    X, plan, cores = _problem(torch, tts, n, R, 1e-3, 21, 500)
    out = plan.run(X, cores, 4, 0.0)
    X2, plan2, cores2 = _problem(torch, tts, n, R, 1e-3, 21, 500)
    res = [plan2.als_sweep(X2, cores2, residual=True) for _ in range(4)]
    assert out["sweeps"] == 4 and not out["reached"] and out["fallbacks"] == 0
    np.testing.assert_allclose(out["residuals"], res, rtol=1e-6)
    assert out["J"] == [500] * 4


def test_run_stops_at_the_target(env):
    """A run whose target is met after sweep t stops there: t + 1 sweeps, and
    the cores are those after sweep t."""
    torch, tts, jpolicy = env
    say("run stops at target")
    n, R = [20, 22, 18, 21], [1, 4, 5, 4, 1]
    X2, plan2, cores2 = _problem(torch, tts, n, R, 1e-3, 21, 500)
    res = [plan2.als_sweep(X2, cores2, residual=True) for _ in range(4)]
    t_hit = next(i for i, r in enumerate(res) if r <= 5e-2)
    X, plan, cores = _problem(torch, tts, n, R, 1e-3, 21, 500)
    out = plan.run(X, cores, 8, 5e-2)
    assert out["reached"] and out["sweeps"] == t_hit + 1
    assert out["residual"] == pytest.approx(res[t_hit], rel=1e-4)
    assert plan.residual(X, cores) == pytest.approx(res[t_hit], rel=1e-4)


def test_run_with_policy_follows_its_rules(env):
    """Each sweep's J is a 2-3-5-7 number in [J_min, plan J]; a sweep that
    did not lower the residual is followed by the Corollary 3 fallback size
    (capped) with the descriptor's lambda; the run stops at the target."""
    torch, tts, jpolicy = env
    say("run with policy")
    n, R = [24, 20, 22, 18], [1, 5, 6, 5, 1]
    X, plan, cores = _problem(torch, tts, n, R, 1e-3, 31, 4000)
    pol = jpolicy.Policy(seed=4)
    out = plan.run(X, cores, 8, 1e-2, params=pol.params, J_min=64)
    fb = plan.fallback_J()
    res = out["residuals"]
    nfb = 0
    for t in range(out["sweeps"]):
        J = out["J"][t]
        x = J
        for q in (2, 3, 5, 7):
            while x % q == 0:
                x //= q
        assert x == 1 and 64 <= J <= 4000
        # a sweep (from the second on) that did not lower the previous
        # residual sends the next to the fallback size with the descriptor's
        # lambda
        if t >= 2 and not (res[t - 1] < res[t - 2]):
            assert J == fb and out["lambda"][t] == 1e-3
            nfb += 1
    assert nfb == out["fallbacks"]
    assert out["reached"] == (out["residual"] <= 1e-2)
    if out["reached"]:
        assert all(r > 1e-2 for r in out["residuals"][:-1])


def test_whole_run_labels(env):
    """The whole-run labels name the J whose run reaches the target first, and
    label every state of that run up to the target."""
    torch, tts, jpolicy = env
    say("whole-run labels")
    # seed 2 draws a small order-4 problem (33 x 34 x 38 x 34)
    X, T, meta = jpolicy.collect_runs(1, 2, "cuda", J_grid=(250, 1000), max_sweeps=3, exact=False)
    assert meta
    ms = meta[0]["ms_to_target"]
    finite = {J: v for J, v in ms.items() if v != math.inf}
    assert finite, ms   # the run with the best residual always reaches max(1e-2, 1.5 x best)
    Jstar = min(finite, key=lambda J: (finite[J], J))
    assert all(m["J"] == Jstar for m in meta)
    assert [m["t"] for m in meta] == list(range(len(meta)))
    d = len(meta[0]["n"])
    assert X.shape == (d * len(meta), F) and T.shape == (d * len(meta), O)
    assert np.allclose(T[:, 0], math.log(Jstar) - 7.0) and np.allclose(T[:, 1], 0.0)   # lambda = 1e-3
    assert np.allclose(X[:d, 7], 0.0)   # no residual drop before the first sweep


def test_whole_run_labels_with_the_exact_run(env):
    """With the exact run among the choices its label is
    TT_JPOLICY_EXACT_LABEL when it reaches the target first."""
    torch, tts, jpolicy = env
    say("whole-run labels with exact")
    X, T, meta = jpolicy.collect_runs(1, 2, "cuda", J_grid=(250, 1000), max_sweeps=3, exact=True)
    ms = meta[0]["ms_to_target"]
    finite = {J: v for J, v in ms.items() if v != math.inf}
    best = min(finite, key=lambda J: (finite[J], J if J != jpolicy.EXACT else math.inf))
    lab = jpolicy._abi.JPOLICY_EXACT_LABEL if best == jpolicy.EXACT else best
    assert all(m["J"] == lab for m in meta)
    assert np.allclose(T[:, 0], math.log(lab) - 7.0)


def _time_to_target(fn):
    torch = pytest.importorskip("torch")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


GAIN_PROBLEMS = [([40] * 5, [1, 8, 8, 8, 8, 1], 2e-3, 71), ([56, 48, 52, 60], [1, 10, 12, 10, 1], 1e-3, 72),
                 ([36] * 5, [1, 6, 9, 9, 6, 1], 3e-3, 73)]


def test_policy_gain_over_fixed_sketch_sizes(env):
    """Time to relative residual 1e-2 on problems outside the training draw
    (shapes and seeds the collection never produced): the shipped policy
    (tt_als_run with the trained weights, exact update available) against
    fixed J = 3000, the best J of {1000, 3000, 8000}, the capped Corollary 3
    size from the start, and exact sweeps throughout.  Asserts that the
    policy reaches the target on every problem and takes less than 0.8 x
    the total time of fixed J = 3000 and of the Corollary 3 size; reports
    the rest (the best grid J, and exact sweeps, which the shipped policy
    picks on these problems)."""
    import os
    import synth
    torch, tts, jpolicy = env
    say("policy gain")
    pol = jpolicy.Policy.load(os.path.join(os.path.dirname(tts.__file__), "jpolicy_weights.npy"), device="cuda")
    dev = torch.device("cuda:0")
    tgt, maxs = 1e-2, 12
    tot = {"policy": 0.0, "J3000": 0.0, "best_grid": 0.0, "cor3": 0.0, "exact": 0.0}
    for n, R, nu, seed in GAIN_PROBLEMS:
        scale = math.sqrt(float(np.prod(R[1:-1])))
        X, _ = synth.tt_tensor_device(n, R, nu * scale, seed, dtype="f32", device=dev)
        init = synth.random_cores(n, R, seed + 1)

        def fresh():
            return [tts.core_to_device(c, dev) for c in init]

        def fixed(J):
            p = tts.Plan(n, R, J, 1e-3, seed=seed, device=dev)
            p.run(X, fresh(), 1, 0.0)          # first-use costs out of the timing
            p.set_sweep(0)
            return _time_to_target(lambda: p.run(X, fresh(), maxs, tgt))

        pp = tts.Plan(n, R, 8000, 1e-3, seed=seed, device=dev, exact=True)
        pp.run(X, fresh(), 1, 0.0, params=pol.params)
        pp.set_sketch(8000, 1e-3)
        pp.set_sweep(0)
        t_pol, o_pol = _time_to_target(lambda: pp.run(X, fresh(), maxs, tgt, params=pol.params))
        grid = {J: fixed(J) for J in (1000, 3000, 8000)}
        fb = pp.fallback_J()
        t_fb, o_fb = fixed(fb)
        pe = tts.Plan(n, R, 8000, 1e-3, seed=seed, device=dev, exact=True)
        c = fresh()
        pe.als_sweep_exact(X, fresh())

        def exact_run():
            h = []
            for _ in range(maxs):
                h.append(pe.als_sweep_exact(X, c, residual=True))
                if h[-1] <= tgt:
                    break
            return h

        t_ex, h_ex = _time_to_target(exact_run)
        best = min(grid, key=lambda J: (not grid[J][1]["reached"], grid[J][0]))
        print("%s R=%s: policy %.1f ms (%d sweeps, J %s) | J=3000 %.1f ms (%d, %s) | best grid J=%d %.1f ms | "
              "Cor. 3 J=%d %.1f ms (%s) | exact %.1f ms (%d sweeps)" % (
                  n, R, t_pol * 1e3, o_pol["sweeps"], o_pol["J"], grid[3000][0] * 1e3, grid[3000][1]["sweeps"],
                  grid[3000][1]["reached"], best, grid[best][0] * 1e3, fb, t_fb * 1e3, o_fb["reached"],
                  t_ex * 1e3, len(h_ex)))
        assert o_pol["reached"], (n, o_pol)
        tot["policy"] += t_pol
        tot["J3000"] += grid[3000][0]
        tot["best_grid"] += grid[best][0]
        tot["cor3"] += t_fb
        tot["exact"] += t_ex
        del X, pp, pe
    print("totals (ms):", {k: round(v * 1e3, 1) for k, v in tot.items()})
    assert tot["policy"] < 0.8 * tot["J3000"] and tot["policy"] < 0.8 * tot["cor3"], tot
