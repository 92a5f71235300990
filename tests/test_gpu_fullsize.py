"""GPU parity at the full sizes of the two dense workloads, in the launch
configuration bench.py times (same shapes, J, seed and sketch kernels):

  * 200^4 FP32 tensor from a random TT with ranks 10 plus noise 1e-2, J=4000;
  * 64^5 tensor stored BF16 from a random TT with ranks 8 plus noise 1e-3,
    J=3000.

The oracle cannot sketch 1.6e9 entries in seconds, so the data sketches are
compared on sampled columns: column c of Y_k is the data sketch of the
sub-tensor with i_k = c, which the oracle computes as a tensor whose mode k
has the single index c (the mode-k table is not used for Y_k).  Tolerance as
for the small cases: 1e-5 relative per column (FP32 work type).

The residual pass is checked at full size by a property that holds at any
size: for the noise-free tensor and the cores that generated it, the exact
relative residual is the rounding of X to its storage type (unit roundoff
2^-8 for BF16) plus the FP32 rounding of the TT values, so it stays below
2^-8 + 1e-5 (BF16) or 1e-5 (FP32); a wrong slab or rank index gives O(1).

End to end, ten sweeps from random cores at each full size must settle at
the noise floor, the residual of the generating cores.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import sketch

pytestmark = pytest.mark.gpu

CASES = {
    # name: n, ranks, J, noise, stored dtype, gram mode, (k = 0 kernel, k >= 1 kernel)
    "200^4 f32": ([200] * 4, [1, 10, 10, 10, 1], 4000, 1e-2, "f32", "work", ("k_sketch_mode0", "k_sketch_gs")),
    "64^5 bf16": ([64] * 5, [1, 8, 8, 8, 8, 1], 3000, 1e-3, "bf16", "bf16", ("k_sketch_mode0", "k_sketch_gs")),
}
SEED = 2023   # bench.py's default seed


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_08093_amd as m
    return m


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_size_sketch_sampled_columns(tts, name):
    n, R, J, noise, xd, gram, kernels = CASES[name]
    d = len(n)
    say("full-size sketch columns", name)
    X, _ = synth.tt_tensor_device(n, R, noise, SEED, dtype=xd, device="cuda")
    plan = tts.Plan(n, R, J, 1e-3, seed=SEED, x_dtype=xd, work_dtype="f32", gram=gram, device="cuda")
    hs, vs = [], []
    for s in range(d):
        h, v = plan.get_tables(s)
        hs.append(h)
        vs.append(v)
    Xv = X.view(*n[::-1])   # torch dims (i_{d-1}, ..., i_0): i_0 fastest
    # the sweep's sketches: Y_1 from the outer sketch of the k = 0 pass; at
    # 200^4 that pass also writes the inner sketch that Y_2 and Y_3 come from
    # (one pass over X), at 64^5 BF16 each mode k >= 2 takes its own pass
    assert plan.sketch_sources() == ([0, 0, 0, 0] if name == "200^4 f32" else [0, 0, 2, 3, 4])
    Yall = [y.cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
            for k, y in enumerate(plan.sketch_tensor_all(X))]
    for k in range(d):
        assert plan.sketch_kernel(k) == (kernels[0] if k == 0 else kernels[1]), k
        say("mode", k, plan.sketch_kernel(k))
        Y = plan.sketch_tensor(X, k).cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        for c in (n[k] // 2 + 1, n[k] - 1):
            sub = Xv.select(d - 1 - k, c).contiguous().float().cpu().numpy().astype(np.float64).reshape(-1)
            nsub = list(n)
            nsub[k] = 1
            Yo = sketch.data_sketch(sub, nsub, k, hs, vs, J)[:, 0]
            assert rel(Y[:, c], Yo) < 1e-5, (k, c, rel(Y[:, c], Yo))
            assert rel(Yall[k][:, c], Yo) < 1e-5, (k, c, rel(Yall[k][:, c], Yo))
            # element-wise: the largest deviation against the column's largest entry
            assert np.abs(Yall[k][:, c] - Yo).max() < 1e-5 * np.abs(Yo).max(), (k, c)
        # every column of the fused result against the per-mode pass
        assert rel(Yall[k], Y) < 1e-5, (k, rel(Yall[k], Y))
    del X, Xv, plan
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_size_residual_of_generating_cores(tts, name):
    n, R, J, _, xd, gram, _ = CASES[name]
    say("full-size residual", name)
    X, cores = synth.tt_tensor_device(n, R, 0.0, SEED, dtype=xd, device="cuda")
    plan = tts.Plan(n, R, J, 1e-3, seed=SEED, x_dtype=xd, work_dtype="f32", gram=gram, device="cuda")
    dev_cores = [tts.core_to_device(c, "cuda") for c in cores]
    r = plan.residual(X, dev_cores)
    bound = (2.0 ** -8 if xd == "bf16" else 0.0) + 1e-5
    assert 0.0 <= r < bound, r
    del X, plan, dev_cores
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_size_sweeps_reach_the_noise_floor(tts, name):
    # Ten sweeps of the method from random cores, the bench's configuration.
    # The generating cores are a feasible point of the rank-R problem, so the
    # fit can at best reach their residual (the noise floor: the added noise,
    # and for BF16 storage the rounding of X) less the little noise a rank-R
    # model absorbs.  Each sketched solve is a (1 + eps)-approximation of the
    # exact one, so the sweeps settle just above that floor (measured 1.03x at
    # 200^4 and 1.11x at 64^5); 0.95-1.25x is required.
    n, R, J, noise, xd, gram, _ = CASES[name]
    say("full-size sweeps", name)
    X, cores = synth.tt_tensor_device(n, R, noise, SEED, dtype=xd, device="cuda")
    plan = tts.Plan(n, R, J, 1e-3, seed=SEED, x_dtype=xd, work_dtype="f32", gram=gram, device="cuda")
    floor = plan.residual(X, [tts.core_to_device(c, "cuda") for c in cores])
    dc = [tts.core_to_device(c, "cuda") for c in synth.random_cores(n, R, SEED + 1)]
    res = [plan.als_sweep(X, dc, residual=True) for _ in range(10)]
    print("floor", floor, "residuals", res)
    assert 0.95 * floor <= res[-1] <= 1.25 * floor, (floor, res)
    del X, plan, dc
    torch.cuda.empty_cache()


def test_full_size_batched_form_matches_single_plans(tts):
    # The batched workload at full size (256 uneven TTs, 36.6 GB), autotuned
    # and graph-captured as bench.py runs it: after three sweeps, sampled
    # problems (the largest, the smallest and six more) agree with single
    # plans run on the same tensors, tables and starting cores.  The k = 0
    # kernels of the two forms add bucket contributions in different orders
    # in FP32, which three sweeps carry into the cores, so the tolerance is
    # that of the small batched test: 1e-4 relative on the residual.
    say("full-size batched form")
    shapes = synth.batched_shapes(256, SEED)
    probs = [dict(n=n, ranks=R, J=1024, lam=1e-3, seed=SEED + 17 * i) for i, (n, R) in enumerate(shapes)]
    Xs = [synth.tt_tensor_device(p["n"], p["ranks"], 1e-3, SEED + 31 * i, dtype="f32", device="cuda")[0]
          for i, p in enumerate(probs)]
    init = [synth.random_cores(p["n"], p["ranks"], SEED + 7 * i + 1) for i, p in enumerate(probs)]
    batch = tts.Batch(probs, device="cuda")
    batch.autotune(Xs, reps=1)
    batch.set_graph(True)
    cores = [[tts.core_to_device(c, "cuda") for c in init[i]] for i in range(len(probs))]
    for _ in range(2):
        batch.sweep(Xs, cores)
    res_b = batch.sweep(Xs, cores, residuals=True)
    sizes = [int(np.prod(p["n"])) for p in probs]
    rng = synth.rng(5)
    sample = {int(np.argmax(sizes)), int(np.argmin(sizes))} | set(int(i) for i in rng.choice(len(probs), 6, replace=False))
    for i in sorted(sample):
        p = probs[i]
        say("problem", i, p["n"], p["ranks"])
        plan = tts.Plan(p["n"], p["ranks"], p["J"], p["lam"], seed=p["seed"], serial=True, device="cuda")
        cs = [tts.core_to_device(c, "cuda") for c in init[i]]
        for _ in range(2):
            plan.als_sweep(Xs[i], cs)
        r = plan.als_sweep(Xs[i], cs, residual=True)
        assert abs(res_b[i] - r) <= 1e-4 * r + 1e-9, (i, res_b[i], r)
    del Xs, batch, cores
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_size_exact_sweeps(tts, name):
    """Exact (unsketched) proximal sweeps at full size: from the generating
    cores on the noise-free tensor the residual stays at the storage
    rounding; from random cores on the noisy tensor three sweeps reach the
    noise floor (the residual of the generating cores), within 5 %."""
    n, R, J, noise, xd, gram, _ = CASES[name]
    say("full-size exact sweeps", name)
    X, gen = synth.tt_tensor_device(n, R, noise, SEED, dtype=xd, device="cuda")
    plan = tts.Plan(n, R, J, 1e-3, seed=SEED, x_dtype=xd, work_dtype="f32", gram=gram, device="cuda", exact=True)
    floor = plan.residual(X, [tts.core_to_device(c, "cuda") for c in gen])
    cores = [tts.core_to_device(c, "cuda") for c in synth.random_cores(n, R, SEED + 1)]
    res = [plan.als_sweep_exact(X, cores, residual=True) for _ in range(3)]
    print(name, "floor %.6e" % floor, "exact sweeps", res)
    assert res[-1] <= 1.05 * floor, (res, floor)
    del X, plan, cores
    torch.cuda.empty_cache()
