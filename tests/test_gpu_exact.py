"""GPU parity of the exact (unsketched) proximal update against the FP64
oracle: A_(k) H_k by mode-by-mode contraction of X (tt_exact_rhs), the
proximal step with the Gram factors of arbitrary cores (tt_prox_exact), exact
sweeps (tt_als_sweep_exact) against the oracle's exact passes, the sketched
sweep with an injective sketch against the exact sweep, and the exact sweep
as the fallback of tt_als_run.  Tolerances: FP64 work 1e-10, FP32 work 1e-5,
norm-wise and element-wise; residuals within 1e-4."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import als, solve

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


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def colmax(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(np.shape(a)[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(np.shape(b)[0], -1)
    den = np.abs(b).max(axis=0)
    err = np.abs(a - b).max(axis=0)
    return float(np.max(np.where(den > 0, err / np.where(den > 0, den, 1.0), err)))


def to_dev_x(Xh, dtype):
    t = synth.to_dtype_host(Xh, dtype)
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(t)
    return t.cuda()


CASES = [
    # n, ranks, x dtype, work dtype
    ([16, 16, 16, 16], [1, 3, 3, 3, 1], "f64", "f64"),
    ([12, 9, 10, 7], [1, 4, 5, 3, 1], "f32", "f32"),
    ([6, 5, 4, 5, 6], [1, 3, 4, 4, 3, 1], "f64", "f64"),
    ([64, 8, 8, 8], [1, 8, 8, 8, 1], "bf16", "f32"),
    ([30, 40], [1, 7, 1], "f32", "f32"),
    ([5, 150, 3], [1, 5, 3, 1], "f32", "f32"),        # long middle mode: K-sliced contractions
    ([13, 11, 9], [1, 13, 9, 1], "f64", "f64"),        # ranks at the feasibility limit
    ([200, 4, 2, 2], [1, 16, 4, 2, 1], "f32", "f32"),  # rank 16 (full MFMA tile), long fibres
]


@pytest.mark.parametrize("n,R,xd,wd", CASES)
def test_exact_rhs_matches_oracle(tts, n, R, xd, wd):
    say("exact rhs", n, R, xd, wd)
    Xh, _ = synth.tt_tensor_host(n, R, 0.05, 51)
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))
    cores = synth.random_cores(n, R, 52)
    plan = tts.Plan(n, R, 16, 1e-3, x_dtype=xd, work_dtype=wd, exact=True)
    X = to_dev_x(Xh, xd)
    dc = [tts.core_to_device(c) for c in cores]
    tol = 1e-10 if wd == "f64" else 1e-5
    for k in range(len(n)):
        B = plan.exact_rhs(X, dc, k).cpu().numpy().astype(np.float64).reshape(n[k], -1, order="F")
        want = als.exact_rhs(Xo, n, cores, k)
        assert rel(B, want) < tol and colmax(B, want) < 10 * tol, (k, rel(B, want), colmax(B, want))


@pytest.mark.parametrize("n,R,xd,wd", CASES[:4])
def test_prox_exact_matches_oracle(tts, n, R, xd, wd):
    # arbitrary (not orthonormal) cores: the Gram factors of H_k^T H_k matter
    say("prox exact", n, R, xd, wd)
    Xh, _ = synth.tt_tensor_host(n, R, 0.05, 53)
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))
    cores = synth.random_cores(n, R, 54, scale=0.7)
    lam = 0.3
    plan = tts.Plan(n, R, 16, lam, x_dtype=xd, work_dtype=wd, exact=True)
    X = to_dev_x(Xh, xd)
    dc = [tts.core_to_device(c) for c in cores]
    tol = 1e-10 if wd == "f64" else 1e-5
    for k in range(len(n)):
        G = tts.core_to_host(plan.prox_exact(X, dc, k), cores[k].shape)
        plan.sync_status()
        want = als.prox_exact(Xo, n, cores, k, lam)
        assert rel(G, want) < tol, (k, rel(G, want))
    # in place (G_new aliases cores[k])
    plan.prox_exact(X, dc, 1, dc[1])
    assert rel(tts.core_to_host(dc[1], cores[1].shape), als.prox_exact(Xo, n, cores, 1, lam)) < tol


@pytest.mark.parametrize("n,R,xd,wd", [CASES[0], CASES[1], CASES[2], CASES[3]])
def test_exact_sweeps_match_oracle(tts, n, R, xd, wd):
    say("exact sweeps", n, R, xd, wd)
    Xh, _ = synth.tt_tensor_host(n, R, 1e-2, 55)
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))
    init = synth.random_cores(n, R, 56)
    lam = 1e-3
    plan = tts.Plan(n, R, 16, lam, x_dtype=xd, work_dtype=wd, exact=True)
    X = to_dev_x(Xh, xd)
    dc = [tts.core_to_device(c) for c in init]
    ref = [c.copy() for c in init]
    for t in range(3):
        r = plan.als_sweep_exact(X, dc, residual=True)
        ref = als.sweep_exact(Xo, n, ref, lam)
        ro = als.rel_residual(Xo, ref)
        got = [tts.core_to_host(c, g.shape) for c, g in zip(dc, ref)]
        d_tt = rel(als.tt_full(got), als.tt_full(ref))
        print("sweep %d: residual %.9e oracle %.9e, TT rel diff %.2e" % (t, r, ro, d_tt))
        assert abs(r - ro) < (1e-10 if wd == "f64" else 1e-4), (t, r, ro)
        assert d_tt < (1e-9 if wd == "f64" else 1e-4), (t, d_tt)
    assert plan.get_sweep() == 3


def test_injective_sketched_sweep_equals_exact_sweep(tts):
    # with h_s(i) = i prod_{t<s} n_t, v = +1 and J = N, S^T S = I, so the
    # sketched sweep is the exact one: two GPU paths that share no kernel
    say("injective sketch vs exact sweep")
    n, R, lam = [4, 5, 3], [1, 2, 3, 1], 0.1
    Xh = synth.rng(35).standard_normal(60)
    init = synth.random_cores(n, R, 36)
    X = torch.from_numpy(Xh).cuda()
    ps = tts.Plan(n, R, 60, lam, x_dtype="f64", work_dtype="f64")
    stride = 1
    for s, ns in enumerate(n):
        ps.set_tables(s, np.arange(ns) * stride, np.ones(ns, dtype=np.int8))
        stride *= ns
    pe = tts.Plan(n, R, 60, lam, x_dtype="f64", work_dtype="f64", exact=True)
    a = [tts.core_to_device(c) for c in init]
    b = [tts.core_to_device(c) for c in init]
    for _ in range(2):
        ps.als_sweep(X, a)
        pe.als_sweep_exact(X, b)
    for x, y, c in zip(a, b, init):
        assert rel(tts.core_to_host(x, c.shape), tts.core_to_host(y, c.shape)) < 1e-10


def test_exact_needs_the_flag(tts):
    say("exact without flag")
    plan = tts.Plan([6, 5, 4], [1, 2, 2, 1], 16, 1e-3)
    X = torch.zeros(120, dtype=torch.float32, device="cuda")
    dc = [torch.zeros(c, dtype=torch.float64, device="cuda") for c in (12, 20, 8)]
    with pytest.raises(tts.TTError) as ei:
        plan.exact_rhs(X, dc, 0)
    assert ei.value.status == 7


def test_run_falls_back_to_exact_sweeps(tts):
    """A policy that always asks for J = 4 makes sketched sweeps that do not
    lower the residual; each is followed by an exact sweep (recorded as
    J = 0, with the descriptor's lambda), since the Corollary 3 size exceeds
    N / n_k here."""
    say("run with exact fallback")
    from paper_2309_08093_amd import _abi
    n, R = [10, 9, 8, 7], [1, 4, 4, 3, 1]
    Xh, _ = synth.tt_tensor_host(n, R, 1e-3, 57)
    X = torch.from_numpy(Xh.astype(np.float32)).cuda()
    plan = tts.Plan(n, R, 512, 1e-3, seed=58, exact=True)
    assert any(tts.sketch_size_bound(R[k] * R[k + 1], len(n) - 1) >= np.prod(n) / n[k] for k in range(len(n)))
    params = torch.zeros(_abi.JPOLICY_PARAMS, dtype=torch.float32, device="cuda")
    params[-2] = math.log(4.0) - 7.0            # output bias: ln J - 7 with J = 4
    cores = [tts.core_to_device(c) for c in synth.random_cores(n, R, 59)]
    out = plan.run(X, cores, 8, 1e-9, params=params, J_min=4)
    res, Js, lams = out["residuals"], out["J"], out["lambda"]
    print("residuals", res, "\nJ", Js)
    nfb = 0
    for t in range(out["sweeps"]):
        if t >= 2 and not (res[t - 1] < res[t - 2]):
            assert Js[t] == 0 and lams[t] == 1e-3, t
            nfb += 1
        else:
            assert Js[t] == 4, t
    assert nfb == out["fallbacks"] and nfb >= 1
    # an exact sweep leaves the tensor near its noise floor
    floor = als.rel_residual(Xh.astype(np.float32).astype(np.float64), synth.tt_tensor_host(n, R, 0.0, 57)[1])
    best = min(r for t, r in enumerate(res) if t >= 1 and Js[t] == 0)
    assert best < 50 * floor + 1e-3, (best, floor)
