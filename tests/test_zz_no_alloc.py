"""The allocation-free residual entry point (tt_residual_noalloc) against the
plan-based one (tt_residual) and the FP64 oracle: same inputs, consecutive
calls with a smaller input second, the path whose G_0 x G_1 table does not
fit in the static scratch, and the size check."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import als

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def tts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_08093_amd as m
    return m


def _inputs(tts, n, R, xd, seed):
    Xh, _ = synth.tt_tensor_host(n, R, 0.05, seed)
    cores = synth.random_cores(n, R, seed + 1)
    X = synth.to_dtype_host(Xh, xd)
    X = (torch.from_numpy(X) if isinstance(X, np.ndarray) else X).cuda()
    Xo = synth.upcast_host(synth.to_dtype_host(Xh, xd))
    return X, Xo, cores, [tts.core_to_device(c) for c in cores]


# larger input first, then a smaller one: the second call reuses the scratch
# the first one filled
CASES = [
    ([40, 30, 20, 12], [1, 5, 6, 4, 1], "f32", "f32"),
    ([16, 16, 16, 16], [1, 3, 3, 3, 1], "f64", "f64"),
    ([64, 8, 8, 8], [1, 8, 8, 8, 1], "bf16", "f32"),
    ([9, 7], [1, 3, 1], "f32", "f32"),
]


def test_noalloc_matches_plan_residual(tts):
    for i, (n, R, xd, wd) in enumerate(CASES):
        say("noalloc residual", n, R, xd, wd)
        X, Xo, cores, dc = _inputs(tts, n, R, xd, 20 + i)
        plan = tts.Plan(n, R, 16, 1e-3, x_dtype=xd, work_dtype=wd)
        want = plan.residual(X, dc)
        got = tts.residual_noalloc(X, dc, n, R, xd, wd)
        # same kernels and launch shape as the plan's residual
        assert got == want, (got, want)
        ref = als.rel_residual(Xo, cores)
        assert abs(got - ref) <= (1e-12 if wd == "f64" else 1e-5) * ref, (got, ref)
        again = tts.residual_noalloc(X, dc, n, R, xd, wd)
        assert again == got


def test_noalloc_without_room_for_the_slab_table(tts):
    # n_0 n_1 R_2 = 4096 * 2048 * 2 FP32 values = 64 MiB > the scratch, so each
    # task forms its rows of G_0 x G_1 itself; the plan keeps the table
    n, R = [4096, 2048, 2], [1, 2, 2, 1]
    say("noalloc residual, no slab table", n, R)
    X, Xo, cores, dc = _inputs(tts, n, R, "f32", 40)
    plan = tts.Plan(n, R, 16, 1e-3, x_dtype="f32", work_dtype="f32")
    want = plan.residual(X, dc)
    got = tts.residual_noalloc(X, dc, n, R, "f32", "f32")
    assert abs(got - want) <= 1e-6 * want, (got, want)
    assert abs(got - als.rel_residual(Xo, cores)) <= 1e-5 * want
    # and a smaller call after it
    n2, R2 = [12, 10, 8], [1, 3, 2, 1]
    X2, Xo2, cores2, dc2 = _inputs(tts, n2, R2, "f32", 41)
    got2 = tts.residual_noalloc(X2, dc2, n2, R2, "f32", "f32")
    assert abs(got2 - als.rel_residual(Xo2, cores2)) <= 1e-5 * got2


def test_noalloc_rejects_scratch_beyond_the_limit(tts):
    # u(o) alone needs 4096 * 4096 outer tuples * R_2 = 2 FP32 values = 128 MiB
    n, R = [2, 2, 4096, 4096], [1, 2, 2, 2, 1]
    say("noalloc residual, too large", n, R)
    X = torch.zeros(int(np.prod(n)), dtype=torch.float32, device="cuda")
    dc = [torch.zeros(R[k] * n[k] * R[k + 1], dtype=torch.float64, device="cuda") for k in range(4)]
    with pytest.raises(tts.TTError) as ei:
        tts.residual_noalloc(X, dc, n, R, "f32", "f32")
    assert ei.value.status == 2 and "TT_NOALLOC_SCRATCH_BYTES" in str(ei.value)
    # the library still works after the rejected call
    n2, R2 = [12, 10, 8], [1, 3, 2, 1]
    X2, Xo2, cores2, dc2 = _inputs(tts, n2, R2, "f32", 42)
    got = tts.residual_noalloc(X2, dc2, n2, R2, "f32", "f32")
    assert abs(got - als.rel_residual(Xo2, cores2)) <= 1e-5 * got
