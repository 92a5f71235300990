"""GPU parity of the O(nnz) sparse-input data sketch (tt_sketch_sparse,
tt_sketch_sparse_all) against the oracle's definition over the stored
entries: bit-exact on integer values, 1e-5 (FP32 work) / 1e-12 (FP64 work)
on Gaussian values, against the dense sketch of the densified tensor, empty
input, and a coordinate out of range."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import sketch

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
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a, float) - b) / (nb if nb > 0 else 1.0)


def coo(n, nnz, seed):
    g = synth.rng(seed)
    c = np.stack([g.integers(0, ns, size=nnz) for ns in n], axis=1).astype(np.int32)
    if nnz > 8:
        c[5] = c[2]                     # a repeated coordinate
    return c


def tables_of(plan):
    hs, vs = [], []
    for s in range(plan.d):
        h, v = plan.get_tables(s)
        hs.append(h)
        vs.append(v)
    return hs, vs


CASES = [([16, 16, 16, 16], 256, "f64", "f64", 5000), ([200, 50, 30], 4000, "f32", "f32", 20000),
         ([8, 9, 7, 6, 5], 3000, "bf16", "f32", 3000), ([40, 30], 60, "f32", "f32", 700),
         ([13, 11, 9, 7], 1, "f32", "f32", 500)]


@pytest.mark.parametrize("n,J,xd,wd,nnz", CASES)
def test_sparse_sketch_matches_oracle(tts, n, J, xd, wd, nnz):
    say("sparse sketch", n, J, xd, nnz)
    plan = tts.Plan(n, [1] * (len(n) + 1), J, 1e-3, seed=62, x_dtype=xd, work_dtype=wd)
    hs, vs = tables_of(plan)
    c = coo(n, nnz, 63)
    dc = torch.from_numpy(c).cuda()
    # integer values: every sum exact
    vi = synth.rng(64).integers(-4, 5, size=nnz).astype(np.float64)
    dv = synth.to_dtype_host(vi, xd)
    dv = (torch.from_numpy(dv) if isinstance(dv, np.ndarray) else dv).cuda()
    alls = plan.sketch_sparse_all(dc, dv)
    for k in range(len(n)):
        want = sketch.data_sketch_sparse(c, vi, n, k, hs, vs, J)
        got = plan.sketch_sparse(dc, dv, k).cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        assert np.array_equal(got, want), k
        got_all = alls[k].cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        assert np.array_equal(got_all, want), k
    # Gaussian values
    vg = synth.rng(65).standard_normal(nnz)
    tv = synth.to_dtype_host(vg, xd)
    vo = synth.upcast_host(tv)
    dv = (torch.from_numpy(tv) if isinstance(tv, np.ndarray) else tv).cuda()
    tol = 1e-12 if wd == "f64" else 1e-5
    for k in range(len(n)):
        want = sketch.data_sketch_sparse(c, vo, n, k, hs, vs, J)
        got = plan.sketch_sparse(dc, dv, k).cpu().numpy().astype(np.float64).reshape(J, n[k], order="F")
        assert rel(got, want) < tol, (k, rel(got, want))
    plan.sync_status()


def test_sparse_equals_dense_sketch_on_gpu(tts):
    # two GPU paths that share no kernel: the sparse scatter over the stored
    # entries and the dense sketch of the densified tensor
    say("sparse vs dense")
    n, J = [37, 12, 11, 13], 40
    c = coo(n, 4000, 66)
    v = synth.rng(67).integers(-3, 4, size=4000).astype(np.float64)
    X = np.zeros(n, order="F")
    np.add.at(X, tuple(c.T.astype(np.int64)), v)
    plan = tts.Plan(n, [1] * 5, J, 1e-3, seed=68)
    Xd = torch.from_numpy(X.reshape(-1, order="F").astype(np.float32)).cuda()
    sp = plan.sketch_sparse_all(torch.from_numpy(c).cuda(), torch.from_numpy(v.astype(np.float32)).cuda())
    for k in range(4):
        assert torch.equal(sp[k], plan.sketch_tensor(Xd, k)), k


def test_sparse_empty_and_bad_coordinates(tts):
    say("sparse empty and out of range")
    n, J = [6, 5, 4], 16
    plan = tts.Plan(n, [1, 1, 1, 1], J, 1e-3)
    empty = torch.zeros((0, 3), dtype=torch.int32, device="cuda")
    Y = plan.sketch_sparse(empty, torch.zeros(0, dtype=torch.float32, device="cuda"), 1)
    assert torch.count_nonzero(Y).item() == 0
    c = coo(n, 50, 69)
    c[7, 2] = 4                          # i_2 = 4 is outside [0, 4)
    v = np.ones(50)
    hs, vs = tables_of(plan)
    got = plan.sketch_sparse(torch.from_numpy(c).cuda(), torch.ones(50, dtype=torch.float32, device="cuda"), 0)
    with pytest.raises(tts.TTError) as ei:
        plan.sync_status()
    assert ei.value.status == 1
    keep = np.ones(50, bool)
    keep[7] = False
    want = sketch.data_sketch_sparse(c[keep], v[keep], n, 0, hs, vs, J)
    assert np.array_equal(got.cpu().numpy().astype(np.float64).reshape(J, n[0], order="F"), want)
    plan.sync_status()   # cleared
