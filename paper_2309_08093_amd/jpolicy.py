"""Sketch-size policy: training data from the method's own runs, training on
the GPU with the library's forward / backward / Adam kernels, and use.

The network and its kernels are in the C ABI (tt_jpolicy_*, tt_als_run);
this module marshals arrays and runs the label-collection loop, in which
every sweep, residual and feature vector is computed by the library.

Two label designs (one label per sweep state; the d feature rows of a state,
one per core update, all carry it as (ln J* - 7, log10 lambda* + 3), and
their residual drop is that of the previous sweep, as in tt_als_run):

* "runs" (default): from the problem's start, one run per J of a geometric
  grid at lambda = 1e-3, and one run of exact (unsketched) sweeps, each up to
  a fixed number of sweeps, timed with its residual check after every sweep
  (as tt_als_run runs).  The target is max(1e-2, 1.5 x the best residual any
  run reached); J* is the choice whose run reaches it first (the exact run
  is labelled J = TT_JPOLICY_EXACT_LABEL), and the states of that run up to
  the target are labelled J*.  This is the quantity a run is judged by, the
  time to a target.
* "sweep": starting from the same cores and sweep index, one sweep per J;
  J* maximises that sweep's residual drop per second, lambda* is the best of
  a grid at J*, and the run continues from that sweep.  Greedy: a larger
  first drop need not remove a sweep before a target is reached.
"""
import json
import math
import time

import numpy as np
import torch

from . import _abi
from ._abi import check

_lib = _abi.load()

F, H, O, P = _abi.JPOLICY_FEATURES, _abi.JPOLICY_HIDDEN, _abi.JPOLICY_OUTPUTS, _abi.JPOLICY_PARAMS


def _ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    import ctypes
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def init_params(seed):
    """He-uniform weights, zero biases, in the C ABI's parameter layout."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for a, b in [(F, H), (H, H), (H, H), (H, O)]:
        lim = math.sqrt(6.0 / a)
        out.append(g.uniform(-lim, lim, size=(b, a)).reshape(-1))
        out.append(np.zeros(b))
    theta = np.concatenate(out).astype(np.float32)
    assert theta.size == P
    return theta


def encode_targets(J, lam):
    return np.array([math.log(J) - 7.0, math.log10(lam) + 3.0], dtype=np.float32)


class Policy:
    """Parameters on the device plus Adam moments."""

    def __init__(self, params=None, device="cuda", seed=0):
        self.device = torch.device(device)
        theta = init_params(seed) if params is None else np.asarray(params, dtype=np.float32).reshape(-1)
        if theta.size != P:
            raise ValueError("policy needs %d parameters" % P)
        self.params = torch.from_numpy(theta.copy()).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    @classmethod
    def load(cls, path, device="cuda"):
        return cls(np.load(path, allow_pickle=False), device=device)

    def save(self, path):
        np.save(path, self.params.detach().cpu().numpy())

    def _rows(self, A, width):
        A = torch.as_tensor(A, dtype=torch.float32)
        A = A.to(self.device).contiguous()
        if A.dim() != 2 or A.shape[1] != width:
            raise ValueError("expected B x %d rows" % width)
        return A

    def forward(self, feats):
        X = self._rows(feats, F)
        Y = torch.empty((X.shape[0], O), dtype=torch.float32, device=self.device)
        check(_lib.tt_jpolicy_forward(_ptr(self.params), _ptr(X), X.shape[0], _ptr(Y), _stream(self.device)),
              "tt_jpolicy_forward")
        return Y

    def loss_grad(self, feats, targets):
        X = self._rows(feats, F)
        T = self._rows(targets, O)
        g = torch.empty_like(self.params)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        check(_lib.tt_jpolicy_loss_grad(_ptr(self.params), _ptr(X), _ptr(T), X.shape[0], _ptr(g), _ptr(loss),
                                        _stream(self.device)), "tt_jpolicy_loss_grad")
        return loss, g

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        check(_lib.tt_jpolicy_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(grad), P, self.step, lr, beta1,
                                   beta2, eps, _stream(self.device)), "tt_jpolicy_adam")

    def fit(self, feats, targets, steps=3000, lr=1e-3, batch=256, seed=0, log_every=500, log=None):
        """Minibatch Adam on the device.  Returns the loss every log_every steps."""
        X = self._rows(feats, F)
        T = self._rows(targets, O)
        n = X.shape[0]
        g = np.random.Generator(np.random.PCG64(seed))
        hist = []
        order = g.permutation(n)
        pos = 0
        for it in range(steps):
            if pos + batch > n:
                order = g.permutation(n)
                pos = 0
            idx = torch.from_numpy(order[pos:pos + batch].copy()).to(self.device)
            pos += batch
            loss, grad = self.loss_grad(X.index_select(0, idx), T.index_select(0, idx))
            self.adam(grad, lr=lr)
            if (it + 1) % log_every == 0 or it == 0:
                hist.append((it + 1, float(loss.item())))
                if log:
                    log("[policy] step %d loss %.5f" % hist[-1])
        return hist

    def mse(self, feats, targets):
        """Full-batch loss with the current parameters (chunks of 4096)."""
        X = self._rows(feats, F)
        T = self._rows(targets, O)
        tot = 0.0
        for a in range(0, X.shape[0], 4096):
            loss, _ = self.loss_grad(X[a:a + 4096], T[a:a + 4096])
            tot += float(loss.item()) * min(4096, X.shape[0] - a)
        return tot / X.shape[0]


def random_problem(g):
    """Shape, ranks and relative noise of one training run: order 4-5, modes
    in [30, 40], ranks U[2, 12] clipped to feasibility, noise log-uniform in
    [1e-4, 1e-1] relative to the entry scale; one run in six is a large order-5
    tensor with modes in [50, 64] (up to 1.07e9 entries), so that the
    features of large tensors are inside the training range."""
    import synth
    if g.uniform() < 1.0 / 6.0:
        d = 5
        n = [int(x) for x in g.integers(50, 65, size=d)]
    else:
        d = int(g.integers(4, 6))
        n = [int(x) for x in g.integers(30, 41, size=d)]
    R = [1] + [int(x) for x in g.integers(2, 13, size=d - 1)] + [1]
    R = synth.clip_ranks(n, R)
    nu = float(10 ** g.uniform(-4, -1))
    return n, R, nu


def collect(n_tensors, seed, device="cuda", J_grid=(250, 500, 1000, 2000, 4000, 8000),
            lam_grid=(1e-4, 1e-3, 1e-2, 1e-1), sweeps=5, log=None):
    """Labelled (features, targets) from n_tensors runs; see the module doc."""
    import synth
    from . import Plan, core_to_device
    dev = torch.device(device)
    g = np.random.Generator(np.random.PCG64(seed))
    feats, targs, meta = [], [], []
    Jmax = max(J_grid)
    t0 = time.time()
    stream = torch.cuda.current_stream(dev)
    for i in range(n_tensors):
        n, R, nu = random_problem(g)
        s_i = int(g.integers(1, 2 ** 31))
        scale = math.sqrt(float(np.prod(R[1:-1])))
        X, _ = synth.tt_tensor_device(n, R, nu * scale, s_i, dtype="f32", device=dev)
        plan = Plan(n, R, Jmax, 1e-3, seed=s_i, x_dtype="f32", work_dtype="f32", device=dev, serial=True)
        cores = [core_to_device(c, dev) for c in synth.random_cores(n, R, s_i + 1)]
        hist = [1.0]        # hist[s + 1]: residual after sweep s; 1 before the first (tt_als_run's convention)
        for t in range(sweeps):
            state = [c.clone() for c in cores]

            def trial(J, lam):
                for c, s0 in zip(cores, state):
                    c.copy_(s0)
                plan.set_sweep(t)
                plan.set_sketch(J, lam)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                plan.als_sweep(X, cores)
                e1.record(stream)
                res = plan.residual(X, cores)
                return math.log10(hist[-1] / res), res, e0.elapsed_time(e1)

            runs = {J: trial(J, 1e-3) for J in J_grid}
            rate = {J: r[0] / r[2] for J, r in runs.items()}
            Jstar = max(J_grid, key=lambda J: (rate[J], -J)) if max(rate.values()) > 0 else Jmax
            best = None
            for lam in lam_grid:
                dr, res, _ = trial(Jstar, lam)
                if best is None or dr > best[0]:
                    best = (dr, res, lam, [c.clone() for c in cores])
            dr, res, lam, cbest = best
            drop = math.log10(hist[t - 1] / hist[t]) if t >= 1 else 0.0
            F_rows = plan.features(t, drop)
            feats.append(F_rows)
            targs.append(np.repeat(encode_targets(Jstar, lam)[None, :], len(n), axis=0))
            meta.append({"n": n, "R": R, "noise": nu, "t": t, "J": Jstar, "lambda": lam,
                         "drops": {J: r[0] for J, r in runs.items()}, "ms": {J: r[2] for J, r in runs.items()},
                         "res": res})
            for c, cb in zip(cores, cbest):
                c.copy_(cb)
            hist.append(res)
        del X, plan, cores
        if log and (i + 1) % 20 == 0:
            log("[collect] %d/%d tensors, %d rows, %.0f s" % (i + 1, n_tensors, sum(len(f) for f in feats),
                                                          time.time() - t0))
    return np.concatenate(feats).astype(np.float32), np.concatenate(targs).astype(np.float32), meta


EXACT = 0   # key of the exact run among the J choices


def collect_runs(n_tensors, seed, device="cuda", J_grid=(250, 500, 1000, 2000, 4000, 8000), lam=1e-3,
                 max_sweeps=8, exact=True, log=None):
    """Labelled (features, targets) from whole runs to a target; see the
    module doc.  Returns the same layout as collect()."""
    import synth
    from . import Plan, core_to_device
    dev = torch.device(device)
    g = np.random.Generator(np.random.PCG64(seed))
    feats, targs, meta = [], [], []
    Jmax = max(J_grid)
    t0 = time.time()
    for i in range(n_tensors):
        n, R, nu = random_problem(g)
        s_i = int(g.integers(1, 2 ** 31))
        scale = math.sqrt(float(np.prod(R[1:-1])))
        X, _ = synth.tt_tensor_device(n, R, nu * scale, s_i, dtype="f32", device=dev)
        plan = Plan(n, R, Jmax, lam, seed=s_i, x_dtype="f32", work_dtype="f32", device=dev, serial=True,
                    exact=exact)
        init = synth.random_cores(n, R, s_i + 1)
        scratch = [core_to_device(c, dev) for c in init]   # first-use costs out of the timings
        plan.als_sweep(X, scratch)
        if exact:
            plan.als_sweep_exact(X, scratch)
        plan.residual(X, scratch)
        runs = {}
        choices = tuple(J_grid) + ((EXACT,) if exact else ())
        for J in choices:
            cores = [core_to_device(c, dev) for c in init]
            plan.set_sketch(Jmax if J == EXACT else J, lam)
            plan.set_sweep(0)
            sweep = plan.als_sweep_exact if J == EXACT else plan.als_sweep
            torch.cuda.synchronize()
            t_acc, times, res = 0.0, [], []
            for _ in range(max_sweeps):
                ta = time.perf_counter()
                sweep(X, cores)
                r = plan.residual(X, cores)   # synchronises
                t_acc += time.perf_counter() - ta
                times.append(t_acc)
                res.append(r)
            runs[J] = (times, res)
        best = min(min(r) for _, r in runs.values())
        tau = max(1e-2, 1.5 * best)

        def reach(J):
            times, res = runs[J]
            for s, r in enumerate(res):
                if r <= tau:
                    return times[s], s + 1
            return math.inf, None

        # ties go to the smaller sketch; the exact run ranks above every J
        Jstar = min(choices, key=lambda J: (reach(J)[0], J if J != EXACT else math.inf))
        T_star = reach(Jstar)[1]
        Jlab = _abi.JPOLICY_EXACT_LABEL if Jstar == EXACT else Jstar
        h = [1.0] + runs[Jstar][1]   # h[s + 1]: residual after sweep s
        for t in range(T_star):
            drop = math.log10(h[t - 1] / h[t]) if t >= 1 else 0.0
            feats.append(plan.features(t, drop))
            targs.append(np.repeat(encode_targets(Jlab, lam)[None, :], len(n), axis=0))
            meta.append({"n": n, "R": R, "noise": nu, "t": t, "J": Jlab, "lambda": lam, "target": tau,
                         "ms_to_target": {J: reach(J)[0] * 1e3 for J in choices}})
        del X, plan, scratch
        if log and (i + 1) % 20 == 0:
            log("[collect] %d/%d tensors, %d rows, %.0f s" % (i + 1, n_tensors, sum(len(f) for f in feats),
                                                          time.time() - t0))
    return np.concatenate(feats).astype(np.float32), np.concatenate(targs).astype(np.float32), meta


def main():
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="collect labels from method runs and train the sketch-size policy")
    ap.add_argument("--tensors", type=int, default=400)
    ap.add_argument("--sweeps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--labels", choices=("runs", "sweep"), default="runs")
    ap.add_argument("--max-sweeps", type=int, default=8, help="sweeps per run of the 'runs' labels")
    ap.add_argument("--out", required=True, help="prefix of the weights (.npy) and summary (.json) files")
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    if args.labels == "runs":
        X, T, meta = collect_runs(args.tensors, args.seed, dev, max_sweeps=args.max_sweeps, log=log)
    else:
        X, T, meta = collect(args.tensors, args.seed, dev, sweeps=args.sweeps, log=log)
    np.savez(args.out + "_data.npz", X=X, T=T)
    g = np.random.Generator(np.random.PCG64(args.seed + 1))
    perm = g.permutation(len(meta))
    nval = max(1, len(meta) // 10)
    d_of = [len(m["n"]) for m in meta]
    starts = np.cumsum([0] + d_of)
    rows = lambda ids: np.concatenate([np.arange(starts[i], starts[i + 1]) for i in ids])
    val, tr = rows(perm[:nval]), rows(perm[nval:])
    pol = Policy(seed=args.seed + 2, device=dev)
    base = float(np.mean((T[val] - T[tr].mean(axis=0)) ** 2))
    hist = pol.fit(X[tr], T[tr], steps=args.steps, lr=args.lr, seed=args.seed + 3, log=log)
    summary = {"tensors": args.tensors, "rows": int(len(X)), "train_rows": int(len(tr)), "val_rows": int(len(val)),
               "steps": args.steps, "lr": args.lr, "train_loss": hist, "val_mse": pol.mse(X[val], T[val]),
               "val_mse_of_mean_predictor": base,
               "label_J_counts": {str(J): int(sum(1 for m in meta if m["J"] == J)) for J in sorted({m["J"] for m in meta})},
               "label_lambda_counts": {str(l): int(sum(1 for m in meta if m["lambda"] == l))
                                       for l in sorted({m["lambda"] for m in meta})}}
    pol.save(args.out + ".npy")
    with open(args.out + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    log(json.dumps({k: v for k, v in summary.items() if k != "train_loss"}))


if __name__ == "__main__":
    main()
