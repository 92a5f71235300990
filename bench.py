"""Benchmark of the TT-TS hot path on one MI355X.

A step is one full sweep of Algorithm 1 (right-to-left orthogonalisation,
d interface sketches, d data-sketch passes over X, d MFMA Gram + FP64 solves,
d-1 QR + absorb steps) on a synthetic tensor resident in HBM.

Default workload: dense 200^4 FP32 tensor (1.6e9 entries, 6.4 GB) built from a
random TT with ranks 10 plus N(0, 1e-2^2) noise; J = 4000, lambda = 1e-3.
Prints one JSON line: value = sketched X entries per second over the timed
sweeps (d * N entries per sweep), the roofline of the dominant kernel (the
k >= 1 data-sketch kernel, timed live with HIP events on the plan's stream),
the plain-FP32 time to relative residual 1e-2, and a CPU baseline (the FP64
oracle's data sketch on a bounded slab of the same tensor).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

CONFIGS = {
    # name: n, ranks, J, lambda, noise, x dtype, work dtype, gram mode, description
    "c2": dict(n=[200] * 4, r=[1, 10, 10, 10, 1], J=4000, lam=1e-3, noise=1e-2, xd="f32", wd="f32", gram="work",
               desc="dense 200^4 FP32 tensor (1.6e9 entries) from a random TT with ranks 10 plus noise 1e-2; "
                    "J=4000, lambda=1e-3"),
    "c1": dict(n=[16] * 4, r=[1, 3, 3, 3, 1], J=256, lam=1e-3, noise=1e-3, xd="f64", wd="f64", gram="work",
               desc="dense 16^4 FP64 tensor from a random TT with ranks 3 plus noise 1e-3; J=256, lambda=1e-3"),
    "c3": dict(n=[64] * 5, r=[1, 8, 8, 8, 8, 1], J=3000, lam=1e-3, noise=1e-3, xd="bf16", wd="f32", gram="bf16",
               desc="dense 64^5 tensor stored BF16 from a random TT with ranks 8 plus noise 1e-3; BF16 MFMA Gram; "
                    "J=3000, lambda=1e-3"),
    "c3f32": dict(n=[64] * 5, r=[1, 8, 8, 8, 8, 1], J=3000, lam=1e-3, noise=1e-3, xd="f32", wd="f32", gram="work",
                  desc="dense 64^5 FP32 tensor from a random TT with ranks 8 plus noise 1e-3; J=3000, lambda=1e-3"),
}
XBYTES = {"f64": 8, "f32": 4, "bf16": 2}
# workload names of the committed profile summaries
PROFILE_TAG = {"c1": "16x4_f64", "c2": "200x4_f32", "c3": "64x5_bf16", "c3f32": "64x5_f32", "c4": "256_uneven_tt_f32"}
# batched workload: 256 independent problems, order U{3,4,5}, n_i U[20,60],
# inner ranks U[2,8] (clipped to feasibility), FP32, noise 1e-3, J=1024, lambda=1e-3
BATCH = dict(count=256, J=1024, lam=1e-3, noise=1e-3)


def cpu_info():
    """Host CPU description from /proc/cpuinfo (first processor) and the
    affinity mask."""
    info, first, procs, packages = {}, True, 0, set()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if procs:
                        first = False
                    continue
                key, val = (x.strip() for x in line.split(":", 1))
                if key == "processor":
                    procs += 1
                elif key == "physical id":
                    packages.add(val)
                elif first and key in ("vendor_id", "cpu family", "model", "model name", "stepping", "cpu MHz",
                                       "cache size", "siblings", "cpu cores"):
                    info[key.replace(" ", "_")] = val
    except OSError:
        pass
    info["logical_cpus"] = procs
    info["packages"] = len(packages) or None
    info["cpus_visible"] = len(os.sched_getaffinity(0))
    return info


def cpu_workers():
    """Oracle workers for the all-core CPU baseline, forked before anything
    touches the GPU: one per visible CPU, at most 16 (one GPU's share of
    the host)."""
    import multiprocessing
    w = max(1, min(16, len(os.sched_getaffinity(0))))
    return multiprocessing.get_context("fork").Pool(w), w


def _oracle_slab(job):
    """Worker: the oracle's data sketch of every mode over the slab
    a <= i_{d-1} < b of the FP64 sample in the file `path`; returns its own
    seconds."""
    import numpy as np
    from oracle import sketch
    path, n, a, b, hs, vs, J = job
    inner = int(np.prod(n[:-1]))
    part = np.array(np.memmap(path, dtype=np.float64, mode="r", offset=8 * a * inner, shape=((b - a) * inner,)))
    nsl = list(n[:-1]) + [b - a]
    hs2 = list(hs[:-1]) + [hs[-1][a:b]]
    vs2 = list(vs[:-1]) + [vs[-1][a:b]]
    t0 = time.perf_counter()
    for k in range(len(n)):
        sketch.data_sketch(part, nsl, k, hs2, vs2, J)
    return time.perf_counter() - t0


def cpu_baseline(X, cfg, plan, budget_entries, pool=None, workers=1):
    """FP64 oracle data sketch (numpy) on a slab of X, the first few indices
    of the last mode, all modes sketched once: on one core in this process,
    and split by last-mode index over the worker pool (all cores)."""
    import numpy as np
    import torch
    from oracle import sketch

    n = cfg["n"]
    inner = int(np.prod(n[:-1]))
    ns = max(1, min(n[-1], budget_entries // inner))
    slab = X.view(n[-1], inner)[:ns].contiguous()
    Xs = slab.to("cpu", torch.float64).numpy().reshape(-1)
    del slab
    nsl = list(n[:-1]) + [ns]
    hs, vs = [], []
    for s in range(len(n)):
        h, v = plan.get_tables(s)
        hs.append(h[: nsl[s]])
        vs.append(v[: nsl[s]])
    t0 = time.perf_counter()
    for k in range(len(n)):
        sketch.data_sketch(Xs, nsl, k, hs, vs, plan.J)
    dt1 = time.perf_counter() - t0
    entries = len(n) * Xs.size
    out = {"value": entries / dt1, "unit": "entries/s", "cores": 1, "kind": "oracle",
           "sample": "numpy FP64 data sketch of all %d modes over the slab i_%d < %d (%d entries; one core %.1f s)"
                     % (len(n), len(n) - 1, ns, Xs.size, dt1),
           "single_core": {"value": entries / dt1, "seconds": dt1},
           "host": cpu_info()}
    if pool is not None:
        # the sample goes to the workers through a memory-backed file; each
        # worker copies its slab in before its clock starts
        import tempfile
        shm_dir = None
        try:
            st = os.statvfs("/dev/shm")
            if st.f_bavail * st.f_frsize >= 2 * Xs.nbytes:
                shm_dir = "/dev/shm"
        except OSError:
            pass
        fd, path = tempfile.mkstemp(suffix=".f64", dir=shm_dir)
        try:
            with os.fdopen(fd, "wb") as f:
                Xs.tofile(f)
            jobs = [(path, nsl, a, a + 1, hs, vs, plan.J) for a in range(ns)]
            t0 = time.perf_counter()
            per = pool.map(_oracle_slab, jobs, chunksize=1)
            dtw = time.perf_counter() - t0
        finally:
            os.unlink(path)
        used = min(workers, ns)
        out.update({"value": entries / dtw, "cores": used,
                    "sample": out["sample"] + "; the same slab split by i_%d over %d worker processes: %.2f s wall"
                                              % (len(n) - 1, used, dtw),
                    "all_cores": {"value": entries / dtw, "seconds": dtw, "workers": used,
                                  "worker_seconds": round(float(sum(per)), 3),
                                  "note": "wall time includes each worker's copy of its slab from the shared file"}})
    return out


POLICY_WEIGHTS = os.path.join(ROOT, "paper_2309_08093_amd", "jpolicy_weights.npy")


def timed_plain(plan, X, cores, target, max_sweeps):
    """Fixed J and lambda.  The time to the target is the wall clock of the
    sweeps and of the exact residual check after each one (a run cannot stop
    without it), as for the policy-driven run; the sweeps alone, timed with
    events on the plan's stream, are reported as sweep_seconds."""
    import torch
    stream = plan.stream
    t_ms, hist = 0.0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max_sweeps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.als_sweep(X, cores)
        e1.record(stream)
        hist.append(plan.residual(X, cores))   # synchronises
        t_ms += e0.elapsed_time(e1)
        if hist[-1] <= target:
            break
    wall = time.perf_counter() - t0
    return {"seconds": wall, "sweep_seconds": t_ms * 1e-3, "sweeps": len(hist), "residuals": hist,
            "reached": bool(hist[-1] <= target)}


def timed_learned(plan, X, cores, params, target, max_sweeps, ref_plan=None, X_ref=None, J_min=256):
    """Policy-driven run (tt_als_run): the residual check after each sweep is
    a policy input, so the whole call, checks included, is timed."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = plan.run(X, cores, max_sweeps, target, params=params, J_min=J_min)
    torch.cuda.synchronize()
    out["seconds"] = time.perf_counter() - t0
    if ref_plan is not None:
        out["residual_vs_fp32_data"] = ref_plan.residual(X_ref, cores)
    return out


def warm(plan, X, init, dev, params=None):
    """One untimed sweep (and policy call) on scratch cores, so that first-use
    costs (code-object loading, stream creation) stay out of the timings; the
    plan is then reset to sweep 0 with its descriptor's J and lambda."""
    import paper_2309_08093_amd as tts
    import torch
    J0, lam0 = plan.get_sketch()
    c = [tts.core_to_device(x, dev) for x in init]
    if params is not None:
        plan.run(X, c, 1, 0.0, params=params)
    else:
        plan.als_sweep(X, c)
    plan.residual(X, c)
    torch.cuda.synchronize()
    plan.set_sketch(J0, lam0)
    plan.set_sweep(0)


def exact_section(cfg, X, init, args, dev):
    """The exact (unsketched) proximal ALS on the same tensor: ms per sweep,
    time to relative residual 1e-2, and the two contraction passes over X
    (the right chain of core 0 and the left interface of core d-1), each
    timed alone with its algorithmic bytes (X read once plus the first
    intermediate written)."""
    import numpy as np
    import torch
    import paper_2309_08093_amd as tts
    n, R = cfg["n"], cfg["r"]
    d = len(n)
    N = int(np.prod(n))
    xb = XBYTES[cfg["xd"]]
    wb = 8 if cfg["wd"] == "f64" else 4
    plan = tts.Plan(n, R, cfg["J"], cfg["lam"], seed=args.seed, x_dtype=cfg["xd"], work_dtype=cfg["wd"],
                    gram=cfg["gram"], device=dev, serial=True, exact=True)
    cores = [tts.core_to_device(c, dev) for c in init]
    plan.als_sweep_exact(X, cores)
    torch.cuda.synchronize()
    stream = plan.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record(stream)
    for _ in range(reps):
        plan.als_sweep_exact(X, cores)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_sweep = e0.elapsed_time(e1) / reps
    passes = {}
    # the right chain of core 0 contracts the two slowest modes in one pass
    # (merged cores) when d >= 3, so its first write is N / (n_{d-2} n_{d-1})
    # R_{d-2} values
    right_inter = N // (n[-1] * n[-2]) * R[d - 2] if d >= 3 else N // n[-1] * R[d - 1]
    for k, name, inter in ((0, "right_chain_k0", right_inter), (d - 1, "left_interfaces_k%d" % (d - 1),
                                                                N // n[0] * R[1])):
        plan.exact_rhs(X, cores, k)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            plan.exact_rhs(X, cores, k)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nbytes = N * xb + inter * wb
        passes[name] = {"ms": round(ms, 4), "bytes": nbytes, "GB/s": round(nbytes / ms / 1e6, 1),
                        "frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBPS, 4)}
    cores2 = [tts.core_to_device(c, dev) for c in init]
    plan.set_sweep(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = []
    for _ in range(30):
        hist.append(plan.als_sweep_exact(X, cores2, residual=True))
        if hist[-1] <= 1e-2:
            break
    wall = time.perf_counter() - t0
    return {"ms_per_sweep": ms_sweep, "passes_over_x": passes,
            "time_to_rel_residual_1e-2": {"seconds": wall, "sweeps": len(hist), "residuals": hist,
                                          "reached": bool(hist[-1] <= 1e-2)}}


def sparse_section(cfg, args, dev, density=0.01):
    """O(nnz) sketches of a random sparse tensor of the workload's shape: all d
    sketches from one pass over the nonzeros (tt_sketch_sparse_all)."""
    import numpy as np
    import torch
    import paper_2309_08093_amd as tts
    n = cfg["n"]
    d = len(n)
    N = int(np.prod(n))
    nnz = int(N * density)
    g = torch.Generator(device=dev)
    g.manual_seed(args.seed + 101)
    coords = torch.stack([torch.randint(0, ns, (nnz,), generator=g, device=dev, dtype=torch.int32) for ns in n],
                         dim=1).contiguous()
    vals = torch.randn(nnz, generator=g, device=dev).to(getattr(torch, {"f64": "float64", "f32": "float32",
                                                                         "bf16": "bfloat16"}[cfg["xd"]]))
    plan = tts.Plan(n, [1] * (d + 1), cfg["J"], cfg["lam"], seed=args.seed, x_dtype=cfg["xd"], work_dtype=cfg["wd"],
                    device=dev)
    plan.sketch_sparse_all(coords, vals)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(plan.stream)
    for _ in range(reps):
        plan.sketch_sparse_all(coords, vals)
    e1.record(plan.stream)
    torch.cuda.synchronize()
    plan.sync_status()
    ms = e0.elapsed_time(e1) / reps
    nbytes = nnz * (4 * d + XBYTES[cfg["xd"]])
    return {"nnz": nnz, "density": density, "ms_all_modes": round(ms, 4), "nonzeros_per_s": nnz / (ms * 1e-3),
            "sketched_entries_per_s": d * nnz / (ms * 1e-3), "input_GB/s": round(nbytes / ms / 1e6, 1),
            "note": "one pass over COO coordinates and values; FP64 atomics into the %d sketches" % d}


# the synthetic workloads of Sec. 5: order 6, n_k = 10 (10^6 entries), FP32,
# from zero cores, 100 sweeps; name: (tensor, rank, sketch size, sigma)
PAPER_WORKLOADS = [
    ("tt6_r5_noise0.1_m150_sigma0.5", ("tt6", 0.1), 5, 150, 0.5),
    ("tt6_r5_noise0.01_m200_sigma0.5", ("tt6", 0.01), 5, 200, 0.5),
    ("sinc_r5_m45_sigma0", ("fn", "sinc"), 5, 45, 0.0),
    ("sinc_r5_m45_sigma0.5", ("fn", "sinc"), 5, 45, 0.5),
    ("osc_r13_m1000_sigma0.5", ("fn", "osc"), 13, 1000, 0.5),
]


def paper_workloads_section(args, dev, sweeps=100, exact_sweeps=10, runs=10):
    """Sec. 5 synthetic workloads: per workload, `sweeps` sketched sweeps
    (TT-TS) from zero cores with per-sweep HIP-event times (median), the final
    exact residual and core change (the paper's accuracy measure), and
    `exact_sweeps` unsketched sweeps (TT-ALS) for the same tensor; for the
    random-TT workloads also `runs` independent runs advanced as one batch
    with the sweep captured in a hipGraph (the paper averages ten runs)."""
    import numpy as np
    import torch
    import paper_2309_08093_amd as tts
    import synth
    n = synth.PAPER_N

    def start(R, lam):
        # zero cores as in the paper; sigma = 0 starts from Gaussian cores, since
        # the zero start's first subproblems are singular without the proximal term
        return synth.random_cores(n, R, 5) if lam == 0.0 else synth.zero_cores(n, R)

    def tensor(src, seed):
        if src[0] == "tt6":
            return synth.paper_tt6(seed, src[1])[0]
        return synth.function_tensor(src[1])

    out = {}
    for name, src, r, J, lam in PAPER_WORKLOADS:
        R = synth.function_ranks(r)
        Xh = tensor(src, args.seed)
        X = torch.from_numpy(Xh.astype(np.float32)).to(dev)
        ent = {"ranks": R, "J": J, "sigma": lam}
        try:
            plan = tts.Plan(n, R, J, lam, seed=args.seed, device=dev, exact=True)
            cores = [tts.core_to_device(c, dev) for c in start(R, lam)]
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(sweeps + 1)]
            torch.cuda.synchronize()
            ev[0].record(plan.stream)
            prev = None
            for t in range(sweeps):
                if t == sweeps - 1:
                    prev = [c.clone() for c in cores]
                    ev[t].record(plan.stream)   # the copy stays out of the last interval
                plan.als_sweep(X, cores)
                ev[t + 1].record(plan.stream)
            torch.cuda.synchronize()
            per = [ev[t].elapsed_time(ev[t + 1]) for t in range(sweeps)]
            ent["tt_ts"] = {"sweeps": sweeps, "ms_per_sweep_median": round(float(np.median(per)), 4),
                            "ms_total": round(float(sum(per)), 3), "rel_residual": plan.residual(X, cores),
                            "core_change_last_sweep": plan.core_change(prev, cores)}
            ex = [tts.core_to_device(c, dev) for c in start(R, lam)]
            exr, exms = [], []
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            for t in range(exact_sweeps):
                e0.record(plan.stream)
                plan.als_sweep_exact(X, ex)
                e1.record(plan.stream)
                torch.cuda.synchronize()
                exms.append(e0.elapsed_time(e1))
            ent["tt_als_exact"] = {"sweeps": exact_sweeps, "ms_per_sweep_median": round(float(np.median(exms)), 4),
                                   "rel_residual": plan.residual(X, ex)}
            plan.sync_status()
        except tts.TTError as e:
            ent["error"] = str(e)
        if src[0] == "tt6":
            probs = [dict(n=n, ranks=R, J=J, lam=lam, seed=args.seed + i) for i in range(runs)]
            Xs = [torch.from_numpy(tensor(src, args.seed + 100 + i).astype(np.float32)).to(dev) for i in range(runs)]
            b = tts.Batch(probs, device=dev)
            b.set_graph(True)
            cb = [[tts.core_to_device(c, dev) for c in synth.zero_cores(n, R)] for _ in range(runs)]
            b.sweep(Xs, cb)                      # capture
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(b.stream)
            for _ in range(sweeps - 2):
                b.sweep(Xs, cb)
            e1.record(b.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / (sweeps - 2)
            res = b.sweep(Xs, cb, residuals=True)
            ent["batched_runs"] = {"runs": runs, "sweeps": sweeps, "ms_per_sweep_all_runs": round(ms, 4),
                                   "rel_residual_mean": float(np.mean(res)), "rel_residual_max": float(np.max(res))}
            del b, Xs, cb
        out[name] = ent
        print("[bench] %s %s" % (name, json.dumps(ent)), file=sys.stderr, flush=True)
    return out


def compare_forms(seed, dev, log):
    """Time to a target relative residual: plain FP32 at fixed J vs mixed
    precision (BF16 X, BF16 MFMA Gram) with the learned sketch-size policy,
    whose choices include the unsketched update (J recorded as 0)."""
    import numpy as np
    import torch
    import paper_2309_08093_amd as tts
    from paper_2309_08093_amd import jpolicy
    import synth
    if not os.path.exists(POLICY_WEIGHTS):
        return {"error": "no trained policy weights at %s" % POLICY_WEIGHTS}
    pol = jpolicy.Policy.load(POLICY_WEIGHTS, device=dev)
    out = {}
    # 64^5 random TT, ranks 8, noise 1e-3: FP32 twin vs BF16 storage
    n, R = [64] * 5, [1, 8, 8, 8, 8, 1]
    log("[bench] compare on 64^5: plain FP32 J=3000 vs mixed + learned J")
    X32, _ = synth.tt_tensor_device(n, R, 1e-3, seed, dtype="f32", device=dev)
    X16 = X32.to(torch.bfloat16)
    init = synth.random_cores(n, R, seed + 1)
    p32 = tts.Plan(n, R, 3000, 1e-3, seed=seed, x_dtype="f32", work_dtype="f32", device=dev)
    p16 = tts.Plan(n, R, 8000, 1e-3, seed=seed, x_dtype="bf16", work_dtype="f32", gram="bf16", device=dev,
                   exact=True)
    warm(p32, X32, init, dev)
    warm(p16, X16, init, dev, params=pol.params)
    c = [tts.core_to_device(x, dev) for x in init]
    plain = timed_plain(p32, X32, c, 1e-2, 30)
    c = [tts.core_to_device(x, dev) for x in init]
    mixed = timed_learned(p16, X16, c, pol.params, 1e-2, 30, ref_plan=p32, X_ref=X32)
    # the precision form alone, at the plain form's fixed J (same run loop)
    p16f = tts.Plan(n, R, 3000, 1e-3, seed=seed, x_dtype="bf16", work_dtype="f32", gram="bf16", device=dev)
    warm(p16f, X16, init, dev)
    c = [tts.core_to_device(x, dev) for x in init]
    mixed_fixed = timed_learned(p16f, X16, c, None, 1e-2, 30)
    out["tt_64x5_r8"] = {"target": 1e-2, "plain_fp32_J3000": plain, "mixed_bf16_learned": mixed,
                         "mixed_bf16_J3000": mixed_fixed,
                         "speedup": plain["seconds"] / mixed["seconds"] if mixed.get("reached") else None}
    del X32, X16, p32, p16, p16f
    torch.cuda.empty_cache()
    # video-shaped smooth tensor 240x320x3x100, ranks 12: the 1e-2 noise is a
    # relative floor of 0.032, rank-12 truncation leaves 0.085 (TT-SVD) and the
    # sketched sweeps level off at 0.15-0.20 for J in [500, 8000], so the
    # target is 0.2
    n, R = [240, 320, 3, 100], [1, 12, 12, 12, 1]
    tgt = 0.2
    log("[bench] compare on 240x320x3x100: plain FP32 fixed J grid vs mixed + learned J")
    Xh = synth.sinusoid_tensor_host(n, 20, 1e-2, seed)
    X32 = torch.from_numpy(Xh).to(dev, torch.float32)
    X16 = torch.from_numpy(Xh).to(dev).to(torch.bfloat16)
    del Xh
    init = synth.random_cores(n, R, seed + 3)
    grid = {}
    for J in (500, 1000, 2000, 3000, 4000, 8000):
        p = tts.Plan(n, R, J, 1e-3, seed=seed, x_dtype="f32", work_dtype="f32", device=dev)
        warm(p, X32, init, dev)
        c = [tts.core_to_device(x, dev) for x in init]
        grid[J] = timed_plain(p, X32, c, tgt, 30)
        del p
    reached = {J: r["seconds"] for J, r in grid.items() if r["reached"]}
    bestJ = min(reached, key=reached.get) if reached else None
    p16 = tts.Plan(n, R, 8000, 1e-3, seed=seed, x_dtype="bf16", work_dtype="f32", gram="bf16", device=dev,
                   exact=True)
    pref = tts.Plan(n, R, 3000, 1e-3, seed=seed, x_dtype="f32", work_dtype="f32", device=dev)
    warm(p16, X16, init, dev, params=pol.params)
    c = [tts.core_to_device(x, dev) for x in init]
    mixed = timed_learned(p16, X16, c, pol.params, tgt, 30, ref_plan=pref, X_ref=X32)
    out["video_240x320x3x100_r12"] = {
        "target": tgt, "plain_fp32": {str(J): r for J, r in grid.items()}, "plain_best_J": bestJ,
        "mixed_bf16_learned": mixed,
        "speedup_vs_J3000": grid[3000]["seconds"] / mixed["seconds"] if grid[3000]["reached"] and mixed["reached"]
        else None,
        "speedup_vs_best_fixed_J": reached[bestJ] / mixed["seconds"] if bestJ and mixed["reached"] else None}
    return out


def batched_section(args, dev, steps, warmup, cache=None):
    """Batched workload: one step = one batched sweep (captured in a hipGraph)
    of every problem; returns the timing, the per-step sketch launches and
    the dominant launch's roofline."""
    import numpy as np
    import torch
    import paper_2309_08093_amd as tts
    import synth

    def log(m):
        print(m, file=sys.stderr, flush=True)

    shapes = synth.batched_shapes(BATCH["count"], args.seed)
    probs = [dict(n=n, ranks=R, J=BATCH["J"], lam=BATCH["lam"], seed=args.seed + 17 * i)
             for i, (n, R) in enumerate(shapes)]
    Ns = [int(np.prod(p["n"])) for p in probs]
    ds = [len(p["n"]) for p in probs]
    log("[bench] generating %d problems, %d entries (%.1f GB FP32)" % (len(probs), sum(Ns), 4e-9 * sum(Ns)))
    Xs = [synth.tt_tensor_device(p["n"], p["ranks"], BATCH["noise"], args.seed + 31 * i, dtype="f32", device=dev)[0]
          for i, p in enumerate(probs)]
    batch = tts.Batch(probs, device=dev)
    cores = [[tts.core_to_device(c, dev) for c in synth.random_cores(p["n"], p["ranks"], args.seed + 7 * i + 1)]
             for i, p in enumerate(probs)]
    log("[bench] autotune")
    t_tune = time.perf_counter()
    batch.autotune(Xs, reps=2, cache=cache)
    t_tune = time.perf_counter() - t_tune
    tuning = batch.get_tuning()
    batch.set_graph(True)
    log("[bench] warmup %d sweeps (the first captures the graph)" % max(1, warmup))
    for _ in range(max(1, warmup)):
        batch.sweep(Xs, cores)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    log("[bench] timing %d batched sweeps" % steps)
    t0 = time.perf_counter()
    evs[0].record(stream)
    for t in range(steps):
        batch.sweep(Xs, cores)
        evs[t + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [evs[t].elapsed_time(evs[t + 1]) for t in range(steps)]
    ms_per_step = float(np.median(per))
    entries = sum(d * N for d, N in zip(ds, Ns))
    # the batched data-sketch launches, one step at a time, timed with events on
    # the stream they run on.  Problems whose plans take Y_1 from the outer
    # sketch of the k = 0 pass: step 0 writes that sketch (J n_0 n_1 FP32
    # values) and reads it back for Y_0 (k_bsketch_0), and step 1 reads it
    # instead of X.
    fused = [batch.sketch_sources(i)[1] == 0 if len(p["n"]) > 1 else False for i, p in enumerate(probs)]
    zo = [4 * p["J"] * p["n"][0] * p["n"][1] if f else 0 for p, f in zip(probs, fused)]
    sk = {}
    for k in range(max(ds)):
        nbytes = 4 * sum(N for d, N in zip(ds, Ns) if d > k)
        if k == 0:
            nbytes += 2 * sum(zo)
        elif k == 1:
            nbytes = 4 * sum(N for d, N, f in zip(ds, Ns, fused) if d > 1 and not f) + sum(zo)
        batch.sketch_launch(Xs, k)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            batch.sketch_launch(Xs, k)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        kern = batch.sketch_kernel(k)
        if k == 0 and any(fused):
            kern = "kb_zo+" + kern
        if k == 1 and any(fused):
            kern = "kb_y1_outer+" + kern
        sk[k] = {"kernel": kern if k == 0 else kern + "+k_breduce", "avg_launch_ms": round(ms, 4),
                 "bytes": nbytes, "GB/s": round(nbytes / ms / 1e6, 1),
                 "frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBPS, 4)}
    dom = max(sk, key=lambda k: sk[k]["avg_launch_ms"])   # the step with the longest sketch launch
    rf = {"bound": "hbm", "achieved": sk[dom]["GB/s"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
          "frac": sk[dom]["frac"], "traffic": stored_traffic("k_bsketch", "c4", "batch.hip", step=dom),
          "kernel": "%s (step %d)" % (sk[dom]["kernel"], dom),
          "avg_launch_ms": sk[dom]["avg_launch_ms"], "bytes_per_launch": sk[dom]["bytes"]}
    res = batch.sweep(Xs, cores, residuals=True)
    out = {"value": entries / (ms_per_step * 1e-3), "unit": "entries/s", "ms_per_step": ms_per_step,
           "ms_per_step_note": "median of %d graph-replayed sweeps; mean %.3f" % (steps, sum(per) / steps),
           "workload": "%d independent random TTs, order U{3,4,5}, n_i U[20,60], ranks U[2,8], FP32, noise 1e-3, "
                       "J=%d, lambda=%g; one batched sweep per step, captured in a hipGraph"
                       % (BATCH["count"], BATCH["J"], BATCH["lam"]),
           "problems": len(probs), "total_entries": sum(Ns),
           "problems_with_outer_sketch": int(sum(fused)),
           "tuning": {"steps": tuning, "seconds": round(t_tune, 3),
                      "from_cache": bool(getattr(batch, "tuned_from_cache", False))},
           "hbm_gbps_sweep": 4 * entries / (ms_per_step * 1e-3) / 1e9, "wall_s_timed": wall, "roofline": rf,
           "batched_sketch_steps": sk,
           "residuals_after": {"median": float(np.median(res)), "max": float(np.max(res))}}
    del Xs, cores, batch
    torch.cuda.empty_cache()
    return out


def run_batched(args):
    """The batched workload as the bench line itself (--config c4)."""
    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    b = batched_section(args, dev, args.steps, args.warmup, cache=args.tune_cache)
    out = {
        "metric": "sketched X entries/s (HBM GB/s) + time-to-rel-residual 1e-2, mixed vs plain FP32",
        "value": b["value"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": b["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": b["workload"], "problems": b["problems"], "total_entries": b["total_entries"],
                   "problems_with_outer_sketch": b["problems_with_outer_sketch"], "tuning": b["tuning"]},
        "hbm_gbps_sweep": b["hbm_gbps_sweep"], "wall_s_timed": b["wall_s_timed"], "roofline": b["roofline"],
        "batched_sketch_steps": b["batched_sketch_steps"], "residuals_after": b["residuals_after"],
    }
    print(json.dumps(out), flush=True)


def source_digest(source="k_sketch.hip"):
    """sha256 of a data-sketch kernel source: a stored counter reading is
    used only while the kernel it was taken from is unchanged."""
    import hashlib
    path = os.path.join(ROOT, "paper_2309_08093_amd", "csrc", source)
    try:
        return hashlib.sha256(open(path, "rb").read()).hexdigest()
    except OSError:
        return None


def stored_traffic(kernel, config, source="k_sketch.hip", step=None):
    """HBM bytes per launch of `kernel` on `config` from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a device copy of known size),
    or None if there is none for the current kernel source."""
    tag = PROFILE_TAG.get(config, config)
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s_%s.txt" % (kernel, tag))
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        if ln.startswith("JSON: "):
            rec = json.loads(ln[6:])
            if rec.get("source_sha256") == source_digest(source) and rec.get("step") == step:
                return rec["traffic_bytes_per_launch"]
    return None


def probe_traffic(plan, X, d, J, n, dev):
    """The data sketches of a sweep as the sweep runs them (tt_sketch_tensor_all:
    the fused k = 0 pass when the plan fuses, then the other passes), one
    launch of every single-mode data sketch, and one device-to-device copy of
    X, bracketed by prints: the workload of the FETCH_SIZE / WRITE_SIZE runs."""
    import torch
    Ys = [torch.empty(J * n[k], dtype=plan.wdtype, device=dev) for k in range(d)]
    for k in range(d):                      # warm (fibre lists, caches of tables)
        plan.sketch_tensor(X, k, Ys[k])
    plan.sketch_tensor_all(X)
    torch.cuda.synchronize()
    plan.sketch_tensor_all(X)
    torch.cuda.synchronize()
    print("[probe] all sketches of a sweep, sources %s" % (plan.sketch_sources(),), flush=True)
    for k in range(d):
        plan.sketch_tensor(X, k, Ys[k])
        torch.cuda.synchronize()
        print("[probe] sketch k=%d kernel=%s" % (k, plan.sketch_kernel(k)), flush=True)
    dst = torch.empty_like(X)
    dst.copy_(X)
    torch.cuda.synchronize()
    print("[probe] copy bytes=%d" % (X.numel() * X.element_size()), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS) + ["c4"])
    ap.add_argument("--seed", type=int, default=2023)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-target", action="store_true")
    ap.add_argument("--no-isolated", action="store_true",
                    help="skip the isolated per-mode sketch timings (profile runs of the timed sweeps alone)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the mixed + learned-J vs plain FP32 time-to-target comparison")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact (unsketched) sweeps")
    ap.add_argument("--no-sparse", action="store_true", help="skip the sparse-input sketch timing")
    ap.add_argument("--no-paper-workloads", action="store_true",
                    help="skip the order-6 synthetic workloads of the paper's experiments")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched workload (256 uneven TTs) in the default line")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file the batched autotuner reads its choices from and writes them to")
    ap.add_argument("--cpu-entries", type=int, default=128_000_000)
    ap.add_argument("--overlap", action="store_true",
                    help="the overlapped schedule (data sketches on a second stream beside the core updates; "
                         "the library's default and this script's)")
    ap.add_argument("--serial", action="store_true", help="time the serial schedule instead of the overlapped one")
    ap.add_argument("--reserve-cus", type=int, default=None,
                    help="CUs kept free of the overlapped data sketches (library default if omitted)")
    ap.add_argument("--probe-traffic", action="store_true",
                    help="run each data sketch once and one device copy of X, then exit (for HBM counter runs)")
    args = ap.parse_args()
    if args.serial and args.overlap:
        ap.error("--serial and --overlap together")
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the data sketch would shard by slabs of the last mode plus one all-reduce of J x n_k "
              "per core update); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline's workers are forked before torch or HIP is loaded
    pool, workers = (None, 1)
    if not args.no_cpu_baseline and args.config != "c4" and not args.probe_traffic:
        pool, workers = cpu_workers()

    import numpy as np
    import torch
    import paper_2309_08093_amd as tts
    import synth

    if args.config == "c4":
        return run_batched(args)
    cfg = CONFIGS[args.config]
    n, R, J, lam = cfg["n"], cfg["r"], cfg["J"], cfg["lam"]
    d = len(n)
    N = int(np.prod(n))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print("[bench] generating %s on the device" % cfg["desc"], file=sys.stderr, flush=True)
    X, _ = synth.tt_tensor_device(n, R, cfg["noise"], args.seed, dtype=cfg["xd"], device=dev)
    init = synth.random_cores(n, R, args.seed + 1)
    plan = tts.Plan(n, R, J, lam, seed=args.seed, x_dtype=cfg["xd"], work_dtype=cfg["wd"], gram=cfg["gram"],
                    device=dev, serial=args.serial)
    if args.reserve_cus is not None:
        plan.set_overlap(args.reserve_cus)
    cores = [tts.core_to_device(c, dev) for c in init]
    torch.cuda.synchronize()
    if args.probe_traffic:
        probe_traffic(plan, X, d, J, n, dev)
        return

    print("[bench] warmup %d sweeps" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        plan.als_sweep(X, cores)
    torch.cuda.synchronize()

    print("[bench] timing %d sweeps" % args.steps, file=sys.stderr, flush=True)
    # only the data-sketch launches are bracketed by events in the timed
    # sweeps: every event record leaves a gap of a few microseconds on the
    # GPU, and timing all ~60 launches of a sweep would lengthen it by ~4 %
    plan.profile(True, ["sketch_k0", "sketch_k"])
    plan.profile_read()
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for t in range(args.steps):
        plan.als_sweep(X, cores)
        evs[t + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    ms_total = evs[0].elapsed_time(evs[-1])
    per_step = [evs[t].elapsed_time(evs[t + 1]) for t in range(args.steps)]
    ms_per_step = float(np.median(per_step))
    entries_per_s = d * N / (ms_per_step * 1e-3)
    xbytes = XBYTES[cfg["xd"]]

    # the data sketches dominate: the k = 0 pass (which also writes the
    # J x n_0 x n_1 outer sketch when Y_1 is derived from it) and the k >= 2
    # (or k >= 1) passes, one launch each per sweep
    src = plan.sketch_sources()
    fused = src[1] == 0
    wbytes = 8 if cfg["wd"] == "f64" else 4
    outer_bytes = J * n[0] * n[1] * wbytes if fused else 0

    def roof(cls, kernel, nbytes, traffic_kernels):
        ms, cnt = prof[cls]
        if cnt == 0:
            return None
        avg_s = ms / cnt * 1e-3
        gbps = nbytes / avg_s / 1e9
        parts = [stored_traffic(t, args.config) for t in traffic_kernels]
        return {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": None if None in parts else sum(parts),
                "kernel": kernel, "avg_launch_ms": round(ms / cnt, 4), "launches": cnt,
                "bytes_per_launch": nbytes}

    # the inner-sketch pass of mode 2 (k_sketch_zi: X read, the J x n_2...n_{d-1}
    # sketch of every slab over modes 0 and 1 written) when Y_3.. come from it
    # joint: the k = 0 pass (k_sketch_zoi) writes both intermediates, and
    # every Y_k comes from them (one pass over X)
    joint = d >= 4 and all(src[k] == 0 for k in range(1, d))
    inner = joint or (d >= 4 and all(src[k] == 2 for k in range(3, d)))
    inner_bytes = J * (N // (n[0] * n[1])) * wbytes if inner else 0
    kern_k = ["k_sketch_zi"] if inner else sorted(set(plan.sketch_kernel(k) for k in range(1, d) if src[k] == k))
    rfk = roof("sketch_k", "+".join(kern_k), N * xbytes + inner_bytes, ["+".join(kern_k)])
    # the fused k = 0 pass: k_sketch_zo (X read, outer sketch written) and
    # k_sketch_y0_zo (Y_0 from the outer sketch, read once)
    k0_kernels = (["k_sketch_zoi", "k_sketch_y0_zo"] if joint else ["k_sketch_zo", "k_sketch_y0_zo"] if fused
                  else [plan.sketch_kernel(0)])
    k0_bytes = N * xbytes + 2 * outer_bytes + (inner_bytes if joint else 0)
    rf0 = roof("sketch_k0", "+".join(k0_kernels), k0_bytes, k0_kernels)
    rf, rf_other = (rfk, rf0) if prof["sketch_k"][0] >= prof["sketch_k0"][0] else (rf0, rfk)
    # per-class times from separate sweeps with every class timed
    n_cls = min(args.steps, 5)
    plan.profile(True)
    plan.profile_read()
    for _ in range(n_cls):
        plan.als_sweep(X, cores)
    prof_all = plan.profile_read()
    plan.profile(False)
    kernels = {k: round(v[0] / n_cls, 4) for k, v in prof_all.items()}

    out = {
        "metric": "sketched X entries/s (HBM GB/s) + time-to-rel-residual 1e-2, mixed vs plain FP32",
        "value": entries_per_s,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_note": "median of the timed sweeps (HIP events between sweeps); mean %.4f, min %.4f, max %.4f"
                            % (ms_total / args.steps, min(per_step), max(per_step)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": cfg["xd"],
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "n": n, "ranks": R, "J": J, "lambda": lam,
                   "step": "one sweep of Algorithm 1 (%d data sketches from %d passes over X)"
                           % (d, sum(1 for k in range(d) if src[k] == k)),
                   "sketch_sources": src,
                   "schedule": "serial" if args.serial else "data sketches overlapped on a second stream",
                   "reserved_cus": None if args.serial else ("library default" if args.reserve_cus is None
                                                             else args.reserve_cus)},
        "hbm_gbps_sweep": (sum(1 for k in range(d) if src[k] == k) * N * xbytes + 3 * outer_bytes
                           + (d - 1) * inner_bytes) / (ms_per_step * 1e-3) / 1e9,
        "hbm_gbps_sweep_note": "passes over X plus the outer sketch written once and read twice (Y_0, Y_1) and the "
                               "inner sketch written once and read d - 2 times (Y_2 .. Y_{d-1}), per sweep time",
        "wall_s_timed": wall,
        "roofline": rf,
        "roofline_other_sketch": rf_other,
        "kernels_ms_per_step": kernels,
        "kernels_ms_per_step_note": "%d further sweeps with every kernel class timed by HIP events" % n_cls,
    }

    # the other schedule, for comparison: the serial one runs every kernel on
    # the plan's stream; the overlapped one runs the data sketches beside the
    # core updates
    if not args.no_isolated:
        plan2 = tts.Plan(n, R, J, lam, seed=args.seed, x_dtype=cfg["xd"], work_dtype=cfg["wd"], gram=cfg["gram"],
                         device=dev, serial=not args.serial)
        cores3 = [tts.core_to_device(c, dev) for c in init]
        for _ in range(max(3, args.warmup)):
            plan2.als_sweep(X, cores3)
        torch.cuda.synchronize()
        evs2 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        evs2[0].record(stream)
        for t in range(args.steps):
            plan2.als_sweep(X, cores3)
            evs2[t + 1].record(stream)
        torch.cuda.synchronize()
        ms2 = float(np.median([evs2[t].elapsed_time(evs2[t + 1]) for t in range(args.steps)]))
        if args.serial:
            out["overlapped_schedule"] = {
                "ms_per_step": ms2, "value": d * N / (ms2 * 1e-3), "unit": "entries/s",
                "reserved_cus": "the library default (none when the k = 0 pass writes both intermediates, else the "
                                "CUs of one XCD)",
                "note": "data sketches on a side stream beside the core updates; median over the timed sweeps"}
        else:
            out["serial_schedule"] = {"ms_per_step": ms2, "value": d * N / (ms2 * 1e-3), "unit": "entries/s",
                                      "note": "every kernel on the plan's stream; median over the timed sweeps"}
        del plan2, cores3

    # each data sketch alone on the plan's stream (no concurrent core updates)
    iso = {}
    if args.no_isolated:
        d_iso = 0
    else:
        d_iso = d
    Ytmp = [torch.empty(J * n[k], dtype=plan.wdtype, device=dev) for k in range(d)]
    for k in range(d_iso):
        plan.sketch_tensor(X, k, Ytmp[k])
        torch.cuda.synchronize()
        plan.profile(True)
        plan.profile_read()
        for _ in range(5):
            plan.sketch_tensor(X, k, Ytmp[k])
        pr = plan.profile_read()
        plan.profile(False)
        ms, cnt = pr["sketch_k0" if k == 0 else "sketch_k"]
        gbps = N * xbytes / (ms / cnt * 1e-3) / 1e9
        iso[k] = {"kernel": plan.sketch_kernel(k), "avg_launch_ms": round(ms / cnt, 4), "GB/s": round(gbps, 1),
                  "frac": round(gbps / HBM_PEAK_GBPS, 4)}
    out["sketch_isolated"] = iso
    del Ytmp
    if not args.no_isolated:
        # all d sketches of a sweep alone (tt_sketch_tensor_all): the fused
        # k = 0 pass, the k >= 2 passes, and the rest (sorts, Y_1 stage, sums)
        plan.sketch_tensor_all(X)
        torch.cuda.synchronize()
        plan.profile(True, ["sketch_k0", "sketch_k", "sketch_aux"])
        plan.profile_read()
        for _ in range(5):
            plan.sketch_tensor_all(X)
        pr = plan.profile_read()
        plan.profile(False)
        k0ms = pr["sketch_k0"][0] / 5
        out["sketch_all_isolated"] = {
            "ms_per_call": {c: round(pr[c][0] / 5, 4) for c in ("sketch_k0", "sketch_k", "sketch_aux")},
            "k0_pass": {"kernel": "+".join(k0_kernels), "bytes": k0_bytes,
                        "GB/s": round(k0_bytes / (k0ms * 1e-3) / 1e9, 1),
                        "frac": round(k0_bytes / (k0ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}}
        if inner and not joint:
            kms = pr["sketch_k"][0] / 5
            kb = N * xbytes + inner_bytes
            out["sketch_all_isolated"]["inner_pass"] = {
                "kernel": "k_sketch_zi", "bytes": kb, "GB/s": round(kb / (kms * 1e-3) / 1e9, 1),
                "frac": round(kb / (kms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}

    if not args.no_time_to_target:
        print("[bench] time to relative residual 1e-2", file=sys.stderr, flush=True)
        cores2 = [tts.core_to_device(c, dev) for c in init]
        plan.set_sweep(0)
        tt = timed_plain(plan, X, cores2, 1e-2, 30)
        tt["form"] = "plain " + cfg["xd"]
        out["time_to_rel_residual_1e-2"] = tt

    if not args.no_sparse:
        print("[bench] sparse sketches", file=sys.stderr, flush=True)
        out["sparse"] = sparse_section(cfg, args, dev)

    if not args.no_paper_workloads:
        print("[bench] paper's synthetic workloads", file=sys.stderr, flush=True)
        out["paper_workloads"] = paper_workloads_section(args, dev)

    if not args.no_exact:
        print("[bench] exact sweeps", file=sys.stderr, flush=True)
        out["exact"] = exact_section(cfg, X, init, args, dev)

    if not args.no_batched:
        print("[bench] batched workload", file=sys.stderr, flush=True)
        out["batched_256_uneven_tt"] = batched_section(args, dev, 5, 1, cache=args.tune_cache)

    if not args.no_compare:
        out["mixed_learned_vs_plain"] = compare_forms(args.seed, dev,
                                                      lambda m: print(m, file=sys.stderr, flush=True))

    if not args.no_cpu_baseline:
        print("[bench] CPU baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(X, cfg, plan, args.cpu_entries, pool, workers)
    if pool is not None:
        pool.close()
        pool.join()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
