"""Seeded synthetic inputs for the TT-TensorSketch path and its oracle.

This module only makes inputs: random TT cores, the dense tensor they
represent plus Gaussian noise, smooth separable signals, and the starting
cores handed to the solver.  It holds none of the method's arithmetic (no
hashing, sketching, solving or orthogonalisation) and imports neither the
oracle nor the HIP package; both sides receive the same arrays from here.

Layout: a d-way tensor is a flat array with i_0 varying fastest (numpy
order='F').  On a torch device the flat tensor is contiguous and equals a
row-major tensor of shape (n_{d-1}, ..., n_0).
"""
import numpy as np

try:  # torch is optional for the host-only paths
    import torch
except Exception:  # pragma: no cover
    torch = None


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def tt_ranks(d, r):
    """(1, r, ..., r, 1)."""
    return [1] + [int(r)] * (d - 1) + [1]


def clip_ranks(n, ranks):
    """Clip inner ranks so that R[k] <= R[k-1] n[k-1] and R[k] <= n[k] R[k+1]."""
    R = list(ranks)
    d = len(n)
    for k in range(1, d):
        R[k] = min(R[k], R[k - 1] * n[k - 1])
    for k in range(d - 1, 0, -1):
        R[k] = min(R[k], n[k] * R[k + 1])
    return R


def random_cores(n, ranks, seed, scale=1.0):
    """Cores (R[k], n[k], R[k+1]) with iid N(0, scale^2) entries, FP64."""
    g = rng(seed)
    return [scale * g.standard_normal((ranks[k], n[k], ranks[k + 1])) for k in range(len(n))]


def zero_cores(n, ranks):
    return [np.zeros((ranks[k], n[k], ranks[k + 1])) for k in range(len(n))]


def _chain_left(cores, m):
    T = np.ones((1, 1))
    for G in cores[:m]:
        r0, nk, r1 = G.shape
        T = (T @ G.reshape(r0, nk * r1, order="F")).reshape(-1, r1, order="F")
    return T                                    # prod_{k<m} n_k  x  R[m]


def _chain_right(cores, m):
    U = np.ones((1, 1))
    for G in reversed(cores[m:]):
        r0, nk, r1 = G.shape
        U = (G.reshape(r0 * nk, r1, order="F") @ U).reshape(r0, -1, order="F")
    return U                                    # R[m]  x  prod_{k>=m} n_k


def dense_from_cores_host(cores):
    """Dense tensor of a TT (FP64, flat, i_0 fastest)."""
    m = max(1, len(cores) // 2)
    return (_chain_left(cores, m) @ _chain_right(cores, m)).reshape(-1, order="F")


def tt_tensor_host(n, ranks, noise, seed, scale=1.0):
    """(X fp64 flat, true cores).  X = [[cores]] + noise * N(0,1) iid."""
    cores = random_cores(n, ranks, seed, scale)
    X = dense_from_cores_host(cores)
    if noise:
        X = X + noise * rng(seed + 7919).standard_normal(X.size)
    return X, cores


def to_dtype_host(X, dtype):
    """Round a host FP64 array to 'f64' | 'f32' | 'bf16' (RNE).  Returns a
    numpy array (float64/float32) or a torch CPU bf16 tensor."""
    if dtype == "f64":
        return np.ascontiguousarray(X, dtype=np.float64)
    if dtype == "f32":
        return np.ascontiguousarray(X, dtype=np.float32)
    if dtype == "bf16":
        return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(torch.bfloat16)
    raise ValueError(dtype)


def upcast_host(X):
    """Host FP64 copy of what ``to_dtype_host`` returned."""
    if torch is not None and isinstance(X, torch.Tensor):
        return X.to(torch.float64).numpy()
    return np.asarray(X, dtype=np.float64)


TORCH_DTYPES = {"f64": "float64", "f32": "float32", "bf16": "bfloat16"}


def tt_tensor_device(n, ranks, noise, seed, dtype="f32", device="cuda", scale=1.0, chunk=1 << 26):
    """Large inputs built on the device: X = [[cores]] + noise, stored in
    ``dtype``.  The product of the two half-chains is formed in FP32 (FP64
    when dtype == 'f64') by torch.matmul, the noise by a seeded torch
    generator; results are deterministic for a given device and seed."""
    tdt = getattr(torch, TORCH_DTYPES[dtype])
    cdt = torch.float64 if dtype == "f64" else torch.float32
    cores = random_cores(n, ranks, seed, scale)
    m = max(1, len(n) // 2)
    L = torch.from_numpy(_chain_left(cores, m)).to(device=device, dtype=cdt)     # NL x r
    Rt = torch.from_numpy(_chain_right(cores, m)).to(device=device, dtype=cdt)   # r x NR
    NL, NR = L.shape[0], Rt.shape[1]
    X = torch.empty(NL * NR, dtype=tdt, device=device)
    Xv = X.view(NR, NL)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed + 7919)
    rows = max(1, chunk // NL)
    for r0 in range(0, NR, rows):
        r1 = min(NR, r0 + rows)
        blk = Rt[:, r0:r1].t() @ L.t()                # (r1-r0) x NL, flat = col*NL + row
        if noise:
            blk += noise * torch.randn(blk.shape, generator=gen, device=device, dtype=cdt)
        Xv[r0:r1] = blk.to(tdt)
    return X, cores


def sinusoid_factors(n, terms, seed):
    """Amplitudes a_p = 1/p and per-mode factors sin(2 pi f i / n_k + phi) with
    f ~ U[0.5, 4], phi ~ U[0, 2 pi)."""
    g = rng(seed)
    facs = []
    for p in range(terms):
        facs.append([np.sin(2 * np.pi * g.uniform(0.5, 4.0) * np.arange(nk) / nk + g.uniform(0, 2 * np.pi))
                     for nk in n])
    amps = [1.0 / (p + 1) for p in range(terms)]
    return amps, facs


def sinusoid_tensor_host(n, terms=20, noise=1e-2, seed=0):
    """Sum of ``terms`` separable sinusoid products plus N(0, noise^2) noise
    (a smooth, video-shaped stand-in for the paper's real-data tensors)."""
    amps, facs = sinusoid_factors(n, terms, seed)
    X = np.zeros(int(np.prod(n)))
    for a, f in zip(amps, facs):
        t = np.array([a])
        for v in f:
            t = np.kron(v, t)                     # new mode is the slower index
        X += t
    if noise:
        X += noise * rng(seed + 104729).standard_normal(X.size)
    return X


# ---- the synthetic workloads of Sec. 5 (Experimental Results for Synthetic
# Data): order 6, n_k = 10, 10^6 entries -------------------------------------

PAPER_N = [10] * 6


def paper_tt6(seed, noise, r=5):
    """First synthetic experiment: a random TT of equal inner ranks r whose
    core entries are iid N(0, 1), plus iid N(0, noise^2) noise on every entry
    (noise is an absolute standard deviation: 0.1 or 0.01 in the paper).
    Returns (X fp64 flat, true cores)."""
    return tt_tensor_host(PAPER_N, clip_ranks(PAPER_N, tt_ranks(6, r)), noise, seed)


def function_points(name, points=10 ** 6):
    """Sample points of the second synthetic experiment: 'sinc' on [-5, 5]
    (both ends included) and 'osc' on (0, 1] (x = j / points, j = 1..points:
    the function has no value at 0)."""
    if name == "sinc":
        return np.linspace(-5.0, 5.0, points)
    if name == "osc":
        return np.arange(1, points + 1, dtype=np.float64) / points
    raise ValueError("unknown function %r" % name)


def function_tensor(name, points=10 ** 6):
    """f at the points of ``function_points``, in order, as a flat tensor with
    i_0 fastest, i.e. folded column-major into 10 x ... x 10:
    'sinc': sin(pi x) / (pi x) (1 at x = 0); 'osc': sin(4 / x) cos(x^2)."""
    x = function_points(name, points)
    if name == "sinc":
        return np.sinc(x)
    return np.sin(4.0 / x) * np.cos(x * x)


def function_ranks(r, n=PAPER_N):
    """TT ranks (1, r, ..., r, 1) clipped to what a tensor of shape n admits
    (R_1 <= n_0, R_{d-1} <= n_{d-1}, ...)."""
    return clip_ranks(n, tt_ranks(len(n), r))


def batched_shapes(count, seed, order=(3, 5), nrange=(20, 60), rrange=(2, 8)):
    """Shapes and ranks of ``count`` independent problems: order uniform in
    [order[0], order[1]], each n_i uniform in nrange, each inner rank uniform
    in rrange, clipped to feasibility."""
    g = rng(seed)
    out = []
    for _ in range(count):
        d = int(g.integers(order[0], order[1] + 1))
        n = [int(x) for x in g.integers(nrange[0], nrange[1] + 1, size=d)]
        R = [1] + [int(x) for x in g.integers(rrange[0], rrange[1] + 1, size=d - 1)] + [1]
        out.append((n, clip_ranks(n, R)))
    return out
