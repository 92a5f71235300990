"""MI355X (gfx950) randomized proximal TT-ALS with TensorSketch.

Thin Python binding over the C ABI of ``libttsketch.so`` (include/tt_sketch.h):
argument checking and marshalling only.  Every step of the method runs in the
library's HIP kernels; torch supplies device memory and the stream.  There is
no fallback: if the library is missing, importing this package raises.

Layouts (see the header): X is a contiguous device tensor whose flat order has
mode 0 fastest (a row-major torch tensor of shape (n_{d-1}, ..., n_0));
core k is a contiguous float64 device tensor of R_k * n_k * R_{k+1} entries,
first index fastest; Y and SH are column-major J x n_k and J x R_k R_{k+1}.
"""
import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import TTError, check

_lib = _abi.load()

_DT = {"f64": _abi.TT_F64, "f32": _abi.TT_F32, "bf16": _abi.TT_BF16}
_TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
_GRAM = {"work": _abi.TT_GRAM_WORK, "bf16": _abi.TT_GRAM_BF16}


def version():
    return _lib.tt_version().decode()


def core_to_device(core, device="cuda"):
    """numpy core (R_k, n_k, R_{k+1}) -> flat float64 device tensor (first index fastest)."""
    flat = np.ascontiguousarray(np.asarray(core, dtype=np.float64).reshape(-1, order="F"))
    return torch.from_numpy(flat).to(device)


def core_to_host(t, shape):
    """flat device core -> numpy (R_k, n_k, R_{k+1})."""
    return t.detach().to("cpu", torch.float64).numpy().reshape(tuple(shape), order="F")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """One TT-TS problem: shape, ranks, sketch size J, proximal lambda, seed,
    storage type of X and work type; owns a device workspace (a torch
    tensor) and runs on a HIP stream (torch's current stream by default)."""

    def __init__(self, n, ranks, J, lam, seed=0, x_dtype="f32", work_dtype="f32", gram="work",
                 device="cuda", stream=None, serial=False, fuse=None, exact=False, inner=None):
        self.n = [int(x) for x in n]
        self.ranks = [int(x) for x in ranks]
        self.d = len(self.n)
        self.J = int(J)
        self.lam = float(lam)
        self.x_dtype, self.work_dtype = x_dtype, work_dtype
        self.device = torch.device(device)
        if x_dtype not in _DT or work_dtype not in ("f64", "f32") or gram not in _GRAM:
            raise ValueError("bad dtype or gram mode")
        if len(self.ranks) != self.d + 1:
            raise ValueError("ranks must have d+1 entries")
        self._n_arr = (ctypes.c_int64 * self.d)(*self.n)
        self._r_arr = (ctypes.c_int64 * (self.d + 1))(*self.ranks)
        flags = (_abi.TT_FLAG_SERIAL if serial else 0) | (_abi.TT_FLAG_EXACT if exact else 0) | \
            {None: 0, True: _abi.TT_FLAG_FUSE, False: _abi.TT_FLAG_NO_FUSE}[fuse] | \
            {None: 0, True: _abi.TT_FLAG_INNER, False: _abi.TT_FLAG_NO_INNER}[inner]
        desc = _abi.PlanDesc(self.d, self._n_arr, self._r_arr, self.J, self.lam, int(seed) & (2 ** 64 - 1),
                             _DT[x_dtype], _DT[work_dtype], _GRAM[gram], flags)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        ws = ctypes.c_size_t(0)
        h = ctypes.c_void_p()
        check(_lib.tt_sketch_plan(ctypes.byref(desc), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(ws),
                                  ctypes.byref(h)), "tt_sketch_plan")
        self._h = h
        self.workspace_bytes = ws.value
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        check(_lib.tt_plan_bind_workspace(self._h, ctypes.c_void_p(aligned), self.workspace_bytes),
              "tt_plan_bind_workspace")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.tt_plan_destroy(h)
            self._h = None

    # -- shapes
    @property
    def N(self):
        return int(np.prod(self.n))

    def core_shape(self, k):
        return (self.ranks[k], self.n[k], self.ranks[k + 1])

    def s(self, k):
        return self.ranks[k] * self.ranks[k + 1]

    @property
    def wdtype(self):
        return _TORCH[self.work_dtype]

    # -- argument checks
    def _check_X(self, X):
        if not (isinstance(X, torch.Tensor) and X.device.type == "cuda" and X.is_contiguous()
                and X.dtype == _TORCH[self.x_dtype] and X.numel() == self.N):
            raise ValueError("X must be a contiguous %s device tensor with %d entries" % (self.x_dtype, self.N))

    def _check_work(self, T, numel, name):
        if not (isinstance(T, torch.Tensor) and T.device.type == "cuda" and T.is_contiguous()
                and T.dtype == self.wdtype and T.numel() == numel):
            raise ValueError("%s must be a contiguous %s device tensor with %d entries" % (name, self.work_dtype, numel))

    def _check_core(self, G, k):
        numel = self.ranks[k] * self.n[k] * self.ranks[k + 1]
        if not (isinstance(G, torch.Tensor) and G.device.type == "cuda" and G.is_contiguous()
                and G.dtype == torch.float64 and G.numel() == numel):
            raise ValueError("core %d must be a contiguous float64 device tensor with %d entries" % (k, numel))

    def _cores(self, cores, skip=None):
        if len(cores) != self.d:
            raise ValueError("need %d cores" % self.d)
        ptrs = []
        for k, G in enumerate(cores):
            if k == skip and G is None:
                ptrs.append(None)
                continue
            self._check_core(G, k)
            ptrs.append(G.data_ptr())
        return _abi.ptr_array(ptrs)

    # -- tables
    def set_sweep(self, t):
        check(_lib.tt_plan_set_sweep(self._h, int(t)), "tt_plan_set_sweep")

    def get_sweep(self):
        t = ctypes.c_int64()
        check(_lib.tt_plan_get_sweep(self._h, ctypes.byref(t)), "tt_plan_get_sweep")
        return t.value

    def get_tables(self, s):
        ns = self.n[s]
        h = (ctypes.c_int32 * ns)()
        v = (ctypes.c_int8 * ns)()
        check(_lib.tt_plan_get_tables(self._h, int(s), h, v), "tt_plan_get_tables")
        return np.array(h, dtype=np.int64), np.array(v, dtype=np.int8)

    def set_tables(self, s, h, v):
        ns = self.n[s]
        h = np.asarray(h, dtype=np.int32)
        v = np.asarray(v, dtype=np.int8)
        if h.shape != (ns,) or v.shape != (ns,):
            raise ValueError("tables of mode %d need %d entries" % (s, ns))
        check(_lib.tt_plan_set_tables(self._h, int(s), (ctypes.c_int32 * ns)(*h.tolist()),
                                      (ctypes.c_int8 * ns)(*v.tolist())), "tt_plan_set_tables")

    # -- the hot path
    def sketch_tensor(self, X, k, Y=None):
        self._check_X(X)
        if Y is None:
            Y = torch.empty(self.J * self.n[k], dtype=self.wdtype, device=self.device)
        self._check_work(Y, self.J * self.n[k], "Y")
        check(_lib.tt_sketch_tensor(self._h, _ptr(X), int(k), _ptr(Y)), "tt_sketch_tensor")
        return Y

    def sketch_tensor_all(self, X, Yall=None):
        """All d data sketches of the current sweep; returns [Y_0, ..., Y_{d-1}]
        as views of one buffer (Y_k flat J x n_k, column-major)."""
        self._check_X(X)
        total = self.J * sum(self.n)
        if Yall is None:
            Yall = torch.empty(total, dtype=self.wdtype, device=self.device)
        self._check_work(Yall, total, "Yall")
        check(_lib.tt_sketch_tensor_all(self._h, _ptr(X), _ptr(Yall)), "tt_sketch_tensor_all")
        out, off = [], 0
        for nk in self.n:
            out.append(Yall[off:off + self.J * nk])
            off += self.J * nk
        return out

    def _check_sparse(self, coords, vals):
        if not (isinstance(coords, torch.Tensor) and coords.device.type == "cuda" and coords.is_contiguous()
                and coords.dtype == torch.int32 and coords.dim() == 2 and coords.shape[1] == self.d):
            raise ValueError("coords must be a contiguous int32 device tensor of shape (nnz, d)")
        nnz = coords.shape[0]
        if not (isinstance(vals, torch.Tensor) and vals.device.type == "cuda" and vals.is_contiguous()
                and vals.dtype == _TORCH[self.x_dtype] and vals.numel() == nnz):
            raise ValueError("vals must be a contiguous %s device tensor of nnz values" % self.x_dtype)
        return nnz

    def sketch_sparse(self, coords, vals, k, Y=None):
        """Y_k of the sparse tensor given by COO coords (nnz x d int32) and vals."""
        nnz = self._check_sparse(coords, vals)
        if Y is None:
            Y = torch.empty(self.J * self.n[k], dtype=self.wdtype, device=self.device)
        self._check_work(Y, self.J * self.n[k], "Y")
        check(_lib.tt_sketch_sparse(self._h, nnz, _ptr(coords), _ptr(vals), int(k), _ptr(Y)), "tt_sketch_sparse")
        return Y

    def sketch_sparse_all(self, coords, vals):
        """[Y_0, ..., Y_{d-1}] of the sparse tensor, one pass over the nonzeros."""
        nnz = self._check_sparse(coords, vals)
        total = self.J * sum(self.n)
        Yall = torch.empty(total, dtype=self.wdtype, device=self.device)
        check(_lib.tt_sketch_sparse_all(self._h, nnz, _ptr(coords), _ptr(vals), _ptr(Yall)), "tt_sketch_sparse_all")
        out, off = [], 0
        for nk in self.n:
            out.append(Yall[off:off + self.J * nk])
            off += self.J * nk
        return out

    def exact_rhs(self, X, cores, k, B=None):
        """A_(k) H_k (n_k x R_k R_{k+1}, column-major, work type) by the exact
        contraction of X with the cores (plan made with exact=True)."""
        self._check_X(X)
        arr, keep = self._cores(cores, skip=k)
        numel = self.n[k] * self.s(k)
        if B is None:
            B = torch.empty(numel, dtype=self.wdtype, device=self.device)
        self._check_work(B, numel, "B")
        check(_lib.tt_exact_rhs(self._h, _ptr(X), arr, int(k), _ptr(B)), "tt_exact_rhs")
        return B

    def prox_exact(self, X, cores, k, G_new=None):
        """Exact proximal update of core k (G_old = cores[k])."""
        self._check_X(X)
        arr, keep = self._cores(cores)
        if G_new is None:
            G_new = torch.empty_like(cores[k])
        self._check_core(G_new, k)
        check(_lib.tt_prox_exact(self._h, _ptr(X), arr, int(k), _ptr(G_new)), "tt_prox_exact")
        return G_new

    def als_sweep_exact(self, X, cores, residual=False):
        """One sweep of exact proximal ALS (every sketch replaced by S = I)."""
        self._check_X(X)
        arr, keep = self._cores(cores)
        out = ctypes.c_double()
        check(_lib.tt_als_sweep_exact(self._h, _ptr(X), arr, ctypes.byref(out) if residual else None),
              "tt_als_sweep_exact")
        return out.value if residual else None

    def sketch_sources(self):
        """src[k] = k if Y_k takes its own pass over X, else the mode whose
        pass writes the intermediate it comes from."""
        arr = (ctypes.c_int32 * self.d)()
        check(_lib.tt_plan_sketch_sources(self._h, arr), "tt_plan_sketch_sources")
        return list(arr)

    def sketch_interface(self, cores, k, SH=None):
        arr, keep = self._cores(cores, skip=k)
        if SH is None:
            SH = torch.empty(self.J * self.s(k), dtype=self.wdtype, device=self.device)
        self._check_work(SH, self.J * self.s(k), "SH")
        check(_lib.tt_sketch_interface(self._h, arr, int(k), _ptr(SH)), "tt_sketch_interface")
        return SH

    def prox_solve(self, k, SH, Y, G_old, G_new=None):
        self._check_work(SH, self.J * self.s(k), "SH")
        self._check_work(Y, self.J * self.n[k], "Y")
        self._check_core(G_old, k)
        if G_new is None:
            G_new = torch.empty_like(G_old)
        self._check_core(G_new, k)
        check(_lib.tt_prox_solve(self._h, int(k), _ptr(SH), _ptr(Y), _ptr(G_old), _ptr(G_new)), "tt_prox_solve")
        return G_new

    def left_orth_absorb(self, cores, k):
        arr, keep = self._cores(cores)
        check(_lib.tt_left_orth_absorb(self._h, arr, int(k)), "tt_left_orth_absorb")

    def right_orthogonalize(self, cores):
        arr, keep = self._cores(cores)
        check(_lib.tt_right_orthogonalize(self._h, arr), "tt_right_orthogonalize")

    def residual(self, X, cores):
        self._check_X(X)
        arr, keep = self._cores(cores)
        out = ctypes.c_double()
        check(_lib.tt_residual(self._h, _ptr(X), arr, ctypes.byref(out)), "tt_residual")
        return out.value

    def core_change(self, prev, cur):
        """max_k ||cur_k - prev_k|| / ||cur_k|| (tt_core_change)."""
        a, ka = self._cores(prev)
        b, kb = self._cores(cur)
        out = ctypes.c_double()
        check(_lib.tt_core_change(self._h, a, b, ctypes.byref(out)), "tt_core_change")
        return out.value

    def als_sweep(self, X, cores, residual=False):
        self._check_X(X)
        arr, keep = self._cores(cores)
        if residual:
            out = ctypes.c_double()
            check(_lib.tt_als_sweep(self._h, _ptr(X), arr, ctypes.byref(out)), "tt_als_sweep")
            return out.value
        check(_lib.tt_als_sweep(self._h, _ptr(X), arr, None), "tt_als_sweep")
        return None

    def profile(self, enable=True, classes=None):
        """Time the launches of `classes` (names from _abi.PROF_CLASSES; all
        if None) with HIP events; enable=False stops measurement."""
        mask = 0
        if enable:
            names = _abi.PROF_CLASSES if classes is None else classes
            for c in names:
                mask |= 1 << _abi.PROF_CLASSES.index(c)
        check(_lib.tt_plan_profile(self._h, mask), "tt_plan_profile")

    def profile_read(self):
        """{class: (total ms, launches)} since the last read (synchronises)."""
        nc = len(_abi.PROF_CLASSES)
        ms = (ctypes.c_double * nc)()
        cnt = (ctypes.c_int64 * nc)()
        check(_lib.tt_plan_profile_read(self._h, nc, ms, cnt), "tt_plan_profile_read")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(_abi.PROF_CLASSES)}

    def set_sketch(self, J, lam):
        """Sketch size and proximal parameter from now on (J <= the plan's J)."""
        check(_lib.tt_plan_set_sketch(self._h, int(J), float(lam)), "tt_plan_set_sketch")

    def get_sketch(self):
        J = ctypes.c_int64()
        lam = ctypes.c_double()
        check(_lib.tt_plan_get_sketch(self._h, ctypes.byref(J), ctypes.byref(lam)), "tt_plan_get_sketch")
        return J.value, lam.value

    def fallback_J(self, eps=0.5, delta=0.1):
        """Corollary 3 sketch size of this plan, capped at its J."""
        J = ctypes.c_int64()
        check(_lib.tt_plan_fallback_J(self._h, float(eps), float(delta), ctypes.byref(J)), "tt_plan_fallback_J")
        return J.value

    def features(self, t, last_drop):
        """Policy features of the d core updates at sweep t (numpy d x F)."""
        out = (ctypes.c_float * (self.d * _abi.JPOLICY_FEATURES))()
        check(_lib.tt_jpolicy_features(self._h, int(t), float(last_drop), out), "tt_jpolicy_features")
        return np.frombuffer(out, dtype=np.float32).reshape(self.d, _abi.JPOLICY_FEATURES).copy()

    def choose(self, params, t, last_drop, J_min=64):
        """(J, lambda) the policy network picks for sweep t; J = 0 is the
        unsketched update (plans with exact=True only)."""
        J = ctypes.c_int64()
        lam = ctypes.c_double()
        check(_lib.tt_jpolicy_choose(self._h, _ptr(params), int(t), float(last_drop), int(J_min), ctypes.byref(J),
                                     ctypes.byref(lam)), "tt_jpolicy_choose")
        return J.value, lam.value

    def run(self, X, cores, max_sweeps, target, params=None, J_min=64):
        """Sweeps until the exact residual <= target (tt_als_run).  Returns a
        dict with the per-sweep residuals, J and lambda and the run stats."""
        self._check_X(X)
        arr, keep = self._cores(cores)
        if params is not None and not (isinstance(params, torch.Tensor) and params.dtype == torch.float32
                                       and params.is_contiguous() and params.numel() == _abi.JPOLICY_PARAMS
                                       and params.device.type == "cuda"):
            raise ValueError("params must be a contiguous float32 device tensor of %d entries" % _abi.JPOLICY_PARAMS)
        res = (ctypes.c_double * max_sweeps)()
        Js = (ctypes.c_int64 * max_sweeps)()
        lams = (ctypes.c_double * max_sweeps)()
        st = _abi.RunStats()
        check(_lib.tt_als_run(self._h, _ptr(X), arr, None if params is None else _ptr(params), int(max_sweeps),
                              float(target), int(J_min), res, Js, lams, ctypes.byref(st)), "tt_als_run")
        n = st.sweeps
        return {"sweeps": n, "reached": bool(st.reached), "fallbacks": st.fallbacks, "residual": st.residual,
                "residuals": list(res[:n]), "J": list(Js[:n]), "lambda": list(lams[:n])}

    def set_overlap(self, reserved_cus):
        """CUs kept free of the overlapped data sketches (see tt_plan_set_overlap)."""
        check(_lib.tt_plan_set_overlap(self._h, int(reserved_cus)), "tt_plan_set_overlap")

    def sketch_kernel(self, k):
        """Name of the data-sketch kernel tt_sketch_tensor runs for mode k."""
        path = ctypes.c_int32()
        check(_lib.tt_plan_sketch_path(self._h, int(k), ctypes.byref(path)), "tt_plan_sketch_path")
        return _abi.SKETCH_PATHS[path.value]

    def sync_status(self):
        check(_lib.tt_plan_sync_status(self._h), "tt_plan_sync_status")


class Batch:
    """Many independent problems advanced together (tt_batch_*).  problems:
    list of dicts with keys n, ranks, J, lam, seed; FP32 X and work."""

    def __init__(self, problems, device="cuda", stream=None):
        self.device = torch.device(device)
        self.problems = [dict(p) for p in problems]
        self.count = len(problems)
        self._keep = []
        descs = (_abi.PlanDesc * self.count)()
        for i, pr in enumerate(self.problems):
            n = (ctypes.c_int64 * len(pr["n"]))(*pr["n"])
            r = (ctypes.c_int64 * len(pr["ranks"]))(*pr["ranks"])
            self._keep += [n, r]
            descs[i] = _abi.PlanDesc(len(pr["n"]), n, r, int(pr["J"]), float(pr.get("lam", 1e-3)),
                                     int(pr.get("seed", i)) & (2 ** 64 - 1), _abi.TT_F32, _abi.TT_F32,
                                     _abi.TT_GRAM_WORK, 0)
        self._descs = descs
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        ws = ctypes.c_size_t(0)
        h = ctypes.c_void_p()
        check(_lib.tt_batch_plan(self.count, ctypes.cast(descs, ctypes.c_void_p), ctypes.c_void_p(stream.cuda_stream),
                                 ctypes.byref(ws), ctypes.byref(h)), "tt_batch_plan")
        self._h = h
        self.workspace_bytes = ws.value
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        check(_lib.tt_batch_bind_workspace(self._h, ctypes.c_void_p(aligned), self.workspace_bytes),
              "tt_batch_bind_workspace")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.tt_batch_destroy(h)
            self._h = None

    def _xs(self, Xs):
        if len(Xs) != self.count:
            raise ValueError("need %d tensors" % self.count)
        for X, pr in zip(Xs, self.problems):
            if not (isinstance(X, torch.Tensor) and X.device.type == "cuda" and X.is_contiguous()
                    and X.dtype == torch.float32 and X.numel() == int(np.prod(pr["n"]))):
                raise ValueError("each X must be a contiguous float32 device tensor of its problem's size")
        return _abi.ptr_array([X.data_ptr() for X in Xs])

    def _cores(self, cores):
        if len(cores) != self.count:
            raise ValueError("need %d core lists" % self.count)
        inner, keep = [], []
        for cs, pr in zip(cores, self.problems):
            n, R = pr["n"], pr["ranks"]
            if len(cs) != len(n):
                raise ValueError("core list of the wrong length")
            for k, G in enumerate(cs):
                if not (isinstance(G, torch.Tensor) and G.dtype == torch.float64 and G.is_contiguous()
                        and G.numel() == R[k] * n[k] * R[k + 1] and G.device.type == "cuda"):
                    raise ValueError("core %d must be a contiguous float64 device tensor" % k)
            arr, a = _abi.ptr_array([G.data_ptr() for G in cs])
            inner.append(arr)
            keep.append(a)
        outer = (ctypes.POINTER(ctypes.c_void_p) * self.count)(*inner)
        return ctypes.cast(outer, ctypes.c_void_p), (outer, keep)

    def plan_tables(self, i, s):
        """(h, v) of problem i, mode s (host copies)."""
        ph = ctypes.c_void_p()
        check(_lib.tt_batch_get_plan(self._h, int(i), ctypes.byref(ph)), "tt_batch_get_plan")
        ns = self.problems[i]["n"][s]
        h = (ctypes.c_int32 * ns)()
        v = (ctypes.c_int8 * ns)()
        check(_lib.tt_plan_get_tables(ph, int(s), h, v), "tt_plan_get_tables")
        return np.array(h, dtype=np.int64), np.array(v, dtype=np.int8)

    def sketch_sources(self, i):
        """tt_plan_sketch_sources of problem i's plan: entry k is the mode
        whose pass produces Y_k (0 at k = 1: Y_1 from the outer sketch)."""
        ph = ctypes.c_void_p()
        check(_lib.tt_batch_get_plan(self._h, int(i), ctypes.byref(ph)), "tt_batch_get_plan")
        d = len(self.problems[i]["n"])
        src = (ctypes.c_int32 * d)()
        check(_lib.tt_plan_sketch_sources(ph, src), "tt_plan_sketch_sources")
        return list(src)

    def set_graph(self, enable=True):
        check(_lib.tt_batch_set_graph(self._h, 1 if enable else 0), "tt_batch_set_graph")

    def sketch_tensor(self, Xs, k):
        """Batched data sketch of step k: list of J x n_k (flat, column-major)
        FP32 tensors, None for problems of order <= k."""
        xs, keep = self._xs(Xs)
        Ys, ptrs = [], []
        for pr in self.problems:
            if len(pr["n"]) > k:
                Y = torch.empty(int(pr["J"]) * pr["n"][k], dtype=torch.float32, device=self.device)
                Ys.append(Y)
                ptrs.append(Y.data_ptr())
            else:
                Ys.append(None)
                ptrs.append(None)
        ya, ykeep = _abi.ptr_array(ptrs)
        check(_lib.tt_batch_sketch_tensor(self._h, xs, int(k), ya), "tt_batch_sketch_tensor")
        return Ys

    def sketch_kernel(self, k):
        """Name of the data-sketch kernel the batched launch of step k runs."""
        path = ctypes.c_int32()
        check(_lib.tt_batch_sketch_path(self._h, int(k), ctypes.byref(path)), "tt_batch_sketch_path")
        return _abi.BSKETCH_PATHS[path.value]

    def sketch_launch(self, Xs, k):
        """The batched data-sketch launch of step k without copying results out."""
        xs, keep = self._xs(Xs)
        check(_lib.tt_batch_sketch_tensor(self._h, xs, int(k), None), "tt_batch_sketch_tensor")

    def sweep(self, Xs, cores, residuals=False):
        xs, keep = self._xs(Xs)
        cs, ckeep = self._cores(cores)
        if residuals:
            out = (ctypes.c_double * self.count)()
            check(_lib.tt_batch_sweep(self._h, xs, cs, out), "tt_batch_sweep")
            return list(out)
        check(_lib.tt_batch_sweep(self._h, xs, cs, None), "tt_batch_sweep")
        return None

    def get_tuning(self):
        """Per step: dict(workgroups, entries_per_lane, fibres_in_flight,
        gram_kchunk) (tt_batch_get_tuning)."""
        F = _abi.BATCH_TUNE_FIELDS
        buf = (ctypes.c_int64 * (_abi.MAX_ORDER * F))()
        check(_lib.tt_batch_get_tuning(self._h, buf), "tt_batch_get_tuning")
        dmax = max(len(p["n"]) for p in self.problems)
        names = ("workgroups", "entries_per_lane", "fibres_in_flight", "gram_kchunk")
        return [dict(zip(names, buf[k * F:(k + 1) * F])) for k in range(dmax)]

    def set_tuning(self, steps):
        """Restore get_tuning()'s list (tt_batch_set_tuning)."""
        F = _abi.BATCH_TUNE_FIELDS
        buf = (ctypes.c_int64 * (_abi.MAX_ORDER * F))()
        check(_lib.tt_batch_get_tuning(self._h, buf), "tt_batch_get_tuning")
        for k, st in enumerate(steps):
            buf[k * F:(k + 1) * F] = [int(st["workgroups"]), int(st["entries_per_lane"]),
                                      int(st["fibres_in_flight"]), int(st["gram_kchunk"])]
        check(_lib.tt_batch_set_tuning(self._h, buf), "tt_batch_set_tuning")

    def step_keys(self):
        """Cache key of each step's tuning: the step, the number of problems
        taking part, their total mode-0 fibres (the data sketch's units), the
        largest n_0, their total n_k (columns), the largest J, the data type
        and the device."""
        dmax = max(len(p["n"]) for p in self.problems)
        dev = torch.cuda.get_device_name(self.device) if torch.cuda.is_available() else "none"
        keys = []
        for k in range(dmax):
            ps = [p for p in self.problems if len(p["n"]) > k]
            units = sum(int(np.prod(p["n"])) // int(p["n"][0]) for p in ps)
            keys.append("k=%d|problems=%d|fibres=%d|n0max=%d|columns=%d|J=%d|dtype=f32|device=%s|%s" % (
                k, len(ps), units, max(p["n"][0] for p in ps), sum(p["n"][k] for p in ps),
                max(int(p["J"]) for p in ps), dev, version()))
        return keys

    def autotune(self, Xs, reps=3, cache=None):
        """Tune every step (tt_batch_autotune) and return the workgroup count
        per step.  With cache (a JSON file path), steps whose key
        (step_keys) is in the file take the stored tuning instead, and a
        fresh tuning is written back."""
        import json
        import os
        keys = self.step_keys()
        db = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                db = json.load(f)
        if cache and all(k in db for k in keys):
            self.set_tuning([db[k] for k in keys])
            self.tuned_from_cache = True
            return [st["workgroups"] for st in self.get_tuning()]
        xs, keep = self._xs(Xs)
        dmax = max(len(p["n"]) for p in self.problems)
        out = (ctypes.c_int64 * dmax)()
        check(_lib.tt_batch_autotune(self._h, xs, int(reps), out), "tt_batch_autotune")
        self.tuned_from_cache = False
        if cache:
            db.update(dict(zip(keys, self.get_tuning())))
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(db, f, indent=1)
            os.replace(tmp, cache)
        return list(out)


def residual_noalloc(X, cores, n, ranks, x_dtype="f32", work_dtype="f32", stream=None):
    """tt_residual_noalloc: ||X - [[G]]|| / ||X|| with the library's static
    device scratch (no plan, no workspace, nothing allocated)."""
    n = [int(x) for x in n]
    ranks = [int(x) for x in ranks]
    d = len(n)
    if len(ranks) != d + 1 or len(cores) != d:
        raise ValueError("need d + 1 ranks and d cores")
    if x_dtype not in _DT or work_dtype not in ("f64", "f32"):
        raise ValueError("bad dtype")
    if not (isinstance(X, torch.Tensor) and X.device.type == "cuda" and X.is_contiguous()
            and X.dtype == _TORCH[x_dtype] and X.numel() == int(np.prod(n))):
        raise ValueError("X must be a contiguous %s device tensor with %d entries" % (x_dtype, int(np.prod(n))))
    ptrs = []
    for k, G in enumerate(cores):
        numel = ranks[k] * n[k] * ranks[k + 1]
        if not (isinstance(G, torch.Tensor) and G.device.type == "cuda" and G.is_contiguous()
                and G.dtype == torch.float64 and G.numel() == numel):
            raise ValueError("core %d must be a contiguous float64 device tensor with %d entries" % (k, numel))
        ptrs.append(G.data_ptr())
    arr, keep = _abi.ptr_array(ptrs)
    if stream is None:
        stream = torch.cuda.current_stream(X.device)
    out = ctypes.c_double()
    check(_lib.tt_residual_noalloc(d, (ctypes.c_int64 * d)(*n), (ctypes.c_int64 * (d + 1))(*ranks), _DT[x_dtype],
                                   _DT[work_dtype], _ptr(X), arr, ctypes.c_void_p(stream.cuda_stream),
                                   ctypes.byref(out)), "tt_residual_noalloc")
    return out.value


def sketch_size_bound(s, q, eps=0.5, delta=0.1):
    """Corollary 3 sketch size m for s unknowns per column and q sketched modes."""
    m = ctypes.c_double()
    check(_lib.tt_sketch_size_bound(int(s), int(q), float(eps), float(delta), ctypes.byref(m)), "tt_sketch_size_bound")
    return m.value


__all__ = ["Plan", "Batch", "TTError", "core_to_device", "core_to_host", "version", "sketch_size_bound"]
