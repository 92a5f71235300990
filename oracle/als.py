"""One outer iteration of Algorithm 1 (TT-TS, Sec. 3) and its measurements.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  FP64 throughout.
"""
import numpy as np

from . import sketch, solve, tables


def tt_full(cores):
    """Dense [[G_0, ..., G_{d-1}]] as a flat array in i_0-fastest order
    (Sec. 2.1: A(i) = G_0(i_0) G_1(i_1) ... G_{d-1}(i_{d-1}))."""
    return sketch.left_product(cores, len(cores)).reshape(-1, order="F")


def rel_residual(X, cores):
    """|| [[G]] - A ||_F / || A ||_F, the objective of Sec. 3 (lrtt) made
    relative; accumulated in FP64."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, order="F")
    return float(np.linalg.norm(tt_full(cores) - X) / np.linalg.norm(X))


def core_change(old, new):
    """The paper's accuracy measure (Sec. 5, first paragraph):
    max_k ||G_k^{(t+1)} - G_k^{(t)}||_F / ||G_k^{(t+1)}||_F."""
    return max(float(np.linalg.norm(b - a) / np.linalg.norm(b)) for a, b in zip(old, new))


def sweep(X, n, cores, J, lam, seed=0, t=0, tabs=None, interface="cyclic", record=None, gram="fp64"):
    """One while-pass of Algorithm 1.

    1. right-to-left orthogonalisation of all cores;
    2. TensorSketch tables S_s for this pass (``tabs`` = (hs, vs) overrides);
    3. for k = 0..d-1: SH_k = S H_k; Y_k = S A_(k)^T; proximal update (ite)
       with G_k^{(t)} = the core's value just before its update; if k < d-1,
       QR of G_k^L, G_k <- Q, G_{k+1} <- R G_{k+1}^R.

    ``record`` (a list) receives per-k dicts with the step inputs/outputs so
    that a GPU step can be compared on identical inputs.  ``gram="bf16"``
    models the mixed-precision form (not from the paper): the normal
    equations are formed from the BF16 roundings of SH and Y
    (``solve.round_bf16``); everything else stays FP64.
    """
    d = len(n)
    cores = solve.right_orthogonalize(cores)
    if tabs is None:
        hs, vs = tables.sweep_tables(seed, t, n, J)
    else:
        hs, vs = tabs
    for k in range(d):
        if interface == "explicit":
            SH = sketch.interface_explicit(cores, n, k, hs, vs, J)
        else:
            SH = sketch.interface_cyclic(cores, k, hs, vs, J)
        Y = sketch.data_sketch(X, n, k, hs, vs, J)
        G_old = cores[k]
        if gram == "bf16":
            G_new = solve.prox_update(solve.round_bf16(SH), solve.round_bf16(Y), G_old, lam)
        else:
            G_new = solve.prox_update(SH, Y, G_old, lam)
        if record is not None:
            record.append(dict(k=k, cores_in=[c.copy() for c in cores], SH=SH, Y=Y,
                               G_old=G_old.copy(), G_new=G_new.copy()))
        cores[k] = G_new
        if k < d - 1:
            cores[k], cores[k + 1] = solve.left_orth_absorb(cores[k], cores[k + 1])
    return cores


def exact_rhs(X, n, cores, k):
    """A_(k) H_k (n_k x R_k R_{k+1}) with H_k = G_{>k}^T (x) G_{<k} formed
    explicitly (Sec. 3, under (lrtt_sub4)); tiny sizes only."""
    return sketch.unfold(X, n, k) @ sketch.interface_matrix(cores, k)


def prox_exact(X, n, cores, k, lam):
    """Minimiser of the unsketched proximal subproblem (lrtt_sub_prox):
    (ite) with S^T S = I, i.e. the proximal update with SH = H_k and
    Y = A_(k)^T."""
    return solve.prox_update(sketch.interface_matrix(cores, k), sketch.unfold(X, n, k).T, cores[k], lam)


def sweep_exact(X, n, cores, lam):
    """One while-pass of Algorithm 1 with every sketched subproblem replaced
    by the exact one (lrtt_sub_prox): right-to-left orthogonalisation, then for
    k = 0..d-1 the exact proximal update and, for k < d-1, QR + absorb."""
    d = len(n)
    cores = solve.right_orthogonalize(cores)
    for k in range(d):
        cores[k] = prox_exact(X, n, cores, k, lam)
        if k < d - 1:
            cores[k], cores[k + 1] = solve.left_orth_absorb(cores[k], cores[k + 1])
    return cores


def run(X, n, cores, J, lam, seed, sweeps, interface="cyclic"):
    """``sweeps`` passes; returns (cores, residual history, core-change history)."""
    res, chg = [], []
    for t in range(sweeps):
        new = sweep(X, n, cores, J, lam, seed=seed, t=t, interface=interface)
        chg.append(core_change(cores, new))
        cores = new
        res.append(rel_residual(X, cores))
    return cores, res, chg
