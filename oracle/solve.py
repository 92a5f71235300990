"""Sketched proximal update, QR with sign normalisation, orthogonalisation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  FP64 throughout.
"""
import numpy as np


def core_unfold2(G):
    """Mode-2 unfolding G_(2) of a core (R[k], n_k, R[k+1]): n_k x R[k]R[k+1],
    column alpha + beta*R[k] (Sec. 1.2 matricization applied to a 3-way core)."""
    r0, nk, r1 = G.shape
    return np.transpose(G, (1, 0, 2)).reshape(nk, r0 * r1, order="F")


def core_fold2(G2, r0, r1):
    """Inverse of ``core_unfold2``."""
    nk = G2.shape[0]
    return np.transpose(G2.reshape(nk, r0, r1, order="F"), (1, 0, 2))


def prox_update(SH, Y, G_old, lam):
    """Closed-form minimiser of the sketched proximal subproblem (Sec. 3,
    (lrtt_sub4)-(ite), reading the printed 'S S^T' as S^T S, the only
    dimensionally consistent product):

        G_(2)^{new} = (Y^T SH + lam G_(2)^{old}) (SH^T SH + lam I)^{-1}

    SH = S H_k (J x s), Y = S A_(k)^T (J x n_k), G_old (R[k], n_k, R[k+1]).
    The s x s system is solved by LU (numpy.linalg.solve) on the normal
    equations M Z = B with M = SH^T SH + lam I, B = SH^T Y + lam G_(2)^T.
    """
    G_old = np.asarray(G_old, dtype=np.float64)
    r0, nk, r1 = G_old.shape
    SH = np.asarray(SH, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    s = r0 * r1
    M = SH.T @ SH + lam * np.eye(s)
    B = SH.T @ Y + lam * core_unfold2(G_old).T
    Z = np.linalg.solve(M, B)            # s x n_k, row alpha + beta*R[k]
    return core_fold2(Z.T, r0, r1)


def round_bf16(A):
    """Round to BF16 the way the precision form feeds its Gram: first to the
    FP32 work type, then to BF16 (the upper 16 bits of an IEEE binary32,
    round to nearest, ties to even), returned as FP64 values.

    BF16 is not from the paper; the mixed-precision form computes M and B
    from BF16 copies of SH and Y.  Finite inputs only."""
    x = np.ascontiguousarray(np.asarray(A, dtype=np.float64).astype(np.float32))
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(A))


def prox_update_stacked(SH, Y, G_old, lam):
    """Same minimiser via the stacked least-squares form used in the proof of
    Theorem 5 (Sec. 4): min || [SH; sqrt(lam) I] Z - [Y; sqrt(lam) G_(2)^T] ||_F,
    solved with numpy.linalg.lstsq.  Used as an independent check."""
    G_old = np.asarray(G_old, dtype=np.float64)
    r0, nk, r1 = G_old.shape
    s = r0 * r1
    A = np.vstack([SH, np.sqrt(lam) * np.eye(s)])
    B = np.vstack([Y, np.sqrt(lam) * core_unfold2(G_old).T])
    Z = np.linalg.lstsq(A, B, rcond=None)[0]
    return core_fold2(Z.T, r0, r1)


def qr_pos(A):
    """Reduced Householder QR (LAPACK via numpy) normalised so diag(R) >= 0.

    Column j of Q and row j of R are negated where R[j, j] < 0.  For a zero
    column LAPACK's reflector is the identity (tau = 0), so a zero matrix gives
    Q = the leading identity columns and R = 0.
    """
    Q, R = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="reduced")
    sg = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * sg[None, :], R * sg[:, None]


def left_orth_absorb(Gk, Gk1):
    """Algorithm 1, inner loop, k < d: [Q, R] = qr(G_k^L); G_k <- Q;
    G_{k+1} <- R G_{k+1}^R (reshaped back)."""
    r0, nk, r1 = Gk.shape
    Q, R = qr_pos(Gk.reshape(r0 * nk, r1, order="F"))
    r1b, nk1, r2 = Gk1.shape
    newk = Q.reshape(r0, nk, r1, order="F")
    newk1 = (R @ Gk1.reshape(r1b, nk1 * r2, order="F")).reshape(r1, nk1, r2, order="F")
    return newk, newk1


def right_orthogonalize(cores):
    """Right-to-left orthogonalisation (Algorithm 1, first step of the while
    loop).  For k = d-1 .. 1: LQ of G_k^R (R[k] x n_k R[k+1]) computed as the QR
    of its transpose, (G_k^R)^T = Q R  =>  G_k^R = R^T Q^T;  G_k <- Q^T;
    G_{k-1}^L <- G_{k-1}^L R^T.  Afterwards cores 1..d-1 have orthonormal rows
    in their right unfolding."""
    cores = [np.array(G, dtype=np.float64) for G in cores]
    d = len(cores)
    for k in range(d - 1, 0, -1):
        r0, nk, r1 = cores[k].shape
        Q, R = qr_pos(cores[k].reshape(r0, nk * r1, order="F").T)
        cores[k] = Q.T.reshape(r0, nk, r1, order="F")
        p0, pn, p1 = cores[k - 1].shape
        cores[k - 1] = (cores[k - 1].reshape(p0 * pn, p1, order="F") @ R.T).reshape(p0, pn, p1, order="F")
    return cores
