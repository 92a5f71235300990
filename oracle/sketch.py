"""TensorSketch of the data tensor and of the TT interface (oracle side, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Everything here is the plain definition written out:
  * ``tensorsketch_matrix`` builds S = Omega D of Sec. 2.2 (Definition of
    TensorSketch, (eqn_h) combined hash and (eqn_v) combined sign) entry by
    entry.
  * ``data_sketch`` computes S A_(k)^T of the sketched subproblem (Sec. 3,
    (lrtt_sub4)) by visiting every tensor entry once and adding its signed value
    to its bucket: each column of S holds exactly one +-1.
  * ``interface_explicit`` forms H_k = G_{>k}^T (x) G_{<k} (Sec. 3, its
    definition under (lrtt_sub4)) and multiplies by the explicit S.
  * ``interface_cyclic`` computes the same S H_k without FFTs: a CountSketch
    adds the mode hashes mod J, i.e. each core contributes a cyclic shift of
    the bucket axis (the identity behind Lemma 1 / Theorem 1 of Sec. 3,
    used here in its shift form rather than its Fourier form).
"""
import numpy as np


def tensorsketch_matrix(hs, vs, J):
    """Explicit TensorSketch matrix over the listed modes (first mode fastest).

    Column j <-> (i_0, ..., i_{q-1}) with j = sum_s i_s prod_{t<s} n_t; row
    (sum_s h_s(i_s)) mod J holds prod_s v_s(i_s) (Sec. 2.2, (eqn_h)-(eqn_v)).
    """
    sizes = [len(h) for h in hs]
    ncols = int(np.prod(sizes)) if sizes else 1
    S = np.zeros((J, ncols))
    for j in range(ncols):
        rem, b, sg = j, 0, 1
        for h, v, ns in zip(hs, vs, sizes):
            i = rem % ns
            rem //= ns
            b += int(h[i])
            sg *= int(v[i])
        S[b % J, j] += sg
    return S


def unfold(X, n, k):
    """Mode-k matricization A_(k): n_k x prod_{s!=k} n_s, columns i_0-fastest
    with mode k skipped (Sec. 1.2, definition of the mode-k matricization)."""
    T = np.asarray(X).reshape(tuple(n), order="F")
    T = np.moveaxis(T, k, 0)
    return T.reshape(n[k], -1, order="F")


def data_sketch_explicit(X, n, k, hs, vs, J):
    """S_{-k} A_(k)^T with S_{-k} built explicitly (tiny sizes only)."""
    others = [s for s in range(len(n)) if s != k]
    S = tensorsketch_matrix([hs[s] for s in others], [vs[s] for s in others], J)
    return S @ unfold(X, n, k).T


def data_sketch(X, n, k, hs, vs, J, slab_entries=1 << 24):
    """Y_k = S_{-k} A_(k)^T by visiting every entry once (FP64 accumulation).

    Entry (i_0..i_{d-1}) adds prod_{s!=k} v_s(i_s) * A(i) to
    Y_k[(sum_{s!=k} h_s(i_s)) mod J, i_k].  Y_k is J x n_k.  The tensor is
    processed in slabs of whole last-mode indices to bound memory.
    """
    n = [int(x) for x in n]
    d = len(n)
    X = np.asarray(X).reshape(-1, order="F")
    N = int(np.prod(n))
    if X.size != N:
        raise ValueError("X has %d entries, shape needs %d" % (X.size, N))
    Y = np.zeros(J * n[k])
    inner = N // n[-1]
    per_slab = max(1, slab_entries // max(inner, 1))
    for i_last0 in range(0, n[-1], per_slab):
        i_last1 = min(n[-1], i_last0 + per_slab)
        idx = np.arange(i_last0 * inner, i_last1 * inner, dtype=np.int64)
        bucket = np.zeros(idx.size, dtype=np.int64)
        sign = np.ones(idx.size, dtype=np.float64)
        col = None
        rem = idx.copy()
        for s in range(d):
            i_s = rem % n[s]
            rem //= n[s]
            if s == k:
                col = i_s
            else:
                bucket += hs[s][i_s]
                sign *= vs[s][i_s]
        bucket %= J
        Y += np.bincount(bucket + J * col, weights=sign * X[idx].astype(np.float64),
                         minlength=J * n[k])
    return Y.reshape(J, n[k], order="F")


def left_product(cores, k):
    """G_{<k} (prod_{i<k} n_i x R[k]); G_{<0} = [[1]] (Sec. 3, definition of H_k under (lrtt_sub4))."""
    T = np.ones((1, 1))
    for i in range(k):
        G = np.asarray(cores[i], dtype=np.float64)
        r0, ni, r1 = G.shape
        T = (T @ G.reshape(r0, ni * r1, order="F")).reshape(-1, r1, order="F")
    return T


def right_product(cores, k):
    """G_{>k} (R[k+1] x prod_{i>k} n_i); G_{>d-1} = [[1]]."""
    d = len(cores)
    U = np.ones((1, 1))
    for i in range(d - 1, k, -1):
        G = np.asarray(cores[i], dtype=np.float64)
        r0, ni, r1 = G.shape
        U = (G.reshape(r0 * ni, r1, order="F") @ U).reshape(r0, -1, order="F")
    return U


def interface_matrix(cores, k):
    """H_k = G_{>k}^T (x) G_{<k}; column alpha + beta*R[k] (Sec. 3, definition of H_k under (lrtt_sub4))."""
    return np.kron(right_product(cores, k).T, left_product(cores, k))


def interface_explicit(cores, n, k, hs, vs, J):
    """S_{-k} H_k with both factors explicit (tiny sizes only)."""
    others = [s for s in range(len(n)) if s != k]
    S = tensorsketch_matrix([hs[s] for s in others], [vs[s] for s in others], J)
    return S @ interface_matrix(cores, k)


def _shift(P, h):
    """Rows moved down cyclically by h: out[b] = P[(b - h) mod J]."""
    return np.roll(P, int(h), axis=0)


def sketched_left(cores, k, hs, vs, J):
    """S_{<k} G_{<k} (J x R[k]) by one cyclic-shift recursion per core.

    P_0 = e_0 (J x 1).  Core i maps P_i (J x R[i]) to
    P_{i+1}[b, beta] = sum_j v_i[j] sum_alpha P_i[(b - h_i[j]) mod J, alpha] G_i[alpha, j, beta].
    """
    P = np.zeros((J, 1))
    P[0, 0] = 1.0
    for i in range(k):
        G = np.asarray(cores[i], dtype=np.float64)
        Pn = np.zeros((J, G.shape[2]))
        for j in range(G.shape[1]):
            Pn += vs[i][j] * (_shift(P, hs[i][j]) @ G[:, j, :])
        P = Pn
    return P


def sketched_right(cores, k, hs, vs, J):
    """S_{>k} G_{>k}^T (J x R[k+1]), the mirrored recursion from core d-1."""
    d = len(cores)
    Q = np.zeros((J, 1))
    Q[0, 0] = 1.0
    for i in range(d - 1, k, -1):
        G = np.asarray(cores[i], dtype=np.float64)
        Qn = np.zeros((J, G.shape[0]))
        for j in range(G.shape[1]):
            Qn += vs[i][j] * (_shift(Q, hs[i][j]) @ G[:, j, :].T)
        Q = Qn
    return Q


def interface_cyclic(cores, k, hs, vs, J):
    """S_{-k} H_k (J x R[k]R[k+1]) without FFTs.

    The combined hash of a row of H_k is (h_<(left) + h_>(right)) mod J and
    its sign is the product, so column (alpha, beta) is the cyclic
    convolution over the bucket axis of left column alpha and right column
    beta.  Written as an explicit sum over the left bucket b'.
    """
    P = sketched_left(cores, k, hs, vs, J)
    Q = sketched_right(cores, k, hs, vs, J)
    rk, rk1 = P.shape[1], Q.shape[1]
    out = np.zeros((J, rk * rk1))
    for bp in range(J):
        Qs = _shift(Q, bp)                       # Qs[b] = Q[(b - bp) mod J]
        # out[b, alpha + beta*rk] += P[bp, alpha] * Q[(b - bp) mod J, beta]
        out += np.einsum("bq,p->bpq", Qs, P[bp]).reshape(J, rk * rk1, order="F")
    return out


def data_sketch_sparse(coords, vals, n, k, hs, vs, J):
    """Y_k from the nonzeros of a COO tensor: nonzero e with indices
    coords[e] adds prod_{s!=k} v_s(i_s) vals[e] to Y_k[(sum_{s!=k} h_s(i_s)) mod
    J, i_k] (the definition of the data sketch restricted to stored entries;
    repeated coordinates add)."""
    coords = np.asarray(coords, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    Y = np.zeros((J, int(n[k])))
    bucket = np.zeros(len(vals), dtype=np.int64)
    sign = np.ones(len(vals))
    for s in range(len(n)):
        if s != k:
            bucket += np.asarray(hs[s], dtype=np.int64)[coords[:, s]]
            sign *= np.asarray(vs[s], dtype=np.float64)[coords[:, s]]
    np.add.at(Y, (bucket % J, coords[:, k]), sign * vals)
    return Y
