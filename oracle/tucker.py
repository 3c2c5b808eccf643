"""Truncated higher-order SVD (oracle; test infrastructure only).

The paper compresses the coefficient tensors with TT-cross followed by
TT-rounding (Sec. 2.1, "Tensor Train Decomposition") and states the online
algebra in terms of the resulting cores (Sec. 4.2 far field, Sec. 4.3 near
field, App. PTTK review).  This build compresses the same tensors with a
truncated HOSVD (Tucker format) over grouped modes instead; the online algebra
keeps the paper's shape: a small parameter-dependent core contracted with the
parametric vectors, between fixed spatial factors.  For a near-field tensor
with one parameter the Tucker format is a truncated SVD of the (n_s n_t) x p
matrix, the same format as the paper's two-core TT.

Reading of the tolerance: the paper's eps_tol is a relative error estimated in
the max norm by a heuristic.  Here it is a relative Frobenius-norm bound: each
of the N modes keeps the smallest rank r with
    sum_{j > r} s_j^2 <= (tol^2 / N) * ||M||_F^2,
which gives ||M - M_hat||_F <= tol * ||M||_F for the truncated HOSVD.

Reading of the cut: the leading-r subspace of a matrix is unique only when
s_r > s_{r+1}, and a backward-stable SVD determines it to about
eps ||A|| / (s_r - s_{r+1}).  Tensors with symmetric geometry (a translation
class whose offset is symmetric under swapping two axes) have exactly
degenerate singular pairs, and the rule above can cut between the two members
of a pair; two correct SVD routines then keep different vectors of the pair and
their truncations differ by about s_r.  So the cut is moved past every
following singular value within relative CLUSTER_GAP of the last one kept: a
cluster of (numerically) equal singular values is kept or dropped as a whole,
which only ever raises the rank and keeps the bound above.
"""

import numpy as np


def unfold(T, m):
    """Mode-m unfolding: rows indexed by mode m, columns by the remaining modes."""
    return np.moveaxis(T, m, 0).reshape(T.shape[m], -1)


def mode_product(T, A, m):
    """Mode-m product T x_m A (Sec. 2.1): y[.., j, ..] = sum_i T[.., i, ..] A[j, i]."""
    out = np.tensordot(A, T, axes=([1], [m]))   # new axis first
    return np.moveaxis(out, 0, m)


CLUSTER_GAP = 1e-4


def truncation_rank(s, thr):
    """Smallest r >= 0 with sum_{j >= r} s_j^2 <= thr (0-based tail), moved past every
    following singular value s_r with s_{r-1} - s_r <= CLUSTER_GAP * s_{r-1}."""
    s = np.asarray(s, dtype=np.float64)
    s2 = s ** 2
    # tail[r] = sum_{j >= r} s2[j], summed from the smallest value upward
    tail = np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]])
    r = len(s2)
    for q in range(len(tail)):
        if tail[q] <= thr:
            r = q
            break
    while 0 < r < len(s) and s[r - 1] - s[r] <= CLUSTER_GAP * s[r - 1]:
        r += 1
    return r


def thosvd(T, tol):
    """Truncated HOSVD of T.

    Returns (core, factors, svals): factors[m] has orthonormal columns
    (T.shape[m] x r_m); core = T x_1 U_1^T ... x_N U_N^T, computed from the
    original T (not sequentially truncated); svals[m] are the mode-m singular
    values.  A zero tensor gives all ranks 0.
    """
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    normsq = float(np.sum(T * T))
    thr = (tol * tol / N) * normsq
    factors, svals = [], []
    for m in range(N):
        U, s, _ = np.linalg.svd(unfold(T, m), full_matrices=False)
        r = 0 if normsq == 0.0 else truncation_rank(s, thr)
        factors.append(U[:, :r].copy())
        svals.append(s)
    core = T
    for m in range(N):
        core = mode_product(core, factors[m].T, m)
    return core, factors, svals


def reconstruct(core, factors):
    """Tucker reconstruction core x_1 U_1 ... x_N U_N."""
    T = core
    for m, U in enumerate(factors):
        T = mode_product(T, U, m)
    return T
