"""Pins of the oracle's tensor-train path (TT-cross, TT-rounding, the conversion of the
cores into L, H(theta), R and the core-by-core coupling of Alg. "Modified H^2-Matrix
MVM") against exact low-rank structure, library SVDs, brute-force contractions and
polynomial exactness.  None needs a GPU."""

import numpy as np
import pytest

from oracle import cheb, hmat, kernels, tt


def _rand_tt(rng, dims, ranks):
    r = [1] + list(ranks) + [1]
    return [rng.standard_normal((r[k], m, r[k + 1])) for k, m in enumerate(dims)]


def _entry(X):
    return lambda idx: X[tuple(idx.T)]


# ---------------------------------------------------------------- ACA
def test_aca_skeleton_of_exact_low_rank_matrix():
    """Partially pivoted ACA of a rank-4 matrix stops at rank 4 and its cross
    M(:, J) M(I, J)^-1 M(I, :) is the matrix itself (Gaussian elimination identity)."""
    rng = np.random.default_rng(0)
    M = rng.standard_normal((40, 4)) @ rng.standard_normal((4, 33))
    rows, cols, _, _ = tt.aca(lambda i: M[i], lambda j: M[:, j], 40, 33, 1e-13, 0)
    assert len(rows) == 4 and len(set(rows)) == 4 and len(set(cols)) == 4
    S = M[:, cols] @ np.linalg.solve(M[np.ix_(rows, cols)], M[rows])
    assert np.max(np.abs(S - M)) <= 1e-12 * np.max(np.abs(M))


def test_aca_pivots_are_largest_residual_entries():
    """The first column pivot is the largest entry of the start row, the second row pivot
    the largest entry of the first residual column (partial pivoting)."""
    rng = np.random.default_rng(1)
    M = rng.standard_normal((12, 9))
    rows, cols, _, _ = tt.aca(lambda i: M[i], lambda j: M[:, j], 12, 9, 1e-14, 3)
    assert rows[0] == 3 and cols[0] == int(np.argmax(np.abs(M[3])))
    u = M[:, cols[0]] - 0.0
    u[3] = 0.0
    assert rows[1] == int(np.argmax(np.abs(u)))


def test_aca_tie_rule_takes_first_index():
    """Exactly equal magnitudes (symmetric geometry) pick the lowest index."""
    M = np.array([[1.0, -2.0, 2.0], [0.5, 1.0, 3.0]])
    rows, cols, _, _ = tt.aca(lambda i: M[i], lambda j: M[:, j], 2, 3, 1e-14, 0)
    assert cols[0] == 1


# ---------------------------------------------------------------- TT-cross
@pytest.mark.parametrize("dims,ranks", [([4, 5, 3, 6, 4], [2, 3, 3, 2]), ([7, 11], [3]), ([5, 4, 6], [2, 2])])
def test_tt_cross_recovers_exact_tt(dims, ranks):
    """A tensor with exact TT ranks r is recovered with ranks <= r and to rounding level,
    evaluating fewer entries than the tensor has when it is large enough."""
    rng = np.random.default_rng(2)
    X = tt.tt_full(_rand_tt(rng, dims, ranks))
    cores, ev = tt.tt_cross(_entry(X), dims, 1e-13)
    got = [c.shape[2] for c in cores[:-1]]
    assert all(g <= r for g, r in zip(got, ranks))
    assert np.max(np.abs(tt.tt_full(cores) - X)) <= 1e-11 * np.max(np.abs(X))
    assert ev <= X.size


def test_tt_full_entry_formula():
    """tt_full against the entry formula of Sec. 2.1 (product of core slices), entry by entry."""
    rng = np.random.default_rng(3)
    cores = _rand_tt(rng, [3, 4, 2], [2, 3])
    X = tt.tt_full(cores)
    for i in range(3):
        for j in range(4):
            for k in range(2):
                v = (cores[0][:, i, :] @ cores[1][:, j, :] @ cores[2][:, k, :])[0, 0]
                assert abs(X[i, j, k] - v) <= 1e-13 * (1 + abs(v))


# ---------------------------------------------------------------- TT-rounding
def test_tt_rounding_exact_ranks_of_redundant_tt():
    """Rounding at tol = 0 (numerically) of a TT with redundant ranks gives the ranks of the
    unfoldings (numpy's SVD) and the same tensor."""
    rng = np.random.default_rng(4)
    dims = [4, 5, 6, 3]
    X = tt.tt_full(_rand_tt(rng, dims, [2, 3, 2]))
    # redundant representation: sum of the TT with itself has ranks doubled, same content x2
    A = _rand_tt(rng, dims, [2, 3, 2])
    XA = tt.tt_full(A)
    B = [np.concatenate([A[0], A[0]], axis=2)]
    for G in A[1:-1]:
        r0, m, r1 = G.shape
        Z = np.zeros((2 * r0, m, 2 * r1))
        Z[:r0, :, :r1] = G
        Z[r0:, :, r1:] = G
        B.append(Z)
    B.append(np.concatenate([A[-1], A[-1]], axis=0))
    R = tt.tt_round(B, 1e-14)
    for k in range(len(dims) - 1):
        unf = XA.reshape(int(np.prod(dims[:k + 1])), -1, order="F")
        assert R[k].shape[2] == np.linalg.matrix_rank(unf)
    np.testing.assert_allclose(tt.tt_full(R), 2 * XA, atol=1e-12 * np.max(np.abs(XA)))
    assert X.shape == XA.shape


def test_tt_rounding_error_bound_and_first_rank():
    """||X - round(X)||_F <= tol ||X||_F; and the first rank is the delta-truncation rank of
    the first unfolding's singular values from numpy's SVD (after the right-to-left
    orthogonalisation the first core's unfolding has exactly those singular values),
    delta = tol / sqrt(N - 1) ||X||_F."""
    from oracle.tucker import truncation_rank
    rng = np.random.default_rng(5)
    dims = [6, 7, 5, 6]
    cores = _rand_tt(rng, dims, [5, 6, 5])
    for k, G in enumerate(cores):
        cores[k] = G * (0.3 ** np.arange(G.shape[2]))[None, None, :]
    X = tt.tt_full(cores)
    s_np = np.linalg.svd(X.reshape(dims[0], -1, order="F"), compute_uv=False)
    for tol in (1e-1, 1e-3, 1e-6):
        R = tt.tt_round(cores, tol)
        assert np.linalg.norm(tt.tt_full(R) - X) <= tol * np.linalg.norm(X) * (1 + 1e-12)
        delta2 = tol * tol / (len(dims) - 1) * float(np.sum(X * X))
        assert R[0].shape[2] == max(1, truncation_rank(s_np, delta2))


# ---------------------------------------------------------------- kernel tensors
def _far_tensor(kernel, d, ps, pt, lo_s, hi_s, lo_t, hi_t, th_lo, th_hi, dth=1):
    ns = [cheb.chebyshev_nodes(lo_s[k], hi_s[k], ps) for k in range(d)]
    nt = [cheb.chebyshev_nodes(lo_t[k], hi_t[k], ps) for k in range(d)]
    th = [cheb.chebyshev_nodes(th_lo[k], th_hi[k], pt) for k in range(dth)]
    dims = [ps] * d + [pt] * dth + [ps] * d
    idx = np.indices(dims).reshape(len(dims), -1).T
    x = np.stack([ns[k][idx[:, k]] for k in range(d)], -1)
    y = np.stack([nt[k][idx[:, d + dth + k]] for k in range(d)], -1)
    t = np.stack([th[k][idx[:, d + k]] for k in range(dth)], -1)
    return kernel(x, y, t).reshape(dims), th


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-8])
def test_tt_compress_kernel_tensor_within_tolerance(tol):
    """TT-cross + TT-rounding of a far tensor (3-D Matern-3/2, offset (2, 0, 1)) lands within
    tol ||M||_F (the reading: the cross at tol / 10, rounding at tol)."""
    M, _ = _far_tensor(kernels.matern32, 3, 5, 11, [0, 0, 0], [.25] * 3, [.5, 0, .25], [.75, .25, .5],
                       [0.1], [1.0])
    cores, ev = tt.tt_compress(_entry(M), list(M.shape), tol)
    assert np.linalg.norm(tt.tt_full(cores) - M) <= tol * np.linalg.norm(M)
    assert ev <= M.size


@pytest.mark.parametrize("d,dth,kernel", [(2, 1, kernels.gaussian), (3, 1, kernels.matern32),
                                          (2, 2, kernels.aniso_gaussian), (2, 2, kernels.matern)])
def test_tt_far_factors_and_core_by_core_coupling(d, dth, kernel):
    """C x_hat three ways agree to rounding: Alg. "Modified H^2-Matrix MVM" applied core by core,
    L H(theta) R^T from the converted factors, and the brute-force contraction
    sum_{k, j} M^[i, k, j] v(theta)_k x_hat_j of the full TT tensor."""
    ps, pt = 4, 5
    lo, hi = ([0.3, 0.6], [1.0, 2.5]) if kernel is kernels.matern else ([0.1] * dth, [0.6] * dth)
    M, th = _far_tensor(kernel, d, ps, pt, [0] * d, [.25] * d, [.5] + [0] * (d - 1), [.75] + [.25] * (d - 1),
                        lo, hi, dth)
    cores, _ = tt.tt_compress(_entry(M), list(M.shape), 1e-10)
    core, facs = tt.far_factors(cores, d, dth)
    rng = np.random.default_rng(7)
    P = ps ** d
    xh = rng.standard_normal((P, 2))
    theta = [0.5 * (a + b) + 0.1 * (b - a) for a, b in zip(lo, hi)]
    vs = [cheb.lagrange(th[k], np.array(theta[k])) for k in range(dth)]
    H = core
    for k in range(dth):
        H = np.tensordot(H, facs[1 + k].T @ vs[k], axes=([1], [0]))
    y_fac = facs[0] @ H @ (facs[-1].T @ xh)
    y_alg5 = tt.implicit_coupling_apply(cores, d, dth, vs, xh)
    Mh = tt.tt_full(cores)
    # flatten (i_1..i_d) and (j_1..j_d) little-endian
    Mflat = Mh.reshape([P] + [pt] * dth + [P], order="F")
    W = Mflat
    for k in range(dth):
        W = np.tensordot(W, vs[k], axes=([1], [0]))
    y_brute = W @ xh
    scale = np.max(np.abs(y_brute))
    assert np.max(np.abs(y_alg5 - y_brute)) <= 1e-13 * scale
    assert np.max(np.abs(y_fac - y_brute)) <= 1e-13 * scale


# ---------------------------------------------------------------- PH2 in TT mode
def _pts(n, d, seed):
    return np.random.default_rng(seed).random((n, d))


def _model(kernel, n, d, l, eta2, p_s, p_theta, tol, lo=(0.1,), hi=(0.5,), seed=9, compress="tt"):
    return hmat.PH2(_pts(n, d, seed), l_max=l, eta2=eta2, kernel=kernels.KERNELS[kernel][0], theta_lo=lo,
                    theta_hi=hi, p_s=p_s, p_theta=p_theta, tol=tol, compress=compress)


def test_tt_model_reproduces_polynomial_kernel():
    """A kernel of degree 2 in x, y and theta is interpolated exactly, and its tensors have
    exact low TT ranks, so the TT model's MVM equals the dense K(theta) x."""
    for d, l, eta2 in ((2, 3, 2), (3, 2, 3)):
        m = _model("poly_test", 700, d, l, eta2, 3, 3, 1e-12)
        x = np.random.default_rng(2).standard_normal((700, 2))
        for th in (0.1, 0.37):
            ref = m.exact_dense(th) @ x
            y = m.matvec(m.instantiate(th), x)
            assert np.max(np.abs(y - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_tt_model_mirror_classes_and_near_blocks_are_transposes():
    """TT mode: a class below its mirror and a near block (s, t), s > t, are the transposes of
    the compressed ones (same factors, up to the contraction order's rounding)."""
    m = _model("gaussian", 600, 2, 3, 2, 5, 7, 1e-8)
    vs = m.theta_vectors(0.23)
    for key in range(len(m.classes)):
        mk = m._mirror_key(key)
        if mk is not None:
            a, b = m.coupling(key, vs), m.coupling(mk, vs).T
            assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))
    idx = {tuple(b): i for i, b in enumerate(m.near)}
    for bi, (s, u) in enumerate(m.near):
        if s > u:
            np.testing.assert_array_equal(m.near_block(bi, vs), m.near_block(idx[(u, s)], vs).T)


@pytest.mark.parametrize("kernel,lo,hi,th", [("matern32", (0.05,), (0.5,), 0.21),
                                             ("gaussian", (0.1,), (0.5,), 0.33)])
def test_tt_model_close_to_tucker_model(kernel, lo, hi, th):
    """The TT and the Tucker compressions of the same tensors at tol approximate the same
    interpolant: their MVMs differ by O(tol) (each within a few tol of it)."""
    tol = 1e-8
    mt = _model(kernel, 800, 2, 3, 2, 5, 7, tol, lo, hi)
    mu = _model(kernel, 800, 2, 3, 2, 5, 7, tol, lo, hi, compress="tucker")
    x = np.random.default_rng(3).standard_normal((800, 2))
    yt = mt.matvec(mt.instantiate(th), x)
    yu = mu.matvec(mu.instantiate(th), x)
    assert np.max(np.abs(yt - yu)) <= 100 * tol * np.max(np.abs(yu))
    assert mt.tt_evals > 0
