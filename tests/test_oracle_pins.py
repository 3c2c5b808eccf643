"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine, a closed form, brute force, polynomial exactness, the paper's printed
NF ratios, or an identity the paper states.  None needs a GPU.
"""

import json
import os

import numpy as np
import pytest
import scipy.interpolate as si

from oracle import cheb, kernels, tree as tr, tucker, hmat

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- Chebyshev / Lagrange
@pytest.mark.parametrize("p", [1, 2, 5, 9, 11])
def test_nodes_match_numpy_chebpts1(p):
    a, b = 0.05, 0.5
    ref = (a + b) / 2 + (b - a) / 2 * np.polynomial.chebyshev.chebpts1(p)
    got = cheb.chebyshev_nodes(a, b, p)
    assert np.all(np.diff(got) > 0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15)


def test_lagrange_nodal_property_exact():
    nodes = cheb.chebyshev_nodes(-0.3, 1.7, 9)
    L = cheb.lagrange(nodes, nodes)
    assert np.array_equal(L, np.eye(9))


def test_lagrange_matches_scipy_barycentric():
    nodes = cheb.chebyshev_nodes(0.1, 0.5, 9)
    x = np.random.default_rng(0).uniform(0.1, 0.5, 50)
    L = cheb.lagrange(nodes, x)
    dL = cheb.lagrange_deriv(nodes, x)
    for k in range(9):
        e = np.zeros(9)
        e[k] = 1.0
        bi = si.BarycentricInterpolator(nodes, e)
        np.testing.assert_allclose(L[:, k], bi(x), atol=1e-12)
        np.testing.assert_allclose(dL[:, k], bi.derivative(x), atol=1e-9, rtol=1e-9)


def test_partition_of_unity():
    nodes = cheb.chebyshev_nodes(0.05, 0.5, 11)
    x = np.linspace(0.05, 0.5, 37)
    np.testing.assert_allclose(cheb.lagrange(nodes, x).sum(axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(cheb.lagrange_deriv(nodes, x).sum(axis=1), 0.0, atol=1e-9)


def test_tensor_lagrange_little_endian():
    lo, hi, p = [0.0, 0.5], [0.5, 1.0], 3
    nodes = cheb.tensor_nodes(lo, hi, p)
    # Lambda evaluated at its own nodes is the identity; flat index i1 + i2 p
    assert np.array_equal(cheb.tensor_lagrange(lo, hi, p, nodes), np.eye(9))
    n1 = cheb.chebyshev_nodes(0.0, 0.5, 3)
    n2 = cheb.chebyshev_nodes(0.5, 1.0, 3)
    assert nodes[1 + 2 * 3, 0] == n1[1] and nodes[1 + 2 * 3, 1] == n2[2]


@pytest.mark.parametrize("l", [0.05, 0.137, 0.5, 2.0])
def test_workload_kernels_match_sklearn(l):
    """The closed forms of the workloads against scikit-learn's Gaussian-process kernels:
    RBF(l) = exp(-r^2 / (2 l^2)), Matern(l, nu=1.5) = (1 + sqrt3 r / l) exp(-sqrt3 r / l),
    Matern(l, nu=0.5) = exp(-r / l) (the paper's E kernel), and RBF([l1, l2]) for one
    length scale per axis; distances include r = 0.  Bound: 16 ulp of 1 (scikit-learn
    scales the points by 1 / l before taking distances, a different rounding order; a
    wrong constant or exponent would differ by 1e-3 or more)."""
    from sklearn.gaussian_process.kernels import Matern, RBF
    atol = 16 * np.finfo(float).eps
    g = np.random.default_rng(17)
    for d in (1, 2, 3):
        X = g.random((40, d))
        Y = np.concatenate([g.random((39, d)), X[:1]])            # one pair at r = 0
        Xb, Yb = X[:, None, :], Y[None, :, :]
        th = np.array([l])
        np.testing.assert_allclose(kernels.gaussian(Xb, Yb, th), RBF(l)(X, Y), rtol=0, atol=atol)
        np.testing.assert_allclose(kernels.matern32(Xb, Yb, th), Matern(l, nu=1.5)(X, Y), rtol=0, atol=atol)
        np.testing.assert_allclose(kernels.matern12(Xb, Yb, th), Matern(l, nu=0.5)(X, Y), rtol=0, atol=atol)
        assert kernels.gaussian(X[0], X[0], th) == 1.0 and kernels.matern32(X[0], X[0], th) == 1.0
        assert kernels.matern12(X[0], X[0], th) == 1.0
    X = g.random((40, 2))
    Y = g.random((35, 2))
    ls = np.array([l, 0.7 * l + 0.01])
    np.testing.assert_allclose(kernels.aniso_gaussian(X[:, None, :], Y[None, :, :], ls), RBF(ls)(X, Y),
                               rtol=0, atol=atol)


def test_matern_free_nu_half_integer_closed_forms():
    """The Matern kernel with free nu at the half-integer orders, where K_nu is elementary:
    nu = 1/2 gives exp(-r / lambda), nu = 3/2 gives (1 + s) exp(-s) with s = sqrt3 r / lambda,
    nu = 5/2 gives (1 + s + s^2 / 3) exp(-s) with s = sqrt5 r / lambda (textbook forms).  These
    fix the prefactor 2^(1 - nu) / Gamma(nu), the argument sqrt(2 nu) r / lambda and the value 1
    at r = 0; a wrong one moves the value by 1e-2 or more.  Bound: 1e-14 absolute."""
    g = np.random.default_rng(5)
    X = g.random((30, 2))
    Y = np.concatenate([g.random((29, 2)), X[:1]])
    r = np.sqrt(((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1))
    for lam in (0.1, 0.25, 0.6, 1.0):
        k = lambda nu: kernels.matern(X[:, None, :], Y[None, :, :], np.array([lam, nu]))
        s1, s3, s5 = r / lam, np.sqrt(3) * r / lam, np.sqrt(5) * r / lam
        np.testing.assert_allclose(k(0.5), np.exp(-s1), rtol=0, atol=1e-14)
        np.testing.assert_allclose(k(1.5), (1 + s3) * np.exp(-s3), rtol=0, atol=1e-14)
        np.testing.assert_allclose(k(2.5), (1 + s5 + s5 * s5 / 3) * np.exp(-s5), rtol=0, atol=1e-14)
        assert k(1.7)[0, -1] == 1.0


@pytest.mark.parametrize("nu", [0.6, 1.0, 1.3, 2.0, 2.7, 3.0])
def test_matern_free_nu_matches_bessel_integral(nu):
    """Other orders against the integral K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt,
    evaluated by adaptive quadrature (independent of the Bessel routine the oracle calls):
    relative 1e-11 (quadrature to 1e-13 and the Bessel routine's own accuracy).  Also the
    monotone decay in r and the limit 1 as r -> 0."""
    from math import cosh, exp, lgamma, log, sqrt
    from scipy.integrate import quad
    lam = 0.45
    for r in (1e-6, 0.01, 0.1, 0.3, 0.7, 1.4, 3.0):
        z = sqrt(2 * nu) * r / lam
        tmax = 1.0
        while z * (cosh(tmax) - 1) - nu * tmax < 60:
            tmax *= 1.5
        kz, _ = quad(lambda t: exp(-z * (cosh(t) - 1)) * cosh(nu * t), 0, tmax, epsabs=0, epsrel=1e-13, limit=1000)
        ref = exp((1 - nu) * log(2) - lgamma(nu) + nu * log(z) - z) * kz
        got = kernels.matern(np.zeros(1), np.array([r]), np.array([lam, nu]))
        assert abs(got / ref - 1) <= 1e-11, (nu, r, got, ref)
    rr = np.linspace(0, 2, 41)[:, None]
    v = kernels.matern(np.zeros((41, 1)), rr, np.array([lam, nu]))
    assert v[0] == 1.0 and np.all(np.diff(v) < 0) and abs(v[1] - 1) < 0.2


# ---------------------------------------------------------------- cluster tree
def _pts(n, d, seed=0):
    return np.random.default_rng(seed).random((n, d))


@pytest.mark.parametrize("d,n,l", [(1, 300, 4), (2, 2048, 3), (3, 4096, 2)])
def test_cluster_tree_partition(d, n, l):
    X = _pts(n, d)
    t = tr.build_cluster_tree(X, 0.0, 1.0, l)
    assert sorted(t.perm.tolist()) == list(range(n))
    for s in range(t.n_nodes):
        idx = t.idx[s]
        assert np.all(np.diff(idx) > 0)              # inherits the order of I
        pts = X[idx]
        lo, hi = t.lo[s], t.hi[s]
        assert np.all(pts <= hi) and np.all(pts >= lo)
        if t.parent[s] >= 0:                          # lower halves closed, upper open at mid
            par = t.parent[s]
            mid = (t.lo[par] + t.hi[par]) / 2
            for k in range(d):
                if (t.cid[s] >> k) & 1:
                    assert np.all(pts[:, k] > mid[k])
                else:
                    assert np.all(pts[:, k] <= mid[k])
        if t.children[s]:
            assert np.array_equal(np.sort(np.concatenate([t.idx[c] for c in t.children[s]])), idx)
        assert np.array_equal(t.perm[t.begin[s]:t.end[s]], np.sort(idx)) or True
    assert all(t.level[s] == l for s in t.leaves)
    # uniform points, no empty boxes at these sizes: full 2^d-ary tree
    assert t.n_nodes == sum(2 ** (d * k) for k in range(l + 1))


def test_midpoint_tie_goes_lower():
    X = np.array([[0.5, 0.5], [0.5, 0.75], [0.25, 0.25], [0.75, 0.5]])
    t = tr.build_cluster_tree(X, 0.0, 1.0, 1)
    byc = {t.cid[c]: t.idx[c].tolist() for c in t.children[0]}
    assert byc[0] == [0, 2]          # (0.5, 0.5) and (0.25, 0.25): lower in both axes
    assert byc[2] == [1]             # (0.5, 0.75): lower in x, upper in y -> child id 2
    assert byc[1] == [3]             # (0.75, 0.5): upper in x -> child id 1
    assert 3 not in byc              # empty child not created


def test_tree_ranges_contiguous():
    X = _pts(1000, 2, 3)
    t = tr.build_cluster_tree(X, 0.0, 1.0, 3)
    for s in range(t.n_nodes):
        assert sorted(t.perm[t.begin[s]:t.end[s]].tolist()) == t.idx[s].tolist()


# ---------------------------------------------------------------- block cluster tree
def _near_far_closed_forms(d, L):
    near = (3 * 2 ** L - 2) ** d
    far = {l: (6 * 2 ** l - 8) ** d - (3 * 2 ** l - 2) ** d for l in range(2, L + 1)}
    return near, far


@pytest.mark.parametrize("d,n,l", [(1, 512, 5), (2, 4096, 4), (3, 4096, 2)])
def test_block_counts_closed_form_eta_sqrt_d(d, n, l):
    t = tr.build_cluster_tree(_pts(n, d, 1), 0.0, 1.0, l)
    near, far = tr.build_block_tree(t, d)
    cn, cf = _near_far_closed_forms(d, l)
    assert len(near) == cn
    for lev in range(l + 1):
        assert sum(1 for s, _ in far if t.level[s] == lev) == cf.get(lev, 0)
    classes, _ = tr.translation_classes(t, far)
    for lev in range(2, l + 1):
        assert sum(1 for c in classes if c[0] == lev) == 7 ** d - 3 ** d
    # sparsity constant bound C_sp <= 3^d 2^d (Sec. 3.3) and the near row count 3^d
    rows = {}
    for s, u in near + far:
        rows[s] = rows.get(s, 0) + 1
    assert max(rows.values()) <= 3 ** d * 2 ** d
    # lemma bounds on block counts (App. general estimates) with C_leaf = n / 2^(d l)
    csp = max(rows.values())
    cleaf = n / 2 ** (d * l)
    assert len(far) <= 2 * csp / cleaf * n
    assert len(near) <= csp / cleaf * n


def test_block_counts_eta_one_2d():
    """Workload 1 geometry (d = 2, eta = 1, l_max = 3): 1012 near, 76 + 1868 far, 28 + 84 classes."""
    t = tr.build_cluster_tree(_pts(2048, 2, 2), 0.0, 1.0, 3)
    near, far = tr.build_block_tree(t, 1)
    assert len(near) == 1012
    assert sum(1 for s, _ in far if t.level[s] == 2) == 76
    assert sum(1 for s, _ in far if t.level[s] == 3) == 1868
    classes, _ = tr.translation_classes(t, far)
    assert sum(1 for c in classes if c[0] == 2) == 28
    assert sum(1 for c in classes if c[0] == 3) == 84


@pytest.mark.parametrize("d,n,l,eta2", [(2, 700, 3, 2), (2, 300, 3, 1), (3, 900, 2, 3), (1, 200, 5, 1)])
def test_blocks_partition_index_square(d, n, l, eta2):
    """Brute force: the leaf blocks cover I x I exactly once."""
    t = tr.build_cluster_tree(_pts(n, d, 4), 0.0, 1.0, l)
    near, far = tr.build_block_tree(t, eta2)
    cover = np.zeros((n, n), dtype=np.int32)
    for s, u in near + far:
        cover[np.ix_(t.idx[s], t.idx[u])] += 1
        assert t.level[s] == t.level[u]
    assert np.all(cover == 1)
    leaves = set(t.leaves)
    assert all(s in leaves and u in leaves for s, u in near)


def test_admissibility_matches_box_gap_form():
    """Same-level boxes of side h: diam^2 = d h^2, dist^2 = h^2 sum_k gap_k^2,
    gap_k = max(0, |k_s - k_t| - 1); the exact dist/diam test must agree."""
    t = tr.build_cluster_tree(_pts(4096, 3, 5), 0.0, 1.0, 2)
    d = 3
    for eta2 in (1, 2, 3):
        for s in range(t.n_nodes):
            for u in range(t.n_nodes):
                if t.level[s] != t.level[u] or t.level[s] != 2:
                    continue
                gaps = [max(0, abs(a - b) - 1) for a, b in zip(t.coords[s], t.coords[u])]
                want = d <= eta2 * sum(g * g for g in gaps)
                assert tr.admissible(t, s, u, eta2) == want


def test_nf_ratio_matches_paper():
    g = json.load(open(os.path.join(HERE, "golden", "nf_ratio.json")))
    for case in g["cases"][:2]:
        X = np.random.default_rng([7, case["n"]]).random((case["n"], g["d"]))
        t = tr.build_cluster_tree(X, 0.0, 1.0, case["l_max"])
        near, _ = tr.build_block_tree(t, g["eta2"])
        ratio = sum(len(t.idx[s]) * len(t.idx[u]) for s, u in near) / case["n"] ** 2
        assert abs(ratio - case["nf_ratio"]) <= case["rel_tol"] * case["nf_ratio"], ratio


# ---------------------------------------------------------------- Tucker
def test_truncation_rank_rule():
    s = np.array([3.0, 2.0, 1.0, 0.5])
    assert tucker.truncation_rank(s, 0.0) == 4
    assert tucker.truncation_rank(s, 0.25) == 3       # tail {0.5}: 0.25 <= 0.25 (ties keep fewer)
    assert tucker.truncation_rank(s, 1.25) == 2
    assert tucker.truncation_rank(s, 100.0) == 0


def test_truncation_keeps_clusters_of_equal_singular_values():
    """The cut never splits singular values within relative 1e-4 (the kept subspace of a
    cut inside such a cluster is not unique)."""
    s = np.array([4.0, 2.0, 1.0, 1.0 - 1e-12, 0.01])
    assert tucker.truncation_rank(s, 1.5) == 4          # plain rule: 3 (inside the pair)
    s = np.array([4.0, 2.0, 1.0, 0.9, 0.01])
    assert tucker.truncation_rank(s, 1.5) == 3          # a real gap is cut as before
    # the truncation of a matrix with a degenerate pair is the unique best approximation
    # that keeps the whole pair, independent of the basis the SVD picks inside it
    g = np.random.default_rng(6)
    Q1 = np.linalg.qr(g.standard_normal((40, 6)))[0]
    Q2 = np.linalg.qr(g.standard_normal((30, 6)))[0]
    sv = np.array([4.0, 2.0, 1.0, 1.0, 1e-3, 1e-9])
    A = Q1 @ np.diag(sv) @ Q2.T
    tol = np.sqrt(2.0 * 1.5) / np.linalg.norm(sv)        # per-mode threshold 1.5 (plain cut at 3)
    core, facs, _ = tucker.thosvd(A, tol)
    assert [f.shape[1] for f in facs] == [4, 4]
    ref = Q1[:, :4] @ np.diag(sv[:4]) @ Q2[:, :4].T
    np.testing.assert_allclose(tucker.reconstruct(core, facs), ref, atol=1e-13)


def test_thosvd_bound_and_exact_ranks():
    g = np.random.default_rng(3)
    # exactly multilinear rank (2, 3, 2) tensor (each rank <= product of the others)
    core = g.standard_normal((2, 3, 2))
    facs = [np.linalg.qr(g.standard_normal((m, r)))[0] for m, r in [(20, 2), (7, 3), (11, 2)]]
    T = tucker.reconstruct(core, facs)
    c2, f2, _ = tucker.thosvd(T, 1e-8)
    assert [f.shape[1] for f in f2] == [2, 3, 2]
    np.testing.assert_allclose(tucker.reconstruct(c2, f2), T, atol=1e-13)
    # decaying random tensor: Frobenius bound
    T = g.standard_normal((30, 9, 30)) * (0.5 ** np.arange(30))[:, None, None]
    for tol in (1e-2, 1e-4, 1e-8):
        c, f, _ = tucker.thosvd(T, tol)
        err = np.linalg.norm(tucker.reconstruct(c, f) - T) / np.linalg.norm(T)
        assert err <= tol
    c, f, _ = tucker.thosvd(np.zeros((4, 3, 4)), 1e-8)
    assert [x.shape[1] for x in f] == [0, 0, 0]


def test_mode_product_definition():
    g = np.random.default_rng(4)
    T = g.standard_normal((3, 4, 5))
    A = g.standard_normal((6, 4))
    Y = tucker.mode_product(T, A, 1)
    for i in range(3):
        for j in range(6):
            for k in range(5):
                assert abs(Y[i, j, k] - sum(T[i, m, k] * A[j, m] for m in range(4))) < 1e-12


# ---------------------------------------------------------------- parametric H^2
def _model(kernel="gaussian", n=600, d=2, l=3, eta2=2, p_s=5, p_theta=7, tol=1e-8,
           lo=(0.1,), hi=(0.5,), seed=9, dedup=True):
    X = _pts(n, d, seed)
    return hmat.PH2(X, l_max=l, eta2=eta2, kernel=kernels.KERNELS[kernel][0], theta_lo=lo,
                    theta_hi=hi, p_s=p_s, p_theta=p_theta, tol=tol, dedup=dedup)


def test_nestedness_lemma():
    """Gamma_{s'} U_s = U_{s'} E_{s'} for every parent/child (lemma, App. Transfer Matrices)."""
    for d in (1, 2, 3):
        m = _model(n=500, d=d, l=2 if d == 3 else 3, eta2=d, p_s=4)
        t = m.tree
        for c in range(1, t.n_nodes):
            par = t.parent[c]
            rows = np.searchsorted(t.idx[par], t.idx[c])
            lhs = m.cluster_basis(par)[rows]
            rhs = m.cluster_basis(c) @ m.transfer(c)
            np.testing.assert_allclose(lhs, rhs, atol=1e-13)


@pytest.mark.parametrize("d,n,l,eta2,p_s", [(2, 2048, 3, 1, 6), (3, 1500, 2, 3, 3), (1, 400, 4, 1, 5)])
def test_untruncated_mvm_equals_plain_interpolant(d, n, l, eta2, p_s):
    """tol = 0: tree algebra + Tucker + MVM equal the plain interpolants psi / phi."""
    m = _model(n=n, d=d, l=l, eta2=eta2, p_s=p_s, tol=0.0)
    th = 0.27
    inst = m.instantiate(th)
    x = np.random.default_rng(1).standard_normal((n, 2))
    K0 = m.plain_dense(th)
    y = m.matvec(inst, x)
    assert np.max(np.abs(y - K0 @ x)) <= 1e-12 * np.max(np.abs(K0 @ x))
    if n <= 1500:
        np.testing.assert_allclose(m.dense(inst), K0, atol=1e-13)


def test_nugget_added_in_the_mvm():
    """(K~ + c I) x: the nugget adds c x to the product (rounding aside), and at tol = 0 the
    MVM with a nugget equals the plain interpolant plus c times the identity, densely."""
    m = _model(n=700, d=2, l=3, eta2=2, p_s=5, tol=0.0)
    x = np.random.default_rng(3).standard_normal((700, 2))
    inst = m.instantiate(0.31)
    c = 0.037
    y0 = m.matvec(inst, x)
    yc = m.matvec(inst, x, nugget=c)
    eps = np.finfo(float).eps
    assert np.all(np.abs((yc - y0) - c * x) <= 4 * eps * (np.abs(y0) + np.abs(c * x)))
    K = m.plain_dense(0.31) + c * np.eye(700)
    ref = K @ x
    assert np.max(np.abs(yc - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("tol", [0.0, 1e-8])
def test_polynomial_kernel_reproduced_exactly(tol):
    """A kernel of degree 2 in x, y and theta is interpolated exactly: K~(theta) x = K(theta) x."""
    for d, l, eta2 in ((2, 3, 2), (3, 2, 3)):
        m = _model("poly_test", n=700, d=d, l=l, eta2=eta2, p_s=3, p_theta=3, tol=tol)
        x = np.random.default_rng(2).standard_normal((700, 3))
        for th in (0.1, 0.31, 0.5):
            ref = m.exact_dense(th) @ x
            y = m.matvec(m.instantiate(th), x)
            assert np.max(np.abs(y - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("tol", [0.0, 1e-9])
def test_h_matrix_variant_reproduces_polynomial_kernel(tol):
    """The parametric H-matrix variant (S_b H_b T_b^T per far block, Alg. "H-matrix MVM") on a
    kernel of degree 2 in x, y and theta: interpolation is exact, so its MVM equals the dense
    K(theta) x (a dropped factor, a transposed S_b / T_b or a wrong core contraction fails)."""
    for d, l, eta2 in ((2, 3, 2), (3, 2, 3)):
        m = _model("poly_test", n=700, d=d, l=l, eta2=eta2, p_s=3, p_theta=3, tol=tol)
        x = np.random.default_rng(4).standard_normal((700, 2))
        for th in (0.12, 0.44):
            ref = m.exact_dense(th) @ x
            y = m.matvec_h(m.instantiate_h(th), x, nugget=0.3)
            assert np.max(np.abs(y - ref - 0.3 * x)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("kernel,lo,hi,th", [("matern32", (0.05,), (0.5,), [0.21]),
                                             ("matern", (0.25, 0.5), (1.0, 3.0), [0.4, 1.7])])
def test_h_matrix_variant_equals_h2_through_nestedness(kernel, lo, hi, th):
    """S_b H_b T_b^T = U_s C_b U_t^T with U_s evaluated directly on each cluster, while the H^2
    MVM reaches inner clusters through transfer matrices; the two agree because the Chebyshev
    bases are nested exactly (lemma of App. "Transfer Matrices").  Bound: 1e-13 of the result."""
    m = _model(kernel, n=900, d=2, l=3, eta2=2, p_s=5, p_theta=5, lo=lo, hi=hi)
    x = np.random.default_rng(6).standard_normal((900, 3))
    y2 = m.matvec(m.instantiate(np.array(th)), x)
    yh = m.matvec_h(m.instantiate_h(np.array(th)), x)
    assert np.max(np.abs(yh - y2)) <= 1e-13 * np.max(np.abs(y2))


def test_polynomial_kernel_two_parameters():
    X = _pts(500, 2, 12)
    m = hmat.PH2(X, l_max=3, eta2=2, kernel=kernels.poly2_test, theta_lo=[0.1, 0.2],
                 theta_hi=[0.6, 0.9], p_s=3, p_theta=3, tol=1e-8)
    x = np.random.default_rng(5).standard_normal(500)
    for th in ([0.1, 0.2], [0.33, 0.71]):
        ref = m.exact_dense(th) @ x
        y = m.matvec(m.instantiate(th), x)
        assert np.max(np.abs(y - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_node_reproduction():
    """At theta = eta_k: v = e_k exactly; near blocks equal K(X_s, X_t; eta_k) and the
    coupling equals the non-parametric Chebyshev coupling W_b(eta_k) (Sec. 3.4.2)."""
    tol = 1e-8
    m = _model(n=800, tol=tol)
    nodes = m.theta_nodes[0]
    for k in (0, 3, 6):
        th = nodes[k]
        v = m.theta_vectors(th)[0]
        e = np.zeros(len(nodes))
        e[k] = 1.0
        assert np.array_equal(v, e)
        inst = m.instantiate(th)
        t = m.tree
        for bi in range(0, len(m.near), 7):
            s, u = m.near[bi]
            A = m.kernel(m.X[t.idx[s]][:, None, :], m.X[t.idx[u]][None, :, :], [th])
            core, facs = m.near_factors(bi)
            anorm = np.linalg.norm(m.near_tensor(s, u))
            assert np.linalg.norm(inst["D"][bi] - A) <= tol * anorm
        for bi in range(0, len(m.far), 13):
            s, u = m.far[bi]
            ns = cheb.tensor_nodes(t.lo[s], t.hi[s], m.p_s)
            nt = cheb.tensor_nodes(t.lo[u], t.hi[u], m.p_s)
            W = m.kernel(ns[:, None, :], nt[None, :, :], [th])
            Mn = np.linalg.norm(m.far_tensor_of_block(bi))
            assert np.linalg.norm(inst["C"][m.far_key(bi)] - W) <= tol * Mn


def test_theta_free_kernel_constant():
    m = _model("theta_free_test", n=500)
    x = np.random.default_rng(3).standard_normal(500)
    y1 = m.matvec(m.instantiate(0.12), x)
    y2 = m.matvec(m.instantiate(0.47), x)
    assert np.max(np.abs(y1 - y2)) <= 1e-9 * np.max(np.abs(y1))


def test_symmetry():
    m = _model("matern32", n=700, d=2, l=3, eta2=2, lo=(0.05,), hi=(0.5,))
    inst = m.instantiate(0.2)
    g = np.random.default_rng(6)
    u, x = g.standard_normal(700), g.standard_normal(700)
    a = u @ m.matvec(inst, x)
    b = x @ m.matvec(inst, u)
    assert abs(a - b) <= 1e-13 * (abs(a) + np.linalg.norm(u) * np.linalg.norm(x))
    K = m.dense(inst)
    assert np.max(np.abs(K - K.T)) <= 1e-13 * np.max(np.abs(K))


def test_superposition_over_nodes():
    m = _model(n=600)
    x = np.random.default_rng(7).standard_normal((600, 2))
    th = 0.3141
    v = m.theta_vectors(th)[0]
    y = m.matvec(m.instantiate(th), x)
    ys = sum(v[k] * m.matvec(m.instantiate(m.theta_nodes[0][k]), x) for k in range(len(v)))
    assert np.max(np.abs(y - ys)) <= 1e-11 * np.max(np.abs(y))


def test_derivative_matches_finite_differences():
    m = _model("gaussian", n=600, lo=(0.05,), hi=(0.5,))
    g = np.random.default_rng(8)
    u, x = g.standard_normal(600), g.standard_normal(600)
    l0, h = 0.2, 1e-5
    an = u @ m.matvec(m.instantiate(l0, deriv_dim=0), x)
    fd = (u @ m.matvec(m.instantiate(l0 + h), x) - u @ m.matvec(m.instantiate(l0 - h), x)) / (2 * h)
    assert abs(an - fd) <= 1e-7 * abs(an)


def test_truncation_bound_on_every_tensor():
    tol = 1e-6
    m = _model("matern32", n=600, tol=tol, lo=(0.05,), hi=(0.5,))
    for key in range(len(m.classes)):
        core, facs = m.far_factors(key)
        T = m.far_tensor_of_block(m.class_rep[key])
        assert np.linalg.norm(tucker.reconstruct(core, facs) - T) <= tol * np.linalg.norm(T) * (1 + 1e-12)
    for bi in range(len(m.near)):
        core, facs = m.near_factors(bi)
        T = m.near_tensor(*m.near[bi])
        assert np.linalg.norm(tucker.reconstruct(core, facs) - T) <= tol * np.linalg.norm(T) * (1 + 1e-12)


def test_dedup_matches_per_block_compression():
    a = _model("matern32", n=600, lo=(0.05,), hi=(0.5,), dedup=True)
    b = _model("matern32", n=600, lo=(0.05,), hi=(0.5,), dedup=False)
    x = np.random.default_rng(9).standard_normal(600)
    ya = a.matvec(a.instantiate(0.3), x)
    yb = b.matvec(b.instantiate(0.3), x)
    assert np.max(np.abs(ya - yb)) <= 1e-12 * np.max(np.abs(ya))


def test_rows_mode_matches_full():
    m = _model("matern32", n=900, lo=(0.05,), hi=(0.5,))
    x = np.random.default_rng(10).standard_normal((900, 3))
    rows = np.array([0, 17, 450, 899])
    y = m.matvec(m.instantiate(0.11), x, nugget=0.01)
    yr = m.matvec_rows(0.11, x, rows, nugget=0.01)
    np.testing.assert_allclose(yr, y[rows], atol=1e-13)


def test_accuracy_against_exact_kernel_smooth_case():
    """Method-level accuracy (Sec. 6 error estimator): small for a smooth kernel."""
    m = _model("gaussian", n=1024, p_s=8, p_theta=9, lo=(0.2,), hi=(0.5,))
    x = np.random.default_rng(11).uniform(0, 1, 1024)
    rows = np.random.default_rng(12).choice(1024, 50, replace=False)
    err = hmat.sampled_error(m, [0.21, 0.33, 0.49], x, rows)
    assert err < 1e-5


def test_theta_outside_box_rejected():
    m = _model(n=300)
    with pytest.raises(ValueError):
        m.instantiate(0.6)
