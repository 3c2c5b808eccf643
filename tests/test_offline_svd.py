"""The library's offline SVD (Householder QR + one-sided Jacobi, host C++) against LAPACK
on the tensors where the two could disagree, through a host-only harness that compiles
the library's offline.cpp into a test shared object.  No GPU.

The case: 3-D Matern-3/2, p_s = 5, p_theta = 7, l in [0.05, 0.5], tol 1e-8.  Far classes
whose box offset is symmetric under swapping two axes have exactly degenerate pairs of
mode singular values, and the Frobenius rank rule can cut between the two members of a
pair (relative gap ~1e-10).  The leading-r subspace is then not unique: each SVD keeps a
different vector of the pair, both truncations satisfy the tolerance bound, and they differ
by about s_r (~1e-8 ||M||), far above rounding.  The rank rule therefore keeps a cluster of
equal singular values whole (relative gap <= 1e-4); with it the two sides keep the same
subspace and their truncations agree to rounding.
"""

import ctypes as C
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from oracle import hmat, kernels, tucker
from paper_2511_03109_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("harness") / "offline_harness.so")
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "host_harness", "offline_harness.cpp"),
           os.path.join(ROOT, "paper_2511_03109_amd", "csrc", "special.cpp"),
           os.path.join(ROOT, "paper_2511_03109_amd", "csrc", "tt.cpp"),
           os.path.join(HERE, "host_harness", "gpu_stub.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    lib = C.CDLL(out)
    dp = C.POINTER(C.c_double)
    lib.harness_left_sv.argtypes = [dp, C.c_int64, C.c_int64, dp, dp]
    lib.harness_left_sv.restype = C.c_int
    lib.harness_thosvd.argtypes = [dp, C.POINTER(C.c_int64), C.c_int, C.c_double, C.POINTER(C.c_int), dp]
    lib.harness_thosvd.restype = None
    lib.harness_tt.argtypes = [dp, C.POINTER(C.c_int), C.c_int, C.c_double, C.POINTER(C.c_int), dp]
    lib.harness_tt.restype = C.c_int64
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _lib_left_sv(lib, X):
    X = np.asfortranarray(X, dtype=np.float64)
    m, q = X.shape
    k = min(m, q)
    s = np.empty(k)
    U = np.empty((m, k), order="F")
    sweeps = lib.harness_left_sv(_ptr(X), m, q, _ptr(s), _ptr(U))
    return s, U, sweeps


def _lib_thosvd(lib, T, tol):
    T = np.asfortranarray(T, dtype=np.float64)
    dims = np.array(T.shape, dtype=np.int64)
    ranks = np.empty(T.ndim, dtype=np.int32)
    rec = np.empty(T.shape, order="F")
    lib.harness_thosvd(_ptr(T), dims.ctypes.data_as(C.POINTER(C.c_int64)), T.ndim, tol,
                       ranks.ctypes.data_as(C.POINTER(C.c_int)), _ptr(rec))
    return ranks, rec


def _plain_rank(s, thr):
    s2 = s ** 2
    tail = np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]])
    return int(np.argmax(tail <= thr))


@pytest.fixture(scope="module")
def degenerate_case():
    n, d = 2000, 3
    X = np.random.default_rng([11, d, n]).random((n, d))
    om = hmat.PH2(X, l_max=2, eta2=Fraction(3), kernel=kernels.matern32, theta_lo=[0.05], theta_hi=[0.5],
                  p_s=5, p_theta=7, tol=1e-8)
    found = []
    for key in range(len(om.classes)):
        M = om.far_tensor_of_block(om.class_rep[key])
        thr = (om.tol ** 2 / M.ndim) * float(np.sum(M * M))
        for m in (0, M.ndim - 1):
            s = np.linalg.svd(tucker.unfold(M, m), compute_uv=False)
            r = _plain_rank(s, thr)
            if 0 < r < len(s) and (s[r - 1] - s[r]) / s[r - 1] < 1e-6:
                found.append((key, m, M, r))
    assert found, "the case has no cut inside a degenerate pair"
    return om, found[:4]


def test_singular_values_match_lapack_and_cut_is_degenerate(harness, degenerate_case):
    om, found = degenerate_case
    for key, m, M, r in found:
        A = tucker.unfold(M, m)
        s_np = np.linalg.svd(A, compute_uv=False)
        s_lib, U_lib, sweeps = _lib_left_sv(harness, A)
        rel = np.max(np.abs(s_lib - s_np)) / s_np[0]
        gap = (s_np[r - 1] - s_np[r]) / s_np[r - 1]
        print(f"class {key} mode {m}: singular values vs LAPACK {rel:.1e} (of s_1), Jacobi sweeps {sweeps}, "
              f"cut r = {r}, relative gap s_r/s_r+1 - 1 = {gap:.1e}")
        assert rel <= 1e-14
        assert sweeps <= 40
        assert gap < 1e-6


def test_plain_cut_is_ambiguous_but_within_bound(harness, degenerate_case):
    """At the plain rule's cut both sides' truncations meet the tolerance, yet keep different
    subspaces: the difference of the two projections of M is ~s_r, not rounding."""
    om, found = degenerate_case
    key, m, M, r = found[0]
    A = tucker.unfold(M, m)
    U_np, s_np, _ = np.linalg.svd(A, full_matrices=False)
    _, U_lib, _ = _lib_left_sv(harness, A)
    nA = np.linalg.norm(A)
    P_np = U_np[:, :r] @ (U_np[:, :r].T @ A)
    P_lib = U_lib[:, :r] @ (U_lib[:, :r].T @ A)
    bound = om.tol / np.sqrt(M.ndim) * nA
    e_np, e_lib = np.linalg.norm(A - P_np), np.linalg.norm(A - P_lib)
    diff = np.linalg.norm(P_np - P_lib)
    print(f"plain cut r = {r}: truncation errors {e_np / nA:.2e}, {e_lib / nA:.2e} (bound {bound / nA:.2e}); "
          f"difference of the two truncations {diff / nA:.2e} of ||M||, s_r = {s_np[r - 1] / nA:.2e}")
    assert e_np <= bound and e_lib <= bound
    assert diff > 1e3 * np.finfo(float).eps * nA
    # keeping the whole pair removes the ambiguity
    r2 = tucker.truncation_rank(s_np, (om.tol ** 2 / M.ndim) * nA ** 2)
    assert r2 > r
    Q_np = U_np[:, :r2] @ (U_np[:, :r2].T @ A)
    Q_lib = U_lib[:, :r2] @ (U_lib[:, :r2].T @ A)
    print(f"cluster cut r = {r2}: difference {np.linalg.norm(Q_np - Q_lib) / nA:.2e} of ||M||")
    assert np.linalg.norm(Q_np - Q_lib) <= 1e-13 * nA


def test_library_thosvd_equals_oracle_on_degenerate_classes(harness, degenerate_case):
    """With the cluster rule, the library's truncated HOSVD of every degenerate class has the
    oracle's ranks and reconstruction to rounding."""
    om, found = degenerate_case
    for key, M in {key: M for key, _, M, _ in found}.items():
        core, facs, _ = tucker.thosvd(M, om.tol)
        rec_o = tucker.reconstruct(core, facs)
        ranks, rec_l = _lib_thosvd(harness, M, om.tol)
        diff = np.linalg.norm(rec_l - rec_o) / np.linalg.norm(M)
        print(f"class {key}: ranks {list(ranks)} vs {[f.shape[1] for f in facs]}, reconstructions differ {diff:.1e}")
        assert list(ranks) == [f.shape[1] for f in facs]
        assert diff <= 1e-13


def test_jacobi_reports_convergence_on_random_matrices(harness):
    g = np.random.default_rng(8)
    for m, q in ((200, 30), (30, 200), (64, 64)):
        A = g.standard_normal((m, q)) @ np.diag(0.7 ** np.arange(q))[:q, :q] if m >= q else g.standard_normal((m, q))
        s_lib, U, sweeps = _lib_left_sv(harness, A)
        s_np = np.linalg.svd(A, compute_uv=False)
        assert np.max(np.abs(s_lib - s_np)) <= 1e-13 * s_np[0]
        assert 1 <= sweeps <= 40
        k = min(m, q)
        np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-13)


def test_jacobi_converges_on_graded_and_underflowing_unfoldings(harness):
    """Two unfoldings on which the one-sided Jacobi iteration used to rotate until its sweep
    cap: a 3-D Matern-1/2 far class whose singular values span 12 orders of magnitude (pairs
    whose cosine sits at the rounding noise of a 64-term inner product), and a near tensor of
    the anisotropic Gaussian whose smallest singular value is ~1e-160 (squared column norms
    underflow).  With sqrt(k) eps as the rotation threshold and columns below eps times the
    largest left alone, both converge in a few sweeps and still match LAPACK."""
    X = np.random.default_rng([5, 3, 1100]).random((1100, 3))
    om = hmat.PH2(X, l_max=2, eta2=Fraction(3), kernel=kernels.matern12, theta_lo=[0.05], theta_hi=[0.5],
                  p_s=4, p_theta=7, tol=1e-8)
    mats = []
    for key in range(len(om.classes)):
        M = om.far_tensor_of_block(om.class_rep[key])
        A = tucker.unfold(M, 2)
        s = np.linalg.svd(A, compute_uv=False)
        if s[-1] < 1e-11 * s[0]:
            mats.append(A)
    Xm = inputs.points_for(3, 3000)
    om2 = hmat.PH2(Xm, l_max=4, eta2=Fraction(2), kernel=kernels.aniso_gaussian, theta_lo=[0.05, 0.05],
                   theta_hi=[0.5, 0.5], p_s=5, p_theta=7, tol=1e-8)
    for bi, (s_, u_) in enumerate(om2.near):
        if s_ > u_:
            continue
        A = tucker.unfold(om2.near_tensor(s_, u_), 1)
        sv = np.linalg.svd(A, compute_uv=False)
        if sv[-1] < 1e-100 * sv[0]:
            mats.append(A)
    assert len(mats) >= 3
    for A in mats:
        s_lib, U, sweeps = _lib_left_sv(harness, A)
        s_np = np.linalg.svd(A, compute_uv=False)
        print(f"{A.shape}: sweeps {sweeps}, s_min/s_max {s_np[-1] / s_np[0]:.1e}, "
              f"singular values vs LAPACK {np.max(np.abs(s_lib - s_np)) / s_np[0]:.1e}")
        assert sweeps <= 30
        assert np.max(np.abs(s_lib - s_np)) <= 1e-13 * s_np[0]


# ---------------------------------------------------------------- TT-cross (tt.cpp vs oracle.tt)
def _lib_tt(lib, T, tol):
    T = np.asfortranarray(T, dtype=np.float64)
    dims = np.array(T.shape, dtype=np.int32)
    ranks = np.empty(T.ndim + 1, dtype=np.int32)
    rec = np.empty(T.shape, order="F")
    ev = lib.harness_tt(_ptr(T), dims.ctypes.data_as(C.POINTER(C.c_int)), T.ndim, tol,
                        ranks.ctypes.data_as(C.POINTER(C.c_int)), _ptr(rec))
    return ranks, rec, ev


def _tt_cases():
    """Far tensors (modes i_1..i_d, k, j_1..j_d) of symmetric and asymmetric classes and near
    tensors (e, k) of a 2-D Gaussian and a 3-D Matern-3/2 model."""
    out = []
    for kern, d, n, l, eta2, lo, hi in (("gaussian", 2, 900, 3, 2, 0.05, 0.5), ("matern32", 3, 1500, 2, 3, 0.05, 0.5)):
        X = np.random.default_rng([5, d]).random((n, d))
        m = hmat.PH2(X, l_max=l, eta2=eta2, kernel=kernels.KERNELS[kern][0], theta_lo=[lo], theta_hi=[hi],
                     p_s=4, p_theta=7, tol=1e-8)
        seen = 0
        for key, (lev, off) in enumerate(m.classes):
            if tuple(off) < tuple(-c for c in off) or seen >= 4:
                continue
            M = m.far_tensor_of_block(m.class_rep[key])
            out.append(M.reshape((4,) * d + (7,) + (4,) * d, order="F"))
            seen += 1
        for bi in (0, len(m.near) // 2):
            s, u = m.near[bi]
            if s <= u:
                out.append(m.near_tensor(s, u))
    return out


@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_library_tt_cross_equals_oracle(harness, tol):
    """The library's TT-cross + TT-rounding (tt.cpp) takes the same pivots as the oracle's on the
    same tensors: the ranks agree exactly and the two TT tensors agree to rounding (1e-10 of the
    largest entry; different pivots would differ by about tol).  Both are within tol ||M||_F."""
    from oracle import tt
    for M in _tt_cases():
        ranks, rec, ev = _lib_tt(harness, M, tol)
        cores, ev_o = tt.tt_compress(lambda idx: M[tuple(idx.T)], list(M.shape), tol)
        assert list(ranks[1:-1]) == [c.shape[2] for c in cores[:-1]]
        assert ev == ev_o
        full = tt.tt_full(cores)
        assert np.max(np.abs(rec - full)) <= 1e-10 * np.max(np.abs(M))
        assert np.linalg.norm(rec - M) <= tol * np.linalg.norm(M)
