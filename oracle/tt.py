"""Tensor-train compression by cross approximation (oracle; test infrastructure only).

Paper: Sec. 2.1 ("Tensor Train Decomposition": TT format, cores G_i of size
r_{i-1} x m_i x r_i, the reshapes G^{1} and G^{2}; TT-cross with partially
pivoted ACA on each supercore; TT-rounding afterwards), App. PTTK review
(L_b from the spatial target cores, H_b(theta) from the parameter cores, R_b
from the spatial source cores), Sec. 4.3 (near tensors in TT format) and
Alg. "Modified H^2-Matrix MVM" (the coupling applied core by core).

The paper names its algorithms (a variant of the greedy cross of Savostyanov,
partially pivoted ACA, a max-norm error heuristic, TT-rounding) without printing
them.  The reading taken here:

* Index sets.  I_k holds r_k multi-indices of modes 0..k-1 (left), J_k holds
  multi-indices of modes k..N-1 (right).  All start from one index (the middle
  node of every mode).
* Supercore k (modes k, k+1) is the matrix with rows (alpha, i_k), alpha over
  I_k, alpha fastest, and columns (i_{k+1}, beta), beta over J_{k+2}, i_{k+1}
  fastest -- the column-major reshape of Sec. 2.1.
* ACA with partial pivoting on a supercore: start at the row of the first
  left index with the middle node of mode k; residual row, column pivot =
  largest residual entry, residual column, next row pivot = largest entry of
  that column among unused rows.  A new term u v^T is rejected, and the ACA
  stops, when ||u|| ||v|| <= tol ||S||_F (S the approximation with it, its norm
  updated incrementally) or when its pivot is at rounding level (ZERO_RTOL of the
  largest entry seen); the first term is always kept unless the row vanishes.
  A vanishing residual row is skipped for the next candidate row (largest entry
  of the last residual column, else the first unused row) until all rows are tried.
  Ties: the first index within relative PIVOT_RTOL of the largest magnitude, so
  that rounding cannot reorder exact ties.
* A sweep runs over the supercores left to right; the row pivots of
  supercore k become I_{k+1}, its column pivots J_{k+1}.  Sweeps alternate
  direction.  After every left-to-right sweep from the second on, the max-norm
  error is estimated on N_SAMPLES entries drawn with SplitMix64 (relative to the
  largest sampled entry): the reading of the paper's max-norm heuristic.  The
  iteration stops when the estimate is at most check_tol; otherwise the worst
  sample's suffixes join the right index sets before the next left-to-right
  sweep (enrichment).  At most MAX_ENRICH enrichments and MAX_SWEEPS
  left-to-right sweeps.  (The ranks of an ACA-based cross move by one or two
  from sweep to sweep as its index sets change, so they are no stopping test.)
* Cores from the last left-to-right sweep: G_k = A(I_k x m_k, J_{k+1})
  A(I_{k+1}, J_{k+1})^{-1} for k < N-1 and G_{N-1} = A(I_{N-1} x m_{N-1}), the
  interpolation form of the cross; G_k is evaluated as Q Q(I_{k+1}, :)^{-1} from the
  reduced QR of A(I_k x m_k, J_{k+1}) (the same matrix, better conditioned).
* TT-rounding (Oseledets): right-to-left QR orthogonalisation, then left-to-right
  SVD truncation with delta = tol / sqrt(N-1) ||X||_F per unfolding (at least rank
  1), never cutting a cluster of equal singular values (the rule of
  ``tucker.truncation_rank``).
"""

import numpy as np

from .tucker import truncation_rank

PIVOT_RTOL = 1e-6
ZERO_RTOL = 1e-12
MAX_SWEEPS = 16


def _pivot(vals, used):
    """First index not in ``used`` whose |value| is within PIVOT_RTOL of the largest; -1 if all vanish."""
    a = np.abs(vals)
    a = a.copy()
    if used:
        a[np.fromiter(used, dtype=np.int64)] = -1.0
    mx = a.max() if a.size else -1.0
    if not mx > 0.0:
        return -1
    return int(np.flatnonzero(a >= (1.0 - PIVOT_RTOL) * mx)[0])


def aca(get_row, get_col, m, n, tol, i0):
    """Partially pivoted ACA of an m x n matrix given by row and column accessors.

    Returns (rows, cols, raw_rows, raw_cols): the pivot rows and columns in the
    order chosen and the matrix's own rows / columns at them (not residuals).
    A candidate term is kept only while it is above the tolerance and its pivot is
    above ZERO_RTOL times the largest entry seen, so that the pivot submatrix stays
    well conditioned (a pivot at rounding level would make it singular).  A residual
    row that vanishes is skipped: the next row is the unused one with the largest
    entry of the last residual column, else the first unused row, until every row
    has been tried (an exactly low-rank matrix is thereby resolved completely).
    """
    us, vs = [], []
    rows, cols, raw_rows, raw_cols = [], [], [], []
    used_r, used_c = set(), set()
    norm2 = 0.0
    amax = 0.0
    i = i0
    while len(us) < min(m, n):
        a_row = np.asarray(get_row(i), dtype=np.float64)
        amax = max(amax, float(np.max(np.abs(a_row))))
        r = a_row.copy()
        for u_l, v_l in zip(us, vs):
            r -= u_l[i] * v_l
        used_r.add(i)
        j = _pivot(r, used_c)
        if j < 0 or abs(r[j]) <= ZERO_RTOL * amax:
            # vanishing residual row: try another row
            if len(used_r) == m:
                break
            nxt = _pivot(us[-1], used_r) if us else -1
            i = nxt if nxt >= 0 else min(set(range(m)) - used_r)
            continue
        v = r / r[j]
        a_col = np.asarray(get_col(j), dtype=np.float64)
        amax = max(amax, float(np.max(np.abs(a_col))))
        u = a_col.copy()
        for u_l, v_l in zip(us, vs):
            u -= v_l[j] * u_l
        used_c.add(j)
        cross = 0.0
        for u_l, v_l in zip(us, vs):
            cross += float(np.dot(u_l, u)) * float(np.dot(v_l, v))
        uu, vv = float(np.dot(u, u)), float(np.dot(v, v))
        norm2_new = norm2 + 2.0 * cross + uu * vv
        if us and np.sqrt(uu * vv) <= tol * np.sqrt(max(norm2_new, 0.0)):
            break
        norm2 = norm2_new
        us.append(u)
        vs.append(v)
        rows.append(i)
        cols.append(j)
        raw_rows.append(a_row)
        raw_cols.append(a_col)
        if len(used_r) == m:
            break
        i = _pivot(u, used_r)
        if i < 0:
            i = min(set(range(m)) - used_r)
    return rows, cols, raw_rows, raw_cols

MAX_ENRICH = 8
N_SAMPLES = 256
SAMPLE_SEED = 0x5EED


def splitmix64(state):
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): returns (next state, output), uint64."""
    mask = (1 << 64) - 1
    state = (state + 0x9E3779B97F4A7C15) & mask
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
    return state, z ^ (z >> 31)


def sample_indices(dims, rnd):
    """N_SAMPLES multi-indices for the error check of enrichment round ``rnd``: sample s,
    mode k takes the next SplitMix64 output (seed SAMPLE_SEED + rnd) modulo m_k."""
    st = SAMPLE_SEED + rnd
    out = np.empty((N_SAMPLES, len(dims)), dtype=np.int64)
    for s in range(N_SAMPLES):
        for k, m in enumerate(dims):
            st, z = splitmix64(st)
            out[s, k] = z % m
    return out


def tt_entries(cores, idx):
    """TT entries at the multi-indices idx (rows), by the entry formula of Sec. 2.1."""
    out = np.empty(idx.shape[0])
    for s in range(idx.shape[0]):
        v = cores[0][:, idx[s, 0], :]
        for k in range(1, len(cores)):
            v = v @ cores[k][:, idx[s, k], :]
        out[s] = v[0, 0]
    return out


def sample_error(cores, ent, dims, rnd):
    """Max-norm error estimate of the reading of the paper's heuristic: relative to the
    largest sampled entry; returns (error, worst multi-index)."""
    idx = sample_indices(dims, rnd)
    x = ent(idx)
    e = np.abs(x - tt_entries(cores, idx))
    scale = np.max(np.abs(x))
    w = int(np.argmax(e))
    return (float(e[w] / scale) if scale > 0 else 0.0), idx[w]


def tt_cross(entry, dims, tol, start=None, check_tol=None):
    """TT approximation of the tensor with mode sizes ``dims`` (column-major
    multi-indices) whose entries ``entry(idx)`` returns for an integer array idx of
    shape (k, N).  Returns (cores, evals): cores[k] of shape (r_k, m_k, r_{k+1}),
    r_0 = r_N = 1, and the number of distinct entries evaluated.  ``tol`` is the ACA
    tolerance of every supercore; ``check_tol`` (default tol) the max-norm tolerance of
    the sampled error check."""
    dims = [int(m) for m in dims]
    if check_tol is None:
        check_tol = tol
    N = len(dims)
    if start is None:
        start = [m // 2 for m in dims]
    evals = [0]
    # every entry is evaluated at most once (the sweeps revisit supercore entries)
    strides = np.cumprod([1] + dims[:-1]).astype(np.int64)
    cache = np.full(int(np.prod(dims)), np.nan)

    def ent(idx):
        idx = np.asarray(idx, dtype=np.int64).reshape(-1, N)
        lin = idx @ strides
        miss = np.unique(lin[np.isnan(cache[lin])])
        if miss.size:
            mi = (miss[:, None] // strides[None, :]) % np.asarray(dims, dtype=np.int64)[None, :]
            cache[miss] = np.asarray(entry(mi), dtype=np.float64).reshape(-1)
            evals[0] += miss.size
        return cache[lin]

    if N == 1:
        return [ent(np.arange(dims[0])[:, None]).reshape(1, dims[0], 1)], evals[0]
    left = [np.zeros((1, 0), dtype=np.int64)] + [np.array([start[:k]], dtype=np.int64) for k in range(1, N)]
    right = [np.array([start[k:]], dtype=np.int64) for k in range(N)] + [np.zeros((1, 0), dtype=np.int64)]

    def supercore(k):
        """ACA of supercore k; returns (row multi-indices, col multi-indices, aca result)."""
        Il, Jr = left[k], right[k + 2]
        a, mk, mk1, b = Il.shape[0], dims[k], dims[k + 1], Jr.shape[0]
        # row rho = alpha + a i ; col c = i' + mk1 beta
        rows_mi = np.concatenate([np.tile(Il, (mk, 1)), np.repeat(np.arange(mk), a)[:, None]], axis=1)
        cols_mi = np.concatenate([np.tile(np.arange(mk1), b)[:, None], np.repeat(Jr, mk1, axis=0)], axis=1)

        def get_row(rho):
            full = np.concatenate([np.broadcast_to(rows_mi[rho], (cols_mi.shape[0], k + 1)), cols_mi], axis=1)
            return ent(full)

        def get_col(c):
            full = np.concatenate([rows_mi, np.broadcast_to(cols_mi[c], (rows_mi.shape[0], N - k - 1))], axis=1)
            return ent(full)

        i0 = 0 + a * start[k]
        res = aca(get_row, get_col, a * mk, mk1 * b, tol, i0)
        return rows_mi, cols_mi, res

    def assemble(last):
        cores = []
        rl = 1
        for k in range(N - 1):
            rp, cp, raw_rows, raw_cols = last[k]
            C = np.stack(raw_cols, axis=1)                   # (r_k m_k) x r_{k+1}
            # C A^{-1} with A = C[rp] the pivot submatrix, formed as Q Q[rp]^{-1} from C = Q R:
            # the same matrix, but Q[rp] is far better conditioned than A
            Q, _ = np.linalg.qr(C)
            G = np.linalg.solve(Q[rp, :].T, Q.T).T
            cores.append(G.reshape(rl, dims[k], len(rp), order="F"))
            rl = len(rp)
            if k == N - 2:
                # last core: the supercore's own rows at the pivot rows, A(I_{N-1} x m_{N-1})
                Rw = np.stack(raw_rows, axis=0)              # r x m_{N-1}
                cores.append(Rw.reshape(rl, dims[N - 1], 1, order="F"))
        return cores

    def sweep(order):
        out = {}
        for k in order:
            rows_mi, cols_mi, res = supercore(k)
            if not res[0]:
                return None
            left[k + 1] = rows_mi[res[0]]
            right[k + 1] = cols_mi[res[1]]
            out[k] = res
        return out

    zero = [np.zeros((1, m, 1)) for m in dims]
    rounds = 0
    cores = None
    for it in range(MAX_SWEEPS):
        last = sweep(range(N - 1))
        if last is None:
            return zero, evals[0]
        cores = assemble(last)
        worst = None
        if it >= 1:
            err, w = sample_error(cores, ent, dims, rounds)
            if err <= check_tol or rounds == MAX_ENRICH:
                break
            rounds += 1
            worst = w
        if sweep(range(N - 2, -1, -1)) is None:
            return zero, evals[0]
        if worst is not None:
            # enrichment: the worst sampled index joins every right index set, so that the
            # next left-to-right sweep sees the directions the cross has missed
            for k in range(1, N):
                suf = np.asarray(worst[k:], dtype=np.int64)[None, :]
                if not np.any(np.all(right[k] == suf, axis=1)):
                    right[k] = np.concatenate([right[k], suf], axis=0)
    return cores, evals[0]


def tt_full(cores):
    """The full tensor of a TT (Sec. 2.1 entry formula), column-major multi-indices."""
    X = cores[0].reshape(-1, cores[0].shape[2], order="F")  # (m_0) x r_1
    for G in cores[1:]:
        r0, m, r1 = G.shape
        X = (X @ G.reshape(r0, m * r1, order="F")).reshape(-1, r1, order="F")
    return X.reshape([G.shape[1] for G in cores], order="F")


def tt_round(cores, tol):
    """TT-rounding: right-to-left QR, then left-to-right truncated SVD with
    delta = tol / sqrt(N-1) ||X||_F (at least rank 1 per unfolding)."""
    cores = [np.array(G, dtype=np.float64) for G in cores]
    N = len(cores)
    if N == 1:
        return cores
    for k in range(N - 1, 0, -1):
        r0, m, r1 = cores[k].shape
        Q, R = np.linalg.qr(cores[k].reshape(r0, m * r1, order="F").T)
        cores[k] = Q.T.reshape(Q.shape[1], m, r1, order="F")
        a0, m0, a1 = cores[k - 1].shape
        cores[k - 1] = (cores[k - 1].reshape(a0 * m0, a1, order="F") @ R.T).reshape(a0, m0, R.shape[0], order="F")
    delta2 = (tol * tol / (N - 1)) * float(np.sum(cores[0] * cores[0]))
    for k in range(N - 1):
        a0, m, a1 = cores[k].shape
        U, s, Vt = np.linalg.svd(cores[k].reshape(a0 * m, a1, order="F"), full_matrices=False)
        r = max(1, truncation_rank(s, delta2))
        cores[k] = U[:, :r].reshape(a0, m, r, order="F")
        b0, mb, b1 = cores[k + 1].shape
        SV = s[:r, None] * Vt[:r, :]
        cores[k + 1] = (SV @ cores[k + 1].reshape(b0, mb * b1, order="F")).reshape(r, mb, b1, order="F")
    return cores


def far_factors(cores, d, d_theta):
    """App. PTTK review: L (P x r_d) from the spatial target cores, R (P x r_{d+dθ}) from
    the spatial source cores (node index little-endian over the axes), and the parameter
    cores as a Tucker core (r_d, p_theta[, p_theta], r_{d+dθ}) with identity parameter
    factors, so that H(theta) = core contracted with v_1(theta_1) [, v_2(theta_2)]."""
    L = cores[0].reshape(cores[0].shape[1], cores[0].shape[2], order="F")
    for G in cores[1:d]:
        r0, m, r1 = G.shape
        L = (L @ G.reshape(r0, m * r1, order="F")).reshape(-1, r1, order="F")
    Y = cores[-1].reshape(cores[-1].shape[0], cores[-1].shape[1], order="F")     # r x m
    for G in reversed(cores[d + d_theta:-1]):
        r0, m, r1 = G.shape
        Y = (G.reshape(r0 * m, r1, order="F") @ Y).reshape(r0, -1, order="F")
    R = Y.T
    core = cores[d]
    if d_theta == 2:
        G1, G2 = cores[d], cores[d + 1]
        core = np.einsum("akc,clb->aklb", G1, G2)
    p = cores[d].shape[1]
    return core, [L] + [np.eye(p)] * d_theta + [R]


def near_factors(cores, d_theta):
    """Sec. 4.3 in TT form: U_e = reshape(G_1, [N_e, r_1]) and the parameter cores as a
    Tucker core (r_1, p_theta[, p_theta]) with identity parameter factors."""
    U = cores[0].reshape(cores[0].shape[1], cores[0].shape[2], order="F")
    if d_theta == 1:
        core = cores[1][:, :, 0]
    else:
        core = np.einsum("akc,cl->akl", cores[1], cores[2][:, :, 0])
    p = cores[1].shape[1]
    return core, [U] + [np.eye(p)] * d_theta


def implicit_coupling_apply(cores, d, d_theta, vs, xh):
    """Alg. "Modified H^2-Matrix MVM", multiplication stage for one far block: C x_hat with C
    kept as TT cores.  The source-side cores are applied from the last one down (each a
    reshape of z times G^{1} transposed), then H(theta) from the parameter cores and the
    vectors v_i, then the target-side cores from the last one down (G^{2} times a
    reshape of z).  xh: (P,) or (P, R)."""
    xh = np.asarray(xh, dtype=np.float64)
    Rr = 1 if xh.ndim == 1 else xh.shape[1]
    N = len(cores)
    p = cores[-1].shape[1]
    out = []
    for c in range(Rr):
        z = xh if xh.ndim == 1 else xh[:, c]
        rr = 1
        for i in range(d):
            G = cores[N - 1 - i]
            r0, m, r1 = G.shape
            Z = z.reshape(p ** (d - i - 1), m * r1, order="F")
            z = (Z @ G.reshape(r0, m * r1, order="F").T).reshape(-1, order="F")
            rr = r0
        H = np.eye(cores[d].shape[0])
        for i in range(d_theta):
            G = cores[d + i]
            H = H @ np.tensordot(G, vs[i], axes=([1], [0]))
        z = H @ z.reshape(rr)
        for i in range(d):
            G = cores[d - 1 - i]
            r0, m, r1 = G.shape
            Z = z.reshape(r1, p ** i, order="F")
            z = (G.reshape(r0 * m, r1, order="F") @ Z).reshape(-1, order="F")
        out.append(z)
    return out[0] if xh.ndim == 1 else np.stack(out, axis=1)


CROSS_TOL_FACTOR = 0.1
CHECK_TOL_FACTOR = 10.0


def tt_compress(entry, dims, tol):
    """TT-cross at CROSS_TOL_FACTOR * tol followed by TT-rounding at tol (Sec. 2.1: the cross
    approximation is rounded afterwards).  Reading: the cross runs ten times tighter than
    the target so that the rounded TT stays within about tol ||X||_F (the cross alone
    lands at a few times its own tolerance).  The sampled max-norm check runs at
    CHECK_TOL_FACTOR * tol: it is there to catch directions the cross has missed, whose
    error is orders of magnitude above the tolerance, while an ACA resolved to its
    Frobenius tolerance shows max-norm errors of a few times that tolerance, which further
    sweeps would not reduce.  Returns (cores, evals)."""
    cores, evals = tt_cross(entry, dims, CROSS_TOL_FACTOR * tol, check_tol=CHECK_TOL_FACTOR * tol)
    return tt_round(cores, tol), evals
