// Tensor-train compression of the offline stage's tensors (Sec. 2.1 "Tensor Train
// Decomposition" of arxiv 2511.03109): TT-cross with partially pivoted ACA on each supercore,
// followed by TT-rounding.  The paper names the algorithms (a variant of Savostyanov's greedy
// cross, partially pivoted ACA, a max-norm error heuristic, TT-rounding) without printing them;
// the reading implemented here:
//
//  * Index sets: I_k (r_k multi-indices of modes 0..k-1) and J_k (of modes k..N-1), all started
//    from one index, the middle node of every mode.
//  * Supercore k (modes k, k+1): rows (alpha, i_k), alpha over I_k and fastest; columns
//    (i_{k+1}, beta), beta over J_{k+2}, i_{k+1} fastest (the column-major reshape).
//  * ACA with partial pivoting: start at row (first left index, middle node of mode k); residual
//    row, column pivot = its largest entry, residual column, next row pivot = the largest entry
//    of that column among unused rows.  A new term u v^T is rejected (and the ACA stops) when
//    |u| |v| <= tol |S|_F, S the approximation with it (norm updated incrementally), or when its
//    pivot is at rounding level (ZERO_RTOL of the largest entry seen); the first term is always
//    kept.  A vanishing residual row is skipped for the next candidate (largest entry of the last
//    residual column among unused rows, else the first unused row) until every row was tried.
//    Ties: the first index within relative PIVOT_RTOL of the largest magnitude, so rounding
//    cannot reorder exact ties (symmetric geometry produces them).
//  * Sweeps alternate direction; pivots of supercore k become I_{k+1} and J_{k+1}.  After every
//    left-to-right sweep from the second on, the max-norm error is estimated on N_SAMPLES entries
//    drawn with SplitMix64 (relative to the largest sampled entry); the iteration stops when it is
//    at most the check tolerance, else the worst sample's suffixes join the right index sets
//    before the next left-to-right sweep (enrichment).  At most MAX_ENRICH enrichments and
//    MAX_SWEEPS sweeps.  (The ranks of an ACA-based cross move by one or two from sweep to sweep
//    as its index sets change, so they are no stopping test.)
//  * Cores from the last left-to-right sweep: G_k = A(I_k x m_k, J_{k+1}) A(I_{k+1}, J_{k+1})^-1,
//    G_{N-1} = A(I_{N-1} x m_{N-1}): the interpolation form of the cross, with G_k evaluated as
//    Q Q(I_{k+1}, :)^-1 from the reduced QR of A(I_k x m_k, J_{k+1}) (same matrix, better
//    conditioned).
//  * TT-rounding (Oseledets): right-to-left QR orthogonalisation, then left-to-right truncated
//    SVD with delta = tol / sqrt(N-1) |X|_F per unfolding (rank >= 1), with the cluster rule of
//    truncation_rank.
//  * The cross runs at tol / 10 and the rounding at tol, so that the rounded TT lands within about
//    tol |X|_F (the cross alone lands at a few times its own tolerance).  The sampled check runs
//    at 10 tol: it catches directions the cross has missed (errors orders of magnitude above the
//    tolerance); an ACA resolved to its Frobenius tolerance shows max-norm errors of a few times
//    that tolerance, which further sweeps would not reduce.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <unordered_map>

#include "ph_host.hpp"

namespace ph {
namespace {

constexpr double PIVOT_RTOL = 1e-6;
constexpr double ZERO_RTOL = 1e-12;
constexpr int MAX_SWEEPS = 16;
constexpr int MAX_ENRICH = 8;
constexpr int N_SAMPLES = 256;
constexpr uint64_t SAMPLE_SEED = 0x5EED;
constexpr double CROSS_TOL_FACTOR = 0.1;
constexpr double CHECK_TOL_FACTOR = 10.0;

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
uint64_t splitmix64(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// First index not marked used whose magnitude is within PIVOT_RTOL of the largest; -1 if all
// unused entries vanish.
int pivot(const std::vector<double>& v, const std::vector<char>& used) {
  double mx = -1.0;
  for (size_t i = 0; i < v.size(); ++i)
    if (!used[i]) mx = std::max(mx, std::fabs(v[i]));
  if (!(mx > 0.0)) return -1;
  const double thr = (1.0 - PIVOT_RTOL) * mx;
  for (size_t i = 0; i < v.size(); ++i)
    if (!used[i] && std::fabs(v[i]) >= thr) return (int)i;
  return -1;
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

// The tensor seen through its accessor, every entry evaluated at most once: a dense cache for
// tensors up to DENSE_MAX entries, a hash map beyond (the cross touches a small part of those).
constexpr int64_t DENSE_MAX = (int64_t)1 << 24;
struct Tensor {
  EntryFn fn;
  const void* ctx;
  std::vector<int> dims;
  std::vector<int64_t> stride;
  bool dense;
  std::vector<double> val;
  std::vector<char> have;
  std::unordered_map<int64_t, double> sparse;
  int64_t evals = 0;
  Tensor(EntryFn f, const void* c, const std::vector<int>& d) : fn(f), ctx(c), dims(d) {
    int64_t s = 1;
    for (int m : dims) {
      stride.push_back(s);
      s *= m;
    }
    dense = s <= DENSE_MAX;
    if (dense) {
      val.assign((size_t)s, 0.0);
      have.assign((size_t)s, 0);
    }
  }
  int N() const { return (int)dims.size(); }
  // out[s] = X[idx row s], idx count x N row-major
  void get(const std::vector<int32_t>& idx, double* out) {
    const int n = N();
    const int64_t count = (int64_t)idx.size() / n;
    std::vector<int64_t> lin((size_t)count);
    std::vector<int32_t> miss;
    std::vector<int64_t> miss_lin;
    std::unordered_map<int64_t, int> queued;   // sparse mode: entries queued in this call
    for (int64_t s = 0; s < count; ++s) {
      int64_t l = 0;
      for (int k = 0; k < n; ++k) l += stride[k] * idx[(size_t)s * n + k];
      lin[s] = l;
      const bool known = dense ? have[l] != 0 : (sparse.count(l) != 0 || queued.count(l) != 0);
      if (!known) {
        if (dense) have[l] = 2;   // queued
        else queued.emplace(l, 0);
        miss.insert(miss.end(), idx.begin() + s * n, idx.begin() + (s + 1) * n);
        miss_lin.push_back(l);
      }
    }
    if (!miss_lin.empty()) {
      std::vector<double> v(miss_lin.size());
      fn(ctx, miss.data(), (int64_t)miss_lin.size(), v.data());
      for (size_t q = 0; q < miss_lin.size(); ++q) {
        if (dense) {
          val[miss_lin[q]] = v[q];
          have[miss_lin[q]] = 1;
        } else {
          sparse.emplace(miss_lin[q], v[q]);
        }
      }
      evals += (int64_t)miss_lin.size();
    }
    for (int64_t s = 0; s < count; ++s) out[s] = dense ? val[lin[s]] : sparse.find(lin[s])->second;
  }
};

struct Aca {
  std::vector<int> rows, cols;
  std::vector<std::vector<double>> raw_rows, raw_cols;   // the matrix's own rows / columns
};

// Partially pivoted ACA of the m x n matrix given by row(i, out) and col(j, out).
template <typename RowF, typename ColF>
Aca aca(RowF row, ColF col, int m, int n, double tol, int i0) {
  Aca out;
  std::vector<std::vector<double>> us, vs;
  std::vector<char> used_r((size_t)m, 0), used_c((size_t)n, 0);
  int n_used_r = 0;
  double norm2 = 0.0, amax = 0.0;
  int i = i0;
  auto first_unused = [&]() {
    for (int q = 0; q < m; ++q)
      if (!used_r[q]) return q;
    return -1;
  };
  while ((int)us.size() < std::min(m, n)) {
    std::vector<double> a_row((size_t)n);
    row(i, a_row.data());
    for (double x : a_row) amax = std::max(amax, std::fabs(x));
    std::vector<double> r = a_row;
    for (size_t l = 0; l < us.size(); ++l) {
      const double ui = us[l][i];
      for (int j = 0; j < n; ++j) r[j] -= ui * vs[l][j];
    }
    used_r[i] = 1;
    ++n_used_r;
    const int j = pivot(r, used_c);
    if (j < 0 || std::fabs(r[j]) <= ZERO_RTOL * amax) {
      // vanishing residual row: try another row
      if (n_used_r == m) break;
      const int nxt = us.empty() ? -1 : pivot(us.back(), used_r);
      i = nxt >= 0 ? nxt : first_unused();
      continue;
    }
    std::vector<double> v((size_t)n);
    const double piv = r[j];
    for (int q = 0; q < n; ++q) v[q] = r[q] / piv;
    std::vector<double> a_col((size_t)m);
    col(j, a_col.data());
    for (double x : a_col) amax = std::max(amax, std::fabs(x));
    std::vector<double> u = a_col;
    for (size_t l = 0; l < us.size(); ++l) {
      const double vj = vs[l][j];
      for (int q = 0; q < m; ++q) u[q] -= vj * us[l][q];
    }
    used_c[j] = 1;
    double cross = 0.0;
    for (size_t l = 0; l < us.size(); ++l) cross += dot(us[l], u) * dot(vs[l], v);
    const double uu = dot(u, u), vv = dot(v, v);
    const double norm2_new = norm2 + 2.0 * cross + uu * vv;
    if (!us.empty() && std::sqrt(uu * vv) <= tol * std::sqrt(std::max(norm2_new, 0.0))) break;
    norm2 = norm2_new;
    out.rows.push_back(i);
    out.cols.push_back(j);
    out.raw_rows.push_back(std::move(a_row));
    out.raw_cols.push_back(std::move(a_col));
    us.push_back(std::move(u));
    vs.push_back(std::move(v));
    if (n_used_r == m) break;
    i = pivot(us.back(), used_r);
    if (i < 0) i = first_unused();
  }
  return out;
}

// X = C A^-1 for C (mr x r) and A (r x r), column-major: LU of A^T with partial pivoting, then
// A^T X^T = C^T solved for every row of C.
std::vector<double> right_solve(const std::vector<double>& C, int64_t mr, const std::vector<double>& A, int r) {
  std::vector<double> L((size_t)r * r);   // A^T, column-major
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) L[(size_t)i + (size_t)r * j] = A[(size_t)j + (size_t)r * i];
  std::vector<int> perm(r);
  for (int i = 0; i < r; ++i) perm[i] = i;
  for (int k = 0; k < r; ++k) {
    int p = k;
    double best = std::fabs(L[(size_t)k + (size_t)r * k]);
    for (int i = k + 1; i < r; ++i) {
      const double v = std::fabs(L[(size_t)i + (size_t)r * k]);
      if (v > best) { best = v; p = i; }
    }
    if (best == 0.0) fail(PH_EUNSUPPORTED, "TT-cross: singular pivot submatrix");
    if (p != k) {
      for (int j = 0; j < r; ++j) std::swap(L[(size_t)k + (size_t)r * j], L[(size_t)p + (size_t)r * j]);
      std::swap(perm[k], perm[p]);
    }
    const double d = L[(size_t)k + (size_t)r * k];
    for (int i = k + 1; i < r; ++i) {
      const double f = L[(size_t)i + (size_t)r * k] / d;
      L[(size_t)i + (size_t)r * k] = f;
      for (int j = k + 1; j < r; ++j) L[(size_t)i + (size_t)r * j] -= f * L[(size_t)k + (size_t)r * j];
    }
  }
  std::vector<double> X((size_t)mr * r), b((size_t)r);
  for (int64_t row = 0; row < mr; ++row) {
    for (int i = 0; i < r; ++i) b[i] = C[(size_t)row + (size_t)mr * perm[i]];
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < i; ++j) b[i] -= L[(size_t)i + (size_t)r * j] * b[j];
    for (int i = r - 1; i >= 0; --i) {
      for (int j = i + 1; j < r; ++j) b[i] -= L[(size_t)i + (size_t)r * j] * b[j];
      b[i] /= L[(size_t)i + (size_t)r * i];
    }
    for (int i = 0; i < r; ++i) X[(size_t)row + (size_t)mr * i] = b[i];
  }
  return X;
}

// index sets: multi-indices stored row-major (count x width)
struct IndexSet {
  int width = 0;
  std::vector<int32_t> v;
  int count() const { return width == 0 ? (int)(v.empty() ? 1 : v.size()) : (int)(v.size() / width); }
};

struct Cross {
  Tensor& X;
  std::vector<int> dims, start;
  std::vector<IndexSet> left, right;   // left[0..N-1], right[0..N]
  int N;
  explicit Cross(Tensor& x) : X(x), dims(x.dims), N(x.N()) {
    for (int m : dims) start.push_back(m / 2);
    left.resize(N);
    right.resize(N + 1);
    for (int k = 0; k < N; ++k) {
      left[k].width = k;
      left[k].v.assign(start.begin(), start.begin() + k);
    }
    for (int k = 0; k <= N; ++k) {
      right[k].width = N - k;
      right[k].v.assign(start.begin() + k, start.end());
    }
  }
  static int cnt(const IndexSet& s) { return s.width == 0 ? 1 : (int)(s.v.size() / s.width); }

  // ACA of supercore k; updates left[k+1], right[k+1]; false for a zero supercore
  bool supercore(int k, Aca* keep) {
    const IndexSet& Il = left[k];
    const IndexSet& Jr = right[k + 2];
    const int a = cnt(Il), b = cnt(Jr), mk = dims[k], mk1 = dims[k + 1];
    const int m = a * mk, n = mk1 * b;
    std::vector<int32_t> idx;
    auto row = [&](int rho, double* out) {
      const int al = rho % a, i = rho / a;
      idx.assign((size_t)n * N, 0);
      for (int c = 0; c < n; ++c) {
        int32_t* p = idx.data() + (size_t)c * N;
        for (int q = 0; q < k; ++q) p[q] = Il.v[(size_t)al * k + q];
        p[k] = i;
        p[k + 1] = c % mk1;
        const int be = c / mk1;
        for (int q = 0; q < N - k - 2; ++q) p[k + 2 + q] = Jr.v[(size_t)be * (N - k - 2) + q];
      }
      X.get(idx, out);
    };
    auto col = [&](int c, double* out) {
      const int i1 = c % mk1, be = c / mk1;
      idx.assign((size_t)m * N, 0);
      for (int rho = 0; rho < m; ++rho) {
        int32_t* p = idx.data() + (size_t)rho * N;
        const int al = rho % a;
        for (int q = 0; q < k; ++q) p[q] = Il.v[(size_t)al * k + q];
        p[k] = rho / a;
        p[k + 1] = i1;
        for (int q = 0; q < N - k - 2; ++q) p[k + 2 + q] = Jr.v[(size_t)be * (N - k - 2) + q];
      }
      X.get(idx, out);
    };
    Aca res = aca(row, col, m, n, tol_, a * start[k]);
    if (res.rows.empty()) return false;
    IndexSet nl, nr;
    nl.width = k + 1;
    nr.width = N - k - 1;
    for (int rho : res.rows) {
      const int al = rho % a;
      for (int q = 0; q < k; ++q) nl.v.push_back(Il.v[(size_t)al * k + q]);
      nl.v.push_back(rho / a);
    }
    for (int c : res.cols) {
      nr.v.push_back(c % mk1);
      const int be = c / mk1;
      for (int q = 0; q < N - k - 2; ++q) nr.v.push_back(Jr.v[(size_t)be * (N - k - 2) + q]);
    }
    left[k + 1] = std::move(nl);
    right[k + 1] = std::move(nr);
    if (keep) *keep = std::move(res);
    return true;
  }
  double tol_ = 0;
};

// value of the TT at one multi-index (product of the core slices)
double tt_entry(const TensorTrain& t, const int32_t* ix) {
  std::vector<double> v(1, 1.0), w;
  for (size_t k = 0; k < t.cores.size(); ++k) {
    const int r0 = t.ranks[k], m = t.dims[k], r1 = t.ranks[k + 1];
    const double* G = t.cores[k].data();
    w.assign((size_t)r1, 0.0);
    for (int b = 0; b < r1; ++b) {
      double s = 0;
      for (int a = 0; a < r0; ++a) s += v[a] * G[(size_t)a + (size_t)r0 * (ix[k] + (size_t)m * b)];
      w[b] = s;
    }
    v.swap(w);
  }
  return v[0];
}

TensorTrain zero_tt(const std::vector<int>& dims) {
  TensorTrain t;
  t.dims = dims;
  t.ranks.assign(dims.size() + 1, 1);
  for (int m : dims) t.cores.emplace_back((size_t)m, 0.0);
  return t;
}

void qr_reduced(const std::vector<double>& A, int64_t m, int k, std::vector<double>& Q, std::vector<double>& R,
                int& q);

TensorTrain tt_cross(Tensor& X, double tol, double check_tol) {
  const int N = X.N();
  const std::vector<int>& dims = X.dims;
  TensorTrain out;
  out.dims = dims;
  if (N == 1) {
    out.ranks = {1, 1};
    out.cores.emplace_back((size_t)dims[0]);
    std::vector<int32_t> idx(dims[0]);
    for (int i = 0; i < dims[0]; ++i) idx[i] = i;
    X.get(idx, out.cores[0].data());
    return out;
  }
  Cross cr(X);
  cr.tol_ = tol;
  std::vector<Aca> last((size_t)N - 1);
  auto assemble = [&]() {
    TensorTrain t;
    t.dims = dims;
    t.ranks.assign(N + 1, 1);
    int rl = 1;
    for (int k = 0; k < N - 1; ++k) {
      const Aca& a = last[k];
      const int r = (int)a.rows.size();
      const int64_t mr = (int64_t)rl * dims[k];
      std::vector<double> C((size_t)mr * r), A((size_t)r * r);
      for (int l = 0; l < r; ++l)
        for (int64_t q = 0; q < mr; ++q) C[(size_t)q + (size_t)mr * l] = a.raw_cols[l][q];
      // C A^-1 with A = C(pivot rows) is formed as Q Q(pivot rows)^-1 from C = Q R: the same
      // matrix, but Q(pivot rows) is far better conditioned than A
      std::vector<double> Q, Rq;
      int q;
      qr_reduced(C, mr, r, Q, Rq, q);
      for (int l = 0; l < r; ++l)
        for (int p = 0; p < r; ++p) A[(size_t)p + (size_t)r * l] = Q[(size_t)a.rows[p] + (size_t)mr * l];
      t.cores.push_back(right_solve(Q, mr, A, r));
      t.ranks[k + 1] = r;
      rl = r;
      if (k == N - 2) {
        // last core: the supercore's own rows at the pivot rows, A(I_{N-1} x m_{N-1})
        std::vector<double> G((size_t)r * dims[N - 1]);
        for (int p = 0; p < r; ++p)
          for (int i = 0; i < dims[N - 1]; ++i) G[(size_t)p + (size_t)r * i] = a.raw_rows[p][i];
        t.cores.push_back(std::move(G));
      }
    }
    return t;
  };
  int rounds = 0;
  TensorTrain cores;
  for (int it = 0; it < MAX_SWEEPS; ++it) {
    for (int k = 0; k < N - 1; ++k)
      if (!cr.supercore(k, &last[k])) return zero_tt(dims);
    cores = assemble();
    std::vector<int32_t> worst;
    if (it >= 1) {
      // sampled max-norm check (SplitMix64 stream of this enrichment round)
      uint64_t st = SAMPLE_SEED + (uint64_t)rounds;
      std::vector<int32_t> idx((size_t)N_SAMPLES * N);
      for (int s = 0; s < N_SAMPLES; ++s)
        for (int k = 0; k < N; ++k) idx[(size_t)s * N + k] = (int32_t)(splitmix64(st) % (uint64_t)dims[k]);
      std::vector<double> x((size_t)N_SAMPLES);
      X.get(idx, x.data());
      double emax = -1, scale = 0;
      int w = 0;
      for (int s = 0; s < N_SAMPLES; ++s) {
        const double e = std::fabs(x[s] - tt_entry(cores, idx.data() + (size_t)s * N));
        if (e > emax) { emax = e; w = s; }
        scale = std::max(scale, std::fabs(x[s]));
      }
      const double err = scale > 0 ? emax / scale : 0.0;
      if (err <= check_tol || rounds == MAX_ENRICH) break;
      ++rounds;
      worst.assign(idx.begin() + (size_t)w * N, idx.begin() + (size_t)(w + 1) * N);
    }
    for (int k = N - 2; k >= 0; --k)
      if (!cr.supercore(k, nullptr)) return zero_tt(dims);
    if (!worst.empty()) {
      // enrichment: the worst sample's suffixes join the right index sets
      for (int k = 1; k < N; ++k) {
        IndexSet& J = cr.right[k];
        const int wdt = N - k, c = Cross::cnt(J);
        bool found = false;
        for (int q = 0; q < c && !found; ++q)
          found = std::equal(worst.begin() + k, worst.end(), J.v.begin() + (size_t)q * wdt);
        if (!found) J.v.insert(J.v.end(), worst.begin() + k, worst.end());
      }
    }
  }
  cores.evals = X.evals;
  return cores;
}

// Reduced QR of the m x k matrix A (any shape): Q (m x q) and R (q x k), q = min(m, k).
void qr_reduced(const std::vector<double>& A, int64_t m, int k, std::vector<double>& Q, std::vector<double>& R,
                int& q) {
  q = (int)std::min<int64_t>(m, k);
  if (m >= k) {
    std::vector<double> W = A, tau((size_t)k);
    householder_qr(W.data(), m, k, tau.data());
    R.assign((size_t)q * k, 0.0);
    for (int c = 0; c < k; ++c)
      for (int i = 0; i <= c; ++i) R[(size_t)i + (size_t)q * c] = W[(size_t)i + (size_t)m * c];
    Q.assign((size_t)m * q, 0.0);
    for (int c = 0; c < q; ++c) Q[(size_t)c + (size_t)m * c] = 1.0;
    apply_q(W.data(), m, k, tau.data(), Q.data(), q);
  } else {
    // wide: QR of the leading m x m block, R = Q^T A
    std::vector<double> W(A.begin(), A.begin() + (size_t)m * m), tau((size_t)m);
    householder_qr(W.data(), m, (int)m, tau.data());
    Q.assign((size_t)m * m, 0.0);
    for (int c = 0; c < m; ++c) Q[(size_t)c + (size_t)m * c] = 1.0;
    apply_q(W.data(), m, (int)m, tau.data(), Q.data(), (int)m);
    R.assign((size_t)m * k, 0.0);
    for (int c = 0; c < k; ++c)
      for (int i = 0; i < m; ++i) {
        double s = 0;
        for (int64_t p = 0; p < m; ++p) s += Q[(size_t)p + (size_t)m * i] * A[(size_t)p + (size_t)m * c];
        R[(size_t)i + (size_t)m * c] = s;
      }
  }
}

void tt_round(TensorTrain& t, double tol) {
  const int N = (int)t.cores.size();
  if (N < 2) return;
  // right-to-left orthogonalisation: G_k^{1} = R^T Q^T, G_k <- Q^T, G_{k-1}^{2} <- G_{k-1}^{2} R^T
  for (int k = N - 1; k >= 1; --k) {
    const int r0 = t.ranks[k], m = t.dims[k], r1 = t.ranks[k + 1];
    const int64_t mm = (int64_t)m * r1;
    std::vector<double> Mt((size_t)mm * r0);   // (G^{1})^T: mm x r0
    const std::vector<double>& G = t.cores[k];
    for (int a = 0; a < r0; ++a)
      for (int64_t c = 0; c < mm; ++c) Mt[(size_t)c + (size_t)mm * a] = G[(size_t)a + (size_t)r0 * c];
    std::vector<double> Q, R;
    int q;
    qr_reduced(Mt, mm, r0, Q, R, q);
    std::vector<double> Gn((size_t)q * mm);
    for (int a = 0; a < q; ++a)
      for (int64_t c = 0; c < mm; ++c) Gn[(size_t)a + (size_t)q * c] = Q[(size_t)c + (size_t)mm * a];
    t.cores[k] = std::move(Gn);
    const int a0 = t.ranks[k - 1], m0 = t.dims[k - 1];
    const int64_t rows = (int64_t)a0 * m0;
    const std::vector<double>& P = t.cores[k - 1];   // rows x r0
    std::vector<double> Pn((size_t)rows * q, 0.0);
    for (int b = 0; b < q; ++b)
      for (int a = 0; a < r0; ++a) {
        const double w = R[(size_t)b + (size_t)q * a];   // (R^T)[a, b]
        if (w == 0.0) continue;
        for (int64_t i = 0; i < rows; ++i) Pn[(size_t)i + (size_t)rows * b] += P[(size_t)i + (size_t)rows * a] * w;
      }
    t.cores[k - 1] = std::move(Pn);
    t.ranks[k] = q;
  }
  double nrm2 = 0;
  for (double v : t.cores[0]) nrm2 += v * v;
  const double delta2 = (tol * tol / (N - 1)) * nrm2;
  for (int k = 0; k < N - 1; ++k) {
    const int a0 = t.ranks[k], m = t.dims[k], a1 = t.ranks[k + 1];
    const int64_t rows = (int64_t)a0 * m;
    const std::vector<double>& G = t.cores[k];   // rows x a1
    LeftSV sv = left_sv(G.data(), rows, a1);
    t.sweeps = std::max(t.sweeps, sv.sweeps);
    const int r = std::max(1, truncation_rank(sv.s.data(), sv.kk, delta2));
    // G <- U_r, next core <- (U_r^T G) G_{k+1}^{1}
    std::vector<double> SV((size_t)r * a1, 0.0);
    for (int c = 0; c < a1; ++c)
      for (int i = 0; i < r; ++i) {
        double s = 0;
        for (int64_t p = 0; p < rows; ++p) s += sv.U[(size_t)p + (size_t)rows * i] * G[(size_t)p + (size_t)rows * c];
        SV[(size_t)i + (size_t)r * c] = s;
      }
    t.cores[k].assign(sv.U.begin(), sv.U.begin() + (size_t)rows * r);
    const int m1 = t.dims[k + 1], b1 = t.ranks[k + 2];
    const int64_t cols = (int64_t)m1 * b1;
    const std::vector<double>& H = t.cores[k + 1];   // a1 x cols
    std::vector<double> Hn((size_t)r * cols, 0.0);
    for (int64_t c = 0; c < cols; ++c)
      for (int b = 0; b < a1; ++b) {
        const double h = H[(size_t)b + (size_t)a1 * c];
        if (h == 0.0) continue;
        for (int i = 0; i < r; ++i) Hn[(size_t)i + (size_t)r * c] += SV[(size_t)i + (size_t)r * b] * h;
      }
    t.cores[k + 1] = std::move(Hn);
    t.ranks[k + 1] = r;
  }
}

}  // namespace

TensorTrain tt_compress(EntryFn entry, const void* ctx, const std::vector<int>& dims, double tol) {
  Tensor X(entry, ctx, dims);
  TensorTrain t = tt_cross(X, CROSS_TOL_FACTOR * tol, CHECK_TOL_FACTOR * tol);
  const int64_t ev = X.evals;
  tt_round(t, tol);
  t.evals = ev;
  return t;
}

}  // namespace ph
