// Offline stage on the host, FP64 (Alg. "Offline Stage: Parametric H^2-matrix",
// arxiv 2511.03109).
//
//  * Chebyshev nodes of the first kind, ascending:
//      eta_i = (a+b)/2 - (b-a)/2 cos((2i-1) pi / (2p))      (Sec. 2.2)
//    Lagrange basis by the product formula of Sec. 2.2.
//  * Leaf cluster-basis factors [U_{s,k}]_{ij} = l_j^{(B_{s,k})}(x_{s,i,k}) (Sec. 3.2).
//  * Transfer factors (Sec. 3.4.1 with the orientation of the transfer lemma):
//      [E_{s',k}]_{j,i} = l_i^{(B_{s,k})}(eta_j^{(B_{s',k})}).
//    The Lagrange basis is invariant under affine maps of the interval, so the
//    factor only depends on whether s' is the lower or the upper half of s along
//    axis k; the two matrices are formed on [0, 1].
//  * Far tensors (App. PTTK review) M[i, k, j] = kappa(eta_i^{(B_s)}, eta_j^{(B_t)}; eta_k),
//    one per translation class (Sec. 5.2), built on the boxes of the class's first
//    far block; near tensors (Sec. 4.3) A_b[e, k] = kappa(x_{s,i}, x_{t,j}; eta_k),
//    e = i + j n_s.
//  * Compression: truncated HOSVD (Tucker) over the grouped modes; per mode the
//    smallest rank r with sum_{j>r} s_j^2 <= (tol^2 / N) ||M||_F^2 (N = number of
//    modes), giving ||M - M^||_F <= tol ||M||_F.  The cut never splits a cluster of
//    equal singular values (s_r - s_{r+1} <= 1e-4 s_r): the kept subspace is then
//    unique, so any backward-stable SVD keeps the same one (symmetric geometry gives
//    exactly degenerate pairs).  Singular values and vectors of
//    each unfolding come from a Householder QR of the tall orientation followed by a
//    one-sided (Hestenes) Jacobi SVD of the small triangular factor.
//  * Symmetry: kappa(x, y) = kappa(y, x), so A_{ts} is A_{st} with the pair index
//    transposed and M_{(l,-o)}[i,k,j] = M_{(l,o)}[j,k,i]; only near blocks with
//    s <= t and classes with offset >= 0 (lexicographic) are compressed.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

#include "kernel_fn.hpp"
#include "ph_host.hpp"

namespace ph {

namespace {

void cheb_nodes(double a, double b, int p, double* out) {
  for (int i = 1; i <= p; ++i)
    out[i - 1] = (a + b) / 2.0 - (b - a) / 2.0 * std::cos((2.0 * i - 1.0) * M_PI / (2.0 * p));
}

// l_k(x) for k = 0..p-1 by the product formula
void lagrange_all(const double* nodes, int p, double x, double* out) {
  for (int k = 0; k < p; ++k) {
    double v = 1.0;
    for (int i = 0; i < p; ++i)
      if (i != k) v *= (x - nodes[i]) / (nodes[k] - nodes[i]);
    out[k] = v;
  }
}

}  // namespace

// ---- dense linear algebra (column-major) ---------------------------------------------

// Householder QR of the m x k matrix A (m >= k, leading dimension m), in place.
// On return the upper triangle of A holds R, the columns below the diagonal hold
// the Householder vectors v_j (v_j[j] = 1 implied), tau[j] their scalars.
void householder_qr(double* A, int64_t m, int k, double* tau) {
  for (int j = 0; j < k; ++j) {
    double* a = A + (int64_t)j * m;
    double norm2 = 0;
    for (int64_t i = j + 1; i < m; ++i) norm2 += a[i] * a[i];
    double alpha = a[j];
    if (norm2 == 0.0) {
      tau[j] = 0.0;
      continue;
    }
    double beta = -std::copysign(std::sqrt(alpha * alpha + norm2), alpha);
    double scale = 1.0 / (alpha - beta);
    for (int64_t i = j + 1; i < m; ++i) a[i] *= scale;
    tau[j] = (beta - alpha) / beta;
    a[j] = beta;
    // apply H_j = I - tau v v^T to the remaining columns
    for (int c = j + 1; c < k; ++c) {
      double* b = A + (int64_t)c * m;
      double dot = b[j];
      for (int64_t i = j + 1; i < m; ++i) dot += a[i] * b[i];
      dot *= tau[j];
      b[j] -= dot;
      for (int64_t i = j + 1; i < m; ++i) b[i] -= dot * a[i];
    }
  }
}

// Y (m x r, leading dimension m) <- Q Y, with Q = H_0 H_1 ... H_{k-1} from householder_qr.
void apply_q(const double* A, int64_t m, int k, const double* tau, double* Y, int r) {
  for (int j = k - 1; j >= 0; --j) {
    if (tau[j] == 0.0) continue;
    const double* a = A + (int64_t)j * m;
    for (int c = 0; c < r; ++c) {
      double* y = Y + (int64_t)c * m;
      double dot = y[j];
      for (int64_t i = j + 1; i < m; ++i) dot += a[i] * y[i];
      dot *= tau[j];
      y[j] -= dot;
      for (int64_t i = j + 1; i < m; ++i) y[i] -= dot * a[i];
    }
  }
}

constexpr int JACOBI_MAX_SWEEPS = 80;

// One-sided Jacobi SVD of the k x k matrix W (overwritten): W V = U S.
// Outputs s (descending), U and V (k x k column-major).  Returns the number of sweeps
// that rotated; JACOBI_MAX_SWEEPS + 1 when the last allowed sweep still rotated (not
// converged).
int jacobi_svd(double* W, int k, double* s, double* U, double* V) {
  std::vector<double> Vw((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) Vw[(size_t)i * k + i] = 1.0;
  // rotation threshold: the rounding level of a k-term inner product (sqrt(k) eps); with eps
  // alone a pair whose cosine sits at its own rounding noise can keep rotating
  const double tol = std::sqrt((double)k) * 2.220446049250313e-16;
  int sweeps = 0;
  std::vector<double> cn(k), tmp((size_t)k * k);
  std::vector<int> ord(k);
  for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
    // de Rijk's ordering: columns by decreasing norm at the start of every sweep, so that
    // the large singular directions are separated first (graded matrices, whose small
    // columns are otherwise rotated against noise for many sweeps)
    for (int j = 0; j < k; ++j) {
      double a = 0;
      for (int i = 0; i < k; ++i) a += W[(size_t)j * k + i] * W[(size_t)j * k + i];
      cn[j] = a;
    }
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cn[a] > cn[b]; });
    bool perm = false;
    for (int j = 0; j < k; ++j) perm |= ord[j] != j;
    if (perm) {
      for (double* M : {W, Vw.data()}) {
        for (int j = 0; j < k; ++j)
          std::copy(M + (size_t)ord[j] * k, M + (size_t)ord[j] * k + k, tmp.data() + (size_t)j * k);
        std::copy(tmp.begin(), tmp.end(), M);
      }
    }
    // columns below eps times the largest are at the rounding level of the factorisation
    // (their squared norms can underflow): they are not rotated
    const double cmax = *std::max_element(cn.begin(), cn.end());
    const double small = 4.930380657631324e-32 * cmax;   // eps^2 cmax
    bool rotated = false;
    for (int p = 0; p < k - 1; ++p) {
      for (int q = p + 1; q < k; ++q) {
        double* wp = W + (size_t)p * k;
        double* wq = W + (size_t)q * k;
        double al = 0, be = 0, ga = 0;
        for (int i = 0; i < k; ++i) {
          al += wp[i] * wp[i];
          be += wq[i] * wq[i];
          ga += wp[i] * wq[i];
        }
        if (al <= small || be <= small) continue;
        if (std::fabs(ga) <= tol * std::sqrt(al) * std::sqrt(be)) continue;
        rotated = true;
        double zeta = (be - al) / (2.0 * ga);
        double t = std::copysign(1.0, zeta) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t);
        double sn = c * t;
        for (int i = 0; i < k; ++i) {
          double x = wp[i], y = wq[i];
          wp[i] = c * x - sn * y;
          wq[i] = sn * x + c * y;
        }
        double* vp = Vw.data() + (size_t)p * k;
        double* vq = Vw.data() + (size_t)q * k;
        for (int i = 0; i < k; ++i) {
          double x = vp[i], y = vq[i];
          vp[i] = c * x - sn * y;
          vq[i] = sn * x + c * y;
        }
      }
    }
    if (!rotated) break;
    sweeps = sweep + 1 == JACOBI_MAX_SWEEPS ? JACOBI_MAX_SWEEPS + 1 : sweep + 1;
  }
  std::vector<double> nrm(k);
  for (int j = 0; j < k; ++j) {
    double a = 0;
    for (int i = 0; i < k; ++i) a += W[(size_t)j * k + i] * W[(size_t)j * k + i];
    nrm[j] = std::sqrt(a);
  }
  std::vector<int> order(k);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
  for (int jj = 0; jj < k; ++jj) {
    int j = order[jj];
    s[jj] = nrm[j];
    for (int i = 0; i < k; ++i) {
      U[(size_t)jj * k + i] = nrm[j] > 0 ? W[(size_t)j * k + i] / nrm[j] : (i == jj ? 1.0 : 0.0);
      V[(size_t)jj * k + i] = Vw[(size_t)j * k + i];
    }
  }
  return sweeps;
}

// Smallest r >= 0 with sum_{j >= r} s_j^2 <= thr (tail summed from the smallest value up),
// then moved past every following s_r with s_{r-1} - s_r <= CLUSTER_GAP s_{r-1}: a cluster of
// equal singular values is kept or dropped as a whole.
constexpr double CLUSTER_GAP = 1e-4;
int truncation_rank(const double* s, int k, double thr) {
  std::vector<double> tail(k + 1, 0.0);
  for (int j = k - 1; j >= 0; --j) tail[j] = tail[j + 1] + s[j] * s[j];
  int r = k;
  for (int q = 0; q <= k; ++q)
    if (tail[q] <= thr) {
      r = q;
      break;
    }
  while (r > 0 && r < k && s[r - 1] - s[r] <= CLUSTER_GAP * s[r - 1]) ++r;
  return r;
}

// Left singular vectors (first r columns) and singular values of the m x q matrix X
// given by an accessor that fills it column-major.  Chooses the tall orientation.

// X column-major m x q (leading dimension m).
LeftSV left_sv(const double* X, int64_t m, int64_t q) {
  LeftSV out;
  out.m = m;
  if (m >= q) {
    // tall: X = Q R, R = U_R S V_R^T  ->  left sv = Q U_R
    int k = (int)q;
    std::vector<double> A(X, X + m * q), tau(k);
    householder_qr(A.data(), m, k, tau.data());
    std::vector<double> R((size_t)k * k, 0.0), UR((size_t)k * k), VR((size_t)k * k);
    for (int c = 0; c < k; ++c)
      for (int i = 0; i <= c; ++i) R[(size_t)c * k + i] = A[(size_t)c * m + i];
    out.s.resize(k);
    out.sweeps = jacobi_svd(R.data(), k, out.s.data(), UR.data(), VR.data());
    out.U.assign((size_t)m * k, 0.0);
    for (int c = 0; c < k; ++c)
      for (int i = 0; i < k; ++i) out.U[(size_t)c * m + i] = UR[(size_t)c * k + i];
    apply_q(A.data(), m, k, tau.data(), out.U.data(), k);
    out.kk = k;
  } else {
    // wide: X^T = Q R, R = U_R S V_R^T  ->  X = V_R S (Q U_R)^T, left sv = V_R
    int k = (int)m;
    std::vector<double> A((size_t)q * m), tau(k);
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < q; ++j) A[(size_t)i * q + j] = X[(size_t)j * m + i];
    householder_qr(A.data(), q, k, tau.data());
    std::vector<double> R((size_t)k * k, 0.0), UR((size_t)k * k), VR((size_t)k * k);
    for (int c = 0; c < k; ++c)
      for (int i = 0; i <= c; ++i) R[(size_t)c * k + i] = A[(size_t)c * q + i];
    out.s.resize(k);
    out.sweeps = jacobi_svd(R.data(), k, out.s.data(), UR.data(), VR.data());
    out.U = VR;
    out.kk = k;
  }
  return out;
}

namespace {

// Mode-m unfolding of a column-major tensor with dims n[0..N-1] (first index fastest),
// written column-major as n[m] x (prod of the others).
std::vector<double> unfold(const std::vector<double>& T, const std::vector<int64_t>& n, int m) {
  int64_t left = 1, right = 1;
  for (int i = 0; i < m; ++i) left *= n[i];
  for (size_t i = m + 1; i < n.size(); ++i) right *= n[i];
  const int64_t mid = n[m];
  std::vector<double> X((size_t)mid * left * right);
  for (int64_t rr = 0; rr < right; ++rr)
    for (int64_t i = 0; i < mid; ++i)
      for (int64_t l = 0; l < left; ++l)
        X[(size_t)i + mid * (l + left * rr)] = T[(size_t)l + left * (i + mid * rr)];
  return X;
}

// Y = T x_m A^T, A (n[m] x r column-major): Y[.., a, ..] = sum_i T[.., i, ..] A[i, a]
std::vector<double> mode_contract(const std::vector<double>& T, std::vector<int64_t>& n, int m,
                                  const double* A, int r) {
  int64_t left = 1, right = 1;
  for (int i = 0; i < m; ++i) left *= n[i];
  for (size_t i = m + 1; i < n.size(); ++i) right *= n[i];
  const int64_t mid = n[m];
  std::vector<double> Y((size_t)left * r * right, 0.0);
  for (int64_t rr = 0; rr < right; ++rr)
    for (int a = 0; a < r; ++a)
      for (int64_t i = 0; i < mid; ++i) {
        const double w = A[(size_t)a * mid + i];
        const double* src = T.data() + (size_t)left * (i + mid * rr);
        double* dst = Y.data() + (size_t)left * (a + r * rr);
        for (int64_t l = 0; l < left; ++l) dst[l] += w * src[l];
      }
  n[m] = r;
  return Y;
}

struct Tucker {
  std::vector<std::vector<double>> factors;  // column-major n[m] x r[m]
  std::vector<int> ranks;
  std::vector<double> core;                  // column-major r[0] x r[1] x ...
  int sweeps = 0;                            // most Jacobi sweeps of any mode
};

// Truncated HOSVD of the column-major tensor T with dims n.
Tucker thosvd(const std::vector<double>& T, const std::vector<int64_t>& n, double tol) {
  const int N = (int)n.size();
  double normsq = 0;
  for (double v : T) normsq += v * v;
  const double thr = (tol * tol / N) * normsq;
  Tucker out;
  for (int m = 0; m < N; ++m) {
    int64_t rest = 1;
    for (int i = 0; i < N; ++i)
      if (i != m) rest *= n[i];
    LeftSV sv;
    if (m == 0) {
      sv = left_sv(T.data(), n[0], rest);
    } else {
      std::vector<double> X = unfold(T, n, m);
      sv = left_sv(X.data(), n[m], rest);
    }
    int r = normsq == 0.0 ? 0 : truncation_rank(sv.s.data(), sv.kk, thr);
    out.sweeps = std::max(out.sweeps, sv.sweeps);
    out.ranks.push_back(r);
    out.factors.emplace_back(sv.U.begin(), sv.U.begin() + (size_t)n[m] * r);
  }
  std::vector<int64_t> dims = n;
  std::vector<double> core = T;
  for (int m = 0; m < N; ++m) core = mode_contract(core, dims, m, out.factors[m].data(), out.ranks[m]);
  out.core = std::move(core);
  return out;
}

// TT of a far tensor (modes i_1..i_d, k_1..k_dth, j_1..j_d, each index little-endian) in the
// form of the online stage (App. PTTK review): L = G_0 .. G_{d-1} contracted (P x r_d), R from
// G_{d+dth} .. G_{N-1} (P x r_{d+dth}), identity parameter factors and the parameter cores as
// core[a, k_1, (k_2,) b], so that H(theta) = core contracted with v_1 (and v_2).
Tucker tt_far_tucker(const TensorTrain& t, int d, int dth) {
  const int N = (int)t.cores.size();
  Tucker out;
  out.sweeps = t.sweeps;
  // L: rows (i_1 .. i_k) little-endian
  std::vector<double> L = t.cores[0];
  int64_t rows = t.dims[0];
  int rl = t.ranks[1];
  for (int k = 1; k < d; ++k) {
    const int m = t.dims[k], r1 = t.ranks[k + 1];
    const std::vector<double>& G = t.cores[k];
    std::vector<double> Ln((size_t)rows * m * r1, 0.0);
    for (int b = 0; b < r1; ++b)
      for (int i = 0; i < m; ++i)
        for (int a = 0; a < rl; ++a) {
          const double w = G[(size_t)a + (size_t)rl * (i + (size_t)m * b)];
          const double* src = L.data() + (size_t)rows * a;
          double* dst = Ln.data() + (size_t)rows * (i + (size_t)m * b);
          for (int64_t q = 0; q < rows; ++q) dst[q] += src[q] * w;
        }
    L.swap(Ln);
    rows *= m;
    rl = r1;
  }
  // R: Y (r x (j_k .. j_d)) built from the last core backwards, then transposed
  int rr = t.ranks[N - 1];
  int64_t cols = t.dims[N - 1];
  std::vector<double> Y = t.cores[N - 1];   // rr x m
  for (int k = N - 2; k >= d + dth; --k) {
    const int r0 = t.ranks[k], m = t.dims[k];
    const std::vector<double>& G = t.cores[k];   // r0 x m x rr
    std::vector<double> Yn((size_t)r0 * m * cols, 0.0);   // [a + r0 (j + m rest)]
    for (int64_t c = 0; c < cols; ++c)
      for (int q = 0; q < rr; ++q) {
        const double y = Y[(size_t)q + (size_t)rr * c];
        if (y == 0.0) continue;
        for (int j = 0; j < m; ++j)
          for (int a = 0; a < r0; ++a)
            Yn[(size_t)a + (size_t)r0 * (j + (size_t)m * c)] += G[(size_t)a + (size_t)r0 * (j + (size_t)m * q)] * y;
      }
    Y.swap(Yn);
    cols *= m;
    rr = r0;
  }
  std::vector<double> R((size_t)cols * rr);
  for (int b = 0; b < rr; ++b)
    for (int64_t j = 0; j < cols; ++j) R[(size_t)j + (size_t)cols * b] = Y[(size_t)b + (size_t)rr * j];
  const int pt = t.dims[d];
  std::vector<double> core;
  if (dth == 1) {
    core = t.cores[d];
  } else {
    const int rm = t.ranks[d + 1];
    const std::vector<double>& G1 = t.cores[d];       // rl x pt x rm
    const std::vector<double>& G2 = t.cores[d + 1];   // rm x pt x rr
    core.assign((size_t)rl * pt * pt * rr, 0.0);
    for (int b = 0; b < rr; ++b)
      for (int k2 = 0; k2 < pt; ++k2)
        for (int c = 0; c < rm; ++c) {
          const double g2 = G2[(size_t)c + (size_t)rm * (k2 + (size_t)pt * b)];
          for (int k1 = 0; k1 < pt; ++k1)
            for (int a = 0; a < rl; ++a)
              core[(size_t)a + (size_t)rl * (k1 + (size_t)pt * (k2 + (size_t)pt * b))] +=
                  G1[(size_t)a + (size_t)rl * (k1 + (size_t)pt * c)] * g2;
        }
  }
  std::vector<double> I((size_t)pt * pt, 0.0);
  for (int k = 0; k < pt; ++k) I[(size_t)k * pt + k] = 1.0;
  out.ranks.push_back(rl);
  out.factors.push_back(std::move(L));
  for (int k = 0; k < dth; ++k) {
    out.ranks.push_back(pt);
    out.factors.push_back(I);
  }
  out.ranks.push_back(rr);
  out.factors.push_back(std::move(R));
  out.core = std::move(core);
  return out;
}

// TT of a near tensor (modes e, k_1 (, k_2)) in the form of the online stage (Sec. 4.3):
// U_e = G_0 (N_e x r_1), identity parameter factors, core[a, k_1 (, k_2)] from the parameter cores.
Tucker tt_near_tucker(const TensorTrain& t, int dth) {
  Tucker out;
  out.sweeps = t.sweeps;
  const int r1 = t.ranks[1], pt = t.dims[1];
  std::vector<double> core;
  if (dth == 1) {
    core = t.cores[1];   // r1 x pt x 1
  } else {
    const int r2 = t.ranks[2];
    const std::vector<double>& G1 = t.cores[1];   // r1 x pt x r2
    const std::vector<double>& G2 = t.cores[2];   // r2 x pt x 1
    core.assign((size_t)r1 * pt * pt, 0.0);
    for (int k2 = 0; k2 < pt; ++k2)
      for (int c = 0; c < r2; ++c) {
        const double g2 = G2[(size_t)c + (size_t)r2 * k2];
        for (int k1 = 0; k1 < pt; ++k1)
          for (int a = 0; a < r1; ++a)
            core[(size_t)a + (size_t)r1 * (k1 + (size_t)pt * k2)] += G1[(size_t)a + (size_t)r1 * (k1 + (size_t)pt * c)] * g2;
      }
  }
  std::vector<double> I((size_t)pt * pt, 0.0);
  for (int k = 0; k < pt; ++k) I[(size_t)k * pt + k] = 1.0;
  out.ranks.push_back(r1);
  out.factors.push_back(t.cores[0]);
  for (int k = 0; k < dth; ++k) {
    out.ranks.push_back(pt);
    out.factors.push_back(I);
  }
  out.core = std::move(core);
  return out;
}

// Entry accessors for the cross: kernel values at the Chebyshev nodes of a class (far) or at
// the point pairs of a near block, evaluated on demand
struct FarCtx {
  ph_kernel kernel;
  int d, dth, ps, P;
  const double* ns;     // P x d target nodes
  const double* nt;     // P x d source nodes
  const double* grid;   // parameter nodes, 2 per grid point, k_1 fastest
  int pt;
};
void far_entries(const void* c, const int32_t* idx, int64_t count, double* out) {
  const FarCtx& f = *static_cast<const FarCtx*>(c);
  const int N = 2 * f.d + f.dth;
  for (int64_t s = 0; s < count; ++s) {
    const int32_t* ix = idx + s * N;
    int i = 0, j = 0, st = 1;
    for (int k = 0; k < f.d; ++k) {
      i += st * ix[k];
      j += st * ix[f.d + f.dth + k];
      st *= f.ps;
    }
    const int kk = ix[f.d] + (f.dth == 2 ? f.pt * ix[f.d + 1] : 0);
    out[s] = kernel_value(f.kernel, f.d, &f.ns[(size_t)i * f.d], &f.nt[(size_t)j * f.d], &f.grid[2 * kk]);
  }
}
struct NearCtx {
  ph_kernel kernel;
  int d, dth, pt;
  int32_t ns;
  const double* xs;     // points of the target cluster (tree order), ns x d
  const double* xt;     // points of the source cluster
  const double* grid;
};
void near_entries(const void* c, const int32_t* idx, int64_t count, double* out) {
  const NearCtx& f = *static_cast<const NearCtx*>(c);
  const int N = 1 + f.dth;
  for (int64_t s = 0; s < count; ++s) {
    const int32_t* ix = idx + s * N;
    const int32_t i = ix[0] % f.ns, j = ix[0] / f.ns;
    const int kk = ix[1] + (f.dth == 2 ? f.pt * ix[2] : 0);
    out[s] = kernel_value(f.kernel, f.d, &f.xs[(size_t)i * f.d], &f.xt[(size_t)j * f.d], &f.grid[2 * kk]);
  }
}

// A failure inside an OpenMP loop is recorded (the first one) and raised after the loop: an
// exception must not leave a parallel region.
struct LoopError {
  std::mutex mu;
  int code = 0;
  std::string msg;
  void record(int c, const std::string& m) {
    std::lock_guard<std::mutex> g(mu);
    if (code == 0) {
      code = c;
      msg = m;
    }
  }
  template <typename F>
  void guard(F&& f) {
    try {
      f();
    } catch (const Failure& e) {
      record(e.code, e.what());
    } catch (const std::bad_alloc&) {
      record(PH_ENOMEM, "ph_offline_compress: out of host memory");
    } catch (const std::exception& e) {
      record(PH_EINVAL, e.what());   // as the C ABI maps other exceptions
    }
  }
  void raise() {
    if (code != 0) fail(code, msg);
  }
};

}  // namespace

int kernel_dtheta(ph_kernel k, int d) {
  switch (k) {
    case PH_KERNEL_GAUSSIAN:
    case PH_KERNEL_MATERN32:
    case PH_KERNEL_MATERN12:
    case PH_KERNEL_POLY_TEST:
      return 1;
    case PH_KERNEL_ANISO_GAUSSIAN:
      return d;
    case PH_KERNEL_POLY2_TEST:
    case PH_KERNEL_MATERN:
      return 2;
  }
  return -1;
}

double kernel_value(ph_kernel k, int d, const double* x, const double* y, const double* th) {
  if (k == PH_KERNEL_MATERN) return kernel_eval(k, d, x, y, th, bessel_order(th[1]));
  return kernel_eval(k, d, x, y, th, BesselOrder{});
}

std::shared_ptr<HostModel> offline_host(const TreeData& t, const ph_offline_opts& o, bool gpu, Compress comp) {
  const bool use_tt = comp == Compress::TT;
  if (use_tt && gpu) fail(PH_EUNSUPPORTED, "ph_offline_compress: TT-cross runs on the host only");
  const int d = t.d;
  if (o.p_s < 1 || o.p_s > 16 || o.p_theta < 1 || o.p_theta > 16)
    fail(PH_EINVAL, "ph_offline_compress: p_s and p_theta must be in 1..16");
  if (!(o.tol >= 0.0)) fail(PH_EINVAL, "ph_offline_compress: tol must be >= 0");
  const int dth = kernel_dtheta(o.kernel, d);
  if (dth < 0) fail(PH_EUNSUPPORTED, "ph_offline_compress: unknown kernel");
  if (o.kernel == PH_KERNEL_ANISO_GAUSSIAN && d > 2)
    fail(PH_EUNSUPPORTED, "ph_offline_compress: anisotropic Gaussian supports d <= 2");
  if (o.d_theta != dth) fail(PH_EUNSUPPORTED, "ph_offline_compress: d_theta does not match the kernel");
  for (int k = 0; k < dth; ++k)
    if (!(o.theta_lo[k] < o.theta_hi[k])) fail(PH_EINVAL, "ph_offline_compress: need theta_lo < theta_hi");
  if (o.kernel == PH_KERNEL_MATERN && !(o.theta_lo[0] > 0 && o.theta_lo[1] > 0))
    fail(PH_EINVAL, "ph_offline_compress: the Matern kernel needs lambda > 0 and nu > 0 on all of Theta");
  int P = 1;
  for (int k = 0; k < d; ++k) P *= o.p_s;
  if (P > 128) fail(PH_EUNSUPPORTED, "ph_offline_compress: p_s^d must be <= 128");

  auto m = std::make_shared<HostModel>();
  m->d = d; m->p_s = o.p_s; m->P = P; m->p_theta = o.p_theta; m->d_theta = dth;
  m->kernel = o.kernel; m->tol = o.tol;
  for (int k = 0; k < dth; ++k) { m->th_lo[k] = o.theta_lo[k]; m->th_hi[k] = o.theta_hi[k]; }
  const int ps = o.p_s, pt = o.p_theta;
  int nthreads = o.num_threads > 0 ? o.num_threads : omp_get_max_threads();

  // parameter grid: q = p^dth nodes, little-endian (k_1 fastest)
  const int q = dth == 1 ? pt : pt * pt;
  std::vector<double> thn(2 * 16), grid((size_t)q * 2, 0.0);
  for (int k = 0; k < dth; ++k) cheb_nodes(o.theta_lo[k], o.theta_hi[k], pt, thn.data() + 16 * k);
  for (int kk = 0; kk < q; ++kk) {
    grid[2 * kk] = thn[kk % pt];
    if (dth == 2) grid[2 * kk + 1] = thn[16 + kk / pt];
  }

  // leaf factors
  const int64_t n = t.n;
  m->U.assign((size_t)n * d * ps, 0.0);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
  for (int64_t li = 0; li < (int64_t)t.leaves.size(); ++li) {
    int32_t s = t.leaves[li];
    double nodes[16];
    for (int k = 0; k < d; ++k) {
      cheb_nodes(t.box_lo[s * d + k], t.box_hi[s * d + k], ps, nodes);
      for (int64_t i = t.begin[s]; i < t.end[s]; ++i)
        lagrange_all(nodes, ps, t.pts_t[i * d + k], m->U.data() + (i * d + k) * ps);
    }
  }
  // transfer factors on the reference interval
  {
    double par[16], ch[16], row[16];
    cheb_nodes(0.0, 1.0, ps, par);
    m->E.assign((size_t)2 * ps * ps, 0.0);
    for (int h = 0; h < 2; ++h) {
      cheb_nodes(h ? 0.5 : 0.0, h ? 1.0 : 0.5, ps, ch);
      for (int j = 0; j < ps; ++j) {
        lagrange_all(par, ps, ch[j], row);
        for (int i = 0; i < ps; ++i) m->E[((size_t)h * ps + j) * ps + i] = row[i];
      }
    }
  }

  // ---- far classes
  const int64_t ncls = t.n_classes();
  m->class_src.assign(ncls, -1);
  m->class_tr.assign(ncls, 0);
  std::vector<int32_t> canon;
  {
    std::map<std::vector<int32_t>, int32_t> bykey;
    for (int64_t c = 0; c < ncls; ++c) {
      std::vector<int32_t> kk{t.class_level[c]};
      for (int k = 0; k < d; ++k) kk.push_back(t.class_off[c * d + k]);
      bykey[kk] = (int32_t)c;
    }
    for (int64_t c = 0; c < ncls; ++c) {
      std::vector<int32_t> off(t.class_off.begin() + c * d, t.class_off.begin() + (c + 1) * d);
      std::vector<int32_t> neg(d);
      for (int k = 0; k < d; ++k) neg[k] = -off[k];
      if (off >= neg) {  // lexicographic, offset >= its negative
        ClassStored cs{};
        cs.cls = (int32_t)c;
        std::vector<int32_t> mk{t.class_level[c]};
        mk.insert(mk.end(), neg.begin(), neg.end());
        auto it = bykey.find(mk);
        cs.mirror = (it != bykey.end() && it->second != c) ? it->second : -1;
        m->class_src[c] = (int32_t)m->cstore.size();
        if (cs.mirror >= 0) {
          m->class_src[cs.mirror] = (int32_t)m->cstore.size();
          m->class_tr[cs.mirror] = 1;
        }
        m->cstore.push_back(cs);
      }
    }
  }
  const int64_t nfc = (int64_t)m->cstore.size();
  std::vector<Tucker> ftuck(nfc);
  int64_t evals_far = 0;
  LoopError lerr;   // failures of the TT compression inside the parallel loops
  // Chebyshev nodes of the two boxes of each stored class's first far block (P x d each)
  std::vector<double> cnodes((size_t)nfc * 2 * P * d);
  for (int64_t ci = 0; ci < nfc; ++ci) {
    const int32_t c = m->cstore[ci].cls;
    const int32_t b = t.class_first_block[c];
    const int32_t s = t.far[2 * b], u = t.far[2 * b + 1];
    double* ns = cnodes.data() + (size_t)ci * 2 * P * d;
    double* nt = ns + (size_t)P * d;
    for (int k = 0; k < d; ++k) {
      double bs[16], bt[16];
      cheb_nodes(t.box_lo[s * d + k], t.box_hi[s * d + k], ps, bs);
      cheb_nodes(t.box_lo[u * d + k], t.box_hi[u * d + k], ps, bt);
      int stride = 1;
      for (int kk = 0; kk < k; ++kk) stride *= ps;
      for (int i = 0; i < P; ++i) {
        ns[(size_t)i * d + k] = bs[(i / stride) % ps];
        nt[(size_t)i * d + k] = bt[(i / stride) % ps];
      }
    }
  }
  // kernel tensors on the GPU (kernel-tensor generation of the offline stage), else per class
  // on the host inside the compression loop
  std::unique_ptr<GpuTensorGen> gen;
  std::vector<double> Mall;
  if (gpu) {
    gen.reset(new GpuTensorGen(t, o.kernel, grid.data(), q));
    Mall.resize((size_t)nfc * P * q * P);
    gen->far(cnodes, (int)nfc, P, Mall.data());
  }
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) reduction(+ : evals_far)
  for (int64_t ci = 0; ci < nfc; ++ci) {
    const double* ns = cnodes.data() + (size_t)ci * 2 * P * d;
    const double* nt = ns + (size_t)P * d;
    if (use_tt) {
      FarCtx fc{o.kernel, d, dth, ps, P, ns, nt, grid.data(), pt};
      std::vector<int> tdims(d, ps);
      for (int k = 0; k < dth; ++k) tdims.push_back(pt);
      for (int k = 0; k < d; ++k) tdims.push_back(ps);
      lerr.guard([&] {
        TensorTrain tt = tt_compress(far_entries, &fc, tdims, o.tol);
        evals_far += tt.evals;
        ftuck[ci] = tt_far_tucker(tt, d, dth);
      });
      continue;
    }
    std::vector<double> M((size_t)P * q * P);
    if (gpu) {
      std::memcpy(M.data(), Mall.data() + (size_t)ci * P * q * P, M.size() * sizeof(double));
    } else {
      for (int j = 0; j < P; ++j)
        for (int kk = 0; kk < q; ++kk)
          for (int i = 0; i < P; ++i)
            M[(size_t)i + P * (kk + (size_t)q * j)] =
                kernel_value(o.kernel, d, &ns[(size_t)i * d], &nt[(size_t)j * d], &grid[2 * kk]);
    }
    evals_far += (int64_t)P * q * P;
    std::vector<int64_t> dims{P};
    if (dth == 1) dims.push_back(pt);
    else { dims.push_back(pt); dims.push_back(pt); }
    dims.push_back(P);
    ftuck[ci] = thosvd(M, dims, o.tol);
  }
  lerr.raise();
  for (const Tucker& tk : ftuck) m->svd_sweeps_max = std::max(m->svd_sweeps_max, tk.sweeps);
  for (int64_t ci = 0; ci < nfc; ++ci) {
    ClassStored& cs = m->cstore[ci];
    Tucker& tk = ftuck[ci];
    cs.rL = tk.ranks.front();
    cs.rR = tk.ranks.back();
    cs.r1 = tk.ranks[1];
    cs.r2 = dth == 2 ? tk.ranks[2] : 1;
    cs.L_off = (int64_t)m->ff_L.size();
    m->ff_L.insert(m->ff_L.end(), tk.factors.front().begin(), tk.factors.front().end());
    cs.R_off = (int64_t)m->ff_R.size();
    m->ff_R.insert(m->ff_R.end(), tk.factors.back().begin(), tk.factors.back().end());
    cs.th1_off = (int64_t)m->ff_theta.size();
    m->ff_theta.insert(m->ff_theta.end(), tk.factors[1].begin(), tk.factors[1].end());
    cs.th2_off = (int64_t)m->ff_theta.size();
    if (dth == 2) m->ff_theta.insert(m->ff_theta.end(), tk.factors[2].begin(), tk.factors[2].end());
    cs.core_off = (int64_t)m->ff_core.size();
    m->ff_core.insert(m->ff_core.end(), tk.core.begin(), tk.core.end());
  }
  // far-field panels Chat_q = L G_q R^T (the coupling is linear in the parametric weights,
  // so C(theta) = L H(theta) R^T = sum_q w_q(theta) Chat_q; the online stage then streams
  // these panels once for all parameter values)
  {
    int64_t tot = 0;
    for (int64_t ci = 0; ci < nfc; ++ci) {
      m->cstore[ci].chat_off = tot;
      tot += (int64_t)m->cstore[ci].r1 * m->cstore[ci].r2 * P * P;
    }
    m->ff_chat.assign((size_t)tot, 0.0);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t ci = 0; ci < nfc; ++ci) {
      const ClassStored& cs = m->cstore[ci];
      const Tucker& tk = ftuck[ci];
      const double* L = tk.factors.front().data();   // P x rL
      const double* Rf = tk.factors.back().data();   // P x rR
      std::vector<double> T1((size_t)P * cs.rR);
      for (int k2 = 0; k2 < cs.r2; ++k2)
        for (int k1 = 0; k1 < cs.r1; ++k1) {
          std::fill(T1.begin(), T1.end(), 0.0);
          for (int b = 0; b < cs.rR; ++b)
            for (int a = 0; a < cs.rL; ++a) {
              const double g = tk.core[(size_t)a + (size_t)cs.rL * (k1 + (size_t)cs.r1 * (k2 + (size_t)cs.r2 * b))];
              for (int i = 0; i < P; ++i) T1[(size_t)i + (size_t)P * b] += L[(size_t)i + (size_t)P * a] * g;
            }
          double* out = &m->ff_chat[(size_t)cs.chat_off + (size_t)(k1 + cs.r1 * k2) * P * P];
          for (int b = 0; b < cs.rR; ++b)
            for (int j = 0; j < P; ++j) {
              const double r = Rf[(size_t)j + (size_t)P * b];
              for (int i = 0; i < P; ++i) out[(size_t)i + (size_t)P * j] += T1[(size_t)i + (size_t)P * b] * r;
            }
        }
    }
  }

  // ---- near blocks (s <= t stored)
  const int64_t nn = t.n_near();
  m->near_src.assign(nn, -1);
  m->near_tr.assign(nn, 0);
  {
    std::map<std::pair<int32_t, int32_t>, int32_t> idx;
    for (int64_t b = 0; b < nn; ++b) idx[{t.near[2 * b], t.near[2 * b + 1]}] = (int32_t)b;
    for (int64_t b = 0; b < nn; ++b) {
      int32_t s = t.near[2 * b], u = t.near[2 * b + 1];
      if (s > u) continue;
      NearStored ns{};
      ns.s = s; ns.t = u;
      ns.s_begin = t.begin[s]; ns.t_begin = t.begin[u];
      ns.ns = (int32_t)t.size(s); ns.nt = (int32_t)t.size(u);
      ns.b_st = (int32_t)b;
      ns.b_ts = -1;
      m->near_src[b] = (int32_t)m->nstore.size();
      if (s != u) {
        auto it = idx.find({u, s});
        if (it == idx.end()) fail(PH_ESTATE, "near block list is not symmetric");
        ns.b_ts = it->second;
        m->near_src[it->second] = (int32_t)m->nstore.size();
        m->near_tr[it->second] = 1;
      }
      m->nstore.push_back(ns);
    }
  }
  const int64_t nst = (int64_t)m->nstore.size();
  std::vector<Tucker> ntuck(nst);
  std::vector<int64_t> near_evals(nst, -1);   // TT-cross: distinct entries evaluated per block
  int64_t evals_near = 0;
  // near tensor of stored block bi from src (GPU-generated) or evaluated here, then compressed
  auto near_one = [&](int64_t bi, const double* src) {
    const NearStored& b = m->nstore[bi];
    const int64_t Ne = (int64_t)b.ns * b.nt;
    if (use_tt) {
      NearCtx nc{o.kernel, d, dth, pt, b.ns, &t.pts_t[(size_t)b.s_begin * d], &t.pts_t[(size_t)b.t_begin * d],
                 grid.data()};
      std::vector<int> tdims{(int)Ne};
      for (int k = 0; k < dth; ++k) tdims.push_back(pt);
      lerr.guard([&] {
        TensorTrain tt = tt_compress(near_entries, &nc, tdims, o.tol);
        near_evals[bi] = tt.evals;
        ntuck[bi] = tt_near_tucker(tt, dth);
      });
      return;
    }
    std::vector<double> A((size_t)Ne * q);
    if (src) {
      std::memcpy(A.data(), src, A.size() * sizeof(double));
    } else {
      for (int kk = 0; kk < q; ++kk)
        for (int32_t j = 0; j < b.nt; ++j) {
          const double* y = &t.pts_t[(size_t)(b.t_begin + j) * d];
          double* col = A.data() + (size_t)kk * Ne + (size_t)j * b.ns;
          for (int32_t i = 0; i < b.ns; ++i)
            col[i] = kernel_value(o.kernel, d, &t.pts_t[(size_t)(b.s_begin + i) * d], y, &grid[2 * kk]);
        }
    }
    std::vector<int64_t> dims{Ne};
    if (dth == 1) dims.push_back(pt);
    else { dims.push_back(pt); dims.push_back(pt); }
    ntuck[bi] = thosvd(A, dims, o.tol);
  };
  if (!gpu) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t bi = 0; bi < nst; ++bi) near_one(bi, nullptr);
  } else {
    // batches of at most 64 M tensor entries (512 MB) generated on the GPU, then compressed
    constexpr int64_t BATCH = (int64_t)1 << 26;
    for (int64_t b0 = 0; b0 < nst;) {
      std::vector<NearJob> jobs;
      int64_t tot = 0, b1 = b0;
      while (b1 < nst) {
        const NearStored& b = m->nstore[b1];
        const int64_t e = (int64_t)b.ns * b.nt * q;
        if (tot > 0 && tot + e > BATCH) break;
        jobs.push_back(NearJob{b.s_begin, b.t_begin, tot, b.ns, b.nt});
        tot += e;
        ++b1;
      }
      const int64_t nj = b1 - b0;
      if (dth == 1 && q <= 16) {
        // one parameter: the tensor A (Ne x q) is compressed on the GPU.  R of A = QR comes
        // back; its SVD R = U_R S V^T gives the singular values and right singular vectors of
        // A, the rank r follows the rule of the host HOSVD (both modes share the singular
        // values), and the factors are U_e = A V_r S_r^-1 (formed on the GPU), Theta = V_r,
        // core = S_r: the blocks U_e S_r Theta^T v(theta) = A V_r V_r^T v(theta).
        std::vector<double> R((size_t)nj * q * q);
        gen->near_qr(jobs, q, tot, R.data());
        std::vector<std::vector<double>> sv(nj), vr(nj);
        std::vector<int> sweeps(nj, 0);
        std::vector<int32_t> rk(nj, 0);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
        for (int64_t jb = 0; jb < nj; ++jb) {
          std::vector<double> W(R.begin() + jb * q * q, R.begin() + (jb + 1) * q * q), U((size_t)q * q), V((size_t)q * q);
          sv[jb].assign(q, 0.0);
          sweeps[jb] = jacobi_svd(W.data(), q, sv[jb].data(), U.data(), V.data());
          double normsq = 0;
          for (double v : sv[jb]) normsq += v * v;
          rk[jb] = normsq == 0.0 ? 0 : truncation_rank(sv[jb].data(), q, (o.tol * o.tol / 2) * normsq);
          vr[jb] = V;
        }
        std::vector<double> Wm;
        std::vector<int64_t> woff(nj), uoff(nj);
        int64_t utot = 0;
        for (int64_t jb = 0; jb < nj; ++jb) {
          woff[jb] = (int64_t)Wm.size();
          for (int k = 0; k < rk[jb]; ++k)
            for (int c = 0; c < q; ++c) Wm.push_back(vr[jb][(size_t)k * q + c] / sv[jb][k]);
          uoff[jb] = utot;
          utot += (int64_t)m->nstore[b0 + jb].ns * m->nstore[b0 + jb].nt * rk[jb];
        }
        std::vector<double> Ubuf((size_t)utot);
        gen->near_factors(jobs, q, Wm, woff, rk, uoff, utot, Ubuf.data());
        for (int64_t jb = 0; jb < nj; ++jb) {
          const int64_t Ne = (int64_t)m->nstore[b0 + jb].ns * m->nstore[b0 + jb].nt;
          const int r = rk[jb];
          Tucker& tk = ntuck[b0 + jb];
          tk.ranks = {r, r};
          tk.sweeps = sweeps[jb];
          tk.factors.clear();
          tk.factors.emplace_back(Ubuf.begin() + uoff[jb], Ubuf.begin() + uoff[jb] + Ne * r);
          tk.factors.emplace_back(vr[jb].begin(), vr[jb].begin() + (size_t)q * r);
          tk.core.assign((size_t)r * r, 0.0);
          for (int k = 0; k < r; ++k) tk.core[(size_t)k * r + k] = sv[jb][k];
        }
      } else {
        std::vector<double> buf((size_t)tot);
        gen->near(jobs, q, buf.data(), tot);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
        for (int64_t bi = b0; bi < b1; ++bi) near_one(bi, buf.data() + jobs[bi - b0].off);
      }
      b0 = b1;
    }
  }
  lerr.raise();
  for (int64_t bi = 0; bi < nst; ++bi)
    evals_near += near_evals[bi] >= 0 ? near_evals[bi] : (int64_t)m->nstore[bi].ns * m->nstore[bi].nt * q;
  for (const Tucker& tk : ntuck) m->svd_sweeps_max = std::max(m->svd_sweeps_max, tk.sweeps);
  if (m->svd_sweeps_max > JACOBI_MAX_SWEEPS)
    fail(PH_EUNSUPPORTED, "ph_offline_compress: a one-sided Jacobi SVD was still rotating after " +
                              std::to_string(JACOBI_MAX_SWEEPS) + " sweeps (not converged)");
  {
    size_t totP = 0, totC = 0, totT = 0;
    for (int64_t bi = 0; bi < nst; ++bi) {
      const Tucker& tk = ntuck[bi];
      const NearStored& b = m->nstore[bi];
      totP += (size_t)((b.ns + 15) / 16 * 16) * b.nt * tk.ranks[0];
      totC += tk.core.size();
      for (size_t f = 1; f < tk.factors.size(); ++f) totT += tk.factors[f].size();
    }
    m->nf_P.reserve(totP);
    m->nf_core.reserve(totC);
    m->nf_theta.reserve(totT);
  }
  for (int64_t bi = 0; bi < nst; ++bi) {
    NearStored& b = m->nstore[bi];
    Tucker& tk = ntuck[bi];
    b.r_e = tk.ranks[0];
    b.r1 = tk.ranks[1];
    b.r2 = dth == 2 ? tk.ranks[2] : 1;
    // rank-outer [k][i + j ldp] with the pair index padded to a leading dimension that is a
    // multiple of 16 entries, so every column starts on a 128-byte boundary
    b.ldp = (b.ns + 15) / 16 * 16;
    b.P_off = (int64_t)m->nf_P.size();
    {
      const int64_t Ne = (int64_t)b.ns * b.nt, Nep = (int64_t)b.ldp * b.nt;
      m->nf_P.resize(m->nf_P.size() + (size_t)Nep * b.r_e, 0.0);
      double* dst = m->nf_P.data() + b.P_off;
      for (int k = 0; k < b.r_e; ++k)
        for (int32_t j = 0; j < b.nt; ++j)
          std::memcpy(dst + k * Nep + (int64_t)j * b.ldp, tk.factors[0].data() + k * Ne + (int64_t)j * b.ns,
                      sizeof(double) * b.ns);
    }
    m->near_factor_entries += (int64_t)b.ns * b.nt * b.r_e;
    b.core_off = (int64_t)m->nf_core.size();
    m->nf_core.insert(m->nf_core.end(), tk.core.begin(), tk.core.end());
    b.th1_off = (int64_t)m->nf_theta.size();
    m->nf_theta.insert(m->nf_theta.end(), tk.factors[1].begin(), tk.factors[1].end());
    b.th2_off = (int64_t)m->nf_theta.size();
    if (dth == 2) m->nf_theta.insert(m->nf_theta.end(), tk.factors[2].begin(), tk.factors[2].end());
    tk = Tucker();
  }
  m->kernel_evals = evals_far + evals_near;
  return m;
}

// TT ranks of the far tensor of every translation class after TT-cross + TT-rounding (Sec. 2.1),
// for comparisons of the compression itself; no model is built, so P = p_s^d (up to 4096) and
// p_theta (up to 64) are not limited by the online stage's kernels.  ranks: n_classes x (N + 1),
// N = 2 d + d_theta; a mirrored class reports its stored class's ranks in reverse order.
std::vector<int32_t> tt_far_ranks(const TreeData& t, const ph_offline_opts& o, int64_t* evals_out) {
  const int d = t.d;
  if (o.p_s < 1 || o.p_s > 16 || o.p_theta < 1 || o.p_theta > 64)
    fail(PH_EINVAL, "ph_tt_far_ranks: p_s must be in 1..16 and p_theta in 1..64");
  if (!(o.tol >= 0.0)) fail(PH_EINVAL, "ph_tt_far_ranks: tol must be >= 0");
  const int dth = kernel_dtheta(o.kernel, d);
  if (dth < 0) fail(PH_EUNSUPPORTED, "ph_tt_far_ranks: unknown kernel");
  if (o.kernel == PH_KERNEL_ANISO_GAUSSIAN && d > 2)
    fail(PH_EUNSUPPORTED, "ph_tt_far_ranks: anisotropic Gaussian supports d <= 2");
  if (o.d_theta != dth) fail(PH_EUNSUPPORTED, "ph_tt_far_ranks: d_theta does not match the kernel");
  for (int k = 0; k < dth; ++k)
    if (!(o.theta_lo[k] < o.theta_hi[k])) fail(PH_EINVAL, "ph_tt_far_ranks: need theta_lo < theta_hi");
  if (o.kernel == PH_KERNEL_MATERN && !(o.theta_lo[0] > 0 && o.theta_lo[1] > 0))
    fail(PH_EINVAL, "ph_tt_far_ranks: the Matern kernel needs lambda > 0 and nu > 0 on all of Theta");
  const int ps = o.p_s, pt = o.p_theta;
  int P = 1;
  for (int k = 0; k < d; ++k) P *= ps;
  const int N = 2 * d + dth;
  const int q = dth == 1 ? pt : pt * pt;
  std::vector<double> thn((size_t)2 * pt), grid((size_t)q * 2, 0.0);
  for (int k = 0; k < dth; ++k) cheb_nodes(o.theta_lo[k], o.theta_hi[k], pt, thn.data() + (size_t)pt * k);
  for (int kk = 0; kk < q; ++kk) {
    grid[2 * kk] = thn[kk % pt];
    if (dth == 2) grid[2 * kk + 1] = thn[(size_t)pt + kk / pt];
  }
  const int64_t ncls = t.n_classes();
  std::map<std::vector<int32_t>, int32_t> bykey;
  for (int64_t c = 0; c < ncls; ++c) {
    std::vector<int32_t> kk{t.class_level[c]};
    for (int k = 0; k < d; ++k) kk.push_back(t.class_off[c * d + k]);
    bykey[kk] = (int32_t)c;
  }
  // stored classes (offset >= its negative) and, for the others, the stored class they mirror
  std::vector<int32_t> src(ncls, -1), canon;
  for (int64_t c = 0; c < ncls; ++c) {
    std::vector<int32_t> off(t.class_off.begin() + c * d, t.class_off.begin() + (c + 1) * d), neg(d);
    for (int k = 0; k < d; ++k) neg[k] = -off[k];
    if (off >= neg) {
      canon.push_back((int32_t)c);
    } else {
      std::vector<int32_t> mk{t.class_level[c]};
      mk.insert(mk.end(), neg.begin(), neg.end());
      auto it = bykey.find(mk);
      if (it == bykey.end()) fail(PH_ESTATE, "far class list is not symmetric");
      src[c] = it->second;
    }
  }
  std::vector<int32_t> ranks((size_t)ncls * (N + 1), 0);
  int64_t evals = 0;
  LoopError lerr;
  const int nthreads = o.num_threads > 0 ? o.num_threads : omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) reduction(+ : evals)
  for (int64_t ci = 0; ci < (int64_t)canon.size(); ++ci) {
    lerr.guard([&] {
      const int32_t c = canon[ci];
      const int32_t b = t.class_first_block[c];
      const int32_t s = t.far[2 * b], u = t.far[2 * b + 1];
      std::vector<double> ns((size_t)P * d), nt((size_t)P * d);
      for (int k = 0; k < d; ++k) {
        double bs[16], bt[16];
        cheb_nodes(t.box_lo[s * d + k], t.box_hi[s * d + k], ps, bs);
        cheb_nodes(t.box_lo[u * d + k], t.box_hi[u * d + k], ps, bt);
        int stride = 1;
        for (int kk = 0; kk < k; ++kk) stride *= ps;
        for (int i = 0; i < P; ++i) {
          ns[(size_t)i * d + k] = bs[(i / stride) % ps];
          nt[(size_t)i * d + k] = bt[(i / stride) % ps];
        }
      }
      FarCtx fc{o.kernel, d, dth, ps, P, ns.data(), nt.data(), grid.data(), pt};
      std::vector<int> tdims(d, ps);
      for (int k = 0; k < dth; ++k) tdims.push_back(pt);
      for (int k = 0; k < d; ++k) tdims.push_back(ps);
      TensorTrain tt = tt_compress(far_entries, &fc, tdims, o.tol);
      evals += tt.evals;
      for (int k = 0; k <= N; ++k) ranks[(size_t)c * (N + 1) + k] = tt.ranks[k];
    });
  }
  lerr.raise();
  for (int64_t c = 0; c < ncls; ++c)
    if (src[c] >= 0)
      for (int k = 0; k <= N; ++k) ranks[(size_t)c * (N + 1) + k] = ranks[(size_t)src[c] * (N + 1) + (N - k)];
  if (evals_out) *evals_out = evals;
  return ranks;
}

// Parametric H-matrix far field (Def. "Parametric H-matrix"; App. PTTK, offline phase 3).
// For far block b = (s, t) of class c with stored class q: S_b = U_s A and T_b = U_t B, where
// (A, B) = (L_q, R_q), or (R_q, L_q) when c is the mirror of q (its far tensor is the transpose),
// and U_s is the tensor Chebyshev basis of cluster s (nodes on its own box, index little-endian
// over the axes) evaluated at the cluster's points in tree order.  The block's coupling is then
// S_b H_q(theta) T_b^T, or S_b H_q(theta)^T T_b^T for a mirrored class.
void hmatrix_far_host(const TreeData& t, HostModel& m, int num_threads) {
  const int d = t.d, ps = m.p_s, P = m.P;
  const int64_t nfar = t.n_far();
  const int nthreads = num_threads > 0 ? num_threads : omp_get_max_threads();
  m.hblk.assign(nfar, HBlock{});
  int64_t offS = 0, offT = 0;
  for (int64_t b = 0; b < nfar; ++b) {
    HBlock& h = m.hblk[b];
    h.s = t.far[2 * b];
    h.t = t.far[2 * b + 1];
    const int32_t c = t.far_class[b];
    h.q = m.class_src[c];
    h.tr = m.class_tr[c];
    const ClassStored& cs = m.cstore[h.q];
    h.rs = h.tr ? cs.rR : cs.rL;
    h.rt = h.tr ? cs.rL : cs.rR;
    h.s_begin = t.begin[h.s];
    h.t_begin = t.begin[h.t];
    h.ns = t.size(h.s);
    h.nt = t.size(h.t);
    h.lds = (int32_t)((h.ns + 15) / 16 * 16);
    h.ldt = (int32_t)((h.nt + 15) / 16 * 16);
    h.S_off = offS;
    h.T_off = offT;
    offS += (int64_t)h.lds * h.rs;
    offT += (int64_t)h.ldt * h.rt;
  }
  m.hS.assign((size_t)offS, 0.0);
  m.hT.assign((size_t)offT, 0.0);
  // rows of U_node A for the points [begin, begin + np) of a node, into out (column-major, ld)
  auto project = [&](int32_t node, int64_t begin, int64_t np, const double* A, int r, double* out, int64_t ld) {
    double nodes[3][16], lk[3][16];
    for (int k = 0; k < d; ++k) cheb_nodes(t.box_lo[node * d + k], t.box_hi[node * d + k], ps, nodes[k]);
    std::vector<double> u(P);
    for (int64_t i = 0; i < np; ++i) {
      for (int k = 0; k < d; ++k) lagrange_all(nodes[k], ps, t.pts_t[(begin + i) * d + k], lk[k]);
      for (int mi = 0; mi < P; ++mi) {
        double v = 1.0;
        int rem = mi;
        for (int k = 0; k < d; ++k) {
          v *= lk[k][rem % ps];
          rem /= ps;
        }
        u[mi] = v;
      }
      for (int a = 0; a < r; ++a) {
        double acc = 0.0;
        for (int mi = 0; mi < P; ++mi) acc += u[mi] * A[(size_t)mi + (size_t)P * a];
        out[(size_t)i + (size_t)ld * a] = acc;
      }
    }
  };
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
  for (int64_t b = 0; b < nfar; ++b) {
    const HBlock& h = m.hblk[b];
    const ClassStored& cs = m.cstore[h.q];
    const double* L = m.ff_L.data() + cs.L_off;   // P x rL
    const double* R = m.ff_R.data() + cs.R_off;   // P x rR
    project(h.s, h.s_begin, h.ns, h.tr ? R : L, h.rs, m.hS.data() + h.S_off, h.lds);
    project(h.t, h.t_begin, h.nt, h.tr ? L : R, h.rt, m.hT.data() + h.T_off, h.ldt);
  }
  m.hformat = true;
}

}  // namespace ph
