// Host-only test harness: the offline stage's own SVD, truncated HOSVD (offline.cpp, compiled
// into this translation unit) and TT compression (tt.cpp, linked beside it) behind a small C
// interface, so that a CPU test can compare them with LAPACK's and with the oracle's on the
// same tensors.  Test infrastructure; not part of the library.
#include "../../paper_2511_03109_amd/csrc/offline.cpp"

extern "C" {

// Left singular vectors and singular values of the column-major m x q matrix X:
// s_out[min(m, q)], U_out[m x min(m, q)] column-major.  Returns the Jacobi sweep count.
int harness_left_sv(const double* X, int64_t m, int64_t q, double* s_out, double* U_out) {
  ph::LeftSV sv = ph::left_sv(X, m, q);
  for (int i = 0; i < sv.kk; ++i) s_out[i] = sv.s[i];
  for (size_t i = 0; i < sv.U.size(); ++i) U_out[i] = sv.U[i];
  return sv.sweeps;
}

// Truncated HOSVD of the column-major tensor T (dims[0..N-1], first index fastest) with
// the library's rank rule: ranks[N] and the reconstruction core x_1 U_1 ... x_N U_N into
// recon (same size as T).
void harness_thosvd(const double* T, const int64_t* dims, int N, double tol, int* ranks, double* recon) {
  std::vector<int64_t> n(dims, dims + N);
  int64_t total = 1;
  for (int64_t v : n) total *= v;
  std::vector<double> t(T, T + total);
  ph::Tucker tk = ph::thosvd(t, n, tol);
  for (int m = 0; m < N; ++m) ranks[m] = tk.ranks[m];
  // expand mode by mode: Y = core x_m U_m
  std::vector<int64_t> cur(tk.ranks.begin(), tk.ranks.end());
  std::vector<double> Y = tk.core;
  for (int m = 0; m < N; ++m) {
    int64_t left = 1, right = 1;
    for (int i = 0; i < m; ++i) left *= cur[i];
    for (int i = m + 1; i < N; ++i) right *= cur[i];
    const int64_t r = cur[m], full = n[m];
    std::vector<double> Z((size_t)left * full * right, 0.0);
    const double* U = tk.factors[m].data();   // full x r, column-major
    for (int64_t rr = 0; rr < right; ++rr)
      for (int64_t a = 0; a < r; ++a)
        for (int64_t i = 0; i < full; ++i) {
          const double u = U[(size_t)a * full + i];
          const double* src = Y.data() + (size_t)left * (a + r * rr);
          double* dst = Z.data() + (size_t)left * (i + full * rr);
          for (int64_t l = 0; l < left; ++l) dst[l] += u * src[l];
        }
    Y.swap(Z);
    cur[m] = full;
  }
  for (int64_t i = 0; i < total; ++i) recon[i] = Y[(size_t)i];
}

// TT-cross + TT-rounding (tt_compress) of the column-major tensor T with dims[0..N-1]: the TT
// ranks into ranks[0..N] and the TT's full tensor into recon; returns the number of distinct
// entries the cross evaluated.
static void dense_entries(const void* c, const int32_t* idx, int64_t count, double* out) {
  const auto* ctx = static_cast<const std::pair<const double*, std::vector<int64_t>>*>(c);
  const int N = (int)ctx->second.size();
  for (int64_t s = 0; s < count; ++s) {
    int64_t l = 0;
    for (int k = 0; k < N; ++k) l += ctx->second[k] * idx[s * N + k];
    out[s] = ctx->first[l];
  }
}

int64_t harness_tt(const double* T, const int* dims, int N, double tol, int* ranks, double* recon) {
  std::vector<int> d(dims, dims + N);
  std::vector<int64_t> stride;
  int64_t s = 1;
  for (int m : d) {
    stride.push_back(s);
    s *= m;
  }
  std::pair<const double*, std::vector<int64_t>> ctx{T, stride};
  ph::TensorTrain tt = ph::tt_compress(dense_entries, &ctx, d, tol);
  for (int k = 0; k <= N; ++k) ranks[k] = tt.ranks[k];
  // full tensor: X (rows x r) grown core by core
  std::vector<double> X = tt.cores[0];
  int64_t rows = d[0];
  for (int k = 1; k < N; ++k) {
    const int r0 = tt.ranks[k], m = d[k], r1 = tt.ranks[k + 1];
    std::vector<double> Y((size_t)rows * m * r1, 0.0);
    for (int b = 0; b < r1; ++b)
      for (int i = 0; i < m; ++i)
        for (int a = 0; a < r0; ++a) {
          const double g = tt.cores[k][(size_t)a + (size_t)r0 * (i + (size_t)m * b)];
          for (int64_t q = 0; q < rows; ++q) Y[(size_t)q + (size_t)rows * (i + (size_t)m * b)] += X[(size_t)q + (size_t)rows * a] * g;
        }
    X.swap(Y);
    rows *= m;
  }
  for (int64_t i = 0; i < rows; ++i) recon[i] = X[(size_t)i];
  return tt.evals;
}

}  // extern "C"
