// Host-only test harness: the offline stage's own SVD and truncated HOSVD (offline.cpp,
// compiled into this translation unit) behind a small C interface, so that a CPU test can
// compare them with LAPACK's on the same tensors.  Test infrastructure; not part of the
// library.
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

}  // extern "C"
