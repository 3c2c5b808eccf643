// Conjugate gradients for (K~(theta) + nugget I) a = y on the device, in FP64 or with
// FP64 iterative refinement around a low-precision inner solver: the residual
// r = y - (K~ + nugget I) a is always formed with the FP64 instance, and each
// correction d solves (K~_lo + nugget I) d = r approximately with CG on an FP32 / BF16
// instance of the same theta.  Vector updates and inner products are HIP kernels; the
// inner products use the fixed-order two-pass reduction, so a solve is reproducible.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ph_device.hpp"

namespace ph {

constexpr int DOT_BLOCKS = 256;

// Vectors of R right-hand sides are [R][n]; column r of every kernel below is blockIdx.y.
// Inner products: part[r][b] = sum over the elements e = b, b + NB, ... of column r of u[e] v[e]
// (FP64), then a fixed-order workgroup tree reduction per column.
template <typename S>
__global__ void __launch_bounds__(NT) k_vdot_partial(const S* __restrict__ u, const S* __restrict__ v,
                                                     double* __restrict__ part, int64_t n) {
  __shared__ double red[NT];
  const int64_t col = blockIdx.y;
  const S* uc = u + col * n;
  const S* vc = v + col * n;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)DOT_BLOCKS * NT)
    acc += (double)uc[e] * (double)vc[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[col * DOT_BLOCKS + blockIdx.x] = red[0];
}

// out[r stride] = sum_b part[r][b], one workgroup per column
__global__ void __launch_bounds__(NT) k_vdot_final(const double* __restrict__ part, double* __restrict__ out,
                                                   int stride) {
  __shared__ double red[NT];
  const int col = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < DOT_BLOCKS; b += NT) acc += part[col * DOT_BLOCKS + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)col * stride] = red[0];
}

// y += alpha_r x per column (host scalars, one per column)
template <typename S>
__global__ void k_axpy(S* __restrict__ y, const S* __restrict__ x, const double* __restrict__ alpha, int64_t n) {
  const int64_t col = blockIdx.y;
  const double a = alpha[col];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[col * n + i] = (S)((double)y[col * n + i] + a * (double)x[col * n + i]);
}

// CG scalars on the device, per column sc[r][...] = {rr, pq, rr_new, alpha, beta, stop, active,
// iterations}: the vector kernels read alpha / beta of their column from sc and do nothing once
// its `active` is 0 (converged or lost positive definiteness), so iterations are launched in
// batches without a host round trip per inner product.
enum { SC_RR, SC_PQ, SC_RRN, SC_ALPHA, SC_BETA, SC_STOP, SC_ACTIVE, SC_IT, SC_N };

__global__ void k_cg_alpha(double* sc, int R) {
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    double* c = sc + (int64_t)r * SC_N;
    if (c[SC_ACTIVE] == 0.0) continue;
    const double pq = c[SC_PQ];
    if (!(pq > 0)) {   // loss of positive definiteness in the low precision: stop
      c[SC_ACTIVE] = 0.0;
      continue;
    }
    c[SC_ALPHA] = c[SC_RR] / pq;
  }
}

__global__ void k_cg_beta(double* sc, int R) {
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    double* c = sc + (int64_t)r * SC_N;
    if (c[SC_ACTIVE] == 0.0) continue;
    const double rn = c[SC_RRN];
    c[SC_BETA] = rn / c[SC_RR];
    c[SC_RR] = rn;
    c[SC_IT] += 1.0;
    if (!(rn > c[SC_STOP])) c[SC_ACTIVE] = 0.0;   // converged (p is not needed any more)
  }
}

// y += sign alpha x (alpha of the column from sc) while the column is active
template <typename S>
__global__ void k_axpy_dev(S* __restrict__ y, const S* __restrict__ x, const double* __restrict__ sc, double sign,
                           int64_t n) {
  const int64_t col = blockIdx.y;
  const double* c = sc + col * SC_N;
  if (c[SC_ACTIVE] == 0.0) return;
  const double a = sign * c[SC_ALPHA];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[col * n + i] = (S)((double)y[col * n + i] + a * (double)x[col * n + i]);
}

// p = r + beta p (beta of the column from sc) while the column is active
template <typename S>
__global__ void k_xpby_dev(S* __restrict__ p, const S* __restrict__ r, const double* __restrict__ sc, int64_t n) {
  const int64_t col = blockIdx.y;
  const double* c = sc + col * SC_N;
  if (c[SC_ACTIVE] == 0.0) return;
  const double b = c[SC_BETA];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[col * n + i] = (S)((double)r[col * n + i] + b * (double)p[col * n + i]);
}

// dst = (D) src * scale_r per column
template <typename D, typename S>
__global__ void k_convert(D* __restrict__ dst, const S* __restrict__ src, const double* __restrict__ scale, int64_t n) {
  const int64_t col = blockIdx.y;
  const double f = scale[col];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[col * n + i] = (D)((double)src[col * n + i] * f);
}

namespace {

struct Solver {
  hipStream_t st;
  int64_t n;
  int R;
  DevArr<double> part, dots, sc, coef;
  double* host = nullptr;   // pinned, R SC_N doubles
  Solver(hipStream_t s, int64_t n_, int R_) : st(s), n(n_), R(R_) {
    part.alloc((size_t)DOT_BLOCKS * R);
    dots.alloc(R);
    sc.alloc((size_t)SC_N * R);
    coef.alloc(R);
    PH_HIP(hipHostMalloc((void**)&host, (size_t)SC_N * R * sizeof(double), hipHostMallocDefault));
  }
  ~Solver() {
    if (host) (void)hipHostFree(host);
  }
  unsigned gv() const { return (unsigned)grid_for(n); }
  // inner products of the R columns into device scalars (out[r stride]), no host round trip
  template <typename S>
  void dot_dev(const S* u, const S* v, double* out, int stride) {
    launch(PH_STAGE_SOLVE, k_vdot_partial<S>, dim3(DOT_BLOCKS, (unsigned)R), dim3(NT), st, u, v, part.p, n);
    launch(PH_STAGE_SOLVE, k_vdot_final, dim3((unsigned)R), dim3(NT), st, (const double*)part.p, out, stride);
  }
  // inner products of the R columns, read back to the host
  template <typename S>
  std::vector<double> dot(const S* u, const S* v) {
    dot_dev(u, v, dots.p, 1);
    PH_HIP(hipMemcpyAsync(host, dots.p, R * sizeof(double), hipMemcpyDeviceToHost, st));
    PH_HIP(hipStreamSynchronize(st));
    return std::vector<double>(host, host + R);
  }
  void upload_coef(const std::vector<double>& c) {   // per-column scalars (stream is synchronised)
    std::copy(c.begin(), c.end(), host);
    PH_HIP(hipMemcpyAsync(coef.p, host, R * sizeof(double), hipMemcpyHostToDevice, st));
    PH_HIP(hipStreamSynchronize(st));
  }
  template <typename S>
  void axpy(S* y, const S* x, const std::vector<double>& a) {
    upload_coef(a);
    launch(PH_STAGE_SOLVE, k_axpy<S>, dim3(gv(), (unsigned)R), dim3(NT), st, y, x, (const double*)coef.p, n);
  }
  template <typename D, typename S>
  void convert(D* dst, const S* src, const std::vector<double>& scale) {
    upload_coef(scale);
    launch(PH_STAGE_SOLVE, k_convert<D, S>, dim3(gv(), (unsigned)R), dim3(NT), st, dst, src, (const double*)coef.p,
           n);
  }
};

// (K + nugget I) v for one slot and the R right-hand sides of instance `in`
template <typename S>
void apply(InstData& in, const S* v, S* out, int64_t R, double nugget, hipStream_t st) {
  if (in.dt == PH_F64)
    matvec_impl<double, double>(in, (const double*)v, (double*)out, R, 1.0, 0.0, nugget, st);
  else if (in.dt == PH_F32)
    matvec_impl<float, float>(in, (const float*)v, (float*)out, R, 1.0, 0.0, nugget, st);
  else
    matvec_impl<float, bf16>(in, (const float*)v, (float*)out, R, 1.0, 0.0, nugget, st);
}

// CG from x = 0 on (K + nugget I) x = b for the R columns until ||r_c|| <= rtol_c ||b_c|| or
// maxit iterations; each column stops on its own (the product is applied to all R at once).
// Returns the largest number of iterations of a column; rel_out[c] the recursive relative
// residual of column c.  Vectors r, p, q are caller scratch of R n entries.
template <typename S>
int cg(Solver& sv, InstData& in, const S* b, S* x, S* r, S* p, S* q, double nugget, const std::vector<double>& rtol,
       int maxit, std::vector<double>& rel_out) {
  const int64_t n = sv.n;
  const int R = sv.R;
  PH_HIP(hipMemsetAsync(x, 0, (size_t)R * n * sizeof(S), sv.st));
  PH_HIP(hipMemcpyAsync(r, b, (size_t)R * n * sizeof(S), hipMemcpyDeviceToDevice, sv.st));
  PH_HIP(hipMemcpyAsync(p, b, (size_t)R * n * sizeof(S), hipMemcpyDeviceToDevice, sv.st));
  const std::vector<double> bb = sv.dot(b, b);
  bool active = false;
  for (int c = 0; c < R; ++c) {
    const double stop = rtol[c] * rtol[c] * bb[c];
    const bool act = bb[c] > 0 && bb[c] > stop && maxit > 0;
    const double h[SC_N] = {bb[c], 0, 0, 0, 0, stop, act ? 1.0 : 0.0, 0};
    std::copy(h, h + SC_N, sv.host + (size_t)c * SC_N);   // pinned staging (stream synchronised by dot)
    active = active || act;
  }
  PH_HIP(hipMemcpyAsync(sv.sc.p, sv.host, (size_t)R * SC_N * sizeof(double), hipMemcpyHostToDevice, sv.st));
  double* sc = sv.sc.p;
  const unsigned gv = sv.gv();
  // batches of CHK iterations between host checks; iterations after convergence are no-ops
  // (at most CHK - 1 products are wasted)
  constexpr int CHK = 8;
  int launched = 0;
  while (active && launched < maxit) {
    const int nb = std::min(CHK, maxit - launched);
    for (int k = 0; k < nb; ++k) {
      apply<S>(in, p, q, R, nugget, sv.st);
      sv.dot_dev(p, q, sc + SC_PQ, SC_N);
      launch(PH_STAGE_SOLVE, k_cg_alpha, dim3(1), dim3(64), sv.st, sc, R);
      launch(PH_STAGE_SOLVE, k_axpy_dev<S>, dim3(gv, (unsigned)R), dim3(NT), sv.st, x, (const S*)p, (const double*)sc,
             1.0, n);
      launch(PH_STAGE_SOLVE, k_axpy_dev<S>, dim3(gv, (unsigned)R), dim3(NT), sv.st, r, (const S*)q, (const double*)sc,
             -1.0, n);
      sv.dot_dev(r, r, sc + SC_RRN, SC_N);
      launch(PH_STAGE_SOLVE, k_cg_beta, dim3(1), dim3(64), sv.st, sc, R);
      launch(PH_STAGE_SOLVE, k_xpby_dev<S>, dim3(gv, (unsigned)R), dim3(NT), sv.st, p, (const S*)r, (const double*)sc,
             n);
    }
    launched += nb;
    PH_HIP(hipMemcpyAsync(sv.host, sc, (size_t)R * SC_N * sizeof(double), hipMemcpyDeviceToHost, sv.st));
    PH_HIP(hipStreamSynchronize(sv.st));
    active = false;
    for (int c = 0; c < R; ++c) active = active || sv.host[(size_t)c * SC_N + SC_ACTIVE] != 0.0;
  }
  int its = 0;
  rel_out.assign(R, 0.0);
  for (int c = 0; c < R; ++c) {
    const double* h = sv.host + (size_t)c * SC_N;
    const double rr = launched == 0 ? bb[c] : h[SC_RR];
    rel_out[c] = bb[c] > 0 ? std::sqrt(rr / bb[c]) : 0.0;
    its = std::max(its, launched == 0 ? 0 : (int)h[SC_IT]);
  }
  return its;
}

}  // namespace

void cg_solve_impl(InstData& hi, InstData* lo, const double* y, double* a, int64_t R_, double nugget, double tol,
                   int max_iter, int inner_max, double inner_tol, ph_cg_stats* stats, hipStream_t st) {
  const int64_t n = hi.m->n;
  const int R = (int)R_;
  Solver sv(st, n, R);
  DevArr<double> r, w;
  r.alloc((size_t)R * n);
  w.alloc((size_t)R * n);
  ph_cg_stats s{};
  const std::vector<double> yy = sv.dot(y, y);
  std::vector<double> rel(R, 1.0);
  auto true_residual = [&]() {   // r = y - (K + nugget I) a  (FP64 instance), per column
    PH_HIP(hipMemcpyAsync(r.p, y, (size_t)R * n * sizeof(double), hipMemcpyDeviceToDevice, st));
    matvec_impl<double, double>(hi, a, r.p, R, -1.0, 1.0, nugget, st);
    const std::vector<double> rr = sv.dot(r.p, r.p);
    for (int c = 0; c < R; ++c) rel[c] = yy[c] > 0 ? std::sqrt(rr[c] / yy[c]) : 0.0;
  };
  auto worst = [&]() { return *std::max_element(rel.begin(), rel.end()); };
  PH_HIP(hipMemsetAsync(a, 0, (size_t)R * n * sizeof(double), st));
  PH_HIP(hipMemcpyAsync(r.p, y, (size_t)R * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (!lo) {
    // plain FP64 CG, restarted from the true residual if a recursive one drifted
    DevArr<double> x, p, q;
    x.alloc((size_t)R * n);
    p.alloc((size_t)R * n);
    q.alloc((size_t)R * n);
    while (s.inner_iterations < max_iter) {
      std::vector<double> rt(R), rec;
      for (int c = 0; c < R; ++c) rt[c] = rel[c] > 0 ? tol / rel[c] : 1.0;
      s.inner_iterations += cg<double>(sv, hi, r.p, x.p, w.p, p.p, q.p, nugget, rt, max_iter - s.inner_iterations, rec);
      sv.axpy(a, x.p, std::vector<double>(R, 1.0));
      true_residual();
      ++s.outer_steps;
      bool stalled = false;
      for (int c = 0; c < R; ++c) stalled = stalled || rec[c] >= 1.0;
      if (worst() <= tol || stalled) break;
    }
  } else {
    // iterative refinement: inner solves in the instance's low precision
    DevArr<float> b32, x32, r32, p32, q32;
    b32.alloc((size_t)R * n);
    x32.alloc((size_t)R * n);
    r32.alloc((size_t)R * n);
    p32.alloc((size_t)R * n);
    q32.alloc((size_t)R * n);
    while (s.outer_steps < max_iter && worst() > tol) {
      // scale each residual column to unit norm for the FP32 solve
      const std::vector<double> rr = sv.dot(r.p, r.p);
      std::vector<double> inv(R), rn(R);
      bool any = false;
      for (int c = 0; c < R; ++c) {
        rn[c] = std::sqrt(rr[c]);
        inv[c] = rn[c] > 0 ? 1.0 / rn[c] : 0.0;
        any = any || rn[c] > 0;
      }
      if (!any) break;
      sv.convert(b32.p, r.p, inv);
      std::vector<double> rec;
      s.inner_iterations += cg<float>(sv, *lo, b32.p, x32.p, r32.p, p32.p, q32.p, nugget,
                                      std::vector<double>(R, inner_tol), inner_max, rec);
      sv.convert(w.p, x32.p, rn);
      sv.axpy(a, w.p, std::vector<double>(R, 1.0));
      const double prev = worst();
      true_residual();
      ++s.outer_steps;
      if (!(worst() < prev)) break;   // refinement no longer contracts
    }
  }
  s.rel_residual = worst();
  s.converged = s.rel_residual <= tol;
  if (stats) *stats = s;
}

}  // namespace ph
