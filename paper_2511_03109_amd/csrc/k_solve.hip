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

template <typename S>
__global__ void __launch_bounds__(NT) k_vdot_partial(const S* __restrict__ u, const S* __restrict__ v,
                                                     double* __restrict__ part, int64_t n) {
  __shared__ double red[NT];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)DOT_BLOCKS * NT)
    acc += (double)u[e] * (double)v[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(NT) k_vdot_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[NT];
  double acc = 0.0;
  for (int b = threadIdx.x; b < DOT_BLOCKS; b += NT) acc += part[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// y += alpha x
template <typename S>
__global__ void k_axpy(S* __restrict__ y, const S* __restrict__ x, double alpha, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (S)((double)y[i] + alpha * (double)x[i]);
}

// p = r + beta p
template <typename S>
__global__ void k_xpby(S* __restrict__ p, const S* __restrict__ r, double beta, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (S)((double)r[i] + beta * (double)p[i]);
}

// dst = (D) src * scale
// CG scalars on the device, sc = {rr, pq, rr_new, alpha, beta, stop, active, iterations}:
// the vector kernels read alpha / beta from sc and do nothing once `active` is 0 (converged
// or lost positive definiteness), so iterations are launched in batches without a host
// round trip per inner product.
enum { SC_RR, SC_PQ, SC_RRN, SC_ALPHA, SC_BETA, SC_STOP, SC_ACTIVE, SC_IT, SC_N };

__global__ void k_cg_alpha(double* sc) {
  if (threadIdx.x != 0 || sc[SC_ACTIVE] == 0.0) return;
  const double pq = sc[SC_PQ];
  if (!(pq > 0)) {   // loss of positive definiteness in the low precision: stop
    sc[SC_ACTIVE] = 0.0;
    return;
  }
  sc[SC_ALPHA] = sc[SC_RR] / pq;
}

__global__ void k_cg_beta(double* sc) {
  if (threadIdx.x != 0 || sc[SC_ACTIVE] == 0.0) return;
  const double rn = sc[SC_RRN];
  sc[SC_BETA] = rn / sc[SC_RR];
  sc[SC_RR] = rn;
  sc[SC_IT] += 1.0;
  if (!(rn > sc[SC_STOP])) sc[SC_ACTIVE] = 0.0;   // converged (p is not needed any more)
}

// y += sign alpha x (alpha from sc) while active
template <typename S>
__global__ void k_axpy_dev(S* __restrict__ y, const S* __restrict__ x, const double* __restrict__ sc, double sign,
                           int64_t n) {
  if (sc[SC_ACTIVE] == 0.0) return;
  const double a = sign * sc[SC_ALPHA];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (S)((double)y[i] + a * (double)x[i]);
}

// p = r + beta p (beta from sc) while active
template <typename S>
__global__ void k_xpby_dev(S* __restrict__ p, const S* __restrict__ r, const double* __restrict__ sc, int64_t n) {
  if (sc[SC_ACTIVE] == 0.0) return;
  const double b = sc[SC_BETA];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (S)((double)r[i] + b * (double)p[i]);
}

template <typename D, typename S>
__global__ void k_convert(D* __restrict__ dst, const S* __restrict__ src, double scale, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (D)((double)src[i] * scale);
}

namespace {

struct Solver {
  hipStream_t st;
  int64_t n;
  DevArr<double> part, dots, sc;
  double* host = nullptr;   // pinned, SC_N doubles
  Solver(hipStream_t s, int64_t n_) : st(s), n(n_) {
    part.alloc(DOT_BLOCKS);
    dots.alloc(1);
    sc.alloc(SC_N);
    PH_HIP(hipHostMalloc((void**)&host, SC_N * sizeof(double), hipHostMallocDefault));
  }
  // inner product into a device scalar, no host round trip
  template <typename S>
  void dot_dev(const S* u, const S* v, double* out) {
    launch(PH_STAGE_SOLVE, k_vdot_partial<S>, dim3(DOT_BLOCKS), dim3(NT), st, u, v, part.p, n);
    launch(PH_STAGE_SOLVE, k_vdot_final, dim3(1), dim3(NT), st, (const double*)part.p, out);
  }
  ~Solver() {
    if (host) (void)hipHostFree(host);
  }
  template <typename S>
  double dot(const S* u, const S* v) {
    launch(PH_STAGE_SOLVE, k_vdot_partial<S>, dim3(DOT_BLOCKS), dim3(NT), st, u, v, part.p, n);
    launch(PH_STAGE_SOLVE, k_vdot_final, dim3(1), dim3(NT), st, (const double*)part.p, dots.p);
    PH_HIP(hipMemcpyAsync(host, dots.p, sizeof(double), hipMemcpyDeviceToHost, st));
    PH_HIP(hipStreamSynchronize(st));
    return *host;
  }
  template <typename S>
  void axpy(S* y, const S* x, double a) {
    launch(PH_STAGE_SOLVE, k_axpy<S>, dim3((unsigned)grid_for(n)), dim3(NT), st, y, x, a, n);
  }
  template <typename S>
  void xpby(S* p, const S* r, double b) {
    launch(PH_STAGE_SOLVE, k_xpby<S>, dim3((unsigned)grid_for(n)), dim3(NT), st, p, r, b, n);
  }
  template <typename D, typename S>
  void convert(D* dst, const S* src, double scale) {
    launch(PH_STAGE_SOLVE, k_convert<D, S>, dim3((unsigned)grid_for(n)), dim3(NT), st, dst, src, scale, n);
  }
};

// (K + nugget I) v for one slot and one right-hand side of instance `in`
template <typename S>
void apply(InstData& in, const S* v, S* out, double nugget, hipStream_t st) {
  if (in.dt == PH_F64)
    matvec_impl<double, double>(in, (const double*)v, (double*)out, 1, 1.0, 0.0, nugget, st);
  else if (in.dt == PH_F32)
    matvec_impl<float, float>(in, (const float*)v, (float*)out, 1, 1.0, 0.0, nugget, st);
  else
    matvec_impl<float, bf16>(in, (const float*)v, (float*)out, 1, 1.0, 0.0, nugget, st);
}

// CG from x = 0 on (K + nugget I) x = b until ||r|| <= rtol ||b|| or maxit iterations;
// returns the iterations taken.  Vectors r, p, q are caller scratch of length n.
template <typename S>
int cg(Solver& sv, InstData& in, const S* b, S* x, S* r, S* p, S* q, double nugget, double rtol, int maxit,
       double* rel_out) {
  const int64_t n = sv.n;
  PH_HIP(hipMemsetAsync(x, 0, n * sizeof(S), sv.st));
  PH_HIP(hipMemcpyAsync(r, b, n * sizeof(S), hipMemcpyDeviceToDevice, sv.st));
  PH_HIP(hipMemcpyAsync(p, b, n * sizeof(S), hipMemcpyDeviceToDevice, sv.st));
  const double bb = sv.dot(b, b);
  const double stop = rtol * rtol * bb;
  const double h[SC_N] = {bb, 0, 0, 0, 0, stop, (bb > 0 && bb > stop && maxit > 0) ? 1.0 : 0.0, 0};
  std::copy(h, h + SC_N, sv.host);   // pinned staging (the stream was synchronised by dot)
  PH_HIP(hipMemcpyAsync(sv.sc.p, sv.host, SC_N * sizeof(double), hipMemcpyHostToDevice, sv.st));
  double* sc = sv.sc.p;
  const unsigned gv = (unsigned)grid_for(n);
  // batches of CHK iterations between host checks; iterations after convergence are no-ops
  // (at most CHK - 1 products are wasted)
  constexpr int CHK = 8;
  int launched = 0;
  bool active = h[SC_ACTIVE] != 0.0;
  while (active && launched < maxit) {
    const int nb = std::min(CHK, maxit - launched);
    for (int k = 0; k < nb; ++k) {
      apply<S>(in, p, q, nugget, sv.st);
      sv.dot_dev(p, q, sc + SC_PQ);
      launch(PH_STAGE_SOLVE, k_cg_alpha, dim3(1), dim3(64), sv.st, sc);
      launch(PH_STAGE_SOLVE, k_axpy_dev<S>, dim3(gv), dim3(NT), sv.st, x, (const S*)p, (const double*)sc, 1.0, n);
      launch(PH_STAGE_SOLVE, k_axpy_dev<S>, dim3(gv), dim3(NT), sv.st, r, (const S*)q, (const double*)sc, -1.0, n);
      sv.dot_dev(r, r, sc + SC_RRN);
      launch(PH_STAGE_SOLVE, k_cg_beta, dim3(1), dim3(64), sv.st, sc);
      launch(PH_STAGE_SOLVE, k_xpby_dev<S>, dim3(gv), dim3(NT), sv.st, p, (const S*)r, (const double*)sc, n);
    }
    launched += nb;
    PH_HIP(hipMemcpyAsync(sv.host, sc, SC_N * sizeof(double), hipMemcpyDeviceToHost, sv.st));
    PH_HIP(hipStreamSynchronize(sv.st));
    active = sv.host[SC_ACTIVE] != 0.0;
  }
  if (launched == 0) {
    sv.host[SC_RR] = bb;
    sv.host[SC_IT] = 0;
  }
  const double rr = sv.host[SC_RR];
  if (rel_out) *rel_out = bb > 0 ? std::sqrt(rr / bb) : 0.0;
  return (int)sv.host[SC_IT];
}

}  // namespace

void cg_solve_impl(InstData& hi, InstData* lo, const double* y, double* a, double nugget, double tol,
                   int max_iter, int inner_max, double inner_tol, ph_cg_stats* stats, hipStream_t st) {
  const int64_t n = hi.m->n;
  Solver sv(st, n);
  DevArr<double> r, w;
  r.alloc(n);
  w.alloc(n);
  ph_cg_stats s{};
  const double yy = sv.dot(y, y);
  auto true_residual = [&]() {   // r = y - (K + nugget I) a  (FP64 instance)
    PH_HIP(hipMemcpyAsync(r.p, y, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    matvec_impl<double, double>(hi, a, r.p, 1, -1.0, 1.0, nugget, st);
    return yy > 0 ? std::sqrt(sv.dot(r.p, r.p) / yy) : 0.0;
  };
  if (!lo) {
    // plain FP64 CG, restarted from the true residual if the recursive one drifted
    DevArr<double> x, p, q;
    x.alloc(n);
    p.alloc(n);
    q.alloc(n);
    PH_HIP(hipMemsetAsync(a, 0, n * sizeof(double), st));
    double rel = 1.0;
    PH_HIP(hipMemcpyAsync(r.p, y, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    while (s.inner_iterations < max_iter) {
      double rec = 0;
      s.inner_iterations += cg<double>(sv, hi, r.p, x.p, w.p, p.p, q.p, nugget, tol / rel, max_iter - s.inner_iterations,
                                       &rec);
      sv.axpy(a, x.p, 1.0);
      rel = true_residual();
      ++s.outer_steps;
      if (rel <= tol || rec >= 1.0) break;
    }
    s.rel_residual = rel;
    s.converged = rel <= tol;
  } else {
    // iterative refinement: inner solves in the instance's low precision
    DevArr<float> b32, x32, r32, p32, q32;
    b32.alloc(n);
    x32.alloc(n);
    r32.alloc(n);
    p32.alloc(n);
    q32.alloc(n);
    PH_HIP(hipMemsetAsync(a, 0, n * sizeof(double), st));
    PH_HIP(hipMemcpyAsync(r.p, y, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    double rel = 1.0;
    while (s.outer_steps < max_iter && rel > tol) {
      // scale the residual to unit norm for the FP32 solve
      const double rn = std::sqrt(sv.dot(r.p, r.p));
      if (!(rn > 0)) break;
      sv.convert(b32.p, r.p, 1.0 / rn);
      double rec = 0;
      s.inner_iterations += cg<float>(sv, *lo, b32.p, x32.p, r32.p, p32.p, q32.p, nugget, inner_tol, inner_max, &rec);
      sv.convert(w.p, x32.p, rn);
      sv.axpy(a, w.p, 1.0);
      const double prev = rel;
      rel = true_residual();
      ++s.outer_steps;
      if (!(rel < prev)) break;   // refinement no longer contracts
    }
    s.rel_residual = rel;
    s.converged = rel <= tol;
  }
  if (stats) *stats = s;
}

}  // namespace ph
