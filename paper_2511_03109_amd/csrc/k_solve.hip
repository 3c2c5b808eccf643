// Conjugate gradients for (K~(theta) + nugget I) a = y on the device, in FP64 or with
// FP64 iterative refinement around a low-precision inner solver: the residual
// r = y - (K~ + nugget I) a is always formed with the FP64 instance, and each
// correction d solves (K~_lo + nugget I) d = r approximately with CG on an FP32 / BF16
// instance of the same theta.  Vector updates and inner products are HIP kernels; the
// inner products use the fixed-order two-pass reduction, so a solve is reproducible.
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
template <typename D, typename S>
__global__ void k_convert(D* __restrict__ dst, const S* __restrict__ src, double scale, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (D)((double)src[i] * scale);
}

namespace {

struct Solver {
  hipStream_t st;
  int64_t n;
  DevArr<double> part, dots;
  double* host = nullptr;   // pinned, 1 double
  Solver(hipStream_t s, int64_t n_) : st(s), n(n_) {
    part.alloc(DOT_BLOCKS);
    dots.alloc(1);
    PH_HIP(hipHostMalloc((void**)&host, sizeof(double), hipHostMallocDefault));
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
  double rr = bb;
  const double stop = rtol * rtol * bb;
  int it = 0;
  while (it < maxit && rr > stop && bb > 0) {
    apply<S>(in, p, q, nugget, sv.st);
    const double pq = sv.dot(p, q);
    if (!(pq > 0)) break;   // loss of positive definiteness in the low precision: stop
    const double alpha = rr / pq;
    sv.axpy(x, p, alpha);
    sv.axpy(r, q, -alpha);
    const double rr_new = sv.dot(r, r);
    sv.xpby(p, r, rr_new / rr);
    rr = rr_new;
    ++it;
  }
  if (rel_out) *rel_out = bb > 0 ? std::sqrt(rr / bb) : 0.0;
  return it;
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
