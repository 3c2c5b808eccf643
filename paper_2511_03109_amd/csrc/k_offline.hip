// Offline stage on the GPU: the kernel tensors of Alg. "Offline Stage: Parametric H²-matrix"
// (near tensors [A_b]_{(ij), k} = kappa(x_{s,i}, x_{t,j}; eta_k), Sec. 4.3; far tensors
// [M_b]_{i,k,j} = kappa(eta_i^{(B_s)}, eta_j^{(B_t)}; eta_k), App. PTTK) evaluated by GPU
// threads with the same kernel functions as the host (kernel_fn.hpp).  For one parameter the
// near tensors are also compressed here: a Householder QR per block gives R, the host takes the
// SVD of the small R (one-sided Jacobi) and the truncation rank, and the factor A V_r S_r^-1 is
// formed on the GPU; the far tensors and the near tensors of two parameters are compressed on
// the host.
#include <vector>

#include "kernel_fn.hpp"
#include "ph_device.hpp"

namespace ph {

// one workgroup per (job, chunk of NT pairs); every thread evaluates its pair at all q nodes
__global__ void __launch_bounds__(NT) k_near_tensors(const double* __restrict__ pts, const NearJob* __restrict__ jobs,
                                                     const double* __restrict__ grid,
                                                     const BesselOrder* __restrict__ orders, int q, int d,
                                                     ph_kernel kern, double* __restrict__ out) {
  const NearJob jb = jobs[blockIdx.y];
  const int64_t Ne = (int64_t)jb.ns * jb.nt;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < Ne; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e % jb.ns, j = e / jb.ns;
    double x[3], y[3];
    for (int k = 0; k < d; ++k) {
      x[k] = pts[(jb.s_begin + i) * d + k];
      y[k] = pts[(jb.t_begin + j) * d + k];
    }
    for (int kk = 0; kk < q; ++kk)
      out[jb.off + kk * Ne + e] = kernel_eval(kern, d, x, y, grid + 2 * kk, orders[kk]);
  }
}

// one workgroup per (class, chunk of entries) of the P x q x P far tensors
__global__ void __launch_bounds__(NT) k_far_tensors(const double* __restrict__ nodes, const double* __restrict__ grid,
                                                    const BesselOrder* __restrict__ orders, int P, int q, int d,
                                                    ph_kernel kern, double* __restrict__ out) {
  const int64_t c = blockIdx.y;
  const int64_t per = (int64_t)P * q * P;
  const double* a = nodes + c * 2 * P * d;
  const double* b = a + (int64_t)P * d;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < per; e += (int64_t)gridDim.x * NT) {
    const int i = (int)(e % P);
    const int64_t rest = e / P;
    const int kk = (int)(rest % q), j = (int)(rest / q);
    out[c * per + e] = kernel_eval(kern, d, a + (int64_t)i * d, b + (int64_t)j * d, grid + 2 * kk, orders[kk]);
  }
}

// Householder QR of each job's near tensor A (Ne x q, column-major, q <= 16) in place, one
// workgroup per job: for column j the reflector v = x - alpha e_1 (x = A[j:, j], alpha = -sign(x_0)
// ||x||) is formed and applied to the columns j + 1 .. q - 1 (their q - 1 - j inner products with
// v in one pass over the rows, reduced through LDS, then the rank-one update).  R (q x q,
// column-major, zero below the diagonal) goes to R[job q q].  Only R is needed: the factors are
// formed from A and the SVD of R (k_near_factor).
__global__ void __launch_bounds__(NT) k_near_qr(double* __restrict__ A, const NearJob* __restrict__ jobs, int q,
                                                double* __restrict__ R) {
  __shared__ double red[NT / WAVE][17];
  __shared__ double sh[17];
  const NearJob jb = jobs[blockIdx.x];
  const int64_t Ne = (int64_t)jb.ns * jb.nt;
  double* a = A + jb.off;
  double* Rj = R + (int64_t)blockIdx.x * q * q;
  const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
  // block-wide sums of the NV values v[0..NV-1] of every thread, into sh[0..NV-1]
  auto reduce = [&](double* v, int nv) {
    for (int c = 0; c < nv; ++c) {
      double x = v[c];
      for (int off = WAVE / 2; off > 0; off >>= 1) x += __shfl_down(x, off, WAVE);
      if (lane == 0) red[wave][c] = x;
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
      double s = 0;
      for (int w = 0; w < NT / WAVE; ++w) s += red[w][threadIdx.x];
      sh[threadIdx.x] = s;
    }
    __syncthreads();
  };
  for (int e = threadIdx.x; e < q * q; e += NT) Rj[e] = 0.0;
  for (int j = 0; j < q && j < Ne; ++j) {
    double* x = a + (int64_t)j * Ne;
    double part[17];
    part[0] = 0;
    for (int64_t i = j + threadIdx.x; i < Ne; i += NT) part[0] += x[i] * x[i];
    reduce(part, 1);
    const double nrm2 = sh[0];
    const double x0 = x[j];
    __syncthreads();
    // zero column: R[j][j] = 0 and no reflection
    const double nrm = sqrt(nrm2);
    const double alpha = x0 >= 0 ? -nrm : nrm;
    const double v0 = x0 - alpha;
    const double vtv = v0 * v0 + (nrm2 - x0 * x0);
    if (threadIdx.x == 0) Rj[(int64_t)j * q + j] = alpha;
    const int nc = q - 1 - j;
    if (nrm2 > 0.0 && nc > 0 && vtv > 0) {
      for (int c = 0; c < nc; ++c) part[c] = 0;
      for (int64_t i = j + threadIdx.x; i < Ne; i += NT) {
        const double vi = i == j ? v0 : x[i];
        for (int c = 0; c < nc; ++c) part[c] += vi * a[(int64_t)(j + 1 + c) * Ne + i];
      }
      reduce(part, nc);
      double f[16];
      for (int c = 0; c < nc; ++c) f[c] = 2.0 * sh[c] / vtv;
      __syncthreads();
      for (int64_t i = j + threadIdx.x; i < Ne; i += NT) {
        const double vi = i == j ? v0 : x[i];
        for (int c = 0; c < nc; ++c) a[(int64_t)(j + 1 + c) * Ne + i] -= f[c] * vi;
      }
      __syncthreads();
    }
    // row j of R in the later columns
    if ((int)threadIdx.x < nc) Rj[(int64_t)(j + 1 + threadIdx.x) * q + j] = a[(int64_t)(j + 1 + threadIdx.x) * Ne + j];
    __syncthreads();
  }
}

// U_job = A_job W_job (Ne x r, W q x r column-major at woff), column-major into U at uoff
__global__ void __launch_bounds__(NT) k_near_factor(const double* __restrict__ A, const NearJob* __restrict__ jobs,
                                                    int q, const double* __restrict__ W,
                                                    const int64_t* __restrict__ woff, const int32_t* __restrict__ rk,
                                                    const int64_t* __restrict__ uoff, double* __restrict__ U) {
  const NearJob jb = jobs[blockIdx.y];
  const int64_t Ne = (int64_t)jb.ns * jb.nt;
  const int r = rk[blockIdx.y];
  const double* a = A + jb.off;
  const double* w = W + woff[blockIdx.y];
  double* u = U + uoff[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < Ne; e += (int64_t)gridDim.x * NT) {
    double av[16];
    for (int c = 0; c < q; ++c) av[c] = a[(int64_t)c * Ne + e];
    for (int k = 0; k < r; ++k) {
      double s = 0;
      for (int c = 0; c < q; ++c) s += av[c] * w[(int64_t)k * q + c];
      u[(int64_t)k * Ne + e] = s;
    }
  }
}

struct GpuTensorGen::Impl {
  int d, q;
  ph_kernel kernel;
  hipStream_t st = nullptr;
  DevArr<double> pts, grid;
  DevArr<BesselOrder> orders;
  DevArr<double> A, Q;          // near tensors of the current batch and their QR copy
  DevArr<NearJob> jobs;
};

GpuTensorGen::GpuTensorGen(const TreeData& t, ph_kernel kernel, const double* grid, int q) : p_(new Impl) {
  p_->d = t.d;
  p_->q = q;
  p_->kernel = kernel;
  PH_HIP(hipStreamCreateWithFlags(&p_->st, hipStreamNonBlocking));
  p_->pts.upload(t.pts_t.data(), t.pts_t.size(), p_->st);
  p_->grid.upload(grid, (size_t)2 * q, p_->st);
  std::vector<BesselOrder> ord(q, BesselOrder{});
  if (kernel == PH_KERNEL_MATERN)
    for (int kk = 0; kk < q; ++kk) ord[kk] = bessel_order(grid[2 * kk + 1]);
  p_->orders.upload(ord.data(), ord.size(), p_->st);
  PH_HIP(hipStreamSynchronize(p_->st));
}

GpuTensorGen::~GpuTensorGen() {
  if (p_->st) (void)hipStreamDestroy(p_->st);
  delete p_;
}

void GpuTensorGen::near(const std::vector<NearJob>& jobs, int q, double* out, int64_t total) {
  if (jobs.empty() || total == 0) return;
  DevArr<NearJob> dj;
  DevArr<double> dout;
  dj.upload(jobs.data(), jobs.size(), p_->st);
  dout.alloc((size_t)total);
  int64_t maxe = 0;
  for (const NearJob& j : jobs) maxe = std::max<int64_t>(maxe, (int64_t)j.ns * j.nt);
  const unsigned gx = (unsigned)std::min<int64_t>((maxe + NT - 1) / NT, 1024);
  for (size_t j0 = 0; j0 < jobs.size(); j0 += 65535) {
    const unsigned nj = (unsigned)std::min<size_t>(65535, jobs.size() - j0);
    launch(PH_STAGE_NEAR_INST, k_near_tensors, dim3(gx, nj), dim3(NT), p_->st, (const double*)p_->pts.p,
           (const NearJob*)dj.p + j0, (const double*)p_->grid.p, (const BesselOrder*)p_->orders.p, q, p_->d,
           p_->kernel, dout.p);
  }
  PH_HIP(hipMemcpyAsync(out, dout.p, (size_t)total * sizeof(double), hipMemcpyDeviceToHost, p_->st));
  PH_HIP(hipStreamSynchronize(p_->st));
}

void GpuTensorGen::near_qr(const std::vector<NearJob>& jobs, int q, int64_t total, double* R) {
  if (jobs.empty()) return;
  if (q > 16) fail(PH_EUNSUPPORTED, "GPU near-tensor QR supports at most 16 parameter nodes");
  p_->jobs.upload(jobs.data(), jobs.size(), p_->st);
  if (p_->A.n < (size_t)total) {
    p_->A.alloc((size_t)total);
    p_->Q.alloc((size_t)total);
  }
  int64_t maxe = 0;
  for (const NearJob& j : jobs) maxe = std::max<int64_t>(maxe, (int64_t)j.ns * j.nt);
  const unsigned gx = (unsigned)std::min<int64_t>((maxe + NT - 1) / NT, 1024);
  DevArr<double> dR;
  dR.alloc(jobs.size() * q * q);
  for (size_t j0 = 0; j0 < jobs.size(); j0 += 65535) {
    const unsigned nj = (unsigned)std::min<size_t>(65535, jobs.size() - j0);
    launch(PH_STAGE_NEAR_INST, k_near_tensors, dim3(gx, nj), dim3(NT), p_->st, (const double*)p_->pts.p,
           (const NearJob*)p_->jobs.p + j0, (const double*)p_->grid.p, (const BesselOrder*)p_->orders.p, q, p_->d,
           p_->kernel, p_->A.p);
  }
  PH_HIP(hipMemcpyAsync(p_->Q.p, p_->A.p, (size_t)total * sizeof(double), hipMemcpyDeviceToDevice, p_->st));
  for (size_t j0 = 0; j0 < jobs.size(); j0 += 65535) {
    const unsigned nj = (unsigned)std::min<size_t>(65535, jobs.size() - j0);
    launch(PH_STAGE_NEAR_INST, k_near_qr, dim3(nj), dim3(NT), p_->st, p_->Q.p, (const NearJob*)p_->jobs.p + j0, q,
           dR.p + j0 * q * q);
  }
  PH_HIP(hipMemcpyAsync(R, dR.p, jobs.size() * q * q * sizeof(double), hipMemcpyDeviceToHost, p_->st));
  PH_HIP(hipStreamSynchronize(p_->st));
}

void GpuTensorGen::near_factors(const std::vector<NearJob>& jobs, int q, const std::vector<double>& W,
                                const std::vector<int64_t>& woff, const std::vector<int32_t>& rk,
                                const std::vector<int64_t>& uoff, int64_t utotal, double* out) {
  if (jobs.empty() || utotal == 0) return;
  DevArr<double> dW, dU;
  DevArr<int64_t> dwo, duo;
  DevArr<int32_t> drk;
  dW.upload(W.data(), W.size(), p_->st);
  dwo.upload(woff.data(), woff.size(), p_->st);
  duo.upload(uoff.data(), uoff.size(), p_->st);
  drk.upload(rk.data(), rk.size(), p_->st);
  dU.alloc((size_t)utotal);
  int64_t maxe = 0;
  for (const NearJob& j : jobs) maxe = std::max<int64_t>(maxe, (int64_t)j.ns * j.nt);
  const unsigned gx = (unsigned)std::min<int64_t>((maxe + NT - 1) / NT, 1024);
  for (size_t j0 = 0; j0 < jobs.size(); j0 += 65535) {
    const unsigned nj = (unsigned)std::min<size_t>(65535, jobs.size() - j0);
    launch(PH_STAGE_NEAR_INST, k_near_factor, dim3(gx, nj), dim3(NT), p_->st, (const double*)p_->A.p,
           (const NearJob*)p_->jobs.p + j0, q, (const double*)dW.p, (const int64_t*)dwo.p + j0,
           (const int32_t*)drk.p + j0, (const int64_t*)duo.p + j0, dU.p);
  }
  PH_HIP(hipMemcpyAsync(out, dU.p, (size_t)utotal * sizeof(double), hipMemcpyDeviceToHost, p_->st));
  PH_HIP(hipStreamSynchronize(p_->st));
}

void GpuTensorGen::far(const std::vector<double>& nodes, int n_cls, int P, double* out) {
  if (n_cls == 0) return;
  DevArr<double> dn, dout;
  dn.upload(nodes.data(), nodes.size(), p_->st);
  const int64_t per = (int64_t)P * p_->q * P;
  dout.alloc((size_t)per * n_cls);
  const unsigned gx = (unsigned)std::min<int64_t>((per + NT - 1) / NT, 1024);
  for (int c0 = 0; c0 < n_cls; c0 += 65535) {
    const unsigned nc = (unsigned)std::min(65535, n_cls - c0);
    launch(PH_STAGE_FAR_INST, k_far_tensors, dim3(gx, nc), dim3(NT), p_->st,
           (const double*)dn.p + (int64_t)c0 * 2 * P * p_->d, (const double*)p_->grid.p,
           (const BesselOrder*)p_->orders.p, P, p_->q, p_->d, p_->kernel, dout.p + (int64_t)c0 * per);
  }
  PH_HIP(hipMemcpyAsync(out, dout.p, (size_t)per * n_cls * sizeof(double), hipMemcpyDeviceToHost, p_->st));
  PH_HIP(hipStreamSynchronize(p_->st));
}

}  // namespace ph
