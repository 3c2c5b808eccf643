// Device side of the parametric H^2 library for MI355X (gfx950): model upload,
// online stage (instantiation) and the H^2 matrix-vector product, plus the C ABI.
//
// Paper: arxiv 2511.03109.  Online stage: Alg. "Online Stage" and Alg. PTTK
// online (parametric vectors v_k(theta_k), App. PTTK review); near field
// D_b(theta) = reshape(P_b c_b(theta), [n_s, n_t]) (Sec. 4.3); far field
// C(theta) = L H(theta) R^T (Sec. 4.2).  MVM: Alg. "H^2-matrix MVM" with
// FastForward / FastBackward and the coupling y_hat_s += C x_hat_t of Alg.
// "Modified H^2-Matrix MVM".
//
// Layouts (device):
//   x, y (caller)      slot-major [T][R][n], column-major n x R per slot, original order
//   xt, yt (scratch)   [n][R], tree order, R fastest
//   xh, yh (scratch)   [node][P][R], R fastest
//   D (instance)       per slot, canonical near blocks back to back, each n_s x n_t
//                      column-major
//   C (instance)       per slot, one P x P column-major matrix per translation class
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ph_host.hpp"

namespace ph {

static thread_local std::string g_last_error;

#define PH_HIP(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) ::ph::fail(PH_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
struct DevArr {
  T* p = nullptr;
  size_t n = 0;
  DevArr() = default;
  DevArr(const DevArr&) = delete;
  DevArr& operator=(const DevArr&) = delete;
  ~DevArr() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    void* q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      fail(PH_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    p = static_cast<T*>(q);
    n = count;
  }
  void upload(const T* h, size_t count, hipStream_t s) {
    alloc(count);
    if (count) PH_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  size_t bytes() const { return n * sizeof(T); }
};

// per stored near block (s <= t), shared layout host/device
struct NearDev {
  int64_t s_begin, t_begin, P_off, core_off, th1_off, th2_off, D_st, D_ts;
  int32_t ns, nt, r_e, r1, r2, pad;
};

// per stored far class (offset >= 0)
struct ClassDev {
  int64_t L_off, R_off, core_off, th1_off, th2_off, C_off, Cm_off, S_off;
  int32_t rL, r1, r2, rR;
};

struct DeviceModel {
  std::shared_ptr<const TreeData> tree;
  int d = 0, p_s = 0, P = 0, p_theta = 0, d_theta = 0, l_max = 0, min_far = -1;
  double th_lo[2] = {0, 0}, th_hi[2] = {0, 0};
  int64_t n = 0, n_nodes = 0, n_leaves = 0, n_near = 0, n_classes = 0, N_nf = 0;
  int64_t n_stored_near = 0, n_stored_cls = 0, n_tiles = 0, ff_scratch = 0;
  int64_t near_factor_entries = 0, kernel_evals = 0;
  double near_rank_mean = 0, far_rank_mean = 0;
  int near_rank_max = 0, far_rank_max = 0;
  std::vector<int32_t> near_rank_canon;   // per canonical near block (-1 if transposed copy)
  std::vector<int32_t> class_ranks;       // per class, 2 + d_theta entries
  std::vector<int64_t> D_off_host;        // per canonical near block, n_near + 1
  // device arrays
  DevArr<double> U, E;
  DevArr<int64_t> perm;
  DevArr<int32_t> first_child, nchild, cid, parent;
  DevArr<int64_t> nbegin, nend;
  DevArr<NearDev> nstore;
  DevArr<double> nf_P, nf_core, nf_theta;
  DevArr<int32_t> tiles;                  // 3 per tile: stored block, i0, j0
  DevArr<int64_t> near_rowptr;            // per leaf index
  DevArr<int64_t> near_tb, near_D;        // per canonical near block: tau begin, D offset
  DevArr<int32_t> near_nt;
  DevArr<ClassDev> cstore;
  DevArr<double> ff_L, ff_R, ff_core, ff_theta;
  DevArr<int64_t> far_rowptr;             // per node
  DevArr<int32_t> far_tau, far_cls;
  int64_t device_bytes = 0;
};

struct InstData {
  std::shared_ptr<const DeviceModel> m;
  int T = 1;
  ph_dtype dt = PH_F64;
  int grad_dim = -1;
  size_t esize = 8;
  DevArr<char> D, C;
  DevArr<double> v, ffs;
  int64_t Rcap = 0;
  DevArr<char> xt, yt, xh, yh;
};

// ---- per-kernel timing with HIP events (enabled by ph_trace_enable)
struct TraceRec {
  int stage;
  hipEvent_t a, b;
};
static std::mutex g_trace_mu;
static bool g_trace_on = false;
static std::vector<TraceRec> g_trace_recs;
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t pooled_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  PH_HIP(hipEventCreate(&e));
  return e;
}

// Launch a kernel on stream st; when tracing, bracket it with events tagged by stage.
template <typename K, typename... Args>
static void launch(int stage, K kernel, dim3 grid, dim3 block, hipStream_t st, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  const bool tr = g_trace_on;
  if (tr) {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    a = pooled_event();
    b = pooled_event();
  }
  if (tr) PH_HIP(hipEventRecord(a, st));
  hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
  PH_HIP(hipGetLastError());
  if (tr) {
    PH_HIP(hipEventRecord(b, st));
    std::lock_guard<std::mutex> lk(g_trace_mu);
    g_trace_recs.push_back({stage, a, b});
  }
}

constexpr int NT = 256;       // threads per workgroup
constexpr int TILE = 32;      // near-field instantiation tile edge
constexpr int MAXT = 64;      // parameter values per theta-vector launch

// ------------------------------------------------------------------ kernels
struct ThetaPack {
  double th[MAXT * 2];
  double lo[2], hi[2];
  int count, dth, p, grad_dim;
};

// v[(t*dth + k)*p + i] = l_i(theta_{t,k}) on [lo_k, hi_k] (product formula, Sec. 2.2),
// or its derivative for k == grad_dim.
__global__ void k_theta_vectors(ThetaPack tp, double* __restrict__ v, int t0) {
  const int total = tp.count * tp.dth * tp.p;
  for (int o = threadIdx.x; o < total; o += blockDim.x) {
    const int i = o % tp.p;
    const int k = (o / tp.p) % tp.dth;
    const int t = o / (tp.p * tp.dth);
    const double a = tp.lo[k], b = tp.hi[k], x = tp.th[t * 2 + k];
    double nodes[16];
    for (int q = 0; q < tp.p; ++q)
      nodes[q] = (a + b) / 2.0 - (b - a) / 2.0 * cos((2.0 * (q + 1) - 1.0) * M_PI / (2.0 * tp.p));
    double val;
    if (k != tp.grad_dim) {
      val = 1.0;
      for (int q = 0; q < tp.p; ++q)
        if (q != i) val *= (x - nodes[q]) / (nodes[i] - nodes[q]);
    } else {
      val = 0.0;
      for (int m = 0; m < tp.p; ++m) {
        if (m == i) continue;
        double term = 1.0 / (nodes[i] - nodes[m]);
        for (int q = 0; q < tp.p; ++q)
          if (q != i && q != m) term *= (x - nodes[q]) / (nodes[i] - nodes[q]);
        val += term;
      }
    }
    v[((size_t)(t0 + t) * tp.dth + k) * tp.p + i] = val;
  }
}

// Far field, one workgroup per (stored class, slot):
//   w_k = Theta_k^T v_k,  H = core x_theta w,  S = H R^T,  C = L S  (and C^T for the mirror).
template <typename S>
__global__ void __launch_bounds__(NT) k_far_instantiate(
    const ClassDev* __restrict__ cls, const double* __restrict__ L, const double* __restrict__ R,
    const double* __restrict__ core, const double* __restrict__ th, const double* __restrict__ v,
    double* __restrict__ scratch, int64_t scratch_per_slot, S* __restrict__ C, int64_t C_per_slot,
    int P, int p, int dth) {
  __shared__ double w1[16], w2[16];
  const ClassDev c = cls[blockIdx.x];
  const int t = blockIdx.y;
  const double* vt = v + (size_t)t * dth * p;
  for (int a = threadIdx.x; a < c.r1; a += blockDim.x) {
    double s = 0;
    for (int q = 0; q < p; ++q) s += th[c.th1_off + q + (size_t)p * a] * vt[q];
    w1[a] = s;
  }
  if (dth == 2) {
    for (int a = threadIdx.x; a < c.r2; a += blockDim.x) {
      double s = 0;
      for (int q = 0; q < p; ++q) s += th[c.th2_off + q + (size_t)p * a] * vt[p + q];
      w2[a] = s;
    }
  } else if (threadIdx.x == 0) {
    w2[0] = 1.0;
  }
  __syncthreads();
  double* H = scratch + (size_t)t * scratch_per_slot + c.S_off;
  double* Sm = H + (size_t)c.rL * c.rR;
  for (int o = threadIdx.x; o < c.rL * c.rR; o += blockDim.x) {
    const int a = o % c.rL, b = o / c.rL;
    double s = 0;
    for (int k2 = 0; k2 < c.r2; ++k2)
      for (int k1 = 0; k1 < c.r1; ++k1)
        s += core[c.core_off + a + (size_t)c.rL * (k1 + (size_t)c.r1 * (k2 + (size_t)c.r2 * b))] *
             w1[k1] * w2[k2];
    H[o] = s;
  }
  __threadfence_block();
  __syncthreads();
  for (int o = threadIdx.x; o < c.rL * P; o += blockDim.x) {
    const int a = o % c.rL, j = o / c.rL;
    double s = 0;
    for (int b = 0; b < c.rR; ++b) s += H[a + (size_t)c.rL * b] * R[c.R_off + j + (size_t)P * b];
    Sm[o] = s;
  }
  __threadfence_block();
  __syncthreads();
  S* Ct = C + (size_t)t * C_per_slot;
  for (int o = threadIdx.x; o < P * P; o += blockDim.x) {
    const int i = o % P, j = o / P;
    double s = 0;
    for (int a = 0; a < c.rL; ++a) s += L[c.L_off + i + (size_t)P * a] * Sm[a + (size_t)c.rL * j];
    Ct[c.C_off + o] = (S)s;
    if (c.Cm_off >= 0) Ct[c.Cm_off + j + (size_t)P * i] = (S)s;
  }
}

// Near field, one workgroup per (TILE x TILE tile of a stored block, slot):
//   c = core x_theta (Theta_k^T v_k);  D[i + j n_s] = sum_k P[k][i + j n_s] c[k]
// written to D_st and, through an LDS transpose, to D_ts = D_st^T.
template <typename S>
__global__ void __launch_bounds__(NT) k_near_instantiate(
    const NearDev* __restrict__ blocks, const int32_t* __restrict__ tiles,
    const double* __restrict__ Pf, const double* __restrict__ core, const double* __restrict__ th,
    const double* __restrict__ v, S* __restrict__ D, int64_t D_per_slot, int p, int dth) {
  __shared__ double w1[16], w2[16], cc[256];
  __shared__ double tile[TILE][TILE + 1];
  const int32_t bi = tiles[3 * blockIdx.x], i0 = tiles[3 * blockIdx.x + 1], j0 = tiles[3 * blockIdx.x + 2];
  const NearDev b = blocks[bi];
  const int t = blockIdx.y;
  const double* vt = v + (size_t)t * dth * p;
  for (int a = threadIdx.x; a < b.r1; a += blockDim.x) {
    double s = 0;
    for (int q = 0; q < p; ++q) s += th[b.th1_off + q + (size_t)p * a] * vt[q];
    w1[a] = s;
  }
  if (dth == 2) {
    for (int a = threadIdx.x; a < b.r2; a += blockDim.x) {
      double s = 0;
      for (int q = 0; q < p; ++q) s += th[b.th2_off + q + (size_t)p * a] * vt[p + q];
      w2[a] = s;
    }
  } else if (threadIdx.x == 0) {
    w2[0] = 1.0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < b.r_e; k += blockDim.x) {
    double s = 0;
    for (int k2 = 0; k2 < b.r2; ++k2)
      for (int k1 = 0; k1 < b.r1; ++k1)
        s += core[b.core_off + k + (size_t)b.r_e * (k1 + (size_t)b.r1 * k2)] * w1[k1] * w2[k2];
    cc[k] = s;
  }
  __syncthreads();
  const int64_t Ne = (int64_t)b.ns * b.nt;
  S* Dt = D + (size_t)t * D_per_slot;
  const int ti = threadIdx.x % TILE, tj0 = threadIdx.x / TILE;
  const int i = i0 + ti;
  for (int tj = tj0; tj < TILE; tj += NT / TILE) {
    const int j = j0 + tj;
    if (i < b.ns && j < b.nt) {
      const int64_t e = i + (int64_t)j * b.ns;
      const double* pe = Pf + b.P_off + e;
      double s = 0;
      for (int k = 0; k < b.r_e; ++k) s += pe[(size_t)k * Ne] * cc[k];
      Dt[b.D_st + e] = (S)s;
      tile[tj][ti] = s;
    }
  }
  if (b.D_ts < 0) return;
  __syncthreads();
  // transposed block (t, s): element (j, i) at j + i n_t
  const int tj = threadIdx.x % TILE, ti0 = threadIdx.x / TILE;
  const int j = j0 + tj;
  for (int tii = ti0; tii < TILE; tii += NT / TILE) {
    const int ii = i0 + tii;
    if (ii < b.ns && j < b.nt) Dt[b.D_ts + j + (int64_t)ii * b.nt] = (S)tile[tj][tii];
  }
}

template <typename S>
__global__ void k_fill_zero(S* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (S)0;
}

// xt[t][r] = x[perm[t] + r n]
template <typename S>
__global__ void k_perm_in(const S* __restrict__ x, S* __restrict__ xt, const int64_t* __restrict__ perm,
                          int64_t n, int64_t R) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n * R;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = o / R, r = o % R;
    xt[o] = x[perm[t] + r * n];
  }
}

// y[perm[t] + r n] = alpha (yt[t][r] + nugget xt[t][r]) + beta y[...]
template <typename S>
__global__ void k_perm_out(S* __restrict__ y, const S* __restrict__ yt, const S* __restrict__ xt,
                           const int64_t* __restrict__ perm, int64_t n, int64_t R, double alpha,
                           double beta, double nugget) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n * R;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = o / R, r = o % R;
    const int64_t dst = perm[t] + r * n;
    double val = alpha * ((double)yt[o] + nugget * (double)xt[o]);
    if (beta != 0.0) val += beta * (double)y[dst];
    y[dst] = (S)val;
  }
}

// Leaf step of FastForward: x_hat_s[i][r] = sum_{pts} prod_k U_k[pt][i_k] x[pt][r].
template <typename S>
__global__ void __launch_bounds__(NT) k_leaf_up(const S* __restrict__ xt, S* __restrict__ xh,
                                                const double* __restrict__ U,
                                                const int64_t* __restrict__ nbegin,
                                                const int64_t* __restrict__ nend, int32_t leaf0,
                                                int d, int ps, int P, int64_t R) {
  constexpr int CH = 64;
  __shared__ double Us[CH * 3 * 16];
  const int32_t s = leaf0 + blockIdx.x;
  const int64_t b = nbegin[s], e = nend[s];
  const int64_t outs = (int64_t)P * R;
  for (int64_t obase = 0; obase < outs; obase += NT * 8) {
    double acc[8];
    for (int q = 0; q < 8; ++q) acc[q] = 0;
    for (int64_t c0 = b; c0 < e; c0 += CH) {
      const int cn = (int)min<int64_t>(CH, e - c0);
      __syncthreads();
      for (int o = threadIdx.x; o < cn * d * ps; o += NT) Us[o] = U[c0 * d * ps + o];
      __syncthreads();
      for (int q = 0; q < 8; ++q) {
        const int64_t o = obase + threadIdx.x + (int64_t)q * NT;
        if (o >= outs) break;
        const int64_t r = o % R;
        int ii = (int)(o / R);
        int idx[3];
        for (int k = 0; k < d; ++k) { idx[k] = ii % ps; ii /= ps; }
        double a = acc[q];
        for (int pt = 0; pt < cn; ++pt) {
          double u = Us[(pt * d) * ps + idx[0]];
          for (int k = 1; k < d; ++k) u *= Us[(pt * d + k) * ps + idx[k]];
          a += u * (double)xt[(c0 + pt) * R + r];
        }
        acc[q] = a;
      }
    }
    for (int q = 0; q < 8; ++q) {
      const int64_t o = obase + threadIdx.x + (int64_t)q * NT;
      if (o < outs) xh[(size_t)s * outs + o] = (S)acc[q];
    }
  }
}

// E_c[j][i] = prod_k E[h_k][j_k][i_k] with h_k = bit k of the child id.
__device__ inline double transfer_entry(const double* Es, int ps, int d, int cid, int j, int i) {
  double e = 1.0;
  for (int k = 0; k < d; ++k) {
    const int h = (cid >> k) & 1;
    e *= Es[(h * ps + (j % ps)) * ps + (i % ps)];
    j /= ps;
    i /= ps;
  }
  return e;
}

// Inner step of FastForward: x_hat_s = sum_{children c} E_c^T x_hat_c, one workgroup per parent.
template <typename S>
__global__ void __launch_bounds__(NT) k_transfer_up(S* __restrict__ xh, const double* __restrict__ E,
                                                    const int32_t* __restrict__ first_child,
                                                    const int32_t* __restrict__ nchild,
                                                    const int32_t* __restrict__ cid, int32_t node0,
                                                    int d, int ps, int P, int64_t R) {
  __shared__ double Es[2 * 16 * 16];
  for (int o = threadIdx.x; o < 2 * ps * ps; o += NT) Es[o] = E[o];
  __syncthreads();
  const int32_t s = node0 + blockIdx.x;
  const int64_t outs = (int64_t)P * R;
  const int32_t f = first_child[s], nc = nchild[s];
  for (int64_t o = threadIdx.x; o < outs; o += NT) {
    const int64_t r = o % R;
    const int i = (int)(o / R);
    double acc = 0;
    for (int c = 0; c < nc; ++c) {
      const int32_t ch = f + c;
      const int cc = cid[ch];
      const S* xc = xh + (size_t)ch * outs;
      for (int j = 0; j < P; ++j) acc += transfer_entry(Es, ps, d, cc, j, i) * (double)xc[(int64_t)j * R + r];
    }
    xh[(size_t)s * outs + o] = (S)acc;
  }
}

// Coupling: y_hat_s = sum over far blocks (s, t) of C_class x_hat_t, one workgroup per node.
template <typename S>
__global__ void __launch_bounds__(NT) k_coupling(const S* __restrict__ xh, S* __restrict__ yh,
                                                 const S* __restrict__ C,
                                                 const int64_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ ftau,
                                                 const int32_t* __restrict__ fcls, int32_t node0,
                                                 int P, int64_t R) {
  const int32_t s = node0 + blockIdx.x;
  const int64_t b0 = rowptr[s], b1 = rowptr[s + 1];
  if (b0 == b1) return;
  const int64_t outs = (int64_t)P * R;
  for (int64_t o = threadIdx.x; o < outs; o += NT) {
    const int64_t r = o % R;
    const int i = (int)(o / R);
    double acc = 0;
    for (int64_t bb = b0; bb < b1; ++bb) {
      const S* Cc = C + (size_t)fcls[bb] * P * P;
      const S* xt = xh + (size_t)ftau[bb] * outs;
      for (int j = 0; j < P; ++j) acc += (double)Cc[i + (size_t)P * j] * (double)xt[(int64_t)j * R + r];
    }
    yh[(size_t)s * outs + o] = (S)acc;
  }
}

// FastBackward inner step: y_hat_c += E_c y_hat_parent, one workgroup per child.
template <typename S>
__global__ void __launch_bounds__(NT) k_transfer_down(S* __restrict__ yh, const double* __restrict__ E,
                                                      const int32_t* __restrict__ parent_of,
                                                      const int32_t* __restrict__ cid, int32_t node0,
                                                      int d, int ps, int P, int64_t R) {
  __shared__ double Es[2 * 16 * 16];
  for (int o = threadIdx.x; o < 2 * ps * ps; o += NT) Es[o] = E[o];
  __syncthreads();
  const int32_t c = node0 + blockIdx.x;
  const int32_t par = parent_of[c];
  const int cc = cid[c];
  const int64_t outs = (int64_t)P * R;
  const S* yp = yh + (size_t)par * outs;
  for (int64_t o = threadIdx.x; o < outs; o += NT) {
    const int64_t r = o % R;
    const int j = (int)(o / R);
    double acc = (double)yh[(size_t)c * outs + o];
    for (int i = 0; i < P; ++i) acc += transfer_entry(Es, ps, d, cc, j, i) * (double)yp[(int64_t)i * R + r];
    yh[(size_t)c * outs + o] = (S)acc;
  }
}

// Leaf step of FastBackward plus the near field, one workgroup per leaf s:
//   y_s[i][r] = sum_i' U_s[i][i'] y_hat_s[i'][r] + sum_{near t} sum_j D_st[i + j n_s] x_t[j][r]
template <typename S>
__global__ void __launch_bounds__(NT) k_leaf_near(
    const S* __restrict__ xt, S* __restrict__ yt, const S* __restrict__ yh, const S* __restrict__ D,
    const double* __restrict__ U, const int64_t* __restrict__ nbegin, const int64_t* __restrict__ nend,
    const int64_t* __restrict__ rowptr, const int64_t* __restrict__ ntb, const int32_t* __restrict__ nnt,
    const int64_t* __restrict__ nD, int32_t leaf0, int use_far, int d, int ps, int P, int64_t R) {
  const int32_t li = blockIdx.x;
  const int32_t s = leaf0 + li;
  const int64_t b = nbegin[s], ns = nend[s] - b;
  const int64_t outs = ns * R;
  const int64_t pP = (int64_t)P * R;
  for (int64_t o = threadIdx.x; o < outs; o += NT) {
    const int64_t i = o % ns, r = o / ns;
    double acc = 0;
    if (use_far) {
      const double* Ui = U + (b + i) * d * ps;
      for (int ip = 0; ip < P; ++ip) {
        int q = ip;
        double u = 1.0;
        for (int k = 0; k < d; ++k) { u *= Ui[k * ps + q % ps]; q /= ps; }
        acc += u * (double)yh[(size_t)s * pP + (int64_t)ip * R + r];
      }
    }
    for (int64_t bb = rowptr[li]; bb < rowptr[li + 1]; ++bb) {
      const S* Db = D + nD[bb];
      const int64_t tb = ntb[bb];
      const int nt = nnt[bb];
      for (int j = 0; j < nt; ++j) acc += (double)Db[i + (int64_t)j * ns] * (double)xt[(tb + j) * R + r];
    }
    yt[(b + i) * R + r] = (S)acc;
  }
}

// ------------------------------------------------------------------ model upload
static std::shared_ptr<DeviceModel> upload_model(std::shared_ptr<const TreeData> tp, HostModel& hm,
                                                 hipStream_t st) {
  const TreeData& t = *tp;
  auto m = std::make_shared<DeviceModel>();
  m->tree = tp;
  m->d = hm.d; m->p_s = hm.p_s; m->P = hm.P; m->p_theta = hm.p_theta; m->d_theta = hm.d_theta;
  m->l_max = t.l_max; m->min_far = t.min_far_level;
  for (int k = 0; k < 2; ++k) { m->th_lo[k] = hm.th_lo[k]; m->th_hi[k] = hm.th_hi[k]; }
  m->n = t.n; m->n_nodes = t.n_nodes(); m->n_leaves = (int64_t)t.leaves.size();
  m->n_near = t.n_near(); m->n_classes = t.n_classes(); m->N_nf = t.near_entries;
  m->n_stored_near = (int64_t)hm.nstore.size();
  m->n_stored_cls = (int64_t)hm.cstore.size();
  m->kernel_evals = hm.kernel_evals;
  m->near_factor_entries = hm.near_factor_entries;

  // canonical near D offsets
  m->D_off_host.assign(m->n_near + 1, 0);
  for (int64_t b = 0; b < m->n_near; ++b)
    m->D_off_host[b + 1] = m->D_off_host[b] + t.size(t.near[2 * b]) * t.size(t.near[2 * b + 1]);

  // near stored blocks and tiles
  std::vector<NearDev> nd(hm.nstore.size());
  std::vector<int32_t> tiles;
  m->near_rank_canon.assign(m->n_near, -1);
  double wsum = 0, rsum = 0;
  for (size_t q = 0; q < hm.nstore.size(); ++q) {
    const NearStored& s = hm.nstore[q];
    NearDev& x = nd[q];
    x.s_begin = s.s_begin; x.t_begin = s.t_begin;
    x.P_off = s.P_off; x.core_off = s.core_off; x.th1_off = s.th1_off; x.th2_off = s.th2_off;
    x.D_st = m->D_off_host[s.b_st];
    x.D_ts = s.b_ts >= 0 ? m->D_off_host[s.b_ts] : -1;
    x.ns = s.ns; x.nt = s.nt; x.r_e = s.r_e; x.r1 = s.r1; x.r2 = s.r2; x.pad = 0;
    m->near_rank_canon[s.b_st] = s.r_e;
    const double w = (double)s.ns * s.nt * (s.b_ts >= 0 ? 2 : 1);
    wsum += w;
    rsum += w * s.r_e;
    m->near_rank_max = std::max(m->near_rank_max, s.r_e);
    for (int32_t j0 = 0; j0 < s.nt; j0 += TILE)
      for (int32_t i0 = 0; i0 < s.ns; i0 += TILE) {
        tiles.push_back((int32_t)q);
        tiles.push_back(i0);
        tiles.push_back(j0);
      }
  }
  m->near_rank_mean = wsum > 0 ? rsum / wsum : 0;
  m->n_tiles = (int64_t)tiles.size() / 3;

  // far classes
  const int P = hm.P;
  std::vector<ClassDev> cd(hm.cstore.size());
  int64_t soff = 0;
  double fr = 0;
  m->class_ranks.assign(m->n_classes * (2 + hm.d_theta), 0);
  for (size_t q = 0; q < hm.cstore.size(); ++q) {
    const ClassStored& c = hm.cstore[q];
    ClassDev& x = cd[q];
    x.L_off = c.L_off; x.R_off = c.R_off; x.core_off = c.core_off;
    x.th1_off = c.th1_off; x.th2_off = c.th2_off;
    x.C_off = (int64_t)c.cls * P * P;
    x.Cm_off = c.mirror >= 0 ? (int64_t)c.mirror * P * P : -1;
    x.S_off = soff;
    soff += (int64_t)c.rL * c.rR + (int64_t)c.rL * P;
    x.rL = c.rL; x.r1 = c.r1; x.r2 = c.r2; x.rR = c.rR;
    fr += 0.5 * (c.rL + c.rR);
    m->far_rank_max = std::max({m->far_rank_max, c.rL, c.rR});
    int32_t* cr = &m->class_ranks[(size_t)c.cls * (2 + hm.d_theta)];
    cr[0] = c.rL; cr[1] = c.r1; if (hm.d_theta == 2) cr[2] = c.r2; cr[1 + hm.d_theta] = c.rR;
    if (c.mirror >= 0) {
      int32_t* mr = &m->class_ranks[(size_t)c.mirror * (2 + hm.d_theta)];
      mr[0] = c.rR; mr[1] = c.r1; if (hm.d_theta == 2) mr[2] = c.r2; mr[1 + hm.d_theta] = c.rL;
    }
  }
  m->far_rank_mean = cd.empty() ? 0 : fr / cd.size();
  m->ff_scratch = soff;

  // CSR of near blocks by target leaf (canonical list is sorted by sigma)
  const int32_t leaf0 = t.leaves.empty() ? 0 : t.leaves.front();
  std::vector<int64_t> nrow(m->n_leaves + 1, 0), ntb(m->n_near), nD(m->n_near);
  std::vector<int32_t> nnt(m->n_near);
  for (int64_t b = 0; b < m->n_near; ++b) {
    const int32_t s = t.near[2 * b], u = t.near[2 * b + 1];
    nrow[s - leaf0 + 1]++;
    ntb[b] = t.begin[u];
    nnt[b] = (int32_t)t.size(u);
    nD[b] = m->D_off_host[b];
  }
  for (int64_t i = 0; i < m->n_leaves; ++i) nrow[i + 1] += nrow[i];
  // CSR of far blocks by target node
  std::vector<int64_t> frow(m->n_nodes + 1, 0);
  std::vector<int32_t> ftau(t.n_far()), fcls(t.n_far());
  for (int64_t b = 0; b < t.n_far(); ++b) {
    frow[t.far[2 * b] + 1]++;
    ftau[b] = t.far[2 * b + 1];
    fcls[b] = t.far_class[b];
  }
  for (int64_t i = 0; i < m->n_nodes; ++i) frow[i + 1] += frow[i];

  m->U.upload(hm.U.data(), hm.U.size(), st);
  m->E.upload(hm.E.data(), hm.E.size(), st);
  m->perm.upload(t.perm.data(), t.perm.size(), st);
  m->first_child.upload(t.first_child.data(), t.first_child.size(), st);
  m->nchild.upload(t.nchild.data(), t.nchild.size(), st);
  m->cid.upload(t.cid.data(), t.cid.size(), st);
  m->parent.upload(t.parent.data(), t.parent.size(), st);
  m->nbegin.upload(t.begin.data(), t.begin.size(), st);
  m->nend.upload(t.end.data(), t.end.size(), st);
  m->nstore.upload(nd.data(), nd.size(), st);
  m->nf_P.upload(hm.nf_P.data(), hm.nf_P.size(), st);
  m->nf_core.upload(hm.nf_core.data(), hm.nf_core.size(), st);
  m->nf_theta.upload(hm.nf_theta.data(), hm.nf_theta.size(), st);
  m->tiles.upload(tiles.data(), tiles.size(), st);
  m->near_rowptr.upload(nrow.data(), nrow.size(), st);
  m->near_tb.upload(ntb.data(), ntb.size(), st);
  m->near_D.upload(nD.data(), nD.size(), st);
  m->near_nt.upload(nnt.data(), nnt.size(), st);
  m->cstore.upload(cd.data(), cd.size(), st);
  m->ff_L.upload(hm.ff_L.data(), hm.ff_L.size(), st);
  m->ff_R.upload(hm.ff_R.data(), hm.ff_R.size(), st);
  m->ff_core.upload(hm.ff_core.data(), hm.ff_core.size(), st);
  m->ff_theta.upload(hm.ff_theta.data(), hm.ff_theta.size(), st);
  m->far_rowptr.upload(frow.data(), frow.size(), st);
  m->far_tau.upload(ftau.data(), ftau.size(), st);
  m->far_cls.upload(fcls.data(), fcls.size(), st);
  PH_HIP(hipStreamSynchronize(st));  // host staging buffers die with this call
  m->device_bytes = (int64_t)(m->U.bytes() + m->E.bytes() + m->perm.bytes() + m->first_child.bytes() +
                              m->nchild.bytes() + m->cid.bytes() + m->parent.bytes() + m->nbegin.bytes() + m->nend.bytes() +
                              m->nstore.bytes() + m->nf_P.bytes() + m->nf_core.bytes() +
                              m->nf_theta.bytes() + m->tiles.bytes() + m->near_rowptr.bytes() +
                              m->near_tb.bytes() + m->near_D.bytes() + m->near_nt.bytes() +
                              m->cstore.bytes() + m->ff_L.bytes() + m->ff_R.bytes() +
                              m->ff_core.bytes() + m->ff_theta.bytes() + m->far_rowptr.bytes() +
                              m->far_tau.bytes() + m->far_cls.bytes());
  return m;
}

// ------------------------------------------------------------------ online stage
static int64_t grid_for(int64_t work) { return std::max<int64_t>(1, std::min<int64_t>((work + NT - 1) / NT, 65536)); }

template <typename S>
static void instantiate_impl(InstData& in, const double* theta, hipStream_t st) {
  const DeviceModel& m = *in.m;
  for (int t0 = 0; t0 < in.T; t0 += MAXT) {
    ThetaPack tp{};
    tp.count = std::min(MAXT, in.T - t0);
    tp.dth = m.d_theta;
    tp.p = m.p_theta;
    tp.grad_dim = in.grad_dim;
    for (int k = 0; k < 2; ++k) { tp.lo[k] = m.th_lo[k]; tp.hi[k] = m.th_hi[k]; }
    for (int t = 0; t < tp.count; ++t)
      for (int k = 0; k < m.d_theta; ++k) tp.th[t * 2 + k] = theta[(size_t)(t0 + t) * m.d_theta + k];
    launch(PH_STAGE_THETA, k_theta_vectors, dim3(1), dim3(NT), st, tp, in.v.p, t0);
  }
  const int64_t Cps = m.n_classes * m.P * m.P;
  if (m.n_stored_cls > 0)
    launch(PH_STAGE_FAR_INST, k_far_instantiate<S>, dim3((unsigned)m.n_stored_cls, in.T), dim3(NT), st,
                       m.cstore.p, m.ff_L.p, m.ff_R.p, m.ff_core.p, m.ff_theta.p, in.v.p, in.ffs.p,
                       m.ff_scratch, (S*)in.C.p, Cps, m.P, m.p_theta, m.d_theta);
  if (m.n_tiles > 0)
    launch(PH_STAGE_NEAR_INST, k_near_instantiate<S>, dim3((unsigned)m.n_tiles, in.T), dim3(NT), st,
                       m.nstore.p, m.tiles.p, m.nf_P.p, m.nf_core.p, m.nf_theta.p, in.v.p, (S*)in.D.p,
                       m.N_nf, m.p_theta, m.d_theta);
  PH_HIP(hipGetLastError());
}

template <typename S>
static void matvec_impl(InstData& in, const S* x, S* y, int64_t R, double alpha, double beta,
                        double nugget, hipStream_t st) {
  const DeviceModel& m = *in.m;
  const TreeData& t = *m.tree;
  if (R > in.Rcap) {
    in.xt.alloc((size_t)m.n * R * sizeof(S));
    in.yt.alloc((size_t)m.n * R * sizeof(S));
    in.xh.alloc((size_t)m.n_nodes * m.P * R * sizeof(S));
    in.yh.alloc((size_t)m.n_nodes * m.P * R * sizeof(S));
    in.Rcap = R;
  }
  S* xt = (S*)in.xt.p;
  S* yt = (S*)in.yt.p;
  S* xh = (S*)in.xh.p;
  S* yh = (S*)in.yh.p;
  const int32_t leaf0 = t.leaves.front();
  const int64_t Cps = m.n_classes * m.P * m.P;
  const bool use_far = m.min_far >= 0;
  for (int slot = 0; slot < in.T; ++slot) {
    const S* xs = x + (size_t)slot * m.n * R;
    S* ys = y + (size_t)slot * m.n * R;
    const S* Ds = (const S*)in.D.p + (size_t)slot * m.N_nf;
    const S* Cs = (const S*)in.C.p + (size_t)slot * Cps;
    launch(PH_STAGE_PERM_IN, k_perm_in<S>, dim3((unsigned)grid_for(m.n * R)), dim3(NT), st, xs, xt, m.perm.p,
                       m.n, R);
    if (use_far) {
      launch(PH_STAGE_LEAF_UP, k_leaf_up<S>, dim3((unsigned)m.n_leaves), dim3(NT), st, xt, xh, m.U.p,
                         m.nbegin.p, m.nend.p, leaf0, m.d, m.p_s, m.P, R);
      for (int l = m.l_max - 1; l >= m.min_far; --l) {
        const int32_t a = t.level_start[l], b = t.level_start[l + 1];
        launch(PH_STAGE_TRANSFER_UP, k_transfer_up<S>, dim3((unsigned)(b - a)), dim3(NT), st, xh, m.E.p,
                           m.first_child.p, m.nchild.p, m.cid.p, a, m.d, m.p_s, m.P, R);
      }
      const int32_t a0 = t.level_start[m.min_far];
      const int64_t nn = m.n_nodes - a0;
      launch(PH_STAGE_ZERO, k_fill_zero<S>, dim3((unsigned)grid_for(nn * m.P * R)), dim3(NT), st,
                         yh + (size_t)a0 * m.P * R, nn * m.P * R);
      launch(PH_STAGE_COUPLING, k_coupling<S>, dim3((unsigned)nn), dim3(NT), st, xh, yh, Cs, m.far_rowptr.p,
                         m.far_tau.p, m.far_cls.p, a0, m.P, R);
      for (int l = m.min_far; l < m.l_max; ++l) {
        const int32_t a = t.level_start[l + 1], b = t.level_start[l + 2];
        launch(PH_STAGE_TRANSFER_DOWN, k_transfer_down<S>, dim3((unsigned)(b - a)), dim3(NT), st, yh, m.E.p,
                           m.parent.p, m.cid.p, a, m.d, m.p_s, m.P, R);
      }
    }
    launch(PH_STAGE_LEAF_NEAR, k_leaf_near<S>, dim3((unsigned)m.n_leaves), dim3(NT), st, xt, yt, yh, Ds, m.U.p,
                       m.nbegin.p, m.nend.p, m.near_rowptr.p, m.near_tb.p, m.near_nt.p, m.near_D.p, leaf0,
                       use_far ? 1 : 0, m.d, m.p_s, m.P, R);
    launch(PH_STAGE_PERM_OUT, k_perm_out<S>, dim3((unsigned)grid_for(m.n * R)), dim3(NT), st, ys, yt, xt,
                       m.perm.p, m.n, R, alpha, beta, nugget);
  }
  PH_HIP(hipGetLastError());
}

}  // namespace ph

// ====================================================================== C ABI
struct ph_tree {
  std::shared_ptr<const ph::TreeData> p;
};
struct ph_model {
  std::shared_ptr<const ph::DeviceModel> p;
};
struct ph_inst {
  std::shared_ptr<ph::InstData> p;
};

namespace {

template <typename F>
int guarded(F&& f) {
  try {
    ph::g_last_error.clear();
    f();
    return PH_OK;
  } catch (const ph::Failure& e) {
    ph::g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    ph::g_last_error = "host allocation failed";
    return PH_ENOMEM;
  } catch (const std::exception& e) {
    ph::g_last_error = e.what();
    return PH_EINVAL;
  } catch (...) {
    ph::g_last_error = "unknown failure";
    return PH_EINVAL;
  }
}

void need(bool ok, const char* msg) {
  if (!ok) ph::fail(PH_EINVAL, msg);
}

int inst_common(const ph_model* m, const double* theta, int T, int dim, ph_dtype dt, void* stream,
                ph_inst** inout) {
  return guarded([&] {
    need(m && m->p, "model is NULL");
    need(theta != nullptr, "theta is NULL");
    need(inout != nullptr, "inout is NULL");
    need(T >= 1, "T must be >= 1");
    need(dt == PH_F64 || dt == PH_F32, "dtype must be PH_F64 or PH_F32");
    const ph::DeviceModel& md = *m->p;
    if (dim >= 0) need(dim < md.d_theta, "gradient dimension out of range");
    for (int t = 0; t < T; ++t)
      for (int k = 0; k < md.d_theta; ++k) {
        const double v = theta[(size_t)t * md.d_theta + k];
        if (!(v >= md.th_lo[k] && v <= md.th_hi[k]))
          ph::fail(PH_EDOMAIN, "theta outside the parameter box");
      }
    hipStream_t st = (hipStream_t)stream;
    std::shared_ptr<ph::InstData> in;
    if (*inout) {
      in = (*inout)->p;
      need(in && in->m.get() == &md && in->T == T && in->dt == dt,
           "instance does not match (model, T, dtype)");
      in->grad_dim = dim;
    } else {
      in = std::make_shared<ph::InstData>();
      in->m = m->p;
      in->T = T;
      in->dt = dt;
      in->grad_dim = dim;
      in->esize = dt == PH_F64 ? sizeof(double) : sizeof(float);
      in->D.alloc((size_t)T * md.N_nf * in->esize);
      in->C.alloc((size_t)T * md.n_classes * md.P * md.P * in->esize);
      in->v.alloc((size_t)T * md.d_theta * md.p_theta);
      in->ffs.alloc((size_t)T * std::max<int64_t>(md.ff_scratch, 1));
    }
    if (dt == PH_F64) ph::instantiate_impl<double>(*in, theta, st);
    else ph::instantiate_impl<float>(*in, theta, st);
    if (!*inout) *inout = new ph_inst{in};
  });
}

}  // namespace

extern "C" {

const char* ph_last_error(void) { return ph::g_last_error.c_str(); }

const char* ph_version(void) { return "ph-mi355x 0.1 (gfx950)"; }

int ph_build_tree(const double* pts, int64_t n, const ph_tree_opts* opts, ph_tree** out) {
  return guarded([&] {
    need(opts != nullptr && out != nullptr, "opts or out is NULL");
    auto t = ph::build_tree(pts, n, *opts);
    *out = new ph_tree{t};
  });
}

int ph_tree_info_get(const ph_tree* t, ph_tree_info* info) {
  return guarded([&] {
    need(t && t->p && info, "NULL argument");
    const ph::TreeData& d = *t->p;
    info->n = d.n;
    info->d = d.d;
    info->l_max = d.l_max;
    info->n_nodes = d.n_nodes();
    info->n_leaves = (int64_t)d.leaves.size();
    info->n_near = d.n_near();
    info->n_far = d.n_far();
    info->n_classes = d.n_classes();
    info->near_entries = d.near_entries;
    info->min_far_level = d.min_far_level;
  });
}

int ph_tree_perm(const ph_tree* t, int64_t* perm) {
  return guarded([&] {
    need(t && t->p && perm, "NULL argument");
    std::memcpy(perm, t->p->perm.data(), t->p->perm.size() * sizeof(int64_t));
  });
}

int ph_tree_nodes(const ph_tree* t, int32_t* level, int32_t* coords, int64_t* begin, int64_t* end,
                  int32_t* parent) {
  return guarded([&] {
    need(t && t->p, "NULL tree");
    const ph::TreeData& d = *t->p;
    const size_t nn = (size_t)d.n_nodes();
    if (level) std::memcpy(level, d.level.data(), nn * sizeof(int32_t));
    if (coords) std::memcpy(coords, d.coords.data(), nn * d.d * sizeof(int32_t));
    if (begin) std::memcpy(begin, d.begin.data(), nn * sizeof(int64_t));
    if (end) std::memcpy(end, d.end.data(), nn * sizeof(int64_t));
    if (parent) std::memcpy(parent, d.parent.data(), nn * sizeof(int32_t));
  });
}

int ph_tree_blocks(const ph_tree* t, int32_t* near, int32_t* far, int32_t* far_class) {
  return guarded([&] {
    need(t && t->p, "NULL tree");
    const ph::TreeData& d = *t->p;
    if (near) std::memcpy(near, d.near.data(), d.near.size() * sizeof(int32_t));
    if (far) std::memcpy(far, d.far.data(), d.far.size() * sizeof(int32_t));
    if (far_class) std::memcpy(far_class, d.far_class.data(), d.far_class.size() * sizeof(int32_t));
  });
}

int ph_tree_classes(const ph_tree* t, int32_t* level, int32_t* offset) {
  return guarded([&] {
    need(t && t->p, "NULL tree");
    const ph::TreeData& d = *t->p;
    if (level) std::memcpy(level, d.class_level.data(), d.class_level.size() * sizeof(int32_t));
    if (offset) std::memcpy(offset, d.class_off.data(), d.class_off.size() * sizeof(int32_t));
  });
}

void ph_tree_free(ph_tree* t) { delete t; }

int ph_offline_compress(const ph_tree* t, const ph_offline_opts* opts, void* stream, ph_model** out) {
  return guarded([&] {
    need(t && t->p && opts && out, "NULL argument");
    auto hm = ph::offline_host(*t->p, *opts);
    auto dm = ph::upload_model(t->p, *hm, (hipStream_t)stream);
    *out = new ph_model{dm};
  });
}

int ph_model_info_get(const ph_model* m, ph_model_info* info) {
  return guarded([&] {
    need(m && m->p && info, "NULL argument");
    const ph::DeviceModel& d = *m->p;
    info->n = d.n;
    info->n_near_stored = d.n_stored_near;
    info->n_classes_stored = d.n_stored_cls;
    info->near_entries = d.N_nf;
    info->near_factor_entries = d.near_factor_entries;
    info->near_rank_mean = d.near_rank_mean;
    info->near_rank_max = d.near_rank_max;
    info->far_rank_mean = d.far_rank_mean;
    info->far_rank_max = d.far_rank_max;
    info->device_bytes = d.device_bytes;
    info->kernel_evals = d.kernel_evals;
    info->P = d.P;
    info->p_theta = d.p_theta;
    info->d_theta = d.d_theta;
  });
}

int ph_model_near_ranks(const ph_model* m, int32_t* ranks) {
  return guarded([&] {
    need(m && m->p && ranks, "NULL argument");
    std::memcpy(ranks, m->p->near_rank_canon.data(), m->p->near_rank_canon.size() * sizeof(int32_t));
  });
}

int ph_model_class_ranks(const ph_model* m, int32_t* ranks) {
  return guarded([&] {
    need(m && m->p && ranks, "NULL argument");
    std::memcpy(ranks, m->p->class_ranks.data(), m->p->class_ranks.size() * sizeof(int32_t));
  });
}

void ph_model_free(ph_model* m) { delete m; }

int ph_instantiate(const ph_model* m, const double* theta, int T, ph_dtype dt, void* stream,
                   ph_inst** inout) {
  return inst_common(m, theta, T, -1, dt, stream, inout);
}

int ph_instantiate_grad(const ph_model* m, const double* theta, int T, int dim, ph_dtype dt, void* stream,
                        ph_inst** inout) {
  if (dim < 0) {
    ph::g_last_error = "gradient dimension out of range";
    return PH_EINVAL;
  }
  return inst_common(m, theta, T, dim, dt, stream, inout);
}

int ph_matvec(ph_inst* k, const void* x, void* y, int64_t R, double alpha, double beta, double nugget,
              void* stream) {
  return guarded([&] {
    need(k && k->p, "instance is NULL");
    need(R >= 0, "R must be >= 0");
    if (R == 0) return;
    need(x && y, "x or y is NULL");
    ph::InstData& in = *k->p;
    hipStream_t st = (hipStream_t)stream;
    if (in.dt == PH_F64)
      ph::matvec_impl<double>(in, (const double*)x, (double*)y, R, alpha, beta, nugget, st);
    else
      ph::matvec_impl<float>(in, (const float*)x, (float*)y, R, alpha, beta, nugget, st);
  });
}

int ph_inst_near_block(const ph_inst* k, int t, int64_t b, double* host_out) {
  return guarded([&] {
    need(k && k->p && host_out, "NULL argument");
    const ph::InstData& in = *k->p;
    const ph::DeviceModel& m = *in.m;
    need(t >= 0 && t < in.T, "slot out of range");
    need(b >= 0 && b < m.n_near, "near block index out of range");
    const int64_t off = m.D_off_host[b], cnt = m.D_off_host[b + 1] - off;
    PH_HIP(hipDeviceSynchronize());
    std::vector<char> buf(cnt * in.esize);
    PH_HIP(hipMemcpy(buf.data(), in.D.p + ((size_t)t * m.N_nf + off) * in.esize, buf.size(),
                     hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < cnt; ++i)
      host_out[i] = in.dt == PH_F64 ? ((double*)buf.data())[i] : (double)((float*)buf.data())[i];
  });
}

int ph_inst_coupling(const ph_inst* k, int t, int64_t c, double* host_out) {
  return guarded([&] {
    need(k && k->p && host_out, "NULL argument");
    const ph::InstData& in = *k->p;
    const ph::DeviceModel& m = *in.m;
    need(t >= 0 && t < in.T, "slot out of range");
    need(c >= 0 && c < m.n_classes, "class index out of range");
    const int64_t cnt = (int64_t)m.P * m.P;
    PH_HIP(hipDeviceSynchronize());
    std::vector<char> buf(cnt * in.esize);
    PH_HIP(hipMemcpy(buf.data(), in.C.p + ((size_t)t * m.n_classes * cnt + c * cnt) * in.esize, buf.size(),
                     hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < cnt; ++i)
      host_out[i] = in.dt == PH_F64 ? ((double*)buf.data())[i] : (double)((float*)buf.data())[i];
  });
}

void ph_inst_free(ph_inst* k) { delete k; }

int ph_trace_enable(int on) {
  return guarded([&] {
    std::lock_guard<std::mutex> lk(ph::g_trace_mu);
    ph::g_trace_on = on != 0;
  });
}

int ph_trace_read(ph_trace_stats* out, int reset) {
  return guarded([&] {
    need(out != nullptr, "out is NULL");
    std::lock_guard<std::mutex> lk(ph::g_trace_mu);
    for (int i = 0; i < PH_NUM_STAGES; ++i) {
      out->ms[i] = 0;
      out->count[i] = 0;
    }
    for (auto& r : ph::g_trace_recs) {
      PH_HIP(hipEventSynchronize(r.b));
      float ms = 0;
      PH_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      out->ms[r.stage] += ms;
      out->count[r.stage] += 1;
    }
    if (reset) {
      for (auto& r : ph::g_trace_recs) {
        ph::g_event_pool.push_back(r.a);
        ph::g_event_pool.push_back(r.b);
      }
      ph::g_trace_recs.clear();
    }
  });
}

}  // extern "C"
