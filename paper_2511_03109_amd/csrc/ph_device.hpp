// Device-side data structures shared by the HIP translation units of the library:
// device arrays, the uploaded model, an instance, per-kernel event tracing and the
// CDNA4 matrix-core (MFMA) helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ph_host.hpp"

#define PH_HIP(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) ::ph::fail(PH_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace ph {

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

// per stored near block (s <= t)
struct NearDev {
  int64_t s_begin, t_begin, P_off, core_off, th1_off, th2_off, D_st, D_ts;
  int32_t ns, nt, r_e, r1, r2, pad;
};

// per stored far class (offset >= 0 lexicographically)
struct ClassDev {
  int64_t L_off, R_off, core_off, th1_off, th2_off, C_off, Cm_off, S_off;
  int32_t rL, r1, r2, rR;
};

constexpr int NT = 256;    // threads per workgroup (4 wavefronts of 64)
constexpr int WAVE = 64;
constexpr int TILE = 32;   // near-field instantiation tile edge
constexpr int TC = 8;      // parameter slots processed together by the near-field kernel
constexpr int MAXT = 64;   // parameter values per theta-vector launch
constexpr int RC = 16;     // right-hand sides per MFMA column tile

struct DeviceModel {
  std::shared_ptr<const TreeData> tree;
  int d = 0, p_s = 0, P = 0, Pp = 0, p_theta = 0, d_theta = 0, l_max = 0, min_far = -1, nsib = 0;
  double th_lo[2] = {0, 0}, th_hi[2] = {0, 0};
  int64_t n = 0, n_nodes = 0, n_leaves = 0, n_near = 0, n_classes = 0, N_nf = 0;
  int64_t n_stored_near = 0, n_stored_cls = 0, n_tiles = 0, ff_scratch = 0;
  int64_t n_groups = 0, n_entries = 0, max_group_entries = 0;
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
  // coupling work list: sibling groups (children of one parent at levels >= min_far)
  DevArr<int32_t> grp_targets;            // n_groups x nsib node ids (-1 = absent)
  DevArr<int32_t> grp_entry;              // n_groups + 1
  DevArr<int32_t> ent_cls;                // per entry: class
  DevArr<int32_t> ent_tau;                // per entry: nsib source nodes (-1 = sibling unused)
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
  int Gcap = 0;
  DevArr<char> xt, yt, xh, yh, part;
};

template <typename S>
void instantiate_impl(InstData& in, const double* theta, hipStream_t st);
template <typename S>
void matvec_impl(InstData& in, const S* x, S* y, int64_t R, double alpha, double beta, double nugget,
                 hipStream_t st);

// ---- per-kernel timing with HIP events
struct TraceRec {
  int stage;
  hipEvent_t a, b;
};
extern std::mutex g_trace_mu;
extern bool g_trace_on;
extern std::vector<TraceRec> g_trace_recs;
hipEvent_t pooled_event();  // caller holds g_trace_mu

// Launch a kernel on stream st; when tracing, bracket it with events tagged by stage.
template <typename K, typename... Args>
inline void launch(int stage, K kernel, dim3 grid, dim3 block, hipStream_t st, Args... args) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return;
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

// ---- matrix cores: one wavefront computes a 16 x 16 tile += (16 x 4) (4 x 16).
// Operand layout (both types): lane l holds A[m = l % 16][k = l / 16] and
// B[k = l / 16][n = l % 16].  Result element i of lane l sits at column l % 16 and
// row (l / 16) + 4 i for FP64, row 4 (l / 16) + i for FP32 (checked on gfx950).
template <typename S>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

inline int64_t grid_for(int64_t work) {
  int64_t g = (work + NT - 1) / NT;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return g;
}

}  // namespace ph
