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

// BF16 storage (1 sign, 8 exponent, 7 fraction bits): the upper half of an FP32 value.
// Conversion rounds to nearest, ties to even (NaN stays NaN); widening is exact.
struct bf16 {
  uint16_t bits;
};
__host__ __device__ inline bf16 to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{(uint16_t)((u >> 16) | 0x40)};   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16{(uint16_t)(u >> 16)};
}
__host__ __device__ inline float from_bf16(bf16 h) {
  const uint32_t u = (uint32_t)h.bits << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
// storage of a computed value (double accumulator) and its widening for arithmetic
template <typename DT>
__host__ __device__ inline DT to_store(double x) { return (DT)x; }
template <>
__host__ __device__ inline bf16 to_store<bf16>(double x) { return to_bf16((float)x); }
template <typename S, typename DT>
__host__ __device__ inline S widen(DT x) { return (S)x; }
template <>
__host__ __device__ inline float widen<float, bf16>(bf16 x) { return from_bf16(x); }

// Near-field blocks are stored once per pair (s <= t).  An instantiated block D (n_s x n_t)
// is kept in 16-row panels: entry (i, j) at (i / 16) * 16 n_t + i % 16 + 16 j, rows
// padded to a multiple of 16 with zeros, so every 16 x 16 tile is one contiguous 2 KB
// chunk whichever way the MVM reads it (D_st x_t for s, D_st^T x_s for t).
__host__ __device__ inline int64_t panel_index(int64_t i, int64_t j, int64_t ncols) {
  return (i >> 4) * 16 * ncols + (i & 15) + 16 * j;
}

// Four consecutive stored values (aligned to 4 elements), widened to the compute type.
template <typename S, typename DT>
struct Load4;
template <>
struct Load4<double, double> {
  static __device__ __forceinline__ void get(const double* p, double* o) {
    typedef double v4 __attribute__((ext_vector_type(4)));
    const v4 v = *reinterpret_cast<const v4*>(p);
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
  }
};
template <>
struct Load4<float, float> {
  static __device__ __forceinline__ void get(const float* p, float* o) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = *reinterpret_cast<const v4*>(p);
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
  }
};
template <>
struct Load4<float, bf16> {
  static __device__ __forceinline__ void get(const bf16* p, float* o) {
    typedef unsigned short v4 __attribute__((ext_vector_type(4)));
    const v4 v = *reinterpret_cast<const v4*>(p);
    o[0] = from_bf16(bf16{v[0]}); o[1] = from_bf16(bf16{v[1]});
    o[2] = from_bf16(bf16{v[2]}); o[3] = from_bf16(bf16{v[3]});
  }
};

// per stored near block (s <= t); ldp: leading dimension of the stored factor columns
struct NearDev {
  int64_t s_begin, t_begin, P_off, core_off, th1_off, th2_off, D_st;
  int32_t ns, nt, r_e, r1, r2, ldp;
};

// per stored far class (offset >= 0 lexicographically)
struct ClassDev {
  int64_t chat_off, th1_off, th2_off, C_off, Cm_off;   // chat_off: panels in fragment order
  int32_t rL, r1, r2, rR;
};

constexpr int NT = 256;    // threads per workgroup (4 wavefronts of 64)
constexpr int WAVE = 64;
constexpr int TILE = 32;   // near-field instantiation tile: rows
constexpr int TILE_J = 16; // near-field instantiation tile: columns
constexpr int TC = 8;      // parameter slots processed together by the near-field kernel
constexpr int MAXT = 64;   // parameter values per theta-vector launch
constexpr int RC = 16;     // right-hand sides per MFMA column tile
constexpr int NTG = 16;    // coupling targets per work group (one box of nodes of a level)

// Parametric H-matrix format: a far block (explicit factors S_b, T_b) and a stored class (its
// core, theta factors and the offset of H_q(theta) in the instance's far buffer).
struct HBlkDev {
  int64_t s_begin, t_begin, S_off, T_off, h_off, w_off;
  int32_t ns, nt, rs, rt, lds, ldt, tr, q;
};
struct HClsDev {
  int64_t core_off, th1_off, th2_off, h_off;
  int32_t rL, r1, r2, rR;
};

struct DeviceModel {
  std::shared_ptr<const TreeData> tree;
  int d = 0, p_s = 0, P = 0, Pp = 0, p_theta = 0, d_theta = 0, l_max = 0, min_far = -1;
  double th_lo[2] = {0, 0}, th_hi[2] = {0, 0};
  int64_t n = 0, n_nodes = 0, n_leaves = 0, n_near = 0, n_classes = 0, N_nf = 0, N_nf_pad = 0;
  int64_t n_stored_near = 0, n_stored_cls = 0, n_tiles = 0;
  int64_t n_groups = 0, n_entries = 0, max_group_entries = 0;
  int64_t near_factor_entries = 0, kernel_evals = 0;
  double near_rank_mean = 0, far_rank_mean = 0;
  int near_rank_max = 0, far_rank_max = 0;
  int svd_sweeps_max = 0;
  std::vector<int32_t> near_rank_canon;   // per canonical near block (-1 if transposed copy)
  std::vector<int32_t> class_ranks;       // per class, 2 + d_theta entries
  std::vector<int64_t> D_off_host;        // per canonical near block: offset of its stored block
  std::vector<int32_t> D_tr_host;         // per canonical near block: 1 if stored as its transpose
  std::vector<int32_t> near_src_host;     // per canonical near block: its stored block
  // device arrays
  DevArr<double> U, E;
  DevArr<int64_t> perm, iperm;            // tree position -> point, point -> tree position
  DevArr<int32_t> first_child, nchild, cid, parent;
  DevArr<int64_t> nbegin, nend;
  DevArr<NearDev> nstore;
  DevArr<double> nf_P, nf_core, nf_theta;
  DevArr<int32_t> tiles;                  // 3 per tile: stored block, i0, j0
  DevArr<int64_t> near_rowptr;            // per leaf index
  DevArr<int64_t> near_tb, near_D;        // per canonical near block: tau begin, stored D offset
  DevArr<int32_t> near_nt, near_tr;       // per canonical near block: n_tau, stored transposed
  // single right-hand side (read-once near MVM): per leaf s, its stored blocks D_st (t >= s,
  // ascending t) and the pair buffers z_ut = D_ut^T x_u (u < t) that it gathers; Zt = rows
  // of all pair buffers
  DevArr<int64_t> up_rowptr, up_tb, up_D, up_z;   // up_z: first row of z_st (-1: t = s)
  DevArr<int32_t> up_nt;
  DevArr<int64_t> lo_rowptr, lo_z;
  int64_t Zt = 0;
  int near_xcd = 0;   // near MVM: contiguous leaf ranges per XCD (only if they balance)
  DevArr<int32_t> mvm_items;   // near MVM and leaf-down work items: (leaf index, first row of a 128-row chunk)
  int64_t n_mvm_items = 0;
  DevArr<int32_t> mvm_items64; // the same with 64-row chunks (factored near MVM, one row tile per wave)
  int64_t n_mvm_items64 = 0;
  DevArr<int32_t> near_q;      // per canonical near block (list order of near_rowptr): its stored block
  int KRp = 4;                 // largest near rank rounded up to 4 (to 16 above 16)
  int KM = 4;                  // rank chunk of the factored near MVM: KRp up to 16, else 16
  int64_t max_Nep = 0;         // largest padded factor column (ldp n_t) of a stored near block
  // near factors in the storage type of a factored instance: FP64 as compressed, FP32 and
  // BF16 copies made on the first factored instantiation that needs them (rounded to nearest)
  mutable DevArr<float> nf_P32;
  mutable DevArr<bf16> nf_P16;
  mutable std::mutex lowp_mu;
  template <typename PT>
  const PT* near_factors() const {
    if constexpr (sizeof(PT) == 8) return (const PT*)nf_P.p;
    else if constexpr (sizeof(PT) == 4) return (const PT*)nf_P32.p;
    else return (const PT*)nf_P16.p;
  }
  int gemv_mp = 12;   // single-RHS near MVM: 16-row panels per row chunk (4, 8 or 12)
  DevArr<ClassDev> cstore;
  DevArr<double> ff_chat, ff_theta;       // far panels (r1 r2 of Pp x Pp per class), theta factors
  // parametric H-matrix format (PH_FORMAT_H): per far block S_b, T_b; per stored class the far
  // core; per leaf the far blocks whose target cluster contains it (CSR); the instance's far
  // buffer holds H_q(theta_t) at t h_tot + h_off (h_tot entries per slot); the MVM's scratch W
  // holds w_b = H_b T_b^T x_t (hw_tot entries per slot and 16-column RHS tile)
  int format = PH_FORMAT_H2;
  int64_t n_hblk = 0, n_hcls = 0, h_tot = 0, hw_tot = 0;
  int64_t h_tbytes_max = 0;   // bytes of the largest T_b of a far block
  DevArr<HBlkDev> hblk;
  DevArr<HClsDev> hcls;
  DevArr<double> hcore, hS, hT;
  DevArr<int32_t> hl_ptr, hl_blk;
  // implicit coupling (PH_FORMAT_H2_IMPLICIT, Alg. "Modified H^2-Matrix MVM"): the same block,
  // class and CSR arrays over the coupling's index space (row s Pp + i of x_hat / y_hat is
  // entry i of node s): one block per far block with S_b = L_q, T_b = R_q (swapped for a
  // mirrored class) in hS = [L factors, R factors], per node its row range and work item
  DevArr<int64_t> hx_nbegin, hx_nend;
  DevArr<int32_t> hx_items;
  int64_t n_hx_items = 0;
  // coupling work list: target boxes of NTG nodes of one level (see coupling_groups)
  DevArr<int32_t> grp_targets;            // n_groups x NTG node ids (-1 = absent)
  DevArr<int32_t> grp_entry;              // n_groups + 1
  DevArr<int32_t> ent_cls;                // per entry: class
  DevArr<int32_t> ent_tau;                // per entry: NTG source nodes (-1 = target unused)
  DevArr<int32_t> ent_mask;               // per entry: bit s set if target s uses the class
  // class-list chunks of equal estimated work: for G = 2^c (c = 0..6), box b's chunk g
  // is entries [chunk_first[chunk_off[c] + b (G + 1) + g], ... + g + 1)
  DevArr<int32_t> chunk_first;
  int64_t chunk_off[7] = {0, 0, 0, 0, 0, 0, 0};
  // the same for half boxes (two groups per box, halves adjacent): entries with at least one
  // active target in the half, weights from the half's activity
  DevArr<int32_t> hgrp_targets, hent_cls, hent_tau, hchunk_first;
  int64_t hchunk_off[7] = {0, 0, 0, 0, 0, 0, 0};
  int64_t n_hgroups = 0;
  int64_t device_bytes = 0;
};

struct InstData {
  std::shared_ptr<const DeviceModel> m;
  int T = 1;
  ph_dtype dt = PH_F64;
  int grad_dim = -1;
  std::vector<double> theta;          // T x d_theta, as last instantiated
  size_t esize = 8;                   // element size of C, x_hat, y_hat, I/O (compute type)
  size_t d_esize = 8;                 // element size of the near blocks D (storage type)
  DevArr<char> D, C;
  // BF16 instances: C in the operand order of the BF16 coupling ([slot][class][32-wide K
  // panel][row tile][lane][8]); xb: the matching BF16 copy of x_hat (MVM scratch)
  DevArr<char> Cb, xb;
  DevArr<char> hw;   // parametric H-matrix format: MVM scratch w_b per far block, slot and RHS tile
  // factored near field (no D): c_b(theta_t) per stored block q, rank chunk c and slot t at
  // ((q KRp / KM + c) T + t) KM
  bool factored = false;
  DevArr<char> ccore;
  DevArr<double> v;
  int64_t Rcap = 0;
  int Gcap = 0;
  DevArr<char> xt, yt, xh, yh, part, zb;   // zb: [T][Zt] near-field pair buffers (R = 1)
  DevArr<char> bil;                   // ph_bilinear: K~ x
  DevArr<double> bil_part;            // ph_bilinear: per-block partial sums
  hipStream_t aux = nullptr;          // second stream: near field concurrent with the far chain
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_near = nullptr;       // after the near-field instantiation on aux
  bool near_pending = false;          // instantiated blocks may still be in flight on aux
  DevArr<double> theta_d;             // T x d_theta on the device (read by the theta-vector kernel)
  double* theta_pin = nullptr;        // pinned staging of theta
  hipEvent_t ev_theta = nullptr;      // after the last use of theta_pin
  bool theta_pending = false;
  int graphs = 0;                     // live graphs recorded from this instance (scratch is fixed)
  // launch configuration of the MVM chosen by ph_autotune (0 = default heuristics)
  int tune_chunks = 0, tune_prefetch = 0, tune_overlap = -1;
  int tune_fused_tcb = 0, tune_fused_rt = 0;   // factored near MVM: slots per workgroup, row tiles per wave
  ~InstData() {
    if (aux) (void)hipStreamSynchronize(aux);   // no kernel of this instance may outlive its buffers
    if (ev_near) (void)hipEventDestroy(ev_near);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_theta) (void)hipEventDestroy(ev_theta);
    if (theta_pin) (void)hipHostFree(theta_pin);
    if (aux) (void)hipStreamDestroy(aux);
  }
};

// Make `st` wait for a near-field instantiation still running on the instance's second
// stream (every entry point that reads the instance on a stream calls this first).
inline void join_near(InstData& in, hipStream_t st) {
  if (in.near_pending) {
    PH_HIP(hipStreamWaitEvent(st, in.ev_near, 0));
    in.near_pending = false;
  }
}

// Scratch memory supplied by the caller of matvec_impl instead of the instance's own
// (allocation-free entry point): base (device, 256-byte aligned) and its size in bytes.
struct ExtScratch {
  void* base;
  size_t bytes;
};

// S: compute type (C, x_hat, I/O); DT: storage type of the near blocks D
template <typename S, typename DT>
void instantiate_impl(InstData& in, const double* theta, hipStream_t st);
template <typename S, typename DT>
void matvec_impl(InstData& in, const S* x, S* y, int64_t R, double alpha, double beta, double nugget,
                 hipStream_t st, const ExtScratch* ext = nullptr);
template <typename S, typename DT>
void bilinear_impl(InstData& in, const S* u, const S* x, int64_t R, double* out, hipStream_t st);
// factored near field (k_near_fused.hip)
template <typename S>
void near_cores_launch(InstData& in, hipStream_t st);
template <typename S, typename PT>
void near_fused_launch(InstData& in, const S* xt, S* yt, int64_t Rs, hipStream_t st);
template <typename S, typename PT>
void near_block_eval(const InstData& in, int t, int64_t q, double* dev_out, hipStream_t st);
void make_low_factors(const DeviceModel& m, ph_dtype dt, hipStream_t st);
// Coupling of a PH_BF16 instance on the BF16 matrix cores (k_coupling_bf16.hip; whole target
// boxes, class-list chunks G, Rs a multiple of 16, output to the partials or y_hat): operand
// sizes per slot, whether the model's shape is supported, the C repacking after
// instantiation, and the coupling launch (x_hat repacked into xb for the nodes >= a0, then
// the matrix-core pass)
int64_t coupling_bf16_c_bytes(const DeviceModel& m);
int64_t coupling_bf16_x_bytes(const DeviceModel& m, int64_t Rs);
bool coupling_bf16_supported(const DeviceModel& m, int64_t Rs);
void coupling_bf16_pack_c(const InstData& in, hipStream_t st);
void coupling_bf16_launch(const InstData& in, const float* xh, void* xb, float* out, int G, int64_t Rs, int64_t nrc,
                          int64_t a0, hipStream_t st);
// Parametric H-matrix format (k_hmatrix.hip): H_q(theta_t) for every stored class and slot
// into the instance's far buffer; the far field of the MVM, phase 0: W = H_b T_b^T x_t for
// every far block, phase 1: yt += S_b w_b over the far blocks containing each row
void h_core_launch(const InstData& in, hipStream_t st);
void h_far_launch(const InstData& in, const double* xt, double* yt, double* W, int64_t Rs, int64_t nrc,
                  hipStream_t st, int phase);
// Implicit coupling (k_hmatrix.hip): y_hat_s = sum over the far blocks (s, t) of
// L_q (H_q(theta) (R_q^T x_hat_t)) for every node s of the far levels (written, not added)
void implicit_coupling_launch(const InstData& in, const double* xh, double* yh, double* W, int64_t Rs,
                              int64_t nrc, hipStream_t st);
// CG / iterative refinement for the R right-hand sides [R][n] of y and a (k_solve.hip)
void cg_solve_impl(InstData& hi, InstData* lo, const double* y, double* a, int64_t R, double nugget, double tol,
                   int max_iter, int inner_max, double inner_tol, ph_cg_stats* stats, hipStream_t st);

// ---- per-kernel timing with HIP events
struct TraceRec {
  int stage;
  hipEvent_t a, b;
};
extern std::mutex g_trace_mu;
extern bool g_trace_on;
extern thread_local bool g_capturing;   // recording a graph on this thread: no tracing events
extern std::vector<TraceRec> g_trace_recs;
hipEvent_t pooled_event();  // caller holds g_trace_mu

// Launch a kernel on stream st; when tracing, bracket it with events tagged by stage.
template <typename K, typename... Args>
inline void launch(int stage, K kernel, dim3 grid, dim3 block, hipStream_t st, Args... args) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return;
  hipEvent_t a = nullptr, b = nullptr;
  const bool tr = g_trace_on && !g_capturing;
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

// ---- 16 x 16 x 4 multiply-accumulate used by the hot kernels.
// B operand (both types): lane l holds B[k = l / 16][n = l % 16].
// FP32: one V_MFMA_F32_16X16X4 (A lane l = A[l % 16][l / 16]; result element i of
//   lane l at row 4 (l / 16) + i, column l % 16).
// FP64: four V_MFMA_F64_4X4X4 (4-block) instructions, one per group of 4 rows; in
//   instruction c, lane l holds A[4c + l % 4][l / 16] and block (l % 16) / 4 multiplies
//   it with columns 4 ((l % 16) / 4) .. + 3 of B, so the B register is the same as
//   above; result element c of lane l sits at row 4c + l / 16, column l % 16.  On gfx950
//   this issues at twice the rate of V_MFMA_F64_16X16X4 (measured: 71 vs 34 TFLOP/s).
// load_a(f, lane) builds the A operand from an accessor f(row) of the lane's K column;
// load_tiled(kr, lane) reads it from one K row of a matrix stored in fragment order
// (frag_index below), where the four FP64 values of a lane are adjacent.
template <typename S>
struct Tile16;

template <>
struct Tile16<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  typedef double a_t __attribute__((ext_vector_type(4)));
  template <typename F>
  static __device__ __forceinline__ a_t load_a(F f, int lane) {
    a_t a;
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = f(4 * c + (lane & 3));
    return a;
  }
  static __device__ __forceinline__ a_t load_tiled(const double* kr, int lane) {
    return *reinterpret_cast<const a_t*>(kr + (lane & 3) * 4);
  }
  static __device__ __forceinline__ acc_t mac(a_t a, double b, acc_t acc) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[c], b, acc[c], 0, 0, 0);
    return acc;
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};

template <>
struct Tile16<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  typedef float a_t;
  template <typename F>
  static __device__ __forceinline__ a_t load_a(F f, int lane) {
    return f(lane & 15);
  }
  static __device__ __forceinline__ a_t load_tiled(const float* kr, int lane) {
    const int m = lane & 15;
    return kr[(m & 3) * 4 + (m >> 2)];
  }
  static __device__ __forceinline__ acc_t mac(a_t a, float b, acc_t acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// Fragment order of a Pp x Pp coupling matrix (Pp a multiple of 16): entry (m, k) sits in
// the 16-column panel k / 16, 16-row tile m / 16, and inside the 256-entry tile at
// (k % 16) * 16 + (m % 4) * 4 + (m % 16) / 4.  A panel is one contiguous pipeline stage of
// the coupling kernel, and the four rows 4c + q (c = 0..3) a lane feeds to the FP64
// matrix cores are adjacent.
__host__ __device__ inline int64_t frag_index(int m, int k, int Pp) {
  return (int64_t)(k >> 4) * Pp * 16 + (m >> 4) * 256 + (k & 15) * 16 + (m & 3) * 4 + ((m & 15) >> 2);
}

// Work estimate of one coupling entry with `act` targets using its class, in units of one
// target's matrix-core time per stage: the multiplications plus the fixed cost of a stage
// (panel copy, fragment reads, barrier), which measured about 6 targets' worth on gfx950
// (per workgroup: 1.21 us per stage + 0.21 us per active target and stage).
inline int32_t coupling_entry_weight(int act) { return act + 6; }

// Raw buffer resources (CDNA3/4 word 3: 32-bit data format, no swizzle); a load at
// BUF_OOB lies past any buffer the library creates and returns zeros.
constexpr int BUF_WORD3 = 0x00020000;
constexpr int BUF_OOB = 0x7ffffff0;
constexpr int64_t BUF_MAX_BYTES = 0x7fff0000;

// Raw buffer load of one stored value (byte offset; BUF_OOB returns zero without touching
// memory), so that every load of the loop below is unconditional and the compiler's wait
// counts track the prefetched registers exactly.
// (The offset is passed through an empty asm so that the compiler keeps one load per call
// instead of cloning it into branches for the two offsets of a select.)
template <typename DT>
__device__ __forceinline__ DT bload1(__amdgpu_buffer_rsrc_t r, int off) {
  asm volatile("" : "+v"(off));
  if constexpr (sizeof(DT) == 8) return __builtin_bit_cast(DT, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else if constexpr (sizeof(DT) == 4) return __builtin_bit_cast(DT, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  else return bf16{(uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0)};
}

// Right-hand sides are padded to a multiple of RC in every internal buffer.
inline int64_t rhs_stride(int64_t R) { return (R + RC - 1) / RC * RC; }

inline int64_t grid_for(int64_t work) {
  int64_t g = (work + NT - 1) / NT;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return g;
}

}  // namespace ph
