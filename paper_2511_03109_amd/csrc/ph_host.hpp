// Host-side data structures of the parametric H^2 library: cluster tree, block
// lists, translation classes (Sec. 3.2, 3.3, 5.2 of arxiv 2511.03109) and the
// offline stage's compressed tensors (Alg. "Offline Stage: Parametric H^2").
// Pure C++ (no HIP); the device side uploads what it needs from these.
#pragma once

#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "ph.h"

namespace ph {

// A failure carrying a ph status code; converted to a return code at the C ABI.
struct Failure : std::runtime_error {
  int code;
  Failure(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] inline void fail(int code, const std::string& msg) { throw Failure(code, msg); }

struct TreeData {
  int64_t n = 0;
  int d = 0;
  int l_max = 0;
  double lo = 0, hi = 1;
  int eta2_num = 1, eta2_den = 1;
  std::vector<double> pts_t;       // tree-ordered points, n x d row-major
  std::vector<int64_t> perm;       // tree position -> original index
  // nodes, breadth-first ids
  std::vector<int32_t> level, coords, parent, first_child, nchild, cid;
  std::vector<int64_t> begin, end;
  std::vector<double> box_lo, box_hi;  // n_nodes x d
  std::vector<int32_t> level_start;    // nodes of level l are [level_start[l], level_start[l+1])
  std::vector<int32_t> leaves;         // leaf node ids in tree order
  // leaf blocks, sorted by (level, sigma, tau)
  std::vector<int32_t> near, far, far_class;   // near/far: 2 entries per block
  std::vector<int32_t> class_level, class_off; // class_off: d entries per class
  std::vector<int32_t> class_first_block;      // first far block of each class
  int64_t near_entries = 0;
  int min_far_level = -1;

  int64_t n_nodes() const { return (int64_t)level.size(); }
  int64_t n_near() const { return (int64_t)near.size() / 2; }
  int64_t n_far() const { return (int64_t)far.size() / 2; }
  int64_t n_classes() const { return (int64_t)class_level.size(); }
  int64_t size(int32_t node) const { return end[node] - begin[node]; }
};

std::shared_ptr<TreeData> build_tree(const double* pts, int64_t n, const ph_tree_opts& o);

// Offline stage output (host).  Layout conventions:
//  U        n x d x p_s, tree order: U[(i*d + k)*p_s + j] = l_j^{(B_leaf,k)}(x_{i,k})
//  E        2 x p_s x p_s: E[(h*p_s + j)*p_s + i] = l_i^{parent}(eta_j^{child half h})
//  near P   rank-outer per stored block: P[P_off + k*ldp*n_t + i + j*ldp],
//           ldp = n_s rounded up to a multiple of 16 (padding entries are 0)
//  near core  c-major: core[core_off + k + r_e*(a + r_1*b)]
//  Theta factors (near and far) column-major p_theta x r: th[off + q + p_theta*a]
//  far L, R  column-major P x r
//  far core  core[off + a + r_L*(k_1 + r_1*(k_2 + r_2*b))]
//  far panels  Chat[chat_off + q*P*P + i + P*j] = (L G_q R^T)[i, j], q = k_1 + r_1 k_2,
//              G_q[a, b] = core[a, k_1, k_2, b]; C(theta) = sum_q w_1[k_1] w_2[k_2] Chat_q
struct NearStored {
  int32_t s, t;             // node ids, s <= t
  int64_t s_begin, t_begin; // tree-order offsets
  int32_t ns, nt;
  int32_t ldp;              // leading dimension of the stored factor columns (multiple of 16)
  int32_t r_e, r1, r2;      // r2 = 1 when d_theta = 1
  int64_t P_off, core_off, th1_off, th2_off;
  int32_t b_st, b_ts;       // canonical near indices of (s,t) and (t,s) (b_ts = -1 if s == t)
};

struct ClassStored {
  int32_t cls, mirror;      // class index and its mirror (-1 if none)
  int32_t rL, r1, r2, rR;
  int64_t L_off, R_off, core_off, th1_off, th2_off, chat_off;
};

// Far block of the parametric H-matrix format: S_b (n_s x rs) and T_b (n_t x rt), column-major
// with leading dimensions lds, ldt (n rounded up to 16, zero rows), stored class q of the
// block's translation class and tr = 1 when the block uses the transposed class.
struct HBlock {
  int32_t s, t, q, tr, rs, rt, lds, ldt;
  int64_t s_begin, t_begin, ns, nt, S_off, T_off;
};

struct HostModel {
  int d = 0, p_s = 0, P = 0, p_theta = 0, d_theta = 0;
  ph_kernel kernel = PH_KERNEL_GAUSSIAN;
  double th_lo[2] = {0, 0}, th_hi[2] = {0, 0};
  double tol = 0;
  std::vector<double> U, E;
  std::vector<NearStored> nstore;
  std::vector<double> nf_P, nf_core, nf_theta;
  std::vector<int32_t> near_src, near_tr;   // per canonical near block
  std::vector<ClassStored> cstore;
  std::vector<double> ff_L, ff_R, ff_core, ff_theta, ff_chat;
  std::vector<int32_t> class_src, class_tr; // per class: stored index, transposed?
  int64_t kernel_evals = 0;
  int64_t near_factor_entries = 0;
  int svd_sweeps_max = 0;   // most one-sided Jacobi sweeps any SVD of the stage needed
  // parametric H-matrix format (ph_offline_compress_h): explicit far factors per far block
  bool hformat = false;
  // implicit coupling (ph_offline_compress_tt with PH_COUPLING_IMPLICIT): the online stage forms
  // H_q(theta) only and the MVM applies L_q H_q R_q^T without forming C
  bool implicit = false;
  std::vector<HBlock> hblk;
  std::vector<double> hS, hT;
};

// Compression of the offline stage's tensors: truncated HOSVD, or TT-cross + TT-rounding
enum class Compress { HOSVD, TT };

// gpu: the kernel tensors (near blocks and far classes) are evaluated on the GPU
// (k_offline.hip) and compressed on the host; comp: the compression (TT: host only, the
// entries are evaluated on demand by the cross)
std::shared_ptr<HostModel> offline_host(const TreeData& t, const ph_offline_opts& o, bool gpu = false,
                                        Compress comp = Compress::HOSVD);

// TT ranks r_0 .. r_N of every translation class's far tensor after TT-cross + TT-rounding
// (n_classes x (N + 1), N = 2 d + d_theta; mirrored classes in reverse order), without building
// a model; P up to 4096 and p_theta up to 64.  evals_out: distinct kernel values evaluated.
std::vector<int32_t> tt_far_ranks(const TreeData& t, const ph_offline_opts& o, int64_t* evals_out);

// ---- dense linear algebra of the offline stage (offline.cpp), column-major
// Householder QR of the m x k matrix A (m >= k) in place: R in the upper triangle, the
// reflectors below it (unit leading entry implied) with scalars tau
void householder_qr(double* A, int64_t m, int k, double* tau);
// Y (m x r) <- Q Y with Q from householder_qr
void apply_q(const double* A, int64_t m, int k, const double* tau, double* Y, int r);
// Left singular vectors and singular values (descending) of the m x q matrix X
struct LeftSV {
  std::vector<double> U;  // m x kk, kk = min(m, q)
  std::vector<double> s;  // kk
  int64_t m = 0;
  int kk = 0;
  int sweeps = 0;   // one-sided Jacobi sweeps (more than the cap: not converged)
};
LeftSV left_sv(const double* X, int64_t m, int64_t q);
// smallest r with sum_{j >= r} s_j^2 <= thr, never cutting a cluster of equal values
int truncation_rank(const double* s, int k, double thr);

// ---- tensor train (tt.cpp; Sec. 2.1): TT-cross with partially pivoted ACA per supercore,
// a sampled max-norm check with enrichment, then TT-rounding
struct TensorTrain {
  std::vector<int> dims;                   // m_0 .. m_{N-1}
  std::vector<int> ranks;                  // r_0 = 1 .. r_N = 1
  std::vector<std::vector<double>> cores;  // core k: r_k x m_k x r_{k+1}, column-major
  int64_t evals = 0;                       // distinct tensor entries evaluated
  int sweeps = 0;                          // most Jacobi sweeps of the rounding's SVDs
};
// Entry accessor: out[s] = X[idx[s * N .. s * N + N - 1]] for s < count (multi-indices
// row-major, column-major tensor)
typedef void (*EntryFn)(const void* ctx, const int32_t* idx, int64_t count, double* out);
// TT-cross at a tenth of tol (the sampled max-norm check at 10 tol), then TT-rounding at tol
TensorTrain tt_compress(EntryFn entry, const void* ctx, const std::vector<int>& dims, double tol);

// GPU kernel-tensor generation for the offline stage (k_offline.hip).  A near job is one stored
// near block: out[off + kk Ne + j ns + i] = kappa(x_{s_begin + i}, x_{t_begin + j}; grid[kk]),
// Ne = ns nt.  A far job is one stored class: out[off + i + P (kk + q j)] = kappa(a_i, b_j;
// grid[kk]) with a, b the class's P Chebyshev nodes (P x d each, in nodes[job * 2 P d ...]).
// The generator keeps the tree points, the theta grid and the Bessel orders on the device.
struct NearJob {
  int64_t s_begin, t_begin, off;
  int32_t ns, nt;
};
class GpuTensorGen {
 public:
  GpuTensorGen(const TreeData& t, ph_kernel kernel, const double* grid, int q);
  ~GpuTensorGen();
  // near tensors of the jobs into host memory out (total entries), synchronous
  void near(const std::vector<NearJob>& jobs, int q, double* out, int64_t total);
  // far tensors of n_cls classes (P x q x P each, consecutive) into host memory out
  void far(const std::vector<double>& nodes, int n_cls, int P, double* out);
  // near tensors of the jobs generated on the device (kept for near_factors) and the R factor
  // of a Householder QR of each (q x q column-major, per job) into host memory R; q <= 16
  void near_qr(const std::vector<NearJob>& jobs, int q, int64_t total, double* R);
  // U_job = A_job W_job (Ne x rk[job], W q x rk column-major at woff[job]) for the tensors of the
  // last near_qr, column-major into host memory out at uoff[job] (utotal entries)
  void near_factors(const std::vector<NearJob>& jobs, int q, const std::vector<double>& W,
                    const std::vector<int64_t>& woff, const std::vector<int32_t>& rk,
                    const std::vector<int64_t>& uoff, int64_t utotal, double* out);
 private:
  struct Impl;
  Impl* p_;
};
// The far factors of the parametric H-matrix format from the class factors of offline_host
// (offline_h.cpp); sets m.hformat.
void hmatrix_far_host(const TreeData& t, HostModel& m, int num_threads);

// kernel value kappa(x, y; theta) on the host
double kernel_value(ph_kernel k, int d, const double* x, const double* y, const double* th);
int kernel_dtheta(ph_kernel k, int d);
// e^x K_nu(x) (modified Bessel function of the second kind, nu >= 0, x > 0), the Matern
// kernel 2^(1 - nu) / Gamma(nu) z^nu K_nu(z), z = sqrt(2 nu) r / lambda, and the order
// constants of K_nu (special.cpp; the evaluation itself is kernel_fn.hpp)
struct BesselOrder;
double bessel_k_scaled(double nu, double x);
double matern_value(double r, double lambda, double nu);
BesselOrder bessel_order(double nu);

}  // namespace ph
