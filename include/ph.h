/*
 * ph.h -- C ABI of the MI355X parametric H^2-matrix library (online stage).
 *
 * Method: arxiv 2511.03109, "Parametric Hierarchical Matrix Approximations to
 * Kernel Matrices".  Problem statement (Sec. 1): points X = (x_i) in a box
 * B = [alpha, beta]^d, a parametric kernel kappa(x, y; theta), theta in a
 * parameter box Theta.  Offline, a parametric H^2-matrix K~(theta) is built over
 * Theta; online, for one theta, it is instantiated with no kernel evaluations and
 * applied in an H^2 matrix-vector product.
 *
 * Conventions
 *  - Every function returns an int status: PH_OK (0) or a negative PH_E* code.
 *    The message of the last failure on the calling thread is ph_last_error().
 *    No C++ exception crosses this interface.
 *  - Handles (ph_tree, ph_model, ph_inst) are opaque.  A model keeps what it needs
 *    of its tree and an instance keeps its model alive (reference counting), so
 *    the *_free functions may be called in any order; they accept NULL.
 *  - "Host" pointers are ordinary CPU memory, "device" pointers are HIP device
 *    memory of the current device.  Streams are hipStream_t passed as void*
 *    (NULL = the null stream).  Device work is stream-ordered and asynchronous;
 *    a kernel fault surfaces at the caller's next synchronisation.
 *  - Matrices are column-major (MATLAB order, Sec. 2.1 "Reshape Command"); multi-
 *    indices are flattened little-endian (first index fastest).
 *  - Tree order: the order of points after the cluster-tree partition (leaves in
 *    breadth-first order, each leaf keeping the original order of its points).
 */
#ifndef PH_H
#define PH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------- */
enum {
  PH_OK = 0,
  PH_EINVAL = -1,        /* bad argument (NULL pointer, size, NaN, point outside the box) */
  PH_EDOMAIN = -2,       /* theta outside the parameter box Theta */
  PH_ENOMEM = -3,        /* host or device allocation failed */
  PH_EHIP = -4,          /* a HIP runtime call failed */
  PH_ESTATE = -5,        /* handle used in a state that does not allow the call */
  PH_EUNSUPPORTED = -6   /* valid but not supported combination (kernel, d, d_theta, dtype) */
};

/* ---- kernels ---------------------------------------------------------------------
 * Closed-form stationary, symmetric kernels; r = |x - y|_2.
 *   GAUSSIAN        exp(-r^2 / (2 l^2))                          d_theta = 1, theta = (l)
 *   MATERN32        (1 + sqrt(3) r / l) exp(-sqrt(3) r / l)       d_theta = 1
 *   MATERN12        exp(-r / l)  (the paper's exponential E)     d_theta = 1
 *   ANISO_GAUSSIAN  exp(-sum_k (x_k - y_k)^2 / (2 l_k^2))         d_theta = d (d <= 2)
 *   POLY_TEST       theta^2 r^2 + theta (test kernel; reproduced exactly by p >= 3)
 *   POLY2_TEST      theta_1 r^2 + theta_2^2 (test kernel, d_theta = 2)
 *   MATERN          2^(1 - nu) / Gamma(nu) z^nu K_nu(z), z = sqrt(2 nu) r / lambda, value 1 at
 *                   r = 0; d_theta = 2, theta = (lambda, nu), lambda > 0, nu > 0 (Table "Kernel
 *                   functions", MN, with parameter space (lambda, nu) as in Sec. "Numerical
 *                   Experiments"; K_nu is the modified Bessel function of the second kind,
 *                   evaluated by the library's own routine: Temme's series for z <= 2, the
 *                   minimal solution of the confluent-hypergeometric recurrence above; within
 *                   1.4e-14 relative of quadrature for 0.5 <= nu <= 3).  nu = 1/2 and 3/2 give MATERN12 and MATERN32.
 */
typedef enum {
  PH_KERNEL_GAUSSIAN = 0,
  PH_KERNEL_MATERN32 = 1,
  PH_KERNEL_MATERN12 = 2,
  PH_KERNEL_ANISO_GAUSSIAN = 3,
  PH_KERNEL_POLY_TEST = 4,
  PH_KERNEL_POLY2_TEST = 5,
  PH_KERNEL_MATERN = 6
} ph_kernel;

/* Kernel values on the host (Table "Kernel functions"): out[i] = kappa(x_i, y_i; theta) for
 * i < n, with x, y host arrays of n points (row-major n x d) and theta the d_theta parameters
 * of the kernel (d_theta as for ph_offline_compress).  For exact reference values, e.g. the
 * rows of K(X, X; theta) x that the paper's error estimate compares against.  Errors:
 * PH_EINVAL for a NULL pointer, n < 0 or d outside 1..3, PH_EUNSUPPORTED for an unknown
 * kernel or a kernel / d combination the offline stage rejects, PH_EDOMAIN for a
 * non-positive length scale or nu. */
int ph_kernel_eval(ph_kernel kernel, int d, const double* x, const double* y, int64_t n, const double* theta,
                   double* out);

/* Hierarchical format of a model (Sec. "Parametric H-matrices and H²-matrices").
 *   PH_FORMAT_H2  parametric H²-matrix: nested cluster bases, one coupling matrix
 *                 C_b(theta) = L H(theta) R^T per far block (Def. "Parametric H²-matrix")
 *   PH_FORMAT_H   parametric H-matrix: explicit factors S_b = U_s L_b, T_b = U_t R_b per far
 *                 block and the far core H_b(theta) (Def. "Parametric H-matrix"; App. PTTK
 *                 offline phase 3); MVM by Alg. "H-matrix MVM" with the parametric far field
 *   PH_FORMAT_H2_IMPLICIT  parametric H²-matrix whose couplings stay factored: the online stage
 *                 forms H_q(theta) per stored class only, and the MVM applies
 *                 y_hat_s += L_q (H_q(theta) (R_q^T x_hat_t)) per far block (Alg. "Modified
 *                 H²-Matrix MVM"); from ph_offline_compress_tt with PH_COUPLING_IMPLICIT */
typedef enum { PH_FORMAT_H2 = 0, PH_FORMAT_H = 1, PH_FORMAT_H2_IMPLICIT = 2 } ph_format;

/* Arithmetic of an instance.  PH_F64: FP64 storage and arithmetic, I/O in double.
 * PH_F32: FP32 storage of the instantiated blocks, FP32 arithmetic (matrix cores with
 * FP32 accumulation), I/O in float.  PH_BF16: as PH_F32, but the near-field blocks D_b
 * (the dominant stream) are stored in BF16, rounded to nearest from the FP64
 * instantiation, and widened to FP32 on load.  The instantiation itself is FP64 in all
 * three. */
typedef enum { PH_F64 = 0, PH_F32 = 1, PH_BF16 = 2 } ph_dtype;

typedef struct ph_tree ph_tree;
typedef struct ph_model ph_model;
typedef struct ph_inst ph_inst;

/* ---- cluster tree and block cluster tree ------------------------------------------
 * Sec. 3.2 and Alg. ConstructClusterTree: uniform 2^d-ary subdivision of the box
 * [lo, hi]^d down to level l_max.  A point with x_k <= midpoint goes to the lower
 * half of axis k; children are numbered by the little-endian child id
 * sum_k b_k 2^(k-1) (b_k = 1 for the upper half); children holding no point are
 * not created.  Node ids are breadth-first (level, parent id, child id).
 * Sec. 3.3 and Alg. ConstructBlockClusterTree: starting from root x root, an
 * inadmissible pair whose nodes both have children is split into all child pairs;
 * leaf pairs are far (admissible) or near.  Admissibility (eq. "admissible"),
 * max(diam B_s, diam B_t) <= eta dist(B_s, B_t), is evaluated exactly in integer
 * arithmetic on the box indices, with equality admissible; eta^2 is given as the
 * rational eta2_num / eta2_den.  Far blocks are grouped into translation classes
 * keyed by (level, box offset) (Sec. 5.2).
 */
typedef struct {
  int d;            /* spatial dimension, 1..3 */
  double lo, hi;    /* the root box [lo, hi]^d; every point must lie inside */
  int leaf_size;    /* used when l_max < 0: l_max = smallest l with n <= leaf_size 2^(d l) */
  int l_max;        /* maximum (and leaf) level, >= 0, or -1 to derive it from leaf_size */
  int eta2_num;     /* eta^2 = eta2_num / eta2_den, both > 0 */
  int eta2_den;
} ph_tree_opts;

typedef struct {
  int64_t n;
  int d;
  int l_max;
  int64_t n_nodes, n_leaves, n_near, n_far, n_classes;
  int64_t near_entries;      /* N_nf = sum over near blocks of n_s n_t */
  int min_far_level;         /* smallest level holding a far block, or -1 */
} ph_tree_info;

/* Build the trees.  pts: host, row-major n x d, copied.  Errors: PH_EINVAL for a NULL
 * pointer, n < 1, d outside 1..3, lo >= hi, a NaN or a point outside [lo, hi]^d,
 * l_max > 20 or a non-positive eta2.  *out is owned by the caller (ph_tree_free). */
int ph_build_tree(const double* pts, int64_t n, const ph_tree_opts* opts, ph_tree** out);

int ph_tree_info_get(const ph_tree* t, ph_tree_info* info);

/* perm[t] = original index of the point at tree position t (host, n entries). */
int ph_tree_perm(const ph_tree* t, int64_t* perm);

/* Per node (host arrays of n_nodes entries; coords has n_nodes * d, node-major):
 * level, integer box index at its level, [begin, end) range in tree order, parent
 * (-1 for the root).  Any pointer may be NULL to skip that array. */
int ph_tree_nodes(const ph_tree* t, int32_t* level, int32_t* coords, int64_t* begin,
                  int64_t* end, int32_t* parent);

/* Block lists sorted by (level, sigma, tau): near[2b], near[2b+1] = (sigma, tau) node ids;
 * far likewise, far_class[b] = its translation class.  Any pointer may be NULL. */
int ph_tree_blocks(const ph_tree* t, int32_t* near, int32_t* far, int32_t* far_class);

/* Translation classes sorted by (level, offset lexicographic, axis 1 first):
 * level[c], offset[c * d + k] = k_tau - k_sigma along axis k. */
int ph_tree_classes(const ph_tree* t, int32_t* level, int32_t* offset);

void ph_tree_free(ph_tree* t);

/* ---- offline stage -------------------------------------------------------------------
 * Alg. "Offline Stage: Parametric H^2-matrix": leaf cluster-basis factors
 * [U_{s,k}]_{ij} = l_j^{(B_{s,k})}(x_{s,i,k}) (Sec. 3.2), transfer factors
 * [E_{s',k}]_{j,i} = l_i^{(B_s,k)}(eta_j^{(B_s',k)}) (Sec. 3.4.1, lemma orientation),
 * one far tensor M[i, k_1.., j] = kappa(eta_i^{B_s}, eta_j^{B_t}; eta_k) per
 * translation class (App. PTTK review, Sec. 5.2) and one near tensor
 * A_b[e, k_1..] = kappa(x_{s,i}, x_{t,j}; eta_k), e = i + j n_s, per near block
 * (Sec. 4.3), each compressed by a truncated HOSVD whose mode ranks keep
 * sum_{j>r} s_j^2 <= (tol^2 / N) ||M||_F^2 (N modes), in FP64 on the host, then
 * uploaded.  Symmetry: A_{ts} = A_{st}^T and M_{(l,-o)} = M_{(l,o)}^T exactly, so only
 * near blocks with sigma <= tau and classes with offset >= 0 (lexicographic) are
 * compressed; the others are their transposes.
 */
typedef struct {
  ph_kernel kernel;
  int d_theta;              /* 1 or 2; must match the kernel */
  double theta_lo[2];       /* parameter box Theta = prod_k [theta_lo[k], theta_hi[k]] */
  double theta_hi[2];
  int p_s;                  /* spatial Chebyshev nodes per axis, 1..16; P = p_s^d <= 128 */
  int p_theta;              /* parameter Chebyshev nodes per axis, 1..16 */
  double tol;               /* relative Frobenius tolerance of each compressed tensor, >= 0 */
  int num_threads;          /* host threads for the offline work, 0 = all */
} ph_offline_opts;

typedef struct {
  int64_t n, n_near_stored, n_classes_stored;
  int64_t near_entries;       /* N_nf */
  int64_t near_factor_entries;/* sum over stored near blocks of N_e * r_e */
  double near_rank_mean;      /* entry-weighted mean near rank r_bar */
  int near_rank_max;
  double far_rank_mean;       /* mean of (r_L + r_R)/2 over stored classes */
  int far_rank_max;
  int64_t device_bytes;       /* bytes the model holds on the device */
  int64_t kernel_evals;       /* kernel evaluations done by the offline stage */
  int P, p_theta, d_theta;
  int svd_sweeps_max;         /* most one-sided Jacobi sweeps any SVD of the offline stage took */
} ph_model_info;

/* Offline stage.  stream: the upload stream.  Errors: PH_EINVAL (NULL, bad sizes,
 * theta_lo >= theta_hi), PH_EUNSUPPORTED (kernel / d / d_theta combination, or an SVD
 * whose one-sided Jacobi iteration still rotates after 80 sweeps), PH_ENOMEM, PH_EHIP.
 * Truncation: the rank of each mode is cut as stated above, then moved past every
 * following singular value within relative 1e-4 of the last one kept, so that a cluster
 * of equal singular values (exactly degenerate pairs arise from symmetric geometry) is
 * kept or dropped as a whole and the kept subspace is unique.  *out is owned by the caller (ph_model_free); the tree may be
 * freed right after this call. */
int ph_offline_compress(const ph_tree* t, const ph_offline_opts* opts, void* stream,
                        ph_model** out);

/* ph_offline_compress with the kernel tensors evaluated on the GPU (the kernel-tensor
 * generation of Alg. "Offline Stage: Parametric H²-matrix": the near tensors of the stored near
 * blocks in batches of at most 512 MB and the far tensors of the stored classes, by the same
 * kernel functions as the host), compressed on the host as in ph_offline_compress.  The model is
 * the same up to the rounding of the kernel values (a few ulp).  Errors as ph_offline_compress,
 * plus PH_EHIP / PH_ENOMEM from the GPU. */
int ph_offline_compress_gpu(const ph_tree* t, const ph_offline_opts* opts, void* stream, ph_model** out);

/* Offline stage of the parametric H-matrix format (Alg. "Offline Stage: Parametric H-matrix";
 * App. PTTK offline, phases 1-3): the same near field and far tensors as ph_offline_compress,
 * then S_b = U_s L_b and T_b = U_t R_b for every far block (U_s evaluated on the block's own
 * clusters; (L_b, R_b) swapped for blocks whose class is the mirror of a stored one).  The model
 * supports PH_F64 instances only (PH_EUNSUPPORTED for other dtypes); ph_instantiate forms
 * H_q(theta) per stored class, ph_matvec applies S_b H_b T_b^T per far block.  Errors as
 * ph_offline_compress.  *out is owned by the caller (ph_model_free). */
int ph_offline_compress_h(const ph_tree* t, const ph_offline_opts* opts, void* stream, ph_model** out);

/* Offline stage with the paper's own compression (Sec. 2.1 "Tensor Train Decomposition";
 * Sec. 4.2 / App. PTTK review for the far tensors, Sec. 4.3 for the near tensors): every far
 * tensor M[i_1..i_d, k_1.., j_1..j_d] and near tensor A_b[e, k_1..] is approximated by TT-cross
 * (partially pivoted ACA on each supercore, started from the middle index of every mode,
 * alternating sweeps, a max-norm error check at 10 tol on 256 SplitMix64-sampled entries with
 * enrichment of the index sets) at tol / 10 and then TT-rounded at tol; entries are evaluated on demand,
 * each at most once (ph_model_info.kernel_evals counts them).  The cores are converted exactly
 * into the online form: L_q from the target-side spatial cores, R_q from the source-side ones,
 * the parameter cores as the core of H_q(theta) with identity parameter factors (ranks
 * reported as (r_d, p_theta [, p_theta], r_{d+d_theta})), and U_e = G_1 for the near field.
 * Host only (num_threads threads).  coupling:
 *   PH_COUPLING_MATERIALIZED  format PH_FORMAT_H2: C_q(theta) is formed per class online
 *   PH_COUPLING_IMPLICIT      format PH_FORMAT_H2_IMPLICIT (PH_F64 instances only)
 * Errors as ph_offline_compress; PH_EINVAL for another coupling value. */
typedef enum { PH_COUPLING_MATERIALIZED = 0, PH_COUPLING_IMPLICIT = 1 } ph_coupling;
int ph_offline_compress_tt(const ph_tree* t, const ph_offline_opts* opts, int coupling, void* stream,
                           ph_model** out);

/* The compression of ph_offline_compress_tt on its own (Sec. 2.1; the paper's Rank and
 * Coupling Ratio are functions of these ranks): the TT ranks r_0 .. r_N, N = 2 d + d_theta, of
 * the far tensor of every translation class after TT-cross and TT-rounding, host only, no model
 * built and nothing uploaded, so p_s^d up to 4096 and p_theta up to 64 are accepted (the model
 * entry points stop at 128 and 16).  ranks: host, n_classes x (N + 1) row-major in class order
 * (ph_tree_classes); a class whose offset is lexicographically below its negative reports the
 * ranks of its mirror in reverse order.  kernel_evals (may be NULL): distinct kernel values
 * evaluated.  Errors as ph_offline_compress. */
int ph_tt_far_ranks(const ph_tree* t, const ph_offline_opts* opts, int32_t* ranks, int64_t* kernel_evals);

/* The hierarchical format of a model (ph_format). */
int ph_model_format(const ph_model* m, int* format);

int ph_model_info_get(const ph_model* m, ph_model_info* info);

/* Ranks of the stored near blocks in canonical near order (e-mode rank; -1 for blocks
 * stored as the transpose of another), host array of n_near entries. */
int ph_model_near_ranks(const ph_model* m, int32_t* ranks);

/* Ranks (r_L, r_theta_1, [r_theta_2], r_R) of every class as stored (mirrored classes
 * report their source's ranks swapped), host array of n_classes * (2 + d_theta). */
int ph_model_class_ranks(const ph_model* m, int32_t* ranks);

void ph_model_free(ph_model* m);

/* ---- online stage --------------------------------------------------------------------
 * Alg. "Online Stage" and Alg. PTTK online.  For each theta: parametric vectors
 * v_k(theta_k) = [l_1 .. l_p](theta_k) on [theta_lo[k], theta_hi[k]] (App. PTTK
 * review), far couplings C(theta) = L H(theta) R^T per class with
 * H = core x_theta (Theta_k^T v_k) (Sec. 4.2), near blocks
 * D_b(theta) = reshape(P_b c_b(theta), [n_s, n_t]) with c_b = core x_theta (Theta_k^T v_k)
 * (Sec. 4.3).  No kernel evaluation happens here.
 *
 * theta: host, T x d_theta row-major.  T >= 1 instantiates T independent parameter
 * values into one instance (slot t holds theta[t]).  dt selects the storage and
 * arithmetic (PH_F64, PH_F32 or PH_BF16).
 * *inout: NULL -> a new instance is allocated and returned (owned by the caller,
 * ph_inst_free).  Non-NULL -> that instance is re-instantiated in place; it must come
 * from the same model with the same T and dt (else PH_EINVAL), and no allocation
 * happens.  Any theta outside Theta -> PH_EDOMAIN before anything is enqueued. */
int ph_instantiate(const ph_model* m, const double* theta, int T, ph_dtype dt, void* stream,
                   ph_inst** inout);

/* Form of the near field held by an instance (the far field is always instantiated).
 *   PH_NEAR_BLOCKS    every near block D_b(theta_t) is written to device memory
 *                     (T N_nf entries) and each ph_matvec reads the blocks.  Suited to many
 *                     MVMs at few theta (e.g. a solver at one theta).
 *   PH_NEAR_FACTORED  only the vectors c_b(theta_t) = core_b x_theta (Theta_k^T v_k) are
 *                     formed (Sec. 4.3); each ph_matvec forms the blocks from the stored
 *                     factors P_b in registers and applies them at once, reading every factor
 *                     entry once for up to 8 slots, and no block is ever written.  D_b is
 *                     linear in c_b, so this is the same matrix.  Suited to batches of theta
 *                     with one or a few MVMs each.  In FP64 the blocks it forms are identical
 *                     to those PH_NEAR_BLOCKS writes.  For PH_F32 / PH_BF16 instances the
 *                     factors are streamed as an FP32 / BF16 copy (rounded to nearest, made
 *                     once per model on the first such instance) and the blocks are formed in
 *                     FP32.  Near ranks above 64: PH_EUNSUPPORTED.
 *   PH_NEAR_AUTO      FACTORED when 4 <= T <= 8 and the largest near rank is at most 64, else
 *                     BLOCKS (beyond 8 slots the factors are streamed once per batch of 8).
 * ph_instantiate and ph_instantiate_grad use PH_NEAR_AUTO. */
typedef enum { PH_NEAR_AUTO = 0, PH_NEAR_BLOCKS = 1, PH_NEAR_FACTORED = 2 } ph_near_mode;

/* ph_instantiate (grad_dim = -1) or ph_instantiate_grad (grad_dim >= 0) with an explicit
 * near-field form.  Re-instantiating an existing instance needs the same form (or
 * PH_NEAR_AUTO), else PH_EINVAL. */
int ph_instantiate_ex(const ph_model* m, const double* theta, int T, ph_dtype dt, ph_near_mode near,
                      int grad_dim, void* stream, ph_inst** inout);

/* *factored = 1 if the instance holds the factored near field, else 0. */
int ph_inst_near_mode(const ph_inst* k, int* factored);

/* As ph_instantiate, but the instance holds dK~/dtheta_dim at each theta: the
 * parametric vector of dimension dim is replaced by its derivative v_dim'(theta_dim)
 * (the approximation is linear in each v_k, so this is its exact derivative).
 * 0 <= dim < d_theta.  Use it with ph_matvec. */
int ph_instantiate_grad(const ph_model* m, const double* theta, int T, int dim, ph_dtype dt,
                        void* stream, ph_inst** inout);

/* H^2 matrix-vector product (Alg. "H^2-matrix MVM": FastForward, coupling over the far
 * blocks, near-field products, FastBackward), for every slot t:
 *   y_t = alpha * (K~(theta_t) + nugget I) x_t + beta * y_t.
 * x, y: device, slot-major [T][R][n] with each slot column-major n x R (leading
 * dimension n) in the ORIGINAL point order; double for PH_F64, float for PH_F32 and
 * PH_BF16.
 * x and y must not overlap.  R = 0 is a no-op.  With beta == 0, y is not read.
 * Scratch for R right-hand sides is allocated on the first call with a larger R and
 * kept in the instance. */
int ph_matvec(ph_inst* k, const void* x, void* y, int64_t R, double alpha, double beta,
              double nugget, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid device allocation): ph_matvec with the same arguments, result and
 * errors, whose scratch (x, y in tree order, the upward / downward coefficients, coupling
 * partial sums, single-RHS pair buffers) comes from a fixed array of 64 MiB that the
 * library holds on each GPU it runs on (in its code object, until the process ends)
 * instead of from the instance.  It calls no device allocation: a product that needs more
 * scratch than 64 MiB fails with PH_EINVAL before anything is launched (about
 * T (2 n + (2 + G) n_nodes Pp) R doubles; Pp = P rounded up to 16, G = 4 or 8 coupling
 * chunks, R rounded up to 16 when above 1).  Every call on one GPU uses the same array and
 * leaves its contents behind; calls that overlap on one GPU (concurrent streams or
 * threads) race, so callers serialise them. */
int ph_matvec_noalloc(ph_inst* k, const void* x, void* y, int64_t R, double alpha, double beta,
                      double nugget, void* stream);

/* Bilinear form per parameter slot:  out[t] = sum_r u_t[:, r]^T K~(theta_t) x_t[:, r]
 * (nugget excluded).  With an instance of ph_instantiate_grad(dim) this is
 * dL/dtheta_dim of L = sum_r u_r^T K~(theta) x_r, the parameter gradient of the
 * backward pass of y = K~(theta) x (multilinearity in the parametric vectors, Sec. 4.2
 * and 4.3).  u, x: device, layout of ph_matvec's x; out: device, T doubles.  The
 * product K~ x goes to a scratch buffer of the instance (allocated on the first call
 * with a larger R); the sum over points and right-hand sides is a fixed-order two-pass
 * reduction in FP64, so repeated calls give identical results.  Stream-ordered. */
int ph_bilinear(ph_inst* k, const void* u, const void* x, int64_t R, double* out, void* stream);

/* Solve (K~(theta) + nugget I) a = y by conjugate gradients (K~ is symmetric by
 * construction; it is positive definite up to the approximation error, which the nugget
 * of a regularised system covers).
 *   hi: PH_F64 instance with T = 1.  y, a: device, n doubles, original point order;
 *   a is overwritten (the initial guess is 0).
 *   lo == NULL: plain FP64 CG; max_iter bounds the total CG iterations.
 *   lo != NULL: FP64 iterative refinement.  lo is a PH_F32 or PH_BF16 instance of the
 *     same model and the same theta (else PH_EINVAL); each step forms the residual
 *     r = y - (K~ + nugget I) a with hi in FP64 and adds the correction from an inner
 *     CG on lo (to relative residual inner_tol or inner_max iterations, FP32 vectors);
 *     max_iter bounds the refinement steps, and refinement stops early once the FP64
 *     residual no longer decreases.
 * Stops when ||y - (K~ + nugget I) a|| <= tol ||y|| with the FP64 instance.  Synchronous:
 * it reads inner products back to the host each iteration.  stats may be NULL. */
typedef struct {
  int outer_steps;        /* refinement steps (plain CG: restarts from the true residual) */
  int inner_iterations;   /* CG iterations in total */
  double rel_residual;    /* final FP64 relative residual */
  int converged;          /* rel_residual <= tol */
} ph_cg_stats;
int ph_cg_solve(ph_inst* hi, ph_inst* lo, const double* y, double* a, double nugget, double tol, int max_iter,
                int inner_max, double inner_tol, ph_cg_stats* stats, void* stream);

/* ph_cg_solve for R right-hand sides at once (the batched form): y and a are device [R][n]
 * arrays (column c at c n, original point order), 1 <= R <= 1024.  Every iteration applies the
 * instance to the R search directions in one ph_matvec product, while each column keeps its own
 * CG scalars and stops on its own (refinement: per-column residual scaling and the same FP64
 * residual test per column).  stats: the largest iteration count and the worst final relative
 * residual over the columns; converged when every column meets tol.  Errors as ph_cg_solve. */
int ph_cg_solve_batch(ph_inst* hi, ph_inst* lo, const double* y, double* a, int64_t R, double nugget, double tol,
                      int max_iter, int inner_max, double inner_tol, ph_cg_stats* stats, void* stream);

/* ---- batched launches -----------------------------------------------------------------
 * Launch configuration of ph_matvec picked by measurement (autotuner): for the instance's
 * T slots and R right-hand sides, every combination of coupling class-list chunks
 * (1, 2, 4, 8, 16, at most the longest class list of a target box), register prefetch
 * depth of the coupling pipeline (1, 2) and near field overlapped on a second stream or
 * not is timed (3 runs after a warm-up, HIP events on `stream`), then, for a factored
 * instance, the launch shape of its near-field kernel (8, 4 or 2 parameter slots per
 * workgroup, 1 or 2 row tiles of 16 per wavefront) with the chosen configuration; the
 * fastest is kept in the instance for all later ph_matvec calls.  x, y: as ph_matvec (y is overwritten).
 * Synchronises `stream`.  Must precede ph_graph_create (PH_ESTATE after it).  On any
 * failure the instance keeps the configuration it had before the call. */
typedef struct {
  int chunks, prefetch, overlap;
  double ms;              /* measured time of one ph_matvec with this configuration */
  int fused_tcb;          /* factored near field: parameter slots per workgroup (0: default) */
  int fused_rt;           /* factored near field: 16-row tiles per wavefront (0: default) */
} ph_tune_info;
int ph_autotune(ph_inst* k, const void* x, void* y, int64_t R, void* stream, ph_tune_info* info);

/* Record instantiation + MVM of instance k as one HIP graph: theta vectors, far and near
 * instantiation of all T slots, then y = (K~ + nugget I) x for R right-hand sides (alpha
 * 1, beta 0).  The near field runs on the recording stream, or on the instance's second
 * stream (concurrently with the far field) when ph_autotune selected that.  x, y (device) are
 * bound into the graph.  stream must not be the null stream.  Runs one MVM first to
 * allocate all scratch; afterwards the instance's scratch is fixed (a ph_matvec that
 * would need more fails with PH_ESTATE) until every graph of the instance is freed.
 * *out is caller-owned (ph_graph_free). */
typedef struct ph_graph ph_graph;
int ph_graph_create(ph_inst* k, const void* x, void* y, int64_t R, double nugget, void* stream, ph_graph** out);

/* Replay a recorded graph: with theta != NULL (host, T x d_theta, checked against Theta
 * as ph_instantiate does) the instance is re-instantiated at these values, else at the
 * last ones.  The replay is ordered after every earlier call on the instance (a near-field
 * instantiation still running on its second stream is joined first).  An instance with
 * live graphs cannot be re-instantiated as the other kind (ph_instantiate after
 * ph_instantiate_grad or the reverse: PH_ESTATE).  One graph launch on `stream`; asynchronous (the host waits only for the
 * previous launch's read of its theta staging buffer). */
int ph_graph_launch(ph_graph* g, const double* theta, void* stream);
void ph_graph_free(ph_graph* g);

/* Inspection (tests): copy the instantiated near block of canonical near index b for
 * slot t (n_s x n_t column-major, as double; for a factored instance the block is formed
 * by a kernel in the arithmetic of the MVM) or the coupling matrix of class c (P x P
 * column-major, as double) to host memory.  Synchronises the device.  A parametric H-matrix
 * instance and an implicit-coupling instance form no coupling matrices: ph_inst_coupling
 * returns PH_EUNSUPPORTED for them. */
int ph_inst_near_block(const ph_inst* k, int t, int64_t b, double* host_out);
int ph_inst_coupling(const ph_inst* k, int t, int64_t c, double* host_out);

void ph_inst_free(ph_inst* k);

/* ---- tracing ---------------------------------------------------------------------------
 * When enabled, every kernel launch of ph_instantiate / ph_matvec is bracketed by HIP
 * events on its stream; ph_trace_read waits for the recorded events and returns the
 * summed device time and launch count per stage (and clears them if reset != 0).
 * Process-wide; meant for benchmarking, not for concurrent use from several threads. */
enum {
  PH_STAGE_THETA = 0,         /* parametric vectors v_k(theta_k) */
  PH_STAGE_FAR_INST = 1,      /* far-field couplings C(theta) */
  PH_STAGE_NEAR_INST = 2,     /* near-field blocks D_b(theta) */
  PH_STAGE_PERM_IN = 3,
  PH_STAGE_LEAF_UP = 4,       /* FastForward, leaves */
  PH_STAGE_TRANSFER_UP = 5,   /* FastForward, inner nodes */
  PH_STAGE_COUPLING = 6,      /* y_hat += C x_hat over far blocks */
  PH_STAGE_TRANSFER_DOWN = 7, /* FastBackward, inner nodes */
  PH_STAGE_NEAR_MVM = 8,      /* near-field products y_s = sum_t D_st x_t */
  PH_STAGE_PERM_OUT = 9,
  PH_STAGE_ZERO = 10,         /* reduction of split coupling partial sums */
  PH_STAGE_LEAF_DOWN = 11,    /* FastBackward, leaves */
  PH_STAGE_BILINEAR = 12,     /* reduction of ph_bilinear */
  PH_STAGE_SOLVE = 13,        /* vector updates and inner products of ph_cg_solve */
  PH_STAGE_NEAR_GATHER = 14,  /* near field, one right-hand side: y_t += D_st^T x_s (s < t) */
  PH_NUM_STAGES = 15
};
typedef struct {
  double ms[16];
  int64_t count[16];
} ph_trace_stats;

int ph_trace_enable(int on);
int ph_trace_read(ph_trace_stats* out, int reset);

/* Message of the last failure on this thread ("" if none). */
const char* ph_last_error(void);

/* Library version string. */
const char* ph_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PH_H */
