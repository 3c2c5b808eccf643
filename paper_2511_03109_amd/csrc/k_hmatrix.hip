// Parametric H-matrix format (Def. "Parametric H-matrix"): the online stage forms the far cores
// H_q(theta) (Alg. PTTK online) and the MVM applies every far block as S_b (H_b (T_b^T x_t))
// (Alg. "H-matrix MVM" with the parametric substitution of Sec. "MVM").  The near field is the
// one of the H^2 format.
#include "ph_device.hpp"

namespace ph {

// H_q(theta_t) = sum_{k1, k2} w_1[k1] w_2[k2] core_q[:, k1, k2, :], w_i = Theta_i^T v_i(theta_t),
// column-major rL x rR at Hc[t h_tot + h_off].  One workgroup per (stored class, slot).
__global__ void __launch_bounds__(NT) k_h_core(const HClsDev* __restrict__ cls, const double* __restrict__ core,
                                               const double* __restrict__ th, const double* __restrict__ v,
                                               double* __restrict__ Hc, int64_t h_tot, int p, int dth) {
  __shared__ double w1[16], w2[16];
  const HClsDev c = cls[blockIdx.x];
  const int64_t t = blockIdx.y;
  const double* vt = v + t * dth * p;
  if ((int)threadIdx.x < c.r1) {
    double s = 0;
    for (int q = 0; q < p; ++q) s += th[c.th1_off + q + (int64_t)p * threadIdx.x] * vt[q];
    w1[threadIdx.x] = s;
  } else if ((int)threadIdx.x >= 32 && (int)threadIdx.x < 32 + c.r2) {
    const int a = threadIdx.x - 32;
    double s = 1.0;
    if (dth == 2) {
      s = 0;
      for (int q = 0; q < p; ++q) s += th[c.th2_off + q + (int64_t)p * a] * vt[p + q];
    }
    w2[a] = s;
  }
  __syncthreads();
  double* H = Hc + t * h_tot + c.h_off;
  const int ne = c.rL * c.rR;
  for (int e = threadIdx.x; e < ne; e += NT) {
    const int a = e % c.rL, b = e / c.rL;
    double s = 0;
    for (int k2 = 0; k2 < c.r2; ++k2) {
      double s1 = 0;
      for (int k1 = 0; k1 < c.r1; ++k1)
        s1 += w1[k1] * core[c.core_off + a + (int64_t)c.rL * (k1 + (int64_t)c.r1 * (k2 + (int64_t)c.r2 * b))];
      s += w2[k2] * s1;
    }
    H[e] = s;
  }
}

constexpr int HTB = 8;    // parameter slots per workgroup (S_b and T_b read once for them)

// Offset of entry (m, k), m < 128, k < 16, in a 128 x 16 operand panel staged in LDS in the
// operand order of the FP64 matrix cores (the in-panel part of frag_index): row tile m / 16,
// then (k, m % 4, (m % 16) / 4), so the four rows a lane feeds to one instruction are adjacent.
__device__ __forceinline__ int panel_index(int m, int k) {
  return (m >> 4) * 256 + k * 16 + (m & 3) * 4 + ((m & 15) >> 2);
}

// w_b = H_b(theta_t) (T_b^T x_t) for far block b, one 16-column RHS tile and the slots
// t0 .. t0 + HTB - 1; W[(t nrc + tile) hw_tot + w_off + a 16 + c].  On the FP64 matrix cores:
// T_b is theta-independent, so z_t = T_b^T x_t for all HTB slots comes from one pass over T_b,
// with the ranks as 8 row tiles of 16 and the slots as 8 column tiles of 16 right-hand sides
// (wave w owns rank tiles w and w + 4 of every slot); per step 16 rows of T_b (transposed into
// the operand order) and of every slot's x go through LDS.  Then, slot by slot, z_t goes
// through LDS as the B operand and w_t = H' z_t, H' = H_q (or H_q^T for a mirrored class) read
// from the instance 16 columns per step, on the matrix cores again.
__global__ void __launch_bounds__(NT, 2) k_h_proj(const double* __restrict__ xt, double* __restrict__ W,
                                               const HBlkDev* __restrict__ blks, const double* __restrict__ hT,
                                               const double* __restrict__ Hc, int64_t h_tot, int64_t hw_tot,
                                               int64_t n, int64_t Rs, int nrc, int T) {
  typedef Tile16<double> MF;
  __shared__ __attribute__((aligned(16))) double As[8 * 256];   // A panel: 128 x 16, operand order
  __shared__ __attribute__((aligned(16))) double Bs[HTB][256];  // B: 16 x 16 per slot; phase 2: z (128 x 16)
  double* Bz = &Bs[0][0];
  const HBlkDev b = blks[blockIdx.x];
  const int tile = blockIdx.y;
  const int t0 = blockIdx.z * HTB;
  const int tn = min(HTB, T - t0);
  const int r0 = tile * RC;
  const int rc = (int)min<int64_t>(RC, Rs - r0);
  const int lane = threadIdx.x % WAVE, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const double* T_ = hT + b.T_off;
  // row tiles that hold a row below the rank (rows beyond it stay zero): with ranks up to 64
  // every wave keeps one tile and skips the other
  const bool zt[2] = {wave * 16 < b.rt, (wave + 4) * 16 < b.rt};
  const bool wt[2] = {wave * 16 < b.rs, (wave + 4) * 16 < b.rs};
  MF::acc_t acc[HTB][2];
#pragma unroll
  for (int s = 0; s < HTB; ++s)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[s][j] = (MF::acc_t){0, 0, 0, 0};
  // phase 1: z_t = T_b^T x_t, 16 rows of T_b per step.  The next step's T_b and x values are
  // loaded into registers while the current step is multiplied.  Every load is unconditional
  // (T_b: raw buffer loads, zeros at an out-of-range offset; x: clamped addresses), so the
  // wait for them falls at the next step's LDS stores.  Thread tid holds T_b entry (row i0 + tid % 16, rank
  // tid / 16 + 16 p) and x entry (point i0 + tid / 16, column tid % 16) of slot t0 + p.
  // T_b is read through a raw buffer view (below 2 GiB, checked on the host).
  static_assert(NT == 256 && HTB == 8, "staging map: 8 values of T_b and of x per thread");
  const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)T_, (short)0, (int)((int64_t)b.ldt * b.rt * (int64_t)sizeof(double)), BUF_WORD3);
  const int kT = threadIdx.x % 16, aT = threadIdx.x / 16;   // T_b: row in the step, rank mod 16
  const int kX = threadIdx.x / 16, cX = threadIdx.x % 16;   // x: point in the step, column
  double pa[8], pb[HTB];
  auto stage_load = [&](int64_t i0) {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int a = aT + 16 * p;
      const bool ok = a < b.rt && i0 + kT < b.nt;
      pa[p] = bload1<double>(trs, ok ? (int)((i0 + kT + (int64_t)b.ldt * a) * (int64_t)sizeof(double)) : BUF_OOB);
    }
    // x: a plain load from a clamped, valid address; entries outside the block, the tile or
    // the slots are zeroed when stored (xok below), so the load itself is unconditional
#pragma unroll
    for (int p = 0; p < HTB; ++p) {
      const int64_t tp = t0 + min(p, tn - 1), ip = min<int64_t>(i0 + kX, b.nt - 1);
      pb[p] = xt[(tp * n + b.t_begin + ip) * Rs + r0 + min(cX, rc - 1)];
    }
  };
  auto xok = [&](int64_t i0, int p) { return p < tn && i0 + kX < b.nt && cX < rc; };
  if (b.nt > 0) stage_load(0);   // (an empty source cluster has no step and no load)
  for (int64_t i0 = 0; i0 < b.nt; i0 += 16) {
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 8; ++p) As[panel_index(aT + 16 * p, kT)] = pa[p];
#pragma unroll
    for (int p = 0; p < HTB; ++p) Bs[p][threadIdx.x] = xok(i0, p) ? pb[p] : 0.0;
    __syncthreads();
    stage_load(i0 + 16);   // past the last step: T_b offsets out of range, x clamped (unused)
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int k = kk + (lane >> 4);
      MF::a_t av[2];
#pragma unroll
      for (int j = 0; j < 2; ++j)
        if (zt[j]) av[j] = MF::load_tiled(&As[(wave + 4 * j) * 256 + k * 16], lane);
#pragma unroll
      for (int s = 0; s < HTB; ++s) {
        const double bv = Bs[s][k * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (zt[j]) acc[s][j] = MF::mac(av[j], bv, acc[s][j]);
      }
    }
  }
  // phase 2, slot by slot: w_t = H' z_t (rows of H' beyond rs and columns beyond rt are zero).
  // The steps (slot, 16 columns a0 of H') run as one sequence with the next step's H' values
  // prefetched into registers as in phase 1 (clamped addresses, masked when stored).  Thread
  // tid holds entry (row ap, column a0 + kk) of H' for p < 8: H' = H^T (tr), H[a + rt ap]
  // with a contiguous: kk = tid % 16, ap = tid / 16 + 16 p; H' = H, H[ap + rs a] with ap
  // contiguous: ap = tid % 128, kk = tid / 128 + 2 p.  A block of rank 0 on either side has
  // no step (its w is zero).
  const bool hsteps = b.rs > 0 && b.rt > 0;
  auto h_ap = [&](int p) { return b.tr ? (int)threadIdx.x / 16 + 16 * p : (int)threadIdx.x % 128; };
  auto h_kk = [&](int p) { return b.tr ? (int)threadIdx.x % 16 : (int)threadIdx.x / 128 + 2 * p; };
  double ph[8];
  auto h_load = [&](int s, int a0) {
    const double* H = Hc + (int64_t)(t0 + s) * h_tot + b.h_off;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int ap = min(h_ap(p), b.rs - 1), a = min(a0 + h_kk(p), b.rt - 1);
      ph[p] = b.tr ? H[a + (int64_t)b.rt * ap] : H[ap + (int64_t)b.rs * a];
    }
  };
  if (hsteps) h_load(0, 0);
#pragma unroll
  for (int s = 0; s < HTB; ++s) {
    if (s >= tn) break;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) Bz[((wave + 4 * j) * 16 + MF::row(lane, q)) * 16 + (lane & 15)] = acc[s][j][q];
    const int64_t slot = t0 + s;
    MF::acc_t w2[2] = {(MF::acc_t){0, 0, 0, 0}, (MF::acc_t){0, 0, 0, 0}};
    for (int a0 = 0; hsteps && a0 < b.rt; a0 += 16) {
      // the step after (s, a0); past the last one the current step's addresses are re-read
      int sn = s, an = a0 + 16;
      if (an >= b.rt) {
        an = 0;
        sn = s + 1;
      }
      __syncthreads();
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int ap = h_ap(p), kk = h_kk(p);
        As[panel_index(ap, kk)] = ap < b.rs && a0 + kk < b.rt ? ph[p] : 0.0;
      }
      __syncthreads();
      if (sn < tn) h_load(sn, an);
      else h_load(s, a0);
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const int k = kk + (lane >> 4);
        const double bv = Bz[(a0 + k) * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (!wt[j]) continue;   // rows of w beyond rs are not stored
          const MF::a_t av = MF::load_tiled(&As[(wave + 4 * j) * 256 + k * 16], lane);
          w2[j] = MF::mac(av, bv, w2[j]);
        }
      }
    }
    double* w = W + (slot * nrc + tile) * hw_tot + b.w_off;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ap = (wave + 4 * j) * 16 + MF::row(lane, q);
        if (ap < b.rs) w[ap * 16 + (lane & 15)] = w2[j][q];
      }
  }
}

// yt[rows] (+)= sum over the far blocks b whose target contains the rows of S_b[rows] w_b, for
// one (leaf, 128-row chunk) item, one RHS tile and the slots t0 .. t0 + HTB - 1, on the FP64
// matrix cores: the chunk's rows are 8 row tiles of 16 and the slots 8 column tiles of 16
// right-hand sides (wave w owns row tiles w and w + 4 of every slot).  Per step 16 columns of
// S_b (the chunk's rows, in the operand order) and the matching 16 rows of w_b of every slot go
// through LDS, so S_b is read once for all HTB slots.  ADD: the sum is added to yt; else it is
// written (an item with no blocks then writes zeros).
template <bool ADD>
__global__ void __launch_bounds__(NT, 2) k_h_apply(double* __restrict__ yt, const double* __restrict__ W,
                                                const HBlkDev* __restrict__ blks, const double* __restrict__ hS,
                                                const int32_t* __restrict__ leaf_ptr,
                                                const int32_t* __restrict__ leaf_blk, const int64_t* __restrict__ nbegin,
                                                const int64_t* __restrict__ nend, const int32_t* __restrict__ items,
                                                int32_t leaf0, int64_t hw_tot, int64_t n, int64_t Rs, int nrc, int T) {
  typedef Tile16<double> MF;
  constexpr int CH = 128;
  __shared__ __attribute__((aligned(16))) double As[8 * 256];   // 128 rows x 16 columns of S_b
  __shared__ __attribute__((aligned(16))) double Bs[HTB][256];  // 16 rows of w_b per slot
  const int li = items[2 * blockIdx.x], cstart = items[2 * blockIdx.x + 1];
  const int32_t leaf = leaf0 + li;
  const int tile = blockIdx.y;
  const int t0 = blockIdx.z * HTB;
  const int tn = min(HTB, T - t0);
  const int r0 = tile * RC;
  const int rc = (int)min<int64_t>(RC, Rs - r0);
  const int lane = threadIdx.x % WAVE, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int64_t lb = nbegin[leaf], ln = nend[leaf] - lb;
  const int cn = (int)min<int64_t>(CH, ln - cstart);
  // row tiles that hold a row of the chunk (with chunks of up to 64 rows every wave keeps one)
  const bool rt_[2] = {wave * 16 < cn, (wave + 4) * 16 < cn};
  MF::acc_t acc[HTB][2];
#pragma unroll
  for (int s = 0; s < HTB; ++s)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[s][j] = (MF::acc_t){0, 0, 0, 0};
  // The steps (block e of the chunk's list, 16 columns a0 of S_b) run as one sequence, and the
  // next step's S_b and w values are loaded into registers while the current one is
  // multiplied.  Thread tid holds S_b entry (chunk row tid % 128, column a0 + tid / 128 + 2 p)
  // and w entry (row a0 + tid / 16, column tid % 16) of slot t0 + p.  The loads use clamped,
  // valid addresses and are masked when stored, so they are unconditional and the wait for
  // them falls at the next step's LDS stores; blocks of rank 0 have no step.
  static_assert(NT == 256 && HTB == 8 && CH == 128, "staging map: 8 values of S_b and of w per thread");
  const int rS = threadIdx.x % CH, kS = threadIdx.x / CH;   // S_b: chunk row, column mod 2
  const int kW = threadIdx.x / 16, cW = threadIdx.x % 16;   // w: row in the step, column
  const int e1 = leaf_ptr[li + 1];
  auto seek = [&](int e, HBlkDev& bb) {   // first block at or after e with a step
    for (; e < e1; ++e) {
      bb = blks[leaf_blk[e]];
      if (bb.rs > 0) break;
    }
    return e;
  };
  double pa[8], pb[HTB];
  auto stage_load = [&](const HBlkDev& bb, int a0) {
    // rows of the chunk relative to the block's target cluster
    const double* S = hS + bb.S_off + (lb + cstart - bb.s_begin) + min(rS, cn - 1);
#pragma unroll
    for (int p = 0; p < 8; ++p) pa[p] = S[(int64_t)bb.lds * min(a0 + kS + 2 * p, bb.rs - 1)];
#pragma unroll
    for (int p = 0; p < HTB; ++p)
      pb[p] = W[((int64_t)(t0 + min(p, tn - 1)) * nrc + tile) * hw_tot + bb.w_off + min(a0 + kW, bb.rs - 1) * 16 + cW];
  };
  HBlkDev b{};
  int e = cn > 0 ? seek(leaf_ptr[li], b) : e1, a0 = 0;
  if (e < e1) stage_load(b, 0);
  while (e < e1) {
    // the step after (e, a0); past the last one the current step's addresses are re-read
    HBlkDev bn = b;
    int en = e, an = a0 + 16;
    if (an >= b.rs) {
      an = 0;
      en = seek(e + 1, bn);
    }
    {
      __syncthreads();
#pragma unroll
      for (int p = 0; p < 8; ++p)
        As[panel_index(rS, kS + 2 * p)] = rS < cn && a0 + kS + 2 * p < b.rs ? pa[p] : 0.0;
#pragma unroll
      for (int p = 0; p < HTB; ++p) Bs[p][threadIdx.x] = p < tn && a0 + kW < b.rs ? pb[p] : 0.0;
      __syncthreads();
      if (en < e1) stage_load(bn, an);
      else stage_load(b, a0);
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const int k = kk + (lane >> 4);
        MF::a_t av[2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (rt_[j]) av[j] = MF::load_tiled(&As[(wave + 4 * j) * 256 + k * 16], lane);
#pragma unroll
        for (int s = 0; s < HTB; ++s) {
          const double bv = Bs[s][k * 16 + (lane & 15)];
#pragma unroll
          for (int j = 0; j < 2; ++j)
            if (rt_[j]) acc[s][j] = MF::mac(av[j], bv, acc[s][j]);
        }
      }
    }
    e = en;
    a0 = an;
    b = bn;
  }
  const int c = lane & 15;
  if (c >= rc) return;
#pragma unroll
  for (int s = 0; s < HTB; ++s) {
    if (s >= tn) break;
    double* y = yt + ((int64_t)(t0 + s) * n + lb + cstart) * Rs + r0 + c;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = (wave + 4 * j) * 16 + MF::row(lane, q);
        if (r < cn) {
          if (ADD) y[(int64_t)r * Rs] += acc[s][j][q];
          else y[(int64_t)r * Rs] = acc[s][j][q];
        }
      }
  }
}

void h_core_launch(const InstData& in, hipStream_t st) {
  const DeviceModel& m = *in.m;
  if (m.n_hcls == 0) return;
  launch(PH_STAGE_FAR_INST, k_h_core, dim3((unsigned)m.n_hcls, (unsigned)in.T), dim3(NT), st,
         (const HClsDev*)m.hcls.p, (const double*)m.hcore.p, (const double*)m.ff_theta.p, (const double*)in.v.p,
         (double*)in.C.p, m.h_tot, m.p_theta, m.d_theta);
}

// The projection reads T_b through a raw buffer view of 32-bit range.
static void h_buffer_check(const DeviceModel& m) {
  if (m.h_tbytes_max > BUF_MAX_BYTES) fail(PH_EUNSUPPORTED, "ph_matvec: a far block's T_b exceeds 2 GiB");
}

void h_far_launch(const InstData& in, const double* xt, double* yt, double* W, int64_t Rs, int64_t nrc,
                  hipStream_t st, int phase) {
  const DeviceModel& m = *in.m;
  if (m.n_hblk == 0) return;
  if (in.T > 65535 || nrc > 65535) fail(PH_EUNSUPPORTED, "ph_matvec: too many parameter slots or RHS tiles");
  const unsigned nb = (unsigned)((in.T + HTB - 1) / HTB);
  h_buffer_check(m);
  if (phase == 0)
    launch(PH_STAGE_COUPLING, k_h_proj, dim3((unsigned)m.n_hblk, (unsigned)nrc, nb), dim3(NT), st, xt, W,
           (const HBlkDev*)m.hblk.p, (const double*)m.hT.p, (const double*)in.C.p, m.h_tot, m.hw_tot, m.n, Rs,
           (int)nrc, in.T);
  else
    launch(PH_STAGE_LEAF_DOWN, k_h_apply<true>, dim3((unsigned)m.n_mvm_items, (unsigned)nrc, nb), dim3(NT), st, yt,
           (const double*)W, (const HBlkDev*)m.hblk.p, (const double*)m.hS.p, (const int32_t*)m.hl_ptr.p,
           (const int32_t*)m.hl_blk.p, (const int64_t*)m.nbegin.p, (const int64_t*)m.nend.p,
           (const int32_t*)m.mvm_items.p, m.tree->leaves.front(), m.hw_tot, m.n, Rs, (int)nrc, in.T);
}

// Alg. "Modified H^2-Matrix MVM", multiplication stage with the couplings kept as factors: the
// far blocks are the H-matrix kernels' blocks over the index space of x_hat (node s, entry i at
// row s Pp + i): w_b = H_q(theta) R_q^T x_hat_t, then y_hat_s = sum_b L_q w_b per node (written,
// so nodes of the far levels without far blocks get zeros for the downward pass).
void implicit_coupling_launch(const InstData& in, const double* xh, double* yh, double* W, int64_t Rs,
                              int64_t nrc, hipStream_t st) {
  const DeviceModel& m = *in.m;
  if (in.T > 65535 || nrc > 65535) fail(PH_EUNSUPPORTED, "ph_matvec: too many parameter slots or RHS tiles");
  const unsigned nb = (unsigned)((in.T + HTB - 1) / HTB);
  h_buffer_check(m);
  const int64_t rows = m.n_nodes * m.Pp;
  if (m.n_hblk > 0)
    launch(PH_STAGE_COUPLING, k_h_proj, dim3((unsigned)m.n_hblk, (unsigned)nrc, nb), dim3(NT), st, xh, W,
           (const HBlkDev*)m.hblk.p, (const double*)m.hS.p, (const double*)in.C.p, m.h_tot, m.hw_tot, rows, Rs,
           (int)nrc, in.T);
  if (m.n_hx_items > 0)
    launch(PH_STAGE_COUPLING, k_h_apply<false>, dim3((unsigned)m.n_hx_items, (unsigned)nrc, nb), dim3(NT), st, yh,
           (const double*)W, (const HBlkDev*)m.hblk.p, (const double*)m.hS.p, (const int32_t*)m.hl_ptr.p,
           (const int32_t*)m.hl_blk.p, (const int64_t*)m.hx_nbegin.p, (const int64_t*)m.hx_nend.p,
           (const int32_t*)m.hx_items.p, (int32_t)0, m.hw_tot, rows, Rs, (int)nrc, in.T);
}

}  // namespace ph
