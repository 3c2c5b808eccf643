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
constexpr int HCH = 16;   // rows of T_b / ranks of S_b staged per step

// w_b = H_b(theta_t) (T_b^T x_t) for far block b, one 16-column RHS tile and the slots
// t0 .. t0 + HTB - 1; W[(t nrc + tile) hw_tot + w_off + a 16 + c].  T_b is theta-independent, so
// z_t = T_b^T x_t for all HTB slots comes from one pass over T_b: thread (g, c) = (tid / 16,
// tid % 16) owns ranks g, g + 16, ... and RHS column c of every slot.  Rows of T_b and of the
// slots' x go through LDS in chunks of HCH.  Then, slot by slot, z_t goes through LDS and
// w_t = H' z_t, H' = H_q (or H_q^T for a mirrored class) read from the instance.
__global__ void __launch_bounds__(NT) k_h_proj(const double* __restrict__ xt, double* __restrict__ W,
                                               const HBlkDev* __restrict__ blks, const double* __restrict__ hT,
                                               const double* __restrict__ Hc, int64_t h_tot, int64_t hw_tot,
                                               int64_t n, int64_t Rs, int nrc, int T) {
  // phase 1 (z = T_b^T x for all slots) uses Ts and xs, phase 2 (w = H' z per slot) zs and Hs
  constexpr int P1 = HCH * 129 + HTB * HCH * 16, P2 = 128 * 17 + 128 * (HCH + 1);
  __shared__ double smem[P1 > P2 ? P1 : P2];
  double(*Ts)[129] = reinterpret_cast<double(*)[129]>(smem);
  double(*xs)[HCH][16] = reinterpret_cast<double(*)[HCH][16]>(smem + HCH * 129);
  double(*zs)[17] = reinterpret_cast<double(*)[17]>(smem);
  double(*Hs)[HCH + 1] = reinterpret_cast<double(*)[HCH + 1]>(smem + 128 * 17);
  const HBlkDev b = blks[blockIdx.x];
  const int tile = blockIdx.y;
  const int t0 = blockIdx.z * HTB;
  const int tn = min(HTB, T - t0);
  const int r0 = tile * RC;
  const int rc = (int)min<int64_t>(RC, Rs - r0);
  const int c = threadIdx.x % 16, g = threadIdx.x / 16;
  const double* T_ = hT + b.T_off;
  double acc[HTB][8];
#pragma unroll
  for (int s = 0; s < HTB; ++s)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[s][j] = 0;
  for (int64_t i0 = 0; i0 < b.nt; i0 += HCH) {
    const int cn = (int)min<int64_t>(HCH, b.nt - i0);
    __syncthreads();
    for (int e = threadIdx.x; e < HTB * HCH * 16; e += NT) {
      const int ts = e / (HCH * 16), ii = (e / 16) % HCH, cc = e % 16;
      xs[ts][ii][cc] = (ts < tn && ii < cn && cc < rc)
                           ? xt[((int64_t)(t0 + ts) * n + b.t_begin + i0 + ii) * Rs + r0 + cc] : 0.0;
    }
    for (int e = threadIdx.x; e < HCH * b.rt; e += NT) {
      const int ii = e % HCH, a = e / HCH;
      Ts[ii][a] = ii < cn ? T_[i0 + ii + (int64_t)b.ldt * a] : 0.0;
    }
    __syncthreads();
    for (int ii = 0; ii < cn; ++ii) {
      double tv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) tv[j] = Ts[ii][min(g + 16 * j, 127)];
#pragma unroll
      for (int s = 0; s < HTB; ++s) {
        const double xv = xs[s][ii][c];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[s][j] += tv[j] * xv;
      }
    }
  }
  for (int s = 0; s < tn; ++s) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int a = g + 16 * j;
      if (a < b.rt) zs[a][c] = acc[s][j];
    }
    const int64_t slot = t0 + s;
    const double* H = Hc + slot * h_tot + b.h_off;
    double wacc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) wacc[j] = 0;
    // H' in column chunks of HCH through LDS (coalesced reads of H_q or of H_q^T's rows)
    for (int a0 = 0; a0 < b.rt; a0 += HCH) {
      const int an = min(HCH, b.rt - a0);
      __syncthreads();
      for (int e = threadIdx.x; e < b.rs * HCH; e += NT) {
        int ap, aa;
        if (b.tr) { aa = e % HCH; ap = e / HCH; }
        else { ap = e % b.rs; aa = e / b.rs; }
        Hs[ap][aa] = aa < an ? (b.tr ? H[a0 + aa + (int64_t)b.rt * ap] : H[ap + (int64_t)b.rs * (a0 + aa)]) : 0.0;
      }
      __syncthreads();
      for (int aa = 0; aa < an; ++aa) {
        const double zv = zs[a0 + aa][c];
#pragma unroll
        for (int j = 0; j < 8; ++j) wacc[j] += Hs[min(g + 16 * j, 127)][aa] * zv;
      }
    }
    double* w = W + (slot * nrc + tile) * hw_tot + b.w_off;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int ap = g + 16 * j;
      if (ap < b.rs) w[ap * 16 + c] = wacc[j];
    }
  }
}

// yt[rows] += sum over the far blocks b whose target contains the rows of S_b[rows] w_b, for one
// (leaf, 128-row chunk) item, one RHS tile and the slots t0 .. t0 + HTB - 1.  Thread (g, c) owns
// rows g, g + 16, ... of the chunk and RHS column c of every slot; HCH columns of S_b (the chunk's
// rows) and the matching rows of w_b of every slot go through LDS per step, so S_b is read once
// for all HTB slots.  ADD: the sum is added to yt; else it is written (an item with no blocks
// then writes zeros).
template <bool ADD>
__global__ void __launch_bounds__(NT) k_h_apply(double* __restrict__ yt, const double* __restrict__ W,
                                                const HBlkDev* __restrict__ blks, const double* __restrict__ hS,
                                                const int32_t* __restrict__ leaf_ptr,
                                                const int32_t* __restrict__ leaf_blk, const int64_t* __restrict__ nbegin,
                                                const int64_t* __restrict__ nend, const int32_t* __restrict__ items,
                                                int32_t leaf0, int64_t hw_tot, int64_t n, int64_t Rs, int nrc, int T) {
  constexpr int CH = 128;
  __shared__ double Ss[HCH][CH + 1];
  __shared__ double ws[HTB][HCH][16];
  const int li = items[2 * blockIdx.x], cstart = items[2 * blockIdx.x + 1];
  const int32_t leaf = leaf0 + li;
  const int tile = blockIdx.y;
  const int t0 = blockIdx.z * HTB;
  const int tn = min(HTB, T - t0);
  const int r0 = tile * RC;
  const int rc = (int)min<int64_t>(RC, Rs - r0);
  const int c = threadIdx.x % 16, g = threadIdx.x / 16;
  const int64_t lb = nbegin[leaf], ln = nend[leaf] - lb;
  const int cn = (int)min<int64_t>(CH, ln - cstart);
  double acc[HTB][8];
#pragma unroll
  for (int s = 0; s < HTB; ++s)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[s][j] = 0;
  for (int e = leaf_ptr[li]; e < leaf_ptr[li + 1]; ++e) {
    const HBlkDev b = blks[leaf_blk[e]];
    // rows of the chunk relative to the block's target cluster
    const double* S = hS + b.S_off + (lb + cstart - b.s_begin);
    for (int a0 = 0; a0 < b.rs; a0 += HCH) {
      const int an = min(HCH, b.rs - a0);
      __syncthreads();
      for (int q = threadIdx.x; q < HCH * CH; q += NT) {
        const int aa = q / CH, r = q % CH;
        Ss[aa][r] = (aa < an && r < cn) ? S[r + (int64_t)b.lds * (a0 + aa)] : 0.0;
      }
      for (int q = threadIdx.x; q < HTB * HCH * 16; q += NT) {
        const int ts = q / (HCH * 16), aa = (q / 16) % HCH, cc = q % 16;
        ws[ts][aa][cc] = (ts < tn && aa < an) ? W[((int64_t)(t0 + ts) * nrc + tile) * hw_tot + b.w_off + (a0 + aa) * 16 + cc]
                                              : 0.0;
      }
      __syncthreads();
      for (int aa = 0; aa < an; ++aa) {
        double sv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) sv[j] = Ss[aa][g + 16 * j];
#pragma unroll
        for (int s = 0; s < HTB; ++s) {
          const double wv = ws[s][aa][c];
#pragma unroll
          for (int j = 0; j < 8; ++j) acc[s][j] += sv[j] * wv;
        }
      }
    }
  }
  if (c >= rc) return;
  for (int s = 0; s < tn; ++s) {
    double* y = yt + ((int64_t)(t0 + s) * n + lb + cstart) * Rs + r0 + c;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int r = g + 16 * j;
      if (r < cn) {
        if (ADD) y[(int64_t)r * Rs] += acc[s][j];
        else y[(int64_t)r * Rs] = acc[s][j];
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

void h_far_launch(const InstData& in, const double* xt, double* yt, double* W, int64_t Rs, int64_t nrc,
                  hipStream_t st, int phase) {
  const DeviceModel& m = *in.m;
  if (m.n_hblk == 0) return;
  if (in.T > 65535 || nrc > 65535) fail(PH_EUNSUPPORTED, "ph_matvec: too many parameter slots or RHS tiles");
  const unsigned nb = (unsigned)((in.T + HTB - 1) / HTB);
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
