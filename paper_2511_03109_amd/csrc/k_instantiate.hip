// Online stage kernels (arxiv 2511.03109, Alg. "Online Stage" and Alg. PTTK online):
// parametric vectors, far-field couplings C(theta) = L H(theta) R^T (Sec. 4.2) and
// near-field blocks D_b(theta) = reshape(P_b c_b(theta), [n_s, n_t]) (Sec. 4.3).
// No kernel evaluation happens here.
#include <cstring>

#include "ph_device.hpp"

namespace ph {

struct ThetaBox {
  double lo[2], hi[2];
};

// v[(t*dth + k)*p + i] = l_i(theta_{t,k}) on [lo_k, hi_k] with first-kind Chebyshev
// nodes (product formula, Sec. 2.2); its derivative for k == grad_dim.  theta is a
// device array T x dth (so that a recorded graph can be replayed with new values).
__global__ void k_theta_vectors(const double* __restrict__ theta, ThetaBox box, double* __restrict__ v, int T,
                                int dth, int p, int grad_dim) {
  const int total = T * dth * p;
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < total; o += gridDim.x * blockDim.x) {
    const int i = o % p;
    const int k = (o / p) % dth;
    const int t = o / (p * dth);
    const double a = box.lo[k], b = box.hi[k], x = theta[t * dth + k];
    double nodes[16];
    for (int q = 0; q < p; ++q)
      nodes[q] = (a + b) / 2.0 - (b - a) / 2.0 * cos((2.0 * (q + 1) - 1.0) * M_PI / (2.0 * p));
    double val;
    if (k != grad_dim) {
      val = 1.0;
      for (int q = 0; q < p; ++q)
        if (q != i) val *= (x - nodes[q]) / (nodes[i] - nodes[q]);
    } else {
      val = 0.0;
      for (int m = 0; m < p; ++m) {
        if (m == i) continue;
        double term = 1.0 / (nodes[i] - nodes[m]);
        for (int q = 0; q < p; ++q)
          if (q != i && q != m) term *= (x - nodes[q]) / (nodes[i] - nodes[q]);
        val += term;
      }
    }
    v[((size_t)t * dth + k) * p + i] = val;
  }
}

// Far field, one workgroup per (stored class, slot).
//   w_k = Theta_k^T v_k;  H = core x_theta w  (r_L x r_R, global scratch);
//   St = (H R^T)^T, i.e. St[j + Pp a] = sum_b R[j, b] H[a, b]     (MFMA, M = j, N = a, K = b);
//   C[i + Pp j] = sum_a L[i, a] St[j + Pp a]                     (MFMA, M = i, N = j, K = a);
// the mirrored class receives C^T.  All Pp x Pp entries are written (zero padding), in
// fragment order (frag_index).
template <typename S>
__global__ void __launch_bounds__(NT) k_far_instantiate(
    const ClassDev* __restrict__ cls, const double* __restrict__ L, const double* __restrict__ R,
    const double* __restrict__ core, const double* __restrict__ th, const double* __restrict__ v,
    double* __restrict__ scratch, int64_t scratch_per_slot, S* __restrict__ C, int64_t C_per_slot,
    int P, int Pp, int p, int dth) {
  typedef Mfma<double> MF;
  __shared__ double w1[16], w2[16];
  const ClassDev c = cls[blockIdx.x];
  const int t = blockIdx.y;
  const int lane = threadIdx.x % WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
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
  const int rL = c.rL, rR = c.rR;
  const int rLp = (rL + 15) / 16 * 16;
  double* H = scratch + (size_t)t * scratch_per_slot + c.S_off;
  double* St = H + (size_t)rL * rR;
  for (int o = threadIdx.x; o < rL * rR; o += blockDim.x) {
    const int a = o % rL, b = o / rL;
    double s = 0;
    for (int k2 = 0; k2 < c.r2; ++k2)
      for (int k1 = 0; k1 < c.r1; ++k1)
        s += core[c.core_off + a + (size_t)rL * (k1 + (size_t)c.r1 * (k2 + (size_t)c.r2 * b))] * w1[k1] *
             w2[k2];
    H[o] = s;
  }
  __threadfence_block();
  __syncthreads();
  const int m16 = lane & 15, kq = lane >> 4;
  // St (Pp x rLp): tiles (jt, at)
  {
    const int nj = Pp / 16, na = rLp / 16;
    for (int tile = wave; tile < nj * na; tile += NT / WAVE) {
      const int jt = tile % nj, at = tile / nj;
      MF::acc_t acc = {0, 0, 0, 0};
      const int j = jt * 16 + m16, a = at * 16 + m16;
      for (int b0 = 0; b0 < rR; b0 += 4) {
        const int b = b0 + kq;
        const double av = (j < P && b < rR) ? R[c.R_off + j + (size_t)P * b] : 0.0;
        const double bv = (a < rL && b < rR) ? H[a + (size_t)rL * b] : 0.0;
        acc = MF::mac(av, bv, acc);
      }
      for (int i = 0; i < 4; ++i) St[(jt * 16 + MF::row(lane, i)) + (size_t)Pp * (at * 16 + m16)] = acc[i];
    }
  }
  __threadfence_block();
  __syncthreads();
  S* Ct = C + (size_t)t * C_per_slot;
  {
    const int nt = Pp / 16;
    for (int tile = wave; tile < nt * nt; tile += NT / WAVE) {
      const int it = tile % nt, jt = tile / nt;
      MF::acc_t acc = {0, 0, 0, 0};
      const int i = it * 16 + m16, j = jt * 16 + m16;
      for (int a0 = 0; a0 < rL; a0 += 4) {
        const int a = a0 + kq;
        const double av = (i < P && a < rL) ? L[c.L_off + i + (size_t)P * a] : 0.0;
        const double bv = (a < rL) ? St[j + (size_t)Pp * a] : 0.0;
        acc = MF::mac(av, bv, acc);
      }
      for (int q = 0; q < 4; ++q) {
        const int row = it * 16 + MF::row(lane, q);
        Ct[c.C_off + frag_index(row, j, Pp)] = (S)acc[q];
        if (c.Cm_off >= 0) Ct[c.Cm_off + frag_index(j, row, Pp)] = (S)acc[q];
      }
    }
  }
}

// Near field, one workgroup per TILE x TILE tile of a stored block, all slots:
//   c_t = core x_theta (Theta_k^T v_k(theta_t));  D_t[i + j n_s] = sum_k P[k][i + j n_s] c_t[k]
// Each factor entry is read from HBM once for up to TC slots; D_t is written to the
// (s, t) block and, through an LDS transpose, to the (t, s) block.
template <typename DT>
__global__ void __launch_bounds__(NT) k_near_instantiate(
    const NearDev* __restrict__ blocks, const int32_t* __restrict__ tiles,
    const double* __restrict__ Pf, const double* __restrict__ core, const double* __restrict__ th,
    const double* __restrict__ v, DT* __restrict__ D, int64_t D_per_slot, int T, int p, int dth) {
  __shared__ double w1[TC][16], w2[TC][16], cc[TC][256];
  __shared__ double tile[TILE][TILE + 1];
  const int32_t bi = tiles[3 * blockIdx.x], i0 = tiles[3 * blockIdx.x + 1], j0 = tiles[3 * blockIdx.x + 2];
  const NearDev b = blocks[bi];
  const int64_t Nep = (int64_t)b.ldp * b.nt;                     // padded factor column length
  const int ti = threadIdx.x % TILE, tj0 = threadIdx.x / TILE;   // 8 rows of 32
  const int i = i0 + ti;
  constexpr int NQ = TILE / (NT / TILE);                          // 4 entries per thread
  for (int t0 = 0; t0 < T; t0 += TC) {
    const int tc = min(TC, T - t0);
    __syncthreads();
    for (int o = threadIdx.x; o < tc * b.r1; o += NT) {
      const int tt = o / b.r1, a = o % b.r1;
      const double* vt = v + (size_t)(t0 + tt) * dth * p;
      double s = 0;
      for (int q = 0; q < p; ++q) s += th[b.th1_off + q + (size_t)p * a] * vt[q];
      w1[tt][a] = s;
    }
    for (int o = threadIdx.x; o < tc * b.r2; o += NT) {
      const int tt = o / b.r2, a = o % b.r2;
      double s = 1.0;
      if (dth == 2) {
        const double* vt = v + (size_t)(t0 + tt) * dth * p;
        s = 0;
        for (int q = 0; q < p; ++q) s += th[b.th2_off + q + (size_t)p * a] * vt[p + q];
      }
      w2[tt][a] = s;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < tc * b.r_e; o += NT) {
      const int tt = o / b.r_e, k = o % b.r_e;
      double s = 0;
      for (int k2 = 0; k2 < b.r2; ++k2)
        for (int k1 = 0; k1 < b.r1; ++k1)
          s += core[b.core_off + k + (size_t)b.r_e * (k1 + (size_t)b.r1 * k2)] * w1[tt][k1] * w2[tt][k2];
      cc[tt][k] = s;
    }
    __syncthreads();
    double acc[TC][NQ];
    for (int tt = 0; tt < TC; ++tt)
      for (int q = 0; q < NQ; ++q) acc[tt][q] = 0.0;
    bool ok[NQ];
    int64_t e[NQ], ed[NQ];
    for (int q = 0; q < NQ; ++q) {
      const int j = j0 + tj0 + q * (NT / TILE);
      ok[q] = i < b.ns && j < b.nt;
      e[q] = ok[q] ? i + (int64_t)j * b.ldp : 0;
      ed[q] = ok[q] ? i + (int64_t)j * b.lds : 0;
    }
    const double* pb = Pf + b.P_off;
    int k = 0;
    for (; k < b.r_e; ++k) {
      double pv[NQ];
      for (int q = 0; q < NQ; ++q) pv[q] = ok[q] ? pb[(size_t)k * Nep + e[q]] : 0.0;
#pragma unroll
      for (int tt = 0; tt < TC; ++tt) {
        const double cv = cc[tt][k];
        for (int q = 0; q < NQ; ++q) acc[tt][q] += pv[q] * cv;
      }
    }
#pragma unroll
    for (int tt = 0; tt < TC; ++tt) {
      if (tt >= tc) break;
      DT* Dt = D + (size_t)(t0 + tt) * D_per_slot;
      for (int q = 0; q < NQ; ++q)
        if (ok[q]) Dt[b.D_st + ed[q]] = to_store<DT>(acc[tt][q]);
      if (b.D_ts >= 0) {
        __syncthreads();
        for (int q = 0; q < NQ; ++q) tile[tj0 + q * (NT / TILE)][ti] = acc[tt][q];
        __syncthreads();
        // transposed block (t, s): element (j, i) at j + i n_t
        const int jj = j0 + ti;
        for (int q = 0; q < NQ; ++q) {
          const int ii = i0 + tj0 + q * (NT / TILE);
          if (ii < b.ns && jj < b.nt) Dt[b.D_ts + jj + (int64_t)ii * b.ldt] = to_store<DT>(tile[ti][tj0 + q * (NT / TILE)]);
        }
      }
    }
  }
}

template <typename S, typename DT>
void instantiate_impl(InstData& in, const double* theta, hipStream_t st) {
  const DeviceModel& m = *in.m;
  // theta -> pinned staging -> device.  The staging buffer is rewritten only after the
  // previous copy out of it has run (ev_theta); under graph capture the copy becomes a
  // graph node that reads the staging buffer at replay time.
  const size_t nth = (size_t)in.T * m.d_theta;
  if (theta) {
    if (in.theta_pending) PH_HIP(hipEventSynchronize(in.ev_theta));
    std::memcpy(in.theta_pin, theta, nth * sizeof(double));
  }
  PH_HIP(hipMemcpyAsync(in.theta_d.p, in.theta_pin, nth * sizeof(double), hipMemcpyHostToDevice, st));
  if (!g_capturing) {
    PH_HIP(hipEventRecord(in.ev_theta, st));
    in.theta_pending = true;
  }
  ThetaBox box{};
  for (int k = 0; k < 2; ++k) {
    box.lo[k] = m.th_lo[k];
    box.hi[k] = m.th_hi[k];
  }
  const int64_t nv = (int64_t)in.T * m.d_theta * m.p_theta;
  launch(PH_STAGE_THETA, k_theta_vectors, dim3((unsigned)grid_for(nv)), dim3(NT), st, (const double*)in.theta_d.p,
         box, in.v.p, in.T, m.d_theta, m.p_theta, in.grad_dim);
  const int64_t Cps = m.n_classes * m.Pp * m.Pp;
  launch(PH_STAGE_FAR_INST, k_far_instantiate<S>, dim3((unsigned)m.n_stored_cls, in.T), dim3(NT), st,
         (const ClassDev*)m.cstore.p, (const double*)m.ff_L.p, (const double*)m.ff_R.p,
         (const double*)m.ff_core.p, (const double*)m.ff_theta.p, (const double*)in.v.p, in.ffs.p,
         m.ff_scratch, (S*)in.C.p, Cps, m.P, m.Pp, m.p_theta, m.d_theta);
  launch(PH_STAGE_NEAR_INST, k_near_instantiate<DT>, dim3((unsigned)m.n_tiles), dim3(NT), st,
         (const NearDev*)m.nstore.p, (const int32_t*)m.tiles.p, (const double*)m.nf_P.p,
         (const double*)m.nf_core.p, (const double*)m.nf_theta.p, (const double*)in.v.p, (DT*)in.D.p,
         m.N_nf_pad, in.T, m.p_theta, m.d_theta);
}

template void instantiate_impl<double, double>(InstData&, const double*, hipStream_t);
template void instantiate_impl<float, float>(InstData&, const double*, hipStream_t);
template void instantiate_impl<float, bf16>(InstData&, const double*, hipStream_t);

}  // namespace ph
