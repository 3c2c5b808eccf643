// Online stage kernels (arxiv 2511.03109, Alg. "Online Stage" and Alg. PTTK online):
// parametric vectors, far-field couplings C(theta) = L H(theta) R^T (Sec. 4.2) and
// near-field blocks D_b(theta) = reshape(P_b c_b(theta), [n_s, n_t]) (Sec. 4.3).
// No kernel evaluation happens here.
#include <cstdlib>
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

// Far field, one workgroup per (FT consecutive 16 x 16 tiles of the Pp x Pp coupling, stored
// class), all slots:  w_k = Theta_k^T v_k(theta_t);  C_t = sum_q w_1[k_1] w_2[k_2] Chat_q
// (Sec. 4.2, C = L H(theta) R^T with H linear in the weights, the panels L G_q R^T formed
// offline).  C is in fragment order, where a 16 x 16 tile is 256 contiguous entries, so
// thread p reads and writes entry p of each of its tiles; the mirrored class receives C^T
// (entry (k, m) of the transposed tile).  The weights are formed once per workgroup and
// the FT tiles' panel loads of each q are in flight together.
template <typename S, int FT>
__global__ void __launch_bounds__(NT) k_far_instantiate(const ClassDev* __restrict__ cls,
                                                        const double* __restrict__ chat,
                                                        const double* __restrict__ th, const double* __restrict__ v,
                                                        S* __restrict__ C, int64_t C_per_slot, int Pp, int T, int p,
                                                        int dth) {
  __shared__ double w1[TC][16], w2[TC][16];
  const ClassDev c = cls[blockIdx.y];
  const int nMt = Pp / 16, ntiles = nMt * nMt;
  const int pos = threadIdx.x;                                   // entry of the tile
  const int kl = pos >> 4, ml = (pos & 3) * 4 + ((pos & 15) >> 2);
  int64_t at[FT], mirror_at[FT];
  bool ok[FT];
#pragma unroll
  for (int u = 0; u < FT; ++u) {
    const int tile = blockIdx.x * FT + u;
    ok[u] = tile < ntiles;
    const int mt = tile % nMt, kc = tile / nMt;
    const int m = mt * 16 + ml, k = kc * 16 + kl;
    at[u] = (int64_t)kc * Pp * 16 + mt * 256 + pos;              // = frag_index(m, k)
    mirror_at[u] = frag_index(k, m, Pp);
  }
  const int rq = c.r1 * c.r2;
  const double* cp = chat + c.chat_off;
  for (int t0 = 0; t0 < T; t0 += TC) {
    const int tc = min(TC, T - t0);
    __syncthreads();
    for (int o = threadIdx.x; o < tc * c.r1; o += NT) {
      const int tt = o / c.r1, a = o % c.r1;
      const double* vt = v + (size_t)(t0 + tt) * dth * p;
      double s = 0;
      for (int q = 0; q < p; ++q) s += th[c.th1_off + q + (size_t)p * a] * vt[q];
      w1[tt][a] = s;
    }
    for (int o = threadIdx.x; o < tc * c.r2; o += NT) {
      const int tt = o / c.r2, a = o % c.r2;
      double s = 1.0;
      if (dth == 2) {
        const double* vt = v + (size_t)(t0 + tt) * dth * p;
        s = 0;
        for (int q = 0; q < p; ++q) s += th[c.th2_off + q + (size_t)p * a] * vt[p + q];
      }
      w2[tt][a] = s;
    }
    __syncthreads();
    double acc[FT][TC];
#pragma unroll
    for (int u = 0; u < FT; ++u)
#pragma unroll
      for (int tt = 0; tt < TC; ++tt) acc[u][tt] = 0.0;
    for (int q = 0; q < rq; ++q) {
      double pv[FT];
#pragma unroll
      for (int u = 0; u < FT; ++u) pv[u] = ok[u] ? cp[(int64_t)q * Pp * Pp + at[u]] : 0.0;
      const int k1 = q % c.r1, k2 = q / c.r1;
#pragma unroll
      for (int tt = 0; tt < TC; ++tt) {
        const double w = w1[tt][k1] * w2[tt][k2];
#pragma unroll
        for (int u = 0; u < FT; ++u) acc[u][tt] += pv[u] * w;
      }
    }
#pragma unroll
    for (int tt = 0; tt < TC; ++tt) {
      if (tt >= tc) break;
      S* Ct = C + (size_t)(t0 + tt) * C_per_slot;
#pragma unroll
      for (int u = 0; u < FT; ++u) {
        if (!ok[u]) continue;
        Ct[c.C_off + at[u]] = (S)acc[u][tt];
        if (c.Cm_off >= 0) Ct[c.Cm_off + mirror_at[u]] = (S)acc[u][tt];
      }
    }
  }
}

// Near field, one workgroup per TILE x TILE_J tile of a stored block (s <= t), all slots:
//   c_t = core x_theta (Theta_k^T v_k(theta_t));  D_t(i, j) = sum_k P[k][i + j n_s] c_t[k]
// Each factor entry is read from HBM once for up to TC slots; the factor entries of KB
// ranks are loaded before any is used (KB * NQ loads in flight per thread).  D_t goes to
// the stored block in 16-row panels (panel_index), padding rows as zeros; the (t, s)
// block is its transpose and is not written (the MVM reads the stored block transposed).
template <typename DT>
__global__ void __launch_bounds__(NT) k_near_instantiate(
    const NearDev* __restrict__ blocks, const int32_t* __restrict__ tiles,
    const double* __restrict__ Pf, const double* __restrict__ core, const double* __restrict__ th,
    const double* __restrict__ v, DT* __restrict__ D, int64_t D_per_slot, int T, int p, int dth) {
  constexpr int RS = NT / TILE;                // 8 column steps of the thread grid
  constexpr int NQ = TILE_J / RS;              // 2 entries per thread
  constexpr int KB = 8;
  __shared__ double w1[TC][16], w2[TC][16], cc[TC][256];
  const int32_t bi = tiles[3 * blockIdx.x], i0 = tiles[3 * blockIdx.x + 1], j0 = tiles[3 * blockIdx.x + 2];
  const NearDev b = blocks[bi];
  const int64_t Nep = (int64_t)b.ldp * b.nt;                     // padded factor column length
  const int ti = threadIdx.x % TILE, tj0 = threadIdx.x / TILE;
  const int i = i0 + ti;
  const int nsp = (b.ns + 15) / 16 * 16;
  bool ok[NQ], wr[NQ];
  int64_t e[NQ], ed[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int j = j0 + tj0 + q * RS;
    ok[q] = i < b.ns && j < b.nt;
    wr[q] = i < nsp && j < b.nt;                                  // rows ns..nsp-1 get 0
    e[q] = ok[q] ? i + (int64_t)j * b.ldp : 0;
    ed[q] = wr[q] ? panel_index(i, j, b.nt) : 0;
  }
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
    for (int o = threadIdx.x; o < TC * b.r_e; o += NT) {
      const int tt = o / b.r_e, k = o % b.r_e;
      double s = 0;
      if (tt < tc)
        for (int k2 = 0; k2 < b.r2; ++k2)
          for (int k1 = 0; k1 < b.r1; ++k1)
            s += core[b.core_off + k + (size_t)b.r_e * (k1 + (size_t)b.r1 * k2)] * w1[tt][k1] * w2[tt][k2];
      cc[tt][k] = s;
    }
    __syncthreads();
    double acc[TC][NQ];
#pragma unroll
    for (int tt = 0; tt < TC; ++tt)
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[tt][q] = 0.0;
    const double* pb = Pf + b.P_off;
    for (int k0 = 0; k0 < b.r_e; k0 += KB) {
      double pv[KB][NQ];
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const bool kok = k0 + kk < b.r_e;
#pragma unroll
        for (int q = 0; q < NQ; ++q) pv[kk][q] = (kok && ok[q]) ? pb[(size_t)(k0 + kk) * Nep + e[q]] : 0.0;
      }
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        if (k0 + kk >= b.r_e) break;
#pragma unroll
        for (int tt = 0; tt < TC; ++tt) {
          const double cv = cc[tt][k0 + kk];
#pragma unroll
          for (int q = 0; q < NQ; ++q) acc[tt][q] += pv[kk][q] * cv;
        }
      }
    }
#pragma unroll
    for (int tt = 0; tt < TC; ++tt) {
      if (tt >= tc) break;
      DT* Dt = D + (size_t)(t0 + tt) * D_per_slot + b.D_st;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (wr[q]) Dt[ed[q]] = to_store<DT>(acc[tt][q]);
    }
  }
}

template <typename S, typename DT>
void instantiate_impl(InstData& in, const double* theta, hipStream_t st) {
  const DeviceModel& m = *in.m;
  join_near(in, st);   // a previous near-field instantiation may still read the theta vectors
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
  const int nMt = m.Pp / 16;
  if (m.format != PH_FORMAT_H2) {
    // far cores H_q(theta_t) of the parametric H-matrix format and of the implicit coupling
    h_core_launch(in, st);
  } else {
    constexpr int FT = 4;
    launch(PH_STAGE_FAR_INST, k_far_instantiate<S, FT>, dim3((unsigned)((nMt * nMt + FT - 1) / FT),
           (unsigned)m.n_stored_cls), dim3(NT), st, (const ClassDev*)m.cstore.p, (const double*)m.ff_chat.p,
           (const double*)m.ff_theta.p, (const double*)in.v.p, (S*)in.C.p, Cps, m.Pp, in.T, m.p_theta, m.d_theta);
  }
  if (in.Cb.n > 0) coupling_bf16_pack_c(in, st);   // BF16 copy of C for the BF16 coupling
  if (in.factored) {
    // factored near field: only c_b(theta_t) per stored block (the MVM forms the blocks)
    near_cores_launch<S>(in, st);
    return;
  }
  // The near-field blocks (HBM-bound, the bulk of the instantiation) are written on the
  // instance's second stream: they overlap the far-field panels here and, in a following
  // ph_matvec, the upward pass and the coupling; the near-field MVM runs on the same
  // stream after them, and every other reader of the instance joins it first (join_near).
  const bool serial = std::getenv("PH_SERIAL_MVM") ? std::atoi(std::getenv("PH_SERIAL_MVM")) != 0
                                                   : in.tune_overlap != 1;
  hipStream_t nst = serial ? st : in.aux;
  if (!serial) {
    PH_HIP(hipEventRecord(in.ev_fork, st));          // theta vectors are ready
    PH_HIP(hipStreamWaitEvent(in.aux, in.ev_fork, 0));
  }
  launch(PH_STAGE_NEAR_INST, k_near_instantiate<DT>, dim3((unsigned)m.n_tiles), dim3(NT), nst,
         (const NearDev*)m.nstore.p, (const int32_t*)m.tiles.p, (const double*)m.nf_P.p,
         (const double*)m.nf_core.p, (const double*)m.nf_theta.p, (const double*)in.v.p, (DT*)in.D.p,
         m.N_nf_pad, in.T, m.p_theta, m.d_theta);
  if (!serial) {
    PH_HIP(hipEventRecord(in.ev_near, in.aux));
    in.near_pending = true;
  }
}

template void instantiate_impl<double, double>(InstData&, const double*, hipStream_t);
template void instantiate_impl<float, float>(InstData&, const double*, hipStream_t);
template void instantiate_impl<float, bf16>(InstData&, const double*, hipStream_t);

}  // namespace ph
