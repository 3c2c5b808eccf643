// H^2 matrix-vector product kernels (arxiv 2511.03109, Alg. "H^2-matrix MVM" with
// FastForward / FastBackward; coupling y_hat_s += C_b x_hat_t as in Alg. "Modified
// H^2-Matrix MVM"), for all parameter slots of an instance in one pass.
//
// Scratch layouts (S = double or float):
//   xt, yt   [T][n][R]             tree order, R fastest
//   xh, yh   [T][nodes][Pp][R]     P padded to Pp (multiple of 16) with zero rows
//   part     [G][T][nodes][Pp][R]  coupling partial sums when the class list is split
#include "ph_device.hpp"

namespace ph {

// xt[slot][t][r] = x[slot][r][perm[t]]
template <typename S>
__global__ void k_perm_in(const S* __restrict__ x, S* __restrict__ xt, const int64_t* __restrict__ perm,
                          int64_t n, int64_t R, int64_t total) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t slot = o / (n * R), rem = o % (n * R);
    const int64_t t = rem / R, r = rem % R;
    xt[o] = x[slot * n * R + r * n + perm[t]];
  }
}

// y[slot][r][perm[t]] = alpha (yt + nugget xt) + beta y
template <typename S>
__global__ void k_perm_out(S* __restrict__ y, const S* __restrict__ yt, const S* __restrict__ xt,
                           const int64_t* __restrict__ perm, int64_t n, int64_t R, int64_t total, double alpha,
                           double beta, double nugget) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t slot = o / (n * R), rem = o % (n * R);
    const int64_t t = rem / R, r = rem % R;
    const int64_t dst = slot * n * R + r * n + perm[t];
    double val = alpha * ((double)yt[o] + nugget * (double)xt[o]);
    if (beta != 0.0) val += beta * (double)y[dst];
    y[dst] = (S)val;
  }
}

// FastForward, leaves: x_hat_s = U_s^T x_s on the matrix cores.  M = i (Chebyshev
// multi-index, Pp rows), K = points of the leaf, N = 16 right-hand sides.
// U_s[pt, i] = prod_k U_k[pt][i_k] is formed on the fly from the factor rows in LDS.
template <typename S>
__global__ void __launch_bounds__(NT) k_leaf_up(const S* __restrict__ xt, S* __restrict__ xh,
                                                const double* __restrict__ U,
                                                const int64_t* __restrict__ nbegin,
                                                const int64_t* __restrict__ nend, int32_t leaf0, int d,
                                                int ps, int P, int Pp, int64_t n, int64_t nodes, int64_t R) {
  typedef Mfma<S> MF;
  constexpr int CH = 128;
  __shared__ double Us[CH * 22];
  const int32_t s = leaf0 + blockIdx.x;
  const int r0 = blockIdx.y * RC;
  const int64_t slot = blockIdx.z;
  const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
  const int m16 = lane & 15, kq = lane >> 4;
  const int64_t b = nbegin[s], ns = nend[s] - b;
  const int dps = d * ps, nMt = Pp / 16;
  const S* xs = xt + slot * n * R;
  int dig[2][3];
  bool rowok[2], tileok[2];
  for (int j = 0; j < 2; ++j) {
    const int mt = wave + 4 * j;
    tileok[j] = mt < nMt;
    int ii = mt * 16 + m16;
    rowok[j] = tileok[j] && ii < P;
    for (int k = 0; k < 3; ++k) {
      dig[j][k] = k < d ? ii % ps : 0;
      ii /= ps;
    }
  }
  typename MF::acc_t acc[2];
  for (int j = 0; j < 2; ++j) acc[j] = (typename MF::acc_t){0, 0, 0, 0};
  const bool colok = r0 + m16 < R;
  for (int64_t c0 = 0; c0 < ns; c0 += CH) {
    const int cn = (int)min<int64_t>(CH, ns - c0);
    __syncthreads();
    for (int q = threadIdx.x; q < cn * dps; q += NT) Us[q] = U[(b + c0) * dps + q];
    __syncthreads();
    for (int k0 = 0; k0 < cn; k0 += 4) {
      const int pi = k0 + kq;
      const bool pok = pi < cn;
      const S bv = (pok && colok) ? xs[(b + c0 + pi) * R + r0 + m16] : (S)0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (!tileok[j]) continue;
        double av = 0.0;
        if (rowok[j] && pok) {
          av = Us[pi * dps + dig[j][0]];
          for (int k = 1; k < d; ++k) av *= Us[pi * dps + k * ps + dig[j][k]];
        }
        acc[j] = MF::mac((S)av, bv, acc[j]);
      }
    }
  }
  if (!colok) return;
  S* out = xh + (slot * nodes + s) * Pp * R;
  for (int j = 0; j < 2; ++j) {
    if (!tileok[j]) continue;
    const int mt = wave + 4 * j;
    for (int q = 0; q < 4; ++q) out[(int64_t)(mt * 16 + MF::row(lane, q)) * R + r0 + m16] = acc[j][q];
  }
}

// Apply a per-axis transfer factor along axis k of a p_s^d x RC tensor in LDS:
//   transpose == true:  out[.., a, ..] = sum_j E_h[j][a] in[.., j, ..]   (FastForward, E^T)
//   transpose == false: out[.., j, ..] = sum_a E_h[j][a] in[.., a, ..]   (FastBackward, E)
__device__ inline void kron_axis(const double* __restrict__ Es, int h, int ps, int stride, int P,
                                 const double* __restrict__ src, double* __restrict__ dst, bool transpose) {
  for (int o = threadIdx.x; o < P * RC; o += NT) {
    const int i = o / RC, r = o % RC;
    const int a = (i / stride) % ps;
    const int base = i - a * stride;
    double s = 0;
    for (int j = 0; j < ps; ++j) {
      const double e = transpose ? Es[(h * ps + j) * ps + a] : Es[(h * ps + a) * ps + j];
      s += e * src[(base + j * stride) * RC + r];
    }
    dst[o] = s;
  }
}

// FastForward, inner nodes: x_hat_s = sum_{children c} E_c^T x_hat_c with
// E_c = E_{c,d} (x) ... (x) E_{c,1} applied one axis at a time (FastKron).
template <typename S>
__global__ void __launch_bounds__(NT) k_transfer_up(S* __restrict__ xh, const double* __restrict__ E,
                                                    const int32_t* __restrict__ first_child,
                                                    const int32_t* __restrict__ nchild,
                                                    const int32_t* __restrict__ cid, int32_t node0, int d,
                                                    int ps, int P, int Pp, int64_t nodes, int64_t R) {
  __shared__ double Es[2 * 16 * 16];
  __shared__ double bufA[128 * RC], bufB[128 * RC];
  const int32_t s = node0 + blockIdx.x;
  const int r0 = blockIdx.y * RC;
  const int64_t slot = blockIdx.z;
  const int rc = (int)min<int64_t>(RC, R - r0);
  for (int o = threadIdx.x; o < 2 * ps * ps; o += NT) Es[o] = E[o];
  double acc[8];
  for (int q = 0; q < 8; ++q) acc[q] = 0;
  const int32_t f = first_child[s], nc = nchild[s];
  for (int c = 0; c < nc; ++c) {
    const int32_t ch = f + c;
    const S* in = xh + (slot * nodes + ch) * Pp * R;
    __syncthreads();
    for (int o = threadIdx.x; o < P * RC; o += NT) {
      const int i = o / RC, r = o % RC;
      bufA[o] = r < rc ? (double)in[(int64_t)i * R + r0 + r] : 0.0;
    }
    __syncthreads();
    const int cc = cid[ch];
    double* src = bufA;
    double* dst = bufB;
    int stride = 1;
    for (int k = 0; k < d; ++k) {
      kron_axis(Es, (cc >> k) & 1, ps, stride, P, src, dst, true);
      __syncthreads();
      double* tmp = src;
      src = dst;
      dst = tmp;
      stride *= ps;
    }
    for (int q = 0; q < 8; ++q) {
      const int o = threadIdx.x + q * NT;
      if (o < P * RC) acc[q] += src[o];
    }
  }
  S* out = xh + (slot * nodes + s) * Pp * R;
  for (int q = 0; q < 8; ++q) {
    const int o = threadIdx.x + q * NT;
    const int i = o / RC, r = o % RC;
    if (i < Pp && r < rc) out[(int64_t)i * R + r0 + r] = (S)(i < P ? acc[q] : 0.0);
  }
}

// FastBackward, inner nodes: y_hat_c += E_c y_hat_parent, one workgroup per child.
template <typename S>
__global__ void __launch_bounds__(NT) k_transfer_down(S* __restrict__ yh, const double* __restrict__ E,
                                                      const int32_t* __restrict__ parent_of,
                                                      const int32_t* __restrict__ cid, int32_t node0, int d,
                                                      int ps, int P, int Pp, int64_t nodes, int64_t R) {
  __shared__ double Es[2 * 16 * 16];
  __shared__ double bufA[128 * RC], bufB[128 * RC];
  const int32_t c = node0 + blockIdx.x;
  const int r0 = blockIdx.y * RC;
  const int64_t slot = blockIdx.z;
  const int rc = (int)min<int64_t>(RC, R - r0);
  for (int o = threadIdx.x; o < 2 * ps * ps; o += NT) Es[o] = E[o];
  const S* in = yh + (slot * nodes + parent_of[c]) * Pp * R;
  for (int o = threadIdx.x; o < P * RC; o += NT) {
    const int i = o / RC, r = o % RC;
    bufA[o] = r < rc ? (double)in[(int64_t)i * R + r0 + r] : 0.0;
  }
  __syncthreads();
  const int cc = cid[c];
  double* src = bufA;
  double* dst = bufB;
  int stride = 1;
  for (int k = 0; k < d; ++k) {
    kron_axis(Es, (cc >> k) & 1, ps, stride, P, src, dst, false);
    __syncthreads();
    double* tmp = src;
    src = dst;
    dst = tmp;
    stride *= ps;
  }
  S* out = yh + (slot * nodes + c) * Pp * R;
  for (int o = threadIdx.x; o < P * RC; o += NT) {
    const int i = o / RC, r = o % RC;
    if (r < rc) {
      const int64_t idx = (int64_t)i * R + r0 + r;
      out[idx] = (S)((double)out[idx] + src[o]);
    }
  }
}

// Coupling y_hat_s = sum over far blocks (s, t) of C_class x_hat_t on the matrix cores.
// One workgroup per (sibling group, class chunk, RHS tile, slot): the 2^d children of
// one parent share most translation classes, so each C_class fragment loaded from
// L2 / Infinity Cache feeds up to 2^d MFMAs.  Wave w owns row tiles w and w + 4 of the
// Pp x 16 outputs.  With G > 1 chunks the outputs are partial sums.
template <typename S, int NSIB>
__global__ void __launch_bounds__(NT) k_coupling(
    const S* __restrict__ xh, S* __restrict__ out, const S* __restrict__ C,
    const int32_t* __restrict__ grp_targets, const int32_t* __restrict__ grp_entry,
    const int32_t* __restrict__ ent_cls, const int32_t* __restrict__ ent_tau, int Pp, int64_t nodes,
    int64_t R, int G, int64_t Cps, int64_t part_stride, int T) {
  typedef Mfma<S> MF;
  const int grp = blockIdx.x;
  const int g = blockIdx.y % G;
  const int r0 = (blockIdx.y / G) * RC;
  const int64_t slot = blockIdx.z;
  const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
  const int m16 = lane & 15, kq = lane >> 4;
  const int nMt = Pp / 16;
  const bool t0ok = wave < nMt, t1ok = wave + 4 < nMt;
  const bool colok = r0 + m16 < R;
  typename MF::acc_t acc[NSIB][2];
#pragma unroll
  for (int s = 0; s < NSIB; ++s) {
    acc[s][0] = (typename MF::acc_t){0, 0, 0, 0};
    acc[s][1] = (typename MF::acc_t){0, 0, 0, 0};
  }
  const int e_begin = grp_entry[grp], e_end = grp_entry[grp + 1];
  const int ne = e_end - e_begin;
  const int ea = e_begin + (int)((int64_t)ne * g / G), eb = e_begin + (int)((int64_t)ne * (g + 1) / G);
  const S* xs = xh + slot * nodes * Pp * R;
  const S* Cs = C + slot * Cps;
  for (int e = ea; e < eb; ++e) {
    const S* Cc = Cs + (int64_t)ent_cls[e] * Pp * Pp;
    int tau[NSIB];
#pragma unroll
    for (int s = 0; s < NSIB; ++s) tau[s] = ent_tau[(int64_t)e * NSIB + s];
    for (int k0 = 0; k0 < Pp; k0 += 4) {
      const int k = k0 + kq;
      const S a0 = t0ok ? Cc[(wave * 16 + m16) + (int64_t)Pp * k] : (S)0;
      const S a1 = t1ok ? Cc[((wave + 4) * 16 + m16) + (int64_t)Pp * k] : (S)0;
#pragma unroll
      for (int s = 0; s < NSIB; ++s) {
        if (tau[s] < 0) continue;
        const S bv = colok ? xs[((int64_t)tau[s] * Pp + k) * R + r0 + m16] : (S)0;
        if (t0ok) acc[s][0] = MF::mac(a0, bv, acc[s][0]);
        if (t1ok) acc[s][1] = MF::mac(a1, bv, acc[s][1]);
      }
    }
  }
  if (!colok) return;
  S* o = out + (int64_t)g * part_stride + slot * nodes * Pp * R;
#pragma unroll
  for (int s = 0; s < NSIB; ++s) {
    const int32_t node = grp_targets[grp * NSIB + s];
    if (node < 0) continue;
    S* on = o + (int64_t)node * Pp * R;
    for (int q = 0; q < 4; ++q) {
      if (t0ok) on[(int64_t)(wave * 16 + MF::row(lane, q)) * R + r0 + m16] = acc[s][0][q];
      if (t1ok) on[(int64_t)((wave + 4) * 16 + MF::row(lane, q)) * R + r0 + m16] = acc[s][1][q];
    }
  }
}

// y_hat[slot][node] = sum_g part[g][slot][node] for nodes >= a0
template <typename S>
__global__ void k_coupling_reduce(S* __restrict__ yh, const S* __restrict__ part, int G, int64_t part_stride,
                                  int64_t node_elems, int64_t a0, int64_t nodes, int64_t total) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t per_slot = (nodes - a0) * node_elems;
    const int64_t slot = o / per_slot, rem = o % per_slot;
    const int64_t idx = slot * nodes * node_elems + a0 * node_elems + rem;
    double s = 0;
    for (int g = 0; g < G; ++g) s += (double)part[(int64_t)g * part_stride + idx];
    yh[idx] = (S)s;
  }
}

// Near field and the leaf step of FastBackward on the matrix cores, one workgroup per
// (leaf s, RHS tile, slot):
//   y_s = sum_{near t} D_st x_t + U_s y_hat_s
// M = rows of the leaf (row tiles w, w + 4 per wave, in chunks of 128 rows),
// K = columns of each near block, then the Chebyshev multi-index for U_s y_hat_s.
template <typename S>
__global__ void __launch_bounds__(NT) k_leaf_near(
    const S* __restrict__ xt, S* __restrict__ yt, const S* __restrict__ yh, const S* __restrict__ D,
    const double* __restrict__ U, const int64_t* __restrict__ nbegin, const int64_t* __restrict__ nend,
    const int64_t* __restrict__ rowptr, const int64_t* __restrict__ ntb, const int32_t* __restrict__ nnt,
    const int64_t* __restrict__ nD, int32_t leaf0, int use_far, int d, int ps, int P, int Pp, int64_t n,
    int64_t nodes, int64_t R, int64_t N_nf) {
  typedef Mfma<S> MF;
  constexpr int CH = 128;
  __shared__ double Us[CH * 22];
  const int32_t li = blockIdx.x;
  const int32_t s = leaf0 + li;
  const int r0 = blockIdx.y * RC;
  const int64_t slot = blockIdx.z;
  const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
  const int m16 = lane & 15, kq = lane >> 4;
  const int64_t b = nbegin[s], ns = nend[s] - b;
  const int dps = d * ps;
  const bool colok = r0 + m16 < R;
  const S* xs = xt + slot * n * R;
  const S* Ds = D + slot * N_nf;
  const S* yhs = yh + (slot * nodes + s) * Pp * R;
  const int64_t bb0 = rowptr[li], bb1 = rowptr[li + 1];
  for (int64_t c0 = 0; c0 < ns; c0 += CH) {
    const int cn = (int)min<int64_t>(CH, ns - c0);
    if (use_far) {
      __syncthreads();
      for (int q = threadIdx.x; q < cn * dps; q += NT) Us[q] = U[(b + c0) * dps + q];
      __syncthreads();
    }
    const int i0 = wave * 16 + m16, i1 = (wave + 4) * 16 + m16;   // rows within the chunk
    const bool t0ok = wave * 16 < cn, t1ok = (wave + 4) * 16 < cn;
    const bool r0ok = i0 < cn, r1ok = i1 < cn;
    typename MF::acc_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    for (int64_t bb = bb0; bb < bb1; ++bb) {
      const S* Db = Ds + nD[bb] + c0;
      const int64_t tb = ntb[bb];
      const int nt = nnt[bb];
#pragma unroll 4
      for (int k0 = 0; k0 < nt; k0 += 4) {
        const int j = k0 + kq;
        const bool jok = j < nt;
        const S bv = (jok && colok) ? xs[(tb + j) * R + r0 + m16] : (S)0;
        const S a0 = (jok && r0ok) ? Db[i0 + (int64_t)j * ns] : (S)0;
        const S a1 = (jok && r1ok) ? Db[i1 + (int64_t)j * ns] : (S)0;
        if (t0ok) acc0 = MF::mac(a0, bv, acc0);
        if (t1ok) acc1 = MF::mac(a1, bv, acc1);
      }
    }
    if (use_far) {
      for (int k0 = 0; k0 < Pp; k0 += 4) {
        const int ii = k0 + kq;
        const bool iok = ii < P;
        const S bv = (iok && colok) ? yhs[(int64_t)ii * R + r0 + m16] : (S)0;
        int dg[3];
        int rem = ii;
        for (int k = 0; k < 3; ++k) {
          dg[k] = rem % ps;
          rem /= ps;
        }
        double u0 = 0.0, u1 = 0.0;
        if (iok && r0ok) {
          u0 = Us[m16 * 0 + (wave * 16 + m16) * dps + dg[0]];
          for (int k = 1; k < d; ++k) u0 *= Us[(wave * 16 + m16) * dps + k * ps + dg[k]];
        }
        if (iok && r1ok) {
          u1 = Us[((wave + 4) * 16 + m16) * dps + dg[0]];
          for (int k = 1; k < d; ++k) u1 *= Us[((wave + 4) * 16 + m16) * dps + k * ps + dg[k]];
        }
        if (t0ok) acc0 = MF::mac((S)u0, bv, acc0);
        if (t1ok) acc1 = MF::mac((S)u1, bv, acc1);
      }
    }
    if (colok) {
      S* ys = yt + slot * n * R;
      for (int q = 0; q < 4; ++q) {
        const int ra = wave * 16 + MF::row(lane, q), rb = (wave + 4) * 16 + MF::row(lane, q);
        if (t0ok && ra < cn) ys[(b + c0 + ra) * R + r0 + m16] = acc0[q];
        if (t1ok && rb < cn) ys[(b + c0 + rb) * R + r0 + m16] = acc1[q];
      }
    }
  }
}

template <typename S>
void matvec_impl(InstData& in, const S* x, S* y, int64_t R, double alpha, double beta, double nugget,
                 hipStream_t st) {
  const DeviceModel& m = *in.m;
  const TreeData& t = *m.tree;
  const int64_t T = in.T;
  const int64_t nrc = (R + RC - 1) / RC;
  const bool use_far = m.min_far >= 0;
  // split the class list when the sibling groups alone give too few workgroups
  int G = 1;
  if (use_far && m.n_groups > 0) {
    const int64_t wgs = m.n_groups * nrc * T;
    while (G < 16 && wgs * G < 1024 && m.max_group_entries >= 2 * G) G *= 2;
  }
  if (R > in.Rcap || G > in.Gcap) {
    const int64_t Rc = std::max<int64_t>(R, in.Rcap);
    const int Gc = std::max(G, in.Gcap);
    in.xt.alloc((size_t)T * m.n * Rc * sizeof(S));
    in.yt.alloc((size_t)T * m.n * Rc * sizeof(S));
    in.xh.alloc((size_t)T * m.n_nodes * m.Pp * Rc * sizeof(S));
    in.yh.alloc((size_t)T * m.n_nodes * m.Pp * Rc * sizeof(S));
    if (Gc > 1) in.part.alloc((size_t)Gc * T * m.n_nodes * m.Pp * Rc * sizeof(S));
    in.Rcap = Rc;
    in.Gcap = Gc;
  }
  S* xt = (S*)in.xt.p;
  S* yt = (S*)in.yt.p;
  S* xh = (S*)in.xh.p;
  S* yh = (S*)in.yh.p;
  const int32_t leaf0 = t.leaves.front();
  const int64_t Cps = m.n_classes * m.Pp * m.Pp;
  const int64_t total = T * m.n * R;
  launch(PH_STAGE_PERM_IN, k_perm_in<S>, dim3((unsigned)grid_for(total)), dim3(NT), st, x, xt,
         (const int64_t*)m.perm.p, m.n, R, total);
  if (use_far) {
    launch(PH_STAGE_LEAF_UP, k_leaf_up<S>, dim3((unsigned)m.n_leaves, (unsigned)nrc, (unsigned)T), dim3(NT),
           st, (const S*)xt, xh, (const double*)m.U.p, (const int64_t*)m.nbegin.p, (const int64_t*)m.nend.p,
           leaf0, m.d, m.p_s, m.P, m.Pp, m.n, m.n_nodes, R);
    for (int l = m.l_max - 1; l >= m.min_far; --l) {
      const int32_t a = t.level_start[l], b = t.level_start[l + 1];
      launch(PH_STAGE_TRANSFER_UP, k_transfer_up<S>, dim3((unsigned)(b - a), (unsigned)nrc, (unsigned)T),
             dim3(NT), st, xh, (const double*)m.E.p, (const int32_t*)m.first_child.p,
             (const int32_t*)m.nchild.p, (const int32_t*)m.cid.p, a, m.d, m.p_s, m.P, m.Pp, m.n_nodes, R);
    }
    const int64_t part_stride = T * m.n_nodes * m.Pp * R;
    S* cout = G > 1 ? (S*)in.part.p : yh;
    dim3 cg((unsigned)m.n_groups, (unsigned)(G * nrc), (unsigned)T);
    if (m.nsib == 2)
      launch(PH_STAGE_COUPLING, k_coupling<S, 2>, cg, dim3(NT), st, (const S*)xh, cout, (const S*)in.C.p,
             (const int32_t*)m.grp_targets.p, (const int32_t*)m.grp_entry.p, (const int32_t*)m.ent_cls.p,
             (const int32_t*)m.ent_tau.p, m.Pp, m.n_nodes, R, G, Cps, part_stride, (int)T);
    else if (m.nsib == 4)
      launch(PH_STAGE_COUPLING, k_coupling<S, 4>, cg, dim3(NT), st, (const S*)xh, cout, (const S*)in.C.p,
             (const int32_t*)m.grp_targets.p, (const int32_t*)m.grp_entry.p, (const int32_t*)m.ent_cls.p,
             (const int32_t*)m.ent_tau.p, m.Pp, m.n_nodes, R, G, Cps, part_stride, (int)T);
    else
      launch(PH_STAGE_COUPLING, k_coupling<S, 8>, cg, dim3(NT), st, (const S*)xh, cout, (const S*)in.C.p,
             (const int32_t*)m.grp_targets.p, (const int32_t*)m.grp_entry.p, (const int32_t*)m.ent_cls.p,
             (const int32_t*)m.ent_tau.p, m.Pp, m.n_nodes, R, G, Cps, part_stride, (int)T);
    if (G > 1) {
      const int64_t a0 = t.level_start[m.min_far];
      const int64_t node_elems = (int64_t)m.Pp * R;
      const int64_t rtotal = T * (m.n_nodes - a0) * node_elems;
      launch(PH_STAGE_ZERO, k_coupling_reduce<S>, dim3((unsigned)grid_for(rtotal)), dim3(NT), st, yh,
             (const S*)in.part.p, G, part_stride, node_elems, a0, m.n_nodes, rtotal);
    }
    for (int l = m.min_far; l < m.l_max; ++l) {
      const int32_t a = t.level_start[l + 1], b = t.level_start[l + 2];
      launch(PH_STAGE_TRANSFER_DOWN, k_transfer_down<S>, dim3((unsigned)(b - a), (unsigned)nrc, (unsigned)T),
             dim3(NT), st, yh, (const double*)m.E.p, (const int32_t*)m.parent.p, (const int32_t*)m.cid.p, a,
             m.d, m.p_s, m.P, m.Pp, m.n_nodes, R);
    }
  }
  launch(PH_STAGE_LEAF_NEAR, k_leaf_near<S>, dim3((unsigned)m.n_leaves, (unsigned)nrc, (unsigned)T), dim3(NT),
         st, (const S*)xt, yt, (const S*)yh, (const S*)in.D.p, (const double*)m.U.p,
         (const int64_t*)m.nbegin.p, (const int64_t*)m.nend.p, (const int64_t*)m.near_rowptr.p,
         (const int64_t*)m.near_tb.p, (const int32_t*)m.near_nt.p, (const int64_t*)m.near_D.p, leaf0,
         use_far ? 1 : 0, m.d, m.p_s, m.P, m.Pp, m.n, m.n_nodes, R, m.N_nf);
  launch(PH_STAGE_PERM_OUT, k_perm_out<S>, dim3((unsigned)grid_for(total)), dim3(NT), st, y, (const S*)yt,
         (const S*)xt, (const int64_t*)m.perm.p, m.n, R, total, alpha, beta, nugget);
}

template void matvec_impl<double>(InstData&, const double*, double*, int64_t, double, double, double,
                                  hipStream_t);
template void matvec_impl<float>(InstData&, const float*, float*, int64_t, double, double, double,
                                 hipStream_t);

}  // namespace ph
