// H^2 matrix-vector product kernels (arxiv 2511.03109, Alg. "H^2-matrix MVM" with
// FastForward / FastBackward; coupling y_hat_s += C_b x_hat_t as in Alg. "Modified
// H^2-Matrix MVM"), for all parameter slots of an instance in one pass.
//
// Scratch layouts (S = double or float; Rs = R rounded up to a multiple of 16, the
// padding columns hold zeros, and Rs = 1 for a single right-hand side):
//   xt, yt   [T][n][Rs]             tree order, right-hand side fastest
//   xh, yh   [T][nodes][Pp][Rs]     P padded to Pp (multiple of 16) with zero rows
//   part     [G][T][nodes][Pp][Rs]  coupling partial sums when the class list is split
#include <cstdlib>
#include <type_traits>

#include "ph_device.hpp"

namespace ph {

// xt[slot][t][r] = x[slot][r][perm[t]] (0 for the padding columns r >= R)
template <typename S>
__global__ void k_perm_in(const S* __restrict__ x, S* __restrict__ xt, const int64_t* __restrict__ perm,
                          int64_t n, int64_t R, int64_t Rs, int64_t total) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t slot = o / (n * Rs), rem = o % (n * Rs);
    const int64_t t = rem / Rs, r = rem % Rs;
    xt[o] = r < R ? x[slot * n * R + r * n + perm[t]] : (S)0;
  }
}

// y[slot][r][perm[t]] = alpha (yt + nugget xt) + beta y
template <typename S>
__global__ void k_perm_out(S* __restrict__ y, const S* __restrict__ yt, const S* __restrict__ xt,
                           const int64_t* __restrict__ perm, int64_t n, int64_t R, int64_t Rs, int64_t total,
                           double alpha, double beta, double nugget) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t slot = o / (n * R), rem = o % (n * R);
    const int64_t t = rem / R, r = rem % R;
    const int64_t src = (slot * n + t) * Rs + r;
    const int64_t dst = slot * n * R + r * n + perm[t];
    double val = alpha * ((double)yt[src] + nugget * (double)xt[src]);
    if (beta != 0.0) val += beta * (double)y[dst];
    y[dst] = (S)val;
  }
}

// The same two permutations for Rs >= 16, through an LDS tile of 64 points x 16 right-hand
// sides: the user's rows x[slot][r][j0 .. j0 + 63] are read and y's written as 512-byte
// runs, and each point's 16 values in tree order (iperm[j] = tree position of point j) as
// one 128-byte run, instead of 8-byte accesses scattered by the permutation.
template <typename S>
__global__ void __launch_bounds__(NT) k_perm_in_tile(const S* __restrict__ x, S* __restrict__ xt,
                                                     const int64_t* __restrict__ iperm, int64_t n, int64_t R,
                                                     int64_t Rs) {
  __shared__ S tile[16][65];
  const int64_t j0 = (int64_t)blockIdx.x * 64, slot = blockIdx.z;
  const int r0 = blockIdx.y * RC;
  const int jj = threadIdx.x & 63, rq = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = rq * 4 + k;
    const int64_t j = j0 + jj;
    tile[r][jj] = (j < n && r0 + r < R) ? x[(slot * R + r0 + r) * n + j] : (S)0;
  }
  __syncthreads();
  const int rr = threadIdx.x & 15, jq = threadIdx.x >> 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int jl = jq * 4 + k;
    const int64_t j = j0 + jl;
    if (j < n) xt[(slot * n + iperm[j]) * Rs + r0 + rr] = tile[rr][jl];
  }
}

template <typename S>
__global__ void __launch_bounds__(NT) k_perm_out_tile(S* __restrict__ y, const S* __restrict__ yt,
                                                      const S* __restrict__ xt, const int64_t* __restrict__ iperm,
                                                      int64_t n, int64_t R, int64_t Rs, double alpha, double beta,
                                                      double nugget) {
  __shared__ double tile[16][65];
  const int64_t j0 = (int64_t)blockIdx.x * 64, slot = blockIdx.z;
  const int r0 = blockIdx.y * RC;
  const int rr = threadIdx.x & 15, jq = threadIdx.x >> 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int jl = jq * 4 + k;
    const int64_t j = j0 + jl;
    if (j < n) {
      const int64_t src = (slot * n + iperm[j]) * Rs + r0 + rr;
      tile[rr][jl] = alpha * ((double)yt[src] + nugget * (double)xt[src]);
    }
  }
  __syncthreads();
  const int jj = threadIdx.x & 63, rq = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = rq * 4 + k;
    const int64_t j = j0 + jj;
    if (j < n && r0 + r < R) {
      S* d = y + (slot * R + r0 + r) * n + j;
      double val = tile[r][jj];
      if (beta != 0.0) val += beta * (double)*d;
      *d = (S)val;
    }
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
  const int lane = threadIdx.x % WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
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

// digits (i_0, i_1, i_2) of every multi-index i = i_0 + p_s i_1 + p_s^2 i_2 < P into an LDS
// table (visible after the caller's next barrier)
__device__ inline void multi_index_digits(int* dg, int P, int ps) {
  for (int i = threadIdx.x; i < P; i += NT) {
    int rem = i;
    for (int k = 0; k < 3; ++k) {
      dg[3 * i + k] = rem % ps;
      rem /= ps;
    }
  }
}

// Apply a per-axis transfer factor along axis k of a p_s^d x 2^lc tensor in LDS (2^lc
// right-hand-side columns: 16, or 1 for a single right-hand side):
//   transpose == true:  out[.., a, ..] = sum_j E_h[j][a] in[.., j, ..]   (FastForward, E^T)
//   transpose == false: out[.., j, ..] = sum_a E_h[j][a] in[.., a, ..]   (FastBackward, E)
// (dg: digit `axis` of every multi-index i < P at dg[3 i + axis], a table in LDS)
__device__ inline void kron_axis(const double* __restrict__ Es, int h, int ps, int stride, int axis, int P,
                                 int lc, const int* __restrict__ dg, const double* __restrict__ src,
                                 double* __restrict__ dst, bool transpose) {
  for (int o = threadIdx.x; o < (P << lc); o += NT) {
    const int i = o >> lc, r = o & ((1 << lc) - 1);
    const int a = dg[3 * i + axis];
    const int base = i - a * stride;
    double s = 0;
    for (int j = 0; j < ps; ++j) {
      const double e = transpose ? Es[(h * ps + j) * ps + a] : Es[(h * ps + a) * ps + j];
      s += e * src[((base + j * stride) << lc) + r];
    }
    dst[o] = s;
  }
}

// FastForward, inner nodes: x_hat_s = sum_{children c} E_c^T x_hat_c with
// E_c = E_{c,d} (x) ... (x) E_{c,1} applied one axis at a time (FastKron).
// LC: log2 of the right-hand-side columns held in LDS (4, or 0 for a single one).
template <typename S, int LC>
__global__ void __launch_bounds__(NT) k_transfer_up(S* __restrict__ xh, const double* __restrict__ E,
                                                    const int32_t* __restrict__ first_child,
                                                    const int32_t* __restrict__ nchild,
                                                    const int32_t* __restrict__ cid, int32_t node0, int d,
                                                    int ps, int P, int Pp, int64_t nodes, int64_t R) {
  __shared__ double Es[2 * 16 * 16];
  __shared__ double bufA[128 * RC], bufB[128 * RC];
  __shared__ int Dg[128 * 3];
  const int32_t s = node0 + blockIdx.x;
  const int r0 = blockIdx.y * RC;
  const int64_t slot = blockIdx.z;
  const int rc = (int)min<int64_t>(RC, R - r0);
  constexpr int lc = LC;
  for (int o = threadIdx.x; o < 2 * ps * ps; o += NT) Es[o] = E[o];
  multi_index_digits(Dg, P, ps);
  double acc[8];
  for (int q = 0; q < 8; ++q) acc[q] = 0;
  const int32_t f = first_child[s], nc = nchild[s];
  for (int c = 0; c < nc; ++c) {
    const int32_t ch = f + c;
    const S* in = xh + (slot * nodes + ch) * Pp * R;
    __syncthreads();
    for (int o = threadIdx.x; o < (P << lc); o += NT) {
      const int i = o >> lc, r = o & ((1 << lc) - 1);
      bufA[o] = r < rc ? (double)in[(int64_t)i * R + r0 + r] : 0.0;
    }
    __syncthreads();
    const int cc = cid[ch];
    double* src = bufA;
    double* dst = bufB;
    int stride = 1;
    for (int k = 0; k < d; ++k) {
      kron_axis(Es, (cc >> k) & 1, ps, stride, k, P, lc, Dg, src, dst, true);
      __syncthreads();
      double* tmp = src;
      src = dst;
      dst = tmp;
      stride *= ps;
    }
    for (int q = 0; q < 8; ++q) {
      const int o = threadIdx.x + q * NT;
      if (o < (P << lc)) acc[q] += src[o];
    }
  }
  S* out = xh + (slot * nodes + s) * Pp * R;
  for (int q = 0; q < 8; ++q) {
    const int o = threadIdx.x + q * NT;
    const int i = o >> lc, r = o & ((1 << lc) - 1);
    if (i < Pp && r < rc) out[(int64_t)i * R + r0 + r] = (S)(i < P ? acc[q] : 0.0);
  }
}

// FastBackward, inner nodes: y_hat_c += E_c y_hat_parent, one workgroup per child.
// LC as in k_transfer_up.
template <typename S, int LC>
__global__ void __launch_bounds__(NT) k_transfer_down(S* __restrict__ yh, const double* __restrict__ E,
                                                      const int32_t* __restrict__ parent_of,
                                                      const int32_t* __restrict__ cid, int32_t node0, int d,
                                                      int ps, int P, int Pp, int64_t nodes, int64_t R) {
  __shared__ double Es[2 * 16 * 16];
  __shared__ double bufA[128 * RC], bufB[128 * RC];
  __shared__ int Dg[128 * 3];
  const int32_t c = node0 + blockIdx.x;
  const int r0 = blockIdx.y * RC;
  const int64_t slot = blockIdx.z;
  const int rc = (int)min<int64_t>(RC, R - r0);
  constexpr int lc = LC;
  for (int o = threadIdx.x; o < 2 * ps * ps; o += NT) Es[o] = E[o];
  multi_index_digits(Dg, P, ps);
  const S* in = yh + (slot * nodes + parent_of[c]) * Pp * R;
  for (int o = threadIdx.x; o < (P << lc); o += NT) {
    const int i = o >> lc, r = o & ((1 << lc) - 1);
    bufA[o] = r < rc ? (double)in[(int64_t)i * R + r0 + r] : 0.0;
  }
  __syncthreads();
  const int cc = cid[c];
  double* src = bufA;
  double* dst = bufB;
  int stride = 1;
  for (int k = 0; k < d; ++k) {
    kron_axis(Es, (cc >> k) & 1, ps, stride, k, P, lc, Dg, src, dst, false);
    __syncthreads();
    double* tmp = src;
    src = dst;
    dst = tmp;
    stride *= ps;
  }
  S* out = yh + (slot * nodes + c) * Pp * R;
  for (int o = threadIdx.x; o < (P << lc); o += NT) {
    const int i = o >> lc, r = o & ((1 << lc) - 1);
    if (r < rc) {
      const int64_t idx = (int64_t)i * R + r0 + r;
      out[idx] = (S)((double)out[idx] + src[o]);
    }
  }
}

// Coupling y_hat_s = sum over far blocks (s, t) of C_class x_hat_t on the matrix cores.
// One workgroup of NW wavefronts per (class chunk g, slot, target box, RHS tile); a box
// holds NTG nodes of one level and its work list has one entry per translation class,
// so each C_class panel staged in LDS feeds the MFMAs of every target in the box that
// uses the class.  The class list of every box is cut into G chunks and g is the fastest
// grid index: with G = 8, chunk g of every box lands on XCD g (workgroups are dealt to the
// 8 XCDs round robin), so each XCD's L2 serves about one eighth of the classes.
// Pipeline: stage = (entry, 16-wide K panel).  C is stored in fragment order (frag_index),
// so a stage of C is one contiguous Pp x 16 panel, copied with 16-byte loads; the x_hat
// rows of each used target are copied the same way.  Global loads run PD stages ahead in
// registers, LDS is double buffered, one barrier per stage.  Entry metadata (class,
// sources) is wave-uniform and read with scalar loads.  Waves form a WR x (NW / WR) grid:
// wave (wr, wt) owns row tiles wr + WR j (j < TPW) of targets wt NTW .. wt NTW + NTW - 1;
// FULL: the row tiles are exactly Pp / 16 (no tile test).
// HB: the box is split into HB parts of NTG / HB targets, one workgroup each (the C panel
// is staged by every part).
// PACK (one right-hand side): the 16 targets of the box are the 16 matrix-core columns,
// B[k][c] = x_hat of target c's source for the entry's class (zero if c does not use it),
// so a stage multiplies one C panel by one 16-column tile instead of 16 tiles of which 15
// columns would be padding.  Requires the unpadded single-RHS layout (Rs = 1, r0 = 0).
template <typename S, int NW, int WR, int TPW, int PD, bool FULL, bool PACK = false, int HB = 1, int KG = 1>
__global__ void __launch_bounds__(NW * 64, HB) k_coupling(
    const S* __restrict__ xh, S* __restrict__ out, const S* __restrict__ C,
    const int32_t* __restrict__ grp_targets, const int32_t* __restrict__ grp_entry,
    const int32_t* __restrict__ ent_cls, const int32_t* __restrict__ ent_tau,
    const int32_t* __restrict__ chunk_first, int Pp, int64_t nodes,
    int64_t Rs, int G, int64_t Cps, int64_t part_stride, int n_groups) {
  typedef Tile16<S> MF;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  constexpr int NTH = NW * 64;
  constexpr int NB = PACK ? 1 : NTG / HB;       // 16-column B tiles per workgroup (HB parts per box)
  constexpr int WT = NW / WR, NTW = NB / WT, MT = WR * TPW;
  constexpr int KC = 16;                        // K rows per stage
  constexpr int EPU = 16 / (int)sizeof(S);      // elements per 16-byte unit
  constexpr int AU = (MT * 256 / EPU + NTH - 1) / NTH;   // C units per thread per stage
  constexpr int TSW = PACK ? 1 : NB / NW;       // targets staged per wave
  constexpr int BUT = 256 / EPU / 64;           // x_hat units per lane per target
  static_assert(NB % WT == 0 && (PACK || NB % NW == 0) && BUT >= 1 && (!PACK || HB == 1), "work split");
  static_assert(!PACK || (WT == 1 && NTH >= 256), "packed mode: one column tile, 256 B loaders");
  __shared__ __attribute__((aligned(16))) S As[2][MT * 256];
  __shared__ __attribute__((aligned(16))) S Bs[2][NB][256];
  // grid (chunk g, slot, box + n_groups * RHS tile): boxes are sorted heaviest first and
  // every slot of a box is dispatched before the next box, so the long workgroups start first
  const int g = blockIdx.x;
  const int64_t slot = blockIdx.y;
  // HB = 2: the groups are half boxes (halves adjacent), so the half is the group's parity
  const int grp = blockIdx.z % n_groups;
  const int toff = HB == 2 ? (grp & 1) * NB : 0;   // first target of this part of the box
  const int r0 = (blockIdx.z / n_groups) * RC;
  const int lane = threadIdx.x % WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int wr = wave % WR, wt = wave / WR;
  const int nMt = Pp / 16;
  const int a_units = Pp * KC / EPU;
  typename MF::acc_t acc[NTW][TPW];
#pragma unroll
  for (int s = 0; s < NTW; ++s)
#pragma unroll
    for (int j = 0; j < TPW; ++j) acc[s][j] = (typename MF::acc_t){0, 0, 0, 0};
  // chunk g of this box (boundaries balanced by estimated work, computed on the host)
  const int ea = chunk_first[grp * (G + 1) + g], eb = chunk_first[grp * (G + 1) + g + 1];
  // raw buffer views of this slot's x_hat and C: an offset past the end reads zeros
  // without touching memory (targets that do not use an entry's class)
  const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(xh + slot * nodes * Pp * Rs), (short)0, (int)(nodes * Pp * Rs * (int64_t)sizeof(S)), BUF_WORD3);
  const __amdgpu_buffer_rsrc_t crs =
      __builtin_amdgcn_make_buffer_rsrc((void*)(C + slot * Cps), (short)0, (int)(Cps * (int64_t)sizeof(S)), BUF_WORD3);
  const int nk = Pp / KC;
  const int nsteps = (eb - ea) * nk;
  constexpr int A_LDS_UNITS = MT * 256 / EPU;
  u4 areg[PD][AU], breg[PD][TSW][BUT];
  S preg[PD];   // packed mode: this thread's element (k = tid / 16, column tid % 16) of B
  // every load and LDS store below is unconditional (clamped stage, out-of-range offsets),
  // so the compiler tracks each register's pending load exactly and waits only at stash
  auto fetch = [&](int step, int rb) {
    const int e = ea + step / nk, kc = step % nk;
    const int cbase = (ent_cls[e] * Pp * Pp + kc * Pp * KC) * (int)sizeof(S);
#pragma unroll
    for (int q = 0; q < AU; ++q) {
      const int u = threadIdx.x + q * NTH;
      const int off = (FULL || u < a_units) ? cbase + u * 16 : BUF_OOB;
      areg[rb][q] = __builtin_amdgcn_raw_buffer_load_b128(crs, off, 0, 0);
    }
    if constexpr (PACK) {
      if (NTH == 256 || threadIdx.x < 256) {
        // the 16 sources of the entry are wave-uniform (scalar loads); pick this lane's
        const int c = lane & 15, k = threadIdx.x >> 4;
        int tv = ent_tau[e * NTG];
#pragma unroll
        for (int i = 1; i < NTG; ++i) {
          const int ti = ent_tau[e * NTG + i];
          tv = c == i ? ti : tv;
        }
        const int off = tv >= 0 ? ((tv * Pp + kc * KC + k) * (int)Rs + r0) * (int)sizeof(S) : BUF_OOB;
        if constexpr (sizeof(S) == 8)
          preg[rb] = __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(xrs, off, 0, 0));
        else
          preg[rb] = __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(xrs, off, 0, 0));
      }
    } else {
#pragma unroll
      for (int q = 0; q < TSW; ++q) {
        const int tv = ent_tau[e * NTG + toff + wave * TSW + q];
        const int base = ((tv * Pp + kc * KC) * (int)Rs + r0) * (int)sizeof(S);
#pragma unroll
        for (int h = 0; h < BUT; ++h) {
          const int u = lane + 64 * h;
          const int rel = ((u / (RC / EPU)) * (int)Rs + (u % (RC / EPU)) * EPU) * (int)sizeof(S);
          breg[rb][q][h] = __builtin_amdgcn_raw_buffer_load_b128(xrs, tv >= 0 ? base + rel : BUF_OOB, 0, 0);
        }
      }
    }
  };
  auto stash = [&](int rb, int buf) {
#pragma unroll
    for (int q = 0; q < AU; ++q) {
      const int u = threadIdx.x + q * NTH;
      if (u < A_LDS_UNITS) reinterpret_cast<u4*>(As[buf])[u] = areg[rb][q];
    }
    if constexpr (PACK) {
      if (NTH == 256 || threadIdx.x < 256) Bs[buf][0][threadIdx.x] = preg[rb];
    } else {
#pragma unroll
      for (int q = 0; q < TSW; ++q)
#pragma unroll
        for (int h = 0; h < BUT; ++h) reinterpret_cast<u4*>(Bs[buf][wave * TSW + q])[lane + 64 * h] = breg[rb][q][h];
    }
  };
  // one stage: prefetch stage st + PD into ring slot RF, multiply from LDS buffer BUF,
  // store stage st + 1 (ring slot RS) into the other LDS buffer.  With PD = 2 the loads of
  // stage st + 1 were issued a whole stage earlier, so it is stored first and its LDS
  // writes overlap this stage's matrix-core work; with PD = 1 it is stored last.
  auto body = [&](int st, auto BUF, auto RF, auto RS) {
    constexpr int buf = decltype(BUF)::value;
    if (PD == 2) stash(decltype(RS)::value, buf ^ 1);
    fetch(min(st + PD, nsteps - 1), decltype(RF)::value);
    const int e = ea + st / nk;
    bool use[NTW];
#pragma unroll
    for (int s = 0; s < NTW; ++s) use[s] = PACK || ent_tau[e * NTG + toff + wt * NTW + s] >= 0;
    __builtin_amdgcn_s_setprio(1);   // matrix-core phase first when the other workgroup stages
    // KG K-steps of 4 per group: the fragments of a group are read from LDS together, so the
    // wait before the first target's products is paid once per group rather than per K-step
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4 * KG) {
      typename MF::a_t a[KG][TPW];
      S bv[KG][NTW];
#pragma unroll
      for (int g = 0; g < KG; ++g) {
        const int k = kk + 4 * g + (lane >> 4);
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
          const int mt = wr + WR * j;
          if (FULL || mt < nMt) a[g][j] = MF::load_tiled(&As[buf][mt * 256 + k * 16], lane);
        }
#pragma unroll
        for (int s = 0; s < NTW; ++s) bv[g][s] = Bs[buf][wt * NTW + s][k * 16 + (lane & 15)];
      }
#pragma unroll
      for (int s = 0; s < NTW; ++s) {
        if (!use[s]) continue;
#pragma unroll
        for (int g = 0; g < KG; ++g)
#pragma unroll
          for (int j = 0; j < TPW; ++j)
            if (FULL || wr + WR * j < nMt) acc[s][j] = MF::mac(a[g][j], bv[g][s], acc[s][j]);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if (PD == 1) stash(decltype(RS)::value, buf ^ 1);
    __syncthreads();
  };
  typedef std::integral_constant<int, 0> I0;
  typedef std::integral_constant<int, 1> I1;
  typedef std::integral_constant<int, 1 % PD> R1;
  if (nsteps > 0) {
    fetch(0, 0);
    stash(0, 0);
    if (PD == 2) fetch(min(1, nsteps - 1), 1 % PD);
  }
  __syncthreads();
  // stages in pairs, so that LDS buffers and register ring slots are compile-time
#pragma unroll 1
  for (int st = 0; st < nsteps; st += 2) {
    body(st, I0(), I0(), R1());
    if (st + 1 < nsteps) body(st + 1, I1(), R1(), I0());
  }
  S* o = out + (int64_t)g * part_stride + slot * nodes * Pp * Rs;
  if constexpr (PACK) {
    // column c of the tile is target c of the box, right-hand side 0
    const int32_t node = grp_targets[grp * NTG + (lane & 15)];
    if (node >= 0) {
      S* on = o + (int64_t)node * Pp * Rs + r0;
#pragma unroll
      for (int j = 0; j < TPW; ++j) {
        const int mt = wr + WR * j;
        if (!FULL && mt >= nMt) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) on[(int64_t)(mt * 16 + MF::row(lane, q)) * Rs] = acc[0][j][q];
      }
    }
    return;
  }
#pragma unroll
  for (int s = 0; s < NTW; ++s) {
    const int32_t node = grp_targets[grp * NTG + toff + wt * NTW + s];
    if (node < 0) continue;
    S* on = o + (int64_t)node * Pp * Rs + r0 + (lane & 15);
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int mt = wr + WR * j;
      if (!FULL && mt >= nMt) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) on[(int64_t)(mt * 16 + MF::row(lane, q)) * Rs] = acc[s][j][q];
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

// Near field on the matrix cores, one workgroup per (leaf s, RHS tile, slot):
//   y_s = sum_{near t} D_st x_t        (writes y_s)
// M = rows of the leaf (row tiles w, w + 4 per wave, in chunks of 128 rows), K = the
// columns of each near block.  Only blocks with s <= t are stored (16-row panels,
// panel_index); for t < s the kernel reads the stored (t, s) block transposed.  Either way
// the 16 x 16 tile a wave needs for one group of 16 columns is one contiguous 2 KB chunk:
// direct blocks are read with one 512-byte row of lanes per K-step, transposed ones with
// 32 contiguous bytes per lane, the K index of the group relabelled (j = 4 kq + u instead
// of 4 u + kq; the x operand follows the same relabelling).  The (block, column group)
// sequence is software pipelined: the next group's D and x values are loaded while the
// current one feeds the MFMAs.
template <typename S, typename DT>
__global__ void __launch_bounds__(NT) k_near_mvm(
    const S* __restrict__ xt, S* __restrict__ yt, const DT* __restrict__ D, const int64_t* __restrict__ nbegin,
    const int64_t* __restrict__ nend, const int64_t* __restrict__ rowptr, const int64_t* __restrict__ ntb,
    const int32_t* __restrict__ nnt, const int32_t* __restrict__ ntr, const int64_t* __restrict__ nD,
    const int32_t* __restrict__ items, int32_t leaf0, int64_t n, int64_t R, int64_t N_nf, int xcd) {
  typedef Mfma<S> MF;
  constexpr int CH = 128;
  // One workgroup per work item = (leaf, 128-row chunk of it), so that the large leaves of
  // uneven point sets are spread over several workgroups.  Workgroups are dealt to the 8
  // XCDs round robin; with xcd set, XCD x gets the contiguous item range [x q, x q + q)
  // (q = items / 8), a compact region of space, so that the two reads of a stored block
  // (for s and, transposed, for t) mostly meet in the same L2.  The host sets it only when
  // those ranges carry about equal work (uneven point sets leave it off: one XCD would get
  // the dense region).
  const int nl = gridDim.x, q8 = nl / 8;
  const int32_t it = xcd && (int)blockIdx.x < 8 * q8 ? (int)(blockIdx.x % 8) * q8 + (int)(blockIdx.x / 8)
                                                      : (int)blockIdx.x;
  const int32_t li = items[2 * it], cstart = items[2 * it + 1];
  const int32_t s = leaf0 + li;
  const int r0 = blockIdx.y * RC;
  const int64_t slot = blockIdx.z;
  const int lane = threadIdx.x % WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int m16 = lane & 15, kq = lane >> 4;
  const int64_t b = nbegin[s], ns = nend[s] - b;
  const bool colok = r0 + m16 < R;
  const S* xs = xt + slot * n * R;
  const DT* Ds = D + slot * N_nf;
  const int64_t bb0 = rowptr[li], bb1 = rowptr[li + 1];
  for (int64_t c0 = cstart; c0 < ns && c0 < cstart + CH; c0 += CH) {
    const int cn = (int)min<int64_t>(CH, ns - c0);
    const int64_t i0 = c0 + wave * 16 + m16, i1 = c0 + (wave + 4) * 16 + m16;   // rows of the leaf
    const bool t0ok = wave * 16 < cn, t1ok = (wave + 4) * 16 < cn;
    const bool r0ok = i0 < c0 + cn, r1ok = i1 < c0 + cn;
    typename MF::acc_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    // pipeline state: block bb, column group kb (16 columns = 4 MFMA K-steps)
    int64_t bb = bb0;
    int kb = 0;
    S a0n[4], a1n[4], bn[4];
    auto fetch = [&](int64_t fb, int fk) {
      const DT* Db = Ds + nD[fb];
      const int64_t tb = ntb[fb];
      const int nt = nnt[fb];
      if (ntr[fb] == 0) {
        // stored (s, t): entry (i, j) at panel_index(i, j, nt)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = fk * 16 + u * 4 + kq;
          const bool jok = j < nt;
          bn[u] = (jok && colok) ? xs[(tb + j) * R + r0 + m16] : (S)0;
          a0n[u] = (jok && r0ok) ? widen<S, DT>(Db[panel_index(i0, j, nt)]) : (S)0;
          a1n[u] = (jok && r1ok) ? widen<S, DT>(Db[panel_index(i1, j, nt)]) : (S)0;
        }
      } else {
        // stored (t, s), n_t rows (zero-padded to 16) x n_s columns: entry (i, j) of D_st
        // at panel_index(j, i, ns); this lane's four K-steps u are j = 16 fk + 4 kq + u
        const int jq = fk * 16 + kq * 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          bn[u] = (jq + u < nt && colok) ? xs[(tb + jq + u) * R + r0 + m16] : (S)0;
          a0n[u] = (S)0;
          a1n[u] = (S)0;
        }
        if (r0ok) Load4<S, DT>::get(Db + panel_index(jq, i0, ns), a0n);
        if (r1ok) Load4<S, DT>::get(Db + panel_index(jq, i1, ns), a1n);
      }
    };
    if (bb < bb1) fetch(bb, kb);
    while (bb < bb1) {
      S a0[4], a1[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a0[u] = a0n[u];
        a1[u] = a1n[u];
        bv[u] = bn[u];
      }
      ++kb;
      if (kb * 16 >= nnt[bb]) {
        ++bb;
        kb = 0;
      }
      if (bb < bb1) fetch(bb, kb);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (t0ok) acc0 = MF::mac(a0[u], bv[u], acc0);
        if (t1ok) acc1 = MF::mac(a1[u], bv[u], acc1);
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


// Near field with one right-hand side, every stored block read once.  With R = 1 there is
// no matrix product for the matrix cores, so this is plain FMA streaming: the workgroup of
// leaf s (one per leaf and slot) walks the 4-column groups of its stored blocks D_st, t >= s;
// wave w takes every fourth group, and lane (r = l % 16, c = l / 16) reads rows 16 p + r of
// column 4 g + c of every 16-row panel p (one 512-byte run per panel and wave):
//   y_s[16 p + r] += D[16 p + r][j] x_t[j]   (summed over lanes and waves at the end)
//   z_st[j] = sum_i D[i][j] x_s[i]          (over the lane's panels, then the 16 lanes of
//                                            its column; t > s only)
// z goes to the pair buffer and k_near_gather adds it into y_t.  A chunk covers MP panels
// (chosen on the host from the leaf sizes); larger leaves take several row chunks and later
// chunks add to z (same lane, same element).
// sum over the 16 lanes of each row of the wavefront (valid in lane 15 of the row): DPP
// row shifts with zero fill, on the 32-bit halves of a double
template <int SH, typename S>
__device__ __forceinline__ S row_shr_add(S v) {
  S u;
  if constexpr (sizeof(S) == 8) {
    typedef int i2 __attribute__((ext_vector_type(2)));
    i2 h = __builtin_bit_cast(i2, v);
    h[0] = __builtin_amdgcn_mov_dpp(h[0], 0x110 + SH, 0xf, 0xf, true);
    h[1] = __builtin_amdgcn_mov_dpp(h[1], 0x110 + SH, 0xf, 0xf, true);
    u = __builtin_bit_cast(S, h);
  } else {
    u = __builtin_bit_cast(S, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x110 + SH, 0xf, 0xf, true));
  }
  return v + u;
}
template <typename S>
__device__ __forceinline__ S row_sum16(S v) {
  return row_shr_add<8>(row_shr_add<4>(row_shr_add<2>(row_shr_add<1>(v))));
}

template <typename S, typename DT, int MP>
__global__ void __launch_bounds__(NT) k_near_gemv(
    const S* __restrict__ xt, S* __restrict__ yt, S* __restrict__ zb, const DT* __restrict__ D,
    const int64_t* __restrict__ nbegin, const int64_t* __restrict__ nend, const int64_t* __restrict__ up_rowptr,
    const int64_t* __restrict__ up_tb, const int32_t* __restrict__ up_nt, const int64_t* __restrict__ up_D,
    const int64_t* __restrict__ up_z, int32_t leaf0, int64_t n, int64_t N_nf, int64_t Zt, int xcd) {
  constexpr int SS = (int)sizeof(S), SD = (int)sizeof(DT);
  __shared__ S ysum[4][MP * 16];
  const int nl = gridDim.x, q8 = nl / 8;
  const int32_t li = xcd && (int)blockIdx.x < 8 * q8 ? (int)(blockIdx.x % 8) * q8 + (int)(blockIdx.x / 8)
                                                      : (int)blockIdx.x;
  const int32_t s = leaf0 + li;
  const int64_t slot = blockIdx.y;
  const int lane = threadIdx.x % WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int r = lane & 15, cq = lane >> 4;
  const int64_t b = nbegin[s], ns = nend[s] - b;
  const S* xs = xt + slot * n;
  S* ys = yt + slot * n;
  S* zs = zb + slot * Zt;
  // byte ranges checked on the host (below BUF_MAX_BYTES)
  const __amdgpu_buffer_rsrc_t dr =
      __builtin_amdgcn_make_buffer_rsrc((void*)(D + slot * N_nf), (short)0, (int)(N_nf * SD), BUF_WORD3);
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)xs, (short)0, (int)(n * SS), BUF_WORD3);
  const __amdgpu_buffer_rsrc_t zr = __builtin_amdgcn_make_buffer_rsrc((void*)zs, (short)0, (int)(Zt * SS), BUF_WORD3);
  const int64_t bb0 = up_rowptr[li], bb1 = up_rowptr[li + 1];
  for (int64_t c0 = 0; c0 < ns; c0 += MP * 16) {
    const int cn = (int)min<int64_t>(MP * 16, ns - c0);
    const int np = (cn + 15) >> 4;
    S xsr[MP], yacc[MP];
#pragma unroll
    for (int p = 0; p < MP; ++p) {
      const int i = 16 * p + r;
      xsr[p] = i < cn ? xs[b + c0 + i] : (S)0;
      yacc[p] = (S)0;
    }
    // this wave's groups: the flattened (block, 4-column group) sequence from index `wave`
    // in steps of 4 (wave-uniform)
    int64_t bb = bb0;
    int g = wave;
    // (block indices are made visibly wave-uniform so that the metadata is read with
    // scalar loads, which do not wait on the vector loads in flight)
    auto settle = [&](int64_t& fb, int& fg) {
      while (fb < bb1) {
        const int ngr = (up_nt[__builtin_amdgcn_readfirstlane((int)fb)] + 3) >> 2;
        if (fg < ngr) break;
        fg -= ngr;
        ++fb;
      }
      fb = __builtin_amdgcn_readfirstlane((int)fb);
      fg = __builtin_amdgcn_readfirstlane(fg);
    };
    settle(bb, g);
    S v[MP], vn[MP], xc = (S)0, xcn = (S)0;
    auto fetch = [&](int64_t fb, int fg, S (&vo)[MP], S& xo) {
      const bool valid = fb < bb1;
      const int fc = __builtin_amdgcn_readfirstlane((int)(valid ? fb : bb1 - 1));
      const int nt = up_nt[fc];
      const int col = 4 * fg + cq;
      const bool ok = valid && col < nt;
      const int dbase = (int)up_D[fc] + (int)panel_index((int)c0 + r, col, nt);
#pragma unroll
      for (int p = 0; p < MP; ++p)
        vo[p] = widen<S, DT>(bload1<DT>(dr, ok && p < np ? (dbase + 16 * p * nt) * SD : BUF_OOB));
      xo = bload1<S>(xr, ok ? (int)((up_tb[fc] + col) * SS) : BUF_OOB);
    };
    if (bb < bb1) fetch(bb, g, v, xc);
    while (bb < bb1) {
      const int bu = __builtin_amdgcn_readfirstlane((int)bb);
      const int nt = up_nt[bu];
      const int64_t zo = up_z[bu];
      const int col = 4 * g + cq;
      const bool zok = zo >= 0 && col < nt;
      // after the first chunk: the partial z of this column (issued before the prefetch)
      const S zold = bload1<S>(zr, zok && c0 > 0 ? (int)((zo + col) * SS) : BUF_OOB);
      g += 4;
      settle(bb, g);
      fetch(bb, g, vn, xcn);
      S zacc = (S)0;
#pragma unroll
      for (int p = 0; p < MP; ++p) {
        yacc[p] += v[p] * xc;
        zacc += v[p] * xsr[p];
      }
      if (zo >= 0) {
        zacc = row_sum16(zacc);
        if (zok && r == 15) zs[zo + col] = zold + zacc;
      }
#pragma unroll
      for (int p = 0; p < MP; ++p) v[p] = vn[p];
      xc = xcn;
    }
    // sum y over the four columns of a lane group, then over the waves (fixed order)
#pragma unroll
    for (int p = 0; p < MP; ++p) {
      S t = yacc[p];
      t += __shfl_xor(t, 16);
      t += __shfl_xor(t, 32);
      if (cq == 0) ysum[wave][16 * p + r] = t;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cn; i += NT)
      ys[b + c0 + i] = ysum[0][i] + ysum[1][i] + ysum[2][i] + ysum[3][i];
    __syncthreads();
  }
}

// y_t += sum of the pair buffers z_ut (u < t) of leaf t in list order (one right-hand side),
// one workgroup per (leaf, slot)
template <typename S>
__global__ void __launch_bounds__(NT) k_near_gather(S* __restrict__ yt, const S* __restrict__ zb,
                                                    const int64_t* __restrict__ nbegin,
                                                    const int64_t* __restrict__ nend,
                                                    const int64_t* __restrict__ lo_rowptr,
                                                    const int64_t* __restrict__ lo_z, int32_t leaf0, int64_t n,
                                                    int64_t Zt) {
  const int32_t li = blockIdx.x, s = leaf0 + li;
  const int64_t slot = blockIdx.y;
  const int64_t b = nbegin[s], ns = nend[s] - b;
  const int64_t q0 = lo_rowptr[li], q1 = lo_rowptr[li + 1];
  if (q0 == q1) return;
  S* ys = yt + slot * n + b;
  const S* zs = zb + slot * Zt;
  for (int64_t i = threadIdx.x; i < ns; i += NT) {
    S acc = ys[i];
    for (int64_t q = q0; q < q1; ++q) acc += zs[lo_z[q] + i];
    ys[i] = acc;
  }
}

// FastBackward, leaves: y_s += U_s y_hat_s on the matrix cores, one workgroup per
// (leaf, RHS tile, slot); U_s[i, i'] = prod_k U_k[i][i'_k] formed from factor rows in LDS.
template <typename S>
__global__ void __launch_bounds__(NT) k_leaf_down(S* __restrict__ yt, const S* __restrict__ yh,
                                                  const double* __restrict__ U,
                                                  const int64_t* __restrict__ nbegin,
                                                  const int64_t* __restrict__ nend,
                                                  const int32_t* __restrict__ items, int32_t leaf0, int d,
                                                  int ps, int P, int Pp, int64_t n, int64_t nodes, int64_t R) {
  typedef Mfma<S> MF;
  constexpr int CH = 128;
  __shared__ double Us[CH * 22];
  __shared__ int Dg[128 * 3];   // per multi-index i < Pp: offsets k ps + i_k of its d digits in a Us row
  // one workgroup per (leaf, 128-row chunk): the chunks of a leaf are independent here
  const int32_t s = leaf0 + items[2 * blockIdx.x], cstart = items[2 * blockIdx.x + 1];
  const int r0 = blockIdx.y * RC;
  const int64_t slot = blockIdx.z;
  const int lane = threadIdx.x % WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int m16 = lane & 15, kq = lane >> 4;
  const int64_t b = nbegin[s], ns = nend[s] - b;
  const int dps = d * ps;
  const bool colok = r0 + m16 < R;
  const S* yhs = yh + (slot * nodes + s) * Pp * R;
  for (int i = threadIdx.x; i < Pp; i += NT) {
    int rem = i;
    for (int k = 0; k < 3; ++k) {
      Dg[i * 3 + k] = k * ps + rem % ps;
      rem /= ps;
    }
  }
  S* ys = yt + slot * n * R;
  for (int64_t c0 = cstart; c0 < ns && c0 < cstart + CH; c0 += CH) {
    const int cn = (int)min<int64_t>(CH, ns - c0);
    __syncthreads();
    for (int q = threadIdx.x; q < cn * dps; q += NT) Us[q] = U[(b + c0) * dps + q];
    __syncthreads();
    const int i0 = wave * 16 + m16, i1 = (wave + 4) * 16 + m16;
    const bool t0ok = wave * 16 < cn, t1ok = (wave + 4) * 16 < cn;
    const bool r0ok = i0 < cn, r1ok = i1 < cn;
    typename MF::acc_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    // y_hat values of 8 K-steps are loaded together (one global load per K-step otherwise
    // leaves the loop waiting on memory latency at every step)
    for (int kb = 0; kb < Pp; kb += 32) {
      S by[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int iq = kb + 4 * q + kq;
        by[q] = (iq < P && colok) ? yhs[(int64_t)iq * R + r0 + m16] : (S)0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int ii = kb + 4 * q + kq;
        if (kb + 4 * q >= Pp) break;
        const bool iok = ii < P;
        const int* dg = &Dg[(iok ? ii : 0) * 3];
        double u0 = 0.0, u1 = 0.0;
        if (iok && r0ok) {
          u0 = Us[i0 * dps + dg[0]];
          for (int k = 1; k < d; ++k) u0 *= Us[i0 * dps + dg[k]];
        }
        if (iok && r1ok) {
          u1 = Us[i1 * dps + dg[0]];
          for (int k = 1; k < d; ++k) u1 *= Us[i1 * dps + dg[k]];
        }
        if (t0ok) acc0 = MF::mac((S)u0, by[q], acc0);
        if (t1ok) acc1 = MF::mac((S)u1, by[q], acc1);
      }
    }
    if (colok) {
      for (int q = 0; q < 4; ++q) {
        const int ra = wave * 16 + MF::row(lane, q), rb = (wave + 4) * 16 + MF::row(lane, q);
        if (t0ok && ra < cn) {
          S* p = ys + (b + c0 + ra) * R + r0 + m16;
          *p = *p + acc0[q];
        }
        if (t1ok && rb < cn) {
          S* p = ys + (b + c0 + rb) * R + r0 + m16;
          *p = *p + acc1[q];
        }
      }
    }
  }
}

static inline int ilog2(int g) {
  int c = 0;
  while ((1 << c) < g) ++c;
  return c;
}

template <typename S, typename DT>
void matvec_impl(InstData& in, const S* x, S* y, int64_t R, double alpha, double beta, double nugget,
                 hipStream_t st, const ExtScratch* ext) {
  const DeviceModel& m = *in.m;
  const TreeData& t = *m.tree;
  const int64_t T = in.T;
  // one right-hand side is stored unpadded (the coupling packs box targets instead)
  const int64_t Rs = R == 1 ? 1 : rhs_stride(R);
  const int64_t nrc = (Rs + RC - 1) / RC;
  // parametric H-matrix format: explicit far factors per block instead of the H^2 far chain
  const bool hfmt = m.format == PH_FORMAT_H;
  const bool use_far = m.min_far >= 0 && !hfmt;
  const bool use_hfar = hfmt && m.n_hblk > 0;
  // implicit coupling (Alg. "Modified H^2-Matrix MVM"): the H^2 chain with L_q H_q R_q^T
  // applied per far block instead of the formed C
  const bool imp = m.format == PH_FORMAT_H2_IMPLICIT && use_far;
  const bool need_w = use_hfar || imp;
  if (m.format != PH_FORMAT_H2 && sizeof(S) != sizeof(double))
    fail(PH_EUNSUPPORTED, "ph_matvec: H-matrix and implicit-coupling models are FP64 only");
  // class-list chunks per target box: 8 (one per XCD) unless the lists are too short;
  // PH_COUPLING_CHUNKS overrides (tuning)
  // launch configuration: environment override (tuning sweeps), else ph_autotune's
  // choice, else the heuristic (8 chunks, prefetch 1, near field overlapped)
  // Pp = 128: each box in two halves of 8 targets (4 waves, 64 KB of LDS), so two
  // workgroups share a CU and their stage barriers fall at different times; one
  // workgroup per box: 5.54 ms, halves: 5.28 ms on the benchmark (PH_COUPLING_HALF=0
  // selects whole boxes; quarters measured 5.4-5.6 ms)
  int hb = 2;
  if (const char* env = std::getenv("PH_COUPLING_HALF")) hb = std::atoi(env) == 0 ? 1 : 2;
  // BF16 instances with right-hand-side tiles: the coupling on the BF16 matrix cores (whole
  // boxes); PH_BF16_COUPLING=0 keeps the FP32 products
  bool bf16_mc = sizeof(DT) == 2 && in.Cb.n > 0 && use_far && coupling_bf16_supported(m, Rs);
  if (const char* env = std::getenv("PH_BF16_COUPLING")) bf16_mc = bf16_mc && std::atoi(env) != 0;
  if (Rs == 1 || m.Pp / 16 != 8 || bf16_mc) hb = 1;
  int G = 1;   // a power of two <= 64 (half boxes double the workgroups: 4 chunks)
  if (use_far && m.n_groups > 0) G = m.max_group_entries >= 16 ? 8 / hb : (m.max_group_entries >= 4 ? 2 : 1);
  if (in.tune_chunks > 0) G = in.tune_chunks;
  if (const char* env = std::getenv("PH_COUPLING_CHUNKS")) {
    const int g = std::atoi(env);
    if (g >= 1 && g <= 64 && (g & (g - 1)) == 0) G = g;
  }
  if (imp) G = 1;   // the implicit coupling writes y_hat directly
  // PH_SERIAL_MVM=1 runs the near field on the caller's stream (no overlap; profiling)
  bool serial = in.tune_overlap != 1;   // default: one stream (sharing the GPU measured no gain)
  if (const char* env = std::getenv("PH_SERIAL_MVM")) serial = std::atoi(env) != 0;
  hipStream_t nst = serial ? st : in.aux;
  // the single-RHS near kernel addresses a slot's blocks, x and pair buffer with 32-bit
  // byte offsets
  const bool gemv_ok = m.N_nf_pad * (int64_t)in.d_esize <= BUF_MAX_BYTES &&
                       m.n * (int64_t)sizeof(S) <= BUF_MAX_BYTES && m.Zt * (int64_t)sizeof(S) <= BUF_MAX_BYTES;
  const bool need_zb = Rs == 1 && gemv_ok && m.Zt > 0 && !in.factored;
  if (use_far && (m.n_nodes * m.Pp * Rs * (int64_t)sizeof(S) > BUF_MAX_BYTES ||
                  m.n_classes * m.Pp * m.Pp * (int64_t)sizeof(S) > BUF_MAX_BYTES))
    fail(PH_EUNSUPPORTED, "ph_matvec: per-slot coupling buffers exceed 2 GiB (reduce R)");
  S *xt, *yt, *xh, *yh, *partp = nullptr, *zbp = nullptr;
  void* xbp = nullptr;
  double* hwp = nullptr;   // H-matrix format: w_b = H_b T_b^T x_t per far block
  if (ext) {
    // caller-provided scratch (no allocation): the same buffers carved at 256-byte offsets
    size_t off = 0;
    auto carve = [&](size_t bytes) {
      char* q = (char*)ext->base + off;
      off += (bytes + 255) / 256 * 256;
      return (S*)q;
    };
    xt = carve((size_t)T * m.n * Rs * sizeof(S));
    yt = carve((size_t)T * m.n * Rs * sizeof(S));
    xh = carve((size_t)T * m.n_nodes * m.Pp * Rs * sizeof(S));
    yh = carve((size_t)T * m.n_nodes * m.Pp * Rs * sizeof(S));
    if (G > 1) partp = carve((size_t)G * T * m.n_nodes * m.Pp * Rs * sizeof(S));
    if (need_zb) zbp = carve((size_t)T * m.Zt * sizeof(S));
    if (bf16_mc) xbp = carve((size_t)T * coupling_bf16_x_bytes(m, Rs));
    if (need_w) hwp = (double*)carve((size_t)T * nrc * m.hw_tot * sizeof(double));
    if (off > ext->bytes)
      fail(PH_EINVAL, "ph_matvec_noalloc: this MVM needs " + std::to_string(off) + " bytes of scratch, more than the " +
                          std::to_string(ext->bytes) + " the library reserves per GPU");
  } else {
  if (Rs > in.Rcap || G > in.Gcap) {
    if (in.graphs > 0) fail(PH_ESTATE, "ph_matvec: the instance has recorded graphs, its scratch cannot grow");
    const int64_t Rc = std::max<int64_t>(Rs, in.Rcap);
    const int Gc = std::max(G, in.Gcap);
    in.xt.alloc((size_t)T * m.n * Rc * sizeof(S));
    in.yt.alloc((size_t)T * m.n * Rc * sizeof(S));
    in.xh.alloc((size_t)T * m.n_nodes * m.Pp * Rc * sizeof(S));
    in.yh.alloc((size_t)T * m.n_nodes * m.Pp * Rc * sizeof(S));
    if (Gc > 1) in.part.alloc((size_t)Gc * T * m.n_nodes * m.Pp * Rc * sizeof(S));
    in.Rcap = Rc;
    in.Gcap = Gc;
  }
  if (need_zb && in.zb.n == 0) {
    if (in.graphs > 0) fail(PH_ESTATE, "ph_matvec: the instance has recorded graphs, its scratch cannot grow");
    in.zb.alloc((size_t)T * m.Zt * sizeof(S));
  }
  xt = (S*)in.xt.p;
  yt = (S*)in.yt.p;
  xh = (S*)in.xh.p;
  yh = (S*)in.yh.p;
  partp = (S*)in.part.p;
  zbp = (S*)in.zb.p;
  if (bf16_mc) {
    const size_t need = (size_t)T * coupling_bf16_x_bytes(m, Rs);
    if (in.xb.n < need) {
      if (in.graphs > 0) fail(PH_ESTATE, "ph_matvec: the instance has recorded graphs, its scratch cannot grow");
      in.xb.alloc(need);
    }
    xbp = in.xb.p;
  }
  if (need_w) {
    const size_t need = (size_t)T * nrc * m.hw_tot * sizeof(double);
    if (in.hw.n < need) {
      if (in.graphs > 0) fail(PH_ESTATE, "ph_matvec: the instance has recorded graphs, its scratch cannot grow");
      in.hw.alloc(need);
    }
    hwp = (double*)in.hw.p;
  }
  }
  const int32_t leaf0 = t.leaves.front();
  const int64_t Cps = m.n_classes * m.Pp * m.Pp;
  const int64_t total_in = T * m.n * Rs;
  const dim3 ptile((unsigned)((m.n + 63) / 64), (unsigned)nrc, (unsigned)T);
  if (Rs >= RC)
    launch(PH_STAGE_PERM_IN, k_perm_in_tile<S>, ptile, dim3(NT), st, x, xt, (const int64_t*)m.iperm.p, m.n, R, Rs);
  else
    launch(PH_STAGE_PERM_IN, k_perm_in<S>, dim3((unsigned)grid_for(total_in)), dim3(NT), st, x, xt,
           (const int64_t*)m.perm.p, m.n, R, Rs, total_in);
  // The near field (HBM-bound) runs on the instance's second stream, concurrently with
  // the far-field chain (matrix-core bound) on the caller's stream.  (Forking it after
  // the upward pass instead measured slower: it then overlaps the coupling throughout.)
  auto near_field = [&] {
    if (!serial) {
      // aux is already ordered after a pending near-field instantiation
      PH_HIP(hipEventRecord(in.ev_fork, st));
      PH_HIP(hipStreamWaitEvent(in.aux, in.ev_fork, 0));
      in.near_pending = false;   // joined into st below (ev_join follows the near-field MVM)
    } else {
      join_near(in, st);
    }
    const int xcd = m.near_xcd;
    if (in.factored) {
      // blocks formed from the near factors inside the MVM (no D in memory)
      near_fused_launch<S, DT>(in, xt, yt, Rs, nst);
    } else if (Rs == 1 && gemv_ok) {
      // one right-hand side: every stored block read once, transposed products gathered
      auto gemv = [&](auto kern) {
        launch(PH_STAGE_NEAR_MVM, kern, dim3((unsigned)m.n_leaves, (unsigned)T), dim3(NT), nst, (const S*)xt, yt,
               zbp, (const DT*)in.D.p, (const int64_t*)m.nbegin.p, (const int64_t*)m.nend.p,
               (const int64_t*)m.up_rowptr.p, (const int64_t*)m.up_tb.p, (const int32_t*)m.up_nt.p,
               (const int64_t*)m.up_D.p, (const int64_t*)m.up_z.p, leaf0, m.n, m.N_nf_pad, m.Zt, xcd);
      };
      int mp = m.gemv_mp;
      if (const char* e = std::getenv("PH_GEMV_PANELS")) mp = std::atoi(e);   // tuning: 4, 8 or 12
      if (mp <= 4) gemv(k_near_gemv<S, DT, 4>);
      else if (mp <= 8) gemv(k_near_gemv<S, DT, 8>);
      else gemv(k_near_gemv<S, DT, 12>);
      launch(PH_STAGE_NEAR_GATHER, k_near_gather<S>, dim3((unsigned)m.n_leaves, (unsigned)T), dim3(NT), nst, yt,
             (const S*)zbp, (const int64_t*)m.nbegin.p, (const int64_t*)m.nend.p,
             (const int64_t*)m.lo_rowptr.p, (const int64_t*)m.lo_z.p, leaf0, m.n, m.Zt);
    } else {
      launch(PH_STAGE_NEAR_MVM, k_near_mvm<S, DT>, dim3((unsigned)m.n_mvm_items, (unsigned)nrc, (unsigned)T),
             dim3(NT), nst, (const S*)xt, yt, (const DT*)in.D.p, (const int64_t*)m.nbegin.p,
             (const int64_t*)m.nend.p, (const int64_t*)m.near_rowptr.p, (const int64_t*)m.near_tb.p,
             (const int32_t*)m.near_nt.p, (const int32_t*)m.near_tr.p, (const int64_t*)m.near_D.p,
             (const int32_t*)m.mvm_items.p, leaf0, m.n, Rs, m.N_nf_pad, xcd);
    }
    if (!serial) PH_HIP(hipEventRecord(in.ev_join, in.aux));
  };
  near_field();
  if (use_far) {
    launch(PH_STAGE_LEAF_UP, k_leaf_up<S>, dim3((unsigned)m.n_leaves, (unsigned)nrc, (unsigned)T), dim3(NT),
           st, (const S*)xt, xh, (const double*)m.U.p, (const int64_t*)m.nbegin.p, (const int64_t*)m.nend.p,
           leaf0, m.d, m.p_s, m.P, m.Pp, m.n, m.n_nodes, Rs);
    for (int l = m.l_max - 1; l >= m.min_far; --l) {
      const int32_t a = t.level_start[l], b = t.level_start[l + 1];
      launch(PH_STAGE_TRANSFER_UP, Rs == 1 ? k_transfer_up<S, 0> : k_transfer_up<S, 4>,
             dim3((unsigned)(b - a), (unsigned)nrc, (unsigned)T),
             dim3(NT), st, xh, (const double*)m.E.p, (const int32_t*)m.first_child.p,
             (const int32_t*)m.nchild.p, (const int32_t*)m.cid.p, a, m.d, m.p_s, m.P, m.Pp, m.n_nodes, Rs);
    }
    const int64_t part_stride = T * m.n_nodes * m.Pp * Rs;
    const bool pack = Rs == 1;   // packed coupling (box targets as matrix-core columns)
    S* cout = G > 1 ? partp : yh;
    const int64_t ngr = hb == 2 ? m.n_hgroups : m.n_groups;
    if (T > 65535 || ngr * nrc > 65535)
      fail(PH_EUNSUPPORTED, "ph_matvec: too many parameter slots or target boxes x RHS tiles for one launch");
    dim3 cg((unsigned)G, (unsigned)T, (unsigned)(ngr * nrc));
    auto run = [&](auto kern, int nw) {
      if (hb == 2)
        launch(PH_STAGE_COUPLING, kern, cg, dim3(64 * nw), st, (const S*)xh, cout, (const S*)in.C.p,
               (const int32_t*)m.hgrp_targets.p, (const int32_t*)nullptr, (const int32_t*)m.hent_cls.p,
               (const int32_t*)m.hent_tau.p, (const int32_t*)m.hchunk_first.p + m.hchunk_off[ilog2(G)], m.Pp,
               m.n_nodes, Rs, G, Cps, part_stride, (int)ngr);
      else
        launch(PH_STAGE_COUPLING, kern, cg, dim3(64 * nw), st, (const S*)xh, cout, (const S*)in.C.p,
               (const int32_t*)m.grp_targets.p, (const int32_t*)m.grp_entry.p, (const int32_t*)m.ent_cls.p,
               (const int32_t*)m.ent_tau.p, (const int32_t*)m.chunk_first.p + m.chunk_off[ilog2(G)], m.Pp,
               m.n_nodes, Rs, G, Cps, part_stride, (int)ngr);
    };
    if (imp) {
      implicit_coupling_launch(in, (const double*)xh, (double*)yh, hwp, Rs, nrc, st);
    } else if (bf16_mc) {
      coupling_bf16_launch(in, (const float*)xh, xbp, (float*)cout, G, Rs, nrc, t.level_start[m.min_far], st);
    } else {
    // 8 waves (4 row groups x 2 target halves) for Pp > 64, else 4 waves over the targets;
    // register prefetch depth 2 (PH_COUPLING_PD or the autotuner may select 1)
    // (half boxes: depth 1 measured 0.5% faster)
    int pd = in.tune_prefetch > 0 ? in.tune_prefetch : (hb == 2 ? 1 : 2);
    if (const char* env = std::getenv("PH_COUPLING_PD")) pd = std::atoi(env) == 2 ? 2 : 1;
    const int nMt = m.Pp / 16;
    if (pack) {
      // one right-hand side: 4 waves over the row tiles, one 16-target column tile
      if (nMt == 8) {
        if (pd == 2) run(k_coupling<S, 4, 4, 2, 2, true, true>, 4);
        else run(k_coupling<S, 4, 4, 2, 1, true, true>, 4);
      } else if (nMt > 4) {
        run(k_coupling<S, 4, 4, 2, 1, false, true>, 4);
      } else if (nMt == 4) {
        run(k_coupling<S, 4, 4, 1, 1, true, true>, 4);
      } else {
        run(k_coupling<S, 4, 4, 1, 1, false, true>, 4);
      }
    } else if (nMt == 8 && hb == 2) {
      // fragments of two K-steps read per group (KG = 2): 4.75 vs 4.97 ms per launch on the
      // benchmark in a same-box A/B; KG = 4 spills
      if (pd == 2) run(k_coupling<S, 4, 4, 2, 2, true, false, 2>, 4);
      else run(k_coupling<S, 4, 4, 2, 1, true, false, 2, 2>, 4);
    } else if (nMt == 8) {
      if (pd == 2) run(k_coupling<S, 8, 4, 2, 2, true>, 8);
      else run(k_coupling<S, 8, 4, 2, 1, true>, 8);
    } else if (nMt > 4) {
      run(k_coupling<S, 8, 4, 2, 1, false>, 8);
    } else if (nMt == 4) {
      run(k_coupling<S, 4, 1, 4, 1, true>, 4);
    } else if (nMt == 3) {
      run(k_coupling<S, 4, 1, 3, 1, true>, 4);
    } else if (nMt == 2) {
      run(k_coupling<S, 4, 1, 2, 1, true>, 4);
    } else {
      run(k_coupling<S, 4, 1, 1, 1, true>, 4);
    }
    }
    if (G > 1) {
      const int64_t a0 = t.level_start[m.min_far];
      const int64_t node_elems = (int64_t)m.Pp * Rs;
      const int64_t rtotal = T * (m.n_nodes - a0) * node_elems;
      launch(PH_STAGE_ZERO, k_coupling_reduce<S>, dim3((unsigned)grid_for(rtotal)), dim3(NT), st, yh,
             (const S*)partp, G, part_stride, node_elems, a0, m.n_nodes, rtotal);
    }
    for (int l = m.min_far; l < m.l_max; ++l) {
      const int32_t a = t.level_start[l + 1], b = t.level_start[l + 2];
      launch(PH_STAGE_TRANSFER_DOWN, Rs == 1 ? k_transfer_down<S, 0> : k_transfer_down<S, 4>,
             dim3((unsigned)(b - a), (unsigned)nrc, (unsigned)T),
             dim3(NT), st, yh, (const double*)m.E.p, (const int32_t*)m.parent.p, (const int32_t*)m.cid.p, a,
             m.d, m.p_s, m.P, m.Pp, m.n_nodes, Rs);
    }
  }
  if (use_hfar) h_far_launch(in, (const double*)xt, nullptr, hwp, Rs, nrc, st, 0);
  if (!serial) PH_HIP(hipStreamWaitEvent(st, in.ev_join, 0));
  if (use_hfar) h_far_launch(in, nullptr, (double*)yt, hwp, Rs, nrc, st, 1);
  if (use_far)
    launch(PH_STAGE_LEAF_DOWN, k_leaf_down<S>, dim3((unsigned)m.n_mvm_items, (unsigned)nrc, (unsigned)T),
           dim3(NT), st, yt, (const S*)yh, (const double*)m.U.p, (const int64_t*)m.nbegin.p,
           (const int64_t*)m.nend.p, (const int32_t*)m.mvm_items.p, leaf0, m.d, m.p_s, m.P, m.Pp, m.n,
           m.n_nodes, Rs);
  const int64_t total_out = T * m.n * R;
  if (Rs >= RC)
    launch(PH_STAGE_PERM_OUT, k_perm_out_tile<S>, ptile, dim3(NT), st, y, (const S*)yt, (const S*)xt,
           (const int64_t*)m.iperm.p, m.n, R, Rs, alpha, beta, nugget);
  else
    launch(PH_STAGE_PERM_OUT, k_perm_out<S>, dim3((unsigned)grid_for(total_out)), dim3(NT), st, y, (const S*)yt,
           (const S*)xt, (const int64_t*)m.perm.p, m.n, R, Rs, total_out, alpha, beta, nugget);
}

// Bilinear form, first pass: part[t][b] = sum over the elements e = b, b + NB, ... of
// slot t of u[e] v[e] (FP64), then a fixed-order workgroup tree reduction.
constexpr int BIL_BLOCKS = 256;
template <typename S>
__global__ void __launch_bounds__(NT) k_dot_partial(const S* __restrict__ u, const S* __restrict__ v,
                                                    double* __restrict__ part, int64_t per_slot) {
  __shared__ double red[NT];
  const int64_t t = blockIdx.y;
  const S* us = u + t * per_slot;
  const S* vs = v + t * per_slot;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < per_slot; e += (int64_t)BIL_BLOCKS * NT)
    acc += (double)us[e] * (double)vs[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[t * BIL_BLOCKS + blockIdx.x] = red[0];
}

// Second pass: out[t] = sum_b part[t][b] (one workgroup per slot, same fixed order).
__global__ void __launch_bounds__(NT) k_dot_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[NT];
  const int64_t t = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < BIL_BLOCKS; b += NT) acc += part[t * BIL_BLOCKS + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[t] = red[0];
}

template <typename S, typename DT>
void bilinear_impl(InstData& in, const S* u, const S* x, int64_t R, double* out, hipStream_t st) {
  const DeviceModel& m = *in.m;
  const int64_t per_slot = m.n * R;
  const size_t need_bytes = (size_t)in.T * per_slot * sizeof(S);
  if (in.bil.bytes() < need_bytes) in.bil.alloc(need_bytes);
  if (in.bil_part.n < (size_t)in.T * BIL_BLOCKS) in.bil_part.alloc((size_t)in.T * BIL_BLOCKS);
  S* v = (S*)in.bil.p;
  matvec_impl<S, DT>(in, x, v, R, 1.0, 0.0, 0.0, st);
  launch(PH_STAGE_BILINEAR, k_dot_partial<S>, dim3(BIL_BLOCKS, (unsigned)in.T), dim3(NT), st, u, (const S*)v,
         in.bil_part.p, per_slot);
  launch(PH_STAGE_BILINEAR, k_dot_final, dim3((unsigned)in.T), dim3(NT), st, (const double*)in.bil_part.p, out);
}

template void bilinear_impl<double, double>(InstData&, const double*, const double*, int64_t, double*, hipStream_t);
template void bilinear_impl<float, float>(InstData&, const float*, const float*, int64_t, double*, hipStream_t);
template void bilinear_impl<float, bf16>(InstData&, const float*, const float*, int64_t, double*, hipStream_t);

template void matvec_impl<double, double>(InstData&, const double*, double*, int64_t, double, double, double,
                                          hipStream_t, const ExtScratch*);
template void matvec_impl<float, float>(InstData&, const float*, float*, int64_t, double, double, double,
                                        hipStream_t, const ExtScratch*);
template void matvec_impl<float, bf16>(InstData&, const float*, float*, int64_t, double, double, double,
                                       hipStream_t, const ExtScratch*);

}  // namespace ph
