// Factored near field: instances that keep every near block as its factor and core
// (Sec. 4.3: D_b(theta) = reshape(P_b c_b(theta), [n_s, n_t]) is linear in c_b(theta)).
// The instantiation forms only the small vectors c_b(theta_t); the MVM forms each 16 x 4
// piece of D_b(theta_t) in registers from the factor entries, for TCB parameter slots at
// once, and feeds it straight to the matrix cores.  No near block is written to memory and
// each factor entry read from HBM serves TCB slots.
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "ph_device.hpp"

namespace ph {

// c[((q nch + c) T + t) KM + kk] = (core_q x_theta (Theta_k^T v_k(theta_t)))[k] for stored
// block q, slot t and rank k = c KM + kk (rank chunks of KM, nch = KRp / KM chunks; zero for
// r_e <= k < KRp), so that the KM coefficients of the TCB slots a unit of the MVM needs are
// contiguous at compile-time offsets.  The sums run in the same order as in the near-block
// instantiation, so both forms use identical coefficients.
template <typename S>
__global__ void __launch_bounds__(NT) k_near_cores(const NearDev* __restrict__ blocks, const double* __restrict__ core,
                                                   const double* __restrict__ th, const double* __restrict__ v,
                                                   S* __restrict__ cc, int64_t nq, int T, int p, int dth, int KRp,
                                                   int KM) {
  const int64_t total = nq * T * KRp;
  const int nch = KRp / KM;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total; o += (int64_t)gridDim.x * blockDim.x) {
    const int kk = (int)(o % KM);
    const int t = (int)((o / KM) % T);
    const int ch = (int)((o / ((int64_t)KM * T)) % nch);
    const int k = ch * KM + kk;
    const NearDev b = blocks[o / ((int64_t)KRp * T)];
    double s = 0.0;
    if (k < b.r_e) {
      const double* vt = v + (size_t)t * dth * p;
      for (int k2 = 0; k2 < b.r2; ++k2) {
        double w2 = 1.0;
        if (dth == 2) {
          w2 = 0;
          for (int a = 0; a < p; ++a) w2 += th[b.th2_off + a + (size_t)p * k2] * vt[p + a];
        }
        for (int k1 = 0; k1 < b.r1; ++k1) {
          double w1 = 0;
          for (int a = 0; a < p; ++a) w1 += th[b.th1_off + a + (size_t)p * k1] * vt[a];
          s += core[b.core_off + k + (size_t)b.r_e * (k1 + (size_t)b.r1 * k2)] * w1 * w2;
        }
      }
    }
    cc[o] = (S)s;
  }
}

// The matrix-core step of the factored near MVM, y(16 rows x 16 RHS) += d(16 x 4) x(4 x 16),
// with the A operand formed by each lane for its own (row i = l % 16, K = l / 16).
// FP64: four V_MFMA_F64_4X4X4 (4-block) instructions, which issue at twice the rate of
//   V_MFMA_F64_16X16X4 on gfx950.  Block b = (l % 16) / 4 multiplies the rows 4 b .. 4 b + 3
//   that its own lanes formed (no replicated operand) with a 4-column group of x; in
//   instruction q that group is b - q (mod 4), the x register rotated by 4 q lanes within
//   each 16-lane row (DPP row_ror).  Result element q of lane l: row 4 b + l / 16, column
//   4 ((b - q) mod 4) + l % 4.
// FP32: one V_MFMA_F32_16X16X4 (result element q of lane l: row 4 (l / 16) + q, column l % 16).
template <typename S>
struct NearApply;
template <>
struct NearApply<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  template <int N>
  static __device__ __forceinline__ double ror(double v) {
    typedef int i2 __attribute__((ext_vector_type(2)));
    i2 h = __builtin_bit_cast(i2, v);
    h[0] = __builtin_amdgcn_mov_dpp(h[0], 0x120 + N, 0xf, 0xf, false);
    h[1] = __builtin_amdgcn_mov_dpp(h[1], 0x120 + N, 0xf, 0xf, false);
    return __builtin_bit_cast(double, h);
  }
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t acc) {
    acc[0] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, ror<4>(b), acc[1], 0, 0, 0);
    acc[2] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, ror<8>(b), acc[2], 0, 0, 0);
    acc[3] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, ror<12>(b), acc[3], 0, 0, 0);
    return acc;
  }
  static __device__ __forceinline__ int row(int lane, int) { return 4 * ((lane & 15) >> 2) + (lane >> 4); }
  static __device__ __forceinline__ int col(int lane, int q) { return 4 * ((((lane & 15) >> 2) - q) & 3) + (lane & 3); }
};
template <>
struct NearApply<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
  static __device__ __forceinline__ int col(int lane, int) { return lane & 15; }
};

// Near-field MVM from the factors.  One workgroup per (work item = CH-row chunk of a target
// leaf s, 16-column right-hand-side tile, batch of TCB slots); wave w owns row tiles w + 4 r
// (r < RT) of the chunk and walks the leaf's near blocks (s, t) in list order, each in
// K-steps of 4 columns j of t (a unit; ranks in chunks of KM, one chunk when r_e <= KM):
//   d_t(i, j) = sum_k P_b[k](i, j) c_b[k](theta_t)     (FMA, i = row of the lane's tile)
//   y_t(i, :) += d_t(i, j) x_t(j, :)                   (matrix cores, NearApply)
// The stored factor of a pair with s > t is that of (t, s); its entry (i, j) is read at
// j + i ldp instead of i + j ldp, the same code with swapped strides.  Units are software
// pipelined: the next unit's KM factor entries and TCB x values per lane are loaded while
// the current one is computed.  Every load is a raw buffer load at an out-of-range offset
// when masked (zeros, no memory access), and ranks k >= r_e get an empty buffer range.
// The coefficients c_b[k](theta_t) and the block metadata are wave-uniform and read with
// scalar loads (metadata of the current and the next block held in scalar registers), so
// the waves need no LDS and no barrier.
template <typename S, typename PT, int TCB, int RT, int KM>
__global__ void __launch_bounds__(NT) k_near_fused(
    const S* __restrict__ xt, S* __restrict__ yt, const PT* __restrict__ Pf, const S* __restrict__ cc,
    const NearDev* __restrict__ blocks, const int64_t* __restrict__ nbegin, const int64_t* __restrict__ nend,
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ nq, const int32_t* __restrict__ ntr,
    const int64_t* __restrict__ ntb, const int32_t* __restrict__ items, int32_t leaf0, int64_t n, int64_t R,
    int T, int nch, int xcd) {
  typedef NearApply<S> MF;
  constexpr int CH = 64 * RT;
  constexpr int SP = (int)sizeof(PT), SS = (int)sizeof(S);
  const int nl = gridDim.x, q8 = nl / 8;
  const int32_t it = xcd && (int)blockIdx.x < 8 * q8 ? (int)(blockIdx.x % 8) * q8 + (int)(blockIdx.x / 8)
                                                      : (int)blockIdx.x;
  const int32_t li = items[2 * it], cstart = items[2 * it + 1];
  const int32_t s = leaf0 + li;
  const int r0 = blockIdx.y * RC;
  const int slot0 = blockIdx.z * TCB;
  const int tc = min(TCB, T - slot0);
  const int lane = threadIdx.x % WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int m16 = lane & 15, kq = lane >> 4;
  const int64_t b = nbegin[s], ns = nend[s] - b;
  const int cn = (int)min<int64_t>(CH, ns - cstart);
  int irow[RT];
  bool rok[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    irow[r] = cstart + (wave + 4 * r) * 16 + m16;
    rok[r] = (wave + 4 * r) * 16 + m16 < cn;
  }
  const bool colok = r0 + m16 < R;
  // x of this workgroup's tc slots (T n R values in all, byte range checked on the host):
  // slots past tc fall outside the range
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(xt + (int64_t)slot0 * n * R), (short)0, (int)((int64_t)tc * n * R * SS), BUF_WORD3);
  typename MF::acc_t acc[RT][TCB];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int tt = 0; tt < TCB; ++tt) acc[r][tt] = typename MF::acc_t{0, 0, 0, 0};
  const int64_t bb0 = rowptr[li], bb1 = rowptr[li + 1];

  // wave-uniform metadata of a near block of the list.  The coefficients are read through a
  // constant-address-space pointer: uniform loads from it are scalar loads.
  typedef const S __attribute__((address_space(4)))* CPtr;
  struct Meta {
    __amdgpu_buffer_rsrc_t pr;   // factor of the stored block, all r_e ranks
    int nepb;                    // bytes of one rank (padded factor column)
    int xo;                      // byte offset of x(first point of t, r0 + m16) in slot 0
    CPtr cb;                     // c_b(theta_slot0) of rank chunk 0 (chunks T KM apart)
    int ldp, tr, nt, re;
  };
  auto meta = [&](int64_t fb) {
    const int fc = __builtin_amdgcn_readfirstlane((int)fb);
    const int32_t q = nq[fc];
    const NearDev B = blocks[q];
    Meta M;
    M.nepb = B.ldp * B.nt * SP;
    M.pr = __builtin_amdgcn_make_buffer_rsrc((void*)(Pf + B.P_off), (short)0, B.r_e * M.nepb, BUF_WORD3);
    M.xo = (int)((ntb[fc] * R + r0 + m16) * SS);
    M.cb = (CPtr)(cc + ((int64_t)q * nch * T + slot0) * KM);
    M.ldp = B.ldp;
    M.re = B.r_e;
    M.tr = ntr[fc];
    M.nt = M.tr ? B.ns : B.nt;
    return M;
  };
  const int xslot = (int)(n * R * SS);   // bytes of one slot of x
  // loads of one unit into the register set (p, x); x only at the first rank chunk
  auto fetch = [&](const Meta& M, int fg, int fu, int fk, S (&p)[RT][KM], S (&x)[TCB]) {
    const int j = 16 * fg + 4 * fu + kq;
    const bool jok = j < M.nt;
    // masked lanes start at BUF_OOB; adding rank offsets (below 2 GiB in all, checked on
    // the host) keeps them out of range, and ranks k >= r_e fall past the block's range
    int off[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
      off[r] = jok && rok[r] ? (M.tr ? j + irow[r] * M.ldp : irow[r] + j * M.ldp) * SP + fk * KM * M.nepb : BUF_OOB;
#pragma unroll
    for (int kk = 0; kk < KM; ++kk)
#pragma unroll
      for (int r = 0; r < RT; ++r) p[r][kk] = widen<S, PT>(bload1<PT>(M.pr, off[r] + kk * M.nepb));
    if (fk == 0) {
      const int xo = jok && colok ? M.xo + j * (int)(R * SS) : BUF_OOB;
#pragma unroll
      for (int tt = 0; tt < TCB; ++tt) x[tt] = bload1<S>(xr, xo + tt * xslot);
    }
  };
  // a unit of the leaf's sequence: block bb (its metadata M), 16-column group g, K-step u,
  // rank chunk kc; valid while bb < bb1
  struct Unit {
    int64_t bb;
    int g, u, kc;
    Meta M;
  };
  auto next = [&](const Unit& a) {
    Unit b = a;
    if (KM == 16 && ++b.kc * KM < a.M.re) return b;   // below 16 ranks one chunk holds them all
    b.kc = 0;
    if (++b.u < 4) return b;
    b.u = 0;
    if (16 * ++b.g < a.M.nt) return b;
    b.g = 0;
    if (++b.bb < bb1) b.M = meta(b.bb);
    return b;
  };

  if (bb0 < bb1) {
    // two units in flight: the current one is computed while the next one's loads are
    // outstanding (the register sets alternate, so the loop is unrolled twice)
    S p0[RT][KM], p1[RT][KM], x0[TCB], x1[TCB], xv[TCB];
    S d[RT][TCB];
    Unit u0{bb0, 0, 0, 0, meta(bb0)};
    Unit u1 = next(u0);
    fetch(u0.M, u0.g, u0.u, u0.kc, p0, x0);
    auto step = [&](S (&pc)[RT][KM], S (&xc)[TCB], S (&pf)[RT][KM], S (&xf)[TCB]) {
      if (u1.bb < bb1) fetch(u1.M, u1.g, u1.u, u1.kc, pf, xf);
      if (KM < 16 || u0.kc == 0) {
#pragma unroll
        for (int tt = 0; tt < TCB; ++tt) xv[tt] = xc[tt];
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int tt = 0; tt < TCB; ++tt) d[r][tt] = (S)0;
      }
      // coefficients slot by slot, the next slot's loads in flight while the current one's
      // FMAs run: two slots of KM scalars at a time (all TCB KM of them would overflow the
      // scalar registers); the empty asm statements keep the compiler from hoisting them
      const CPtr cbk = u0.M.cb + (int64_t)u0.kc * T * KM;
#pragma unroll
      for (int tt = 0; tt < TCB; ++tt) {
        S cv[KM];
#pragma unroll
        for (int kk = 0; kk < KM; ++kk) cv[kk] = cbk[tt * KM + kk];   // zero for r_e <= k < KRp
#pragma unroll
        for (int kk = 0; kk < KM; ++kk)
#pragma unroll
          for (int r = 0; r < RT; ++r) d[r][tt] += pc[r][kk] * cv[kk];
        asm volatile("" ::: "memory");
      }
      if (KM < 16 || u1.bb >= bb1 || u1.kc == 0) {   // last rank chunk of this K-step
#pragma unroll
        for (int tt = 0; tt < TCB; ++tt)
#pragma unroll
          for (int r = 0; r < RT; ++r) acc[r][tt] = MF::mac(d[r][tt], xv[tt], acc[r][tt]);
      }
      if (u1.bb >= bb1) return false;
      u0 = u1;
      u1 = next(u1);
      return true;
    };
    while (step(p0, x0, p1, x1) && step(p1, x1, p0, x0)) {
    }
  }
#pragma unroll
  for (int tt = 0; tt < TCB; ++tt) {
    if (tt >= tc) break;
    S* ys = yt + (int64_t)(slot0 + tt) * n * R;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = (wave + 4 * r) * 16 + MF::row(lane, q), col = r0 + MF::col(lane, q);
        if (row < cn && col < R) ys[(b + cstart + row) * R + col] = acc[r][tt][q];
      }
  }
}

// One factored near block, evaluated entry by entry for inspection: out (n_s x n_t,
// column-major) = the block the MVM forms for slot t, in the same arithmetic.
template <typename S, typename PT>
__global__ void __launch_bounds__(NT) k_near_block_eval(const NearDev* __restrict__ blocks,
                                                        const PT* __restrict__ Pf, const S* __restrict__ cc,
                                                        int64_t q, int T, int t, int KRp, int KM,
                                                        double* __restrict__ out) {
  const NearDev B = blocks[q];
  const int64_t Ne = (int64_t)B.ns * B.nt, Nep = (int64_t)B.ldp * B.nt;
  const int nch = KRp / KM;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < Ne; o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = o % B.ns, j = o / B.ns;
    S dv = (S)0;
    for (int k = 0; k < B.r_e; ++k)
      dv += widen<S, PT>(Pf[B.P_off + k * Nep + i + j * B.ldp]) * cc[((q * nch + k / KM) * T + t) * KM + k % KM];
    out[o] = (double)dv;
  }
}

// Near factors in a low-precision storage type, rounded to nearest (BF16 via FP32).
template <typename PT>
__global__ void __launch_bounds__(NT) k_round_factors(const double* __restrict__ src, PT* __restrict__ dst, int64_t n) {
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x)
    dst[o] = to_store<PT>(src[o]);
}

// ---- host side

void make_low_factors(const DeviceModel& m, ph_dtype dt, hipStream_t st) {
  std::lock_guard<std::mutex> lk(m.lowp_mu);
  const int64_t n = (int64_t)m.nf_P.n;
  if (dt == PH_F32 && m.nf_P32.n == 0 && n > 0) {
    m.nf_P32.alloc((size_t)n);
    hipLaunchKernelGGL(k_round_factors<float>, dim3((unsigned)grid_for(n)), dim3(NT), 0, st, (const double*)m.nf_P.p,
                       m.nf_P32.p, n);
    PH_HIP(hipGetLastError());
    PH_HIP(hipStreamSynchronize(st));
  } else if (dt == PH_BF16 && m.nf_P16.n == 0 && n > 0) {
    m.nf_P16.alloc((size_t)n);
    hipLaunchKernelGGL(k_round_factors<bf16>, dim3((unsigned)grid_for(n)), dim3(NT), 0, st, (const double*)m.nf_P.p,
                       m.nf_P16.p, n);
    PH_HIP(hipGetLastError());
    PH_HIP(hipStreamSynchronize(st));
  }
}

template <typename S>
void near_cores_launch(InstData& in, hipStream_t st) {
  const DeviceModel& m = *in.m;
  const int64_t total = m.n_stored_near * in.T * m.KRp;
  launch(PH_STAGE_NEAR_INST, k_near_cores<S>, dim3((unsigned)grid_for(total)), dim3(NT), st,
         (const NearDev*)m.nstore.p, (const double*)m.nf_core.p, (const double*)m.nf_theta.p, (const double*)in.v.p,
         (S*)in.ccore.p, m.n_stored_near, in.T, m.p_theta, m.d_theta, m.KRp, m.KM);
}
template void near_cores_launch<double>(InstData&, hipStream_t);
template void near_cores_launch<float>(InstData&, hipStream_t);

// Launch shape of the factored near MVM: TCB slots per workgroup, RT row tiles per wave.
// PH_FUSED_SHAPE = "TCB,RT" overrides (tuning), else ph_autotune's choice, else 8 slots
// (fewer for small T) and 1 row tile.
static void fused_shape(const InstData& in, int& tcb, int& rt) {
  tcb = in.tune_fused_tcb > 0 ? in.tune_fused_tcb : 8;
  rt = in.tune_fused_rt > 0 ? in.tune_fused_rt : 1;
  if (const char* e = std::getenv("PH_FUSED_SHAPE")) {
    int a = 0, c = 0;
    if (std::sscanf(e, "%d,%d", &a, &c) == 2 && (a == 1 || a == 2 || a == 4 || a == 8) && (c == 1 || c == 2)) {
      tcb = a;
      rt = c;
    }
  }
  while (tcb > 1 && tcb / 2 >= in.T) tcb /= 2;
}

template <typename S, typename PT>
void near_fused_launch(InstData& in, const S* xt, S* yt, int64_t Rs, hipStream_t st) {
  const DeviceModel& m = *in.m;
  const TreeData& t = *m.tree;
  int tcb, rt;
  fused_shape(in, tcb, rt);
  if ((int64_t)in.T * m.n * Rs * (int64_t)sizeof(S) > BUF_MAX_BYTES)
    fail(PH_EUNSUPPORTED, "ph_matvec: factored near field needs T n R values below 2 GiB (reduce R or T)");
  if (m.KRp * m.max_Nep * (int64_t)sizeof(PT) > BUF_MAX_BYTES)
    fail(PH_EUNSUPPORTED, "ph_matvec: a near factor exceeds 2 GiB (use PH_NEAR_BLOCKS)");
  const int64_t nrc = (Rs + RC - 1) / RC;
  const int64_t nitems = rt == 2 ? m.n_mvm_items : m.n_mvm_items64;
  const int32_t* items = rt == 2 ? (const int32_t*)m.mvm_items.p : (const int32_t*)m.mvm_items64.p;
  const PT* Pf = m.near_factors<PT>();
  const dim3 grid((unsigned)nitems, (unsigned)nrc, (unsigned)((in.T + tcb - 1) / tcb));
  auto go = [&](auto kern) {
    launch(PH_STAGE_NEAR_MVM, kern, grid, dim3(NT), st, xt, yt, Pf, (const S*)in.ccore.p,
           (const NearDev*)m.nstore.p, (const int64_t*)m.nbegin.p, (const int64_t*)m.nend.p,
           (const int64_t*)m.near_rowptr.p, (const int32_t*)m.near_q.p, (const int32_t*)m.near_tr.p,
           (const int64_t*)m.near_tb.p, items, t.leaves.front(), m.n, Rs, in.T, m.KRp / m.KM, m.near_xcd);
  };
  // rank chunk KM: the largest near rank rounded up to 4 when it is at most 16 (one chunk
  // per K-step), else chunks of 16
  const int km = m.KM;
  auto by_km = [&](auto tcbc, auto rtc) {
    constexpr int A = decltype(tcbc)::value, B = decltype(rtc)::value;
    if (km == 4) go(k_near_fused<S, PT, A, B, 4>);
    else if (km == 8) go(k_near_fused<S, PT, A, B, 8>);
    else if (km == 12) go(k_near_fused<S, PT, A, B, 12>);
    else go(k_near_fused<S, PT, A, B, 16>);
  };
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I4 = std::integral_constant<int, 4>;
  using I8 = std::integral_constant<int, 8>;
  if (rt == 2) {
    if (tcb == 8) by_km(I8(), I2());
    else if (tcb == 4) by_km(I4(), I2());
    else if (tcb == 2) by_km(I2(), I2());
    else by_km(I1(), I2());
  } else {
    if (tcb == 8) by_km(I8(), I1());
    else if (tcb == 4) by_km(I4(), I1());
    else if (tcb == 2) by_km(I2(), I1());
    else by_km(I1(), I1());
  }
}
template void near_fused_launch<double, double>(InstData&, const double*, double*, int64_t, hipStream_t);
template void near_fused_launch<float, float>(InstData&, const float*, float*, int64_t, hipStream_t);
template void near_fused_launch<float, bf16>(InstData&, const float*, float*, int64_t, hipStream_t);

template <typename S, typename PT>
void near_block_eval(const InstData& in, int t, int64_t q, double* dev_out, hipStream_t st) {
  const DeviceModel& m = *in.m;
  hipLaunchKernelGGL((k_near_block_eval<S, PT>), dim3(64), dim3(NT), 0, st, (const NearDev*)m.nstore.p,
                     (const PT*)m.near_factors<PT>(), (const S*)in.ccore.p, q, in.T, t, m.KRp, m.KM, dev_out);
  PH_HIP(hipGetLastError());
}
template void near_block_eval<double, double>(const InstData&, int, int64_t, double*, hipStream_t);
template void near_block_eval<float, float>(const InstData&, int, int64_t, double*, hipStream_t);
template void near_block_eval<float, bf16>(const InstData&, int, int64_t, double*, hipStream_t);

}  // namespace ph
