// Coupling on the BF16 matrix cores (instances of PH_BF16 with 16-column right-hand-side
// tiles): y_hat_s += C_class x_hat_t over the far blocks (Sec. 4.2: the coupling is the
// dense contraction of the far field), with C and x_hat rounded to BF16 (nearest) and
// V_MFMA_F32_16X16X32_BF16 products accumulated in FP32.
#include "ph_device.hpp"

namespace ph {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Operand order.  Both operands are stored as the 16-byte lane units of the matrix-core
// instruction (lane l: A row l % 16, B column l % 16, eight consecutive k = 8 (l / 16) + j),
// so an operand tile is 1 KB that a wave reads with one 16-byte access per lane:
//   C:     [slot][class][k panel kp][row tile mt][lane l][j]: row 16 mt + l % 16,
//          column 32 kp + 8 (l / 16) + j  (zero past Pp)
//   x_hat: [slot][node][RHS tile rt][k panel kp][lane l][j]: row 32 kp + 8 (l / 16) + j
//          (zero past Pp), right-hand side 16 rt + l % 16
__device__ __forceinline__ unsigned int pack_bf16x2(float lo, float hi) {
  return (unsigned int)to_bf16(lo).bits | ((unsigned int)to_bf16(hi).bits << 16);
}

// C (FP32, fragment order frag_index) -> operand order; one thread per lane unit
__global__ void __launch_bounds__(NT) k_pack_c_bf16(const float* __restrict__ C, u4* __restrict__ Cb, int Pp,
                                                    int nMt, int nkp, int64_t units) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
    const int lane = (int)(u % 64);
    int64_t r = u / 64;
    const int mt = (int)(r % nMt);
    r /= nMt;
    const int kp = (int)(r % nkp);
    r /= nkp;   // slot * n_classes + class
    const float* c = C + r * Pp * Pp;
    const int m = mt * 16 + lane % 16, k0 = kp * 32 + 8 * (lane / 16);
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = k0 + j < Pp ? c[frag_index(m, k0 + j, Pp)] : 0.0f;
    Cb[u] = u4{pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]), pack_bf16x2(v[4], v[5]), pack_bf16x2(v[6], v[7])};
  }
}

// x_hat (FP32, [slot][node][Pp][Rs]) of the nodes >= a0 -> operand order
__global__ void __launch_bounds__(NT) k_pack_xh_bf16(const float* __restrict__ xh, u4* __restrict__ xb, int Pp,
                                                     int nkp, int64_t nodes, int64_t Rs, int nrc, int64_t a0,
                                                     int64_t units) {
  const int64_t span = nodes - a0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
    const int lane = (int)(u % 64);
    int64_t r = u / 64;
    const int kp = (int)(r % nkp);
    r /= nkp;
    const int rt = (int)(r % nrc);
    r /= nrc;
    const int64_t node = a0 + r % span, slot = r / span;
    const float* x = xh + (slot * nodes + node) * Pp * Rs + rt * 16 + lane % 16;
    const int k0 = kp * 32 + 8 * (lane / 16);
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = k0 + j < Pp ? x[(int64_t)(k0 + j) * Rs] : 0.0f;
    xb[(((slot * nodes + node) * nrc + rt) * nkp + kp) * 64 + lane] =
        u4{pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]), pack_bf16x2(v[4], v[5]), pack_bf16x2(v[6], v[7])};
  }
}

// One workgroup of 4 wavefronts per (class chunk g, slot, target box, RHS tile): the work
// list, chunking and grid of the FP64 / FP32 coupling (boxes of NTG targets of one level,
// one entry per translation class used in the box, chunk g of every box on XCD g).  A stage
// is one 32-wide K panel of one entry: the NMT operand tiles of C and, for each of the NTG
// targets, the x_hat tile of the source it pairs with under the class (zeros for targets
// that do not use the class), both copied from global memory to LDS as 16-byte units
// (wave w copies the tiles of targets 4 w .. 4 w + 3).
// Wave w owns row tiles w, w + 4 for every target (acc[target][tile], FP32) and skips the
// targets of the entry's mask.  Global loads run two stages ahead in registers, LDS is
// double buffered, one barrier per stage.
template <int NMT>
__global__ void __launch_bounds__(256, 2) k_coupling_bf16(
    const u4* __restrict__ xb, float* __restrict__ out, const u4* __restrict__ Cb,
    const int32_t* __restrict__ grp_targets, const int32_t* __restrict__ ent_cls,
    const int32_t* __restrict__ ent_tau, const int32_t* __restrict__ ent_mask,
    const int32_t* __restrict__ chunk_first, int Pp, int nkp, int64_t nodes, int64_t Rs, int nrc, int G,
    int64_t cb_slot_bytes, int64_t xb_slot_bytes, int64_t part_stride, int n_groups) {
  constexpr int TPW = (NMT + 3) / 4;           // row tiles per wave
  constexpr int AU = (NMT * 64 + 255) / 256;   // C units per thread and stage
  __shared__ u4 As[2][NMT * 64];
  __shared__ u4 Bs[2][NTG][64];
  const int g = blockIdx.x;
  const int64_t slot = blockIdx.y;
  const int grp = blockIdx.z % n_groups;
  const int rt = blockIdx.z / n_groups;
  const int lane = threadIdx.x % WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  __builtin_assume(wave >= 0 && wave < 4);
  f4 acc[NTG][TPW];
#pragma unroll
  for (int s = 0; s < NTG; ++s)
#pragma unroll
    for (int j = 0; j < TPW; ++j) acc[s][j] = f4{0, 0, 0, 0};
  const int ea = chunk_first[grp * (G + 1) + g], eb = chunk_first[grp * (G + 1) + g + 1];
  // raw buffer views of this slot's operands: an offset past the end reads zeros
  const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((const char*)xb + slot * xb_slot_bytes), (short)0, (int)xb_slot_bytes, BUF_WORD3);
  const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((const char*)Cb + slot * cb_slot_bytes), (short)0, (int)cb_slot_bytes, BUF_WORD3);
  const int nsteps = (eb - ea) * nkp;
  u4 areg[2][AU], breg[2][4];
  // every load is unconditional (clamped stage, out-of-range offsets), so the compiler
  // tracks each register's pending load exactly and waits only at stash
  auto fetch = [&](int step, int rb) {
    const int e = ea + step / nkp, kp = step % nkp;
    const int abase = (ent_cls[e] * nkp + kp) * NMT * 1024;
#pragma unroll
    for (int q = 0; q < AU; ++q) {
      const int u = threadIdx.x + 256 * q;
      areg[rb][q] = __builtin_amdgcn_raw_buffer_load_b128(crs, u < NMT * 64 ? abase + u * 16 : BUF_OOB, 0, 0);
    }
    // wave w stages targets 4 w .. 4 w + 3 (their sources: one 16-byte scalar load)
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 tv = *reinterpret_cast<const i4*>(ent_tau + e * NTG + 4 * wave);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int off = tv[q] >= 0 ? (((tv[q] * nrc + rt) * nkp + kp) * 64 + lane) * 16 : BUF_OOB;
      breg[rb][q] = __builtin_amdgcn_raw_buffer_load_b128(xrs, off, 0, 0);
    }
  };
  auto stash = [&](int rb, int buf) {
#pragma unroll
    for (int q = 0; q < AU; ++q) {
      const int u = threadIdx.x + 256 * q;
      if (u < NMT * 64) As[buf][u] = areg[rb][q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[buf][4 * wave + q][lane] = breg[rb][q];
  };
  // stage st from LDS buffer BUF: store stage st + 1 (register slot RS) into the other
  // buffer first (its loads were issued a stage earlier), then issue the loads of stage
  // st + 2 into register slot RF, then the matrix-core work
  auto body = [&](int st, auto BUF, auto RF, auto RS) {
    constexpr int buf = decltype(BUF)::value;
    const int mask = ent_mask[ea + st / nkp];
    stash(decltype(RS)::value, buf ^ 1);
    fetch(min(st + 2, nsteps - 1), decltype(RF)::value);
    u4 a[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j)
      if (wave + 4 * j < NMT) a[j] = As[buf][(wave + 4 * j) * 64 + lane];
    // the B tiles of the targets in the entry's mask (wave-uniform) are all read before the
    // first product, so their LDS latencies overlap
    u4 b[NTG];
#pragma unroll
    for (int s = 0; s < NTG; ++s)
      if ((mask >> s) & 1) b[s] = Bs[buf][s][lane];
#pragma unroll
    for (int s = 0; s < NTG; ++s) {
      if (!((mask >> s) & 1)) continue;
#pragma unroll
      for (int j = 0; j < TPW; ++j)
        if (wave + 4 * j < NMT)
          acc[s][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a[j]), __builtin_bit_cast(b8, b[s]),
                                                              acc[s][j], 0, 0, 0);
    }
    __syncthreads();
  };
  typedef std::integral_constant<int, 0> I0;
  typedef std::integral_constant<int, 1> I1;
  if (nsteps > 0) {
    fetch(0, 0);
    stash(0, 0);
    fetch(min(1, nsteps - 1), 1);
  }
  __syncthreads();
  // stages in pairs, so that LDS buffers and register slots are compile-time
#pragma unroll 1
  for (int st = 0; st < nsteps; st += 2) {
    body(st, I0(), I0(), I1());
    if (st + 1 < nsteps) body(st + 1, I1(), I1(), I0());
  }
  // element i of lane l: row 4 (l / 16) + i of the tile, right-hand side l % 16
  float* o = out + (int64_t)g * part_stride + slot * nodes * Pp * Rs;
#pragma unroll
  for (int s = 0; s < NTG; ++s) {
    const int32_t node = grp_targets[grp * NTG + s];
    if (node < 0) continue;
    float* on = o + (int64_t)node * Pp * Rs + rt * RC + lane % 16;
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      const int mt = wave + 4 * j;
      if (mt >= NMT) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) on[(int64_t)(mt * 16 + 4 * (lane / 16) + i) * Rs] = acc[s][j][i];
    }
  }
}

int64_t coupling_bf16_c_bytes(const DeviceModel& m) {
  const int nkp = (m.Pp + 31) / 32, nMt = m.Pp / 16;
  return m.n_classes * nkp * nMt * 1024;
}

int64_t coupling_bf16_x_bytes(const DeviceModel& m, int64_t Rs) {
  const int nkp = (m.Pp + 31) / 32;
  return m.n_nodes * ((Rs + RC - 1) / RC) * nkp * 1024;
}

bool coupling_bf16_supported(const DeviceModel& m, int64_t Rs) {
  return m.Pp <= 128 && Rs >= RC && coupling_bf16_c_bytes(m) <= BUF_MAX_BYTES &&
         coupling_bf16_x_bytes(m, Rs) <= BUF_MAX_BYTES;
}

void coupling_bf16_pack_c(const InstData& in, hipStream_t st) {
  const DeviceModel& m = *in.m;
  const int nkp = (m.Pp + 31) / 32, nMt = m.Pp / 16;
  const int64_t units = (int64_t)in.T * m.n_classes * nkp * nMt * 64;
  if (units == 0) return;
  launch(PH_STAGE_FAR_INST, k_pack_c_bf16, dim3((unsigned)grid_for(units)), dim3(NT), st, (const float*)in.C.p,
         (u4*)in.Cb.p, m.Pp, nMt, nkp, units);
}

void coupling_bf16_launch(const InstData& in, const float* xh, void* xb, float* out, int G, int64_t Rs, int64_t nrc,
                          int64_t a0, hipStream_t st) {
  const DeviceModel& m = *in.m;
  const int nkp = (m.Pp + 31) / 32, nMt = m.Pp / 16;
  if (nMt < 1 || nMt > 8 || in.T > 65535 || m.n_groups * nrc > 65535)
    fail(PH_EUNSUPPORTED, "ph_matvec: BF16 coupling supports Pp <= 128 and at most 65535 slots / boxes x RHS tiles");
  const int64_t xunits = (int64_t)in.T * (m.n_nodes - a0) * nrc * nkp * 64;
  if (xunits > 0)
    launch(PH_STAGE_COUPLING, k_pack_xh_bf16, dim3((unsigned)grid_for(xunits)), dim3(NT), st, xh, (u4*)xb, m.Pp, nkp,
           m.n_nodes, Rs, (int)nrc, a0, xunits);
  int c = 0;
  while ((1 << c) < G) ++c;
  const int64_t part_stride = (int64_t)in.T * m.n_nodes * m.Pp * Rs;
  auto run = [&](auto kern) {
    launch(PH_STAGE_COUPLING, kern, dim3((unsigned)G, (unsigned)in.T, (unsigned)(m.n_groups * nrc)), dim3(256), st,
           (const u4*)xb, out, (const u4*)in.Cb.p, (const int32_t*)m.grp_targets.p, (const int32_t*)m.ent_cls.p,
           (const int32_t*)m.ent_tau.p, (const int32_t*)m.ent_mask.p, (const int32_t*)m.chunk_first.p + m.chunk_off[c],
           m.Pp, nkp, m.n_nodes, Rs, (int)nrc, G, coupling_bf16_c_bytes(m), coupling_bf16_x_bytes(m, Rs), part_stride,
           (int)m.n_groups);
  };
  switch (nMt) {
    case 1: run(k_coupling_bf16<1>); break;
    case 2: run(k_coupling_bf16<2>); break;
    case 3: run(k_coupling_bf16<3>); break;
    case 4: run(k_coupling_bf16<4>); break;
    case 5: run(k_coupling_bf16<5>); break;
    case 6: run(k_coupling_bf16<6>); break;
    case 7: run(k_coupling_bf16<7>); break;
    default: run(k_coupling_bf16<8>); break;
  }
}

}  // namespace ph
