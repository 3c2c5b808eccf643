// Coupling on the BF16 matrix cores (instances of PH_BF16 with 16-column right-hand-side
// tiles): y_hat_s += C_class x_hat_t over the far blocks, with C and x_hat rounded to BF16
// (nearest) as they are staged into LDS and V_MFMA_F32_16X16X16_BF16 products accumulated
// in FP32 (Sec. 4.2: the coupling is the dense contraction of the far field).
#include "ph_device.hpp"

namespace ph {

// One workgroup of 4 wavefronts per (class chunk g, slot, target box, RHS tile), the work
// list and grid of the FP64 / FP32 coupling (boxes of NTG targets of one level, one entry
// per translation class used in the box, chunks of equal estimated work).  A stage is one
// 16-wide K panel of one entry: the Pp x 16 panel of C and, for each of the NTG targets
// that use the class, the 16 x 16 block of x_hat (K rows of the source node, 16 RHS), both
// as BF16 in LDS:
//   As[m][k]      row-major 16 x 16 tiles (a lane's A operand: row m, k = 4 (l / 16) .. + 3)
//   Bs[t][n][k]   per target, transposed (a lane's B operand: column n, the same 4 k)
// Wave w owns row tiles w, w + 4 (Pp / 16 <= 8) for all targets: acc[target][tile].
// Global loads of the next stage run one stage ahead in registers; LDS is double buffered,
// one barrier per stage.  C is read in the FP32 fragment order of the instance (a 16-byte
// unit holds rows m0, m0 + 4, m0 + 8, m0 + 12 of one column k, frag_index).
__global__ void __launch_bounds__(256) k_coupling_bf16(
    const float* __restrict__ xh, float* __restrict__ out, const float* __restrict__ C,
    const int32_t* __restrict__ grp_targets, const int32_t* __restrict__ ent_cls,
    const int32_t* __restrict__ ent_tau, const int32_t* __restrict__ chunk_first, int Pp, int64_t nodes, int64_t Rs, int G, int64_t Cps,
    int64_t part_stride, int n_groups) {
  typedef short s4 __attribute__((ext_vector_type(4)));
  typedef float f4 __attribute__((ext_vector_type(4)));
  __shared__ __attribute__((aligned(16))) uint16_t As[2][8 * 256];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][NTG][256];
  const int g = blockIdx.x;
  const int64_t slot = blockIdx.y;
  const int grp = blockIdx.z % n_groups;
  const int r0 = (blockIdx.z / n_groups) * RC;
  const int lane = threadIdx.x % WAVE;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int nMt = Pp / 16;
  f4 acc[NTG][2];
#pragma unroll
  for (int s = 0; s < NTG; ++s)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[s][j] = f4{0, 0, 0, 0};
  const int ea = chunk_first[grp * (G + 1) + g], eb = chunk_first[grp * (G + 1) + g + 1];
  const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(xh + slot * nodes * Pp * Rs), (short)0, (int)(nodes * Pp * Rs * (int64_t)sizeof(float)), BUF_WORD3);
  const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(C + slot * Cps), (short)0, (int)(Cps * (int64_t)sizeof(float)), BUF_WORD3);
  const int nk = Pp / 16;
  const int nsteps = (eb - ea) * nk;
  // stage loads: C panel = Pp * 16 floats = nMt * 64 16-byte units (<= 512: 2 per thread);
  // x_hat = NTG targets x 16 k x 16 RHS floats = 1024 16-byte units (4 per thread)
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 areg[2], breg[4];
  auto fetch = [&](int step) {
    const int e = ea + step / nk, kc = step % nk;
    const int cbase = (ent_cls[e] * Pp * Pp + kc * Pp * 16) * 4;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int u = threadIdx.x + 256 * q;
      areg[q] = __builtin_amdgcn_raw_buffer_load_b128(crs, u < nMt * 64 ? cbase + u * 16 : BUF_OOB, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = threadIdx.x + 256 * q;        // target u / 64, k (u % 64) / 4, RHS 4 (u % 4) .. + 3
      const int tgt = u >> 6, k = (u & 63) >> 2, rq = u & 3;
      const int tv = ent_tau[e * NTG + tgt];
      const int off = tv >= 0 ? (((tv * Pp + kc * 16 + k) * (int)Rs) + r0 + 4 * rq) * 4 : BUF_OOB;
      breg[q] = __builtin_amdgcn_raw_buffer_load_b128(xrs, off, 0, 0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int u = threadIdx.x + 256 * q;
      if (u < nMt * 64) {
        // unit u of the panel: tile u / 64, column k = (u % 64) / 4, rows m0 + 4 i with
        // m0 = u % 4 (frag_index)
        const int tile = u >> 6, k = (u & 63) >> 2, m0 = u & 3;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // the element is copied out first: a bit cast of a vector element expression
          // reads element 0 with this compiler
          const unsigned int w = areg[q][i];
          As[buf][tile * 256 + (m0 + 4 * i) * 16 + k] = to_bf16(__builtin_bit_cast(float, w)).bits;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = threadIdx.x + 256 * q;
      const int tgt = u >> 6, k = (u & 63) >> 2, rq = u & 3;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const unsigned int w = breg[q][i];
        Bs[buf][tgt][(4 * rq + i) * 16 + k] = to_bf16(__builtin_bit_cast(float, w)).bits;
      }
    }
  };
  const int m16 = lane & 15, kq = lane >> 4;
  auto body = [&](int st, int buf) {
    if (st + 1 < nsteps) fetch(st + 1);
    const int e = ea + st / nk;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int mt = wave + 4 * j;
      if (mt >= nMt) continue;
      const s4 a = *reinterpret_cast<const s4*>(&As[buf][mt * 256 + m16 * 16 + 4 * kq]);
#pragma unroll
      for (int s = 0; s < NTG; ++s) {
        if (ent_tau[e * NTG + s] < 0) continue;   // wave-uniform
        const s4 b = *reinterpret_cast<const s4*>(&Bs[buf][s][m16 * 16 + 4 * kq]);
        acc[s][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[s][j], 0, 0, 0);
      }
    }
    if (st + 1 < nsteps) stash(buf ^ 1);
    __syncthreads();
  };
  if (nsteps > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  for (int st = 0; st < nsteps; st += 2) {
    body(st, 0);
    if (st + 1 < nsteps) body(st + 1, 1);
  }
  // output: element i of lane l at row 4 (l / 16) + i, column (RHS) l % 16
  float* o = out + (int64_t)g * part_stride + slot * nodes * Pp * Rs;
#pragma unroll
  for (int s = 0; s < NTG; ++s) {
    const int32_t node = grp_targets[grp * NTG + s];
    if (node < 0) continue;
    float* on = o + (int64_t)node * Pp * Rs + r0 + m16;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int mt = wave + 4 * j;
      if (mt >= nMt) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) on[(int64_t)(mt * 16 + 4 * kq + i) * Rs] = acc[s][j][i];
    }
  }
}

void coupling_bf16_launch(const InstData& in, const float* xh, float* out, int G, int64_t Rs, int64_t nrc,
                          hipStream_t st) {
  const DeviceModel& m = *in.m;
  const int64_t Cps = m.n_classes * m.Pp * m.Pp;
  const int64_t part_stride = (int64_t)in.T * m.n_nodes * m.Pp * Rs;
  if (m.Pp > 128 || in.T > 65535 || m.n_groups * nrc > 65535)
    fail(PH_EUNSUPPORTED, "ph_matvec: BF16 coupling supports Pp <= 128 and at most 65535 slots / boxes x RHS tiles");
  int c = 0;
  while ((1 << c) < G) ++c;
  launch(PH_STAGE_COUPLING, k_coupling_bf16, dim3((unsigned)G, (unsigned)in.T, (unsigned)(m.n_groups * nrc)), dim3(256),
         st, xh, out, (const float*)in.C.p, (const int32_t*)m.grp_targets.p, (const int32_t*)m.ent_cls.p,
         (const int32_t*)m.ent_tau.p, (const int32_t*)m.chunk_first.p + m.chunk_off[c], m.Pp, m.n_nodes, Rs, G, Cps,
         part_stride, (int)m.n_groups);
}

}  // namespace ph
