// Model upload, tracing state and the C ABI of the parametric H^2 library (arxiv
// 2511.03109) on MI355X.  The online-stage kernels live in k_instantiate.hip and the
// MVM kernels in k_matvec.hip.
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>

#include "ph_device.hpp"

namespace ph {

static thread_local std::string g_last_error;

std::mutex g_trace_mu;
bool g_trace_on = false;
thread_local bool g_capturing = false;
std::vector<TraceRec> g_trace_recs;
static std::vector<hipEvent_t> g_event_pool;

hipEvent_t pooled_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  PH_HIP(hipEventCreate(&e));
  return e;
}

// ------------------------------------------------------------------ model upload
// The far field of the parametric H-matrix format: per far block its factors and offsets, per
// stored class its core, and per leaf the far blocks whose target cluster contains the leaf.
static void upload_hmatrix(DeviceModel& m, const TreeData& t, const HostModel& hm, hipStream_t st) {
  m.format = PH_FORMAT_H;
  std::vector<HClsDev> hc(hm.cstore.size());
  int64_t hoff = 0;
  for (size_t q = 0; q < hm.cstore.size(); ++q) {
    const ClassStored& c = hm.cstore[q];
    hc[q] = HClsDev{c.core_off, c.th1_off, c.th2_off, hoff, c.rL, c.r1, c.r2, c.rR};
    hoff += (int64_t)c.rL * c.rR;
  }
  m.h_tot = hoff;
  std::vector<HBlkDev> hb(hm.hblk.size());
  int64_t woff = 0;
  std::vector<std::vector<int32_t>> by_target(t.n_nodes());
  for (size_t b = 0; b < hm.hblk.size(); ++b) {
    const HBlock& h = hm.hblk[b];
    hb[b] = HBlkDev{h.s_begin, h.t_begin, h.S_off, h.T_off, hc[h.q].h_off, woff,
                    (int32_t)h.ns, (int32_t)h.nt, h.rs, h.rt, h.lds, h.ldt, h.tr, h.q};
    woff += (int64_t)h.rs * 16;
    m.h_tbytes_max = std::max(m.h_tbytes_max, (int64_t)h.ldt * h.rt * (int64_t)sizeof(double));
    by_target[h.s].push_back((int32_t)b);
  }
  m.hw_tot = woff;
  std::vector<int32_t> lptr{0}, lblk;
  for (int32_t leaf : t.leaves) {
    for (int32_t s = leaf; s >= 0; s = t.parent[s])
      lblk.insert(lblk.end(), by_target[s].begin(), by_target[s].end());
    lptr.push_back((int32_t)lblk.size());
  }
  m.n_hblk = (int64_t)hb.size();
  m.n_hcls = (int64_t)hc.size();
  m.hblk.upload(hb.data(), hb.size(), st);
  m.hcls.upload(hc.data(), hc.size(), st);
  m.hcore.upload(hm.ff_core.data(), hm.ff_core.size(), st);
  m.hS.upload(hm.hS.data(), hm.hS.size(), st);
  m.hT.upload(hm.hT.data(), hm.hT.size(), st);
  m.hl_ptr.upload(lptr.data(), lptr.size(), st);
  m.hl_blk.upload(lblk.data(), lblk.size(), st);
  PH_HIP(hipStreamSynchronize(st));   // host staging buffers die with this call
  m.device_bytes += (int64_t)(m.hblk.bytes() + m.hcls.bytes() + m.hcore.bytes() + m.hS.bytes() + m.hT.bytes() +
                              m.hl_ptr.bytes() + m.hl_blk.bytes());
}

// The implicit coupling (Alg. "Modified H^2-Matrix MVM"): the H-matrix kernels' structures over
// the index space of the coupling (row s Pp + i is entry i of x_hat_s / y_hat_s).  Far block
// (s, t) of class c with stored class q: S_b = L_q, T_b = R_q, or (R_q, L_q) with H_q^T when c is
// the mirror of q; per stored class its core; per node of the far levels its row range, work
// item and far blocks.
static void upload_implicit(DeviceModel& m, const TreeData& t, const HostModel& hm, hipStream_t st) {
  m.format = PH_FORMAT_H2_IMPLICIT;
  const int P = hm.P;
  const int64_t Pp = m.Pp;
  std::vector<HClsDev> hc(hm.cstore.size());
  int64_t hoff = 0;
  for (size_t q = 0; q < hm.cstore.size(); ++q) {
    const ClassStored& c = hm.cstore[q];
    hc[q] = HClsDev{c.core_off, c.th1_off, c.th2_off, hoff, c.rL, c.r1, c.r2, c.rR};
    hoff += (int64_t)c.rL * c.rR;
  }
  m.h_tot = hoff;
  const int64_t Roff = (int64_t)hm.ff_L.size();   // R factors follow the L factors in hS
  std::vector<HBlkDev> hb;
  int64_t woff = 0;
  std::vector<std::vector<int32_t>> by_target(t.n_nodes());
  for (int64_t b = 0; b < t.n_far(); ++b) {
    const int32_t s = t.far[2 * b], u = t.far[2 * b + 1], c = t.far_class[b];
    const int32_t q = hm.class_src[c], tr = hm.class_tr[c];
    const ClassStored& cs = hm.cstore[q];
    const int64_t Lo = cs.L_off, Ro = Roff + cs.R_off;
    HBlkDev h{};
    h.s_begin = (int64_t)s * Pp;
    h.t_begin = (int64_t)u * Pp;
    h.S_off = tr ? Ro : Lo;
    h.T_off = tr ? Lo : Ro;
    h.h_off = hc[q].h_off;
    h.w_off = woff;
    h.ns = P;
    h.nt = P;
    h.rs = tr ? cs.rR : cs.rL;
    h.rt = tr ? cs.rL : cs.rR;
    h.lds = P;
    h.ldt = P;
    h.tr = tr;
    h.q = q;
    woff += (int64_t)h.rs * 16;
    m.h_tbytes_max = std::max(m.h_tbytes_max, (int64_t)h.ldt * h.rt * (int64_t)sizeof(double));
    by_target[s].push_back((int32_t)hb.size());
    hb.push_back(h);
  }
  m.hw_tot = woff;
  const int32_t a0 = t.level_start[t.min_far_level];
  std::vector<int32_t> lptr{0}, lblk, items;
  std::vector<int64_t> nb((size_t)t.n_nodes()), ne((size_t)t.n_nodes());
  for (int32_t s = 0; s < (int32_t)t.n_nodes(); ++s) {
    lblk.insert(lblk.end(), by_target[s].begin(), by_target[s].end());
    lptr.push_back((int32_t)lblk.size());
    nb[s] = (int64_t)s * Pp;
    ne[s] = (int64_t)s * Pp + P;
    if (s >= a0) {
      items.push_back(s);
      items.push_back(0);
    }
  }
  std::vector<double> LR(hm.ff_L);
  LR.insert(LR.end(), hm.ff_R.begin(), hm.ff_R.end());
  m.n_hblk = (int64_t)hb.size();
  m.n_hcls = (int64_t)hc.size();
  m.n_hx_items = (int64_t)items.size() / 2;
  m.hblk.upload(hb.data(), hb.size(), st);
  m.hcls.upload(hc.data(), hc.size(), st);
  m.hcore.upload(hm.ff_core.data(), hm.ff_core.size(), st);
  m.hS.upload(LR.data(), LR.size(), st);
  m.hl_ptr.upload(lptr.data(), lptr.size(), st);
  m.hl_blk.upload(lblk.data(), lblk.size(), st);
  m.hx_nbegin.upload(nb.data(), nb.size(), st);
  m.hx_nend.upload(ne.data(), ne.size(), st);
  m.hx_items.upload(items.data(), items.size(), st);
  PH_HIP(hipStreamSynchronize(st));   // host staging buffers die with this call
  m.device_bytes += (int64_t)(m.hblk.bytes() + m.hcls.bytes() + m.hcore.bytes() + m.hS.bytes() + m.hl_ptr.bytes() +
                              m.hl_blk.bytes() + m.hx_nbegin.bytes() + m.hx_nend.bytes() + m.hx_items.bytes());
}

static std::shared_ptr<DeviceModel> upload_model(std::shared_ptr<const TreeData> tp, HostModel& hm,
                                                 hipStream_t st) {
  const TreeData& t = *tp;
  auto m = std::make_shared<DeviceModel>();
  m->tree = tp;
  m->d = hm.d; m->p_s = hm.p_s; m->P = hm.P; m->p_theta = hm.p_theta; m->d_theta = hm.d_theta;
  m->Pp = (hm.P + 15) / 16 * 16;
  m->l_max = t.l_max; m->min_far = t.min_far_level;
  for (int k = 0; k < 2; ++k) { m->th_lo[k] = hm.th_lo[k]; m->th_hi[k] = hm.th_hi[k]; }
  m->n = t.n; m->n_nodes = t.n_nodes(); m->n_leaves = (int64_t)t.leaves.size();
  m->n_near = t.n_near(); m->n_classes = t.n_classes(); m->N_nf = t.near_entries;
  m->n_stored_near = (int64_t)hm.nstore.size();
  m->n_stored_cls = (int64_t)hm.cstore.size();
  m->kernel_evals = hm.kernel_evals;
  m->near_factor_entries = hm.near_factor_entries;
  m->svd_sweeps_max = hm.svd_sweeps_max;

  // stored near blocks (s <= t): offsets of the instantiated blocks (rows padded to 16)
  std::vector<int64_t> doff(hm.nstore.size() + 1, 0);
  for (size_t q = 0; q < hm.nstore.size(); ++q)
    doff[q + 1] = doff[q] + (int64_t)(hm.nstore[q].ns + 15) / 16 * 16 * hm.nstore[q].nt;
  m->N_nf_pad = doff.back();
  m->D_off_host.assign(m->n_near, 0);
  m->D_tr_host.assign(m->n_near, 0);
  m->near_src_host.assign(m->n_near, 0);
  for (int64_t b = 0; b < m->n_near; ++b) {
    m->D_off_host[b] = doff[hm.near_src[b]];
    m->D_tr_host[b] = hm.near_tr[b];
    m->near_src_host[b] = hm.near_src[b];
  }

  // near stored blocks and tiles
  std::vector<NearDev> nd(hm.nstore.size());
  std::vector<int32_t> tiles;
  m->near_rank_canon.assign(m->n_near, -1);
  double wsum = 0, rsum = 0;
  for (size_t q = 0; q < hm.nstore.size(); ++q) {
    const NearStored& s = hm.nstore[q];
    NearDev& x = nd[q];
    x.s_begin = s.s_begin; x.t_begin = s.t_begin;
    x.P_off = s.P_off; x.core_off = s.core_off; x.th1_off = s.th1_off; x.th2_off = s.th2_off;
    x.D_st = doff[q];
    x.ns = s.ns; x.nt = s.nt; x.r_e = s.r_e; x.r1 = s.r1; x.r2 = s.r2;
    x.ldp = s.ldp;
    m->near_rank_canon[s.b_st] = s.r_e;
    const double w = (double)s.ns * s.nt * (s.b_ts >= 0 ? 2 : 1);
    wsum += w;
    rsum += w * s.r_e;
    m->near_rank_max = std::max(m->near_rank_max, s.r_e);
    for (int32_t j0 = 0; j0 < s.nt; j0 += TILE_J)
      for (int32_t i0 = 0; i0 < (s.ns + 15) / 16 * 16; i0 += TILE) {   // padding rows are written (0)
        tiles.push_back((int32_t)q);
        tiles.push_back(i0);
        tiles.push_back(j0);
      }
  }
  m->near_rank_mean = wsum > 0 ? rsum / wsum : 0;
  m->n_tiles = (int64_t)tiles.size() / 3;

  // far classes: panels Chat_q permuted into fragment order (zero padding to Pp)
  const int P = hm.P;
  const int64_t Pp = m->Pp;
  std::vector<ClassDev> cd(hm.cstore.size());
  double fr = 0;
  int64_t chat_tot = 0;
  for (const ClassStored& c : hm.cstore) chat_tot += (int64_t)c.r1 * c.r2 * Pp * Pp;
  std::vector<double> chat((size_t)chat_tot, 0.0);
  m->class_ranks.assign(m->n_classes * (2 + hm.d_theta), 0);
  int64_t coff = 0;
  for (size_t q = 0; q < hm.cstore.size(); ++q) {
    const ClassStored& c = hm.cstore[q];
    ClassDev& x = cd[q];
    x.th1_off = c.th1_off; x.th2_off = c.th2_off;
    x.C_off = (int64_t)c.cls * Pp * Pp;
    x.Cm_off = c.mirror >= 0 ? (int64_t)c.mirror * Pp * Pp : -1;
    x.chat_off = coff;
    for (int64_t r = 0; r < (int64_t)c.r1 * c.r2; ++r)
      for (int j = 0; j < P; ++j)
        for (int i = 0; i < P; ++i)
          chat[(size_t)(coff + r * Pp * Pp + frag_index(i, j, (int)Pp))] =
              hm.ff_chat[(size_t)(c.chat_off + r * P * P + i + (int64_t)P * j)];
    coff += (int64_t)c.r1 * c.r2 * Pp * Pp;
    x.rL = c.rL; x.r1 = c.r1; x.r2 = c.r2; x.rR = c.rR;
    fr += 0.5 * (c.rL + c.rR);
    m->far_rank_max = std::max({m->far_rank_max, c.rL, c.rR});
    int32_t* cr = &m->class_ranks[(size_t)c.cls * (2 + hm.d_theta)];
    cr[0] = c.rL; cr[1] = c.r1; if (hm.d_theta == 2) cr[2] = c.r2; cr[1 + hm.d_theta] = c.rR;
    if (c.mirror >= 0) {
      int32_t* mr = &m->class_ranks[(size_t)c.mirror * (2 + hm.d_theta)];
      mr[0] = c.rR; mr[1] = c.r1; if (hm.d_theta == 2) mr[2] = c.r2; mr[1 + hm.d_theta] = c.rL;
    }
  }
  m->far_rank_mean = cd.empty() ? 0 : fr / cd.size();

  // CSR of near blocks by target leaf (canonical list is sorted by sigma)
  const int32_t leaf0 = t.leaves.empty() ? 0 : t.leaves.front();
  std::vector<int64_t> nrow(m->n_leaves + 1, 0), ntb(m->n_near), nD(m->n_near);
  std::vector<int32_t> nnt(m->n_near), ntr(m->n_near), nq(m->n_near);
  for (int64_t b = 0; b < m->n_near; ++b) {
    const int32_t s = t.near[2 * b], u = t.near[2 * b + 1];
    nrow[s - leaf0 + 1]++;
    ntb[b] = t.begin[u];
    nnt[b] = (int32_t)t.size(u);
    nD[b] = m->D_off_host[b];
    ntr[b] = m->D_tr_host[b];
    nq[b] = hm.near_src[b];
  }
  // factored near MVM: ranks in chunks of KRp (<= 16, a multiple of 4) or of 16
  int rmax = 1;
  for (const NearStored& q : hm.nstore) {
    rmax = std::max(rmax, q.r_e);
    m->max_Nep = std::max(m->max_Nep, (int64_t)q.ldp * q.nt);
  }
  m->KRp = rmax <= 16 ? (rmax + 3) / 4 * 4 : (rmax + 15) / 16 * 16;
  m->KM = rmax <= 16 ? m->KRp : 16;
  for (int64_t i = 0; i < m->n_leaves; ++i) nrow[i + 1] += nrow[i];
  // near MVM work items, one per 128-row chunk of every leaf (leaf order)
  std::vector<int32_t> items;
  for (int64_t li = 0; li < m->n_leaves; ++li) {
    const int64_t ns = t.size(t.leaves[(size_t)li]);
    for (int64_t c0 = 0; c0 < std::max<int64_t>(ns, 1); c0 += 128) {
      items.push_back((int32_t)li);
      items.push_back((int32_t)c0);
    }
  }
  m->n_mvm_items = (int64_t)items.size() / 2;
  m->mvm_items.upload(items.data(), items.size(), st);
  std::vector<int32_t> items64;
  for (int64_t li = 0; li < m->n_leaves; ++li) {
    const int64_t ns = t.size(t.leaves[(size_t)li]);
    for (int64_t c0 = 0; c0 < std::max<int64_t>(ns, 1); c0 += 64) {
      items64.push_back((int32_t)li);
      items64.push_back((int32_t)c0);
    }
  }
  m->n_mvm_items64 = (int64_t)items64.size() / 2;
  m->mvm_items64.upload(items64.data(), items64.size(), st);
  // XCD-contiguous leaf ranges in the near MVM only when the 8 ranges carry about equal
  // work (entries of the leaf's near blocks): within 5% of the mean
  {
    std::vector<double> rw(8, 0.0);
    const int64_t q8 = m->n_leaves / 8;
    for (int64_t b = 0; b < m->n_near && q8 > 0; ++b) {
      const int64_t li = t.near[2 * b] - leaf0;
      if (li < 8 * q8) rw[li / q8] += (double)t.size(t.near[2 * b]) * t.size(t.near[2 * b + 1]);
    }
    double mx = 0, sum = 0;
    for (double v : rw) {
      mx = std::max(mx, v);
      sum += v;
    }
    m->near_xcd = q8 > 0 && sum > 0 && mx <= 1.05 * sum / 8 ? 1 : 0;
  }
  // single-RHS near MVM: the smallest row chunk (4, 8 or 12 panels) that holds 90% of the
  // leaves in one pass
  {
    std::vector<int64_t> sz;
    for (int32_t v : t.leaves) sz.push_back(t.size(v));
    std::sort(sz.begin(), sz.end());
    const int64_t p90 = sz.empty() ? 0 : sz[(size_t)(0.9 * (double)(sz.size() - 1))];
    m->gemv_mp = p90 <= 64 ? 4 : (p90 <= 128 ? 8 : 12);
  }
  // Each stored block is read twice by the near MVM: directly by the workgroup of one of
  // its leaves and transposed by that of the other.  Ordering every leaf's list by an edge
  // colouring of the near graph (one block per colour and leaf, both leaves of a block at
  // the same colour) puts the two reads at the same list position, so the second one
  // finds the block still in the memory-side cache.  Colour of the pair (s, u): its leaf
  // offset o = coords(u) - coords(s) up to sign (o' with a positive first non-zero
  // component a), and the parity of floor(c_a / o'_a) at the lower end c; the two blocks
  // of a leaf with offsets o' and -o' differ in that parity.  The diagonal block is first.
  {
    const int d = t.d;
    auto canon = [&](int32_t s, int32_t u, std::vector<int32_t>& o) {
      o.resize(d);
      int sg = 0;
      for (int k = 0; k < d; ++k) {
        o[k] = t.coords[(size_t)u * d + k] - t.coords[(size_t)s * d + k];
        if (sg == 0 && o[k] != 0) sg = o[k] > 0 ? 1 : -1;
      }
      if (sg < 0)
        for (int k = 0; k < d; ++k) o[k] = -o[k];
      return sg;   // 0 on the diagonal, +1 when s is the lower end, -1 when u is
    };
    std::map<std::vector<int32_t>, int32_t> rank;
    std::vector<int32_t> o;
    for (int64_t b = 0; b < m->n_near; ++b)
      if (canon(t.near[2 * b], t.near[2 * b + 1], o) != 0) rank.emplace(o, 0);
    int32_t r = 0;
    for (auto& kv : rank) kv.second = r++;
    std::vector<int64_t> color(m->n_near), order(m->n_near);
    for (int64_t b = 0; b < m->n_near; ++b) {
      const int32_t s = t.near[2 * b], u = t.near[2 * b + 1];
      const int sg = canon(s, u, o);
      if (sg == 0) {
        color[b] = 0;
        continue;
      }
      int a = 0;
      while (o[a] == 0) ++a;
      const int32_t lower = sg > 0 ? s : u;
      const int32_t c = t.coords[(size_t)lower * d + a];
      const int32_t par = (c / o[a]) & 1;   // leaf coordinates are non-negative
      color[b] = 1 + 2 * (int64_t)rank[o] + par;
    }
    for (int64_t b = 0; b < m->n_near; ++b) order[b] = b;
    for (int64_t i = 0; i < m->n_leaves; ++i)
      std::stable_sort(order.begin() + nrow[i], order.begin() + nrow[i + 1],
                       [&](int64_t x, int64_t y) { return color[x] < color[y]; });
    auto permute = [&](auto& v) {
      auto w = v;
      for (int64_t b = 0; b < m->n_near; ++b) v[b] = w[order[b]];
    };
    permute(ntb);
    permute(nD);
    permute(nnt);
    permute(ntr);
    permute(nq);
  }
  // Single-RHS near MVM lists.  The workgroup of leaf s streams its stored blocks D_st
  // (t >= s, canonical order) and writes z_st = D_st^T x_s (t > s) into rows
  // [zoff, zoff + n_t) of the pair buffer; leaf t then adds the z of its blocks with s < t.
  // (The host arrays live until the end of the upload: the copies are asynchronous.)
  std::vector<int64_t> urow(m->n_leaves + 1, 0), lrow(m->n_leaves + 1, 0), utb, uD, uz, lz;
  std::vector<int32_t> unt;
  {
    std::vector<int64_t> zoff(hm.nstore.size(), -1);
    int64_t zt = 0;
    for (size_t q = 0; q < hm.nstore.size(); ++q)
      if (hm.nstore[q].s != hm.nstore[q].t) {
        zoff[q] = zt;
        zt += hm.nstore[q].nt;
      }
    m->Zt = zt;
    for (int64_t b = 0; b < m->n_near; ++b) {
      const int32_t s = t.near[2 * b], u = t.near[2 * b + 1];
      const int32_t q = hm.near_src[b];
      if (s <= u) {
        urow[s - leaf0 + 1]++;
        utb.push_back(t.begin[u]);
        unt.push_back((int32_t)t.size(u));
        uD.push_back(m->D_off_host[b]);
        uz.push_back(zoff[q]);
      } else {
        lrow[s - leaf0 + 1]++;
        lz.push_back(zoff[q]);
      }
    }
    for (int64_t i = 0; i < m->n_leaves; ++i) {
      urow[i + 1] += urow[i];
      lrow[i + 1] += lrow[i];
    }
    m->up_rowptr.upload(urow.data(), urow.size(), st);
    m->up_tb.upload(utb.data(), utb.size(), st);
    m->up_nt.upload(unt.data(), unt.size(), st);
    m->up_D.upload(uD.data(), uD.size(), st);
    m->up_z.upload(uz.data(), uz.size(), st);
    m->lo_rowptr.upload(lrow.data(), lrow.size(), st);
    m->lo_z.upload(lz.data(), lz.size(), st);
  }
  // Coupling work list.  The nodes of every level >= min_far are cut into boxes of NTG = 16
  // nodes (4 x 2 x 2 in 3-D, 4 x 4 in 2-D, 16 in 1-D, axis 1 longest); neighbouring
  // targets share most translation classes, so one coupling matrix fetched for a box
  // serves several targets.  For each box, one entry per class used by any of its nodes,
  // holding the source node of every target that uses it (-1 otherwise), classes ascending.
  std::vector<int32_t> gt, gptr{0}, ecls, etau, ewpre, gw;
  std::vector<int32_t> hgt, hgptr{0}, hecls, hetau, hewpre, hgw;   // half boxes
  struct Box {
    std::vector<int32_t> targets, cls, tau, w;
    int64_t wsum = 0;
  };
  std::vector<Box> boxes_all;
  if (t.min_far_level >= 0) {
    static const int box_bits[4][3] = {{0, 0, 0}, {4, 0, 0}, {2, 2, 0}, {2, 1, 1}};
    const int* bits = box_bits[t.d];
    std::vector<std::vector<std::pair<int32_t, int32_t>>> far_of(t.n_nodes());  // node -> (tau, class)
    for (int64_t b = 0; b < t.n_far(); ++b) far_of[t.far[2 * b]].push_back({t.far[2 * b + 1], t.far_class[b]});
    for (int l = t.min_far_level; l <= t.l_max; ++l) {
      std::map<std::vector<int32_t>, std::vector<int32_t>> boxes;   // box coordinates -> NTG slots
      for (int32_t v = t.level_start[l]; v < t.level_start[l + 1]; ++v) {
        std::vector<int32_t> key(t.d);
        int slot = 0, shift = 0;
        for (int k = 0; k < t.d; ++k) {
          const int32_t c = t.coords[(size_t)v * t.d + k];
          key[k] = c >> bits[k];
          slot |= (c & ((1 << bits[k]) - 1)) << shift;
          shift += bits[k];
        }
        auto& slots = boxes[key];
        if (slots.empty()) slots.assign(NTG, -1);
        slots[slot] = v;
      }
      for (auto& bx : boxes) {
        std::map<int32_t, std::vector<int32_t>> bycls;
        for (int sl = 0; sl < NTG; ++sl) {
          const int32_t v = bx.second[sl];
          if (v < 0) continue;
          for (auto& pr : far_of[v]) {
            auto& e = bycls[pr.second];
            if (e.empty()) e.assign(NTG, -1);
            e[sl] = pr.first;
          }
        }
        Box b;
        b.targets = bx.second;
        for (auto& kv : bycls) {
          int act = 0;
          for (int32_t v : kv.second) act += v >= 0;
          b.cls.push_back(kv.first);
          b.tau.insert(b.tau.end(), kv.second.begin(), kv.second.end());
          b.w.push_back(coupling_entry_weight(act));
          b.wsum += b.w.back();
        }
        boxes_all.push_back(std::move(b));
      }
    }
    // heaviest boxes first: workgroups are dispatched in grid order, so the short ones
    // fill the end of the launch
    std::stable_sort(boxes_all.begin(), boxes_all.end(),
                     [](const Box& a, const Box& b) { return a.wsum > b.wsum; });
    for (const Box& b : boxes_all) {
      gt.insert(gt.end(), b.targets.begin(), b.targets.end());
      int32_t pre = 0;
      for (size_t e = 0; e < b.cls.size(); ++e) {
        ecls.push_back(b.cls[e]);
        ewpre.push_back(pre);
        pre += b.w[e];
      }
      etau.insert(etau.end(), b.tau.begin(), b.tau.end());
      gptr.push_back((int32_t)ecls.size());
      gw.push_back(pre);
      m->max_group_entries = std::max<int64_t>(m->max_group_entries, (int64_t)b.cls.size());
    }
    // Half boxes (the 8-target workgroups of Pp = 128): each half keeps only the entries
    // with at least one active target in it (18% of half-entries have none on the 3-D
    // benchmark: their stages would be pure overhead).  Halves of a box stay adjacent, so
    // the half is the parity of the group index.
    for (const Box& b : boxes_all)
      for (int h = 0; h < 2; ++h) {
        hgt.insert(hgt.end(), b.targets.begin(), b.targets.end());
        int32_t pre = 0;
        for (size_t e = 0; e < b.cls.size(); ++e) {
          int act = 0;
          for (int sl = h * (NTG / 2); sl < (h + 1) * (NTG / 2); ++sl) act += b.tau[e * NTG + sl] >= 0;
          if (act == 0) continue;
          hecls.push_back(b.cls[e]);
          hewpre.push_back(pre);
          pre += coupling_entry_weight(act);
          hetau.insert(hetau.end(), b.tau.begin() + e * NTG, b.tau.begin() + (e + 1) * NTG);
        }
        hgptr.push_back((int32_t)hecls.size());
        hgw.push_back(pre);
      }
  }
  m->n_groups = (int64_t)gptr.size() - 1;
  m->n_entries = (int64_t)ecls.size();
  m->n_hgroups = (int64_t)hgptr.size() - 1;

  m->U.upload(hm.U.data(), hm.U.size(), st);
  m->E.upload(hm.E.data(), hm.E.size(), st);
  m->perm.upload(t.perm.data(), t.perm.size(), st);
  std::vector<int64_t> ip(t.perm.size());
  for (size_t i = 0; i < t.perm.size(); ++i) ip[(size_t)t.perm[i]] = (int64_t)i;
  m->iperm.upload(ip.data(), ip.size(), st);
  m->first_child.upload(t.first_child.data(), t.first_child.size(), st);
  m->nchild.upload(t.nchild.data(), t.nchild.size(), st);
  m->cid.upload(t.cid.data(), t.cid.size(), st);
  m->parent.upload(t.parent.data(), t.parent.size(), st);
  m->nbegin.upload(t.begin.data(), t.begin.size(), st);
  m->nend.upload(t.end.data(), t.end.size(), st);
  m->nstore.upload(nd.data(), nd.size(), st);
  m->nf_P.upload(hm.nf_P.data(), hm.nf_P.size(), st);
  m->nf_core.upload(hm.nf_core.data(), hm.nf_core.size(), st);
  m->nf_theta.upload(hm.nf_theta.data(), hm.nf_theta.size(), st);
  m->tiles.upload(tiles.data(), tiles.size(), st);
  m->near_rowptr.upload(nrow.data(), nrow.size(), st);
  m->near_tb.upload(ntb.data(), ntb.size(), st);
  m->near_D.upload(nD.data(), nD.size(), st);
  m->near_nt.upload(nnt.data(), nnt.size(), st);
  m->near_tr.upload(ntr.data(), ntr.size(), st);
  m->near_q.upload(nq.data(), nq.size(), st);
  m->cstore.upload(cd.data(), cd.size(), st);
  if (!hm.implicit) m->ff_chat.upload(chat.data(), chat.size(), st);   // implicit: no formed couplings
  m->ff_theta.upload(hm.ff_theta.data(), hm.ff_theta.size(), st);
  m->grp_targets.upload(gt.data(), gt.size(), st);
  m->grp_entry.upload(gptr.data(), gptr.size(), st);
  m->ent_cls.upload(ecls.data(), ecls.size(), st);
  m->ent_tau.upload(etau.data(), etau.size(), st);
  std::vector<int32_t> emask(ecls.size(), 0);
  for (size_t e = 0; e < ecls.size(); ++e)
    for (int sl = 0; sl < NTG; ++sl) emask[e] |= (etau[e * NTG + sl] >= 0 ? 1 : 0) << sl;
  m->ent_mask.upload(emask.data(), emask.size(), st);
  m->hgrp_targets.upload(hgt.data(), hgt.size(), st);
  m->hent_cls.upload(hecls.data(), hecls.size(), st);
  m->hent_tau.upload(hetau.data(), hetau.size(), st);
  // chunk boundaries: chunk g of G holds the entries whose work prefix lies in
  // [ceil(W g / G), ceil(W (g + 1) / G))
  auto chunks = [](const std::vector<int32_t>& ptr, const std::vector<int32_t>& wpre,
                   const std::vector<int32_t>& wsum, std::vector<int32_t>& out, int64_t* off) {
    for (int c = 0; c < 7; ++c) {
      const int G = 1 << c;
      off[c] = (int64_t)out.size();
      for (size_t b = 0; b + 1 < ptr.size(); ++b) {
        const int32_t e0 = ptr[b], e1 = ptr[b + 1];
        const int64_t W = wsum[b];
        for (int g = 0; g <= G; ++g) {
          const int64_t lim = (W * g + G - 1) / G;
          int32_t e = e0;
          while (e < e1 && wpre[e] < lim) ++e;
          out.push_back(e);
        }
      }
    }
  };
  std::vector<int32_t> cfirst, hcfirst;
  chunks(gptr, ewpre, gw, cfirst, m->chunk_off);
  chunks(hgptr, hewpre, hgw, hcfirst, m->hchunk_off);
  m->chunk_first.upload(cfirst.data(), cfirst.size(), st);
  m->hchunk_first.upload(hcfirst.data(), hcfirst.size(), st);
  PH_HIP(hipStreamSynchronize(st));  // host staging buffers die with this call
  m->device_bytes = (int64_t)(m->U.bytes() + m->E.bytes() + m->perm.bytes() + m->first_child.bytes() +
                              m->iperm.bytes() + m->nchild.bytes() + m->cid.bytes() + m->parent.bytes() + m->nbegin.bytes() + m->nend.bytes() +
                              m->nstore.bytes() + m->nf_P.bytes() + m->nf_core.bytes() +
                              m->nf_theta.bytes() + m->tiles.bytes() + m->near_rowptr.bytes() +
                              m->near_tb.bytes() + m->near_D.bytes() + m->near_nt.bytes() + m->near_tr.bytes() +
                              m->up_rowptr.bytes() + m->up_tb.bytes() + m->up_D.bytes() + m->up_z.bytes() +
                              m->up_nt.bytes() + m->lo_rowptr.bytes() + m->lo_z.bytes() +
                              m->cstore.bytes() + m->ff_chat.bytes() + m->ff_theta.bytes() + m->grp_targets.bytes() +
                              m->grp_entry.bytes() + m->ent_cls.bytes() + m->ent_tau.bytes() + m->ent_mask.bytes() +
                              m->chunk_first.bytes() + m->mvm_items.bytes() + m->mvm_items64.bytes() + m->near_q.bytes() + m->hgrp_targets.bytes() + m->hent_cls.bytes() +
                              m->hent_tau.bytes() + m->hchunk_first.bytes());
  if (hm.hformat) upload_hmatrix(*m, t, hm, st);
  if (hm.implicit) upload_implicit(*m, t, hm, st);
  return m;
}

}  // namespace ph

// ====================================================================== C ABI
struct ph_tree {
  std::shared_ptr<const ph::TreeData> p;
};
struct ph_model {
  std::shared_ptr<const ph::DeviceModel> p;
};
struct ph_inst {
  std::shared_ptr<ph::InstData> p;
};
struct ph_graph {
  std::shared_ptr<ph::InstData> in;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~ph_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (in) --in->graphs;
  }
};

namespace {

template <typename F>
int guarded(F&& f) {
  try {
    ph::g_last_error.clear();
    f();
    return PH_OK;
  } catch (const ph::Failure& e) {
    ph::g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    ph::g_last_error = "host allocation failed";
    return PH_ENOMEM;
  } catch (const std::exception& e) {
    ph::g_last_error = e.what();
    return PH_EINVAL;
  } catch (...) {
    ph::g_last_error = "unknown failure";
    return PH_EINVAL;
  }
}

void need(bool ok, const char* msg) {
  if (!ok) ph::fail(PH_EINVAL, msg);
}

int inst_common(const ph_model* m, const double* theta, int T, int dim, ph_dtype dt, ph_near_mode near,
                void* stream, ph_inst** inout) {
  return guarded([&] {
    need(m && m->p, "model is NULL");
    need(theta != nullptr, "theta is NULL");
    need(inout != nullptr, "inout is NULL");
    need(T >= 1, "T must be >= 1");
    need(dt == PH_F64 || dt == PH_F32 || dt == PH_BF16, "dtype must be PH_F64, PH_F32 or PH_BF16");
    need(near == PH_NEAR_AUTO || near == PH_NEAR_BLOCKS || near == PH_NEAR_FACTORED, "invalid near-field mode");
    const ph::DeviceModel& md = *m->p;
    if (md.format != PH_FORMAT_H2 && dt != PH_F64)
      ph::fail(PH_EUNSUPPORTED, "parametric H-matrix and implicit-coupling models support PH_F64 instances only");
    if (near == PH_NEAR_FACTORED && md.KRp > 64)
      ph::fail(PH_EUNSUPPORTED, "factored near field supports near ranks up to 64");
    // automatic form: factored for one batch of 4..8 slots, where each factor entry read
    // serves every slot (8 slots: 4.4 vs 5.2 ms for the benchmark's near field); from 9 slots
    // on the factors are streamed once per batch of 8, and the written blocks win (64-slot
    // mixture sweep: 20 vs 40 ms per MVM)
    const bool factored = near == PH_NEAR_FACTORED || (near == PH_NEAR_AUTO && T >= 4 && T <= 8 && md.KRp <= 64);
    if (dim >= 0) need(dim < md.d_theta, "gradient dimension out of range");
    for (int t = 0; t < T; ++t)
      for (int k = 0; k < md.d_theta; ++k) {
        const double v = theta[(size_t)t * md.d_theta + k];
        if (!(v >= md.th_lo[k] && v <= md.th_hi[k]))
          ph::fail(PH_EDOMAIN, "theta outside the parameter box");
      }
    hipStream_t st = (hipStream_t)stream;
    std::shared_ptr<ph::InstData> in;
    if (*inout) {
      in = (*inout)->p;
      need(in && in->m.get() == &md && in->T == T && in->dt == dt,
           "instance does not match (model, T, dtype)");
      need(near == PH_NEAR_AUTO || (near == PH_NEAR_FACTORED) == in->factored,
           "instance does not match (near-field mode)");
      // a recorded graph replays the theta-vector launch with the flag it was recorded with
      if (in->graphs > 0 && dim != in->grad_dim)
        ph::fail(PH_ESTATE, "instance has recorded graphs; it cannot switch between K~ and dK~/dtheta");
      in->grad_dim = dim;
    } else {
      in = std::make_shared<ph::InstData>();
      in->m = m->p;
      in->T = T;
      in->dt = dt;
      in->grad_dim = dim;
      in->esize = dt == PH_F64 ? sizeof(double) : sizeof(float);
      in->d_esize = dt == PH_F64 ? sizeof(double) : dt == PH_F32 ? sizeof(float) : sizeof(ph::bf16);
      in->factored = factored;
      if (factored) {
        if (dt != PH_F64) ph::make_low_factors(md, dt, st);
        in->ccore.alloc((size_t)md.n_stored_near * T * md.KRp * in->esize);
      } else {
        in->D.alloc((size_t)T * md.N_nf_pad * in->d_esize);
      }
      if (md.format != PH_FORMAT_H2) in->C.alloc((size_t)T * md.h_tot * sizeof(double));   // H_q(theta_t)
      else in->C.alloc((size_t)T * md.n_classes * md.Pp * md.Pp * in->esize);
      if (md.format == PH_FORMAT_H2 && dt == PH_BF16 && md.min_far >= 0 && md.n_groups > 0 && ph::coupling_bf16_supported(md, ph::RC))
        in->Cb.alloc((size_t)T * ph::coupling_bf16_c_bytes(md));
      in->v.alloc((size_t)T * md.d_theta * md.p_theta);
      in->theta_d.alloc((size_t)T * md.d_theta);
      PH_HIP(hipHostMalloc((void**)&in->theta_pin, (size_t)T * md.d_theta * sizeof(double), hipHostMallocDefault));
      PH_HIP(hipEventCreateWithFlags(&in->ev_theta, hipEventDisableTiming));
      PH_HIP(hipStreamCreateWithFlags(&in->aux, hipStreamNonBlocking));
      PH_HIP(hipEventCreateWithFlags(&in->ev_fork, hipEventDisableTiming));
      PH_HIP(hipEventCreateWithFlags(&in->ev_join, hipEventDisableTiming));
      PH_HIP(hipEventCreateWithFlags(&in->ev_near, hipEventDisableTiming));
    }
    in->theta.assign(theta, theta + (size_t)T * md.d_theta);
    if (dt == PH_F64) ph::instantiate_impl<double, double>(*in, theta, st);
    else if (dt == PH_F32) ph::instantiate_impl<float, float>(*in, theta, st);
    else ph::instantiate_impl<float, ph::bf16>(*in, theta, st);
    if (!*inout) *inout = new ph_inst{in};
  });
}

}  // namespace

extern "C" {

const char* ph_last_error(void) { return ph::g_last_error.c_str(); }

const char* ph_version(void) { return "ph-mi355x 0.1 (gfx950)"; }

int ph_build_tree(const double* pts, int64_t n, const ph_tree_opts* opts, ph_tree** out) {
  return guarded([&] {
    need(opts != nullptr && out != nullptr, "opts or out is NULL");
    auto t = ph::build_tree(pts, n, *opts);
    *out = new ph_tree{t};
  });
}

int ph_tree_info_get(const ph_tree* t, ph_tree_info* info) {
  return guarded([&] {
    need(t && t->p && info, "NULL argument");
    const ph::TreeData& d = *t->p;
    info->n = d.n;
    info->d = d.d;
    info->l_max = d.l_max;
    info->n_nodes = d.n_nodes();
    info->n_leaves = (int64_t)d.leaves.size();
    info->n_near = d.n_near();
    info->n_far = d.n_far();
    info->n_classes = d.n_classes();
    info->near_entries = d.near_entries;
    info->min_far_level = d.min_far_level;
  });
}

int ph_tree_perm(const ph_tree* t, int64_t* perm) {
  return guarded([&] {
    need(t && t->p && perm, "NULL argument");
    std::memcpy(perm, t->p->perm.data(), t->p->perm.size() * sizeof(int64_t));
  });
}

int ph_tree_nodes(const ph_tree* t, int32_t* level, int32_t* coords, int64_t* begin, int64_t* end,
                  int32_t* parent) {
  return guarded([&] {
    need(t && t->p, "NULL tree");
    const ph::TreeData& d = *t->p;
    const size_t nn = (size_t)d.n_nodes();
    if (level) std::memcpy(level, d.level.data(), nn * sizeof(int32_t));
    if (coords) std::memcpy(coords, d.coords.data(), nn * d.d * sizeof(int32_t));
    if (begin) std::memcpy(begin, d.begin.data(), nn * sizeof(int64_t));
    if (end) std::memcpy(end, d.end.data(), nn * sizeof(int64_t));
    if (parent) std::memcpy(parent, d.parent.data(), nn * sizeof(int32_t));
  });
}

int ph_tree_blocks(const ph_tree* t, int32_t* near, int32_t* far, int32_t* far_class) {
  return guarded([&] {
    need(t && t->p, "NULL tree");
    const ph::TreeData& d = *t->p;
    if (near) std::memcpy(near, d.near.data(), d.near.size() * sizeof(int32_t));
    if (far) std::memcpy(far, d.far.data(), d.far.size() * sizeof(int32_t));
    if (far_class) std::memcpy(far_class, d.far_class.data(), d.far_class.size() * sizeof(int32_t));
  });
}

int ph_tree_classes(const ph_tree* t, int32_t* level, int32_t* offset) {
  return guarded([&] {
    need(t && t->p, "NULL tree");
    const ph::TreeData& d = *t->p;
    if (level) std::memcpy(level, d.class_level.data(), d.class_level.size() * sizeof(int32_t));
    if (offset) std::memcpy(offset, d.class_off.data(), d.class_off.size() * sizeof(int32_t));
  });
}

void ph_tree_free(ph_tree* t) { delete t; }

int ph_kernel_eval(ph_kernel kernel, int d, const double* x, const double* y, int64_t n, const double* theta,
                   double* out) {
  return guarded([&] {
    need(x && y && theta && out && n >= 0 && d >= 1 && d <= 3, "NULL argument, n < 0 or d outside 1..3");
    const int dth = ph::kernel_dtheta(kernel, d);
    if (dth < 0 || (kernel == PH_KERNEL_ANISO_GAUSSIAN && d > 2))
      ph::fail(PH_EUNSUPPORTED, "ph_kernel_eval: unknown kernel or unsupported kernel / d combination");
    const bool scale = kernel == PH_KERNEL_GAUSSIAN || kernel == PH_KERNEL_MATERN32 || kernel == PH_KERNEL_MATERN12 ||
                       kernel == PH_KERNEL_ANISO_GAUSSIAN || kernel == PH_KERNEL_MATERN;
    if (scale)
      for (int k = 0; k < dth; ++k)
        if (!(theta[k] > 0)) ph::fail(PH_EDOMAIN, "ph_kernel_eval: length scales and nu must be positive");
    for (int64_t i = 0; i < n; ++i) out[i] = ph::kernel_value(kernel, d, x + i * d, y + i * d, theta);
  });
}

int ph_offline_compress(const ph_tree* t, const ph_offline_opts* opts, void* stream, ph_model** out) {
  return guarded([&] {
    need(t && t->p && opts && out, "NULL argument");
    auto hm = ph::offline_host(*t->p, *opts);
    auto dm = ph::upload_model(t->p, *hm, (hipStream_t)stream);
    *out = new ph_model{dm};
  });
}

int ph_offline_compress_gpu(const ph_tree* t, const ph_offline_opts* opts, void* stream, ph_model** out) {
  return guarded([&] {
    need(t && t->p && opts && out, "NULL argument");
    auto hm = ph::offline_host(*t->p, *opts, true);
    auto dm = ph::upload_model(t->p, *hm, (hipStream_t)stream);
    *out = new ph_model{dm};
  });
}

int ph_offline_compress_h(const ph_tree* t, const ph_offline_opts* opts, void* stream, ph_model** out) {
  return guarded([&] {
    need(t && t->p && opts && out, "NULL argument");
    auto hm = ph::offline_host(*t->p, *opts);
    ph::hmatrix_far_host(*t->p, *hm, opts->num_threads);
    auto dm = ph::upload_model(t->p, *hm, (hipStream_t)stream);
    *out = new ph_model{dm};
  });
}

int ph_offline_compress_tt(const ph_tree* t, const ph_offline_opts* opts, int coupling, void* stream,
                           ph_model** out) {
  return guarded([&] {
    need(t && t->p && opts && out, "NULL argument");
    need(coupling == PH_COUPLING_MATERIALIZED || coupling == PH_COUPLING_IMPLICIT, "invalid coupling form");
    auto hm = ph::offline_host(*t->p, *opts, false, ph::Compress::TT);
    hm->implicit = coupling == PH_COUPLING_IMPLICIT && t->p->min_far_level >= 0;
    auto dm = ph::upload_model(t->p, *hm, (hipStream_t)stream);
    *out = new ph_model{dm};
  });
}

int ph_tt_far_ranks(const ph_tree* t, const ph_offline_opts* opts, int32_t* ranks, int64_t* kernel_evals) {
  return guarded([&] {
    need(t && t->p && opts && ranks, "NULL argument");
    int64_t ev = 0;
    const std::vector<int32_t> r = ph::tt_far_ranks(*t->p, *opts, &ev);
    std::copy(r.begin(), r.end(), ranks);
    if (kernel_evals) *kernel_evals = ev;
  });
}

int ph_model_format(const ph_model* m, int* format) {
  return guarded([&] {
    need(m && m->p && format, "NULL argument");
    *format = m->p->format;
  });
}

int ph_model_info_get(const ph_model* m, ph_model_info* info) {
  return guarded([&] {
    need(m && m->p && info, "NULL argument");
    const ph::DeviceModel& d = *m->p;
    info->n = d.n;
    info->n_near_stored = d.n_stored_near;
    info->n_classes_stored = d.n_stored_cls;
    info->near_entries = d.N_nf;
    info->near_factor_entries = d.near_factor_entries;
    info->near_rank_mean = d.near_rank_mean;
    info->near_rank_max = d.near_rank_max;
    info->far_rank_mean = d.far_rank_mean;
    info->far_rank_max = d.far_rank_max;
    info->device_bytes = d.device_bytes;
    info->kernel_evals = d.kernel_evals;
    info->P = d.P;
    info->p_theta = d.p_theta;
    info->d_theta = d.d_theta;
    info->svd_sweeps_max = d.svd_sweeps_max;
  });
}

int ph_model_near_ranks(const ph_model* m, int32_t* ranks) {
  return guarded([&] {
    need(m && m->p && ranks, "NULL argument");
    std::memcpy(ranks, m->p->near_rank_canon.data(), m->p->near_rank_canon.size() * sizeof(int32_t));
  });
}

int ph_model_class_ranks(const ph_model* m, int32_t* ranks) {
  return guarded([&] {
    need(m && m->p && ranks, "NULL argument");
    std::memcpy(ranks, m->p->class_ranks.data(), m->p->class_ranks.size() * sizeof(int32_t));
  });
}

void ph_model_free(ph_model* m) { delete m; }

int ph_instantiate(const ph_model* m, const double* theta, int T, ph_dtype dt, void* stream,
                   ph_inst** inout) {
  return inst_common(m, theta, T, -1, dt, PH_NEAR_AUTO, stream, inout);
}

int ph_instantiate_ex(const ph_model* m, const double* theta, int T, ph_dtype dt, ph_near_mode near, int grad_dim,
                      void* stream, ph_inst** inout) {
  if (grad_dim < -1) {
    ph::g_last_error = "gradient dimension out of range";
    return PH_EINVAL;
  }
  return inst_common(m, theta, T, grad_dim, dt, near, stream, inout);
}

int ph_inst_near_mode(const ph_inst* k, int* factored) {
  return guarded([&] {
    need(k && k->p && factored, "NULL argument");
    *factored = k->p->factored ? 1 : 0;
  });
}

int ph_instantiate_grad(const ph_model* m, const double* theta, int T, int dim, ph_dtype dt, void* stream,
                        ph_inst** inout) {
  if (dim < 0) {
    ph::g_last_error = "gradient dimension out of range";
    return PH_EINVAL;
  }
  return inst_common(m, theta, T, dim, dt, PH_NEAR_AUTO, stream, inout);
}

int ph_matvec(ph_inst* k, const void* x, void* y, int64_t R, double alpha, double beta, double nugget,
              void* stream) {
  return guarded([&] {
    need(k && k->p, "instance is NULL");
    need(R >= 0, "R must be >= 0");
    if (R == 0) return;
    need(x && y, "x or y is NULL");
    ph::InstData& in = *k->p;
    hipStream_t st = (hipStream_t)stream;
    if (in.dt == PH_F64)
      ph::matvec_impl<double, double>(in, (const double*)x, (double*)y, R, alpha, beta, nugget, st);
    else if (in.dt == PH_F32)
      ph::matvec_impl<float, float>(in, (const float*)x, (float*)y, R, alpha, beta, nugget, st);
    else
      ph::matvec_impl<float, ph::bf16>(in, (const float*)x, (float*)y, R, alpha, beta, nugget, st);
  });
}

// Scratch of ph_matvec_noalloc: one array per GPU, in the code object (no allocation at
// call time).  Its device address is looked up once per device with hipGetSymbolAddress;
// host code uses only that address, never the array's name.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

static void* noalloc_scratch() {
  int dev = -1;
  PH_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) ph::fail(PH_EUNSUPPORTED, "ph_matvec_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess || q == nullptr)
      ph::fail(PH_EHIP, std::string("ph_matvec_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = q;
  }
  return g_scratch_ptr[dev];
}

int ph_matvec_noalloc(ph_inst* k, const void* x, void* y, int64_t R, double alpha, double beta, double nugget,
                      void* stream) {
  return guarded([&] {
    need(k && k->p, "instance is NULL");
    need(R >= 0, "R must be >= 0");
    if (R == 0) return;
    need(x && y, "x or y is NULL");
    ph::InstData& in = *k->p;
    hipStream_t st = (hipStream_t)stream;
    const ph::ExtScratch ext{noalloc_scratch(), NOALLOC_SCRATCH_BYTES};
    if (in.dt == PH_F64)
      ph::matvec_impl<double, double>(in, (const double*)x, (double*)y, R, alpha, beta, nugget, st, &ext);
    else if (in.dt == PH_F32)
      ph::matvec_impl<float, float>(in, (const float*)x, (float*)y, R, alpha, beta, nugget, st, &ext);
    else
      ph::matvec_impl<float, ph::bf16>(in, (const float*)x, (float*)y, R, alpha, beta, nugget, st, &ext);
  });
}

int ph_bilinear(ph_inst* k, const void* u, const void* x, int64_t R, double* out, void* stream) {
  return guarded([&] {
    need(k && k->p, "instance is NULL");
    need(u && x && out, "u, x or out is NULL");
    need(R >= 1, "R must be >= 1");
    ph::InstData& in = *k->p;
    hipStream_t st = (hipStream_t)stream;
    if (in.dt == PH_F64)
      ph::bilinear_impl<double, double>(in, (const double*)u, (const double*)x, R, out, st);
    else if (in.dt == PH_F32)
      ph::bilinear_impl<float, float>(in, (const float*)u, (const float*)x, R, out, st);
    else
      ph::bilinear_impl<float, ph::bf16>(in, (const float*)u, (const float*)x, R, out, st);
  });
}

int ph_cg_solve_batch(ph_inst* hi, ph_inst* lo, const double* y, double* a, int64_t R, double nugget, double tol,
                      int max_iter, int inner_max, double inner_tol, ph_cg_stats* stats, void* stream) {
  return guarded([&] {
    need(hi && hi->p, "FP64 instance is NULL");
    need(y && a, "y or a is NULL");
    need(R >= 1 && R <= 1024, "R must be in 1..1024");
    ph::InstData& h = *hi->p;
    need(h.dt == PH_F64 && h.T == 1, "hi must be a PH_F64 instance with T = 1");
    need(h.grad_dim < 0, "hi must not be a gradient instance");
    need(tol > 0 && max_iter >= 1, "tol must be > 0 and max_iter >= 1");
    need(nugget >= 0, "nugget must be >= 0");
    ph::InstData* l = nullptr;
    if (lo) {
      need(lo->p != nullptr, "low-precision instance is empty");
      l = lo->p.get();
      need(l->dt == PH_F32 || l->dt == PH_BF16, "lo must be a PH_F32 or PH_BF16 instance");
      need(l->m == h.m && l->T == 1 && l->grad_dim < 0 && l->theta == h.theta,
           "lo must instantiate the same model at the same theta");
      need(inner_max >= 1 && inner_tol > 0, "inner_max must be >= 1 and inner_tol > 0");
    }
    ph::cg_solve_impl(h, l, y, a, R, nugget, tol, max_iter, inner_max, inner_tol, stats, (hipStream_t)stream);
  });
}

int ph_cg_solve(ph_inst* hi, ph_inst* lo, const double* y, double* a, double nugget, double tol, int max_iter,
                int inner_max, double inner_tol, ph_cg_stats* stats, void* stream) {
  return ph_cg_solve_batch(hi, lo, y, a, 1, nugget, tol, max_iter, inner_max, inner_tol, stats, stream);
}

int ph_autotune(ph_inst* k, const void* x, void* y, int64_t R, void* stream, ph_tune_info* info) {
  return guarded([&] {
    need(k && k->p, "instance is NULL");
    need(x && y && R >= 1, "x, y must be non-NULL and R >= 1");
    ph::InstData& in = *k->p;
    if (in.graphs > 0) ph::fail(PH_ESTATE, "instance has recorded graphs; tune before recording");
    const ph::DeviceModel& m = *in.m;
    hipStream_t st = (hipStream_t)stream;
    // the events are destroyed, and the instance keeps its previous configuration, also when
    // a trial fails
    struct Events {
      hipEvent_t a = nullptr, b = nullptr;
      ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
      }
    } ev;
    struct Restore {
      ph::InstData& in;
      int chunks, prefetch, overlap, tcb, rt;
      bool done = false;
      ~Restore() {
        if (done) return;
        in.tune_chunks = chunks;
        in.tune_prefetch = prefetch;
        in.tune_overlap = overlap;
        in.tune_fused_tcb = tcb;
        in.tune_fused_rt = rt;
      }
    } restore{in, in.tune_chunks, in.tune_prefetch, in.tune_overlap, in.tune_fused_tcb, in.tune_fused_rt};
    PH_HIP(hipEventCreate(&ev.a));
    PH_HIP(hipEventCreate(&ev.b));
    hipEvent_t a = ev.a, b = ev.b;
    auto run = [&] {
      if (in.dt == PH_F64)
        ph::matvec_impl<double, double>(in, (const double*)x, (double*)y, R, 1.0, 0.0, 0.0, st);
      else if (in.dt == PH_F32)
        ph::matvec_impl<float, float>(in, (const float*)x, (float*)y, R, 1.0, 0.0, 0.0, st);
      else
        ph::matvec_impl<float, ph::bf16>(in, (const float*)x, (float*)y, R, 1.0, 0.0, 0.0, st);
    };
    std::vector<int> chunks{1};
    for (int g : {2, 4, 8, 16})
      if (g <= m.max_group_entries) chunks.push_back(g);
    const int reps = 3;
    auto time_it = [&] {
      run();   // warm-up (allocates scratch for this configuration)
      PH_HIP(hipEventRecord(a, st));
      for (int r = 0; r < reps; ++r) run();
      PH_HIP(hipEventRecord(b, st));
      PH_HIP(hipEventSynchronize(b));
      float ms = 0;
      PH_HIP(hipEventElapsedTime(&ms, a, b));
      return ms / reps;
    };
    float best = 1e30f;
    ph_tune_info bi{};
    for (int ov : {1, 0})
      for (int pd : {1, 2})
        for (int g : chunks) {
          in.tune_chunks = g;
          in.tune_prefetch = pd;
          in.tune_overlap = ov;
          const float ms = time_it();
          if (ms < best) {
            best = ms;
            bi = ph_tune_info{g, pd, ov, (double)ms, in.tune_fused_tcb, in.tune_fused_rt};
          }
        }
    in.tune_chunks = bi.chunks;
    in.tune_prefetch = bi.prefetch;
    in.tune_overlap = bi.overlap;
    if (in.factored) {
      // then the factored near MVM's launch shape with that configuration: slots per
      // workgroup (each factor entry is read once per batch of them) and row tiles per wave
      for (int tcb : {8, 4, 2})
        for (int rt : {1, 2}) {
          if (tcb > 2 && tcb / 2 >= in.T) continue;   // the launch would clamp it
          in.tune_fused_tcb = tcb;
          in.tune_fused_rt = rt;
          const float ms = time_it();
          if (ms < best) {
            best = ms;
            bi.fused_tcb = tcb;
            bi.fused_rt = rt;
            bi.ms = ms;
          }
        }
      in.tune_fused_tcb = bi.fused_tcb;
      in.tune_fused_rt = bi.fused_rt;
    }
    restore.done = true;
    if (info) *info = bi;
  });
}

int ph_graph_create(ph_inst* k, const void* x, void* y, int64_t R, double nugget, void* stream, ph_graph** out) {
  return guarded([&] {
    need(k && k->p && out, "NULL argument");
    need(x && y && R >= 1, "x, y must be non-NULL and R >= 1");
    ph::InstData& in = *k->p;
    hipStream_t st = (hipStream_t)stream;
    need(st != nullptr, "recording needs a non-default stream");
    auto mv = [&] {
      if (in.dt == PH_F64)
        ph::matvec_impl<double, double>(in, (const double*)x, (double*)y, R, 1.0, 0.0, nugget, st);
      else if (in.dt == PH_F32)
        ph::matvec_impl<float, float>(in, (const float*)x, (float*)y, R, 1.0, 0.0, nugget, st);
      else
        ph::matvec_impl<float, ph::bf16>(in, (const float*)x, (float*)y, R, 1.0, 0.0, nugget, st);
    };
    auto inst = [&] {
      if (in.dt == PH_F64) ph::instantiate_impl<double, double>(in, nullptr, st);
      else if (in.dt == PH_F32) ph::instantiate_impl<float, float>(in, nullptr, st);
      else ph::instantiate_impl<float, ph::bf16>(in, nullptr, st);
    };
    mv();   // allocates every scratch buffer the recorded launches use
    PH_HIP(hipStreamSynchronize(st));
    if (in.theta_pending) PH_HIP(hipEventSynchronize(in.ev_theta));
    // (g->in is set only once the graph exists: the destructor releases the instance's
    // graph count, which a failed recording never took)
    auto g = std::make_unique<ph_graph>();
    ph::g_capturing = true;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      try {
        inst();
        mv();
      } catch (...) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(st, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        ph::g_capturing = false;
        throw;
      }
      e = hipStreamEndCapture(st, &g->graph);
    }
    ph::g_capturing = false;
    if (e != hipSuccess) ph::fail(PH_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    PH_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    g->in = k->p;
    ++in.graphs;
    *out = g.release();
  });
}

int ph_graph_launch(ph_graph* g, const double* theta, void* stream) {
  return guarded([&] {
    need(g && g->exec, "graph is NULL");
    ph::InstData& in = *g->in;
    const ph::DeviceModel& md = *in.m;
    if (theta) {
      for (int t = 0; t < in.T; ++t)
        for (int k = 0; k < md.d_theta; ++k) {
          const double v = theta[(size_t)t * md.d_theta + k];
          if (!(v >= md.th_lo[k] && v <= md.th_hi[k])) ph::fail(PH_EDOMAIN, "theta outside the parameter box");
        }
      if (in.theta_pending) PH_HIP(hipEventSynchronize(in.ev_theta));
      std::memcpy(in.theta_pin, theta, (size_t)in.T * md.d_theta * sizeof(double));
      in.theta.assign(theta, theta + (size_t)in.T * md.d_theta);
    }
    hipStream_t st = (hipStream_t)stream;
    // a near-field instantiation of an eager call may still run on the second stream; the
    // replay rewrites the theta vectors and the near blocks it reads
    ph::join_near(in, st);
    PH_HIP(hipGraphLaunch(g->exec, st));
    PH_HIP(hipEventRecord(in.ev_theta, st));
    in.theta_pending = true;
  });
}

void ph_graph_free(ph_graph* g) { delete g; }

int ph_inst_near_block(const ph_inst* k, int t, int64_t b, double* host_out) {
  return guarded([&] {
    need(k && k->p && host_out, "NULL argument");
    const ph::InstData& in = *k->p;
    const ph::DeviceModel& m = *in.m;
    need(t >= 0 && t < in.T, "slot out of range");
    need(b >= 0 && b < m.n_near, "near block index out of range");
    const ph::TreeData& tr = *m.tree;
    const int64_t ns = tr.size(tr.near[2 * b]), nt = tr.size(tr.near[2 * b + 1]);
    const bool trn = m.D_tr_host[b] != 0;
    const int64_t rows = trn ? nt : ns, cols = trn ? ns : nt;     // the stored block
    if (in.factored) {
      // no block in memory: evaluate the stored block from its factor and cores
      ph::DevArr<double> dev;
      dev.alloc((size_t)(rows * cols));
      const int64_t q = m.near_src_host[b];
      PH_HIP(hipDeviceSynchronize());
      if (in.dt == PH_F64) ph::near_block_eval<double, double>(in, t, q, dev.p, nullptr);
      else if (in.dt == PH_F32) ph::near_block_eval<float, float>(in, t, q, dev.p, nullptr);
      else ph::near_block_eval<float, ph::bf16>(in, t, q, dev.p, nullptr);
      std::vector<double> hb((size_t)(rows * cols));
      PH_HIP(hipMemcpy(hb.data(), dev.p, hb.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (int64_t j = 0; j < nt; ++j)
        for (int64_t i = 0; i < ns; ++i) host_out[i + j * ns] = trn ? hb[j + i * rows] : hb[i + j * rows];
      return;
    }
    const int64_t cnt = (rows + 15) / 16 * 16 * cols;
    PH_HIP(hipDeviceSynchronize());
    std::vector<char> buf(cnt * in.d_esize);
    PH_HIP(hipMemcpy(buf.data(), in.D.p + ((size_t)t * m.N_nf_pad + m.D_off_host[b]) * in.d_esize, buf.size(),
                     hipMemcpyDeviceToHost));
    auto val = [&](int64_t idx) {
      return in.dt == PH_F64   ? ((double*)buf.data())[idx]
             : in.dt == PH_F32 ? (double)((float*)buf.data())[idx]
                               : (double)ph::from_bf16(((ph::bf16*)buf.data())[idx]);
    };
    for (int64_t j = 0; j < nt; ++j)
      for (int64_t i = 0; i < ns; ++i)
        host_out[i + j * ns] = trn ? val(ph::panel_index(j, i, cols)) : val(ph::panel_index(i, j, cols));
  });
}

int ph_inst_coupling(const ph_inst* k, int t, int64_t c, double* host_out) {
  return guarded([&] {
    need(k && k->p && host_out, "NULL argument");
    const ph::InstData& in = *k->p;
    const ph::DeviceModel& m = *in.m;
    need(t >= 0 && t < in.T, "slot out of range");
    need(c >= 0 && c < m.n_classes, "class index out of range");
    if (m.format != PH_FORMAT_H2)
      ph::fail(PH_EUNSUPPORTED, "ph_inst_coupling: the instance forms no coupling matrices (H-matrix format or "
                                "implicit coupling)");
    const int64_t cnt = (int64_t)m.Pp * m.Pp;
    PH_HIP(hipDeviceSynchronize());
    std::vector<char> buf(cnt * in.esize);
    PH_HIP(hipMemcpy(buf.data(), in.C.p + ((size_t)t * m.n_classes * cnt + c * cnt) * in.esize, buf.size(),
                     hipMemcpyDeviceToHost));
    for (int j = 0; j < m.P; ++j)
      for (int i = 0; i < m.P; ++i) {
        const int64_t src = ph::frag_index(i, j, m.Pp);
        host_out[i + (int64_t)m.P * j] =
            in.dt == PH_F64 ? ((double*)buf.data())[src] : (double)((float*)buf.data())[src];
      }
  });
}

void ph_inst_free(ph_inst* k) { delete k; }

int ph_trace_enable(int on) {
  return guarded([&] {
    std::lock_guard<std::mutex> lk(ph::g_trace_mu);
    ph::g_trace_on = on != 0;
  });
}

int ph_trace_read(ph_trace_stats* out, int reset) {
  return guarded([&] {
    need(out != nullptr, "out is NULL");
    std::lock_guard<std::mutex> lk(ph::g_trace_mu);
    for (int i = 0; i < PH_NUM_STAGES; ++i) {
      out->ms[i] = 0;
      out->count[i] = 0;
    }
    for (auto& r : ph::g_trace_recs) {
      PH_HIP(hipEventSynchronize(r.b));
      float ms = 0;
      PH_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      out->ms[r.stage] += ms;
      out->count[r.stage] += 1;
    }
    if (reset) {
      for (auto& r : ph::g_trace_recs) {
        ph::g_event_pool.push_back(r.a);
        ph::g_event_pool.push_back(r.b);
      }
      ph::g_trace_recs.clear();
    }
  });
}

}  // extern "C"
