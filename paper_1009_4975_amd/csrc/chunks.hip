// Host-side construction of the octree operator chunks.
//
// Every unconstrained node is owned by exactly one chunk: the chunk holding
// the first element (in space-filling-curve order) that touches it, where an
// element touches a node if the node is one of its vertices or a master of one
// of its hanging vertices.  A chunk is a run of consecutive elements plus the
// halo elements that touch its owned nodes from outside the run, so the chunk
// sees every contribution to its owned rows and can write them directly: the
// operator needs one pass, no atomics in global memory and no second
// reduction pass, and it is deterministic.  Each hanging node is owned (for
// its identity row) by the chunk of the first element having it as a vertex.
//
// Node table order inside a chunk: [owned regular | other regular | owned
// hanging | other hanging]; hanging interpolation is kept as (hanging entry,
// master entry, weight) triples.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace amrto {

namespace {

template <typename V>
hipError_t upload(V*& dst, const std::vector<V>& v) {
  if (dst) (void)hipFree(dst);
  dst = nullptr;
  hipError_t e = hipMalloc((void**)&dst, std::max<size_t>(1, v.size()) * sizeof(V));
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(dst, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice);
  return e;
}

struct Tables {
  std::vector<int32_t> chunk_cnt;  // 8 per chunk
  std::vector<int32_t> ent_elem, tab_node, tab_hbeg;
  std::vector<uint16_t> ent_loc;
  std::vector<uint32_t> trip_hm;
  std::vector<double> trip_w;
};

}  // namespace

int build_chunks(amrto_ctx* ctx, const amrto_mesh* m) {
  const int nn = m->n_nodes, ne = m->n_elems;
  std::vector<int> hidx(nn, -1);
  for (int i = 0; i < m->n_hang; ++i) {
    const int h = m->hang_node[i];
    if (h < 0 || h >= nn || hidx[h] >= 0)
      return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: bad or repeated hanging node");
    hidx[h] = i;
  }
  for (int i = 0; i < m->n_hang; ++i) {
    const int b = m->hang_ptr[i], e = m->hang_ptr[i + 1];
    if (e < b || e - b > 16) return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: hanging node with bad master count");
    for (int k = b; k < e; ++k) {
      const int mm = m->hang_master[k];
      if (mm < 0 || mm >= nn) return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: master out of range");
      if (hidx[mm] >= 0) return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: a master is itself hanging");
      if (!std::isfinite(m->hang_w[k])) return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: bad weight");
    }
  }
  // element -> touched regular nodes (vertices and masters), CSR
  std::vector<int> tptr(ne + 1, 0), tnode;
  tnode.reserve(12L * ne);
  {
    std::vector<int> tmp;
    for (int e = 0; e < ne; ++e) {
      tmp.clear();
      for (int a = 0; a < 8; ++a) {
        const int v = m->elem_nodes[8L * e + a];
        if (hidx[v] < 0) tmp.push_back(v);
        else
          for (int k = m->hang_ptr[hidx[v]]; k < m->hang_ptr[hidx[v] + 1]; ++k) tmp.push_back(m->hang_master[k]);
      }
      std::sort(tmp.begin(), tmp.end());
      tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
      tnode.insert(tnode.end(), tmp.begin(), tmp.end());
      tptr[e + 1] = (int)tnode.size();
    }
  }
  // owner element: first touching element (regular) / first element with it as a vertex (hanging)
  std::vector<int> owner(nn, ne);
  for (int e = 0; e < ne; ++e) {
    for (int k = tptr[e]; k < tptr[e + 1]; ++k) owner[tnode[k]] = std::min(owner[tnode[k]], e);
    for (int a = 0; a < 8; ++a) {
      const int v = m->elem_nodes[8L * e + a];
      if (hidx[v] >= 0) owner[v] = std::min(owner[v], e);
    }
  }
  for (int v = 0; v < nn; ++v)
    if (owner[v] == ne) return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: a node belongs to no element");
  // node -> touching elements (regular nodes), CSR
  std::vector<int> nptr(nn + 1, 0), nelem(tnode.size());
  for (int v : tnode) nptr[v + 1]++;
  for (int v = 0; v < nn; ++v) nptr[v + 1] += nptr[v];
  {
    std::vector<int> fill(nptr.begin(), nptr.end() - 1);
    for (int e = 0; e < ne; ++e)
      for (int k = tptr[e]; k < tptr[e + 1]; ++k) nelem[fill[tnode[k]]++] = e;
  }
  // owned nodes grouped by owner element
  std::vector<int> optr(ne + 1, 0), onode(nn);
  for (int v = 0; v < nn; ++v) optr[owner[v] + 1]++;
  for (int e = 0; e < ne; ++e) optr[e + 1] += optr[e];
  {
    std::vector<int> fill(optr.begin(), optr.end() - 1);
    for (int v = 0; v < nn; ++v) onode[fill[owner[v]]++] = v;
  }

  // Chunk boundaries.  The operator pass of a chunk takes a fixed time plus
  // time in proportion to its entries and, at half that rate, its hanging
  // triples (measured on the octree cantilever), and a launch lasts as long
  // as its heaviest chunk.  Runs of consecutive elements are therefore grown
  // one element at a time (the entry set and node table followed
  // incrementally) while the tables fit and that cost stays under a cap; the
  // cap is the smallest (bisection) that keeps the number of chunks at most
  // what runs of CH_MAX elements give, rounded up to a multiple of 8 (the
  // launch grid is rounded so anyway).  Light runs may exceed CH_MAX
  // elements, up to RUN_MAX, as long as their tables fit.
  constexpr double W_TRIP = 0.5, W_FIX = 390.0;  // cost per entry = 1
  constexpr int RUN_MAX = 4 * CH_MAX;
  std::vector<int> mk_e(ne, -1), mk_n(nn, -1);
  std::vector<std::pair<int, int>> jr_e, jr_n;  // (index, previous stamp) of one element's additions
  int stamp = 0;
  auto plan = [&](double cap, int run_max, long limit, std::vector<int>* ends) -> long {
    long count = 0;
    int b = 0;
    while (b < ne) {
      const int s = stamp++;
      long n_ent = 0, n_tab = 0, n_trip = 0;
      auto add_node = [&](int v) {
        if (mk_n[v] == s) return;
        jr_n.push_back({v, mk_n[v]});
        mk_n[v] = s;
        ++n_tab;
        if (hidx[v] >= 0) n_trip += m->hang_ptr[hidx[v] + 1] - m->hang_ptr[hidx[v]];
      };
      auto add_ent = [&](int f) {
        if (mk_e[f] == s) return;
        jr_e.push_back({f, mk_e[f]});
        mk_e[f] = s;
        ++n_ent;
        for (int a = 0; a < 8; ++a) {
          const int v = m->elem_nodes[8L * f + a];
          add_node(v);
          if (hidx[v] >= 0)
            for (int k = m->hang_ptr[hidx[v]]; k < m->hang_ptr[hidx[v] + 1]; ++k) add_node(m->hang_master[k]);
        }
      };
      int e = b;
      while (e < ne && e - b < run_max) {
        jr_e.clear();
        jr_n.clear();
        const long se = n_ent, st = n_tab, sh = n_trip;
        add_ent(e);
        for (int k = optr[e]; k < optr[e + 1]; ++k) {
          const int v = onode[k];
          if (hidx[v] >= 0) continue;
          for (int j = nptr[v]; j < nptr[v + 1]; ++j) add_ent(nelem[j]);
        }
        const bool fits = n_tab <= TAB_MAX && n_ent <= ENT_MAX && n_trip <= TRIP_MAX;
        if (!fits || (e > b && W_FIX + n_ent + W_TRIP * n_trip > cap)) {
          for (const auto& p : jr_e) mk_e[p.first] = p.second;
          for (const auto& p : jr_n) mk_n[p.first] = p.second;
          n_ent = se;
          n_tab = st;
          n_trip = sh;
          if (e == b) ++e;  // one element alone does not fit: reported when the chunk is built
          break;
        }
        ++e;
      }
      if (ends) ends->push_back(e);
      if (++count > limit) return count;
      b = e;
    }
    return count;
  };
  const long n_fixed = plan(1e300, CH_MAX, ne, nullptr);
  const long target = (n_fixed + 7) / 8 * 8;
  double lo = W_FIX, hi = W_FIX + ENT_MAX + W_TRIP * TRIP_MAX + 1.0;
  const bool balanced = plan(hi, RUN_MAX, target, nullptr) <= target;
  for (int it = 0; balanced && it < 14 && hi - lo > 0.5; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (plan(mid, RUN_MAX, target, nullptr) <= target) hi = mid;
    else lo = mid;
  }
  std::vector<int> ends;
  if (balanced) plan(hi, RUN_MAX, ne, &ends);
  else plan(1e300, CH_MAX, ne, &ends);

  Tables T;
  std::vector<int> mark_e(ne, -1), loc(nn, -1);
  int cid = 0;
  std::vector<int> ents, own_reg, own_h, oth_reg, oth_h;
  std::vector<int> nstamp(nn, -1);
  int e0 = 0;
  size_t run = 0;
  long n_real_entries = 0;
  while (e0 < ne) {
    while (run < ends.size() && ends[run] <= e0) ++run;
    int e1 = run < ends.size() ? ends[run] : ne;
    while (true) {
      // gather the chunk for run [e0, e1)
      ents.clear(); own_reg.clear(); own_h.clear(); oth_reg.clear(); oth_h.clear();
      const int stamp_id = cid;
      for (int e = e0; e < e1; ++e) { mark_e[e] = stamp_id; ents.push_back(e); }
      for (int e = e0; e < e1; ++e)
        for (int k = optr[e]; k < optr[e + 1]; ++k) {
          const int v = onode[k];
          if (hidx[v] >= 0) { own_h.push_back(v); continue; }
          own_reg.push_back(v);
          for (int j = nptr[v]; j < nptr[v + 1]; ++j) {
            const int f = nelem[j];
            if (mark_e[f] != stamp_id) { mark_e[f] = stamp_id; ents.push_back(f); }
          }
        }
      for (int v : own_reg) nstamp[v] = stamp_id;
      for (int v : own_h) nstamp[v] = stamp_id;
      for (int e : ents)
        for (int a = 0; a < 8; ++a) {
          const int v = m->elem_nodes[8L * e + a];
          if (nstamp[v] != stamp_id) {
            nstamp[v] = stamp_id;
            (hidx[v] >= 0 ? oth_h : oth_reg).push_back(v);
          }
          if (hidx[v] >= 0)
            for (int k = m->hang_ptr[hidx[v]]; k < m->hang_ptr[hidx[v] + 1]; ++k) {
              const int mm = m->hang_master[k];
              if (nstamp[mm] != stamp_id) { nstamp[mm] = stamp_id; oth_reg.push_back(mm); }
            }
        }
      const size_t nt = own_reg.size() + oth_reg.size() + own_h.size() + oth_h.size();
      size_t ntrip = 0;
      for (int v : own_h) ntrip += m->hang_ptr[hidx[v] + 1] - m->hang_ptr[hidx[v]];
      for (int v : oth_h) ntrip += m->hang_ptr[hidx[v] + 1] - m->hang_ptr[hidx[v]];
      const bool fits = nt <= (size_t)TAB_MAX && ents.size() <= (size_t)ENT_MAX && ntrip <= (size_t)TRIP_MAX;
      if (fits || e1 - e0 == 1) {
        if (!fits)
          return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: one element's neighbourhood exceeds a chunk table");
        break;
      }
      ++cid;  // fresh stamps for the retry
      e1 = e0 + (e1 - e0) / 2;
    }
    // commit chunk [e0, e1)
    int t = 0;
    for (int v : own_reg) loc[v] = t++;
    for (int v : oth_reg) loc[v] = t++;
    const int nreg = t;
    for (int v : own_h) loc[v] = t++;
    for (int v : oth_h) loc[v] = t++;
    std::sort(ents.begin(), ents.end());
    // this chunk's slots at fixed strides, zero padded (kc = chunks so far)
    const size_t kc = T.chunk_cnt.size() / 8;
    const size_t eb = kc * ENT_MAX, tb = kc * TAB_MAX, hb = kc * TRIP_MAX;
    T.ent_elem.resize(eb + ENT_MAX, 0);
    T.ent_loc.resize(8 * (eb + ENT_MAX), 0);
    T.tab_node.resize(tb + TAB_MAX, 0);
    T.tab_hbeg.resize(tb + TAB_MAX, 0);
    T.trip_hm.resize(hb + TRIP_MAX, 0);
    T.trip_w.resize(hb + TRIP_MAX, 0.0);
    for (size_t i = 0; i < ents.size(); ++i) {
      const int e = ents[i];
      T.ent_elem[eb + i] = e;
      for (int a = 0; a < 8; ++a) T.ent_loc[8 * (eb + i) + a] = (uint16_t)loc[m->elem_nodes[8L * e + a]];
    }
    {
      size_t i = tb;
      for (int v : own_reg) T.tab_node[i++] = v;
      for (int v : oth_reg) T.tab_node[i++] = v;
      for (int v : own_h) T.tab_node[i++] = v;
      for (int v : oth_h) T.tab_node[i++] = v;
    }
    int ntrip = 0;
    auto add_trips = [&](const std::vector<int>& hs) {
      for (int h : hs) {
        T.tab_hbeg[tb + loc[h]] = ntrip;
        for (int k = m->hang_ptr[hidx[h]]; k < m->hang_ptr[hidx[h] + 1]; ++k) {
          T.trip_hm[hb + ntrip] = ((uint32_t)loc[h] << 16) | (uint32_t)loc[m->hang_master[k]];
          T.trip_w[hb + ntrip] = m->hang_w[k];
          ++ntrip;
        }
      }
    };
    add_trips(own_h);
    add_trips(oth_h);
    const int cnt[8] = {(int)ents.size(), t, ntrip, (int)own_reg.size(), nreg, (int)own_h.size(), 0, 0};
    T.chunk_cnt.insert(T.chunk_cnt.end(), cnt, cnt + 8);
    n_real_entries += (long)ents.size();
    ++cid;
    e0 = e1;
  }
  const int nc = (int)(T.chunk_cnt.size() / 8);
  AMRTO_HIP(upload(ctx->d_chunk_cnt, T.chunk_cnt));
  AMRTO_HIP(upload(ctx->d_ent_elem, T.ent_elem));
  AMRTO_HIP(upload(ctx->d_ent_loc, T.ent_loc));
  AMRTO_HIP(upload(ctx->d_tab_node, T.tab_node));
  AMRTO_HIP(upload(ctx->d_trip_hm, T.trip_hm));
  AMRTO_HIP(upload(ctx->d_trip_w, T.trip_w));
  AMRTO_HIP(upload(ctx->d_tab_hbeg, T.tab_hbeg));

  // hanging lists (recovery, masks) and the transpose used for loads
  std::vector<int> hang_node(m->hang_node, m->hang_node + m->n_hang);
  std::vector<int> hang_ptr(m->hang_ptr, m->hang_ptr + m->n_hang + 1);
  const int nhe = m->n_hang ? m->hang_ptr[m->n_hang] : 0;
  std::vector<int> hang_master(m->hang_master, m->hang_master + nhe);
  std::vector<double> hang_w(m->hang_w, m->hang_w + nhe);
  std::vector<int> mt_count(nn, 0);
  for (int k = 0; k < nhe; ++k) mt_count[hang_master[k]]++;
  std::vector<int> mt_node, mt_ptr{0}, mt_h, mt_pos(nn, -1);
  std::vector<double> mt_w;
  for (int v = 0; v < nn; ++v)
    if (mt_count[v] > 0) {
      mt_pos[v] = mt_ptr.back();
      mt_node.push_back(v);
      mt_ptr.push_back(mt_ptr.back() + mt_count[v]);
    }
  mt_h.resize(mt_ptr.back());
  mt_w.resize(mt_ptr.back());
  for (int i = 0; i < m->n_hang; ++i)
    for (int k = hang_ptr[i]; k < hang_ptr[i + 1]; ++k) {
      const int mm = hang_master[k];
      mt_h[mt_pos[mm]] = hang_node[i];
      mt_w[mt_pos[mm]] = hang_w[k];
      mt_pos[mm]++;
    }
  AMRTO_HIP(upload(ctx->d_hang_node, hang_node));
  AMRTO_HIP(upload(ctx->d_hang_ptr, hang_ptr));
  AMRTO_HIP(upload(ctx->d_hang_master, hang_master));
  AMRTO_HIP(upload(ctx->d_hang_w, hang_w));
  AMRTO_HIP(upload(ctx->d_mt_node, mt_node));
  AMRTO_HIP(upload(ctx->d_mt_ptr, mt_ptr));
  AMRTO_HIP(upload(ctx->d_mt_h, mt_h));
  AMRTO_HIP(upload(ctx->d_mt_w, mt_w));
  ctx->n_mt = (int)mt_node.size();
  ctx->n_chunks = nc;
  ctx->n_entries = (int)n_real_entries;
  ctx->n_hang = m->n_hang;
  return AMRTO_OK;
}

}  // namespace amrto
