// Host-side quadtree of the 2-D variant (paper Sec. 4, Sec. 6 and Sec. 7,
// Test 1): leaves with refinement and derefinement, level-one compatibility
// across edges, marking with the two compatibility sweeps, density and
// displacement transfer, and the Q4 finite-element mesh (nodes,
// connectivity, hanging-node interpolation, supports, a point load).
//
// Leaves are (level, anchor) on the finest lattice; a level-l leaf has edge
// 2^(max_level - l).  Leaves are kept in Morton order, so every family of four
// siblings is contiguous.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "amrto.h"

namespace {

struct QLeaf {
  int8_t level;
  int32_t x, y;
};

inline uint64_t spread2(uint64_t v) {
  v &= 0xffffffffULL;
  v = (v | v << 16) & 0x0000ffff0000ffffULL;
  v = (v | v << 8) & 0x00ff00ff00ff00ffULL;
  v = (v | v << 4) & 0x0f0f0f0f0f0f0f0fULL;
  v = (v | v << 2) & 0x3333333333333333ULL;
  v = (v | v << 1) & 0x5555555555555555ULL;
  return v;
}
inline uint64_t morton2(int32_t x, int32_t y) { return spread2((uint64_t)x) | spread2((uint64_t)y) << 1; }
inline uint64_t qkey(int level, int64_t x, int64_t y) {
  return (uint64_t)level << 56 | (uint64_t)(x & 0xfffffff) << 28 | (uint64_t)(y & 0xfffffff);
}

const int kEdge[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};

struct QMesh {
  std::vector<int32_t> xy, elem_nodes;
  std::vector<int8_t> level;
  std::vector<int32_t> anchor;
  std::vector<int32_t> hang_node, hang_ptr, hang_master;
  std::vector<double> hang_w;
  std::vector<uint8_t> fixed;
  std::vector<double> load;
  std::unordered_map<uint64_t, int> node_of;
};

}  // namespace

struct amrto_quadtree {
  int32_t base[2];
  int32_t L;
  int32_t dims[2];
  std::vector<QLeaf> leaves;
  std::vector<double> rho_new;
  QMesh mesh, old_mesh;
  bool has_old = false;

  int32_t size_of(int level) const { return 1 << (L - level); }
  void sort_leaves(std::vector<QLeaf>& v, std::vector<int>* carry) const {
    std::vector<size_t> perm(v.size());
    for (size_t i = 0; i < perm.size(); ++i) perm[i] = i;
    std::sort(perm.begin(), perm.end(), [&](size_t a, size_t b) {
      const uint64_t ka = morton2(v[a].x, v[a].y), kb = morton2(v[b].x, v[b].y);
      return ka != kb ? ka < kb : v[a].level < v[b].level;
    });
    std::vector<QLeaf> s(v.size());
    std::vector<int> c(carry ? carry->size() : 0);
    for (size_t i = 0; i < perm.size(); ++i) {
      s[i] = v[perm[i]];
      if (carry) c[i] = (*carry)[perm[i]];
    }
    v.swap(s);
    if (carry) carry->swap(c);
  }
  std::unordered_map<uint64_t, int> index(const std::vector<QLeaf>& v) const {
    std::unordered_map<uint64_t, int> m;
    m.reserve(v.size() * 2);
    for (size_t i = 0; i < v.size(); ++i) m.emplace(qkey(v[i].level, v[i].x, v[i].y), (int)i);
    return m;
  }
  // the leaf containing the point (hx / 2, hy / 2) (half-lattice units), or -1
  int find(const std::unordered_map<uint64_t, int>& idx, int64_t hx, int64_t hy) const {
    if (hx < 0 || hy < 0 || hx >= 2LL * dims[0] || hy >= 2LL * dims[1]) return -1;
    for (int l = 0; l <= L; ++l) {
      const int64_t s2 = 2LL * size_of(l);
      auto it = idx.find(qkey(l, hx / s2 * (s2 / 2), hy / s2 * (s2 / 2)));
      if (it != idx.end()) return it->second;
    }
    return -1;
  }
};

namespace {

void qsplit(amrto_quadtree* t, const std::vector<uint8_t>& marks, std::vector<int>* src) {
  std::vector<QLeaf> out;
  std::vector<int> s;
  for (size_t i = 0; i < t->leaves.size(); ++i) {
    const QLeaf& f = t->leaves[i];
    if (marks[i] && f.level < t->L) {
      const int32_t h = t->size_of(f.level + 1);
      for (int c = 0; c < 4; ++c) {
        out.push_back({(int8_t)(f.level + 1), f.x + h * (c & 1), f.y + h * (c >> 1)});
        s.push_back(src ? (*src)[i] : (int)i);
      }
    } else {
      out.push_back(f);
      s.push_back(src ? (*src)[i] : (int)i);
    }
  }
  t->sort_leaves(out, &s);
  t->leaves.swap(out);
  if (src) src->swap(s);
}

// level-one closure across edges: a leaf whose same-size edge neighbour cell
// lies in a leaf two or more levels coarser splits that leaf
void qbalance(amrto_quadtree* t, std::vector<int>* src) {
  while (true) {
    auto idx = t->index(t->leaves);
    std::vector<uint8_t> marks(t->leaves.size(), 0);
    bool any = false;
    for (const QLeaf& f : t->leaves) {
      const int64_t s = t->size_of(f.level);
      for (const auto& d : kEdge) {
        const int c = t->find(idx, 2 * (f.x + d[0] * s) + s, 2 * (f.y + d[1] * s) + s);
        if (c >= 0 && t->leaves[c].level < f.level - 1 && !marks[c]) {
          marks[c] = 1;
          any = true;
        }
      }
    }
    if (!any) return;
    qsplit(t, marks, src);
  }
}

}  // namespace

extern "C" {

int amrto_quadtree_create(amrto_quadtree** out, const int32_t base[2], int32_t max_level) {
  if (!out || !base) return AMRTO_EINVAL;
  *out = nullptr;
  if (base[0] < 1 || base[1] < 1 || max_level < 0 || max_level > 20) return AMRTO_EINVAL;
  if ((int64_t)base[0] << max_level > (1 << 27) || (int64_t)base[1] << max_level > (1 << 27)) return AMRTO_EINVAL;
  amrto_quadtree* t = new (std::nothrow) amrto_quadtree();
  if (!t) return AMRTO_ENOMEM;
  t->base[0] = base[0];
  t->base[1] = base[1];
  t->L = max_level;
  t->dims[0] = base[0] << max_level;
  t->dims[1] = base[1] << max_level;
  for (int32_t j = 0; j < base[1]; ++j)
    for (int32_t i = 0; i < base[0]; ++i) t->leaves.push_back({0, i << max_level, j << max_level});
  t->sort_leaves(t->leaves, nullptr);
  *out = t;
  return AMRTO_OK;
}

int amrto_quadtree_destroy(amrto_quadtree* t) {
  delete t;
  return AMRTO_OK;
}

int32_t amrto_quadtree_n_leaves(const amrto_quadtree* t) { return t ? (int32_t)t->leaves.size() : -1; }

int amrto_quadtree_leaves(const amrto_quadtree* t, int8_t* level, int32_t* anchor) {
  if (!t || !level || !anchor) return AMRTO_EINVAL;
  for (size_t i = 0; i < t->leaves.size(); ++i) {
    level[i] = t->leaves[i].level;
    anchor[2 * i] = t->leaves[i].x;
    anchor[2 * i + 1] = t->leaves[i].y;
  }
  return AMRTO_OK;
}

int amrto_quadtree_refine(amrto_quadtree* t, const uint8_t* marks) {
  if (!t || !marks) return AMRTO_EINVAL;
  qsplit(t, std::vector<uint8_t>(marks, marks + t->leaves.size()), nullptr);
  t->mesh = QMesh();
  return AMRTO_OK;
}

int amrto_quadtree_balance(amrto_quadtree* t) {
  if (!t) return AMRTO_EINVAL;
  qbalance(t, nullptr);
  t->mesh = QMesh();
  return AMRTO_OK;
}

int amrto_quadtree_adapt(amrto_quadtree* t, const double* rho, double rho_s, double r_amr, int32_t* n_new) {
  if (!t || !rho || !n_new || !(r_amr >= 0.0)) return AMRTO_EINVAL;
  const size_t n = t->leaves.size();
  auto cen = [&](const QLeaf& f, double* c) {
    const double h = t->size_of(f.level);
    c[0] = f.x + 0.5 * h;
    c[1] = f.y + 0.5 * h;
  };
  // marking: solid, or a solid centre within r_amr (inclusive, centre to centre)
  std::vector<int8_t> mark(n, 0);
  {
    const double cell = std::max(1.0, r_amr);
    std::unordered_map<uint64_t, std::vector<int>> grid;
    auto gk = [](int64_t a, int64_t b) { return (uint64_t)(a + (1 << 20)) << 32 | (uint64_t)(b + (1 << 20)); };
    for (size_t i = 0; i < n; ++i)
      if (rho[i] >= rho_s) {
        double c[2];
        cen(t->leaves[i], c);
        grid[gk((int64_t)std::floor(c[0] / cell), (int64_t)std::floor(c[1] / cell))].push_back((int)i);
      }
    const int reach = (int)std::ceil(r_amr / cell);
    for (size_t i = 0; i < n; ++i) {
      bool near = rho[i] >= rho_s;
      double c[2];
      cen(t->leaves[i], c);
      const int64_t gx = (int64_t)std::floor(c[0] / cell), gy = (int64_t)std::floor(c[1] / cell);
      for (int dy = -reach; dy <= reach && !near; ++dy)
        for (int dx = -reach; dx <= reach && !near; ++dx) {
          auto it = grid.find(gk(gx + dx, gy + dy));
          if (it == grid.end()) continue;
          for (int s : it->second) {
            double d[2];
            cen(t->leaves[s], d);
            if ((d[0] - c[0]) * (d[0] - c[0]) + (d[1] - c[1]) * (d[1] - c[1]) <= r_amr * r_amr) {
              near = true;
              break;
            }
          }
        }
      if (near) mark[i] = t->leaves[i].level < t->L ? 1 : 0;
      else mark[i] = t->leaves[i].level > 0 ? -1 : 0;
    }
  }
  auto parent_key = [&](const QLeaf& f) {
    const int32_t ps = t->size_of(f.level - 1);
    return qkey(f.level - 1, f.x / ps * ps, f.y / ps * ps);
  };
  auto sweep1 = [&](const std::vector<QLeaf>& lv, std::vector<uint8_t>& dm) {
    std::unordered_map<uint64_t, int> cnt;
    for (size_t i = 0; i < lv.size(); ++i)
      if (dm[i]) cnt[parent_key(lv[i])]++;
    for (size_t i = 0; i < lv.size(); ++i)
      if (dm[i] && cnt[parent_key(lv[i])] != 4) dm[i] = 0;
  };
  std::vector<uint8_t> dmark(n), rmark(n);
  for (size_t i = 0; i < n; ++i) {
    dmark[i] = mark[i] == -1;
    rmark[i] = mark[i] == 1;
  }
  sweep1(t->leaves, dmark);
  std::vector<int> src(n);
  for (size_t i = 0; i < n; ++i) src[i] = (int)i;
  qsplit(t, rmark, &src);
  qbalance(t, &src);
  std::vector<int> nsplit(n, 0);
  for (int s : src) nsplit[s]++;
  const size_t m = t->leaves.size();
  std::vector<uint8_t> dm(m, 0);
  for (size_t i = 0; i < m; ++i) dm[i] = dmark[src[i]] && nsplit[src[i]] == 1;
  sweep1(t->leaves, dm);
  // sweep 2: drop families whose parent would meet a leaf two levels finer across an edge
  while (true) {
    std::vector<QLeaf> tent;
    std::vector<uint8_t> is_parent;
    std::vector<double> rsum;
    std::unordered_map<uint64_t, int> pidx;
    for (size_t i = 0; i < m; ++i) {
      const QLeaf& f = t->leaves[i];
      if (dm[i]) {
        const uint64_t pk = parent_key(f);
        auto it = pidx.find(pk);
        if (it == pidx.end()) {
          const int32_t ps = t->size_of(f.level - 1);
          pidx.emplace(pk, (int)tent.size());
          tent.push_back({(int8_t)(f.level - 1), f.x / ps * ps, f.y / ps * ps});
          is_parent.push_back(1);
          rsum.push_back(rho[src[i]]);
        } else {
          rsum[it->second] += rho[src[i]];
        }
      } else {
        tent.push_back(f);
        is_parent.push_back(0);
        rsum.push_back(rho[src[i]]);
      }
    }
    auto idx = t->index(tent);
    std::vector<uint64_t> bad;
    for (const QLeaf& f : tent) {
      const int64_t s = t->size_of(f.level);
      for (const auto& d : kEdge) {
        const int c = t->find(idx, 2 * (f.x + d[0] * s) + s, 2 * (f.y + d[1] * s) + s);
        if (c >= 0 && is_parent[c] && tent[c].level < f.level - 1) bad.push_back(qkey(tent[c].level, tent[c].x, tent[c].y));
      }
    }
    if (bad.empty()) {
      std::vector<int> order(tent.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
      t->sort_leaves(tent, &order);
      t->leaves = tent;
      t->rho_new.resize(tent.size());
      for (size_t i = 0; i < tent.size(); ++i) {
        const int o = order[i];
        t->rho_new[i] = is_parent[o] ? rsum[o] / 4.0 : rsum[o];
      }
      break;
    }
    std::sort(bad.begin(), bad.end());
    bad.erase(std::unique(bad.begin(), bad.end()), bad.end());
    for (size_t i = 0; i < m; ++i)
      if (dm[i] && std::binary_search(bad.begin(), bad.end(), parent_key(t->leaves[i]))) dm[i] = 0;
  }
  t->old_mesh = std::move(t->mesh);
  t->has_old = !t->old_mesh.elem_nodes.empty();
  t->mesh = QMesh();
  *n_new = (int32_t)t->leaves.size();
  return AMRTO_OK;
}

int amrto_quadtree_adapt_result(const amrto_quadtree* t, double* rho_new) {
  if (!t || !rho_new) return AMRTO_EINVAL;
  if (t->rho_new.size() != t->leaves.size()) return AMRTO_ESTATE;
  std::memcpy(rho_new, t->rho_new.data(), t->rho_new.size() * sizeof(double));
  return AMRTO_OK;
}

int amrto_quadtree_build_mesh(amrto_quadtree* t, int32_t n_fixed, const amrto_region* fixed, int32_t load_x,
                              int32_t load_y, int32_t load_comp, double load_total) {
  if (!t || n_fixed < 0 || (n_fixed > 0 && !fixed) || load_comp < 0 || load_comp > 1) return AMRTO_EINVAL;
  QMesh md;
  const size_t ne = t->leaves.size();
  const int64_t SX = t->dims[0] + 1;
  auto lk = [&](int64_t x, int64_t y) { return (uint64_t)(x + SX * y); };
  // nodes: leaf corners, numbered lexicographically (x fastest)
  std::vector<uint64_t> keys;
  keys.reserve(4 * ne);
  for (const QLeaf& f : t->leaves) {
    const int32_t h = t->size_of(f.level);
    for (int a = 0; a < 4; ++a) keys.push_back(lk(f.x + h * (a & 1), f.y + h * (a >> 1)));
  }
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  for (size_t i = 0; i < keys.size(); ++i) {
    md.node_of.emplace(keys[i], (int)i);
    md.xy.push_back((int32_t)(keys[i] % SX));
    md.xy.push_back((int32_t)(keys[i] / SX));
  }
  const int nn = (int)keys.size();
  for (const QLeaf& f : t->leaves) {
    const int32_t h = t->size_of(f.level);
    for (int a = 0; a < 4; ++a) md.elem_nodes.push_back(md.node_of[lk(f.x + h * (a & 1), f.y + h * (a >> 1))]);
    md.level.push_back(f.level);
    md.anchor.push_back(f.x);
    md.anchor.push_back(f.y);
  }
  // hanging nodes: the midpoint of a leaf edge that is a node hangs on the
  // edge's end points (the leaf's bilinear functions there: 1/2, 1/2)
  std::unordered_map<int, std::vector<std::pair<int, double>>> hang;
  for (const QLeaf& f : t->leaves) {
    const int32_t h = t->size_of(f.level);
    if (h < 2) continue;
    const int32_t ex[4][4] = {{0, 0, 1, 0}, {0, 1, 1, 1}, {0, 0, 0, 1}, {1, 0, 1, 1}};  // edges (i0,j0,i1,j1)
    for (const auto& e : ex) {
      const int64_t x0 = f.x + h * e[0], y0 = f.y + h * e[1], x1 = f.x + h * e[2], y1 = f.y + h * e[3];
      auto it = md.node_of.find(lk((x0 + x1) / 2, (y0 + y1) / 2));
      if (it == md.node_of.end()) continue;
      hang[it->second] = {{md.node_of[lk(x0, y0)], 0.5}, {md.node_of[lk(x1, y1)], 0.5}};
    }
  }
  // resolve chains so that masters never hang
  bool changed = true;
  while (changed) {
    changed = false;
    for (auto& kv : hang) {
      std::vector<std::pair<int, double>> out;
      bool any = false;
      for (const auto& mw : kv.second) {
        auto it = hang.find(mw.first);
        if (it == hang.end()) {
          out.push_back(mw);
        } else {
          any = true;
          for (const auto& m2 : it->second) out.push_back({m2.first, mw.second * m2.second});
        }
      }
      if (any) {
        std::sort(out.begin(), out.end());
        std::vector<std::pair<int, double>> merged;
        for (const auto& p : out)
          if (!merged.empty() && merged.back().first == p.first) merged.back().second += p.second;
          else merged.push_back(p);
        kv.second = merged;
        changed = true;
      }
    }
  }
  std::vector<int> hn;
  for (const auto& kv : hang) hn.push_back(kv.first);
  std::sort(hn.begin(), hn.end());
  md.hang_ptr.push_back(0);
  for (int h : hn) {
    md.hang_node.push_back(h);
    for (const auto& mw : hang[h]) {
      md.hang_master.push_back(mw.first);
      md.hang_w.push_back(mw.second);
    }
    md.hang_ptr.push_back((int32_t)md.hang_master.size());
  }
  md.fixed.assign(2 * (size_t)nn, 0);
  for (int r = 0; r < n_fixed; ++r)
    for (int v = 0; v < nn; ++v) {
      bool on = true;
      for (int a = 0; a < 2; ++a)
        if (fixed[r].has[a] && md.xy[2 * v + a] != fixed[r].at[a]) on = false;
      if (on) md.fixed[2 * v] = md.fixed[2 * v + 1] = 1;
    }
  md.load.assign(2 * (size_t)nn, 0.0);
  auto it = md.node_of.find(lk(load_x, load_y));
  if (it == md.node_of.end() || hang.count(it->second)) return AMRTO_EINVAL;
  md.load[2 * it->second + load_comp] = load_total;
  t->mesh = std::move(md);
  return AMRTO_OK;
}

int amrto_quadtree_mesh_sizes(const amrto_quadtree* t, int32_t* n_nodes, int32_t* n_elems, int32_t* n_hang,
                              int32_t* n_hang_entries) {
  if (!t || t->mesh.elem_nodes.empty()) return AMRTO_ESTATE;
  if (n_nodes) *n_nodes = (int32_t)(t->mesh.xy.size() / 2);
  if (n_elems) *n_elems = (int32_t)t->mesh.level.size();
  if (n_hang) *n_hang = (int32_t)t->mesh.hang_node.size();
  if (n_hang_entries) *n_hang_entries = (int32_t)t->mesh.hang_master.size();
  return AMRTO_OK;
}

int amrto_quadtree_mesh_export(const amrto_quadtree* t, int32_t* node_xy, int32_t* elem_nodes, int8_t* elem_level,
                               int32_t* hang_node, int32_t* hang_ptr, int32_t* hang_master, double* hang_w,
                               uint8_t* dof_fixed, double* f_load) {
  if (!t || t->mesh.elem_nodes.empty()) return AMRTO_ESTATE;
  const QMesh& m = t->mesh;
  auto cp = [](auto* dst, const auto& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  cp(node_xy, m.xy);
  cp(elem_nodes, m.elem_nodes);
  cp(elem_level, m.level);
  cp(hang_node, m.hang_node);
  cp(hang_ptr, m.hang_ptr);
  cp(hang_master, m.hang_master);
  cp(hang_w, m.hang_w);
  cp(dof_fixed, m.fixed);
  cp(f_load, m.load);
  return AMRTO_OK;
}

int amrto_quadtree_transfer_nodal(const amrto_quadtree* t, const double* u_old, double* u_new) {
  if (!t || !u_old || !u_new) return AMRTO_EINVAL;
  if (!t->has_old || t->mesh.elem_nodes.empty()) return AMRTO_ESTATE;
  const QMesh& om = t->old_mesh;
  std::vector<QLeaf> old;
  for (size_t e = 0; e < om.level.size(); ++e) old.push_back({om.level[e], om.anchor[2 * e], om.anchor[2 * e + 1]});
  auto idx = t->index(old);
  const int nn = (int)(t->mesh.xy.size() / 2);
  for (int v = 0; v < nn; ++v) {
    const int64_t x = t->mesh.xy[2 * v], y = t->mesh.xy[2 * v + 1];
    // a point a quarter cell towards the interior lies in a leaf whose closed box holds the node
    const int64_t hx = 2 * x + (x >= t->dims[0] ? -1 : 1), hy = 2 * y + (y >= t->dims[1] ? -1 : 1);
    const int e = t->find(idx, hx, hy);
    if (e < 0) return AMRTO_EINVAL;
    const double h = t->size_of(old[e].level);
    const double xi = (x - old[e].x) / h, eta = (y - old[e].y) / h;
    const double w[4] = {(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta};
    for (int c = 0; c < 2; ++c) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a) s += w[a] * u_old[2 * om.elem_nodes[4 * e + a] + c];
      u_new[2 * v + c] = s;
    }
  }
  return AMRTO_OK;
}

}  // extern "C"
