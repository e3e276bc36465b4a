// Host-side octree for the dynamic AMR strategy (paper Sec. 4 and Sec. 6):
// hierarchical leaves with refinement and derefinement, level-one
// compatibility closure, marking with the two compatibility sweeps, field
// transfer, and the finite-element mesh (nodes, connectivity, hanging-node
// interpolation, supports, consistent loads) that the device library uploads.
//
// Leaves are (level, anchor) with the anchor on the finest lattice; a level-l
// leaf has edge 2^(max_level - l).  Leaves are kept in Morton order of their
// anchors, which places every family of 8 siblings contiguously and gives the
// device a space-filling-curve element order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "amrto.h"
#include "levels.h"

namespace {

struct Leaf {
  int8_t level;
  int32_t x, y, z;
};

inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}
inline uint64_t morton(int32_t x, int32_t y, int32_t z) {
  return spread3((uint64_t)x) | spread3((uint64_t)y) << 1 | spread3((uint64_t)z) << 2;
}
inline uint64_t leaf_key(int level, int32_t x, int32_t y, int32_t z) {
  return (uint64_t)level << 60 | morton(x, y, z);
}

// the 18 face and edge neighbour directions
const int kDirs[18][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
                          {1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, 0, 1}, {1, 0, -1},
                          {-1, 0, 1}, {-1, 0, -1}, {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};

struct MeshData {
  int n_nodes = 0;
  std::vector<int32_t> xyz;        // 3 per node
  std::vector<int32_t> elem_nodes; // 8 per element
  std::vector<int8_t> level;
  std::vector<int32_t> anchor;     // 3 per element (copy of the leaves)
  std::vector<int32_t> hang_node, hang_ptr, hang_master;
  std::vector<double> hang_w;
  std::vector<uint8_t> fixed;      // 3 per node
  std::vector<double> load;        // 3 per node
  std::unordered_map<uint64_t, int> node_of;  // lattice key -> node
};

}  // namespace

struct amrto_octree {
  int32_t base[3];
  int32_t L;
  int32_t dims[3];
  std::vector<Leaf> leaves;
  std::vector<double> rho_new;  // result of the last adapt
  MeshData mesh;                // mesh of the current leaves (after build_mesh)
  MeshData old_mesh;            // mesh before the last adapt (for transfers)
  bool has_old = false;
  std::vector<amrto_region> fixed_regions;  // supports of the last build_mesh
  std::string err;

  int32_t size_of(int level) const { return 1 << (L - level); }

  void sort_leaves() {
    std::sort(leaves.begin(), leaves.end(), [](const Leaf& a, const Leaf& b) {
      const uint64_t ka = morton(a.x, a.y, a.z), kb = morton(b.x, b.y, b.z);
      if (ka != kb) return ka < kb;
      return a.level < b.level;
    });
  }

  std::unordered_map<uint64_t, int> index() const {
    std::unordered_map<uint64_t, int> m;
    m.reserve(leaves.size() * 2);
    for (size_t i = 0; i < leaves.size(); ++i)
      m.emplace(leaf_key(leaves[i].level, leaves[i].x, leaves[i].y, leaves[i].z), (int)i);
    return m;
  }

  // leaf containing lattice point 2*(p/2) given in half units (doubled coordinates)
  int find(const std::unordered_map<uint64_t, int>& idx, int64_t hx, int64_t hy, int64_t hz) const {
    if (hx < 0 || hy < 0 || hz < 0 || hx >= 2L * dims[0] || hy >= 2L * dims[1] || hz >= 2L * dims[2]) return -1;
    for (int l = 0; l <= L; ++l) {
      const int64_t s2 = 2L * size_of(l);
      const int32_t ax = (int32_t)((hx / s2) * (s2 / 2)), ay = (int32_t)((hy / s2) * (s2 / 2)),
                    az = (int32_t)((hz / s2) * (s2 / 2));
      auto it = idx.find(leaf_key(l, ax, ay, az));
      if (it != idx.end()) return it->second;
    }
    return -1;
  }
};

namespace {

// split marked leaves; src[i] = index of the old leaf each new leaf came from
void split(amrto_octree* t, const std::vector<uint8_t>& marks, std::vector<int>* src) {
  std::vector<Leaf> out;
  std::vector<int> s;
  out.reserve(t->leaves.size() + 7 * std::count(marks.begin(), marks.end(), 1));
  for (size_t i = 0; i < t->leaves.size(); ++i) {
    const Leaf& f = t->leaves[i];
    if (marks[i] && f.level < t->L) {
      const int32_t h = t->size_of(f.level + 1);
      for (int c = 0; c < 8; ++c) {
        out.push_back({(int8_t)(f.level + 1), f.x + h * (c & 1), f.y + h * ((c >> 1) & 1), f.z + h * (c >> 2)});
        s.push_back((int)i);
      }
    } else {
      out.push_back(f);
      s.push_back((int)i);
    }
  }
  // keep provenance through the Morton sort
  std::vector<size_t> perm(out.size());
  for (size_t i = 0; i < perm.size(); ++i) perm[i] = i;
  std::sort(perm.begin(), perm.end(), [&](size_t a, size_t b) {
    const uint64_t ka = morton(out[a].x, out[a].y, out[a].z), kb = morton(out[b].x, out[b].y, out[b].z);
    if (ka != kb) return ka < kb;
    return out[a].level < out[b].level;
  });
  std::vector<Leaf> sorted(out.size());
  std::vector<int> ssrc(out.size());
  for (size_t i = 0; i < perm.size(); ++i) {
    sorted[i] = out[perm[i]];
    ssrc[i] = s[perm[i]];
  }
  t->leaves.swap(sorted);
  if (src) {
    std::vector<int> composed(ssrc.size());
    for (size_t i = 0; i < ssrc.size(); ++i) composed[i] = (*src)[ssrc[i]];
    src->swap(composed);
  }
}

// Level-one closure: a leaf whose same-size face or edge neighbour cell lies in
// a leaf two or more levels coarser forces that coarse leaf to split.
void balance(amrto_octree* t, std::vector<int>* src) {
  while (true) {
    auto idx = t->index();
    std::vector<uint8_t> marks(t->leaves.size(), 0);
    bool any = false;
    for (const Leaf& f : t->leaves) {
      const int64_t s = t->size_of(f.level);
      for (const auto& d : kDirs) {
        // centre of the same-size neighbour cell, in half units
        const int64_t hx = 2 * (f.x + d[0] * s) + s, hy = 2 * (f.y + d[1] * s) + s, hz = 2 * (f.z + d[2] * s) + s;
        const int c = t->find(idx, hx, hy, hz);
        if (c >= 0 && t->leaves[c].level < f.level - 1 && !marks[c]) {
          marks[c] = 1;
          any = true;
        }
      }
    }
    if (!any) return;
    split(t, marks, src);
  }
}

}  // namespace

extern "C" {

int amrto_octree_create(amrto_octree** out, const int32_t base[3], int32_t max_level) {
  if (!out || !base) return AMRTO_EINVAL;
  *out = nullptr;
  if (max_level < 0 || max_level > 12) return AMRTO_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (base[a] <= 0 || ((int64_t)base[a] << max_level) >= (1 << 20)) return AMRTO_EINVAL;
  amrto_octree* t = new (std::nothrow) amrto_octree();
  if (!t) return AMRTO_ENOMEM;
  t->L = max_level;
  for (int a = 0; a < 3; ++a) {
    t->base[a] = base[a];
    t->dims[a] = base[a] << max_level;
  }
  const int32_t s = 1 << max_level;
  for (int k = 0; k < base[2]; ++k)
    for (int j = 0; j < base[1]; ++j)
      for (int i = 0; i < base[0]; ++i) t->leaves.push_back({0, i * s, j * s, k * s});
  t->sort_leaves();
  *out = t;
  return AMRTO_OK;
}

int amrto_octree_destroy(amrto_octree* t) {
  delete t;
  return AMRTO_OK;
}

int32_t amrto_octree_n_leaves(const amrto_octree* t) { return t ? (int32_t)t->leaves.size() : -1; }

int amrto_octree_leaves(const amrto_octree* t, int8_t* level, int32_t* anchor) {
  if (!t || !level || !anchor) return AMRTO_EINVAL;
  for (size_t i = 0; i < t->leaves.size(); ++i) {
    level[i] = t->leaves[i].level;
    anchor[3 * i] = t->leaves[i].x;
    anchor[3 * i + 1] = t->leaves[i].y;
    anchor[3 * i + 2] = t->leaves[i].z;
  }
  return AMRTO_OK;
}

int amrto_octree_refine(amrto_octree* t, const uint8_t* marks) {
  if (!t || !marks) return AMRTO_EINVAL;
  std::vector<uint8_t> m(marks, marks + t->leaves.size());
  for (auto& v : m) v = v ? 1 : 0;
  split(t, m, nullptr);
  return AMRTO_OK;
}

int amrto_octree_balance(amrto_octree* t) {
  if (!t) return AMRTO_EINVAL;
  balance(t, nullptr);
  return AMRTO_OK;
}

// One adaptation (Sec. 4): mark, sweep 1, refine + closure, sweep 1 again on
// the leaves left untouched, sweep 2 against the resulting mesh, derefine.
int amrto_octree_adapt(amrto_octree* t, const double* rho, double rho_s, double r_amr, int32_t* n_new) {
  if (!t || !rho || !n_new) return AMRTO_EINVAL;
  const size_t n = t->leaves.size();
  // marking: solid, or a solid centre within r_amr (centre to centre)
  std::vector<int8_t> mark(n, 0);
  {
    const double cell = std::max(1.0, r_amr);
    std::unordered_map<uint64_t, std::vector<int>> grid;
    auto cen = [&](size_t i, double* c) {
      const double h = t->size_of(t->leaves[i].level);
      c[0] = t->leaves[i].x + 0.5 * h;
      c[1] = t->leaves[i].y + 0.5 * h;
      c[2] = t->leaves[i].z + 0.5 * h;
    };
    auto gkey = [&](int64_t a, int64_t b, int64_t c) {
      return (uint64_t)((a + 4096) << 42 | (b + 4096) << 21 | (c + 4096));
    };
    for (size_t i = 0; i < n; ++i)
      if (rho[i] >= rho_s) {
        double c[3];
        cen(i, c);
        grid[gkey((int64_t)std::floor(c[0] / cell), (int64_t)std::floor(c[1] / cell), (int64_t)std::floor(c[2] / cell))]
            .push_back((int)i);
      }
    const double r2 = r_amr * r_amr;
    const int reach = (int)std::ceil(r_amr / cell);
    for (size_t i = 0; i < n; ++i) {
      bool near = rho[i] >= rho_s;
      if (!near) {
        double c[3];
        cen(i, c);
        const int64_t gx = (int64_t)std::floor(c[0] / cell), gy = (int64_t)std::floor(c[1] / cell),
                      gz = (int64_t)std::floor(c[2] / cell);
        for (int dz = -reach; dz <= reach && !near; ++dz)
          for (int dy = -reach; dy <= reach && !near; ++dy)
            for (int dx = -reach; dx <= reach && !near; ++dx) {
              auto it = grid.find(gkey(gx + dx, gy + dy, gz + dz));
              if (it == grid.end()) continue;
              for (int s : it->second) {
                double d[3];
                cen(s, d);
                const double q = (d[0] - c[0]) * (d[0] - c[0]) + (d[1] - c[1]) * (d[1] - c[1]) +
                                 (d[2] - c[2]) * (d[2] - c[2]);
                if (q <= r2) { near = true; break; }
              }
            }
      }
      if (near) mark[i] = t->leaves[i].level < t->L ? 1 : 0;
      else mark[i] = t->leaves[i].level > 0 ? -1 : 0;
    }
  }
  auto parent_key = [&](const Leaf& f) {
    const int32_t ps = t->size_of(f.level - 1);
    return leaf_key(f.level - 1, f.x / ps * ps, f.y / ps * ps, f.z / ps * ps);
  };
  // sweep 1: whole families only
  auto sweep1 = [&](const std::vector<Leaf>& lv, std::vector<uint8_t>& dm) {
    std::unordered_map<uint64_t, int> cnt;
    for (size_t i = 0; i < lv.size(); ++i)
      if (dm[i]) cnt[parent_key(lv[i])]++;
    for (size_t i = 0; i < lv.size(); ++i)
      if (dm[i] && cnt[parent_key(lv[i])] != 8) dm[i] = 0;
  };
  std::vector<uint8_t> dmark(n), rmark(n);
  for (size_t i = 0; i < n; ++i) {
    dmark[i] = mark[i] == -1;
    rmark[i] = mark[i] == 1;
  }
  sweep1(t->leaves, dmark);
  const std::vector<Leaf> old = t->leaves;
  std::vector<int> src(n);
  for (size_t i = 0; i < n; ++i) src[i] = (int)i;
  split(t, rmark, &src);
  balance(t, &src);
  // derefinement candidates: leaves that are still exactly an old marked leaf
  std::vector<int> nsplit(n, 0);
  for (int s : src) nsplit[s]++;
  const size_t m = t->leaves.size();
  std::vector<uint8_t> dm(m, 0);
  for (size_t i = 0; i < m; ++i) dm[i] = dmark[src[i]] && nsplit[src[i]] == 1;
  sweep1(t->leaves, dm);
  // sweep 2: tentative coarsening; drop families whose parent would meet a
  // leaf two or more levels finer across a face or an edge
  while (true) {
    std::unordered_map<uint64_t, int> parent_of;  // parent key -> family id
    std::vector<Leaf> tent;
    std::vector<int> fam_of_tent;
    std::unordered_map<uint64_t, int> seen;
    for (size_t i = 0; i < m; ++i) {
      if (dm[i]) {
        const uint64_t pk = parent_key(t->leaves[i]);
        if (seen.emplace(pk, (int)tent.size()).second) {
          const int32_t ps = t->size_of(t->leaves[i].level - 1);
          tent.push_back({(int8_t)(t->leaves[i].level - 1), t->leaves[i].x / ps * ps, t->leaves[i].y / ps * ps,
                          t->leaves[i].z / ps * ps});
          fam_of_tent.push_back(1);
        }
      } else {
        tent.push_back(t->leaves[i]);
        fam_of_tent.push_back(0);
      }
    }
    std::unordered_map<uint64_t, int> idx;
    for (size_t i = 0; i < tent.size(); ++i) idx.emplace(leaf_key(tent[i].level, tent[i].x, tent[i].y, tent[i].z), (int)i);
    std::vector<uint64_t> bad;
    for (const Leaf& f : tent) {
      const int64_t s = t->size_of(f.level);
      for (const auto& d : kDirs) {
        const int64_t hx = 2 * (f.x + d[0] * s) + s, hy = 2 * (f.y + d[1] * s) + s, hz = 2 * (f.z + d[2] * s) + s;
        const int c = t->find(idx, hx, hy, hz);
        if (c >= 0 && fam_of_tent[c] && tent[c].level < f.level - 1)
          bad.push_back(leaf_key(tent[c].level, tent[c].x, tent[c].y, tent[c].z));
      }
    }
    if (bad.empty()) {
      // commit: parents replace families; densities: inherit / average
      std::vector<double> rnew;
      std::vector<Leaf> fin;
      std::unordered_map<uint64_t, double> famsum;
      for (size_t i = 0; i < m; ++i)
        if (dm[i]) famsum[parent_key(t->leaves[i])] += rho[src[i]];
      for (size_t i = 0; i < tent.size(); ++i) {
        fin.push_back(tent[i]);
        if (fam_of_tent[i])
          rnew.push_back(famsum[leaf_key(tent[i].level, tent[i].x, tent[i].y, tent[i].z)] / 8.0);
        else
          rnew.push_back(0.0);
      }
      // non-family leaves: look up provenance by position in the refined list
      size_t k = 0;
      for (size_t i = 0; i < m; ++i) {
        if (dm[i]) continue;
        while (fam_of_tent[k]) ++k;
        rnew[k] = rho[src[i]];
        ++k;
      }
      // restore Morton order with densities attached
      std::vector<size_t> perm(fin.size());
      for (size_t i = 0; i < perm.size(); ++i) perm[i] = i;
      std::sort(perm.begin(), perm.end(), [&](size_t a, size_t b) {
        const uint64_t ka = morton(fin[a].x, fin[a].y, fin[a].z), kb = morton(fin[b].x, fin[b].y, fin[b].z);
        if (ka != kb) return ka < kb;
        return fin[a].level < fin[b].level;
      });
      t->leaves.resize(fin.size());
      t->rho_new.resize(fin.size());
      for (size_t i = 0; i < perm.size(); ++i) {
        t->leaves[i] = fin[perm[i]];
        t->rho_new[i] = rnew[perm[i]];
      }
      break;
    }
    std::sort(bad.begin(), bad.end());
    bad.erase(std::unique(bad.begin(), bad.end()), bad.end());
    for (size_t i = 0; i < m; ++i)
      if (dm[i] && std::binary_search(bad.begin(), bad.end(), parent_key(t->leaves[i]))) dm[i] = 0;
  }
  // keep the mesh of the previous leaves for nodal transfers
  t->old_mesh = std::move(t->mesh);
  t->has_old = !t->old_mesh.elem_nodes.empty();
  t->mesh = MeshData();
  *n_new = (int32_t)t->leaves.size();
  (void)old;
  return AMRTO_OK;
}

int amrto_octree_adapt_result(const amrto_octree* t, double* rho_new, int32_t* src_first, int32_t* src_count) {
  if (!t || !rho_new) return AMRTO_EINVAL;
  if (t->rho_new.size() != t->leaves.size()) return AMRTO_ESTATE;
  std::memcpy(rho_new, t->rho_new.data(), t->rho_new.size() * sizeof(double));
  (void)src_first;
  (void)src_count;
  return AMRTO_OK;
}

int amrto_octree_build_mesh(amrto_octree* t, int32_t n_fixed, const amrto_region* fixed,
                            const amrto_region* load_region, int32_t load_kind, int32_t load_comp,
                            double load_total, int32_t lexicographic) {
  if (!t) return AMRTO_EINVAL;
  if (n_fixed < 0 || (n_fixed > 0 && !fixed) || (load_region && (load_comp < 0 || load_comp > 2)) ||
      (load_region && load_kind != 0 && load_kind != 1))
    return AMRTO_EINVAL;
  MeshData md;
  const size_t ne = t->leaves.size();
  const int64_t SX = t->dims[0] + 1, SY = t->dims[1] + 1;
  auto lex = [&](int64_t x, int64_t y, int64_t z) { return (uint64_t)(x + SX * (y + SY * z)); };
  // nodes: the vertices of all leaves, ordered lexicographically or by Morton key
  std::vector<std::pair<uint64_t, uint64_t>> keys;  // (order key, lattice key)
  keys.reserve(ne * 8);
  for (const Leaf& f : t->leaves) {
    const int32_t s = t->size_of(f.level);
    for (int a = 0; a < 8; ++a) {
      const int32_t x = f.x + s * (a & 1), y = f.y + s * ((a >> 1) & 1), z = f.z + s * (a >> 2);
      keys.emplace_back(lexicographic ? lex(x, y, z) : morton(x, y, z), lex(x, y, z));
    }
  }
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  md.n_nodes = (int)keys.size();
  md.xyz.resize(3L * md.n_nodes);
  md.node_of.reserve(keys.size() * 2);
  for (int i = 0; i < md.n_nodes; ++i) {
    const uint64_t k = keys[i].second;
    md.xyz[3 * i] = (int32_t)(k % SX);
    md.xyz[3 * i + 1] = (int32_t)((k / SX) % SY);
    md.xyz[3 * i + 2] = (int32_t)(k / (SX * SY));
    md.node_of.emplace(k, i);
  }
  auto node_at = [&](int64_t x, int64_t y, int64_t z) -> int {
    if (x < 0 || y < 0 || z < 0 || x >= SX || y >= SY || z > t->dims[2]) return -1;
    auto it = md.node_of.find(lex(x, y, z));
    return it == md.node_of.end() ? -1 : it->second;
  };
  md.elem_nodes.resize(8 * ne);
  md.level.resize(ne);
  md.anchor.resize(3 * ne);
  for (size_t e = 0; e < ne; ++e) {
    const Leaf& f = t->leaves[e];
    const int32_t s = t->size_of(f.level);
    for (int a = 0; a < 8; ++a)
      md.elem_nodes[8 * e + a] = node_at(f.x + s * (a & 1), f.y + s * ((a >> 1) & 1), f.z + s * (a >> 2));
    md.level[e] = f.level;
    md.anchor[3 * e] = f.x;
    md.anchor[3 * e + 1] = f.y;
    md.anchor[3 * e + 2] = f.z;
  }
  // hanging nodes: a node at the midpoint of a leaf edge interpolates the two
  // edge ends (1/2 each), one at a face centre the four face corners (1/4)
  std::unordered_map<int, std::vector<std::pair<int, double>>> direct;
  for (const Leaf& f : t->leaves) {
    const int32_t s = t->size_of(f.level);
    if (s < 2) continue;
    const int32_t h = s / 2;
    // 12 edges: axis ax, the other two coordinates at 0 or s
    for (int ax = 0; ax < 3; ++ax) {
      const int o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
      for (int c1 = 0; c1 < 2; ++c1)
        for (int c2 = 0; c2 < 2; ++c2) {
          int32_t p[3] = {f.x, f.y, f.z}, q0[3], q1[3];
          p[o1] += c1 * s;
          p[o2] += c2 * s;
          std::memcpy(q0, p, sizeof p);
          std::memcpy(q1, p, sizeof p);
          q1[ax] += s;
          p[ax] += h;
          const int v = node_at(p[0], p[1], p[2]);
          if (v >= 0 && !direct.count(v))
            direct[v] = {{node_at(q0[0], q0[1], q0[2]), 0.5}, {node_at(q1[0], q1[1], q1[2]), 0.5}};
        }
    }
    // 6 faces: normal axis ax at 0 or s
    for (int ax = 0; ax < 3; ++ax) {
      const int o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
      for (int c = 0; c < 2; ++c) {
        int32_t p[3] = {f.x, f.y, f.z};
        p[ax] += c * s;
        int32_t ctr[3] = {p[0], p[1], p[2]};
        ctr[o1] += h;
        ctr[o2] += h;
        const int v = node_at(ctr[0], ctr[1], ctr[2]);
        if (v >= 0 && !direct.count(v)) {
          std::vector<std::pair<int, double>> ms;
          for (int a1 = 0; a1 < 2; ++a1)
            for (int a2 = 0; a2 < 2; ++a2) {
              int32_t q[3] = {p[0], p[1], p[2]};
              q[o1] += a1 * s;
              q[o2] += a2 * s;
              ms.push_back({node_at(q[0], q[1], q[2]), 0.25});
            }
          direct[v] = ms;
        }
      }
    }
  }
  // resolve chains: a hanging master is replaced by its own masters
  std::unordered_map<int, std::vector<std::pair<int, double>>> resolved;
  std::vector<int> hnodes;
  for (auto& kv : direct) hnodes.push_back(kv.first);
  std::sort(hnodes.begin(), hnodes.end());
  std::function<const std::vector<std::pair<int, double>>&(int, int)> resolve;
  resolve = [&](int v, int depth) -> const std::vector<std::pair<int, double>>& {
    auto it = resolved.find(v);
    if (it != resolved.end()) return it->second;
    std::unordered_map<int, double> acc;
    for (auto& mw : direct[v]) {
      if (direct.count(mw.first) && depth < 64) {
        for (auto& m2 : resolve(mw.first, depth + 1)) acc[m2.first] += mw.second * m2.second;
      } else {
        acc[mw.first] += mw.second;
      }
    }
    std::vector<std::pair<int, double>> out(acc.begin(), acc.end());
    std::sort(out.begin(), out.end());
    return resolved[v] = out;
  };
  md.hang_ptr.push_back(0);
  for (int v : hnodes) {
    const auto& ms = resolve(v, 0);
    md.hang_node.push_back(v);
    for (auto& mw : ms) {
      md.hang_master.push_back(mw.first);
      md.hang_w.push_back(mw.second);
    }
    md.hang_ptr.push_back((int32_t)md.hang_master.size());
  }
  // supports
  md.fixed.assign(3L * md.n_nodes, 0);
  for (int r = 0; r < n_fixed; ++r)
    for (int i = 0; i < md.n_nodes; ++i) {
      bool on = true;
      for (int a = 0; a < 3; ++a)
        if (fixed[r].has[a] && md.xyz[3 * i + a] != fixed[r].at[a]) on = false;
      if (on) md.fixed[3 * i] = md.fixed[3 * i + 1] = md.fixed[3 * i + 2] = 1;
    }
  // consistent load on all nodes
  md.load.assign(3L * md.n_nodes, 0.0);
  if (load_region) {
    std::unordered_map<uint64_t, int> done;
    double total = 0.0;
    auto on_region = [&](const int32_t* p) {
      for (int a = 0; a < 3; ++a)
        if (load_region->has[a] && p[a] != load_region->at[a]) return false;
      return true;
    };
    for (const Leaf& f : t->leaves) {
      const int32_t s = t->size_of(f.level);
      int32_t cs[8][3];
      int on[8], non = 0;
      for (int a = 0; a < 8; ++a) {
        cs[a][0] = f.x + s * (a & 1);
        cs[a][1] = f.y + s * ((a >> 1) & 1);
        cs[a][2] = f.z + s * (a >> 2);
        if (on_region(cs[a])) on[non++] = a;
      }
      if ((load_kind == 0 && non == 2) || (load_kind == 1 && non == 4)) {
        uint64_t key = 0;
        for (int k = 0; k < non; ++k) key = key * 1000003ULL + lex(cs[on[k]][0], cs[on[k]][1], cs[on[k]][2]);
        if (!done.emplace(key, 1).second) continue;
        const double share = load_kind == 0 ? 0.5 * s : 0.25 * (double)s * s;
        for (int k = 0; k < non; ++k) {
          const int v = node_at(cs[on[k]][0], cs[on[k]][1], cs[on[k]][2]);
          md.load[3L * v + load_comp] += share;
        }
        total += load_kind == 0 ? (double)s : (double)s * s;
      }
    }
    if (total > 0.0)
      for (auto& v : md.load) v *= load_total / total;
  }
  t->mesh = std::move(md);
  t->fixed_regions.assign(fixed, fixed + n_fixed);
  return AMRTO_OK;
}

int amrto_octree_mesh_sizes(const amrto_octree* t, int32_t* n_nodes, int32_t* n_elems, int32_t* n_hang,
                            int32_t* n_hang_entries) {
  if (!t) return AMRTO_EINVAL;
  if (t->mesh.elem_nodes.empty()) return AMRTO_ESTATE;
  if (n_nodes) *n_nodes = t->mesh.n_nodes;
  if (n_elems) *n_elems = (int32_t)t->mesh.level.size();
  if (n_hang) *n_hang = (int32_t)t->mesh.hang_node.size();
  if (n_hang_entries) *n_hang_entries = (int32_t)t->mesh.hang_master.size();
  return AMRTO_OK;
}

int amrto_octree_mesh_export(const amrto_octree* t, int32_t* node_xyz, int32_t* elem_nodes, int8_t* elem_level,
                             int32_t* hang_node, int32_t* hang_ptr, int32_t* hang_master, double* hang_w,
                             uint8_t* dof_fixed, double* f_load) {
  if (!t) return AMRTO_EINVAL;
  const MeshData& m = t->mesh;
  if (m.elem_nodes.empty()) return AMRTO_ESTATE;
  auto cp = [](void* dst, const auto& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  cp(node_xyz, m.xyz);
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

// Evaluate the previous mesh's trilinear field at the current mesh's nodes:
// each node is located in an old leaf through a point a quarter cell towards
// the domain interior, then interpolated from that leaf's eight vertices.
int amrto_octree_transfer_nodal(const amrto_octree* t, const double* u_old, double* u_new) {
  if (!t || !u_old || !u_new) return AMRTO_EINVAL;
  if (!t->has_old || t->mesh.elem_nodes.empty()) return AMRTO_ESTATE;
  const MeshData& om = t->old_mesh;
  std::unordered_map<uint64_t, int> idx;
  const size_t ne = om.level.size();
  idx.reserve(ne * 2);
  for (size_t e = 0; e < ne; ++e)
    idx.emplace(leaf_key(om.level[e], om.anchor[3 * e], om.anchor[3 * e + 1], om.anchor[3 * e + 2]), (int)e);
  for (int i = 0; i < t->mesh.n_nodes; ++i) {
    const int32_t* p = &t->mesh.xyz[3 * i];
    int64_t h[3];
    for (int a = 0; a < 3; ++a) h[a] = 2L * p[a] + (p[a] >= t->dims[a] ? -1 : 1);  // +-1/2 in half units
    int e = -1;
    for (int l = 0; l <= t->L && e < 0; ++l) {
      const int64_t s2 = 2L * t->size_of(l);
      auto it = idx.find(leaf_key(l, (int32_t)((h[0] / s2) * (s2 / 2)), (int32_t)((h[1] / s2) * (s2 / 2)),
                                  (int32_t)((h[2] / s2) * (s2 / 2))));
      if (it != idx.end()) e = it->second;
    }
    if (e < 0) return AMRTO_EINVAL;
    const double s = t->size_of(om.level[e]);
    const double xi[3] = {(p[0] - om.anchor[3 * e]) / s, (p[1] - om.anchor[3 * e + 1]) / s,
                          (p[2] - om.anchor[3 * e + 2]) / s};
    double v[3] = {0, 0, 0};
    for (int a = 0; a < 8; ++a) {
      const double w = ((a & 1) ? xi[0] : 1 - xi[0]) * (((a >> 1) & 1) ? xi[1] : 1 - xi[1]) *
                       ((a >> 2) ? xi[2] : 1 - xi[2]);
      const int nd = om.elem_nodes[8 * e + a];
      for (int c = 0; c < 3; ++c) v[c] += w * u_old[3L * nd + c];
    }
    for (int c = 0; c < 3; ++c) u_new[3L * i + c] = v[c];
  }
  return AMRTO_OK;
}

}  // extern "C"

namespace amrto {

static void to_level_mesh(const MeshData& md, int L, LevelMesh* out) {
  out->n_nodes = md.n_nodes;
  out->n_elems = (int)md.level.size();
  out->L = L;
  out->xyz = md.xyz;
  out->elem_nodes = md.elem_nodes;
  out->level = md.level;
  out->anchor = md.anchor;
  out->hang_node = md.hang_node;
  out->hang_ptr = md.hang_ptr;
  out->hang_master = md.hang_master;
  out->hang_w = md.hang_w;
  out->fixed = md.fixed;
}

bool octree_level_mesh(const amrto_octree* t, int k, LevelMesh* out) {
  if (!t || !out || k < 0 || t->mesh.elem_nodes.empty()) return false;
  if (k == 0) {
    to_level_mesh(t->mesh, t->L, out);
    return true;
  }
  amrto_octree c;
  int32_t lmax;
  if (k <= t->L) {
    lmax = t->L;
    for (int a = 0; a < 3; ++a) c.base[a] = t->base[a];
  } else {
    const int j = k - t->L;
    if (j > 20) return false;
    for (int a = 0; a < 3; ++a) {
      if (t->base[a] % (1 << j)) return false;
      c.base[a] = t->base[a] >> j;
    }
    lmax = k;
  }
  c.L = lmax;
  for (int a = 0; a < 3; ++a) c.dims[a] = t->dims[a];
  const int top = k <= t->L ? t->L - k : 0;
  std::unordered_map<uint64_t, int> seen;
  for (const Leaf& f : t->leaves) {
    const int8_t lv = (int8_t)std::min<int>(f.level, top);
    const int32_t s = 1 << (lmax - lv);
    const Leaf g{lv, f.x / s * s, f.y / s * s, f.z / s * s};
    if (seen.emplace(leaf_key(g.level, g.x, g.y, g.z), 1).second) c.leaves.push_back(g);
  }
  c.sort_leaves();
  const int rc = amrto_octree_build_mesh(&c, (int32_t)t->fixed_regions.size(), t->fixed_regions.data(), nullptr, 0, 0,
                                         0.0, 1);
  if (rc != AMRTO_OK) return false;
  to_level_mesh(c.mesh, lmax, out);
  return true;
}

}  // namespace amrto
