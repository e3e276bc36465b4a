// Host driver for the library's octree, built with g++ together with the
// octree source under AddressSanitizer and UndefinedBehaviorSanitizer: random
// refinement, 2:1 closure, adaptations with random densities, mesh builds and
// nodal transfers, checking the structural invariants of each mesh.  Prints
// "ok" and exits 0 when every check passes.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "amrto.h"

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                   \
    }                                                                 \
  } while (0)

static void check_mesh(amrto_octree* t, const int32_t dims[3]) {
  int32_t nn = 0, ne = 0, nh = 0, nhe = 0;
  CHECK(amrto_octree_mesh_sizes(t, &nn, &ne, &nh, &nhe) == AMRTO_OK);
  CHECK(ne == amrto_octree_n_leaves(t));
  std::vector<int32_t> xyz(3L * nn), en(8L * ne), hn(nh), hp(nh + 1), hm(nhe);
  std::vector<int8_t> lv(ne);
  std::vector<double> hw(nhe), f(3L * nn);
  std::vector<uint8_t> fx(3L * nn);
  CHECK(amrto_octree_mesh_export(t, xyz.data(), en.data(), lv.data(), hn.data(), hp.data(), hm.data(), hw.data(),
                                 fx.data(), f.data()) == AMRTO_OK);
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < 3; ++a) CHECK(xyz[3 * i + a] >= 0 && xyz[3 * i + a] <= dims[a]);
  for (int32_t v : en) CHECK(v >= 0 && v < nn);
  CHECK(hp[0] == 0 && hp[nh] == nhe);
  std::vector<uint8_t> hanging(nn, 0);
  for (int32_t v : hn) {
    CHECK(v >= 0 && v < nn);
    hanging[v] = 1;
  }
  for (int h = 0; h < nh; ++h) {
    CHECK(hp[h + 1] > hp[h]);
    double sw = 0;
    for (int k = hp[h]; k < hp[h + 1]; ++k) {
      CHECK(hm[k] >= 0 && hm[k] < nn && !hanging[hm[k]]);
      CHECK(hw[k] > 0 && hw[k] <= 1);
      sw += hw[k];
    }
    CHECK(std::fabs(sw - 1.0) < 1e-12);
  }
  double total = 0;
  for (double v : f) total += v;
  CHECK(std::fabs(total + 1.0) < 1e-12);  // unit load, negative direction
}

int main() {
  const int32_t base[3] = {4, 2, 3};
  const int L = 3;
  amrto_octree* t = nullptr;
  CHECK(amrto_octree_create(&t, base, L) == AMRTO_OK);
  const int32_t dims[3] = {base[0] << L, base[1] << L, base[2] << L};
  amrto_region fixed{{1, 0, 0}, {0, 0, 0}};
  amrto_region load{{1, 0, 1}, {dims[0], 0, 0}};
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  // random refinement and closure
  for (int pass = 0; pass < 3; ++pass) {
    std::vector<uint8_t> marks(amrto_octree_n_leaves(t));
    for (auto& m : marks) m = U(rng) < 0.2;
    CHECK(amrto_octree_refine(t, marks.data()) == AMRTO_OK);
    CHECK(amrto_octree_balance(t) == AMRTO_OK);
  }
  CHECK(amrto_octree_build_mesh(t, 1, &fixed, &load, 0, 2, -1.0, 0) == AMRTO_OK);
  check_mesh(t, dims);
  // adaptations with random densities, each followed by a transfer
  for (int round = 0; round < 6; ++round) {
    int32_t nn_old = 0;
    CHECK(amrto_octree_mesh_sizes(t, &nn_old, nullptr, nullptr, nullptr) == AMRTO_OK);
    std::vector<double> u_old(3L * nn_old);
    for (auto& v : u_old) v = U(rng) - 0.5;
    std::vector<double> rho(amrto_octree_n_leaves(t));
    for (auto& v : rho) v = U(rng) < 0.3 ? 1.0 : 0.01 + 0.4 * U(rng);
    int32_t n_new = 0;
    CHECK(amrto_octree_adapt(t, rho.data(), 0.5, 1.5, &n_new) == AMRTO_OK);
    CHECK(n_new == amrto_octree_n_leaves(t));
    std::vector<double> rho_new(n_new);
    CHECK(amrto_octree_adapt_result(t, rho_new.data(), nullptr, nullptr) == AMRTO_OK);
    for (double v : rho_new) CHECK(v >= 0.01 && v <= 1.0);
    const amrto_region face{{0, 0, 1}, {0, 0, dims[2]}};
    const bool on_face = round & 1;
    CHECK(amrto_octree_build_mesh(t, 1, &fixed, on_face ? &face : &load, on_face ? 1 : 0, 2, -1.0, round == 5) ==
          AMRTO_OK);
    check_mesh(t, dims);
    int32_t nn = 0;
    CHECK(amrto_octree_mesh_sizes(t, &nn, nullptr, nullptr, nullptr) == AMRTO_OK);
    std::vector<double> u_new(3L * nn);
    CHECK(amrto_octree_transfer_nodal(t, u_old.data(), u_new.data()) == AMRTO_OK);
    for (double v : u_new) CHECK(std::isfinite(v) && std::fabs(v) <= 0.5);
  }
  // rejected arguments
  amrto_octree* bad = nullptr;
  const int32_t zero[3] = {0, 1, 1};
  CHECK(amrto_octree_create(&bad, zero, 2) == AMRTO_EINVAL && bad == nullptr);
  CHECK(amrto_octree_create(&bad, base, 13) == AMRTO_EINVAL);
  CHECK(amrto_octree_build_mesh(t, 1, &fixed, &load, 2, 2, -1.0, 0) == AMRTO_EINVAL);
  CHECK(amrto_octree_destroy(t) == AMRTO_OK);
  std::puts("ok");
  return 0;
}
