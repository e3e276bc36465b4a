// Context, material, mesh upload and the small host helpers of the amrto
// library.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace amrto {

// Unit-cube Q1 element matrix from the index form of linear elasticity,
//   K[(a,c),(b,d)] = int lam dN_a/dx_c dN_b/dx_d + mu dN_a/dx_d dN_b/dx_c
//                    + mu delta_cd grad N_a . grad N_b,
// where each integral of trilinear shape-function products factorises into
// exact one-dimensional integrals (trilinear displacements: paper Sec. 3).
void k0_unit_cube(double nu, double* K) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  auto one_d = [](int ia, int ib, bool da, bool db) -> double {
    if (da && db) return ia == ib ? 1.0 : -1.0;
    if (da) return ia ? 0.5 : -0.5;
    if (db) return ib ? 0.5 : -0.5;
    return ia == ib ? 1.0 / 3.0 : 1.0 / 6.0;
  };
  auto g = [&](int a, int b, int p, int q) {
    double v = 1.0;
    for (int ax = 0; ax < 3; ++ax)
      v *= one_d((a >> ax) & 1, (b >> ax) & 1, ax == p, ax == q);
    return v;
  };
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
          double v = lam * g(a, b, c, d) + mu * g(a, b, d, c);
          if (c == d) v += mu * (g(a, b, 0, 0) + g(a, b, 1, 1) + g(a, b, 2, 2));
          K[(3 * a + c) * 24 + 3 * b + d] = v;
        }
}

uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

int grid_for(long n, int threads, int cap) {
  long g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace amrto

using namespace amrto;

template <typename T>
static void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

template <typename T>
static hipError_t dalloc(T*& p, size_t n) {
  dfree(p);
  if (n == 0) n = 1;
  return hipMalloc((void**)&p, n * sizeof(T));
}

static void free_mesh(amrto_ctx* c) {
  mg_free(c);
  dfree(c->d_fix); dfree(c->d_level); dfree(c->d_elem_nodes);
  dfree(c->d_chunk_cnt); dfree(c->d_ent_elem); dfree(c->d_ent_loc);
  dfree(c->d_tab_node); dfree(c->d_trip_hm); dfree(c->d_trip_w); dfree(c->d_tab_hbeg);
  dfree(c->d_hang_node); dfree(c->d_hang_ptr); dfree(c->d_hang_master); dfree(c->d_hang_w);
  dfree(c->d_mt_node); dfree(c->d_mt_ptr); dfree(c->d_mt_h); dfree(c->d_mt_w);
  c->n_mt = 0;
  dfree(c->d_edesc); dfree(c->d_cmap);
  dfree(c->d_rec_store); dfree(c->d_rec_coef); dfree(c->d_rec_C); dfree(c->d_rr_aw); dfree(c->d_rr_part);
  c->rec_m = 0;
  c->rec_active = false;
  dfree(c->d_coef); dfree(c->d_coef_f); dfree(c->d_dinv); dfree(c->d_dinv_f); dfree(c->d_vol);
  dfree(c->d_r); dfree(c->d_z); dfree(c->d_p); dfree(c->d_q); dfree(c->d_p2); dfree(c->f_p2);
  dfree(c->d_partpq);
  dfree(c->d_cg1_r2); dfree(c->d_cg1_w); dfree(c->d_cg1_w2); dfree(c->d_cg1_s); dfree(c->d_cg1_s2);
  dfree(c->d_cg1_part);
  dfree(c->d_binv); dfree(c->d_binv_f);
  c->binv_valid = false;
  c->n_partpq = 0;
  dfree(c->f_b); dfree(c->f_x); dfree(c->f_r); dfree(c->f_z); dfree(c->f_p); dfree(c->f_q);
  dfree(c->d_cf); dfree(c->d_region); dfree(c->d_cpart); dfree(c->d_cinv); dfree(c->d_cz); dfree(c->d_ct);
  dfree(c->d_cqpart); c->cq_cap = 0;
  dfree(c->d_gram_mask); c->gram_mask_cap = 0; dfree(c->d_gram); c->gram_cap = 0; dfree(c->d_cmask); dfree(c->d_cgeo);
  dfree(c->d_node_xyz); dfree(c->d_cell_ptr); dfree(c->d_cell_elem); dfree(c->d_cell_w);
  dfree(c->d_gn_node); dfree(c->d_gn_w);
  c->coarse_k = 0;
  c->coarse_cap = 0;
  c->grid_cell = 0;
  c->has_mesh = false;
  c->has_density = false;
}

static int upload_material(amrto_ctx* ctx) {
  k0_unit_cube(ctx->nu, ctx->K0);
  float kf[576];
  uint16_t kb[1152];
  for (int i = 0; i < 576; ++i) {
    kf[i] = (float)ctx->K0[i];
    uint16_t hi = f32_to_bf16_rne(kf[i]);
    float rem = (float)(ctx->K0[i] - (double)bf16_to_f32(hi));
    kb[i] = hi;
    kb[576 + i] = f32_to_bf16_rne(rem);
  }
  AMRTO_HIP(hipMemcpyAsync(ctx->d_K0, ctx->K0, sizeof(ctx->K0), hipMemcpyHostToDevice, ctx->stream));
  AMRTO_HIP(hipMemcpyAsync(ctx->d_K0f, kf, sizeof(kf), hipMemcpyHostToDevice, ctx->stream));
  AMRTO_HIP(hipMemcpyAsync(ctx->d_K0bf, kb, sizeof(kb), hipMemcpyHostToDevice, ctx->stream));
  // K0 in the basis of per-component Walsh-Hadamard modes W (W W^T = 8 I):
  // B = W K0 W^T / 64 is block diagonal; block S couples the modes
  // (c, t = S ^ (1 << c)), c = 0, 1, 2, so K0 = W^T B W.
  double kbd[72];
  auto wsign = [](int t, int n) { return (__builtin_popcount(t & n) & 1) ? -1.0 : 1.0; };
  for (int S = 0; S < 8; ++S)
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d) {
        const int t = S ^ (1 << c), tp = S ^ (1 << d);
        double v = 0.0;
        for (int n = 0; n < 8; ++n)
          for (int m = 0; m < 8; ++m) v += wsign(t, n) * ctx->K0[(3 * n + c) * 24 + 3 * m + d] * wsign(tp, m);
        kbd[9 * S + 3 * c + d] = v / 64.0;
      }
  // For a cube of an isotropic material the blocks have a fixed pattern
  // (zero modes, equal entries) with eight distinct values:
  //   B0 = [[a b b][b a b][b b a]]  B7 = [[h i i][i h i][i i h]]
  //   B1 = [[0 0 0][0 d e][0 e d]]  B2 = [[d 0 e][0 0 0][e 0 d]]  B4 = [[d e 0][e d 0][0 0 0]]
  //   B3 = [[f f 0][f f 0][0 0 g]]  B5 = [[f 0 f][0 g 0][f 0 f]]  B6 = [[g 0 0][0 f f][0 f f]]
  {
    const double a = kbd[0], b = kbd[1], d = kbd[9 + 4], e = kbd[9 + 5], f = kbd[27], g = kbd[27 + 8],
                 h = kbd[63], i = kbd[64];
    const double pat[8][9] = {{a, b, b, b, a, b, b, b, a}, {0, 0, 0, 0, d, e, 0, e, d}, {d, 0, e, 0, 0, 0, e, 0, d},
                              {f, f, 0, f, f, 0, 0, 0, g}, {d, e, 0, e, d, 0, 0, 0, 0}, {f, 0, f, 0, g, 0, f, 0, f},
                              {g, 0, 0, 0, f, f, 0, f, f}, {h, i, i, i, h, i, i, i, h}};
    double big = 0.0, dev = 0.0;
    for (int k = 0; k < 72; ++k) big = std::max(big, std::fabs(kbd[k]));
    for (int k = 0; k < 72; ++k) dev = std::max(dev, std::fabs(kbd[k] - pat[k / 9][k % 9]));
    if (!(dev <= 1e-12 * big)) return ctx->fail(AMRTO_EINVAL, "element matrix lost its cube symmetry (material constants?)");
    const double bk[8] = {a - b, b, d, e, f, g, h - i, i};
    std::memcpy(ctx->bk, bk, sizeof bk);
  }
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  return AMRTO_OK;
}

extern "C" {

int amrto_create(amrto_ctx** out, int device, void* stream) {
  if (!out) return AMRTO_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return AMRTO_EINVAL;
  amrto_ctx* ctx = new (std::nothrow) amrto_ctx();
  if (!ctx) return AMRTO_ENOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess) { delete ctx; return AMRTO_EHIP; }
  if (hipMalloc((void**)&ctx->d_K0, 576 * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&ctx->d_K0f, 576 * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&ctx->d_K0bf, 1152 * sizeof(uint16_t)) != hipSuccess ||
      hipMalloc((void**)&ctx->d_part, 8 * RED_BLOCKS * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&ctx->d_scal, S_COUNT * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&ctx->d_oc, OC_WS * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&ctx->h_scal, S_COUNT * sizeof(double)) != hipSuccess) {
    amrto_destroy(ctx);
    return AMRTO_ENOMEM;
  }
  int rc = oc_scratch_attach(ctx);
  if (rc == AMRTO_OK) rc = upload_material(ctx);
  if (rc != AMRTO_OK) { amrto_destroy(ctx); return rc; }
  *out = ctx;
  return AMRTO_OK;
}

int amrto_destroy(amrto_ctx* ctx) {
  if (!ctx) return AMRTO_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  free_mesh(ctx);
  dfree(ctx->d_K0); dfree(ctx->d_K0f); dfree(ctx->d_K0bf);
  dfree(ctx->d_part); dfree(ctx->d_scal); dfree(ctx->d_oc);
  if (ctx->h_scal) (void)hipHostFree(ctx->h_scal);
  delete ctx;
  return AMRTO_OK;
}

const char* amrto_last_error(const amrto_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

int amrto_set_stream(amrto_ctx* ctx, void* stream) {
  if (!ctx) return AMRTO_EINVAL;
  ctx->stream = (hipStream_t)stream;
  return AMRTO_OK;
}

int amrto_set_material(amrto_ctx* ctx, double E0, double Emin, double nu, double p) {
  if (!ctx) return AMRTO_EINVAL;
  if (!(E0 > Emin) || !(Emin >= 0.0) || !(nu > -1.0 && nu < 0.5) || !(p >= 1.0))
    return ctx->fail(AMRTO_EINVAL, "amrto_set_material: need E0 > Emin >= 0, -1 < nu < 0.5, p >= 1");
  AMRTO_HIP(hipSetDevice(ctx->device));
  ctx->E0 = E0; ctx->Emin = Emin; ctx->nu = nu; ctx->p = p;
  ctx->has_density = false;
  ctx->mg_valid = false;
  return upload_material(ctx);
}

int amrto_set_deterministic(amrto_ctx* ctx, int32_t on) {
  if (!ctx) return AMRTO_EINVAL;
  const bool det = on != 0;
  if (det == ctx->deterministic) return AMRTO_OK;
  AMRTO_HIP(hipSetDevice(ctx->device));
  ctx->deterministic = det;
  // what the density determines is formed again in the new mode: the
  // diagonal now, the node-block inverses and multigrid operators when next
  // used (a coarse space keeps its Gram matrix until it is set up again)
  ctx->binv_valid = false;
  ctx->mg_valid = false;
  return ctx->has_density ? launch_diag(ctx) : AMRTO_OK;
}

int amrto_upload_mesh(amrto_ctx* ctx, const amrto_mesh* m) {
  if (!ctx) return AMRTO_EINVAL;
  if (!m || m->n_nodes <= 0 || m->n_elems <= 0 || !m->dof_fixed)
    return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: empty mesh or missing dof_fixed");
  // kernels index DOFs with 32-bit per-lane offsets
  if (3L * m->n_nodes > 2147483647L || 8L * m->n_elems > 2147483647L)
    return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: mesh too large (3 n_nodes and 8 n_elems must be < 2^31)");
  AMRTO_HIP(hipSetDevice(ctx->device));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  free_mesh(ctx);
  const bool uni = (m->elem_nodes == nullptr);
  if (uni) {
    long nx = m->dims[0], ny = m->dims[1], nz = m->dims[2];
    if (nx <= 0 || ny <= 0 || nz <= 0 || nx * ny * nz != m->n_elems ||
        (nx + 1) * (ny + 1) * (nz + 1) != m->n_nodes || m->n_hang != 0)
      return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: uniform brick sizes inconsistent");
    ctx->nx = (int)nx; ctx->ny = (int)ny; ctx->nz = (int)nz;
  } else {
    if (!m->node_xyz) return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: octree mesh needs node_xyz");
    if (m->dims[0] <= 0 || m->dims[1] <= 0 || m->dims[2] <= 0)
      return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: octree mesh needs positive lattice extents");
    for (long i = 0; i < 3L * m->n_nodes; ++i)
      if (m->node_xyz[i] < 0 || m->node_xyz[i] > m->dims[i % 3])
        return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: node coordinate outside the lattice box");
    for (long i = 0; i < 8L * m->n_elems; ++i)
      if (m->elem_nodes[i] < 0 || m->elem_nodes[i] >= m->n_nodes)
        return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: element node index out of range");
    ctx->nx = m->dims[0]; ctx->ny = m->dims[1]; ctx->nz = m->dims[2];
  }
  if (m->max_level < 0 || m->max_level > 16)
    return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: max_level outside [0, 16]");
  ctx->uniform = uni;
  ctx->n_nodes = m->n_nodes;
  ctx->n_elems = m->n_elems;
  ctx->max_level = m->max_level;
  const long n3 = 3L * m->n_nodes;

  // supports: one byte per node, bit c for DOF c
  std::vector<uint8_t> fix(m->n_nodes, 0);
  for (long i = 0; i < n3; ++i)
    if (m->dof_fixed[i]) fix[i / 3] |= (uint8_t)(1u << (i % 3));
  AMRTO_HIP(dalloc(ctx->d_fix, m->n_nodes));
  AMRTO_HIP(hipMemcpy(ctx->d_fix, fix.data(), fix.size(), hipMemcpyHostToDevice));

  // element levels and volumes
  std::vector<int8_t> lev(m->n_elems, (int8_t)m->max_level);
  if (m->elem_level) std::memcpy(lev.data(), m->elem_level, m->n_elems);
  for (int8_t l : lev)
    if (l < 0 || l > m->max_level) return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: element level out of range");
  std::vector<double> vol(m->n_elems);
  for (int e = 0; e < m->n_elems; ++e) {
    double h = (double)(1 << (m->max_level - lev[e]));
    vol[e] = h * h * h;
  }
  AMRTO_HIP(dalloc(ctx->d_level, m->n_elems));
  AMRTO_HIP(hipMemcpy(ctx->d_level, lev.data(), lev.size(), hipMemcpyHostToDevice));
  AMRTO_HIP(dalloc(ctx->d_vol, m->n_elems));
  AMRTO_HIP(hipMemcpy(ctx->d_vol, vol.data(), vol.size() * sizeof(double), hipMemcpyHostToDevice));
  ctx->h_level = lev;

  if (!uni) {
    ctx->h_node_xyz.assign(m->node_xyz, m->node_xyz + n3);
    ctx->h_elem_nodes.assign(m->elem_nodes, m->elem_nodes + 8L * m->n_elems);
    AMRTO_HIP(dalloc(ctx->d_elem_nodes, 8L * m->n_elems));
    AMRTO_HIP(hipMemcpy(ctx->d_elem_nodes, m->elem_nodes, 8L * m->n_elems * sizeof(int32_t), hipMemcpyHostToDevice));
    int rc = build_chunks(ctx, m);
    if (rc != AMRTO_OK) return rc;
    rc = build_cell_map(ctx);
    if (rc != AMRTO_OK) return rc;
  } else {
    ctx->h_node_xyz.clear();
    ctx->h_elem_nodes.clear();
    ctx->n_chunks = 0; ctx->n_hang = 0; ctx->n_entries = 0;
  }

  // density-dependent arrays and the solver workspace
  AMRTO_HIP(dalloc(ctx->d_coef, m->n_elems));
  AMRTO_HIP(dalloc(ctx->d_coef_f, m->n_elems));
  AMRTO_HIP(dalloc(ctx->d_dinv, n3));
  AMRTO_HIP(dalloc(ctx->d_dinv_f, n3));
  AMRTO_HIP(dalloc(ctx->d_r, n3)); AMRTO_HIP(dalloc(ctx->d_z, n3));
  AMRTO_HIP(dalloc(ctx->d_p, n3)); AMRTO_HIP(dalloc(ctx->d_q, n3)); AMRTO_HIP(dalloc(ctx->d_p2, n3));
  AMRTO_HIP(dalloc(ctx->f_p2, n3));
  ctx->n_partpq = apply_blocks(ctx);
  AMRTO_HIP(dalloc(ctx->d_partpq, ctx->n_partpq));
  AMRTO_HIP(dalloc(ctx->d_binv, 6L * m->n_nodes)); AMRTO_HIP(dalloc(ctx->d_binv_f, 6L * m->n_nodes));
  if (!uni) {
    AMRTO_HIP(dalloc(ctx->d_cg1_r2, n3)); AMRTO_HIP(dalloc(ctx->d_cg1_w, n3)); AMRTO_HIP(dalloc(ctx->d_cg1_w2, n3));
    AMRTO_HIP(dalloc(ctx->d_cg1_s, n3)); AMRTO_HIP(dalloc(ctx->d_cg1_s2, n3));
    AMRTO_HIP(dalloc(ctx->d_cg1_part, 6L * cg1_parts(ctx)));
  }
  AMRTO_HIP(dalloc(ctx->f_b, n3)); AMRTO_HIP(dalloc(ctx->f_x, n3)); AMRTO_HIP(dalloc(ctx->f_r, n3)); AMRTO_HIP(dalloc(ctx->f_z, n3));
  AMRTO_HIP(dalloc(ctx->f_p, n3)); AMRTO_HIP(dalloc(ctx->f_q, n3));
  ctx->has_mesh = true;
  return AMRTO_OK;
}

int amrto_mesh_info(const amrto_ctx* ctx, int32_t* n_nodes, int32_t* n_elems, int32_t* n_chunks) {
  if (!ctx) return AMRTO_EINVAL;
  if (n_nodes) *n_nodes = ctx->n_nodes;
  if (n_elems) *n_elems = ctx->n_elems;
  if (n_chunks) *n_chunks = ctx->n_chunks;
  return AMRTO_OK;
}

int amrto_set_density(amrto_ctx* ctx, const double* rho) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_set_density: no mesh uploaded");
  ctx->binv_valid = false;
  if (!rho) return ctx->fail(AMRTO_EINVAL, "amrto_set_density: rho is NULL");
  AMRTO_HIP(hipSetDevice(ctx->device));
  ctx->coarse_k = 0;  // Z^T A~ Z depends on the density
  ctx->mg_valid = false;
  int rc = launch_set_density(ctx, rho);
  if (rc) return rc;
  rc = launch_diag(ctx);
  if (rc) return rc;
  ctx->has_density = true;
  return AMRTO_OK;
}

int amrto_get_diag(amrto_ctx* ctx, double* diag) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, "amrto_get_diag: density not set");
  if (!diag) return ctx->fail(AMRTO_EINVAL, "amrto_get_diag: NULL buffer");
  AMRTO_HIP(hipSetDevice(ctx->device));
  return launch_recip(ctx, ctx->d_dinv, diag, 3L * ctx->n_nodes);
}

int amrto_apply(amrto_ctx* ctx, const void* x, void* y, int prec) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, "amrto_apply: density not set");
  if (prec != AMRTO_FP64 && prec != AMRTO_FP32 && prec != AMRTO_BF16)
    return ctx->fail(AMRTO_EINVAL, "amrto_apply: unknown precision");
  if (!x || !y || x == y) return ctx->fail(AMRTO_EINVAL, "amrto_apply: x and y must be distinct device buffers");
  AMRTO_HIP(hipSetDevice(ctx->device));
  return launch_apply(ctx, x, y, prec);
}

int amrto_project_rhs(amrto_ctx* ctx, const double* f, double* b) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_project_rhs: no mesh");
  if (!f || !b || f == b) return ctx->fail(AMRTO_EINVAL, "amrto_project_rhs: f and b must be distinct");
  AMRTO_HIP(hipSetDevice(ctx->device));
  return launch_project_rhs(ctx, f, b);
}

int amrto_recover(amrto_ctx* ctx, const double* ut, double* u) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_recover: no mesh");
  if (!ut || !u) return ctx->fail(AMRTO_EINVAL, "amrto_recover: NULL buffer");
  AMRTO_HIP(hipSetDevice(ctx->device));
  return launch_recover(ctx, ut, u);
}

}  // extern "C"
