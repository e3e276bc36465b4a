// Two-level preconditioner and warm start from predicted displacement fields.
//
// Coarse space: Z has k = 3 n_fields n_regions columns; column (f, g, c) is
// component c of field f restricted to the nodes of region g (the domain split
// into rx x ry x rz equal boxes).  Z is never stored: a DOF's row of Z is its
// field values placed at the column of its node's region.  With
// E = Z^T A~ Z the preconditioner M^-1 = D^-1 + Z E^-1 Z^T is SPD, so CG stays
// valid whatever the fields are; good fields (a network's prediction of the
// displacement) put the slowest error components into the coarse solve.
//
// Warm start: x0 = V a with a minimising the energy 1/2 x^T A~ x - b^T x over
// the span of given vectors V (for instance the previous solution and a
// prediction), so it is never worse in the energy norm than any of them.
#include <cmath>
#include <vector>

#include "kernels.h"

namespace amrto {

__global__ __launch_bounds__(256) void k_node_region(const int32_t* __restrict__ xyz, int n_nodes, int nx, int ny,
                                                     int nz, int rx, int ry, int rz, uint8_t* __restrict__ region) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_nodes) return;
  int px, py, pz;
  if (xyz) {
    px = xyz[3L * v]; py = xyz[3L * v + 1]; pz = xyz[3L * v + 2];
  } else {
    px = v % (nx + 1); py = (v / (nx + 1)) % (ny + 1); pz = v / ((nx + 1) * (ny + 1));
  }
  const int gx = min(px * rx / nx, rx - 1), gy = min(py * ry / ny, ry - 1), gz = min(pz * rz / nz, rz - 1);
  region[v] = (uint8_t)((gz * ry + gy) * rx + gx);
}

// Affine fields 0..3: (1,1,1), (x,y,z), (y,z,x), (z,x,y) with coordinates
// centred on the node's region and scaled by the largest extent, rounded to
// FP32 once: geo[v] = (dx, dy, dz, region | mask << 8) is what the solve
// kernels read, and the stored fields are made from the same values.
__global__ __launch_bounds__(256) void k_affine_fields(const int32_t* __restrict__ xyz, int n_nodes, int nx, int ny,
                                                       int nz, int rx, int ry, int rz, const uint8_t* __restrict__ cmask,
                                                       float4* __restrict__ geo, double* __restrict__ F) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_nodes) return;
  int px, py, pz;
  if (xyz) {
    px = xyz[3L * v]; py = xyz[3L * v + 1]; pz = xyz[3L * v + 2];
  } else {
    px = v % (nx + 1); py = (v / (nx + 1)) % (ny + 1); pz = v / ((nx + 1) * (ny + 1));
  }
  const int gx = min(px * rx / nx, rx - 1), gy = min(py * ry / ny, ry - 1), gz = min(pz * rz / nz, rz - 1);
  const double s = 1.0 / max(nx, max(ny, nz));
  const float c[3] = {(float)((px - (gx + 0.5) * nx / rx) * s), (float)((py - (gy + 0.5) * ny / ry) * s),
                      (float)((pz - (gz + 0.5) * nz / rz) * s)};
  const int g = (gz * ry + gy) * rx + gx;
  geo[v] = make_float4(c[0], c[1], c[2], __int_as_float(g | ((int)cmask[v] << 8)));
  const long n3 = 3L * n_nodes;
  for (int d = 0; d < 3; ++d) {
    F[3L * v + d] = 1.0;
    F[n3 + 3L * v + d] = (double)c[d];
    F[2 * n3 + 3L * v + d] = (double)c[(d + 1) % 3];
    F[3 * n3 + 3L * v + d] = (double)c[(d + 2) % 3];
  }
}

// cmask[v] = supported components of node v, all three for hanging nodes
__global__ __launch_bounds__(256) void k_cmask(const uint8_t* __restrict__ fix, int n_nodes, uint8_t* __restrict__ cmask) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n_nodes) cmask[v] = fix[v] & 7;
}
__global__ __launch_bounds__(256) void k_cmask_hanging(const int32_t* __restrict__ hang, int n_hang,
                                                       uint8_t* __restrict__ cmask) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < n_hang) cmask[hang[h]] = 7;
}

// r = b - q
__global__ __launch_bounds__(256) void k_sub(const double* __restrict__ b, const double* __restrict__ q, long n,
                                             double* __restrict__ r) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - q[i];
}

// column j = (f n_regions + g) 3 + c of Z as a full vector
__global__ __launch_bounds__(256) void k_make_column(const double* __restrict__ F, long n3, const uint8_t* __restrict__ region,
                                                     int f, int g, int c, double* __restrict__ out) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n3) return;
  out[i] = (region[i / 3] == g && (i % 3) == c) ? F[(long)f * n3 + i] : 0.0;
}

// x = a v (first) or x += a v
__global__ __launch_bounds__(256) void k_axpy_set(double a, const double* __restrict__ v, long n3, int first,
                                                  double* __restrict__ x) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n3) return;
  x[i] = first ? a * v[i] : fma(a, v[i], x[i]);
}

// E[i k + j] = sum over blocks of part[block k + i]; one block per row i
// (deterministic tree)
__global__ __launch_bounds__(256) void k_gram_column(const double* __restrict__ part, int k, int j,
                                                     double* __restrict__ E) {
  __shared__ double sh[8];
  const int i = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < RED_BLOCKS; b += blockDim.x) v += part[(long)i * RED_BLOCKS + b];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) E[(long)i * k + j] = v;
}

__global__ __launch_bounds__(256) void k_dot2_part(const double* __restrict__ a, const double* __restrict__ b, long n,
                                                   double* __restrict__ part) {
  __shared__ double sh[8];
  double s = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) s += a[i] * b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Cholesky of the active principal submatrix of a k x k SPD matrix, dropping
// columns whose pivot falls below tol * max diagonal; returns the inverse
// (zero rows/columns for dropped ones) and the number kept.
static int spd_inverse(std::vector<double> E, int k, std::vector<double>& inv) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < i; ++j) E[i * k + j] = E[j * k + i] = 0.5 * (E[i * k + j] + E[j * k + i]);
  double dmax = 0.0;
  for (int i = 0; i < k; ++i) dmax = std::max(dmax, E[i * k + i]);
  std::vector<int> act;
  std::vector<double> L;
  for (int c = 0; c < k; ++c) {
    // try to append column c to the factor of the active set
    const int m = (int)act.size();
    std::vector<double> row(m);
    for (int i = 0; i < m; ++i) {
      double s = E[act[i] * k + c];
      for (int j = 0; j < i; ++j) s -= L[i * k + j] * row[j];
      row[i] = s / L[i * k + i];
    }
    double d = E[c * k + c];
    for (int j = 0; j < m; ++j) d -= row[j] * row[j];
    if (!(d > 1e-12 * dmax)) continue;
    act.push_back(c);
    L.resize(k * k, 0.0);
    for (int j = 0; j < m; ++j) L[m * k + j] = row[j];
    L[m * k + m] = std::sqrt(d);
  }
  const int m = (int)act.size();
  inv.assign(k * k, 0.0);
  // inverse of the active block: solve L L^T X = I column by column
  for (int col = 0; col < m; ++col) {
    std::vector<double> y(m, 0.0), x(m, 0.0);
    for (int i = 0; i < m; ++i) {
      double s = (i == col) ? 1.0 : 0.0;
      for (int j = 0; j < i; ++j) s -= L[i * k + j] * y[j];
      y[i] = s / L[i * k + i];
    }
    for (int i = m - 1; i >= 0; --i) {
      double s = y[i];
      for (int j = i + 1; j < m; ++j) s -= L[j * k + i] * x[j];
      x[i] = s / L[i * k + i];
    }
    for (int i = 0; i < m; ++i) inv[act[i] * k + act[col]] = x[i];
  }
  return m;
}

}  // namespace amrto

using namespace amrto;

extern "C" {

int amrto_coarse_setup(amrto_ctx* ctx, int32_t affine, const double* const* fields, int32_t n_fields, int32_t rx,
                       int32_t ry, int32_t rz, int32_t* k_kept) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, "amrto_coarse_setup: density not set");
  const int nf = (affine ? 4 : 0) + n_fields;
  const int R = rx * ry * rz;
  const int k = 3 * nf * R;
  if (n_fields < 0 || (n_fields > 0 && !fields) || nf < 1 || nf > COARSE_NFMAX || rx < 1 || ry < 1 || rz < 1 ||
      R > 255 || k > COARSE_KMAX)
    return ctx->fail(AMRTO_EINVAL,
                     "amrto_coarse_setup: need at most 8 fields and 1 <= 3 (4 affine + n_fields) rx ry rz <= 384");
  AMRTO_HIP(hipSetDevice(ctx->device));
  ctx->coarse_k = 0;  // no coarse space unless this setup completes
  const long n3 = 3L * ctx->n_nodes;
  // fields (affine ones generated, caller ones copied), node regions
  if (nf > ctx->coarse_cap) {
    if (ctx->d_cf) (void)hipFree(ctx->d_cf);
    ctx->d_cf = nullptr;
    ctx->coarse_cap = 0;
    AMRTO_HIP(hipMalloc((void**)&ctx->d_cf, nf * n3 * sizeof(double)));
    ctx->coarse_cap = nf;
  }
  if (!ctx->uniform && !ctx->d_node_xyz) {
    AMRTO_HIP(hipMalloc((void**)&ctx->d_node_xyz, n3 * sizeof(int32_t)));
    AMRTO_HIP(hipMemcpy(ctx->d_node_xyz, ctx->h_node_xyz.data(), n3 * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  const int32_t* xyz = ctx->uniform ? nullptr : ctx->d_node_xyz;
  const int gn = (ctx->n_nodes + 255) / 256;
  for (int f = 0; f < n_fields; ++f) {
    if (!fields[f]) return ctx->fail(AMRTO_EINVAL, "amrto_coarse_setup: null field");
    AMRTO_HIP(hipMemcpyAsync(ctx->d_cf + (long)(nf - n_fields + f) * n3, fields[f], n3 * sizeof(double),
                             hipMemcpyDeviceToDevice, ctx->stream));
  }
  if (!ctx->d_region) AMRTO_HIP(hipMalloc((void**)&ctx->d_region, ctx->n_nodes));
  if (!ctx->d_cmask) AMRTO_HIP(hipMalloc((void**)&ctx->d_cmask, ctx->n_nodes));
  hipLaunchKernelGGL(k_cmask, dim3(gn), dim3(256), 0, ctx->stream, ctx->d_fix, ctx->n_nodes, ctx->d_cmask);
  if (ctx->n_hang)
    hipLaunchKernelGGL(k_cmask_hanging, dim3((ctx->n_hang + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_hang_node,
                       ctx->n_hang, ctx->d_cmask);
  ctx->coarse_nf = nf;
  ctx->coarse_R = R;
  ctx->coarse_affine_only = (affine && n_fields == 0) ? 1 : 0;
  if (!ctx->uniform && ctx->coarse_affine_only) {
    // partials of Z^T q and E^-1 Z^T q per operator-pass block (recurrence form)
    const long need = 2L * k * apply_blocks(ctx);
    if (need > ctx->cq_cap) {
      if (ctx->d_cqpart) (void)hipFree(ctx->d_cqpart);
      ctx->d_cqpart = nullptr;
      ctx->cq_cap = 0;
      AMRTO_HIP(hipMalloc((void**)&ctx->d_cqpart, need * sizeof(double)));
      ctx->cq_cap = need;
    }
  }
  if (affine) {
    if (!ctx->d_cgeo) AMRTO_HIP(hipMalloc((void**)&ctx->d_cgeo, ctx->n_nodes * sizeof(float4)));
    hipLaunchKernelGGL(k_affine_fields, dim3(gn), dim3(256), 0, ctx->stream, xyz, ctx->n_nodes, ctx->nx, ctx->ny,
                       ctx->nz, rx, ry, rz, (const uint8_t*)ctx->d_cmask, ctx->d_cgeo, ctx->d_cf);
  }
  {
    int rc = mask_vector_n(ctx, ctx->d_cf, nf);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_node_region, dim3(gn), dim3(256), 0, ctx->stream, xyz, ctx->n_nodes, ctx->nx, ctx->ny, ctx->nz,
                     rx, ry, rz, ctx->d_region);
  if (!ctx->d_cpart) AMRTO_HIP(hipMalloc((void**)&ctx->d_cpart, COARSE_KMAX * RED_BLOCKS * sizeof(double)));
  if (!ctx->d_cinv) AMRTO_HIP(hipMalloc((void**)&ctx->d_cinv, COARSE_KMAX * COARSE_KMAX * sizeof(double)));
  if (!ctx->d_cz) AMRTO_HIP(hipMalloc((void**)&ctx->d_cz, COARSE_KMAX * sizeof(double)));
  if (!ctx->d_ct) AMRTO_HIP(hipMalloc((void**)&ctx->d_ct, COARSE_KMAX * sizeof(double)));
  // E[:, j] = Z^T A~ z_j, gathered on the device (d_cinv holds E until the inverse replaces it)
  const int g1 = (int)((n3 + 255) / 256);
  for (int j = 0; j < k; ++j) {
    const int c = j % 3, g = (j / 3) % R, f = j / (3 * R);
    hipLaunchKernelGGL(k_make_column, dim3(g1), dim3(256), 0, ctx->stream, ctx->d_cf, n3, ctx->d_region, f, g, c,
                       ctx->d_z);
    int rc = apply_stop(ctx, ctx->d_z, ctx->d_q, AMRTO_FP64, nullptr);
    if (rc) return rc;
    rc = launch_zt(ctx, ctx->d_q);
    if (rc) return rc;
    hipLaunchKernelGGL(k_gram_column, dim3(k), dim3(256), 0, ctx->stream, ctx->d_cpart, k, j, ctx->d_cinv);
  }
  std::vector<double> E((long)k * k);
  AMRTO_HIP(hipMemcpyAsync(E.data(), ctx->d_cinv, E.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  for (double e : E)
    if (!std::isfinite(e)) return ctx->fail(AMRTO_EINVAL, "amrto_coarse_setup: a coarse field is not finite");
  std::vector<double> inv;
  const int kept = spd_inverse(E, k, inv);
  AMRTO_HIP(hipMemcpy(ctx->d_cinv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice));
  ctx->coarse_k = k;
  if (k_kept) *k_kept = kept;
  return AMRTO_OK;
}

int amrto_coarse_clear(amrto_ctx* ctx) {
  if (!ctx) return AMRTO_EINVAL;
  ctx->coarse_k = 0;
  return AMRTO_OK;
}

int amrto_energy_combine(amrto_ctx* ctx, const double* b, const double* base, const double* const* vecs_host,
                         int32_t n, double* x0, double* coef_host) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, "amrto_energy_combine: density not set");
  if (!b || !vecs_host || !x0 || n < 1 || n > 8) return ctx->fail(AMRTO_EINVAL, "amrto_energy_combine: 1 <= n <= 8");
  for (int j = 0; j < n; ++j)
    if (!vecs_host[j] || vecs_host[j] == x0)
      return ctx->fail(AMRTO_EINVAL, "amrto_energy_combine: vectors must be non-null and distinct from x0");
  if (base == x0) return ctx->fail(AMRTO_EINVAL, "amrto_energy_combine: base must not alias x0");
  AMRTO_HIP(hipSetDevice(ctx->device));
  const long n3 = 3L * ctx->n_nodes;
  std::vector<double> G(n * n), rhs(n), part(RED_BLOCKS);
  auto dot = [&](const double* a, const double* c, double* out) -> int {
    hipLaunchKernelGGL(k_dot2_part, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, a, c, n3, ctx->d_cpart);
    AMRTO_HIP(hipMemcpyAsync(part.data(), ctx->d_cpart, RED_BLOCKS * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    AMRTO_HIP(hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (double v : part) s += v;
    *out = s;
    return AMRTO_OK;
  };
  if (!ctx->d_cpart) AMRTO_HIP(hipMalloc((void**)&ctx->d_cpart, COARSE_KMAX * RED_BLOCKS * sizeof(double)));
  // the residual of the base: rhs_j = v_j^T (b - A~ base)
  const double* res = b;
  if (base) {
    int rc = apply_stop(ctx, base, ctx->d_q, AMRTO_FP64, nullptr);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sub, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, b, ctx->d_q, n3, ctx->d_r);
    res = ctx->d_r;
  }
  for (int j = 0; j < n; ++j) {
    int rc = apply_stop(ctx, vecs_host[j], ctx->d_q, AMRTO_FP64, nullptr);
    if (rc) return rc;
    for (int i = 0; i <= j; ++i) {
      double v;
      rc = dot(vecs_host[i], ctx->d_q, &v);
      if (rc) return rc;
      G[i * n + j] = G[j * n + i] = v;
    }
    int rc2 = dot(vecs_host[j], res, &rhs[j]);
    if (rc2) return rc2;
  }
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(rhs[i])) return ctx->fail(AMRTO_EINVAL, "amrto_energy_combine: a vector is not finite");
    for (int j = 0; j < n; ++j)
      if (!std::isfinite(G[i * n + j]))
        return ctx->fail(AMRTO_EINVAL, "amrto_energy_combine: a vector is not finite");
  }
  std::vector<double> inv;
  spd_inverse(G, n, inv);
  std::vector<double> a(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a[i] += inv[i * n + j] * rhs[j];
  if (base)
    hipLaunchKernelGGL(k_axpy_set, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, 1.0, base, n3, 1, x0);
  for (int j = 0; j < n; ++j)
    hipLaunchKernelGGL(k_axpy_set, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, a[j], vecs_host[j], n3,
                       (j == 0 && !base) ? 1 : 0, x0);
  if (coef_host)
    for (int i = 0; i < n; ++i) coef_host[i] = a[i];
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

}  // extern "C"
