// Design-side kernels of one SIMP iteration (paper Sec. 3 and Sec. 6):
// compliance and its self-adjoint sensitivity, the distance-weighted filters
// of Eq. (3)-(5), and the Optimality Criteria update with its volume
// multiplier found by a k-ary search.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "internal.h"

namespace amrto {

__device__ __forceinline__ double block_sum_t(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_max_t(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = fmax(s, sh[i]);
  __syncthreads();
  return s;
}

// ------------------------------------------------------------------ compliance
__global__ __launch_bounds__(256) void k_dot_part(const double* __restrict__ a, const double* __restrict__ b, long n,
                                                  double* __restrict__ part) {
  __shared__ double sh[16];
  double s = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  s = block_sum_t(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_sum_part(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
  v = block_sum_t(v, sh);
  if (threadIdx.x == 0) *out = v;
}

// dc_e = -p rho^(p-1) (E0 - Emin) h_e u_e^T K0 u_e
__global__ __launch_bounds__(256) void k_sensitivity(
    const double* __restrict__ u, const double* __restrict__ rho, const int8_t* __restrict__ level,
    const int32_t* __restrict__ elem_nodes, const double* __restrict__ K0, double* __restrict__ dc, int n_elems,
    int nx, int ny, int max_level, double dE, double p) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elems) return;
  int nodes[8];
  if (elem_nodes) {
#pragma unroll
    for (int a = 0; a < 8; ++a) nodes[a] = elem_nodes[8L * e + a];
  } else {
    const int ex = e % nx, ey = (e / nx) % ny, ez = e / (nx * ny);
#pragma unroll
    for (int a = 0; a < 8; ++a)
      nodes[a] = (ex + (a & 1)) + (nx + 1) * ((ey + ((a >> 1) & 1)) + (ny + 1) * (ez + (a >> 2)));
  }
  double ue[24];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) ue[3 * a + c] = u[3L * nodes[a] + c];
  // K0 annihilates rigid translations, so u_e^T K0 u_e is unchanged by
  // subtracting the element mean; doing so removes most of the cancellation
  // when the element mostly translates (small strain energy, large |u|).
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double m = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) m += ue[3 * a + c];
    m *= 0.125;
#pragma unroll
    for (int a = 0; a < 8; ++a) ue[3 * a + c] -= m;
  }
  double w = 0.0;
#pragma unroll
  for (int r = 0; r < 24; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < 24; ++s) acc = fma(K0[r * 24 + s], ue[s], acc);
    w = fma(ue[r], acc, w);
  }
  const double h = (double)(1 << (max_level - level[e]));
  dc[e] = -p * pow(rho[e], p - 1.0) * dE * h * w;
}

// ------------------------------------------------------------------ filters
// weights W_ed = H_de V_d; SENSITIVITY: sum W rho_d in_d / (max(rho_e, 1e-3) sum W)
//                          DENSITY:     sum W in_d / sum W
__global__ __launch_bounds__(256) void k_filter_uniform(
    const double* __restrict__ in, const double* __restrict__ rho, double* __restrict__ out,
    const int4* __restrict__ sten, const double* __restrict__ sw, int n_sten, int nx, int ny, int nz, int mode) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)nx * ny * nz) return;
  const int ex = e % nx, ey = (e / nx) % ny, ez = e / ((long)nx * ny);
  double num = 0.0, den = 0.0;
  for (int s = 0; s < n_sten; ++s) {
    const int4 st = sten[s];
    const int dx = ex + st.x, dy = ey + st.y, dz = ez + st.z;
    if (dx < 0 || dx >= nx || dy < 0 || dy >= ny || dz < 0 || dz >= nz) continue;
    const long d = dx + (long)nx * (dy + (long)ny * dz);
    const double w = sw[s];
    num += w * (mode == AMRTO_FILTER_SENSITIVITY ? rho[d] * in[d] : in[d]);
    den += w;
  }
  out[e] = mode == AMRTO_FILTER_SENSITIVITY ? num / (fmax(rho[e], 1e-3) * den) : num / den;
}

__global__ __launch_bounds__(256) void k_filter_csr(
    const double* __restrict__ in, const double* __restrict__ rho, double* __restrict__ out,
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx, const double* __restrict__ w, int n, int mode) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double num = 0.0, den = 0.0;
  for (int k = ptr[e]; k < ptr[e + 1]; ++k) {
    const int d = idx[k];
    num += w[k] * (mode == AMRTO_FILTER_SENSITIVITY ? rho[d] * in[d] : in[d]);
    den += w[k];
  }
  out[e] = mode == AMRTO_FILTER_SENSITIVITY ? num / (fmax(rho[e], 1e-3) * den) : num / den;
}

// ------------------------------------------------------------------ OC
constexpr int OC_K = 256;      // candidates per pass
constexpr int OC_BLOCKS = 1024;
constexpr int OC_TILE = 64;   // elements per block and step of the volume pass
constexpr int OC_VOL = 2 + OC_BLOCKS * OC_K;

__device__ __forceinline__ double oc_new(double rho, double g, double lam, double eta, double move, double rmin) {
  const double b = g / lam;
  const double f = eta == 0.5 ? sqrt(b) : pow(b, eta);
  const double lo = fmax(rmin, rho - move), hi = fmin(1.0, rho + move);
  return fmin(fmax(rho * f, lo), hi);
}

// ws layout: [0] log lo, [1] log hi, [2..] partial volumes OC_K x nblocks
// (candidate-major), then OC_K candidate volumes at OC_VOL
__global__ __launch_bounds__(OC_K) void k_oc_volumes(
    const double* __restrict__ rho, const double* __restrict__ dc, const double* __restrict__ vol, int n,
    double eta, double move, double rmin, double* __restrict__ ws) {
  // rho (g / lam)^eta = (rho g^eta) lam^-eta: the powers are taken once per
  // element (as a tile is staged) and once per candidate, so a pair costs a
  // product, the move limits and the volume product
  __shared__ double s_rg[OC_TILE], s_lo[OC_TILE], s_hi[OC_TILE], s_v[OC_TILE];
  const double llo = ws[0], lhi = ws[1];
  const int j = threadIdx.x;
  const double lam = exp(llo + (lhi - llo) * (double)j / (double)(OC_K - 1));
  const double ilam = eta == 0.5 ? 1.0 / sqrt(lam) : pow(lam, -eta);
  double acc = 0.0;
  for (int base = blockIdx.x * OC_TILE; base < n; base += gridDim.x * OC_TILE) {
    const int e = base + j;
    __syncthreads();
    if (j < OC_TILE && e < n) {
      const double r = rho[e], g = fmax(-dc[e], 0.0) / vol[e];
      s_rg[j] = r * (eta == 0.5 ? sqrt(g) : pow(g, eta));
      s_lo[j] = fmax(rmin, r - move);
      s_hi[j] = fmin(1.0, r + move);
      s_v[j] = vol[e];
    }
    __syncthreads();
    const int m = min(OC_TILE, n - base);
    for (int t = 0; t < m; ++t) acc += fmin(fmax(s_rg[t] * ilam, s_lo[t]), s_hi[t]) * s_v[t];
  }
  ws[2 + (long)j * gridDim.x + blockIdx.x] = acc;
}

// volume of candidate j = blockIdx.x: its nblocks partials in a fixed tree
__global__ __launch_bounds__(256) void k_oc_candsum(double* __restrict__ ws, int nblocks) {
  __shared__ double sh[8];
  const int j = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += ws[2 + (long)j * nblocks + b];
  v = block_sum_t(v, sh);
  if (threadIdx.x == 0) ws[OC_VOL + j] = v;
}

__global__ __launch_bounds__(OC_K) void k_oc_bracket(double* __restrict__ ws, double v0) {
  __shared__ double s_vol[OC_K];
  const int j = threadIdx.x;
  s_vol[j] = ws[OC_VOL + j];
  __syncthreads();
  if (j == 0) {
    const double llo = ws[0], lhi = ws[1];
    // volume is non-increasing in lam: last candidate whose volume exceeds v0
    int jl = -1;
    for (int t = 0; t < OC_K; ++t)
      if (s_vol[t] > v0) jl = t;
    double nlo, nhi;
    if (jl < 0) { nlo = llo; nhi = llo; }
    else if (jl == OC_K - 1) { nlo = lhi; nhi = lhi; }
    else {
      nlo = llo + (lhi - llo) * (double)jl / (double)(OC_K - 1);
      nhi = llo + (lhi - llo) * (double)(jl + 1) / (double)(OC_K - 1);
    }
    ws[0] = nlo;
    ws[1] = nhi;
  }
}

__global__ __launch_bounds__(256) void k_oc_apply(
    const double* __restrict__ rho, const double* __restrict__ dc, const double* __restrict__ vol, int n,
    double eta, double move, double rmin, double* __restrict__ rho_new, double* __restrict__ ws) {
  __shared__ double sh[16];
  const double lam = exp(0.5 * (ws[0] + ws[1]));
  double ch = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double g = fmax(-dc[e], 0.0) / vol[e];
    const double r = oc_new(rho[e], g, lam, eta, move, rmin);
    ch = fmax(ch, fabs(r - rho[e]));
    rho_new[e] = r;
  }
  ch = block_max_t(ch, sh);
  if (threadIdx.x == 0) ws[2 + blockIdx.x] = ch;
}

__global__ __launch_bounds__(256) void k_oc_finish(double* __restrict__ ws, int nblocks) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) v = fmax(v, ws[2 + i]);
  v = block_max_t(v, sh);
  if (threadIdx.x == 0) {
    ws[2] = v;
    ws[3] = exp(0.5 * (ws[0] + ws[1]));
  }
}

__global__ void k_init_bracket(double* ws, double llo, double lhi) {
  ws[0] = llo;
  ws[1] = lhi;
}

// ------------------------------------------------------------------ host
// Neighbour lists for an octree mesh: all element pairs with centre distance
// below rmin (a hash grid of cell size ceil(rmin) over element centres; a
// coarse element is inserted once at its centre, and the search radius is
// widened by half the largest element edge in each direction).
static int build_neighbours(amrto_ctx* ctx, double rmin) {
  const int ne = ctx->n_elems;
  std::vector<double> cx(ne), cy(ne), cz(ne), vol(ne);
  for (int e = 0; e < ne; ++e) {
    const int n0 = ctx->h_elem_nodes[8L * e];
    const int h = 1 << (ctx->max_level - ctx->h_level[e]);
    cx[e] = ctx->h_node_xyz[3L * n0] + 0.5 * h;
    cy[e] = ctx->h_node_xyz[3L * n0 + 1] + 0.5 * h;
    cz[e] = ctx->h_node_xyz[3L * n0 + 2] + 0.5 * h;
    vol[e] = (double)h * h * h;
  }
  const double cell = std::max(1.0, std::ceil(rmin));
  auto key = [](long a, long b, long c) { return (a * 73856093L) ^ (b * 19349663L) ^ (c * 83492791L); };
  std::unordered_multimap<long, int> grid;
  grid.reserve(ne * 2);
  for (int e = 0; e < ne; ++e)
    grid.emplace(key((long)std::floor(cx[e] / cell), (long)std::floor(cy[e] / cell), (long)std::floor(cz[e] / cell)), e);
  std::vector<int> ptr(ne + 1, 0), idx;
  std::vector<double> w;
  const int reach = (int)std::ceil(rmin / cell);
  for (int e = 0; e < ne; ++e) {
    const long gx = (long)std::floor(cx[e] / cell), gy = (long)std::floor(cy[e] / cell), gz = (long)std::floor(cz[e] / cell);
    std::vector<std::pair<int, double>> nb;
    for (long dz = -reach; dz <= reach; ++dz)
      for (long dy = -reach; dy <= reach; ++dy)
        for (long dx = -reach; dx <= reach; ++dx) {
          auto range = grid.equal_range(key(gx + dx, gy + dy, gz + dz));
          for (auto it = range.first; it != range.second; ++it) {
            const int d = it->second;
            const double ddx = cx[d] - cx[e], ddy = cy[d] - cy[e], ddz = cz[d] - cz[e];
            if (std::fabs(ddx) > rmin || std::fabs(ddy) > rmin || std::fabs(ddz) > rmin) continue;
            const double H = rmin - std::sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
            if (H > 0.0) nb.emplace_back(d, H * vol[d]);
          }
        }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end(), [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
               return a.first == b.first;
             }), nb.end());
    for (auto& pr : nb) { idx.push_back(pr.first); w.push_back(pr.second); }
    ptr[e + 1] = (int)idx.size();
  }
  auto up = [&](auto*& dst, const auto& v) -> hipError_t {
    using T = typename std::remove_reference<decltype(v)>::type::value_type;
    if (dst) (void)hipFree(dst);
    dst = nullptr;
    hipError_t er = hipMalloc((void**)&dst, std::max<size_t>(1, v.size()) * sizeof(T));
    if (er != hipSuccess) return er;
    if (!v.empty()) er = hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return er;
  };
  AMRTO_HIP(up(ctx->d_nb_ptr, ptr));
  AMRTO_HIP(up(ctx->d_nb_idx, idx));
  AMRTO_HIP(up(ctx->d_nb_w, w));
  ctx->filt_rmin = rmin;
  return AMRTO_OK;
}

}  // namespace amrto

using namespace amrto;

extern "C" {

int amrto_compliance(amrto_ctx* ctx, const double* u, const double* f, const double* rho, double* c_host,
                     double* dc) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_compliance: no mesh");
  if (!u || (c_host && !f) || (dc && !rho)) return ctx->fail(AMRTO_EINVAL, "amrto_compliance: NULL buffer");
  AMRTO_HIP(hipSetDevice(ctx->device));
  const long n3 = 3L * ctx->n_nodes;
  if (dc) {
    const int ne = ctx->n_elems;
    hipLaunchKernelGGL(k_sensitivity, dim3((ne + 255) / 256), dim3(256), 0, ctx->stream, u, rho, ctx->d_level,
                       ctx->uniform ? nullptr : ctx->d_elem_nodes, ctx->d_K0, dc, ne, ctx->nx, ctx->ny,
                       ctx->max_level, ctx->E0 - ctx->Emin, ctx->p);
  }
  if (c_host) {
    hipLaunchKernelGGL(k_dot_part, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, f, u, n3, ctx->d_part);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(256), 0, ctx->stream, ctx->d_part, RED_BLOCKS, ctx->d_scal + 6);
    AMRTO_HIP(hipGetLastError());
    AMRTO_HIP(hipMemcpyAsync(ctx->h_scal, ctx->d_scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    AMRTO_HIP(hipStreamSynchronize(ctx->stream));
    *c_host = ctx->h_scal[6];
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_filter(amrto_ctx* ctx, int mode, double rmin, const double* in, const double* rho, double* out) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_filter: no mesh");
  if (mode != AMRTO_FILTER_SENSITIVITY && mode != AMRTO_FILTER_DENSITY)
    return ctx->fail(AMRTO_EINVAL, "amrto_filter: unknown mode");
  if (!(rmin > 0.0) || rmin > 16.0) return ctx->fail(AMRTO_EINVAL, "amrto_filter: rmin must be in (0, 16]");
  if (!in || !out || in == out || (mode == AMRTO_FILTER_SENSITIVITY && !rho))
    return ctx->fail(AMRTO_EINVAL, "amrto_filter: bad buffers");
  AMRTO_HIP(hipSetDevice(ctx->device));
  const int ne = ctx->n_elems;
  if (ctx->uniform) {
    if (ctx->filt_rmin != rmin) {
      // stencil of offsets with H = rmin - |d| > 0 (Eq. (4)); V_d = 1
      std::vector<int32_t> st;
      std::vector<double> wd;
      const int R = (int)std::ceil(rmin);
      for (int dz = -R; dz <= R; ++dz)
        for (int dy = -R; dy <= R; ++dy)
          for (int dx = -R; dx <= R; ++dx) {
            const double H = rmin - std::sqrt((double)(dx * dx + dy * dy + dz * dz));
            if (H > 0.0) {
              st.insert(st.end(), {dx, dy, dz, 0});
              wd.push_back(H);
            }
          }
      if (ctx->d_nb_idx) (void)hipFree(ctx->d_nb_idx);
      if (ctx->d_nb_w) (void)hipFree(ctx->d_nb_w);
      ctx->d_nb_idx = nullptr;
      ctx->d_nb_w = nullptr;
      AMRTO_HIP(hipMalloc((void**)&ctx->d_nb_idx, st.size() * sizeof(int32_t)));
      AMRTO_HIP(hipMalloc((void**)&ctx->d_nb_w, wd.size() * sizeof(double)));
      AMRTO_HIP(hipMemcpy(ctx->d_nb_idx, st.data(), st.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      AMRTO_HIP(hipMemcpy(ctx->d_nb_w, wd.data(), wd.size() * sizeof(double), hipMemcpyHostToDevice));
      ctx->n_sten = (int)wd.size();
      ctx->filt_rmin = rmin;
    }
    hipLaunchKernelGGL(k_filter_uniform, dim3((ne + 255) / 256), dim3(256), 0, ctx->stream, in, rho, out,
                       (const int4*)ctx->d_nb_idx, ctx->d_nb_w, ctx->n_sten, ctx->nx, ctx->ny, ctx->nz, mode);
  } else {
    if (ctx->filt_rmin != rmin) {
      int rc = build_neighbours(ctx, rmin);
      if (rc) return rc;
    }
    hipLaunchKernelGGL(k_filter_csr, dim3((ne + 255) / 256), dim3(256), 0, ctx->stream, in, rho, out, ctx->d_nb_ptr,
                       ctx->d_nb_idx, ctx->d_nb_w, ne, mode);
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_oc_update(amrto_ctx* ctx, const double* rho, const double* dc, double volfrac, double move, double eta,
                    double rho_min, double* rho_new, double* change_host, double* lam_host) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_oc_update: no mesh");
  if (!rho || !dc || !rho_new || rho_new == rho) return ctx->fail(AMRTO_EINVAL, "amrto_oc_update: bad buffers");
  if (!(volfrac > 0.0 && volfrac <= 1.0) || !(move > 0.0) || !(eta > 0.0) || !(rho_min >= 0.0 && rho_min < 1.0))
    return ctx->fail(AMRTO_EINVAL, "amrto_oc_update: bad parameters");
  AMRTO_HIP(hipSetDevice(ctx->device));
  const int ne = ctx->n_elems;
  double vtot = 0.0;
  for (int e = 0; e < ne; ++e) {
    const double h = (double)(1 << (ctx->max_level - ctx->h_level[e]));
    vtot += h * h * h;
  }
  const double v0 = volfrac * vtot;
  const int nblk = std::min(OC_BLOCKS, (ne + OC_TILE - 1) / OC_TILE);
  double* ws = ctx->d_oc;
  // log(lam) in [log 1e-300, log 1e300]; each pass narrows it 255-fold
  hipLaunchKernelGGL(k_init_bracket, dim3(1), dim3(1), 0, ctx->stream, ws, std::log(1e-300), std::log(1e300));
  double width = std::log(1e300) - std::log(1e-300);
  while (width > 1e-14) {
    hipLaunchKernelGGL(k_oc_volumes, dim3(nblk), dim3(OC_K), 0, ctx->stream, rho, dc, ctx->d_vol, ne, eta, move,
                       rho_min, ws);
    hipLaunchKernelGGL(k_oc_candsum, dim3(OC_K), dim3(256), 0, ctx->stream, ws, nblk);
    hipLaunchKernelGGL(k_oc_bracket, dim3(1), dim3(OC_K), 0, ctx->stream, ws, v0);
    width /= (OC_K - 1);
  }
  const int g = std::min(256, (ne + 255) / 256);
  hipLaunchKernelGGL(k_oc_apply, dim3(g), dim3(256), 0, ctx->stream, rho, dc, ctx->d_vol, ne, eta, move, rho_min,
                     rho_new, ws);
  hipLaunchKernelGGL(k_oc_finish, dim3(1), dim3(256), 0, ctx->stream, ws, g);
  AMRTO_HIP(hipGetLastError());
  if (change_host || lam_host) {
    double h[4];
    AMRTO_HIP(hipMemcpyAsync(h, ws, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    AMRTO_HIP(hipStreamSynchronize(ctx->stream));
    if (change_host) *change_host = h[2];
    if (lam_host) *lam_host = h[3];
  }
  return AMRTO_OK;
}

}  // extern "C"
