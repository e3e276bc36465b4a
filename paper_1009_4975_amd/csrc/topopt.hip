// Design-side kernels of one SIMP iteration (paper Sec. 3 and Sec. 6):
// compliance and its self-adjoint sensitivity, the distance-weighted filters
// of Eq. (3)-(5), and the Optimality Criteria update with its volume
// multiplier found by a k-ary search.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

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
// weights W_ed = H_de V_d with H_de = max(rmin - |x_d - x_e|, 0) (Eq. (4));
//   SENSITIVITY: sum W rho_d in_d / (max(rho_e, 1e-3) sum W)   (Eq. (5))
//   DENSITY:     sum W in_d / sum W
// Neither kernel reads a neighbour table: the uniform one walks the box of
// offsets |d_a| <= R with H from a per-block table indexed by |d|^2, the
// octree one probes, per leaf size, the aligned anchors a neighbour of that
// size can have and takes each leaf at its anchor cell.  Nothing is built or allocated per call, and the
// summation order is fixed (z, y, x of the offsets or anchors).
constexpr int FILT_RMAX = 16;                       // largest rmin accepted
constexpr int FILT_D2MAX = 3 * FILT_RMAX * FILT_RMAX;  // largest |d|^2 in the box

__global__ __launch_bounds__(256) void k_filter_uniform(
    const double* __restrict__ in, const double* __restrict__ rho, double* __restrict__ out, int nx, int ny, int nz,
    double rmin, int R, int mode) {
  __shared__ double s_h[FILT_D2MAX + 1];
  const int d2max = 3 * R * R;
  for (int s = threadIdx.x; s <= d2max; s += blockDim.x) s_h[s] = fmax(rmin - sqrt((double)s), 0.0);
  __syncthreads();
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)nx * ny * nz) return;
  const int ex = e % nx, ey = (e / nx) % ny, ez = e / ((long)nx * ny);
  double num = 0.0, den = 0.0;
  for (int dz = -R; dz <= R; ++dz) {
    const int z = ez + dz;
    if (z < 0 || z >= nz) continue;
    for (int dy = -R; dy <= R; ++dy) {
      const int y = ey + dy;
      if (y < 0 || y >= ny) continue;
      for (int dx = -R; dx <= R; ++dx) {
        const int x = ex + dx;
        if (x < 0 || x >= nx) continue;
        const double w = s_h[dx * dx + dy * dy + dz * dz];
        if (w <= 0.0) continue;
        const long d = x + (long)nx * (y + (long)ny * z);
        num += w * (mode == AMRTO_FILTER_SENSITIVITY ? rho[d] * in[d] : in[d]);
        den += w;
      }
    }
  }
  out[e] = mode == AMRTO_FILTER_SENSITIVITY ? num / (fmax(rho[e], 1e-3) * den) : num / den;
}

// Octree: desc[e] = (anchor x, y, z, edge h) on the finest lattice; cmap[c] =
// the leaf covering lattice cell c, with bit 31 set on the leaf's anchor
// (lowest) cell.  A neighbour d of edge h_d satisfies |2 a_d + h_d - (2 a_e +
// h_e)| < 2 rmin per axis, and its anchor a_d is a multiple of h_d: per edge
// size, the few aligned candidate anchors are probed, and a cell counts only
// if it is the anchor of a leaf of that size (every leaf once).
__global__ __launch_bounds__(256) void k_filter_octree(
    const double* __restrict__ in, const double* __restrict__ rho, double* __restrict__ out,
    const int4* __restrict__ desc, const int32_t* __restrict__ cmap, int n, int nx, int ny, int nz, int hmax,
    double rmin, int mode) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int4 de = desc[e];
  const int cx = 2 * de.x + de.w, cy = 2 * de.y + de.w, cz = 2 * de.z + de.w;  // doubled centre
  const double r2 = 2.0 * rmin;
  const double lim2 = r2 * r2;
  double num = 0.0, den = 0.0;
  for (int h = 1; h <= hmax; h <<= 1) {
    // aligned anchors a (multiples of h) with |2 a + h - c| < 2 rmin
    auto lo = [&](int c) { return max(0, (int)ceil(0.5 * ((double)(c - h) - r2) / h) * h); };
    auto hi = [&](int c, int nmax) { return min(nmax - h, (int)floor(0.5 * ((double)(c - h) + r2) / h) * h); };
    const int x0 = lo(cx), x1 = hi(cx, nx), y0 = lo(cy), y1 = hi(cy, ny), z0 = lo(cz), z1 = hi(cz, nz);
    for (int z = z0; z <= z1; z += h)
      for (int y = y0; y <= y1; y += h) {
        const long row = (long)nx * (y + (long)ny * z);
        for (int x = x0; x <= x1; x += h) {
          const int v = cmap[row + x];
          if (v >= 0) continue;  // not an anchor cell
          const int d = v & 0x7fffffff;
          const int4 dd = desc[d];
          if (dd.w != h) continue;  // the anchor of a leaf of another size
          const double ddx = (double)(2 * dd.x + h - cx), ddy = (double)(2 * dd.y + h - cy),
                       ddz = (double)(2 * dd.z + h - cz);
          const double D2 = ddx * ddx + ddy * ddy + ddz * ddz;  // (2 |x_d - x_e|)^2
          if (D2 >= lim2) continue;
          const double H = rmin - 0.5 * sqrt(D2);
          if (H <= 0.0) continue;
          const double w = H * (double)h * h * h;
          num += w * (mode == AMRTO_FILTER_SENSITIVITY ? rho[d] * in[d] : in[d]);
          den += w;
        }
      }
  }
  out[e] = mode == AMRTO_FILTER_SENSITIVITY ? num / (fmax(rho[e], 1e-3) * den) : num / den;
}

// cmap from the element descriptors: leaf e writes e into its h^3 cells and
// e | 2^31 into its anchor cell (leaves tile the box, so every cell is
// written exactly once).
__global__ __launch_bounds__(256) void k_cell_map(const int4* __restrict__ desc, int n, int nx, int ny,
                                                 int32_t* __restrict__ cmap) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int4 d = desc[e];
    for (int k = 0; k < d.w; ++k)
      for (int j = 0; j < d.w; ++j)
        for (int i = 0; i < d.w; ++i) {
          const long c = (d.x + i) + (long)nx * ((d.y + j) + (long)ny * (d.z + k));
          cmap[c] = (i | j | k) ? e : (int32_t)((uint32_t)e | 0x80000000u);
        }
  }
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

// ------------------------------------------------------------------ design difference
// Eq. (10) on the finest lattice: each cell takes the density of the leaf
// covering it (uniform brick: the element of the same index); per block the
// sums of |rho_a - rho_b| and rho_a over a fixed cell range, then one block
// adds the partials in order.
__global__ __launch_bounds__(256) void k_design_diff(const double* __restrict__ ra, const int32_t* __restrict__ cmap_a,
                                                     const double* __restrict__ rb, const int32_t* __restrict__ cmap_b,
                                                     long cells, double* __restrict__ part) {
  __shared__ double sh[16];
  double num = 0.0, den = 0.0;
  for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < cells; c += (long)gridDim.x * blockDim.x) {
    const long ea = cmap_a ? (long)(cmap_a[c] & 0x7fffffff) : c;
    const long eb = cmap_b ? (long)(cmap_b[c] & 0x7fffffff) : c;
    const double a = ra[ea];
    num += fabs(a - rb[eb]);
    den += a;
  }
  num = block_sum_t(num, sh);
  den = block_sum_t(den, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = num;
    part[gridDim.x + blockIdx.x] = den;
  }
}

__global__ __launch_bounds__(256) void k_design_diff_sum(const double* __restrict__ part, int nb,
                                                         double* __restrict__ out) {
  __shared__ double sh[16];
  double num = 0.0, den = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    num += part[i];
    den += part[nb + i];
  }
  num = block_sum_t(num, sh);
  den = block_sum_t(den, sh);
  if (threadIdx.x == 0) {
    out[0] = num;
    out[1] = den;
  }
}

// ------------------------------------------------------------------ OC scratch
// Workspace of amrto_oc_update_noalloc: a file-scope device array (one copy
// per GPU, held until the process ends) instead of the context's buffer.
// Host code never passes `scratch` itself to a kernel: its device address on
// each GPU comes from hipGetSymbolAddress at context creation.
constexpr int OC_SCRATCH_DEVICES = 64;
static __device__ __align__(256) double scratch[OC_WS];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[OC_SCRATCH_DEVICES] = {};

// Called by amrto_create with ctx->device current: looks the array's address
// up once per device and keeps it in the context.
int oc_scratch_attach(amrto_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= OC_SCRATCH_DEVICES)
    return ctx->fail(AMRTO_EINVAL, "amrto_create: device index above the OC scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* ptr = nullptr;
    AMRTO_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return ctx->fail(AMRTO_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[ctx->device] = ptr;
  }
  ctx->d_oc_scratch = (double*)g_scratch_ptr[ctx->device];
  return AMRTO_OK;
}

// ------------------------------------------------------------------ host
// Element descriptors and the lattice cell map of an octree mesh, built at
// mesh upload (the filter reads them; no per-call host work).
int build_cell_map(amrto_ctx* ctx) {
  const int ne = ctx->n_elems;
  const long cells = (long)ctx->nx * ctx->ny * ctx->nz;
  if (cells > (1L << 30))
    return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: finest lattice above 2^30 cells (filter cell map)");
  std::vector<int32_t> desc(4L * ne);
  int hmax = 1;
  for (int e = 0; e < ne; ++e) {
    const int n0 = ctx->h_elem_nodes[8L * e];
    const int h = 1 << (ctx->max_level - ctx->h_level[e]);
    for (int a = 0; a < 3; ++a) desc[4L * e + a] = ctx->h_node_xyz[3L * n0 + a];
    desc[4L * e + 3] = h;
    hmax = std::max(hmax, h);
  }
  ctx->filt_hmax = hmax;
  AMRTO_HIP(hipMalloc((void**)&ctx->d_edesc, std::max<size_t>(1, desc.size()) * sizeof(int32_t)));
  AMRTO_HIP(hipMalloc((void**)&ctx->d_cmap, std::max<long>(1, cells) * sizeof(int32_t)));
  AMRTO_HIP(hipMemcpyAsync(ctx->d_edesc, desc.data(), desc.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           ctx->stream));
  hipLaunchKernelGGL(k_cell_map, dim3(grid_for(ne, 256, 4096)), dim3(256), 0, ctx->stream, (const int4*)ctx->d_edesc,
                     ne, ctx->nx, ctx->ny, ctx->d_cmap);
  AMRTO_HIP(hipGetLastError());
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));  // desc is a host temporary
  return AMRTO_OK;
}

// The OC step on workspace ws (OC_WS doubles on the device); host results
// come back through hbuf (4 doubles).
static int oc_update_ws(amrto_ctx* ctx, double* ws, double* hbuf, const char* name, const double* rho,
                        const double* dc, double volfrac, double move, double eta, double rho_min, double* rho_new,
                        double* change_host, double* lam_host) {
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, std::string(name) + ": no mesh");
  if (!rho || !dc || !rho_new || rho_new == rho) return ctx->fail(AMRTO_EINVAL, std::string(name) + ": bad buffers");
  if (!(volfrac > 0.0 && volfrac <= 1.0) || !(move > 0.0) || !(eta > 0.0) || !(rho_min >= 0.0 && rho_min < 1.0))
    return ctx->fail(AMRTO_EINVAL, std::string(name) + ": bad parameters");
  AMRTO_HIP(hipSetDevice(ctx->device));
  const int ne = ctx->n_elems;
  double vtot = 0.0;
  for (int e = 0; e < ne; ++e) {
    const double h = (double)(1 << (ctx->max_level - ctx->h_level[e]));
    vtot += h * h * h;
  }
  const double v0 = volfrac * vtot;
  const int nblk = std::min(OC_BLOCKS, (ne + OC_TILE - 1) / OC_TILE);
  const int g = std::min(256, (ne + 255) / 256);
  // workspace layout: bracket [0, 2), partial volumes [2, 2 + OC_K nblk),
  // candidate volumes [OC_VOL, OC_VOL + OC_K), per-block changes [2, 2 + g)
  if (OC_VOL + OC_K > OC_WS || 2 + (long)OC_K * nblk > OC_VOL || 2 + g > OC_VOL)
    return ctx->fail(AMRTO_EINVAL, std::string(name) + ": workspace layout exceeds its size");
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
  hipLaunchKernelGGL(k_oc_apply, dim3(g), dim3(256), 0, ctx->stream, rho, dc, ctx->d_vol, ne, eta, move, rho_min,
                     rho_new, ws);
  hipLaunchKernelGGL(k_oc_finish, dim3(1), dim3(256), 0, ctx->stream, ws, g);
  AMRTO_HIP(hipGetLastError());
  if (change_host || lam_host) {
    AMRTO_HIP(hipMemcpyAsync(hbuf, ws, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    AMRTO_HIP(hipStreamSynchronize(ctx->stream));
    if (change_host) *change_host = hbuf[2];
    if (lam_host) *lam_host = hbuf[3];
  }
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
  if (!(rmin > 0.0) || rmin > (double)FILT_RMAX) return ctx->fail(AMRTO_EINVAL, "amrto_filter: rmin must be in (0, 16]");
  if (!in || !out || in == out || (mode == AMRTO_FILTER_SENSITIVITY && !rho))
    return ctx->fail(AMRTO_EINVAL, "amrto_filter: bad buffers");
  AMRTO_HIP(hipSetDevice(ctx->device));
  const int ne = ctx->n_elems;
  if (ctx->uniform) {
    const int R = std::min(FILT_RMAX, (int)std::ceil(rmin));
    hipLaunchKernelGGL(k_filter_uniform, dim3((ne + 255) / 256), dim3(256), 0, ctx->stream, in, rho, out, ctx->nx,
                       ctx->ny, ctx->nz, rmin, R, mode);
  } else {
    hipLaunchKernelGGL(k_filter_octree, dim3((ne + 255) / 256), dim3(256), 0, ctx->stream, in, rho, out,
                       (const int4*)ctx->d_edesc, ctx->d_cmap, ne, ctx->nx, ctx->ny, ctx->nz, ctx->filt_hmax, rmin,
                       mode);
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_oc_update(amrto_ctx* ctx, const double* rho, const double* dc, double volfrac, double move, double eta,
                    double rho_min, double* rho_new, double* change_host, double* lam_host) {
  if (!ctx) return AMRTO_EINVAL;
  double h[4];
  return oc_update_ws(ctx, ctx->d_oc, h, "amrto_oc_update", rho, dc, volfrac, move, eta, rho_min, rho_new,
                      change_host, lam_host);
}

int amrto_oc_update_noalloc(amrto_ctx* ctx, const double* rho, const double* dc, double volfrac, double move,
                            double eta, double rho_min, double* rho_new, double* change_host, double* lam_host) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->d_oc_scratch) return ctx->fail(AMRTO_ESTATE, "amrto_oc_update_noalloc: scratch address not set");
  // the context's pinned scalar mirror receives the host results (slots
  // 0-3; no solve is running while this call synchronises)
  return oc_update_ws(ctx, ctx->d_oc_scratch, ctx->h_scal, "amrto_oc_update_noalloc", rho, dc, volfrac, move, eta,
                      rho_min, rho_new, change_host, lam_host);
}

int amrto_design_difference(amrto_ctx* a, const double* rho_a, const amrto_ctx* b, const double* rho_b,
                            double* D_host) {
  if (!a || !b) return AMRTO_EINVAL;
  amrto_ctx* ctx = a;
  if (!a->has_mesh || !b->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_design_difference: no mesh");
  if (!rho_a || !rho_b || !D_host) return ctx->fail(AMRTO_EINVAL, "amrto_design_difference: NULL argument");
  if (a->device != b->device) return ctx->fail(AMRTO_EINVAL, "amrto_design_difference: contexts on different devices");
  if (a->nx != b->nx || a->ny != b->ny || a->nz != b->nz)
    return ctx->fail(AMRTO_EINVAL, "amrto_design_difference: meshes cover different lattice boxes");
  AMRTO_HIP(hipSetDevice(ctx->device));
  const long cells = (long)a->nx * a->ny * a->nz;
  const int nb = grid_for(cells, 256, RED_BLOCKS);
  // b's mesh and densities are read on a's stream: b's earlier work must be
  // complete (its calls that return host values synchronise)
  hipLaunchKernelGGL(k_design_diff, dim3(nb), dim3(256), 0, ctx->stream, rho_a, a->uniform ? nullptr : a->d_cmap,
                     rho_b, b->uniform ? nullptr : b->d_cmap, cells, ctx->d_part);
  hipLaunchKernelGGL(k_design_diff_sum, dim3(1), dim3(256), 0, ctx->stream, ctx->d_part, nb, ctx->d_scal + 6);
  AMRTO_HIP(hipGetLastError());
  AMRTO_HIP(hipMemcpyAsync(ctx->h_scal, ctx->d_scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  *D_host = ctx->h_scal[6] / ctx->h_scal[7];
  return AMRTO_OK;
}

}  // extern "C"
