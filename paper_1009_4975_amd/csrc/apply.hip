// Matrix-free application of the constrained stiffness operator
//   y = A~ x,  A~ = F T^T K T F + (I - F),   K = sum_e c_e G_e^T K0 G_e
// (paper Sec. 6, Eq. (6)-(8); supported DOFs as identity rows) and the exact
// diagonal of A~ used by the Jacobi preconditioner (the diagonal rescaling
// of Sec. 5).
//
// Two data paths:
//  * uniform brick: implicit connectivity.  A workgroup owns a UT x UT block
//    of node columns over a range of node layers, computes the surrounding
//    (UT+1)^2 element columns one element per thread, marches up one element
//    layer at a time with two node layers of x staged in LDS, and writes every
//    owned node exactly once (no global atomics, deterministic).
//  * octree: elements in space-filling-curve order are cut into chunks whose
//    node tables (vertices plus masters of hanging vertices) fit in LDS.  The
//    hanging interpolation x_h = P x_m and the condensation y_m += P^T y_h
//    happen inside the chunk.  Nodes referenced by one chunk only are stored
//    directly; shared nodes go to per-(chunk, node) slots that a second pass
//    adds in a fixed order (deterministic, no global atomics).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace amrto {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so neighbouring tiles share an L2.
  int per = (nb + 7) >> 3;
  int x = b & 7, i = b >> 3;
  return x * per + i;
}

template <typename T>
__device__ __forceinline__ void contract_valu(const T* __restrict__ K0, const T (&u)[24], T (&out)[24], T s) {
#pragma unroll
  for (int r = 0; r < 24; ++r) {
    T acc = 0;
#pragma unroll
    for (int c = 0; c < 24; ++c) acc = fma(K0[r * 24 + c], u[c], acc);
    out[r] = acc * s;
  }
}

// ------------------------------------------------------------------ uniform brick
template <typename VT>
__global__ __launch_bounds__(256) void k_apply_uniform(
    const VT* __restrict__ x, VT* __restrict__ y, const VT* __restrict__ coef,
    const uint8_t* __restrict__ fix, const VT* __restrict__ K0, int nx, int ny, int nz,
    int tiles_x, int tiles_y, int zchunk, int n_tiles, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ VT xs[2][UN * UN * 3];
  __shared__ VT ys[2][UT * UT * 3];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  if (tile >= n_tiles) return;
  const int tx = tile % tiles_x;
  const int ty = (tile / tiles_x) % tiles_y;
  const int tz = tile / (tiles_x * tiles_y);
  const int ox = tx * UT, oy = ty * UT;  // first owned node column
  const int z0 = tz * zchunk;
  const int z1 = min(z0 + zchunk, nz + 1);  // owned node layers [z0, z1)
  const int tid = threadIdx.x;
  const int i = tid % UE, j = tid / UE;
  const int ex = ox - 1 + i, ey = oy - 1 + j;
  const bool ev = ex >= 0 && ex < nx && ey >= 0 && ey < ny;
  const long sx = nx + 1, sxy = (long)(nx + 1) * (ny + 1);

  auto load_layer = [&](int buf, int k) {
    for (int idx = tid; idx < UN * UN * 3; idx += 256) {
      const int c = idx % 3, nd = idx / 3;
      const int gx = ox - 1 + nd % UN, gy = oy - 1 + nd / UN;
      VT v = 0;
      if (gx >= 0 && gx <= nx && gy >= 0 && gy <= ny) {
        const long node = gx + sx * gy + sxy * k;
        if (!((fix[node] >> c) & 1)) v = x[3 * node + c];
      }
      xs[buf][idx] = v;
    }
  };
  auto store_layer = [&](int buf, int k) {
    for (int idx = tid; idx < UT * UT * 3; idx += 256) {
      const int c = idx % 3, nd = idx / 3;
      const int gx = ox + nd % UT, gy = oy + nd / UT;
      if (gx <= nx && gy <= ny) {
        const long node = gx + sx * gy + sxy * k;
        VT v = ys[buf][idx];
        if ((fix[node] >> c) & 1) v = x[3 * node + c];
        y[3 * node + c] = v;
      }
      ys[buf][idx] = 0;
    }
  };

  for (int idx = tid; idx < UT * UT * 3; idx += 256) { ys[0][idx] = 0; ys[1][idx] = 0; }
  const int kbeg = max(z0 - 1, 0);
  const int kend = min(z1 - 1, nz - 1);
  int cur = 0;
  load_layer(cur, kbeg);
  for (int k = kbeg; k <= kend; ++k) {
    load_layer(cur ^ 1, k + 1);
    __syncthreads();
    if (ev) {
      VT u[24], out[24];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int l = ((j + ((a >> 1) & 1)) * UN + i + (a & 1)) * 3;
        const VT* src = xs[(a >> 2) ? (cur ^ 1) : cur];
        u[3 * a + 0] = src[l + 0];
        u[3 * a + 1] = src[l + 1];
        u[3 * a + 2] = src[l + 2];
      }
      const VT ce = coef[ex + (long)nx * (ey + (long)ny * k)];
      contract_valu<VT>(K0, u, out, ce);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int li = i + (a & 1) - 1, lj = j + ((a >> 1) & 1) - 1;
        const int layer = k + (a >> 2);
        if (li >= 0 && li < UT && lj >= 0 && lj < UT && layer >= z0 && layer < z1) {
          VT* dst = &ys[layer & 1][(lj * UT + li) * 3];
          atomicAdd(dst + 0, out[3 * a + 0]);
          atomicAdd(dst + 1, out[3 * a + 1]);
          atomicAdd(dst + 2, out[3 * a + 2]);
        }
      }
    }
    __syncthreads();
    if (k >= z0) store_layer(k & 1, k);  // node layer k has all its elements
    cur ^= 1;
  }
  if (kend + 1 < z1 && kend + 1 >= z0) {  // top node layer of the brick
    __syncthreads();
    store_layer((kend + 1) & 1, kend + 1);
  }
}

// ------------------------------------------------------------------ octree chunks
struct ChunkArgs {
  const int32_t* chunk_elem;
  const int32_t* chunk_tab;
  const int32_t* chunk_nreg;
  const int32_t* chunk_trip;
  const int32_t* tab_node;
  const int32_t* tab_slot;
  const uint16_t* elem_loc;
  const uint32_t* trip_hm;
  const double* trip_w;
  int n_chunks;
};

template <typename VT>
__global__ __launch_bounds__(256) void k_apply_chunks(
    const VT* __restrict__ x, VT* __restrict__ y, VT* __restrict__ partial,
    const VT* __restrict__ coef, const uint8_t* __restrict__ fix, const VT* __restrict__ K0,
    ChunkArgs ca, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ VT xs[TAB_MAX * 3];
  __shared__ VT ys[TAB_MAX * 3];
  const int c = xcd_remap(blockIdx.x, gridDim.x);
  if (c >= ca.n_chunks) return;
  const int tid = threadIdx.x;
  const int e0 = ca.chunk_elem[c], e1 = ca.chunk_elem[c + 1];
  const int t0 = ca.chunk_tab[c], nt = ca.chunk_tab[c + 1] - t0, nreg = ca.chunk_nreg[c];
  const int h0 = ca.chunk_trip[c], nh = ca.chunk_trip[c + 1] - h0;
  for (int i = tid; i < nt * 3; i += 256) {
    const int t = i / 3, comp = i % 3;
    VT v = 0;
    if (t < nreg) {
      const int node = ca.tab_node[t0 + t];
      if (!((fix[node] >> comp) & 1)) v = x[3L * node + comp];
    }
    xs[i] = v;
    ys[i] = 0;
  }
  __syncthreads();
  for (int i = tid; i < nh * 3; i += 256) {  // x_h = sum_m w_hm x_m  (Eq. (6))
    const int k = i / 3, comp = i % 3;
    const uint32_t hm = ca.trip_hm[h0 + k];
    const int h = hm >> 16, m = hm & 0xffff;
    atomicAdd(&xs[h * 3 + comp], (VT)ca.trip_w[h0 + k] * xs[m * 3 + comp]);
  }
  __syncthreads();
  const int e = e0 + tid;
  if (e < e1) {
    int loc[8];
    const uint4 lv = *reinterpret_cast<const uint4*>(ca.elem_loc + 8L * e);
    loc[0] = lv.x & 0xffff; loc[1] = lv.x >> 16; loc[2] = lv.y & 0xffff; loc[3] = lv.y >> 16;
    loc[4] = lv.z & 0xffff; loc[5] = lv.z >> 16; loc[6] = lv.w & 0xffff; loc[7] = lv.w >> 16;
    VT u[24], out[24];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      u[3 * a + 0] = xs[loc[a] * 3 + 0];
      u[3 * a + 1] = xs[loc[a] * 3 + 1];
      u[3 * a + 2] = xs[loc[a] * 3 + 2];
    }
    contract_valu<VT>(K0, u, out, coef[e]);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      atomicAdd(&ys[loc[a] * 3 + 0], out[3 * a + 0]);
      atomicAdd(&ys[loc[a] * 3 + 1], out[3 * a + 1]);
      atomicAdd(&ys[loc[a] * 3 + 2], out[3 * a + 2]);
    }
  }
  __syncthreads();
  for (int i = tid; i < nh * 3; i += 256) {  // y_m += w_hm y_h  (P^T of Eq. (7))
    const int k = i / 3, comp = i % 3;
    const uint32_t hm = ca.trip_hm[h0 + k];
    const int h = hm >> 16, m = hm & 0xffff;
    atomicAdd(&ys[m * 3 + comp], (VT)ca.trip_w[h0 + k] * ys[h * 3 + comp]);
  }
  __syncthreads();
  for (int i = tid; i < nreg * 3; i += 256) {
    const int t = i / 3, comp = i % 3;
    const int node = ca.tab_node[t0 + t];
    const int slot = ca.tab_slot[t0 + t];
    VT v = ys[i];
    if (slot < 0) {
      if ((fix[node] >> comp) & 1) v = x[3L * node + comp];
      y[3L * node + comp] = v;
    } else {
      partial[3L * slot + comp] = v;
    }
  }
}

// Shared nodes: add the chunk slots in chunk order; hanging nodes: identity.
template <typename VT>
__global__ __launch_bounds__(256) void k_reduce_shared(
    const VT* __restrict__ x, VT* __restrict__ y, const VT* __restrict__ partial,
    const uint8_t* __restrict__ fix, const int32_t* __restrict__ shared_node,
    const int32_t* __restrict__ shared_ptr, const int32_t* __restrict__ slot_list, int n_shared,
    const int32_t* __restrict__ hang_node, int n_hang, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long n1 = 3L * n_shared;
  if (i < n1) {
    const int s = (int)(i / 3), comp = (int)(i % 3);
    const int node = shared_node[s];
    VT v = 0;
    for (int k = shared_ptr[s]; k < shared_ptr[s + 1]; ++k) v += partial[3L * slot_list[k] + comp];
    if ((fix[node] >> comp) & 1) v = x[3L * node + comp];
    y[3L * node + comp] = v;
  } else if (i < n1 + 3L * n_hang) {
    const long k = i - n1;
    const int node = hang_node[k / 3], comp = (int)(k % 3);
    y[3L * node + comp] = x[3L * node + comp];
  }
}

// ------------------------------------------------------------------ diagonal
// Uniform brick: diag = K0[0][0] * sum of c_e over the node's elements
// (every diagonal entry of K0 equals (lambda + 4 mu) / 9).
__global__ __launch_bounds__(256) void k_diag_uniform(
    const double* __restrict__ coef, const uint8_t* __restrict__ fix, double k00,
    double* __restrict__ dinv, int nx, int ny, int nz) {
  const long n = (long)(nx + 1) * (ny + 1) * (nz + 1);
  const long node = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (node >= n) return;
  const int gx = node % (nx + 1);
  const int gy = (node / (nx + 1)) % (ny + 1);
  const int gz = node / ((long)(nx + 1) * (ny + 1));
  double s = 0.0;
  for (int dz = -1; dz <= 0; ++dz)
    for (int dy = -1; dy <= 0; ++dy)
      for (int dx = -1; dx <= 0; ++dx) {
        const int ex = gx + dx, ey = gy + dy, ez = gz + dz;
        if (ex >= 0 && ex < nx && ey >= 0 && ey < ny && ez >= 0 && ez < nz)
          s += coef[ex + (long)nx * (ey + (long)ny * ez)];
      }
  const double d = k00 * s;
  for (int c = 0; c < 3; ++c) dinv[3 * node + c] = ((fix[node] >> c) & 1) ? 1.0 : 1.0 / d;
}

// Octree: per element and component, sum c_e t_a t_b K0[(a,c),(b,c)] over the
// pairs of (vertex a, master m, weight t) expansions that share a master m:
// the diagonal of T^T K T including the cross terms that hanging vertices
// create.  Results use the same exclusive/slot output as the operator.
__global__ __launch_bounds__(256) void k_diag_chunks(
    double* __restrict__ diag, double* __restrict__ partial, const double* __restrict__ coef,
    const double* __restrict__ K0, ChunkArgs ca) {
  __shared__ double ds[TAB_MAX * 3];
  const int c = blockIdx.x;
  if (c >= ca.n_chunks) return;
  const int tid = threadIdx.x;
  const int e0 = ca.chunk_elem[c], e1 = ca.chunk_elem[c + 1];
  const int t0 = ca.chunk_tab[c], nt = ca.chunk_tab[c + 1] - t0, nreg = ca.chunk_nreg[c];
  const int h0 = ca.chunk_trip[c], nh = ca.chunk_trip[c + 1] - h0;
  for (int i = tid; i < nt * 3; i += 256) ds[i] = 0.0;
  __syncthreads();
  const int e = e0 + tid;
  if (e < e1) {
    int ent_m[64], ent_a[64];
    double ent_w[64];
    int ne = 0;
    for (int a = 0; a < 8; ++a) {
      const int l = ca.elem_loc[8L * e + a];
      if (l < nreg) {
        ent_m[ne] = l; ent_a[ne] = a; ent_w[ne] = 1.0; ++ne;
      } else {
        for (int k = 0; k < nh && ne < 64; ++k) {
          const uint32_t hm = ca.trip_hm[h0 + k];
          if ((int)(hm >> 16) == l) {
            ent_m[ne] = hm & 0xffff; ent_a[ne] = a; ent_w[ne] = ca.trip_w[h0 + k]; ++ne;
          }
        }
      }
    }
    const double ce = coef[e];
    for (int p = 0; p < ne; ++p)
      for (int q = 0; q < ne; ++q) {
        if (ent_m[p] != ent_m[q]) continue;
        const double w = ce * ent_w[p] * ent_w[q];
        for (int cc = 0; cc < 3; ++cc)
          atomicAdd(&ds[ent_m[p] * 3 + cc], w * K0[(3 * ent_a[p] + cc) * 24 + 3 * ent_a[q] + cc]);
      }
  }
  __syncthreads();
  for (int i = tid; i < nreg * 3; i += 256) {
    const int t = i / 3, comp = i % 3;
    const int node = ca.tab_node[t0 + t];
    const int slot = ca.tab_slot[t0 + t];
    if (slot < 0) diag[3L * node + comp] = ds[i];
    else partial[3L * slot + comp] = ds[i];
  }
}

__global__ __launch_bounds__(256) void k_diag_finish(
    double* __restrict__ diag, const double* __restrict__ partial, const uint8_t* __restrict__ fix,
    const int32_t* __restrict__ shared_node, const int32_t* __restrict__ shared_ptr,
    const int32_t* __restrict__ slot_list, int n_shared, const int32_t* __restrict__ hang_node,
    int n_hang, int n_nodes, int phase) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (phase == 0) {  // sum slots of shared nodes, identity for hanging nodes
    const long n1 = 3L * n_shared;
    if (i < n1) {
      const int s = (int)(i / 3), comp = (int)(i % 3);
      double v = 0.0;
      for (int k = shared_ptr[s]; k < shared_ptr[s + 1]; ++k) v += partial[3L * slot_list[k] + comp];
      diag[3L * shared_node[s] + comp] = v;
    } else if (i < n1 + 3L * n_hang) {
      const long k = i - n1;
      diag[3L * hang_node[k / 3] + k % 3] = 1.0;
    }
  } else {  // invert; supported DOFs are identity rows
    if (i < 3L * n_nodes) {
      const int node = (int)(i / 3), comp = (int)(i % 3);
      const double d = diag[i];
      diag[i] = ((fix[node] >> comp) & 1) ? 1.0 : 1.0 / d;
    }
  }
}

__global__ void k_to_float(const double* __restrict__ a, float* __restrict__ b, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------------ host side
static ChunkArgs chunk_args(amrto_ctx* ctx) {
  ChunkArgs a;
  a.chunk_elem = ctx->d_chunk_elem; a.chunk_tab = ctx->d_chunk_tab; a.chunk_nreg = ctx->d_chunk_nreg;
  a.chunk_trip = ctx->d_chunk_trip; a.tab_node = ctx->d_tab_node; a.tab_slot = ctx->d_tab_slot;
  a.elem_loc = ctx->d_elem_loc; a.trip_hm = ctx->d_trip_hm; a.trip_w = ctx->d_trip_w;
  a.n_chunks = ctx->n_chunks;
  return a;
}

template <typename VT>
void reduce_shared(amrto_ctx* ctx, const VT* x, VT* y, const double* stop);

void uniform_grid(const amrto_ctx* ctx, int& tiles_x, int& tiles_y, int& zchunk, int& n_tiles, int& grid) {
  tiles_x = (ctx->nx + 1 + UT - 1) / UT;
  tiles_y = (ctx->ny + 1 + UT - 1) / UT;
  const int layers = ctx->nz + 1;
  // aim for ~4 workgroups per CU (256 CUs) with at least 4 layers per chunk
  const int want = 1024;
  int nzc = std::max(1, want / std::max(1, tiles_x * tiles_y));
  zchunk = std::max(4, (layers + nzc - 1) / nzc);
  nzc = (layers + zchunk - 1) / zchunk;
  n_tiles = tiles_x * tiles_y * nzc;
  grid = ((n_tiles + 7) / 8) * 8;
}

template <typename VT>
static int apply_t(amrto_ctx* ctx, const VT* x, VT* y, const VT* coef, const VT* K0, const double* stop) {
  if (ctx->uniform) {
    int tx, ty, zc, nt, grid;
    uniform_grid(ctx, tx, ty, zc, nt, grid);
    hipLaunchKernelGGL(k_apply_uniform<VT>, dim3(grid), dim3(256), 0, ctx->stream, x, y, coef,
                       ctx->d_fix, K0, ctx->nx, ctx->ny, ctx->nz, tx, ty, zc, nt, stop);
  } else {
    const int grid = ((ctx->n_chunks + 7) / 8) * 8;
    hipLaunchKernelGGL(k_apply_chunks<VT>, dim3(grid), dim3(256), 0, ctx->stream, x, y,
                       (VT*)ctx->d_partial, coef, ctx->d_fix, K0, chunk_args(ctx), stop);
    reduce_shared<VT>(ctx, x, y, stop);
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

template <typename VT>
void reduce_shared(amrto_ctx* ctx, const VT* x, VT* y, const double* stop) {
  const long n = 3L * (ctx->n_shared + ctx->n_hang);
  if (n > 0)
    hipLaunchKernelGGL(k_reduce_shared<VT>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, x, y,
                       (const VT*)ctx->d_partial, ctx->d_fix, ctx->d_shared_node, ctx->d_shared_ptr,
                       ctx->d_slot_list, ctx->n_shared, ctx->d_hang_node, ctx->n_hang, stop);
}
template void reduce_shared<float>(amrto_ctx*, const float*, float*, const double*);
template void reduce_shared<double>(amrto_ctx*, const double*, double*, const double*);

ChunkArgs chunk_args_of(amrto_ctx* ctx) { return chunk_args(ctx); }

int apply_stop(amrto_ctx* ctx, const void* x, void* y, int prec, const double* stop) {
  if (prec == AMRTO_FP64)
    return apply_t<double>(ctx, (const double*)x, (double*)y, ctx->d_coef, ctx->d_K0, stop);
  if (prec == AMRTO_FP32)
    return apply_t<float>(ctx, (const float*)x, (float*)y, ctx->d_coef_f, ctx->d_K0f, stop);
  return launch_apply_bf16(ctx, (const float*)x, (float*)y, stop);
}

int launch_apply(amrto_ctx* ctx, const void* x, void* y, int prec) {
  return apply_stop(ctx, x, y, prec, nullptr);
}

int launch_diag(amrto_ctx* ctx) {
  const long n3 = 3L * ctx->n_nodes;
  if (ctx->uniform) {
    const long n = ctx->n_nodes;
    hipLaunchKernelGGL(k_diag_uniform, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_coef,
                       ctx->d_fix, ctx->K0[0], ctx->d_dinv, ctx->nx, ctx->ny, ctx->nz);
  } else {
    hipLaunchKernelGGL(k_diag_chunks, dim3(ctx->n_chunks), dim3(256), 0, ctx->stream, ctx->d_dinv,
                       ctx->d_partial, ctx->d_coef, ctx->d_K0, chunk_args(ctx));
    const long n = 3L * (ctx->n_shared + ctx->n_hang);
    if (n > 0)
      hipLaunchKernelGGL(k_diag_finish, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_dinv,
                         ctx->d_partial, ctx->d_fix, ctx->d_shared_node, ctx->d_shared_ptr,
                         ctx->d_slot_list, ctx->n_shared, ctx->d_hang_node, ctx->n_hang, ctx->n_nodes, 0);
    hipLaunchKernelGGL(k_diag_finish, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_dinv,
                       ctx->d_partial, ctx->d_fix, ctx->d_shared_node, ctx->d_shared_ptr, ctx->d_slot_list,
                       ctx->n_shared, ctx->d_hang_node, ctx->n_hang, ctx->n_nodes, 1);
  }
  hipLaunchKernelGGL(k_to_float, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_dinv,
                     ctx->d_dinv_f, n3);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

// Cut the element sequence into chunks whose node tables fit TAB_MAX entries,
// order each table (regular nodes, then hanging ones), express hanging
// interpolation as (hanging entry, master entry, weight) triples, and give
// every node referenced by two or more chunks one partial slot per chunk.
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
  std::vector<int> stamp(nn, -1), loc(nn, 0);
  std::vector<int> chunk_elem{0}, chunk_tab{0}, chunk_nreg, chunk_trip{0};
  std::vector<int> tab_node;
  std::vector<uint16_t> elem_loc(8L * ne);
  std::vector<uint32_t> trip_hm;
  std::vector<double> trip_w;
  std::vector<int> cur;  // current chunk table (global nodes, insertion order)
  int cid = 0, cur_e0 = 0;

  auto close_chunk = [&](int e_end) -> int {
    // order: regular entries first, hanging entries after
    std::vector<int> reg, hng;
    for (int v : cur) (hidx[v] < 0 ? reg : hng).push_back(v);
    const int nreg = (int)reg.size();
    for (int i = 0; i < nreg; ++i) loc[reg[i]] = i;
    for (size_t i = 0; i < hng.size(); ++i) loc[hng[i]] = nreg + (int)i;
    for (int e = cur_e0; e < e_end; ++e)
      for (int a = 0; a < 8; ++a) elem_loc[8L * e + a] = (uint16_t)loc[m->elem_nodes[8L * e + a]];
    for (size_t i = 0; i < hng.size(); ++i) {
      const int hi = hidx[hng[i]];
      for (int k = m->hang_ptr[hi]; k < m->hang_ptr[hi + 1]; ++k) {
        trip_hm.push_back(((uint32_t)(nreg + i) << 16) | (uint32_t)loc[m->hang_master[k]]);
        trip_w.push_back(m->hang_w[k]);
      }
    }
    for (int v : reg) tab_node.push_back(v);
    for (int v : hng) tab_node.push_back(v);
    chunk_nreg.push_back(nreg);
    chunk_tab.push_back((int)tab_node.size());
    chunk_trip.push_back((int)trip_hm.size());
    chunk_elem.push_back(e_end);
    cur.clear();
    cur_e0 = e_end;
    ++cid;
    return 0;
  };

  std::vector<int> need, uniq;
  for (int e = 0; e < ne; ++e) {
    need.clear();
    for (int a = 0; a < 8; ++a) {
      const int v = m->elem_nodes[8L * e + a];
      need.push_back(v);
      if (hidx[v] >= 0)
        for (int k = m->hang_ptr[hidx[v]]; k < m->hang_ptr[hidx[v] + 1]; ++k) need.push_back(m->hang_master[k]);
    }
    uniq = need;
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    if ((int)uniq.size() > TAB_MAX)
      return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: element needs more nodes than a chunk table holds");
    int fresh = 0;
    for (int v : uniq) fresh += (stamp[v] != cid);
    if (e - cur_e0 >= CH_MAX || (int)cur.size() + fresh > TAB_MAX) close_chunk(e);
    for (int v : uniq)
      if (stamp[v] != cid) { stamp[v] = cid; cur.push_back(v); }
  }
  if (!cur.empty() || cur_e0 < ne) close_chunk(ne);
  const int nc = cid;

  // reference counts of regular nodes over chunks -> exclusive or shared
  std::vector<int> cnt(nn, 0);
  for (int c = 0; c < nc; ++c)
    for (int t = chunk_tab[c]; t < chunk_tab[c] + chunk_nreg[c]; ++t) cnt[tab_node[t]]++;
  for (int v = 0; v < nn; ++v)
    if (hidx[v] < 0 && cnt[v] == 0)
      return ctx->fail(AMRTO_EINVAL, "amrto_upload_mesh: a node belongs to no element");
  std::vector<int> tab_slot(tab_node.size(), -1);
  std::vector<int> shared_id(nn, -1), shared_node;
  for (int v = 0; v < nn; ++v)
    if (cnt[v] >= 2) { shared_id[v] = (int)shared_node.size(); shared_node.push_back(v); }
  std::vector<int> shared_ptr(shared_node.size() + 1, 0);
  for (size_t s = 0; s < shared_node.size(); ++s) shared_ptr[s + 1] = shared_ptr[s] + cnt[shared_node[s]];
  std::vector<int> fill(shared_node.size(), 0), slot_list(shared_ptr.back());
  int n_slots = 0;
  for (int c = 0; c < nc; ++c)
    for (int t = chunk_tab[c]; t < chunk_tab[c] + chunk_nreg[c]; ++t) {
      const int v = tab_node[t];
      if (shared_id[v] >= 0) {
        const int s = shared_id[v];
        tab_slot[t] = n_slots;
        slot_list[shared_ptr[s] + fill[s]++] = n_slots;
        ++n_slots;
      }
    }
  auto up = [&](auto*& dst, const auto& v) -> hipError_t {
    using T = typename std::remove_reference<decltype(v)>::type::value_type;
    if (dst) (void)hipFree(dst);
    dst = nullptr;
    hipError_t e = hipMalloc((void**)&dst, std::max<size_t>(1, v.size()) * sizeof(T));
    if (e != hipSuccess) return e;
    if (!v.empty()) e = hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
  };
  // transpose of the hanging interpolation: master -> (hanging node, weight)
  std::vector<int> mt_count(nn, 0);
  for (int i = 0; i < m->n_hang; ++i)
    for (int k = m->hang_ptr[i]; k < m->hang_ptr[i + 1]; ++k) mt_count[m->hang_master[k]]++;
  std::vector<int> mt_node, mt_ptr{0}, mt_h;
  std::vector<double> mt_w;
  std::vector<int> mt_pos(nn, -1);
  for (int v = 0; v < nn; ++v)
    if (mt_count[v] > 0) {
      mt_pos[v] = mt_ptr.back();
      mt_node.push_back(v);
      mt_ptr.push_back(mt_ptr.back() + mt_count[v]);
    }
  mt_h.resize(mt_ptr.back());
  mt_w.resize(mt_ptr.back());
  for (int i = 0; i < m->n_hang; ++i)
    for (int k = m->hang_ptr[i]; k < m->hang_ptr[i + 1]; ++k) {
      const int mm = m->hang_master[k];
      mt_h[mt_pos[mm]] = m->hang_node[i];
      mt_w[mt_pos[mm]] = m->hang_w[k];
      mt_pos[mm]++;
    }
  AMRTO_HIP(up(ctx->d_mt_node, mt_node));
  AMRTO_HIP(up(ctx->d_mt_ptr, mt_ptr));
  AMRTO_HIP(up(ctx->d_mt_h, mt_h));
  AMRTO_HIP(up(ctx->d_mt_w, mt_w));
  ctx->n_mt = (int)mt_node.size();
  std::vector<int> hang_node(m->hang_node, m->hang_node + m->n_hang);
  std::vector<int> hang_ptr(m->hang_ptr, m->hang_ptr + m->n_hang + 1);
  const int nhe = m->n_hang ? m->hang_ptr[m->n_hang] : 0;
  std::vector<int> hang_master(m->hang_master, m->hang_master + nhe);
  std::vector<double> hang_w(m->hang_w, m->hang_w + nhe);

  AMRTO_HIP(up(ctx->d_chunk_elem, chunk_elem));
  AMRTO_HIP(up(ctx->d_chunk_tab, chunk_tab));
  AMRTO_HIP(up(ctx->d_chunk_nreg, chunk_nreg));
  AMRTO_HIP(up(ctx->d_chunk_trip, chunk_trip));
  AMRTO_HIP(up(ctx->d_tab_node, tab_node));
  AMRTO_HIP(up(ctx->d_tab_slot, tab_slot));
  AMRTO_HIP(up(ctx->d_elem_loc, elem_loc));
  AMRTO_HIP(up(ctx->d_trip_hm, trip_hm));
  AMRTO_HIP(up(ctx->d_trip_w, trip_w));
  AMRTO_HIP(up(ctx->d_shared_node, shared_node));
  AMRTO_HIP(up(ctx->d_shared_ptr, shared_ptr));
  AMRTO_HIP(up(ctx->d_slot_list, slot_list));
  AMRTO_HIP(up(ctx->d_hang_node, hang_node));
  AMRTO_HIP(up(ctx->d_hang_ptr, hang_ptr));
  AMRTO_HIP(up(ctx->d_hang_master, hang_master));
  AMRTO_HIP(up(ctx->d_hang_w, hang_w));
  if (ctx->d_partial) (void)hipFree(ctx->d_partial);
  ctx->d_partial = nullptr;
  AMRTO_HIP(hipMalloc((void**)&ctx->d_partial, std::max<size_t>(1, 3L * n_slots) * sizeof(double)));
  ctx->n_chunks = nc;
  ctx->n_shared = (int)shared_node.size();
  ctx->n_slots = n_slots;
  ctx->n_hang = m->n_hang;
  return AMRTO_OK;
}

}  // namespace amrto
