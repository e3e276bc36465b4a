// Mixed-precision operator apply: the element contraction Y = K0 U for a
// batch of 16 elements runs on the gfx950 matrix cores as
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
//
//   M = 24 DOF rows  -> two 16-row tiles (rows 24..31 are zero padding)
//   K = 24 DOF cols  -> one 32-deep step  (cols 24..31 are zero padding)
//   N = 16 elements of one tile
//
// K0 is split as K0 = hi + lo with both parts in BF16 (two MFMAs per tile
// into the same FP32 accumulator), so the matrix is kept to ~2^-17.  Each
// element's displacements are shifted by their element mean before rounding
// to BF16: K0 annihilates rigid translations, so the shift changes nothing in
// exact arithmetic but removes the large common part that rounding would
// otherwise spoil.  Vectors are FP32; the caller's refinement loop keeps the
// residual and all dot products in FP64.
//
// Operand layout of the 16x16x32 BF16 instruction (lane l, q = l / 16):
//   A[m][k]: lane (m + 16 q) holds k = 8q .. 8q+7
//   B[k][n]: lane (n + 16 q) holds k = 8q .. 8q+7
//   D[m][n]: lane (n + 16 q) holds m = 4q .. 4q+3
#include "internal.h"

namespace amrto {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int xcd_remap_m(int b, int nb) {
  int per = (nb + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ __bf16 bits_to_bf16(uint16_t v) {
  return __builtin_bit_cast(__bf16, v);
}

// A operands for the two M tiles, hi and lo parts: a[tile][part]
__device__ __forceinline__ void load_k0_bf16(const uint16_t* __restrict__ K0bf, bf16x8 (&a)[2][2]) {
  const int lane = threadIdx.x & 63;
  const int m0 = lane & 15, q = lane >> 4;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      bf16x8 v;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int m = m0 + 16 * t, k = 8 * q + i;
        const uint16_t bits = (m < 24 && k < 24) ? K0bf[part * 576 + m * 24 + k] : (uint16_t)0;
        v[i] = bits_to_bf16(bits);
      }
      a[t][part] = v;
    }
}

// B operand from the 24 element values u (already in registers): shift by
// the element mean per component and keep this lane's 8 consecutive DOFs.
__device__ __forceinline__ bf16x8 element_operand(const float (&u)[24], int q) {
  float m[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < 8; ++a) s += u[3 * a + c];
    m[c] = 0.125f * s;
  }
  bf16x8 b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float v0 = u[i] - m[i % 3];
    const float v1 = u[8 + i] - m[(8 + i) % 3];
    const float v2 = u[16 + i] - m[(16 + i) % 3];
    const float v = q == 0 ? v0 : (q == 1 ? v1 : (q == 2 ? v2 : 0.f));
    b[i] = (__bf16)v;
  }
  return b;
}

__device__ __forceinline__ void contract_tile(const bf16x8 (&a)[2][2], bf16x8 b, f32x4& d0, f32x4& d1) {
  f32x4 z = {0.f, 0.f, 0.f, 0.f};
  d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][0], b, z, 0, 0, 0);
  d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][1], b, d0, 0, 0, 0);
  d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][0], b, z, 0, 0, 0);
  d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][1], b, d1, 0, 0, 0);
}

// ------------------------------------------------------------------ uniform brick
// Same tiling and march as the FP64/FP32 uniform kernel; wave w handles the
// element rows j = 4w .. 4w+3 of each layer, one 16-element MFMA tile per row.
__global__ __launch_bounds__(256) void k_apply_uniform_bf16(
    const float* __restrict__ x, float* __restrict__ y, const float* __restrict__ coef,
    const uint8_t* __restrict__ fix, const uint16_t* __restrict__ K0bf, int nx, int ny, int nz,
    int tiles_x, int tiles_y, int zchunk, int n_tiles, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ float xs[2][UN * UN * 3];
  __shared__ float ys[2][UT * UT * 3];
  const int tile = xcd_remap_m(blockIdx.x, gridDim.x);
  if (tile >= n_tiles) return;
  const int tx = tile % tiles_x;
  const int ty = (tile / tiles_x) % tiles_y;
  const int tz = tile / (tiles_x * tiles_y);
  const int ox = tx * UT, oy = ty * UT;
  const int z0 = tz * zchunk;
  const int z1 = min(z0 + zchunk, nz + 1);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int n = lane & 15, q = lane >> 4;
  const long sx = nx + 1, sxy = (long)(nx + 1) * (ny + 1);
  bf16x8 a[2][2];
  load_k0_bf16(K0bf, a);

  auto load_layer = [&](int buf, int k) {
    for (int idx = tid; idx < UN * UN * 3; idx += 256) {
      const int c = idx % 3, nd = idx / 3;
      const int gx = ox - 1 + nd % UN, gy = oy - 1 + nd / UN;
      float v = 0.f;
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
        float v = ys[buf][idx];
        if ((fix[node] >> c) & 1) v = x[3 * node + c];
        y[3 * node + c] = v;
      }
      ys[buf][idx] = 0.f;
    }
  };

  for (int idx = tid; idx < UT * UT * 3; idx += 256) { ys[0][idx] = 0.f; ys[1][idx] = 0.f; }
  const int kbeg = max(z0 - 1, 0);
  const int kend = min(z1 - 1, nz - 1);
  int cur = 0;
  load_layer(cur, kbeg);
  for (int k = kbeg; k <= kend; ++k) {
    load_layer(cur ^ 1, k + 1);
    __syncthreads();
#pragma unroll 1
    for (int row = 0; row < 4; ++row) {
      const int j = 4 * wave + row;
      const int i = n;
      const int ex = ox - 1 + i, ey = oy - 1 + j;
      const bool ev = ex >= 0 && ex < nx && ey >= 0 && ey < ny;
      float u[24];
#pragma unroll
      for (int aa = 0; aa < 8; ++aa) {
        const int l = ((j + ((aa >> 1) & 1)) * UN + i + (aa & 1)) * 3;
        const float* src = xs[(aa >> 2) ? (cur ^ 1) : cur];
        u[3 * aa + 0] = src[l + 0];
        u[3 * aa + 1] = src[l + 1];
        u[3 * aa + 2] = src[l + 2];
      }
      const bf16x8 b = element_operand(u, q);
      f32x4 d0, d1;
      contract_tile(a, b, d0, d1);
      if (ev) {
        const float ce = coef[ex + (long)nx * (ey + (long)ny * k)];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int R = 16 * t + 4 * q + r;
            if (R < 24) {
              const int aa = R / 3, c = R % 3;
              const int li = i + (aa & 1) - 1, lj = j + ((aa >> 1) & 1) - 1;
              const int layer = k + (aa >> 2);
              if (li >= 0 && li < UT && lj >= 0 && lj < UT && layer >= z0 && layer < z1)
                atomicAdd(&ys[layer & 1][(lj * UT + li) * 3 + c], ce * (t ? d1[r] : d0[r]));
            }
          }
      }
    }
    __syncthreads();
    if (k >= z0) store_layer(k & 1, k);
    cur ^= 1;
  }
  if (kend + 1 < z1 && kend + 1 >= z0) {
    __syncthreads();
    store_layer((kend + 1) & 1, kend + 1);
  }
}

// ------------------------------------------------------------------ octree chunks
struct ChunkArgsM {
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

__global__ __launch_bounds__(256) void k_apply_chunks_bf16(
    const float* __restrict__ x, float* __restrict__ y, float* __restrict__ partial,
    const float* __restrict__ coef, const uint8_t* __restrict__ fix, const uint16_t* __restrict__ K0bf,
    ChunkArgsM ca, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ float xs[TAB_MAX * 3];
  __shared__ float ys[TAB_MAX * 3];
  __shared__ uint16_t lsm[CH_MAX * 8];
  const int c = xcd_remap_m(blockIdx.x, gridDim.x);
  if (c >= ca.n_chunks) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int n = lane & 15, q = lane >> 4;
  const int e0 = ca.chunk_elem[c], e1 = ca.chunk_elem[c + 1];
  const int ne = e1 - e0;
  const int t0 = ca.chunk_tab[c], nt = ca.chunk_tab[c + 1] - t0, nreg = ca.chunk_nreg[c];
  const int h0 = ca.chunk_trip[c], nh = ca.chunk_trip[c + 1] - h0;
  bf16x8 a[2][2];
  load_k0_bf16(K0bf, a);
  for (int i = tid; i < nt * 3; i += 256) {
    const int t = i / 3, comp = i % 3;
    float v = 0.f;
    if (t < nreg) {
      const int node = ca.tab_node[t0 + t];
      if (!((fix[node] >> comp) & 1)) v = x[3L * node + comp];
    }
    xs[i] = v;
    ys[i] = 0.f;
  }
  for (int i = tid; i < ne * 8; i += 256) lsm[i] = ca.elem_loc[8L * e0 + i];
  __syncthreads();
  for (int i = tid; i < nh * 3; i += 256) {
    const int k = i / 3, comp = i % 3;
    const uint32_t hm = ca.trip_hm[h0 + k];
    atomicAdd(&xs[(hm >> 16) * 3 + comp], (float)ca.trip_w[h0 + k] * xs[(hm & 0xffff) * 3 + comp]);
  }
  __syncthreads();
  // 16-element tiles, round-robin over the 4 waves
  for (int tb = 16 * wave; tb < ne; tb += 64) {
    const int el = tb + n;
    const bool ev = el < ne;
    float u[24];
#pragma unroll
    for (int aa = 0; aa < 8; ++aa) {
      const int l = ev ? lsm[el * 8 + aa] * 3 : 0;
      u[3 * aa + 0] = ev ? xs[l + 0] : 0.f;
      u[3 * aa + 1] = ev ? xs[l + 1] : 0.f;
      u[3 * aa + 2] = ev ? xs[l + 2] : 0.f;
    }
    const bf16x8 b = element_operand(u, q);
    f32x4 d0, d1;
    contract_tile(a, b, d0, d1);
    if (ev) {
      const float ce = coef[e0 + el];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int R = 16 * t + 4 * q + r;
          if (R < 24) {
            const int l = lsm[el * 8 + R / 3];
            atomicAdd(&ys[l * 3 + R % 3], ce * (t ? d1[r] : d0[r]));
          }
        }
    }
  }
  __syncthreads();
  for (int i = tid; i < nh * 3; i += 256) {
    const int k = i / 3, comp = i % 3;
    const uint32_t hm = ca.trip_hm[h0 + k];
    atomicAdd(&ys[(hm & 0xffff) * 3 + comp], (float)ca.trip_w[h0 + k] * ys[(hm >> 16) * 3 + comp]);
  }
  __syncthreads();
  for (int i = tid; i < nreg * 3; i += 256) {
    const int t = i / 3, comp = i % 3;
    const int node = ca.tab_node[t0 + t];
    const int slot = ca.tab_slot[t0 + t];
    float v = ys[i];
    if (slot < 0) {
      if ((fix[node] >> comp) & 1) v = x[3L * node + comp];
      y[3L * node + comp] = v;
    } else {
      partial[3L * slot + comp] = v;
    }
  }
}

int launch_apply_bf16(amrto_ctx* ctx, const float* x, float* y, const double* stop) {
  if (ctx->uniform) {
    int tx, ty, zc, nt, grid;
    uniform_grid(ctx, tx, ty, zc, nt, grid);
    hipLaunchKernelGGL(k_apply_uniform_bf16, dim3(grid), dim3(256), 0, ctx->stream, x, y, ctx->d_coef_f,
                       ctx->d_fix, ctx->d_K0bf, ctx->nx, ctx->ny, ctx->nz, tx, ty, zc, nt, stop);
  } else {
    ChunkArgsM ca;
    ca.chunk_elem = ctx->d_chunk_elem; ca.chunk_tab = ctx->d_chunk_tab; ca.chunk_nreg = ctx->d_chunk_nreg;
    ca.chunk_trip = ctx->d_chunk_trip; ca.tab_node = ctx->d_tab_node; ca.tab_slot = ctx->d_tab_slot;
    ca.elem_loc = ctx->d_elem_loc; ca.trip_hm = ctx->d_trip_hm; ca.trip_w = ctx->d_trip_w;
    ca.n_chunks = ctx->n_chunks;
    const int grid = ((ctx->n_chunks + 7) / 8) * 8;
    hipLaunchKernelGGL(k_apply_chunks_bf16, dim3(grid), dim3(256), 0, ctx->stream, x, y,
                       (float*)ctx->d_partial, ctx->d_coef_f, ctx->d_fix, ctx->d_K0bf, ca, stop);
    reduce_shared<float>(ctx, x, y, stop);
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

}  // namespace amrto
