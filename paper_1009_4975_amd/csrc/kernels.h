// Device building blocks shared by the operator kernels.
#pragma once

#include "internal.h"

namespace amrto {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int per = (nb + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// deterministic block sum (fixed tree); every thread gets the result
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
  return block_sum(v, sh);
}

// two block sums with one exchange (sh holds 2 x waves entries); each sum
// uses the same fixed tree as block_sum
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  if (lane == 0) {
    sh[w] = a;
    sh[nw + w] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
  for (int i = 0; i < nw; ++i) {
    sa += sh[i];
    sb += sh[nw + i];
  }
  __syncthreads();
  a = sa;
  b = sb;
}

// ------------------------------------------------------------------ element contraction
// K0 commutes with the three mirror maps of the cube (node flip combined with
// a sign change of the mirrored displacement component).  In the basis of
// per-component 8-point Walsh-Hadamard modes, w_c[t] = sum_n (-1)^{t.n} u[3n+c],
// it is block diagonal: the three modes (c, t = S ^ (1 << c)), c = 0, 1, 2,
// sharing the mirror character S form one 3x3 block B_S (8 blocks; rigid
// translations t = 0 fall in zero rows).  So K0 u = W^T B W u costs two
// transforms (add/sub only) and a few multiply-adds (apply.hip: brick_blocks).
template <typename T>
__device__ __forceinline__ void wht8(T (&v)[8]) {
#pragma unroll
  for (int h = 1; h < 8; h <<= 1)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (!(j & h)) {
        const T a = v[j], b = v[j + h];
        v[j] = a + b;
        v[j + h] = a - b;
      }
}

// ------------------------------------------------------------------ BF16 MFMA tile
// Y = K0 U for 16 elements with v_mfma_f32_16x16x32_bf16 (FP32 accumulate):
// M = 24 rows in two 16-row tiles, K = 24 (padded to 32), N = 16 elements.
// K0 is split hi + lo in BF16 (two MFMAs into one accumulator).  Operand
// layout, lane l, q = l / 16:  A[m][k]: lane m + 16q holds k = 8q..8q+7;
// B[k][n]: lane n + 16q holds k = 8q..8q+7;  D[m][n]: lane n + 16q holds
// m = 4q..4q+3.
__device__ __forceinline__ __bf16 bits_to_bf16(uint16_t v) { return __builtin_bit_cast(__bf16, v); }

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
        v[i] = bits_to_bf16((m < 24 && k < 24) ? K0bf[part * 576 + m * 24 + k] : (uint16_t)0);
      }
      a[t][part] = v;
    }
}

// B operand: subtract the element mean per component (K0 annihilates rigid
// translations, so this is exact in real arithmetic), keep this lane's 8
// consecutive DOFs and split each into hi + lo BF16 parts (v ~ hi + lo to
// about 2^-16 relative).  Products: K0hi.uhi + K0lo.uhi + K0hi.ulo, all
// accumulated in FP32; the dropped K0lo.ulo term is ~2^-17 relative.
__device__ __forceinline__ void mfma_tile_bf16(const bf16x8 (&a)[2][2], const float (&u)[24], int q, f32x4& d0,
                                               f32x4& d1) {
  float m[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += u[3 * k + c];
    m[c] = 0.125f * s;
  }
  bf16x8 bh, bl;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float v0 = u[i] - m[i % 3];
    const float v1 = u[8 + i] - m[(8 + i) % 3];
    const float v2 = u[16 + i] - m[(16 + i) % 3];
    const float v = q == 0 ? v0 : (q == 1 ? v1 : (q == 2 ? v2 : 0.f));
    const __bf16 h = (__bf16)v;
    bh[i] = h;
    bl[i] = (__bf16)(v - (float)h);
  }
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
  d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][0], bh, z, 0, 0, 0);
  d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][1], bh, d0, 0, 0, 0);
  d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][0], bl, d0, 0, 0, 0);
  d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][0], bh, z, 0, 0, 0);
  d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][1], bh, d1, 0, 0, 0);
  d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][0], bl, d1, 0, 0, 0);
}

// ------------------------------------------------------------------ fused CG step
// Start of a fused CG iteration (every block computes the same values from
// the same partial sums): convergence test on r.r, then beta = rz_i / rz_{i-1}
// (beta = 0 on the first iteration, p = z).  Returns false when the solve has
// stopped (converged, breakdown, or already flagged).

__device__ __forceinline__ bool cg_prologue(const CgArgs& cg, double& beta, double* sh) {
  if (cg.scal[S_DONE] != 0.0) return false;
  double rz = 0.0, rr = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += blockDim.x) {
    rz += cg.part_in[i];
    rr += cg.part_in[RED_BLOCKS + i];
  }
  block_sum2(rz, rr, sh);
  if (cg.coarse) rz += cg.scal[S_CTZ];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (!(rz == rz) || !(rr == rr) || rr > 1e300 || rz > 1e300) {
    if (lead) cg.scal[S_DONE] = 2.0;
    return false;
  }
  if (rr <= cg.tol2 * cg.scal[S_BB]) {
    if (lead) {
      cg.scal[S_RR] = rr;
      cg.scal[S_ITERS] = cg.it;
      cg.scal[S_DONE] = 1.0;
    }
    return false;
  }
  beta = cg.it == 0 ? 0.0 : rz / cg.scal[S_RZ0 + ((cg.it - 1) & 1)];
  if (lead) {
    cg.scal[S_RZ0 + (cg.it & 1)] = rz;
    cg.scal[S_RR] = rr;
    cg.scal[S_ITERS] = cg.it;
  }
  return true;
}

}  // namespace amrto
