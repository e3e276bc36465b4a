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

// Wave sum with DPP row operations (register-to-register, no LDS round trip
// per step): quad permutes, half-row and row mirrors give every lane its
// row's sum; the broadcasts of lanes 15 and 31 (into rows 1, 3 and 2, 3; the
// other rows add zero) leave the total in lane 63, which is read back to
// every lane.  Fixed order, so the result is deterministic.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xb1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4e, 0xf>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_f64<0x140, 0xf>(v);  // row_mirror
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// bitwise OR over the wave, same DPP steps; every lane gets the result
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_or(uint32_t m) {
  m |= dpp_u32<0xb1, 0xf>(m);
  m |= dpp_u32<0x4e, 0xf>(m);
  m |= dpp_u32<0x141, 0xf>(m);
  m |= dpp_u32<0x140, 0xf>(m);
  m |= dpp_u32<0x142, 0xa>(m);
  m |= dpp_u32<0x143, 0xc>(m);
  return (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
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

// ------------------------------------------------------------------ cube element in mode form
// The mirror-symmetry blocks of K0 (see wht8) for a cube of an isotropic
// material have a fixed pattern with eight distinct entries; the kernels take
// them as arguments.
template <typename VT>
struct BrickK {
  VT c[8];  // a - b, b, d, e, f, g, h - i, i
};

constexpr int DPP_ROW_SHL1 = 0x101;  // lane l reads lane l + 1 of its row of 16
constexpr int DPP_ROW_SHR1 = 0x111;  // lane l reads lane l - 1 of its row of 16

// row shifts; lanes whose source falls outside their row read zero
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// 4-point Walsh-Hadamard transform over the x and y bits of a face:
// (u00, u10, u01, u11) -> modes (0, x, y, xy); its own inverse up to 1/4.
template <typename T>
__device__ __forceinline__ void wht4(T (&u)[4]) {
  const T a0 = u[0] + u[1], a1 = u[0] - u[1], b0 = u[2] + u[3], b1 = u[2] - u[3];
  u[0] = a0 + b0;
  u[1] = a1 + b1;
  u[2] = a0 - b0;
  u[3] = a1 - b1;
}

// o = s B w with the block pattern of the cube (w, o: modes [c][t], t bits
// x, y, z); k[] already scaled by the element coefficient.  Translation modes
// (t = 0) give zero rows and columns.
template <typename T>
__device__ __forceinline__ void brick_blocks(const T (&k)[8], const T (&w)[3][8], T (&o)[3][8]) {
  const T AB = k[0], B = k[1], D = k[2], E = k[3], F = k[4], G = k[5], HI = k[6], I = k[7];
  o[0][0] = 0;
  o[1][0] = 0;
  o[2][0] = 0;
  {  // S = 0: modes (0,1) (1,2) (2,4)
    const T v0 = w[0][1], v1 = w[1][2], v2 = w[2][4];
    const T bt = B * (v0 + v1 + v2);
    o[0][1] = AB * v0 + bt;
    o[1][2] = AB * v1 + bt;
    o[2][4] = AB * v2 + bt;
  }
  {  // S = 7: modes (0,6) (1,5) (2,3)
    const T v0 = w[0][6], v1 = w[1][5], v2 = w[2][3];
    const T it = I * (v0 + v1 + v2);
    o[0][6] = HI * v0 + it;
    o[1][5] = HI * v1 + it;
    o[2][3] = HI * v2 + it;
  }
  {  // S = 1: (1,3) (2,5)
    const T v1 = w[1][3], v2 = w[2][5];
    o[1][3] = D * v1 + E * v2;
    o[2][5] = E * v1 + D * v2;
  }
  {  // S = 2: (0,3) (2,6)
    const T v0 = w[0][3], v2 = w[2][6];
    o[0][3] = D * v0 + E * v2;
    o[2][6] = E * v0 + D * v2;
  }
  {  // S = 4: (0,5) (1,6)
    const T v0 = w[0][5], v1 = w[1][6];
    o[0][5] = D * v0 + E * v1;
    o[1][6] = E * v0 + D * v1;
  }
  {  // S = 3: (0,2) (1,1) | (2,7)
    const T s = F * (w[0][2] + w[1][1]);
    o[0][2] = s;
    o[1][1] = s;
    o[2][7] = G * w[2][7];
  }
  {  // S = 5: (0,4) (2,1) | (1,7)
    const T s = F * (w[0][4] + w[2][1]);
    o[0][4] = s;
    o[2][1] = s;
    o[1][7] = G * w[1][7];
  }
  {  // S = 6: (1,4) (2,2) | (0,7)
    const T s = F * (w[1][4] + w[2][2]);
    o[1][4] = s;
    o[2][2] = s;
    o[0][7] = G * w[0][7];
  }
}

// node layers per workgroup (the march is unrolled for exactly this many):
// FP64 runs two workgroups per CU and gains from longer chunks (fewer
// repeated layers); FP32 runs four and from more workgroups
#ifndef AMRTO_BRICK_Z64
#define AMRTO_BRICK_Z64 20
#endif
template <typename VT>
struct BrickZ { static constexpr int layers = 10; };
template <>
struct BrickZ<double> { static constexpr int layers = AMRTO_BRICK_Z64; };
#ifndef AMRTO_BRICK_PD
#define AMRTO_BRICK_PD 2
#endif
constexpr int BPD = AMRTO_BRICK_PD;  // prefetch distance in layers

// y = c K0 u for one element: mode transform, the eight-constant block
// product (k already scaled by c), inverse transform
template <typename T>
__device__ __forceinline__ void contract_brick(const T (&k)[8], const T (&u)[24], T (&y)[24]) {
  T w[3][8], o[3][8];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int n = 0; n < 8; ++n) w[c][n] = u[3 * n + c];
    wht8(w[c]);
  }
  brick_blocks<T>(k, w, o);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    wht8(o[c]);
#pragma unroll
    for (int n = 0; n < 8; ++n) y[3 * n + c] = o[c][n];
  }
}


// ------------------------------------------------------------------ octree chunk tables
// Chunk c's entries, table and hanging triples sit at fixed strides (c
// ENT_MAX, c TAB_MAX, c TRIP_MAX; the tails are padded with zeros), so their
// addresses follow from c alone and a kernel can request them together with
// the chunk's counts instead of after them.
struct ChunkArgs {
  const int4* chunk_cnt;      // [2 n_chunks]: (entries, table, triples, owned regular), (regular, owned hanging, -, -)
  const int32_t* ent_elem;
  const uint16_t* ent_loc;
  const int32_t* tab_node;
  const uint32_t* trip_hm;
  const double* trip_w;
  const int32_t* tab_hbeg;    // hanging entries: first triple (chunk-relative)
  int n_chunks;
  int det;                    // deterministic mode: LDS accumulation in a fixed order
};

// Deterministic mode for LDS accumulation.  FP64 adds into one LDS slot from
// different waves land in the order the waves happen to run, so the last bits
// of the sums vary from run to run.  wave_turns(f) runs f in each wave of the
// block in turn, wave 0 first, with a barrier after every turn: the adds then
// follow (wave, program order, lane), a fixed order, when no two lanes of one
// add instruction name the same slot (the element loops: per vertex slot and
// component, distinct elements have distinct nodes, since two boxes with the
// same corner in the same octant would overlap), and otherwise the order in
// which the LDS unit applies one instruction's conflicting lanes, which does
// not depend on timing.  Every thread of the block must call it.
template <typename F>
__device__ __forceinline__ void wave_turns(F&& f) {
  const int nw = (int)(blockDim.x >> 6), w = (int)(threadIdx.x >> 6);
  for (int t = 0; t < nw; ++t) {
    if (w == t) f();
    __syncthreads();
  }
}

struct ChunkDims {
  int n0, nent, t0, nt, h0, nh, nown, nreg, nhown;
};

// bases and counts of chunk c (counts zero for a surplus workgroup, have = false)
__device__ __forceinline__ ChunkDims chunk_dims(const ChunkArgs& ca, int c, bool have = true) {
  ChunkDims d;
  d.n0 = c * ENT_MAX;
  d.t0 = c * TAB_MAX;
  d.h0 = c * TRIP_MAX;
  const int4 a = ca.chunk_cnt[2 * c], b = ca.chunk_cnt[2 * c + 1];
  d.nent = have ? a.x : 0;
  d.nt = have ? a.y : 0;
  d.nh = have ? a.z : 0;
  d.nown = have ? a.w : 0;
  d.nreg = have ? b.x : 0;
  d.nhown = have ? b.y : 0;
  return d;
}

template <typename VT>
inline BrickK<VT> brick_k(const amrto_ctx* ctx) {
  BrickK<VT> kc;
  for (int q = 0; q < 8; ++q) kc.c[q] = (VT)ctx->bk[q];
  return kc;
}

inline ChunkArgs chunk_args(amrto_ctx* ctx) {
  ChunkArgs a;
  a.chunk_cnt = (const int4*)ctx->d_chunk_cnt;
  a.ent_elem = ctx->d_ent_elem; a.ent_loc = ctx->d_ent_loc; a.tab_node = ctx->d_tab_node;
  a.trip_hm = ctx->d_trip_hm; a.trip_w = ctx->d_trip_w; a.tab_hbeg = ctx->d_tab_hbeg;
  a.n_chunks = ctx->n_chunks;
  a.det = ctx->deterministic ? 1 : 0;
  return a;
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

// ------------------------------------------------------------------ block-Jacobi

// Inverse 3x3 node blocks are stored as six entries per node:
// (B00, B11, B22, B01, B02, B12) of the symmetric inverse.
// z = B^-1 r for one node from the six stored entries
template <typename VT>
__device__ __forceinline__ void block_apply(const VT* __restrict__ bi, const VT (&r)[3], VT (&z)[3]) {
  z[0] = bi[0] * r[0] + bi[3] * r[1] + bi[4] * r[2];
  z[1] = bi[3] * r[0] + bi[1] * r[1] + bi[5] * r[2];
  z[2] = bi[4] * r[0] + bi[5] * r[1] + bi[2] * r[2];
}

// ------------------------------------------------------------------ fused CG step
// Start of a fused CG iteration (every block computes the same values from
// the same partial sums): convergence test on r.r, then beta = rz_i / rz_{i-1}
// (beta = 0 on the first iteration, p = z).  Returns false when the solve has
// stopped (converged, breakdown, or already flagged).

__device__ __forceinline__ bool cg_prologue(const CgArgs& cg, double& beta, double* sh) {
  // the finished flag is read with the partial sums and tested after them
  // (uniform over the block; nothing is stored before the test)
  const double done = cg.scal[S_DONE];
  double rz = 0.0, rr = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += blockDim.x) {
    rz += cg.part_in[i];
    rr += cg.part_in[RED_BLOCKS + i];
  }
  for (int i = threadIdx.x; i < cg.ck; i += blockDim.x) rz += cg.cct[i] * cg.ccz[i];
  block_sum2(rz, rr, sh);
  if (done != 0.0) return false;
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
