// Jacobi-preconditioned conjugate gradients on A~ (paper Sec. 5: the
// symmetric diagonal rescaling D^-1/2 A D^-1/2 is exactly the Jacobi
// preconditioner of CG; warm start from the previous solution), and a
// mixed-precision variant that runs the Krylov recurrence with FP32 vectors
// and an FP32 or BF16 operator while the iterate, the true residual and all
// dot products stay in FP64 ("reliable updates").
//
// One CG iteration is two passes: the fused operator pass (p = z + beta p,
// q = A~ p, partial p.q; see apply.hip) and the update pass below (alpha,
// x, r, z, partial r.z and r.r).  All scalars live on the device; every
// block re-adds the same partials in the same order, so every block takes
// the same decision without a finalize launch, and a converged or broken
// solve makes the rest of an enqueued batch return at once.
#include <chrono>
#include <cstdio>
#include <cmath>
#include <string>
#include <type_traits>

#include "kernels.h"

namespace amrto {

template <typename VT>
__global__ __launch_bounds__(256) void k_fill(VT* __restrict__ x, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

// zero supported and hanging entries (identity rows with zero right-hand side)
template <typename VT>
__global__ __launch_bounds__(256) void k_mask(VT* __restrict__ x, const uint8_t* __restrict__ fix, long n3) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n3 && ((fix[i / 3] >> (i % 3)) & 1)) x[i] = 0;
}

template <typename VT>
__global__ __launch_bounds__(256) void k_mask_hanging(VT* __restrict__ x, const int32_t* __restrict__ hang_node,
                                                      int n_hang) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < 3L * n_hang) x[3L * hang_node[i / 3] + i % 3] = 0;
}

// r = b - q (q may be NULL: r = b); z = D^-1 r; partials r.z, r.r, b.b
template <typename VT, typename BT>
__global__ __launch_bounds__(256) void k_init(const BT* __restrict__ b, const BT* __restrict__ q,
                                              VT* __restrict__ r, VT* __restrict__ z, const VT* __restrict__ dinv,
                                              long n, double* __restrict__ part) {
  __shared__ double sh[8];
  double rz = 0, rr = 0, bb = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const BT bi = b[i];
    const VT ri = (VT)(q ? (BT)(bi - q[i]) : bi);
    const VT zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    rz += (double)ri * (double)zi;
    rr += (double)ri * (double)ri;
    bb += (double)bi * (double)bi;
  }
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rz;
    part[RED_BLOCKS + blockIdx.x] = rr;
    part[2 * RED_BLOCKS + blockIdx.x] = bb;
  }
}

// bb_mode 0: b.b from the partials; 1: keep scal[S_BB] (set by the caller)
__global__ __launch_bounds__(256) void k_init_scalars(const double* __restrict__ part, double* __restrict__ scal,
                                                      double tol2, int keep_bb, int add_ctz) {
  __shared__ double sh[8];
  double rz = sum_partials(part, RED_BLOCKS, sh);
  if (add_ctz) rz += scal[S_CTZ];
  const double rr = sum_partials(part + RED_BLOCKS, RED_BLOCKS, sh);
  const double bb = sum_partials(part + 2 * RED_BLOCKS, RED_BLOCKS, sh);
  if (threadIdx.x == 0) {
    if (!keep_bb) scal[S_BB] = bb;
    scal[S_RZ0] = rz;
    scal[S_RZ1] = rz;
    scal[S_RR] = rr;
    scal[S_ITERS] = 0.0;
    scal[S_DONE] = (rr <= tol2 * scal[S_BB]) ? 1.0 : ((rr == rr && rr < 1e300) ? 0.0 : 2.0);
  }
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; z = D^-1 r; partials r.z, r.r
template <typename VT>
__global__ __launch_bounds__(256) void k_cg_update(VT* __restrict__ x, VT* __restrict__ r, const VT* __restrict__ p,
                                                   const VT* __restrict__ q, const VT* __restrict__ dinv,
                                                   VT* __restrict__ z, long n, const double* __restrict__ part_pq,
                                                   int n_pq, double* __restrict__ scal, int it,
                                                   double* __restrict__ part) {
  // a finished solve stores nothing; the flag is read with the loads below
  // and tested once they are requested (one round trip instead of two)
  const double done = scal[S_DONE];
  __shared__ double sh[8];
  // the first UPT entries of this thread are requested before the p.q
  // partials are reduced (alpha is not needed to load them)
  constexpr int UPT = 4;
  const long i0 = blockIdx.x * (long)blockDim.x + threadIdx.x, stride = (long)gridDim.x * blockDim.x;
  VT xv[UPT], pv[UPT], rv[UPT], qv[UPT], dv[UPT];
#pragma unroll
  for (int u = 0; u < UPT; ++u) {
    const long i = i0 + u * stride;
    const bool in = i < n;
    xv[u] = in ? x[i] : (VT)0;
    pv[u] = in ? p[i] : (VT)0;
    rv[u] = in ? r[i] : (VT)0;
    qv[u] = in ? q[i] : (VT)0;
    dv[u] = in ? dinv[i] : (VT)0;
  }
  const double pq = sum_partials(part_pq, n_pq, sh);
  if (done != 0.0) return;
  const double rz = scal[S_RZ0 + (it & 1)];
  if (!(pq > 0.0) || !(pq < 1e300) || !(rz == rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_DONE] = 2.0;
    return;
  }
  const VT alpha = (VT)(rz / pq);
  double srz = 0.0, srr = 0.0;
#pragma unroll
  for (int u = 0; u < UPT; ++u) {
    const long i = i0 + u * stride;
    if (i < n) {
      x[i] = xv[u] + alpha * pv[u];
      const VT ri = rv[u] - alpha * qv[u];
      const VT zi = dv[u] * ri;
      r[i] = ri;
      z[i] = zi;
      srz += (double)ri * (double)zi;
      srr += (double)ri * (double)ri;
    }
  }
  for (long i = i0 + UPT * stride; i < n; i += stride) {
    x[i] += alpha * p[i];
    const VT ri = r[i] - alpha * q[i];
    const VT zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    srz += (double)ri * (double)zi;
    srr += (double)ri * (double)ri;
  }
  block_sum2(srz, srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[RED_BLOCKS + blockIdx.x] = srr;
  }
}

// ------------------------------------------------------------------ coarse space
// The coarse space Z: column (f, g, c) is component c of field f on the nodes
// of region g.  Fields are either stored (F, nf x 3n, masked) or, for the
// affine space alone, formed on the fly from a 16-byte node descriptor (FP32
// offsets from the region centre, region, support/hanging bits) instead of
// 96 bytes of stored fields.  The stored fields Z^T A Z was formed from are
// made from the same FP32 offsets, so both views of Z agree exactly.
struct CoarseArgs {
  const double* F;
  int nf, R;
  const uint8_t* region;
  const float4* geo;      // affine space: per node (dx, dy, dz, region | mask << 8); NULL: stored fields
  int det;                // deterministic mode (see zt_loop_acc)
};

// field values of DOF i into fv; returns the DOF's region
__device__ __forceinline__ int coarse_fields(const CoarseArgs& a, long i, long n3, double (&fv)[COARSE_NFMAX]) {
  const int ii = (int)i, v = ii / 3, c = ii - 3 * v;
  if (!a.geo) {
#pragma unroll
    for (int f = 0; f < COARSE_NFMAX; ++f) fv[f] = f < a.nf ? a.F[(long)f * n3 + i] : 0.0;
    return a.region[v];
  }
  const float4 q = a.geo[v];
  const int w = __float_as_int(q.w);
  const double on = ((w >> (8 + c)) & 1) ? 0.0 : 1.0;
  const double d[3] = {(double)q.x, (double)q.y, (double)q.z};
  fv[0] = on;
  fv[1] = on * d[c];
  fv[2] = on * d[c == 2 ? 0 : c + 1];
  fv[3] = on * d[c == 0 ? 2 : c - 1];
#pragma unroll
  for (int f = 4; f < COARSE_NFMAX; ++f) fv[f] = 0.0;
  return w & 0xff;
}

__device__ __forceinline__ int coarse_region(const CoarseArgs& a, int v) {
  return a.geo ? (__float_as_int(a.geo[v].w) & 0xff) : a.region[v];
}

// Z^T v per block.  Each block takes a contiguous DOF range and walks it in
// steps of the block size, so a thread's DOFs stay in one region for long
// stretches: the thread keeps 3 nf running sums in registers for its current
// region and adds them to the block's LDS accumulator only when its region
// changes and at the end.  Fields beyond COARSE_NFMAX are rejected at set-up,
// so the register sums have a fixed size.
struct ZtAcc {
  double s[COARSE_NFMAX][3];
  int g;
};

__device__ __forceinline__ void zt_clear(ZtAcc& a, int g) {
#pragma unroll
  for (int f = 0; f < COARSE_NFMAX; ++f)
#pragma unroll
    for (int c = 0; c < 3; ++c) a.s[f][c] = 0.0;
  a.g = g;
}

__device__ __forceinline__ void zt_flush_lane(ZtAcc& a, double* acc, int nf, int R) {
  if (a.g < 0) return;
#pragma unroll
  for (int f = 0; f < COARSE_NFMAX; ++f)
    if (f < nf)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (a.s[f][c] != 0.0) atomicAdd(&acc[(f * R + a.g) * 3 + c], a.s[f][c]);
}

// add vi F_f[i] (f < nf) for DOF i of component c in region g
__device__ __forceinline__ void zt_add(ZtAcc& a, double* acc, const double (&fv)[COARSE_NFMAX], int nf, int R, int g,
                                       int c, double vi) {
  if (g != a.g) {
    zt_flush_lane(a, acc, nf, R);
    zt_clear(a, g);
  }
#pragma unroll
  for (int f = 0; f < COARSE_NFMAX; ++f) {
    const double v = fv[f] * vi;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) a.s[f][cc] += cc == c ? v : 0.0;
  }
}

// End of the block's range.  When every thread's sums belong to the region of
// the block's first DOF (the usual case), they are transposed through LDS and
// each of the 3 nf columns is summed by one thread in thread order (no atomics,
// deterministic); otherwise each thread adds its own sums atomically.
// Deterministic mode: the lane flushes go to one accumulator per wave (in
// red, which is unused until the end of the block's range), and the end of
// the range adds the waves' accumulators in wave order.  Within a wave the
// flushes follow program order, and one instruction's lanes that name the
// same slot are applied by the LDS unit in an order that does not depend on
// timing, so the sums do not vary from run to run.
__device__ __forceinline__ double* zt_loop_acc(int det, double* acc, double (*red)[256]) {
  return det ? &red[0][0] + (threadIdx.x >> 6) * COARSE_KMAX : acc;
}

__device__ __forceinline__ void zt_loop_clear(int det, double (*red)[256]) {
  static_assert(COARSE_NFMAX * 3 * 256 >= 4 * COARSE_KMAX, "one accumulator per wave of 256 threads fits in red");
  if (det)
    for (int j = threadIdx.x; j < (int)(blockDim.x >> 6) * COARSE_KMAX; j += blockDim.x) (&red[0][0])[j] = 0.0;
}

__device__ __forceinline__ void zt_flush(ZtAcc& a, double* acc, int nf, int R, int g_first,
                                         double (*red)[256], int det) {
  if (det) {
    double* accw = &red[0][0];
    zt_flush_lane(a, accw + (threadIdx.x >> 6) * COARSE_KMAX, nf, R);
    __syncthreads();
    const int k = 3 * nf * R, nw = (int)(blockDim.x >> 6);
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += accw[w * COARSE_KMAX + j];
      acc[j] += s;
    }
    return;
  }
  const bool uniform = __syncthreads_and(a.g == g_first || a.g < 0);
  if (!uniform) {
    zt_flush_lane(a, acc, nf, R);
    return;
  }
  const int t = threadIdx.x;
#pragma unroll
  for (int f = 0; f < COARSE_NFMAX; ++f)
    if (f < nf)
#pragma unroll
      for (int c = 0; c < 3; ++c) red[f * 3 + c][t] = a.g < 0 ? 0.0 : a.s[f][c];
  __syncthreads();
  if (t < 3 * nf) {
    double s = 0.0;
#pragma unroll 8
    for (int u = 0; u < 256; ++u) s += red[t][u];
    acc[((t / 3) * R + g_first) * 3 + t % 3] += s;  // one writer per column; earlier flushes are done
  }
}

// block b's DOF range [lo, hi)
__device__ __forceinline__ void block_range(long n, long& lo, long& hi) {
  const long per = (n + gridDim.x - 1) / gridDim.x;
  lo = blockIdx.x * per;
  hi = lo + per < n ? lo + per : n;
}

// Write this block's Z^T v partials (column-major: part[j nblk + block], so
// the column sums read them coalesced).
__device__ __forceinline__ void zt_store(const double* acc, int k, double* __restrict__ part) {
  for (int j = threadIdx.x; j < k; j += blockDim.x) part[(long)j * gridDim.x + blockIdx.x] = acc[j];
}

template <typename VT>
__global__ __launch_bounds__(256) void k_zt_part(CoarseArgs ca, const VT* __restrict__ v, long n3,
                                                 double* __restrict__ part) {
  __shared__ double acc[COARSE_KMAX];
  __shared__ double red[COARSE_NFMAX * 3][256];
  const int nf = ca.nf, R = ca.R, k = 3 * nf * R;
  for (int j = threadIdx.x; j < k; j += blockDim.x) acc[j] = 0.0;
  zt_loop_clear(ca.det, red);
  __syncthreads();
  double* const acc_l = zt_loop_acc(ca.det, acc, red);
  long lo, hi;
  block_range(n3, lo, hi);
  ZtAcc a;
  zt_clear(a, -1);
#pragma unroll 2
  for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    double fv[COARSE_NFMAX];
    const int g = coarse_fields(ca, i, n3, fv);
    zt_add(a, acc_l, fv, nf, R, g, (int)(i % 3), (double)v[i]);
  }
  zt_flush(a, acc, nf, R, lo < hi ? coarse_region(ca, (int)(lo / 3)) : 0, red, ca.det);
  __syncthreads();
  zt_store(acc, k, part);
}

// Coarse-corrected variant of the update pass: x += alpha p, r -= alpha q,
// the block partials of Z^T r, and partials of r^T D^-1 r and r^T r (then
// k_coarse_sum and k_coarse_cz; z is formed by k_coarse_z or, on octree
// meshes with the affine space, inside the next operator pass).
template <typename VT>
__global__ __launch_bounds__(256) void k_cg_update_coarse(VT* __restrict__ x, VT* __restrict__ r,
                                                          const VT* __restrict__ p, const VT* __restrict__ q,
                                                          const VT* __restrict__ dinv, long n,
                                                          const double* __restrict__ part_pq, int n_pq,
                                                          double* __restrict__ scal, int it, CoarseArgs ca,
                                                          double* __restrict__ part_z, double* __restrict__ part) {
  // a finished solve stores nothing; the flag is read with the loads below
  // and tested once they are requested (one round trip instead of two)
  const double done = scal[S_DONE];
  __shared__ double sh[8];
  __shared__ double acc[COARSE_KMAX];
  __shared__ double red[COARSE_NFMAX * 3][256];
  const int nf = ca.nf, R = ca.R, k = 3 * nf * R;
  long lo, hi;
  block_range(n, lo, hi);
  // the first UPT entries of this thread are requested before the p.q
  // partials are reduced (alpha is not needed to load them)
  constexpr int UPT = 2;
  VT pv0[UPT], qv0[UPT], rv0[UPT], xv0[UPT], dv0[UPT];
#pragma unroll
  for (int u = 0; u < UPT; ++u) {
    const long i = lo + threadIdx.x + u * (long)blockDim.x;
    const bool in = i < hi;
    pv0[u] = in ? p[i] : (VT)0;
    qv0[u] = in ? q[i] : (VT)0;
    rv0[u] = in ? r[i] : (VT)0;
    xv0[u] = in ? x[i] : (VT)0;
    dv0[u] = in ? dinv[i] : (VT)0;
  }
  const double pq = sum_partials(part_pq, n_pq, sh);
  if (done != 0.0) return;
  const double rz = scal[S_RZ0 + (it & 1)];
  if (!(pq > 0.0) || !(pq < 1e300) || !(rz == rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_DONE] = 2.0;
    return;
  }
  for (int j = threadIdx.x; j < k; j += blockDim.x) acc[j] = 0.0;
  zt_loop_clear(ca.det, red);
  __syncthreads();
  double* const acc_l = zt_loop_acc(ca.det, acc, red);
  const VT alpha = (VT)(rz / pq);
  ZtAcc a;
  zt_clear(a, -1);
  double srz = 0.0, srr = 0.0;
  long i = lo + threadIdx.x;
#pragma unroll
  for (int u = 0; u < UPT; ++u, i += blockDim.x) {
    if (i < hi) {
      double fv[COARSE_NFMAX];
      const int g = coarse_fields(ca, i, n, fv);
      x[i] = xv0[u] + alpha * pv0[u];
      const VT rv = rv0[u] - alpha * qv0[u];
      r[i] = rv;
      srz += (double)rv * (double)dv0[u] * (double)rv;
      srr += (double)rv * (double)rv;
      zt_add(a, acc_l, fv, nf, R, g, (int)(i % 3), (double)rv);
    }
  }
#pragma unroll 2
  for (; i < hi; i += blockDim.x) {
    double fv[COARSE_NFMAX];
    const int g = coarse_fields(ca, i, n, fv);
    const VT pi = p[i], qi = q[i], ri = r[i], xi = x[i], di = dinv[i];
    x[i] = xi + alpha * pi;
    const VT rv = ri - alpha * qi;
    r[i] = rv;
    srz += (double)rv * (double)di * (double)rv;
    srr += (double)rv * (double)rv;
    zt_add(a, acc_l, fv, nf, R, g, (int)(i % 3), (double)rv);
  }
  zt_flush(a, acc, nf, R, lo < hi ? coarse_region(ca, (int)(lo / 3)) : 0, red, ca.det);
  __syncthreads();
  zt_store(acc, k, part_z);
  block_sum2(srz, srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[RED_BLOCKS + blockIdx.x] = srr;
  }
}

// The same pass with the block-Jacobi preconditioner (inverse 3x3 node
// blocks): one node per step, since r^T B^-1 r needs a node's three
// components together.
template <typename VT>
__global__ __launch_bounds__(256) void k_cg_update_coarse_b3(VT* __restrict__ x, VT* __restrict__ r,
                                                             const VT* __restrict__ p, const VT* __restrict__ q,
                                                             const VT* __restrict__ binv, long nn,
                                                             const double* __restrict__ part_pq, int n_pq,
                                                             double* __restrict__ scal, int it, CoarseArgs ca,
                                                             double* __restrict__ part_z, double* __restrict__ part) {
  // a finished solve stores nothing; the flag is read with the loads below
  // and tested once they are requested (one round trip instead of two)
  const double done = scal[S_DONE];
  __shared__ double sh[8];
  __shared__ double acc[COARSE_KMAX];
  __shared__ double red[COARSE_NFMAX * 3][256];
  const int nf = ca.nf, R = ca.R, k = 3 * nf * R;
  const long n3 = 3 * nn;
  long lo, hi;
  block_range(nn, lo, hi);
  const double pq = sum_partials(part_pq, n_pq, sh);
  if (done != 0.0) return;
  const double rz = scal[S_RZ0 + (it & 1)];
  if (!(pq > 0.0) || !(pq < 1e300) || !(rz == rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_DONE] = 2.0;
    return;
  }
  for (int j = threadIdx.x; j < k; j += blockDim.x) acc[j] = 0.0;
  zt_loop_clear(ca.det, red);
  __syncthreads();
  double* const acc_l = zt_loop_acc(ca.det, acc, red);
  const VT alpha = (VT)(rz / pq);
  ZtAcc a;
  zt_clear(a, -1);
  double srz = 0.0, srr = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    VT rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[3 * i + c] += alpha * p[3 * i + c];
      rv[c] = r[3 * i + c] - alpha * q[3 * i + c];
      r[3 * i + c] = rv[c];
    }
    block_apply<VT>(binv + 6 * i, rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      srz += (double)rv[c] * (double)zv[c];
      srr += (double)rv[c] * (double)rv[c];
      double fv[COARSE_NFMAX];
      const int g = coarse_fields(ca, 3 * i + c, n3, fv);
      zt_add(a, acc_l, fv, nf, R, g, c, (double)rv[c]);
    }
  }
  zt_flush(a, acc, nf, R, lo < hi ? coarse_region(ca, (int)lo) : 0, red, ca.det);
  __syncthreads();
  zt_store(acc, k, part_z);
  block_sum2(srz, srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[RED_BLOCKS + blockIdx.x] = srr;
  }
}

#ifndef AMRTO_COARSE_REC
#define AMRTO_COARSE_REC 1
#endif
constexpr int CT_REFRESH = 64;

// Update pass of the coarse-space solve in recurrence form (octree mesh,
// affine space; the operator pass formed the per-block partials of Z^T q and
// E^-1 Z^T q).  Blocks below RED_BLOCKS: x += alpha p, r -= alpha q and the
// partials of r^T M r and r^T r, one node per step (M = the Jacobi diagonal,
// 3 entries per node, or with B3 the inverse node blocks, 6 entries).  Block
// RED_BLOCKS + j: ct[j] -= alpha (Z^T q)_j and cz[j] -= alpha (E^-1 Z^T q)_j,
// so that ct = Z^T r and cz = E^-1 ct hold for the new r up to rounding (both
// are formed from r again every CT_REFRESH iterations).
template <typename VT, bool B3>
__global__ __launch_bounds__(256) void k_cg_update_rec(VT* __restrict__ x, VT* __restrict__ r,
                                                       const VT* __restrict__ p, const VT* __restrict__ q,
                                                       const VT* __restrict__ minv, long nn,
                                                       const double* __restrict__ part_pq, int n_pq,
                                                       double* __restrict__ scal, int it,
                                                       const double* __restrict__ qpart, int nb, int kk,
                                                       double* __restrict__ ct, double* __restrict__ cz,
                                                       double* __restrict__ part) {
  // a finished solve stores nothing; the flag is read with the loads below
  // and tested once they are requested (one round trip instead of two)
  const double done = scal[S_DONE];
  __shared__ double sh[16];
  constexpr int MW = B3 ? 6 : 3;
  const bool col = blockIdx.x >= RED_BLOCKS;
  const int j = (int)blockIdx.x - RED_BLOCKS;
  const long i0 = blockIdx.x * (long)blockDim.x + threadIdx.x, stride = (long)RED_BLOCKS * blockDim.x;
  // the first UPT nodes of this thread (meshes larger than the grid give a
  // thread more than one), and the column sums, requested before the p.q
  // partials are reduced
  constexpr int UPT = 2;
  VT xv[UPT][3], pv[UPT][3], rv[UPT][3], qv[UPT][3], mv[UPT][MW];
#pragma unroll
  for (int u = 0; u < UPT; ++u) {
    const long i = i0 + u * stride;
    const bool in = !col && i < nn;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xv[u][c] = in ? x[3 * i + c] : (VT)0;
      pv[u][c] = in ? p[3 * i + c] : (VT)0;
      rv[u][c] = in ? r[3 * i + c] : (VT)0;
      qv[u][c] = in ? q[3 * i + c] : (VT)0;
    }
#pragma unroll
    for (int c = 0; c < MW; ++c) mv[u][c] = in ? minv[MW * i + c] : (VT)0;
  }
  double s1 = 0.0, s2 = 0.0;
  if (col)
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      s1 += qpart[(long)j * nb + b];
      s2 += qpart[(long)(kk + j) * nb + b];
    }
  const double pq = sum_partials(part_pq, n_pq, sh);
  if (done != 0.0) return;
  const double rz = scal[S_RZ0 + (it & 1)];
  if (!(pq > 0.0) || !(pq < 1e300) || !(rz == rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_DONE] = 2.0;
    return;
  }
  const VT alpha = (VT)(rz / pq);
  if (col) {
    block_sum2(s1, s2, sh);
    if (threadIdx.x == 0) {
      ct[j] -= (double)alpha * s1;
      cz[j] -= (double)alpha * s2;
    }
    return;
  }
  double srz = 0.0, srr = 0.0;
  auto node = [&](long i, const VT* xl, const VT* pl, const VT* rl, const VT* ql, const VT* ml) {
    VT rn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[3 * i + c] = xl[c] + alpha * pl[c];
      rn[c] = rl[c] - alpha * ql[c];
      r[3 * i + c] = rn[c];
      srr += (double)rn[c] * (double)rn[c];
    }
    if (B3) {
      VT zn[3];
      block_apply<VT>(ml, rn, zn);
#pragma unroll
      for (int c = 0; c < 3; ++c) srz += (double)rn[c] * (double)zn[c];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) srz += (double)rn[c] * (double)ml[c] * (double)rn[c];
    }
  };
#pragma unroll
  for (int u = 0; u < UPT; ++u) {
    const long i = i0 + u * stride;
    if (i < nn) node(i, xv[u], pv[u], rv[u], qv[u], mv[u]);
  }
  for (long i = i0 + UPT * stride; i < nn; i += stride) {
    VT xl[3], pl[3], rl[3], ql[3], ml[MW];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xl[c] = x[3 * i + c];
      pl[c] = p[3 * i + c];
      rl[c] = r[3 * i + c];
      ql[c] = q[3 * i + c];
    }
#pragma unroll
    for (int c = 0; c < MW; ++c) ml[c] = minv[MW * i + c];
    node(i, xl, pl, rl, ql, ml);
  }
  block_sum2(srz, srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[RED_BLOCKS + blockIdx.x] = srr;
  }
}

// ct[j] = sum_b part[j nblk + b]: one block per coarse column, fixed-tree sum
// (deterministic).
__global__ __launch_bounds__(256) void k_coarse_sum(const double* __restrict__ part, int k, int nblk,
                                                    double* __restrict__ ct, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double sh[8];
  const int j = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += part[(long)j * nblk + b];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) ct[j] = v;
}

// cz = E^-1 ct in one block of G x kp threads: thread (g, j) sums the rows
// i = g, g + G, ... of column j of the symmetric E^-1 (each row read coalesced
// across j), so all of E^-1 is requested at once; the G group sums are added
// in group order and ct^T cz in column order (deterministic).
__global__ __launch_bounds__(1024) void k_coarse_cz(const double* __restrict__ ct_g, int k,
                                                    const double* __restrict__ Einv, double* __restrict__ cz,
                                                    double* __restrict__ ctz, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double ct[COARSE_KMAX], prod[COARSE_KMAX], grp[1024];
  const int kp = ((k + 63) / 64) * 64, G = (int)blockDim.x / kp;
  for (int i = threadIdx.x; i < k; i += blockDim.x) ct[i] = ct_g[i];
  __syncthreads();
  const int j = threadIdx.x % kp, g = threadIdx.x / kp;
  if (j < k && g < G) {
    double s = 0.0;
    for (int i = g; i < k; i += G) s += Einv[(long)i * k + j] * ct[i];
    grp[g * kp + j] = s;
  }
  __syncthreads();
  if (threadIdx.x < k) {
    double s = 0.0;
    for (int q = 0; q < G; ++q) s += grp[q * kp + threadIdx.x];
    cz[threadIdx.x] = s;
    prod[threadIdx.x] = ct[threadIdx.x] * s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < k; ++i) t += prod[i];
    *ctz = t;
  }
}

// z = D^-1 r + Z cz; partials r.z, r.r
template <typename VT>
__global__ __launch_bounds__(256) void k_coarse_z(const VT* __restrict__ r, VT* __restrict__ z,
                                                  const VT* __restrict__ dinv, long n, const double* __restrict__ cz_g,
                                                  CoarseArgs ca, double* __restrict__ part,
                                                  const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double sh[8];
  __shared__ double cz[COARSE_KMAX];
  const int nf = ca.nf, R = ca.R, k = 3 * nf * R;
  for (int j = threadIdx.x; j < k; j += blockDim.x) cz[j] = cz_g[j];
  __syncthreads();
  double srz = 0.0, srr = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double fv[COARSE_NFMAX];
    const int g = coarse_fields(ca, i, n, fv);
    const int c = (int)(i % 3);
    const VT ri = r[i];
    double zi = (double)dinv[i] * (double)ri;
    // the fields are zero on supported and hanging DOFs, so z stays zero there
#pragma unroll
    for (int f = 0; f < COARSE_NFMAX; ++f)
      if (f < nf) zi += fv[f] * cz[(f * R + g) * 3 + c];
    z[i] = (VT)zi;
    srz += (double)ri * zi;
    srr += (double)ri * (double)ri;
  }
  block_sum2(srz, srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[RED_BLOCKS + blockIdx.x] = srr;
  }
}

// r = b - q in FP64 and partials r.r, b.b (true residual)
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ b, const double* __restrict__ q,
                                                  double* __restrict__ r, long n, double* __restrict__ part) {
  __shared__ double sh[8];
  double rr = 0.0, bb = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double ri = b[i] - q[i];
    r[i] = ri;
    rr += ri * ri;
    bb += b[i] * b[i];
  }
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rr;
    part[RED_BLOCKS + blockIdx.x] = bb;
  }
}

__global__ __launch_bounds__(256) void k_residual_scalars(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[8];
  const double rr = sum_partials(part, RED_BLOCKS, sh);
  const double bb = sum_partials(part + RED_BLOCKS, RED_BLOCKS, sh);
  if (threadIdx.x == 0) {
    out[0] = rr;
    out[1] = bb;
  }
}

__global__ void k_set_scalar(double* __restrict__ scal, int idx, double v) { scal[idx] = v; }

// x64 += x32; x32 = 0   (reliable update of the FP64 iterate)
__global__ __launch_bounds__(256) void k_accumulate(double* __restrict__ x, float* __restrict__ d, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) {
    x[i] += (double)d[i];
    d[i] = 0.f;
  }
}

// ------------------------------------------------------------------ host
template <typename VT>
struct Vecs {
  VT *r, *z, *p0, *p1, *q;
  const VT* dinv;
};
static Vecs<double> vecs64(amrto_ctx* c) { return {c->d_r, c->d_z, c->d_p, c->d_p2, c->d_q, c->d_dinv}; }
static Vecs<float> vecs32(amrto_ctx* c) { return {c->f_r, c->f_z, c->f_p, c->f_p2, c->f_q, c->d_dinv_f}; }

static CoarseArgs coarse_args(const amrto_ctx* ctx) {
  CoarseArgs a;
  a.F = ctx->d_cf; a.nf = ctx->coarse_nf; a.R = ctx->coarse_R; a.region = ctx->d_region;
  a.geo = ctx->coarse_affine_only ? ctx->d_cgeo : nullptr;
  a.det = ctx->deterministic ? 1 : 0;
  return a;
}

// G groups of kp threads (kp = columns rounded to whole wavefronts), G as
// large as 1024 threads allow
static int cz_threads(const amrto_ctx* ctx) {
  const int kp = ((ctx->coarse_k + 63) / 64) * 64;
  return (1024 / kp) * kp;
}

// The affine coarse space on an octree mesh is folded into the operator pass
// (z = M1 r + Z cz formed while staging, M1 the Jacobi diagonal or the inverse
// node blocks; r.z = r^T M1 r + ct^T cz), in the recurrence form of
// k_cg_update_rec unless built with AMRTO_COARSE_REC=0.
static bool coarse_fused(const amrto_ctx* ctx) {
  return ctx->coarse_k > 0 && !ctx->uniform && ctx->coarse_affine_only;
}

// with a coarse space: cz = E^-1 Z^T r for the initial residual and either
// z = D^-1 r + Z cz (overwriting the r.z and r.r partials of k_init; b.b
// stays) or, in the fused form, ct^T cz in its scalar slot (the partials of
// k_init already are r^T D^-1 r and r^T r)
// ct = Z^T r and cz = E^-1 ct (and ct^T cz) formed from r
template <typename VT>
static void coarse_exact(amrto_ctx* ctx, const VT* r, const double* stop) {
  hipLaunchKernelGGL(k_zt_part<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, coarse_args(ctx), r,
                     3L * ctx->n_nodes, ctx->d_cpart);
  hipLaunchKernelGGL(k_coarse_sum, dim3(ctx->coarse_k), dim3(256), 0, ctx->stream, ctx->d_cpart, ctx->coarse_k,
                     RED_BLOCKS, ctx->d_ct, stop);
  hipLaunchKernelGGL(k_coarse_cz, dim3(1), dim3(cz_threads(ctx)), 0, ctx->stream, (const double*)ctx->d_ct,
                     ctx->coarse_k, (const double*)ctx->d_cinv, ctx->d_cz, ctx->d_scal + S_CTZ, stop);
}

template <typename VT>
static void coarse_init(amrto_ctx* ctx, const Vecs<VT>& v) {
  if (ctx->coarse_k <= 0) return;
  ctx->coarse_fresh = true;
  const long n3 = 3L * ctx->n_nodes;
  hipLaunchKernelGGL(k_zt_part<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, coarse_args(ctx), v.r, n3,
                     ctx->d_cpart);
  hipLaunchKernelGGL(k_coarse_sum, dim3(ctx->coarse_k), dim3(256), 0, ctx->stream, ctx->d_cpart, ctx->coarse_k,
                     RED_BLOCKS, ctx->d_ct, (const double*)nullptr);
  hipLaunchKernelGGL(k_coarse_cz, dim3(1), dim3(cz_threads(ctx)), 0, ctx->stream, (const double*)ctx->d_ct, ctx->coarse_k,
                     (const double*)ctx->d_cinv, ctx->d_cz, ctx->d_scal + S_CTZ, (const double*)nullptr);
  if (!coarse_fused(ctx))
    hipLaunchKernelGGL(k_coarse_z<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, v.r, v.z, v.dinv, n3, ctx->d_cz,
                       coarse_args(ctx), ctx->d_part, (const double*)nullptr);
}

int launch_zt(amrto_ctx* ctx, const double* v) {
  hipLaunchKernelGGL(k_zt_part<double>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, coarse_args(ctx), v,
                     3L * ctx->n_nodes, ctx->d_cpart);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int mask_vector_n(amrto_ctx* ctx, double* x, int count) {
  for (int i = 0; i < count; ++i) {
    int rc = mask_vector(ctx, x + 3L * ctx->n_nodes * i);
    if (rc) return rc;
  }
  return AMRTO_OK;
}

int mask_vector(amrto_ctx* ctx, double* x) {
  const long n3 = 3L * ctx->n_nodes;
  hipLaunchKernelGGL(k_mask<double>, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, x, ctx->d_fix, n3);
  if (ctx->n_hang)
    hipLaunchKernelGGL(k_mask_hanging<double>, dim3((3L * ctx->n_hang + 255) / 256), dim3(256), 0, ctx->stream, x,
                       ctx->d_hang_node, ctx->n_hang);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

static int read_scalars(amrto_ctx* ctx) {
  AMRTO_HIP(hipMemcpyAsync(ctx->h_scal, ctx->d_scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  return AMRTO_OK;
}

// The two halves of CG iteration `it`: the fused operator pass (p = z + beta
// p_old, q = A~ p, p.q partials; with the fused coarse space z = M1 r + Z cz
// and, in the recurrence form, the Z^T q and E^-1 Z^T q partials) ...
template <typename VT>
static int enqueue_op_pass(amrto_ctx* ctx, const Vecs<VT>& v, int prec, double tol2, int it, bool block3) {
  const bool fused = coarse_fused(ctx);
  const bool rec = fused && AMRTO_COARSE_REC && ctx->d_cqpart;
  VT* pnew = (it & 1) ? v.p1 : v.p0;
  VT* pold = (it & 1) ? v.p0 : v.p1;
  CgArgs cg{ctx->d_scal, ctx->d_part, ctx->d_partpq, 0, it, tol2, (fused && !rec) ? 1 : 0};
  const VT* binv = nullptr;
  if (block3) {
    if constexpr (std::is_same<VT, double>::value) binv = ctx->d_binv;
    else binv = ctx->d_binv_f;
  }
  return fused ? apply_fused_coarse(ctx, v.r, block3 ? (const void*)binv : (const void*)v.dinv, pold, pnew, v.q, prec,
                                    cg, block3, rec ? ctx->d_cqpart : nullptr)
               : apply_fused(ctx, v.z, pold, pnew, v.q, prec, cg);
}

// ... and the update side (alpha, x, r, z = M^-1 r, the r.z and r.r partials,
// and the coarse-space launches that follow it).
template <typename VT>
static int enqueue_update(amrto_ctx* ctx, const Vecs<VT>& v, VT* x, int it, bool block3) {
  const long n3 = 3L * ctx->n_nodes;
  const bool fused = coarse_fused(ctx);
  const bool rec = fused && AMRTO_COARSE_REC && ctx->d_cqpart;
  VT* pnew = (it & 1) ? v.p1 : v.p0;
  const VT* binv = nullptr;
  if (block3) {
    if constexpr (std::is_same<VT, double>::value) binv = ctx->d_binv;
    else binv = ctx->d_binv_f;
  }
  if (rec) {
    const int nb = apply_blocks(ctx);
    if (block3)
      hipLaunchKernelGGL((k_cg_update_rec<VT, true>), dim3(RED_BLOCKS + ctx->coarse_k), dim3(256), 0, ctx->stream,
                         x, v.r, pnew, v.q, binv, (long)ctx->n_nodes, ctx->d_partpq, ctx->n_partpq, ctx->d_scal,
                         it, (const double*)ctx->d_cqpart, nb, ctx->coarse_k, ctx->d_ct, ctx->d_cz,
                         ctx->d_part);
    else
      hipLaunchKernelGGL((k_cg_update_rec<VT, false>), dim3(RED_BLOCKS + ctx->coarse_k), dim3(256), 0,
                         ctx->stream, x, v.r, pnew, v.q, (const VT*)v.dinv, (long)ctx->n_nodes, ctx->d_partpq,
                         ctx->n_partpq, ctx->d_scal, it, (const double*)ctx->d_cqpart, nb, ctx->coarse_k,
                         ctx->d_ct, ctx->d_cz, ctx->d_part);
  } else if (ctx->coarse_k > 0) {
    if (block3)  // coarse_fused holds (checked in amrto_pcg)
      hipLaunchKernelGGL(k_cg_update_coarse_b3<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, x, v.r, pnew,
                         v.q, binv, (long)ctx->n_nodes, ctx->d_partpq, ctx->n_partpq, ctx->d_scal, it,
                         coarse_args(ctx), ctx->d_cpart, ctx->d_part);
    else
      hipLaunchKernelGGL(k_cg_update_coarse<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, x, v.r, pnew, v.q,
                         v.dinv, n3, ctx->d_partpq, ctx->n_partpq, ctx->d_scal, it, coarse_args(ctx),
                         ctx->d_cpart, ctx->d_part);
    hipLaunchKernelGGL(k_coarse_sum, dim3(ctx->coarse_k), dim3(256), 0, ctx->stream, ctx->d_cpart,
                       ctx->coarse_k, RED_BLOCKS, ctx->d_ct, ctx->d_scal + S_DONE);
    hipLaunchKernelGGL(k_coarse_cz, dim3(1), dim3(cz_threads(ctx)), 0, ctx->stream, (const double*)ctx->d_ct, ctx->coarse_k,
                       (const double*)ctx->d_cinv, ctx->d_cz, ctx->d_scal + S_CTZ, ctx->d_scal + S_DONE);
    if (!fused)
      hipLaunchKernelGGL(k_coarse_z<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, v.r, v.z, v.dinv, n3,
                         ctx->d_cz, coarse_args(ctx), ctx->d_part, ctx->d_scal + S_DONE);
  } else if (block3) {
    const int rc = block3_update<VT>(ctx, x, v.r, pnew, v.q, v.z, it);
    if (rc) return rc;
  } else {
    hipLaunchKernelGGL(k_cg_update<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, x, v.r, pnew, v.q, v.dinv,
                       v.z, n3, ctx->d_partpq, ctx->n_partpq, ctx->d_scal, it, ctx->d_part);
  }
  return AMRTO_OK;
}

// enqueue CG iterations [it0, it0 + count) on the current r, z (and p from it0 - 1)
template <typename VT>
static int enqueue_iters(amrto_ctx* ctx, const Vecs<VT>& v, VT* x, int prec, double tol2, int it0, int count,
                         bool block3 = false) {
  const bool fused = coarse_fused(ctx);
  const bool rec = fused && AMRTO_COARSE_REC && ctx->d_cqpart;
  if (rec && ctx->coarse_fresh) {
    ctx->coarse_fresh = false;
    ctx->coarse_exact_it = it0;
  }
  for (int it = it0; it < it0 + count; ++it) {
    // ct and cz follow r by recurrences; every CT_REFRESH iterations they are
    // formed from r again, so rounding cannot accumulate without bound
    if (rec && it - ctx->coarse_exact_it >= CT_REFRESH) {
      coarse_exact(ctx, v.r, ctx->d_scal + S_DONE);
      ctx->coarse_exact_it = it;
    }
    int rc = enqueue_op_pass<VT>(ctx, v, prec, tol2, it, block3);
    if (!rc) rc = enqueue_update<VT>(ctx, v, x, it, block3);
    if (!rc && ctx->rec_active) rc = recycle_store<VT>(ctx, v.r, it);
    if (rc) return rc;
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

static int true_residual(amrto_ctx* ctx, const double* b, const double* x, double* rr, double* bb);

// Time the two halves of one CG iteration of a solver variant: the solve is
// started as amrto_pcg starts it (from x, with a stopping target of zero so
// the recurrence cannot stop) and run for two iterations; then the operator
// pass of iteration 2 is launched `reps` times back to back (it reads the
// same inputs each time and rewrites the same outputs), then its update side
// `reps` times, each group between two events on the context stream.
template <typename VT>
static int pass_times(amrto_ctx* ctx, const double* b, double* x, int prec, bool block3, int reps, float* op_ms,
                      float* up_ms) {
  const long n3 = 3L * ctx->n_nodes;
  const int g1 = (int)((n3 + 255) / 256);
  Vecs<VT> v{};
  VT* xi = nullptr;
  hipLaunchKernelGGL(k_mask<double>, dim3(g1), dim3(256), 0, ctx->stream, x, ctx->d_fix, n3);
  if (ctx->n_hang)
    hipLaunchKernelGGL(k_mask_hanging<double>, dim3((3L * ctx->n_hang + 255) / 256), dim3(256), 0, ctx->stream, x,
                       ctx->d_hang_node, ctx->n_hang);
  if (block3) {
    const int rc = block3_setup(ctx);
    if (rc) return rc;
  }
  if constexpr (std::is_same<VT, double>::value) {
    v = vecs64(ctx);
    xi = x;
    int rc = apply_stop(ctx, x, v.q, AMRTO_FP64, nullptr);
    if (rc) return rc;
    if (block3) {
      rc = block3_init<double, double>(ctx, b, v.q, v.r, v.z);
      if (rc) return rc;
    } else {
      hipLaunchKernelGGL((k_init<double, double>), dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, b, v.q, v.r, v.z,
                         v.dinv, n3, ctx->d_part);
    }
  } else {
    v = vecs32(ctx);
    xi = ctx->f_x;
    hipLaunchKernelGGL(k_fill<float>, dim3(g1), dim3(256), 0, ctx->stream, ctx->f_x, n3);
    double rr, bb;
    int rc = true_residual(ctx, b, x, &rr, &bb);
    if (rc) return rc;
    if (block3) {
      rc = block3_init<float, double>(ctx, ctx->d_r, (const double*)nullptr, v.r, v.z);
      if (rc) return rc;
    } else {
      hipLaunchKernelGGL((k_init<float, double>), dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, ctx->d_r,
                         (const double*)nullptr, v.r, v.z, v.dinv, n3, ctx->d_part);
    }
  }
  coarse_init<VT>(ctx, v);
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(256), 0, ctx->stream, ctx->d_part, ctx->d_scal, 0.0, 0,
                     coarse_fused(ctx) ? 1 : 0);
  int rc = enqueue_iters<VT>(ctx, v, xi, prec, 0.0, 0, 2, block3);
  if (rc) return rc;
  hipEvent_t e[3] = {nullptr, nullptr, nullptr};
  for (auto& ev : e) AMRTO_HIP(hipEventCreate(&ev));
  struct Ev {
    hipEvent_t* e;
    ~Ev() { for (int i = 0; i < 3; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
  } guard{e};
  AMRTO_HIP(hipEventRecord(e[0], ctx->stream));
  for (int i = 0; i < reps && !rc; ++i) rc = enqueue_op_pass<VT>(ctx, v, prec, 0.0, 2, block3);
  AMRTO_HIP(hipEventRecord(e[1], ctx->stream));
  for (int i = 0; i < reps && !rc; ++i) rc = enqueue_update<VT>(ctx, v, xi, 2, block3);
  AMRTO_HIP(hipEventRecord(e[2], ctx->stream));
  if (rc) return rc;
  AMRTO_HIP(hipGetLastError());
  AMRTO_HIP(hipEventSynchronize(e[2]));
  AMRTO_HIP(hipEventElapsedTime(op_ms, e[0], e[1]));
  AMRTO_HIP(hipEventElapsedTime(up_ms, e[1], e[2]));
  // nothing of this run is a result: the finished flag stops any later
  // kernel of this state, and the next solve starts afresh
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, ctx->stream, ctx->d_scal, (int)S_DONE, 2.0);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

// u = M^-1 s with the preconditioner of a solve: M1 = D^-1 (or the inverse
// node blocks) plus, with a coarse space, Z E^-1 Z^T s (FP64 copies).
__global__ __launch_bounds__(256) void k_apply_m1(const double* __restrict__ s, double* __restrict__ u,
                                                  const double* __restrict__ dinv, const double* __restrict__ binv,
                                                  long n_nodes) {
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < n_nodes; v += (long)gridDim.x * blockDim.x) {
    const double r0 = s[3 * v], r1 = s[3 * v + 1], r2 = s[3 * v + 2];
    if (binv) {
      const double* b = binv + 6 * v;  // (B00, B11, B22, B01, B02, B12)
      u[3 * v] = b[0] * r0 + b[3] * r1 + b[4] * r2;
      u[3 * v + 1] = b[3] * r0 + b[1] * r1 + b[5] * r2;
      u[3 * v + 2] = b[4] * r0 + b[5] * r1 + b[2] * r2;
    } else {
      u[3 * v] = dinv[3 * v] * r0;
      u[3 * v + 1] = dinv[3 * v + 1] * r1;
      u[3 * v + 2] = dinv[3 * v + 2] * r2;
    }
  }
}

__global__ __launch_bounds__(256) void k_add_zcz(double* __restrict__ u, long n, const double* __restrict__ cz_g,
                                                 CoarseArgs ca) {
  __shared__ double cz[COARSE_KMAX];
  const int nf = ca.nf, R = ca.R, k = 3 * nf * R;
  for (int j = threadIdx.x; j < k; j += blockDim.x) cz[j] = cz_g[j];
  __syncthreads();
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double fv[COARSE_NFMAX];
    const int g = coarse_fields(ca, i, n, fv);
    const int c = (int)(i % 3);
    double add = 0.0;
#pragma unroll
    for (int f = 0; f < COARSE_NFMAX; ++f)
      if (f < nf) add += fv[f] * cz[(f * R + g) * 3 + c];
    u[i] += add;
  }
}

int apply_precond(amrto_ctx* ctx, const double* s, double* u, bool block3, bool coarse) {
  const long n3 = 3L * ctx->n_nodes;
  hipLaunchKernelGGL(k_apply_m1, dim3(grid_for(ctx->n_nodes, 256, 2048)), dim3(256), 0, ctx->stream, s, u,
                     (const double*)ctx->d_dinv, block3 ? (const double*)ctx->d_binv : nullptr, (long)ctx->n_nodes);
  if (coarse && ctx->coarse_k > 0) {
    hipLaunchKernelGGL(k_zt_part<double>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, coarse_args(ctx), s, n3,
                       ctx->d_cpart);
    hipLaunchKernelGGL(k_coarse_sum, dim3(ctx->coarse_k), dim3(256), 0, ctx->stream, ctx->d_cpart, ctx->coarse_k,
                       RED_BLOCKS, ctx->d_ct, (const double*)nullptr);
    hipLaunchKernelGGL(k_coarse_cz, dim3(1), dim3(cz_threads(ctx)), 0, ctx->stream, (const double*)ctx->d_ct,
                       ctx->coarse_k, (const double*)ctx->d_cinv, ctx->d_cz, ctx->d_scal + S_CTZ,
                       (const double*)nullptr);
    hipLaunchKernelGGL(k_add_zcz, dim3(grid_for(n3, 256, 2048)), dim3(256), 0, ctx->stream, u, n3,
                       (const double*)ctx->d_cz, coarse_args(ctx));
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

// Iterations to enqueue before the next host check.  Every check drains the
// stream (the device idles until the next batch is queued), and every
// iteration queued past convergence is a pair of launches that return at
// once.  So: check_every while nothing is known; then 3/4 of the iterations
// the residual still needs to reach `target`, at the faster of its mean rate
// since rr0 (its iterations ago) and its rate over the last batch (log r.r
// falls about linearly in CG), between check_every and 8 check_every.
int next_batch(double rr0, double rr_prev, double rr, int its, int last, double target, int check_every,
               int left) {
  int n = check_every;
  if (its > 0 && last > 0 && rr0 > 0.0 && rr_prev > 0.0 && target > 0.0 && rr > target && rr < rr0) {
    double rate = std::log(rr / rr0) / its;
    if (rr < rr_prev) rate = std::min(rate, std::log(rr / rr_prev) / last);
    const double need = std::log(target / rr) / rate;
    n = (int)std::min(8.0 * check_every, std::max((double)check_every, 0.75 * need));
  }
  return std::max(1, std::min(n, left));
}

// Plain FP64 Jacobi-PCG from x (masked).  *iters = iterations performed.
static int cg_fp64_run(amrto_ctx* ctx, const double* b, double* x, double rtol, int max_it, int check_every,
                       bool one_reduction, bool block3, int* iters) {
  const long n3 = 3L * ctx->n_nodes;
  const int g1 = (int)((n3 + 255) / 256);
  Vecs<double> v = vecs64(ctx);
  const double tol2 = rtol * rtol;
  hipLaunchKernelGGL(k_mask<double>, dim3(g1), dim3(256), 0, ctx->stream, x, ctx->d_fix, n3);
  if (ctx->n_hang)
    hipLaunchKernelGGL(k_mask_hanging<double>, dim3((3L * ctx->n_hang + 255) / 256), dim3(256), 0, ctx->stream, x,
                       ctx->d_hang_node, ctx->n_hang);
  int rc = apply_stop(ctx, x, v.q, AMRTO_FP64, nullptr);
  if (rc) return rc;
  if (block3) {
    rc = block3_setup(ctx);
    if (!rc) rc = block3_init<double, double>(ctx, b, v.q, v.r, v.z);
    if (rc) return rc;
  } else {
    hipLaunchKernelGGL((k_init<double, double>), dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, b, v.q, v.r, v.z,
                       v.dinv, n3, ctx->d_part);
  }
  coarse_init<double>(ctx, v);
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(256), 0, ctx->stream, ctx->d_part, ctx->d_scal, tol2, 0,
                     coarse_fused(ctx) ? 1 : 0);
  AMRTO_HIP(hipGetLastError());
  if (ctx->rec_active) {
    rc = recycle_begin(ctx, block3);
    if (!rc) rc = recycle_store<double>(ctx, v.r, -1);
    if (rc) return rc;
  }
  // one reduction per iteration where the recurrences allow it (octree mesh,
  // Jacobi preconditioner)
  const bool one = one_reduction && !block3 && ctx->coarse_k <= 0 && !ctx->rec_active && cg1_available(ctx);
  if (one) {
    rc = cg1_init(ctx);
    if (rc) return rc;
  }
  int it = 0, last = 0;
  int status = AMRTO_NOT_CONVERGED;
  double rr0 = 0.0, rr_prev = 0.0;
  while (true) {
    rc = read_scalars(ctx);
    if (rc) return rc;
    const double done = ctx->h_scal[S_DONE];
    if (done == 1.0) { status = AMRTO_OK; break; }
    if (done == 2.0) { status = AMRTO_EBREAKDOWN; break; }
    if (it >= max_it) break;
    const double rr = ctx->h_scal[S_RR];
    if (it == 0) rr0 = rr;
    const int batch = next_batch(rr0, rr_prev, rr, it, last, tol2 * ctx->h_scal[S_BB], check_every, max_it - it);
    rr_prev = rr;
    rc = one ? cg1_enqueue(ctx, x, tol2, it, batch)
             : enqueue_iters<double>(ctx, v, x, AMRTO_FP64, tol2, it, batch, block3);
    if (rc) return rc;
    it += batch;
    last = batch;
  }
  *iters = status == AMRTO_NOT_CONVERGED ? it : (int)ctx->h_scal[S_ITERS];
  return status;
}

// true FP64 residual of A~ x = b: *rel = ||b - A~ x|| / ||b||; r left in d_r
static int true_residual(amrto_ctx* ctx, const double* b, const double* x, double* rr, double* bb) {
  const long n3 = 3L * ctx->n_nodes;
  int rc = apply_stop(ctx, x, ctx->d_q, AMRTO_FP64, nullptr);
  if (rc) return rc;
  hipLaunchKernelGGL(k_residual, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, b, ctx->d_q, ctx->d_r, n3,
                     ctx->d_part);
  hipLaunchKernelGGL(k_residual_scalars, dim3(1), dim3(256), 0, ctx->stream, ctx->d_part, ctx->d_scal + 6);
  AMRTO_HIP(hipGetLastError());
  rc = read_scalars(ctx);
  if (rc) return rc;
  *rr = ctx->h_scal[6];
  *bb = ctx->h_scal[7];
  return AMRTO_OK;
}

// Plain FP64 PCG judged on the true residual.  Over long solves the
// recurrence residual of CG drifts away from b - A~ x (the attainable
// accuracy of the method); when the recurrence claims convergence but the
// true residual is still above the target, the search restarts from the
// current iterate with r = b - A~ x (residual replacement), as long as that
// keeps paying off (at most 8 restarts, each must halve the true residual).
static int cg_fp64(amrto_ctx* ctx, const double* b, double* x, double rtol, int max_it, int check_every,
                   bool one_reduction, bool block3, int* iters, int* restarts, double* rel_out) {
  int total = 0, status = AMRTO_NOT_CONVERGED;
  double best = 1e300;
  *restarts = 0;
  while (true) {
    int it = 0;
    status = cg_fp64_run(ctx, b, x, rtol, max_it - total, check_every, one_reduction, block3, &it);
    ctx->rec_active = false;  // a restart starts another Krylov space: only the first run is recorded
    total += it;
    if (status < 0 && status != AMRTO_EBREAKDOWN) return status;
    double rr, bb;
    int rc = true_residual(ctx, b, x, &rr, &bb);
    if (rc) return rc;
    const double rel = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    *rel_out = rel;
    if (status != AMRTO_OK) break;  // breakdown or iteration cap
    if (rel <= rtol) break;
    if (*restarts >= 8 || !(rel < 0.5 * best) || total >= max_it) {
      status = AMRTO_NOT_CONVERGED;
      break;
    }
    best = rel;
    ++*restarts;
  }
  *iters = total;
  return status;
}

// Mixed precision: the CG recurrence runs in FP32 vectors with an FP32 or
// BF16 operator on d = A~^-1 r0; whenever the recurrence residual has dropped
// by `delta` since the last reliable update (or claims convergence), the FP32
// correction is added to the FP64 iterate, the true FP64 residual replaces the
// recurrence residual and the search continues with the same direction p.
static int cg_mixed(amrto_ctx* ctx, const double* b, double* x, int prec, double rtol, int max_it,
                    int check_every, double delta, bool block3, int* iters, int* updates, double* rel_out) {
  const long n3 = 3L * ctx->n_nodes;
  const int g1 = (int)((n3 + 255) / 256);
  Vecs<float> v = vecs32(ctx);
  float* d = ctx->f_x;  // FP32 correction since the last reliable update
  hipLaunchKernelGGL(k_mask<double>, dim3(g1), dim3(256), 0, ctx->stream, x, ctx->d_fix, n3);
  if (ctx->n_hang)
    hipLaunchKernelGGL(k_mask_hanging<double>, dim3((3L * ctx->n_hang + 255) / 256), dim3(256), 0, ctx->stream, x,
                       ctx->d_hang_node, ctx->n_hang);
  hipLaunchKernelGGL(k_fill<float>, dim3(g1), dim3(256), 0, ctx->stream, d, n3);
  double rr = 0, bb = 0;
  int rc = true_residual(ctx, b, x, &rr, &bb);
  if (rc) return rc;
  const double tol2 = rtol * rtol;
  *updates = 0;
  int it = 0;
  int status = AMRTO_NOT_CONVERGED;
  double rr_ref = rr;  // true r.r at the last reliable update
  int stalls = 0;
  bool restart_scalars = true;
  // The FP32 recurrence can level off above its target (its attainable
  // accuracy on an ill-conditioned system): when its residual has not
  // dropped by 4 in STALL_WIN iterations, a reliable update is made anyway.
  constexpr int STALL_WIN = 2048;
  double rr_rec_best = 1e300;
  int since_gain = 0;
  // this cycle (since the last reliable update): r.r at its start, at the
  // last two checks, its iterations and the last batch
  double cyc_rr0 = rr, cyc_prev = 0.0, cyc_rr = rr;
  int cyc_its = 0, cyc_last = 0;
  while (true) {
    if (!(rr == rr) || rr > 1e300) { status = AMRTO_EBREAKDOWN; break; }
    if (rr <= tol2 * bb) { status = AMRTO_OK; break; }
    if (it >= max_it) break;
    if (restart_scalars) {
      // r32 = r64, z32 = M^-1 r32; r.z, r.r partials for the next operator pass
      if (block3) {
        rc = block3_init<float, double>(ctx, ctx->d_r, (const double*)nullptr, v.r, v.z);
        if (rc) return rc;
      } else {
        hipLaunchKernelGGL((k_init<float, double>), dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, ctx->d_r,
                           (const double*)nullptr, v.r, v.z, v.dinv, n3, ctx->d_part);
      }
      coarse_init<float>(ctx, v);
      if (ctx->rec_active && *updates == 0) {
        // the first cycle (up to the first reliable update) is one Krylov space
        rc = recycle_begin(ctx, block3);
        if (!rc) rc = recycle_store<float>(ctx, v.r, -1);
        if (rc) return rc;
      }
      // the recurrence measures its residual against b.b
      hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, ctx->stream, ctx->d_scal, (int)S_BB, bb);
      if (*updates == 0) {
        hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(256), 0, ctx->stream, ctx->d_part, ctx->d_scal, 0.0, 1,
                           coarse_fused(ctx) ? 1 : 0);
      } else {
        // continue the recurrence (same search direction): clear the stop flag
        hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, ctx->stream, ctx->d_scal, (int)S_DONE, 0.0);
      }
      restart_scalars = false;
      cyc_rr0 = cyc_rr = rr;
      cyc_prev = 0.0;
      cyc_its = cyc_last = 0;
    }
    // the recurrence stops itself when its own residual reaches delta^2 rr_ref
    const double tol_in = std::max(std::sqrt(delta * delta * rr_ref / bb), 0.5 * rtol);
    const int batch = next_batch(cyc_rr0, cyc_prev, cyc_rr, cyc_its, cyc_last, tol_in * tol_in * bb, check_every,
                                 max_it - it);
    rc = enqueue_iters<float>(ctx, v, d, prec, tol_in * tol_in, it, batch, block3);
    if (rc) return rc;
    rc = read_scalars(ctx);
    if (rc) return rc;
    const double done = ctx->h_scal[S_DONE];
    it = done != 0.0 ? (int)ctx->h_scal[S_ITERS] : it + batch;
    if (done == 2.0) { status = AMRTO_EBREAKDOWN; break; }
    bool stagnant = false;
    if (done == 0.0) {
      const double rr_rec = ctx->h_scal[S_RR];
      cyc_prev = cyc_rr;
      cyc_rr = rr_rec;
      cyc_its += batch;
      cyc_last = batch;
      if (rr_rec < 0.25 * rr_rec_best) {
        rr_rec_best = rr_rec;
        since_gain = 0;
      } else {
        since_gain += batch;
        stagnant = since_gain >= STALL_WIN;
      }
    }
    if (done == 1.0 || it >= max_it || stagnant) {
      ctx->rec_active = false;  // a reliable update ends the recorded cycle
      rr_rec_best = 1e300;
      since_gain = 0;
      // reliable update: x64 += d, true residual in FP64
      hipLaunchKernelGGL(k_accumulate, dim3(g1), dim3(256), 0, ctx->stream, x, d, n3);
      rc = true_residual(ctx, b, x, &rr, &bb);
      if (rc) return rc;
      // at the FP64 floor of the true residual the cycles stop paying off:
      // three updates in a row that fail to halve it end the solve
      stalls = (rr > 0.25 * rr_ref) ? stalls + 1 : 0;
      rr_ref = rr;
      ++*updates;
      restart_scalars = true;
      if (stalls >= 3 && !(rr <= tol2 * bb)) break;
    }
  }
  *iters = it;
  *rel_out = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
  return status;
}

}  // namespace amrto

using namespace amrto;

extern "C" {

int amrto_mask(amrto_ctx* ctx, double* x) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_mask: no mesh");
  if (!x) return ctx->fail(AMRTO_EINVAL, "amrto_mask: NULL buffer");
  AMRTO_HIP(hipSetDevice(ctx->device));
  return mask_vector(ctx, x);
}

void amrto_solve_opts_default(amrto_solve_opts* o) {
  if (!o) return;
  o->rtol = 1e-8;
  o->max_it = 20000;
  o->precond = AMRTO_PRECOND_JACOBI;
  o->inner_prec = AMRTO_FP64;
  o->inner_rtol = 0.1;
  o->check_every = 16;
  o->use_coarse = 1;
  o->fallback_fp64 = 1;
  o->single_reduction = 0;
  o->record = 0;
}

int amrto_pcg(amrto_ctx* ctx, const double* b, double* u, const amrto_solve_opts* opts_in,
              amrto_solve_stats* stats) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, "amrto_pcg: density not set");
  if (!b || !u || b == u) return ctx->fail(AMRTO_EINVAL, "amrto_pcg: b and u must be distinct device buffers");
  amrto_solve_opts o;
  amrto_solve_opts_default(&o);
  if (opts_in) o = *opts_in;
  if (!(o.rtol > 0.0) || o.max_it < 0 || o.check_every < 1 || !(o.inner_rtol > 0.0) ||
      !(o.inner_rtol < 1.0))
    return ctx->fail(AMRTO_EINVAL, "amrto_pcg: bad options");
  if (o.inner_prec != AMRTO_FP64 && o.inner_prec != AMRTO_FP32 && o.inner_prec != AMRTO_BF16)
    return ctx->fail(AMRTO_EINVAL, "amrto_pcg: unknown inner precision");
  if (o.precond != AMRTO_PRECOND_JACOBI && o.precond != AMRTO_PRECOND_BLOCK3)
    return ctx->fail(AMRTO_EINVAL, "amrto_pcg: unknown preconditioner");
  const bool block3 = o.precond == AMRTO_PRECOND_BLOCK3;
  if (block3 && o.use_coarse && ctx->coarse_k > 0 && !coarse_fused(ctx))
    return ctx->fail(AMRTO_EINVAL,
                     "amrto_pcg: block-Jacobi with a coarse space needs an octree mesh and the affine space");
  if (o.record && ctx->rec_m <= 0) return ctx->fail(AMRTO_ESTATE, "amrto_pcg: record needs amrto_recycle_setup");
  if (o.record && o.single_reduction) return ctx->fail(AMRTO_EINVAL, "amrto_pcg: record needs the two-pass form");
  AMRTO_HIP(hipSetDevice(ctx->device));
  struct RecOff {
    amrto_ctx* c;
    ~RecOff() { c->rec_active = false; }
  } rec_guard{ctx};
  ctx->rec_active = o.record != 0;
  if (o.record) ctx->rec_coarse = o.use_coarse && ctx->coarse_k > 0;
  // the solve loops read the coarse space from the context
  struct CoarseOff {
    amrto_ctx* c; int k;
    ~CoarseOff() { c->coarse_k = k; }
  } coarse_guard{ctx, ctx->coarse_k};
  if (!o.use_coarse) ctx->coarse_k = 0;
  const auto t0 = std::chrono::steady_clock::now();
  int iters = 0, outer = 0, status, fell_back = 0;
  double rel = 0.0;
  if (o.inner_prec == AMRTO_FP64) {
    status = cg_fp64(ctx, b, u, o.rtol, o.max_it, o.check_every, o.single_reduction != 0, block3, &iters, &outer,
                     &rel);
    if (status < 0 && status != AMRTO_EBREAKDOWN) return status;
  } else {
    if (block3) {
      const int rc = block3_setup(ctx);
      if (rc) return rc;
    }
    status = cg_mixed(ctx, b, u, o.inner_prec, o.rtol, o.max_it, o.check_every, o.inner_rtol, block3, &iters,
                      &outer, &rel);
    if (status < 0 && status != AMRTO_EBREAKDOWN) return status;
    if (status != AMRTO_OK && o.fallback_fp64 && iters < o.max_it) {
      // the plain FP64 solve takes over (and judges), from the mixed iterate
      if (!(rel == rel) || rel > 1e300)
        hipLaunchKernelGGL(k_fill<double>, dim3((int)((3L * ctx->n_nodes + 255) / 256)), dim3(256), 0, ctx->stream, u,
                           3L * ctx->n_nodes);
      int it2 = 0, restarts = 0;
      status = cg_fp64(ctx, b, u, o.rtol, o.max_it - iters, o.check_every, o.single_reduction != 0, block3, &it2,
                       &restarts, &rel);
      if (status < 0 && status != AMRTO_EBREAKDOWN) return status;
      iters += it2;
      fell_back = 1;
    }
  }
  int rc = launch_recover(ctx, u, u);
  if (rc) return rc;
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) {
    stats->iters = iters;
    stats->outer = outer;
    stats->rel_res = rel;
    stats->ms = ms;
    stats->fell_back = fell_back;
  }
  if (status == AMRTO_EBREAKDOWN) return ctx->fail(AMRTO_EBREAKDOWN, "amrto_pcg: breakdown (p^T A p <= 0 or non-finite)");
  if (status == AMRTO_NOT_CONVERGED) {
    char msg[160];
    if (iters >= o.max_it)
      std::snprintf(msg, sizeof msg, "amrto_pcg: iteration cap reached (relative residual %.3e)", rel);
    else
      std::snprintf(msg, sizeof msg,
                    "amrto_pcg: true relative residual %.3e stagnated above rtol (FP64 attainable accuracy)", rel);
    ctx->err = msg;
  }
  return status;
}

int amrto_pcg_pass_times(amrto_ctx* ctx, const double* b, double* u, const amrto_solve_opts* opts_in, int32_t reps,
                         double* op_us, double* update_us) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, "amrto_pcg_pass_times: density not set");
  if (!b || !u || b == u || !op_us || !update_us || reps < 1 || reps > 100000)
    return ctx->fail(AMRTO_EINVAL, "amrto_pcg_pass_times: bad arguments");
  amrto_solve_opts o;
  amrto_solve_opts_default(&o);
  if (opts_in) o = *opts_in;
  if (o.inner_prec != AMRTO_FP64 && o.inner_prec != AMRTO_FP32 && o.inner_prec != AMRTO_BF16)
    return ctx->fail(AMRTO_EINVAL, "amrto_pcg_pass_times: unknown inner precision");
  if (o.precond != AMRTO_PRECOND_JACOBI && o.precond != AMRTO_PRECOND_BLOCK3)
    return ctx->fail(AMRTO_EINVAL, "amrto_pcg_pass_times: unknown preconditioner");
  const bool block3 = o.precond == AMRTO_PRECOND_BLOCK3;
  if (block3 && o.use_coarse && ctx->coarse_k > 0 && !coarse_fused(ctx))
    return ctx->fail(AMRTO_EINVAL, "amrto_pcg_pass_times: block-Jacobi with this coarse space is not a solver variant");
  AMRTO_HIP(hipSetDevice(ctx->device));
  struct CoarseOff {
    amrto_ctx* c; int k;
    ~CoarseOff() { c->coarse_k = k; }
  } coarse_guard{ctx, ctx->coarse_k};
  if (!o.use_coarse) ctx->coarse_k = 0;
  float op = 0.f, up = 0.f;
  const int rc = o.inner_prec == AMRTO_FP64 ? pass_times<double>(ctx, b, u, AMRTO_FP64, block3, reps, &op, &up)
                                            : pass_times<float>(ctx, b, u, o.inner_prec, block3, reps, &op, &up);
  if (rc) return rc;
  *op_us = 1e3 * (double)op / reps;
  *update_us = 1e3 * (double)up / reps;
  return AMRTO_OK;
}

}  // extern "C"
