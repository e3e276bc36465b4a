// Matrix-free application of the constrained stiffness operator
//   y = A~ x,  A~ = F T^T K T F + (I - F),   K = sum_e c_e G_e^T K0 G_e
// (paper Sec. 6, Eq. (6)-(8); supported DOFs as identity rows) and the exact
// diagonal of A~ used by the Jacobi preconditioner (the diagonal rescaling
// of Sec. 5).
//
// Two data paths, both writing every output row exactly once (deterministic,
// no atomics in global memory):
//  * uniform brick: implicit connectivity, workgroups march upwards through
//    a range of node layers of a block of node columns.  FP64 and FP32: one
//    thread per node column, output rows summed in registers (z), across
//    lanes (x) and through LDS (y), no atomics (k_apply_brick).  BF16: rows
//    of 16 elements per MFMA tile, element outputs through LDS to the thread
//    owning each node column, summed in fixed order, no atomics
//    (k_apply_uniform_bf16).
//  * octree: node-owner chunks (chunks.hip).  A chunk stages its node table
//    (vertices plus masters of hanging vertices) in LDS, interpolates hanging
//    values x_h = P x_m, runs its run of elements plus the halo elements around
//    its owned nodes, condenses y_m += P^T y_h and writes its owned rows.
//
// Precisions: FP64 and FP32 contract on the vector ALUs through the mirror-
// symmetry block form of K0 (kernels.h); BF16 contracts on the matrix cores
// (dense K0, FP32 accumulation).  FUSED kernels are one conjugate-gradient
// step: they form p = z + beta p_old while staging the vector, write p and
// q = A~ p, and emit partial sums of p.q.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"

namespace amrto {

constexpr int P_F64 = 0, P_F32 = 1, P_BF16 = 2;
constexpr int LSLOTS = (UN * UN * 3 + 255) / 256;  // load slots per thread

struct UArgs {
  const void* x;     // plain: x;   fused: z
  const void* pold;  // fused: previous search direction
  void* y;           // plain: y;   fused: q
  void* pnew;        // fused: new search direction
  const void* coef;
  const uint8_t* fix;
  const void* kb;    // BF16: K0 hi/lo bits
  int nx, ny, nz, tiles_x, tiles_y, zchunk, n_tiles;
  const double* stop;
  // fused octree pass with the affine coarse space: x holds r and the staged
  // direction is p = (M r + Z cz) + beta p_old; dinv holds M (the Jacobi
  // diagonal, or the inverse 3x3 node blocks)
  const void* dinv = nullptr;
  const float4* geo = nullptr;
  const double* cz = nullptr;
  int coarse_R = 0;
  // recurrence form: the pass writes, per block, Z^T q over its owned nodes
  // and E^-1 Z^T q (column j at zq_part[j nblocks + block], E^-1 Z^T q after
  // the first k columns), and r.z takes ct^T cz from ct and cz; NULL: r.z
  // takes its coarse part from the scalar slot, no partials
  double* zq_part = nullptr;
  const double* einv = nullptr;
  const double* ct = nullptr;
  // multigrid smoothing epilogue (octree, FP64, plain pass): with q = A~ d at
  // the owned nodes (x holds d), mode 1 updates x += d, r -= q and writes the
  // next Chebyshev direction to y; mode 2 updates x and r only; mode 3 sets
  // r -= q and y = D^-1 r / theta.  cheb_scal holds the level's interval
  // (MS_* slots); dinv the diagonal inverse
  int cheb_mode = 0;
  int cheb_step = 0;
  const double* cheb_scal = nullptr;
  double* cheb_x = nullptr;
  double* cheb_r = nullptr;
  // with node blocks: the inverse 3 x 3 node blocks (six entries per node)
  // take the place of D^-1 in the smoothing update
  const double* cheb_binv = nullptr;
};

// ------------------------------------------------------------------ uniform brick, BF16 on the matrix cores
// Node-owner form, no atomics.  A workgroup covers UE x UE element columns
// around UT x UT owned node columns and marches upwards through a range of
// node layers.  Per element layer each wave contracts four rows of 16
// elements, one v_mfma_f32_16x16x32_bf16 tile per row (lane n + 16 q holds
// nodes 2q and 2q + 1 of element n, shifted by the element's node-0 values
// before the hi + lo split), and writes the element outputs K0 u_e to LDS.
// After a barrier the thread owning a node column adds, in fixed order, the
// bottom-face rows of the four elements of this layer around its node, each
// scaled by its c_e, and the top-face rows of the layer below (carried in
// registers).  Node layers rotate through three LDS buffers and are fetched
// two layers ahead; no load waited on inside a step is issued after that
// step's prefetch (waits count loads in issue order, so such a wait would
// also wait for the prefetch).
template <bool FUSED>
__global__ __launch_bounds__(256, FUSED ? 3 : 4) void k_apply_uniform_bf16(UArgs a, CgArgs cg) {
  using VT = float;
  constexpr int NL = UN * UN * 3;  // values of one staged node layer
  // element outputs, row-major: output DOF d of element e at d * YR + e; a
  // stride of 4 mod 16 puts the 64 lanes of a row write (16 elements x 4 lane
  // groups, rows 4q + r) on 64 distinct banks
  constexpr int YR = UE * UE + 4;
  __shared__ VT xs[3][NL];
  __shared__ VT cs[3][UE * UE];  // element coefficients of the staged layers
  __shared__ VT yel[24 * YR];
  __shared__ double sh[16];
  double beta = 0.0;
  if (FUSED) {
    if (!cg_prologue(cg, beta, sh)) return;
  } else if (a.stop && *a.stop != 0.0) {
    return;
  }
  const int tid = threadIdx.x;
  const int ntp = (a.n_tiles + 7) & ~7;
  const int tile = (int)blockIdx.x < ntp ? xcd_remap(blockIdx.x, ntp) : a.n_tiles;
  if (tile >= a.n_tiles) {
    if (FUSED && tid == 0) cg.part_out[cg.part_base + blockIdx.x] = 0.0;
    return;
  }
  const VT* __restrict__ X = (const VT*)a.x;
  const VT* __restrict__ PO = (const VT*)a.pold;
  VT* __restrict__ Y = (VT*)a.y;
  VT* __restrict__ PN = (VT*)a.pnew;
  const VT* __restrict__ coef = (const VT*)a.coef;
  const uint8_t* __restrict__ fix = a.fix;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int tx = tile % a.tiles_x;
  const int ty = (tile / a.tiles_x) % a.tiles_y;
  const int tz = tile / (a.tiles_x * a.tiles_y);
  const int ox = tx * UT, oy = ty * UT;
  const int z0 = tz * a.zchunk;
  const int z1 = min(z0 + a.zchunk, nz + 1);
  const int sx = nx + 1;
  const long sxy = (long)(nx + 1) * (ny + 1);
  const VT vbeta = (VT)beta;
  const bool first = FUSED && cg.it == 0;

  // load slot s of this thread: value tid + 256 s of a staged (UN x UN x 3)
  // layer; addresses of slots outside the mesh are clamped to 0 and their
  // values dropped when staged
  int gnode[LSLOTS];
  uint32_t inside = 0;
#pragma unroll
  for (int s = 0; s < LSLOTS; ++s) {
    const int idx = tid + 256 * s;
    const int nd = idx / 3;
    const int li = nd % UN, lj = nd / UN;
    const int gx = ox - 1 + li, gy = oy - 1 + lj;
    const bool in = idx < NL && gx >= 0 && gx <= nx && gy >= 0 && gy <= ny;
    inside |= (uint32_t)in << s;
    gnode[s] = in ? gx + sx * gy : 0;
  }
  // the node column this thread owns (threads 0 .. UT^2 - 1)
  const int oli = 1 + tid % UT, olj = 1 + tid / UT;
  const int ogx = ox - 1 + oli, ogy = oy - 1 + olj;
  const bool own = tid < UT * UT && ogx <= nx && ogy <= ny;
  const int onode = own ? ogx + sx * ogy : 0;
  // this lane's element in tile r: local (n, 4 wave + r); its DOF group q
  const int lane = tid & 63, wave = tid >> 6;
  const int n = lane & 15, q = lane >> 4;

  // this thread's element column for the coefficient loads: local (tid % UE, tid / UE)
  const int cex = ox - 1 + (tid % UE), cey = oy - 1 + tid / UE;
  const bool cev = cex >= 0 && cex < nx && cey >= 0 && cey < ny;
  const int cid = cev ? cex + nx * cey : 0;
  const long nxy = (long)nx * ny;

  struct Slot {
    VT x[LSLOTS];
    VT po[FUSED ? LSLOTS : 1];
    uint8_t f[LSLOTS];
    uint8_t fo;  // support bits of the owned node
    VT ce;       // coefficient of this thread's element column
  };
  // per-lane offsets within a layer are 32-bit (3 n_nodes < 2^31 is checked
  // at upload), per-layer offsets uniform
  int xoff[LSLOTS];
#pragma unroll
  for (int s = 0; s < LSLOTS; ++s) xoff[s] = 3 * gnode[s] + (tid + 256 * s) % 3;
  auto load = [&](Slot& R, int k) {
    const long kk = min(k, nz);
    const VT* __restrict__ Xl = X + 3 * sxy * kk;
    const VT* __restrict__ Pl = PO + 3 * sxy * kk;
    const uint8_t* __restrict__ Fl = fix + sxy * kk;
#pragma unroll
    for (int s = 0; s < LSLOTS; ++s) {
      R.f[s] = Fl[gnode[s]];
      R.x[s] = Xl[xoff[s]];
      if (FUSED) R.po[s] = Pl[xoff[s]];
    }
    R.fo = Fl[onode];
    R.ce = (coef + nxy * min(k, nz - 1))[cid];
  };
  // stage layer k into ring slot k % 3: masked values (fused: p = z + beta
  // p_old, masked), the owned node's support bits and the coefficients of
  // element layer k (zero outside the mesh)
  uint32_t fring = 0;  // owned node support bits, 3 per ring slot
  auto stage = [&](const Slot& R, int k) {
    const bool lay = k <= nz;
#pragma unroll
    for (int s = 0; s < LSLOTS; ++s) {
      const int idx = tid + 256 * s;
      if (idx < NL) {
        const bool in = ((inside >> s) & 1) && lay;
        VT v = in ? R.x[s] : (VT)0;
        if (FUSED && !first) v += vbeta * (in ? R.po[s] : (VT)0);
        const bool fx = in && ((R.f[s] >> (idx % 3)) & 1);
        xs[k % 3][idx] = fx ? (VT)0 : v;
      }
    }
    const uint32_t ff = (own && lay) ? (uint32_t)(R.fo & 7) : 0u;
    fring = (fring & ~(7u << (3 * (k % 3)))) | (ff << (3 * (k % 3)));
    cs[k % 3][tid] = (cev && k < nz) ? R.ce : (VT)0;
  };

  const int kbeg = max(z0 - 1, 0);
  const int kend = min(z1 - 1, nz - 1);
  // A operand: K0 hi / lo rows 16 t + (lane & 15); slot i of lane group q is
  // column 6 q + i (slots 6, 7 and rows 24..31 zero)
  bf16x8 ka[2][2];
  {
    const uint16_t* __restrict__ kb = (const uint16_t*)a.kb;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        const int m = n + 16 * t;
        bf16x8 w;
#pragma unroll
        for (int i = 0; i < 8; ++i)
          w[i] = bits_to_bf16((m < 24 && i < 6) ? kb[part * 576 + m * 24 + 6 * q + i] : (uint16_t)0);
        ka[t][part] = w;
      }
  }
  Slot S0, S1;
  load(S0, kbeg);
  stage(S0, kbeg);
  load(S0, kbeg + 1);
  stage(S0, kbeg + 1);
  load(S0, kbeg + 2);
  __syncthreads();

  VT carry[3] = {0, 0, 0};
  double dot = 0.0;
  // B operand: lane n + 16 q holds element n's nodes 2q and 2q + 1 (slots
  // 0..5: six consecutive values of one staged layer, component = slot mod 3;
  // slots 6, 7: zero, against zero K0 columns).  Nodes 0..3 lie on the bottom
  // face (layer k), 4..7 on the top face (layer k + 1); the lane's base offset
  // includes this wave's first element row, and a row adds a compile-time
  // offset.
  const int wrow = 4 * wave * UN * 3;
  const int lane_off = wrow + ((q & 1) * UN + n) * 3;
  const int ref_off = wrow + n * 3;  // node 0 of the element (bottom face)
  const VT* __restrict__ xsb = &xs[0][0];
  VT* __restrict__ yeb = yel + 4 * q * YR + 4 * wave * UE + n;
  // element layer k: contract, finish node layer k, stage layer k + 2
  auto step = [&](int k, Slot& Rst, Slot& Rld) {
    // plain apply: x of the owned node (rows of fixed DOFs copy it), requested
    // before the prefetch; the prefetch itself is unconditional (layers past
    // the top are clamped and never staged)
    VT xo[3];
    if (!FUSED) {
      const VT* Xk = X + 3 * (sxy * k + onode);
#pragma unroll
      for (int c = 0; c < 3; ++c) xo[c] = Xk[c];
    }
    load(Rld, k + 3);
    const int bsl = (k % 3) * NL;
    const VT* __restrict__ xl = xsb + (q >= 2 ? ((k + 1) % 3) * NL : bsl) + lane_off;
    const VT* __restrict__ xr = xsb + bsl + ref_off;
    // one element row: operands (K0 annihilates a translation, so any
    // per-component shift of the element's values leaves its product
    // unchanged; taking off node 0's values makes the split relative to the
    // variation within the element), products, and the scaled output rows
    // hi = t with the low 16 bits cleared (truncation: t - hi is exact in
    // FP32 and below 2^-7 |t|), lo = t - hi rounded to BF16; two hi parts
    // pack into one register from their high halves
    auto prep = [&](int r, bf16x8& bh, bf16x8& bl) {
      const int ro = r * UN * 3;
      float sft[3], v[6];
#pragma unroll
      for (int j = 0; j < 3; ++j) sft[j] = xr[ro + j];
#pragma unroll
      for (int i = 0; i < 6; ++i) v[i] = xl[ro + i];
      uint32_t tb[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const float t = v[i] - sft[i % 3];
        tb[i] = __float_as_uint(t);
        bl[i] = (__bf16)(t - __uint_as_float(tb[i] & 0xffff0000u));
      }
      bl[6] = bl[7] = (__bf16)0.f;
      uint32_t hp[4];
#pragma unroll
      for (int i = 0; i < 3; ++i) hp[i] = (tb[2 * i] >> 16) | (tb[2 * i + 1] & 0xffff0000u);
      hp[3] = 0u;
      bh = __builtin_bit_cast(bf16x8, hp);
    };
    auto mm = [&](const bf16x8& bh, const bf16x8& bl, f32x4& d0, f32x4& d1) {
      const f32x4 z = {0.f, 0.f, 0.f, 0.f};
      d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[0][0], bh, z, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[1][0], bh, z, 0, 0, 0);
      d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[0][1], bh, d0, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[1][1], bh, d1, 0, 0, 0);
      d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[0][0], bl, d0, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[1][0], bl, d1, 0, 0, 0);
    };
    // unscaled K0 u_e rows (c_e is applied by the node owner)
    auto put = [&](int r, const f32x4& d0, const f32x4& d1) {
      VT* ye = yeb + r * UE;
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) ye[r4 * YR] = d0[r4];
      if (q < 2) {  // rows 24..31 of the second tile are padding
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) ye[(16 + r4) * YR] = d1[r4];
      }
    };
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bf16x8 bh, bl;
      f32x4 d0, d1;
      prep(r, bh, bl);
      mm(bh, bl, d0, d1);
      put(r, d0, d1);
    }
    __syncthreads();
    // node layer k: carried top rows of element layer k - 1 plus the bottom
    // rows of element layer k, four elements in fixed order
    if (own) {
      VT yb[3] = {0, 0, 0}, yt[3] = {0, 0, 0};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ii = oli - 1 + (e & 1), jj = olj - 1 + (e >> 1);
        const int av = (oli - ii) + 2 * (olj - jj);
        const VT* ye = yel + jj * UE + ii;
        const VT ce = cs[k % 3][jj * UE + ii];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          yb[c] = fmaf(ce, ye[(3 * av + c) * YR], yb[c]);
          yt[c] = fmaf(ce, ye[(3 * (av + 4) + c) * YR], yt[c]);
        }
      }
      if (k >= z0) {
        const long g = 3 * (sxy * k + onode);
        const uint32_t fx = (fring >> (3 * (k % 3))) & 7u;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const VT acc = carry[c] + yb[c];
          const bool fc = (fx >> c) & 1;
          if (FUSED) {
            const VT pn = xs[k % 3][(olj * UN + oli) * 3 + c];
            const VT qv = fc ? (VT)0 : acc;
            PN[g + c] = pn;
            Y[g + c] = qv;
            dot += (double)pn * (double)qv;
          } else {
            Y[g + c] = fc ? xo[c] : acc;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) carry[c] = yt[c];
    }
    if (k + 2 <= nz) stage(Rst, k + 2);
    __syncthreads();
  };
  // S0 holds layer kbeg + 2 (staged at step kbeg); steps alternate the two slots
  for (int k = kbeg; k <= kend; k += 2) {
    step(k, S0, S1);
    if (k + 1 <= kend) step(k + 1, S1, S0);
  }
  // the top node layer of the mesh: only the elements below contribute
  if (own && kend + 1 < z1) {
    const int k = kend + 1;
    const long g = 3 * (sxy * k + onode);
    const uint32_t fx = (fring >> (3 * (k % 3))) & 7u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool fc = (fx >> c) & 1;
      if (FUSED) {
        const VT pn = xs[k % 3][(olj * UN + oli) * 3 + c];
        const VT qv = fc ? (VT)0 : carry[c];
        PN[g + c] = pn;
        Y[g + c] = qv;
        dot += (double)pn * (double)qv;
      } else {
        Y[g + c] = fc ? X[g + c] : carry[c];
      }
    }
  }
  if (FUSED) {
    dot = block_sum(dot, sh);
    if (tid == 0) cg.part_out[cg.part_base + blockIdx.x] = dot;
  }
}

// ------------------------------------------------------------------ uniform brick, node-owner form
// FP64 and FP32.  One thread per node column of a 16 x 16 tile; the thread's
// element column is the one whose lower corner is its node.  Marching up one
// element layer per step, every output row is summed without atomics:
//  * z: an element's top-face outputs stay in the thread's registers and are
//    added to the next element's bottom-face outputs (same node layer);
//  * x: the contributions to the right-hand node move one lane up with DPP
//    (rows of 16 lanes are rows of the tile);
//  * y: the contributions to the node column above go through LDS.
// The element contraction works in the Walsh-Hadamard mode basis and reuses
// transforms along z: the forward transform of a node layer factors into an
// x-y part (computed once per layer, carried to the next element) and a z
// butterfly; the inverse is linear, so the top-face outputs of element k-1
// are carried in mode form and added before one x-y inverse per layer.  The
// block matrix is applied through its eight distinct entries (cube symmetry:
// 33 multiply-adds instead of 72, the element coefficient folded into the
// eight constants).  One barrier per layer.
#ifndef AMRTO_BRICK_OCC64
#define AMRTO_BRICK_OCC64 2
#endif
// workgroups per CU the brick kernel is compiled for
template <typename VT>
struct BrickOcc { static constexpr int blocks = 4 * 256 / BTHREADS; };
template <>
struct BrickOcc<double> { static constexpr int blocks = AMRTO_BRICK_OCC64 * 256 / BTHREADS; };

template <typename VT, bool FUSED>
__global__ __launch_bounds__(BTHREADS, BrickOcc<VT>::blocks) void k_apply_brick(UArgs a, BrickK<VT> kc, CgArgs cg) {
  __shared__ VT xs[4][3][BTHREADS];  // staged node layers L & 3 (masked; fused: p)
  __shared__ VT sb[2][3][BTHREADS];  // partial sums for the node column above
  __shared__ double sh[16];
  double beta = 0.0;
  if (FUSED) {
    if (!cg_prologue(cg, beta, sh)) return;
  } else if (a.stop && *a.stop != 0.0) {
    return;
  }
  const int tid = threadIdx.x;
  // the grid may exceed the tile count (it is shared with the BF16 kernel):
  // spread the tiles over all eight XCDs, surplus workgroups at the end
  const int ntp = (a.n_tiles + 7) & ~7;
  const int tile = (int)blockIdx.x < ntp ? xcd_remap(blockIdx.x, ntp) : a.n_tiles;
  if (tile >= a.n_tiles) {
    if (FUSED && tid == 0) cg.part_out[cg.part_base + blockIdx.x] = 0.0;
    return;
  }
  const VT* __restrict__ X = (const VT*)a.x;
  const VT* __restrict__ PO = (const VT*)a.pold;
  VT* __restrict__ Y = (VT*)a.y;
  VT* __restrict__ PN = (VT*)a.pnew;
  const VT* __restrict__ coef = (const VT*)a.coef;
  const uint8_t* __restrict__ fix = a.fix;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  // z-chunks vary fastest: the chunks of one column of tiles share an XCD
  constexpr int BZ = BrickZ<VT>::layers;
  const int nzc = (nz + 1 + BZ - 1) / BZ;
  const int tz = tile % nzc;
  const int txy = tile / nzc;
  const int tx = txy % a.tiles_x, ty = txy / a.tiles_x;
  const int i = tid & (BT - 1), j = tid >> 4;
  const int gx = tx * BO - 1 + i, gy = ty * BOY - 1 + j;
  const bool nv = gx >= 0 && gx <= nx && gy >= 0 && gy <= ny;
  const bool ev = i < BT - 1 && j < BTY - 1 && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
  const bool owned = nv && i >= 1 && i <= BO && j >= 1 && j <= BOY;
  // per-lane offsets within a layer (32-bit: 3 n_nodes < 2^31 is checked at
  // upload); per-layer offsets are uniform
  const int nid = nv ? gx + (nx + 1) * gy : 0;
  const int eid = ev ? gx + nx * gy : 0;
  const long sxy = (long)(nx + 1) * (ny + 1);
  const long nxy = (long)nx * ny;
  const int z0 = tz * BZ;
  const int z1 = min(z0 + BZ, nz + 1);
  const VT vbeta = (VT)beta;
  const bool first = FUSED && cg.it == 0;
  const int up = min(tid + BT, BTHREADS - 1);  // node column above (top row: unused)
  const int dn = max(tid - BT, 0);            // node column below (row 0: unused)

  // raw loads of node layer L and the coefficient of element layer L.  The
  // loads are unconditional (addresses clamped into the arrays) and the
  // validity is applied when the layer is staged, so a load in flight is
  // never merged with a default value (which would force a wait).
  struct Slot {
    VT x[3];
    VT po[FUSED ? 3 : 1];
    VT ce;
    uint32_t f;
  };
  auto load = [&](Slot& R, int L) {
    const long Lc = min(L, nz);
    const VT* xl = X + 3 * sxy * Lc;
    R.f = fix[sxy * Lc + nid];
#pragma unroll
    for (int c = 0; c < 3; ++c) R.x[c] = xl[3 * nid + c];
    if (FUSED) {
      const VT* pl = PO + 3 * sxy * Lc;
#pragma unroll
      for (int c = 0; c < 3; ++c) R.po[c] = pl[3 * nid + c];
    }
    R.ce = coef[nxy * min(L, nz - 1) + eid];
  };
  // a staged layer in registers: masked values (fused: p), support bits and
  // the coefficient of the element above it
  struct Lay {
    VT v[3];
    VT ce;
    uint32_t f;
  };
  // Stage layer L: masked values (fused: p = z + beta p_old) into LDS.  Rows
  // known at this point are written now: the search direction p (fused) and
  // the identity rows of supported DOFs (plain apply).
  auto stage = [&](const Slot& R, int L, Lay& out) {
    const bool in = nv && L <= nz;
    out.f = in ? R.f : 0u;
    out.ce = (ev && L < nz) ? R.ce : (VT)0;
    const bool mine = owned && L >= z0 && L < z1;
    const long g = 3 * sxy * L + 3 * nid;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool fx = (out.f >> c) & 1;
      VT v = in ? R.x[c] : (VT)0;
      if (!FUSED && mine && fx) Y[g + c] = v;
      if (FUSED && !first) v += vbeta * (in ? R.po[c] : (VT)0);
      v = fx ? (VT)0 : v;
      if (FUSED && mine) PN[g + c] = v;
      out.v[c] = v;
      xs[L & 3][c][tid] = v;
    }
  };
  // x-y modes of a staged layer: own column, right (DPP), above (LDS), above-right
  auto face_modes = [&](const Lay& l, int L, VT (&m)[3][4]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const VT v00 = l.v[c];
      const VT v01 = xs[L & 3][c][up];
      m[c][0] = v00;
      m[c][1] = dpp_mov<DPP_ROW_SHL1>(v00);
      m[c][2] = v01;
      m[c][3] = dpp_mov<DPP_ROW_SHL1>(v01);
      wht4(m[c]);
    }
  };

  const int kbeg = max(z0 - 1, 0);
  const int kend = z1 - 1;
  // layer L is loaded into register set (L - kbeg) % NSL, BPD steps before
  // it is staged (into staged set (L - kbeg) % 3).  The march is unrolled
  // completely (at most BZ + 1 steps), so no value in flight crosses a loop
  // back-edge (where register copies would wait for it).
  constexpr int NSL = BPD + 1;
  Slot S[NSL];
  Lay Ls[3];
  VT fb[3][4], carry[3][4];
  load(S[0], kbeg);
  load(S[1 % NSL], kbeg + 1);
  stage(S[0], kbeg, Ls[0]);
  stage(S[1 % NSL], kbeg + 1, Ls[1]);
#pragma unroll
  for (int q = 2; q < 2 + BPD; ++q) load(S[q % NSL], kbeg + q);
  __syncthreads();
  face_modes(Ls[0], kbeg, fb);
  VT fn[3][4];  // x-y modes of the next layer to contract (k + 1)
  face_modes(Ls[1], kbeg + 1, fn);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int t = 0; t < 4; ++t) carry[c][t] = 0;
  double dot = 0.0;

  // element layer k: contract with the staged layers k (modes fb) and k + 1
  // (modes fn), stage layer k + 2 from Rst into ln, request layer k + 2 + BPD
  // into Rld, finish node layer k and take the modes of layer k + 2
  auto step = [&](int k, Slot& Rld, Slot& Rst, const Lay& lp, Lay& ln) {
    VT w[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        w[c][t] = fb[c][t] + fn[c][t];
        w[c][t + 4] = fb[c][t] - fn[c][t];
        fb[c][t] = fn[c][t];
      }
    VT ks[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ks[q] = lp.ce * kc.c[q];
    VT o[3][8];
    brick_blocks<VT>(ks, w, o);
    VT c00[3], c10[3], c01[3], c11[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      VT m[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        m[t] = o[c][t] + o[c][t + 4] + carry[c][t];
        carry[c][t] = o[c][t] - o[c][t + 4];
      }
      wht4(m);
      c00[c] = m[0];
      c10[c] = m[1];
      c01[c] = m[2];
      c11[c] = m[3];
    }
    VT s0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s0[c] = c00[c] + dpp_mov<DPP_ROW_SHR1>(c10[c]);
      sb[k & 1][c][tid] = c01[c] + dpp_mov<DPP_ROW_SHR1>(c11[c]);
    }
    // layers above the mesh are staged too (as zeros): their modes meet a zero
    // coefficient in the top element layer, and zero times stale LDS or
    // register contents is not zero when those bits are Inf or NaN
    stage(Rst, k + 2, ln);
    load(Rld, k + 2 + BPD);
    __syncthreads();
    // the next layer's modes first: its LDS reads overlap the partial sums'
    if (k < kend) face_modes(ln, k + 2, fn);
    if (owned && k >= z0) {
      VT* yl = Y + 3 * sxy * k;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const VT tot = s0[c] + (j >= 1 ? sb[k & 1][c][dn] : (VT)0);
        const bool fx = (lp.f >> c) & 1;
        if (FUSED) {
          const VT q = fx ? (VT)0 : tot;
          yl[3 * nid + c] = q;
          dot += (double)lp.v[c] * (double)q;
        } else if (!fx) {
          yl[3 * nid + c] = tot;
        }
      }
    }
  };
#pragma unroll
  for (int st = 0; st <= BZ; ++st) {
    const int k = kbeg + st;
    if (k > kend) break;
    step(k, S[(st + 2 + BPD) % NSL], S[(st + 2) % NSL], Ls[st % 3], Ls[(st + 2) % 3]);
  }
  if (FUSED) {
    dot = block_sum(dot, sh);
    if (tid == 0) cg.part_out[cg.part_base + blockIdx.x] = dot;
  }
}

// ------------------------------------------------------------------ octree chunks

// COARSE: 0 plain; 1 stage p from z = D^-1 r + Z cz; 2 the same with the
// inverse 3x3 node blocks (six entries per node in a.dinv) in place of D^-1
// Threads per workgroup of the octree operator pass.  The LDS of a chunk
// allows two workgroups per CU; with 512 threads that is four waves per SIMD
// (twice the latency hiding of 256, and half the per-thread staging, element
// and store work), which needs at most 128 VGPRs: the BF16 coarse-space
// variants need more and keep 256.
constexpr int chunk_threads(int prec, int coarse) { return (coarse && prec == P_BF16) ? 256 : 512; }

// DET: deterministic mode (a template parameter, so that the default kernels
// keep their register budget); see wave_turns
template <typename VT, int PREC, bool FUSED, int COARSE = 0, bool DET = false>
__global__ __launch_bounds__(chunk_threads(PREC, COARSE)) void k_apply_chunks(UArgs a, ChunkArgs ca, BrickK<VT> kc, CgArgs cg) {
  __shared__ VT xs[TAB_MAX * 3];
  __shared__ double ys[TAB_MAX * 3];  // FP64 LDS accumulators (ds_add_f64 runs at full rate on gfx950)
  __shared__ uint16_t lsm[PREC == P_BF16 ? ENT_MAX * 8 : 1];
  __shared__ double sh[16];
  __shared__ uint32_t trip_hm_s[TRIP_MAX];
  __shared__ double trip_w_s[TRIP_MAX];
  __shared__ int hbeg_s[TAB_MAX];
  constexpr int NT = chunk_threads(PREC, COARSE);
  static_assert(NT == 256 || NT == 512, "chunk workgroups have 256 or 512 threads");
  const int tid = threadIdx.x;
  const int c = xcd_remap(blockIdx.x, gridDim.x);
  if (!FUSED && a.stop && *a.stop != 0.0) return;
  const bool have = c < ca.n_chunks;
  const int cc = have ? c : 0;
  const VT* __restrict__ X = (const VT*)a.x;
  const VT* __restrict__ PO = (const VT*)a.pold;
  VT* __restrict__ Y = (VT*)a.y;
  VT* __restrict__ PN = (VT*)a.pnew;
  const VT* __restrict__ coef = (const VT*)a.coef;
  const uint8_t* __restrict__ fix = a.fix;
  // surplus workgroups (the grid is rounded up to a multiple of 8) own nothing
  const ChunkDims cd = chunk_dims(ca, cc, have);
  const int n0 = cd.n0, nent = cd.nent, t0 = cd.t0, nt = cd.nt, h0 = cd.h0, nh = cd.nh;
  const int nown = cd.nown, nreg = cd.nreg, nhown = cd.nhown;
  // Every index this block needs is requested before the CG prologue (which
  // waits on the previous pass's partial sums), so those round trips overlap.
  // The node-table slot is read whole (the chunk's slots sit at fixed strides,
  // zero padded), so it goes out with the count loads rather than after them:
  // the staged vector values depend on it.  Entries and hanging triples are
  // needed later and are read only up to their counts.  Table nodes
  // t = tid + NT r (r < NPT): global node, support bits and the staged values
  // are loaded in one batch (no dependent round trips per component), and the
  // indices stay in registers for the store phase.
  constexpr int NPT = TAB_MAX / NT;
  int gn[NPT];
  uint8_t fb[NPT];
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int t = tid + NT * r;
    const int g = ca.tab_node[t0 + t];
    gn[r] = t < nt ? g : -1;
  }
  // entry metadata of the element loop, prefetched under the staging latency
  constexpr int EPT = ENT_MAX / NT;
  uint4 lvp[EPT];
  int eel[EPT];
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const int en = tid + NT * r;
    eel[r] = 0;
    lvp[r] = make_uint4(0u, 0u, 0u, 0u);
    if (en < nent) {
      eel[r] = ca.ent_elem[n0 + en];
      lvp[r] = *reinterpret_cast<const uint4*>(ca.ent_loc + 8L * (n0 + en));
    }
  }
  // hanging triples and per-entry triple ranges, whole slots; written to LDS
  // once the vector values below are requested
  constexpr int HPT = TRIP_MAX / NT;
  uint32_t thm[HPT];
  double tw[HPT];
  int hbr[NPT];
#pragma unroll
  for (int q = 0; q < HPT; ++q) {
    thm[q] = 0u;
    tw[q] = 0.0;
    if (tid + NT * q < nh) {
      thm[q] = ca.trip_hm[h0 + tid + NT * q];
      tw[q] = ca.trip_w[h0 + tid + NT * q];
    }
  }
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int t = tid + NT * r;
    hbr[r] = (t >= nreg && t < nt) ? ca.tab_hbeg[t0 + t] : 0;
  }
  // raw vector values of the regular table nodes, also requested before the
  // prologue; beta is applied once the prologue has it
  const bool first = FUSED && cg.it == 0;
  constexpr int DW = COARSE == 2 ? 6 : 3;
  VT xv[NPT][3], pv[FUSED ? NPT : 1][3], dv[COARSE ? NPT : 1][DW];
  float4 gv[COARSE ? NPT : 1];
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int t = tid + NT * r;
    fb[r] = 0;
#pragma unroll
    for (int c3 = 0; c3 < 3; ++c3) {
      xv[r][c3] = 0;
      if (FUSED) pv[r][c3] = 0;
    }
#pragma unroll
    for (int k = 0; k < DW; ++k)
      if (COARSE) dv[r][k] = 0;
    if (COARSE) gv[r] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t < nreg && gn[r] >= 0) {
      const long g = 3L * gn[r];
      fb[r] = fix[gn[r]];
#pragma unroll
      for (int c3 = 0; c3 < 3; ++c3) {
        xv[r][c3] = X[g + c3];
        if (FUSED && !first) pv[r][c3] = PO[g + c3];
      }
#pragma unroll
      for (int k = 0; k < DW; ++k)
        if (COARSE) dv[r][k] = ((const VT*)a.dinv)[(long)DW * gn[r] + k];
      if (COARSE) gv[r] = a.geo[gn[r]];
    }
  }
  // Chebyshev smoothing step (plain FP64 pass): the owned rows' r, D^-1 and
  // x, and the step's interval, are requested with the staged vector, so the
  // store phase does not wait on them (each owned row is read and written by
  // its own thread only)
  constexpr bool CHEB = !FUSED && PREC == P_F64;
  double cr[CHEB ? NPT : 1][3], cdi[CHEB ? NPT : 1][6], cxo[CHEB ? NPT : 1][3];
  double c_sigma = 1.0, c_delta = 1.0, c_theta = 1.0;
  if (CHEB && a.cheb_mode) {
    c_sigma = a.cheb_scal[MS_SIGMA];
    c_delta = a.cheb_scal[MS_DELTA];
    c_theta = a.cheb_scal[MS_THETA];
    const double* __restrict__ dinv = (const double*)a.dinv;
    const double* __restrict__ binv = a.cheb_binv;
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int t = tid + NT * r;
      const bool own = t < nown;
      const long v = own ? gn[r] : 0, g = 3L * v;
#pragma unroll
      for (int c3 = 0; c3 < 3; ++c3) {
        cr[r][c3] = own ? a.cheb_r[g + c3] : 0.0;
        cxo[r][c3] = own && a.cheb_mode != 3 ? a.cheb_x[g + c3] : 0.0;
      }
      const bool need = own && a.cheb_mode != 2;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        cdi[r][k] = !need ? 0.0 : (binv ? binv[6 * v + k] : (k < 3 ? dinv[g + k] : 0.0));
    }
  }
  VT cep[EPT];
#pragma unroll
  for (int r = 0; r < EPT; ++r) cep[r] = coef[eel[r]];
#pragma unroll
  for (int q = 0; q < HPT; ++q) {
    trip_hm_s[tid + NT * q] = thm[q];
    trip_w_s[tid + NT * q] = tw[q];
  }
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int t = tid + NT * r;
    if (t >= nreg && t < nt) hbeg_s[t - nreg] = hbr[r];
  }
  __shared__ double czs[COARSE ? COARSE_KMAX : 1];
  CgArgs cgb = cg;
  if (COARSE) {
    for (int j = tid; j < 12 * a.coarse_R; j += NT) czs[j] = a.cz[j];
    if (a.zq_part) {  // recurrence form: r.z adds ct^T cz in the prologue
      cgb.cct = a.ct;
      cgb.ccz = a.cz;
      cgb.ck = 12 * a.coarse_R;
    }
  }
  double beta = 0.0;
  if (FUSED) {
    if (!cg_prologue(cgb, beta, sh)) return;
  }
  if (!have) {
    if (FUSED && tid == 0) cg.part_out[cg.part_base + blockIdx.x] = 0.0;
    if (COARSE && a.zq_part)
      for (int j = tid; j < 24 * a.coarse_R; j += NT) a.zq_part[(long)j * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const VT vbeta = (VT)beta;
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int t = tid + NT * r;
    if (t < nreg) {
      VT zb[3];
      if (COARSE == 2) block_apply<VT>(dv[r], xv[r], zb);
#pragma unroll
      for (int c3 = 0; c3 < 3; ++c3) {
        VT v = xv[r][c3];
        if (COARSE) {
          // z = D^-1 r + Z cz with the affine fields of this node (zero on
          // supported and hanging DOFs, where r and the fields vanish)
          const int w = __float_as_int(gv[r].w), gr = w & 0xff;
          const double on = ((w >> (8 + c3)) & 1) ? 0.0 : 1.0;
          const double d[3] = {(double)gv[r].x, (double)gv[r].y, (double)gv[r].z};
          const int R = a.coarse_R;
          const double zc = czs[gr * 3 + c3] + d[c3] * czs[(R + gr) * 3 + c3] +
                            d[c3 == 2 ? 0 : c3 + 1] * czs[(2 * R + gr) * 3 + c3] +
                            d[c3 == 0 ? 2 : c3 - 1] * czs[(3 * R + gr) * 3 + c3];
          const double zl = COARSE == 2 ? (double)zb[c3] : (double)dv[r][c3] * (double)v;
          v = (VT)(zl + on * zc);
        }
        if (FUSED && !first) v += vbeta * pv[r][c3];
        xs[3 * t + c3] = ((fb[r] >> c3) & 1) ? (VT)0 : v;
      }
    }
  }
  for (int i = tid; i < nt * 3; i += NT) ys[i] = 0.0;
  if (PREC == P_BF16)
    for (int i = tid; i < nent * 8; i += NT) lsm[i] = ca.ent_loc[8L * n0 + i];
  // recurrence form: the regions of the owned regular nodes (a bitmask), and
  // the E^-1 columns of the first two requested now, under the element loop
  __shared__ uint32_t gmask_s[NT / 64];
  uint32_t mall = 0;
  int g0 = -1, g1 = -1;
  // E^-1 columns prefetched: two regions' (FP32, BF16), one region's in FP64
  // (their 24 registers keep the FP64 pass within 128 VGPRs at 512 threads)
  constexpr int EPF = sizeof(VT) == 8 ? 12 : 24;
  double e0[COARSE ? EPF : 1];
  if (COARSE && a.zq_part) {
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < NPT; ++r)
      if (tid + NT * r < nown) m |= 1u << (__float_as_int(gv[r].w) & 31);
    m = wave_or(m);
    if ((tid & 63) == 0) gmask_s[tid >> 6] = m;
  }
  __syncthreads();
  if (COARSE && a.zq_part) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) mall |= gmask_s[w];
    const uint32_t m1 = mall & (mall - 1);
    g0 = mall ? __ffs((int)mall) - 1 : -1;
    g1 = m1 ? __ffs((int)m1) - 1 : -1;
    const int R = a.coarse_R, kk = 12 * R;
#pragma unroll
    for (int u = 0; u < EPF; ++u) {
      const int g = u < 12 ? g0 : g1, v = u % 12;
      e0[u] = (g >= 0 && tid < kk) ? a.einv[(long)(((v / 3) * R + g) * 3 + v % 3) * kk + tid] : 0.0;
    }
  }
  for (int i = tid; i < (nt - nreg) * 3; i += NT) {  // x_h = sum_m w_hm x_m  (Eq. (6))
    const int t = nreg + i / 3, comp = i % 3;
    const int kb = hbeg_s[t - nreg], ke = t + 1 < nt ? hbeg_s[t + 1 - nreg] : nh;
    double v = 0.0;
    for (int k = kb; k < ke; ++k) v += trip_w_s[k] * (double)xs[(trip_hm_s[k] & 0xffff) * 3 + comp];
    xs[t * 3 + comp] = (VT)v;
  }
  __syncthreads();
  if (PREC != P_BF16) {
    // deterministic mode: the waves take turns over whole elements (the
    // contraction stays next to its adds, so the mode costs no registers)
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
      const int en = tid + NT * r;
      const bool ev = en < nent;
      if (!ev && !DET) break;
      auto elem = [&]() {
        if (!ev) return;
        int loc[8];
        const uint4 lv = lvp[r];
        loc[0] = lv.x & 0xffff; loc[1] = lv.x >> 16; loc[2] = lv.y & 0xffff; loc[3] = lv.y >> 16;
        loc[4] = lv.z & 0xffff; loc[5] = lv.z >> 16; loc[6] = lv.w & 0xffff; loc[7] = lv.w >> 16;
        const VT ce = cep[r];
        VT u[24], out[24];
#pragma unroll
        for (int aa = 0; aa < 8; ++aa) {
          u[3 * aa + 0] = xs[loc[aa] * 3 + 0];
          u[3 * aa + 1] = xs[loc[aa] * 3 + 1];
          u[3 * aa + 2] = xs[loc[aa] * 3 + 2];
        }
        VT ks[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) ks[q] = ce * kc.c[q];
        contract_brick<VT>(ks, u, out);
#pragma unroll
        for (int aa = 0; aa < 8; ++aa) {
          atomicAdd(&ys[loc[aa] * 3 + 0], (double)out[3 * aa + 0]);
          atomicAdd(&ys[loc[aa] * 3 + 1], (double)out[3 * aa + 1]);
          atomicAdd(&ys[loc[aa] * 3 + 2], (double)out[3 * aa + 2]);
        }
      };
      if (DET) wave_turns(elem);
      else elem();
    }
  } else {
    bf16x8 ka[2][2];
    load_k0_bf16((const uint16_t*)a.kb, ka);
    const int lane = tid & 63, wave = tid >> 6;
    const int n16 = lane & 15, q4 = lane >> 4;
    // deterministic mode: every wave takes the same number of tile steps and
    // the waves take turns over them; one quarter of the lanes adds at a
    // time, so the lanes of an add instruction hold distinct elements at the
    // same vertex slot
    const int tb_end = DET ? nent + 16 * wave : nent;
    for (int tb = 16 * wave; tb < tb_end; tb += 16 * (NT / 64)) {
      auto tile = [&](bool quarters) {
        const int en = tb + n16;
        const bool ev = en < nent;
        float u[24];
#pragma unroll
        for (int aa = 0; aa < 8; ++aa) {
          const int l = ev ? lsm[en * 8 + aa] * 3 : 0;
          u[3 * aa + 0] = ev ? (float)xs[l + 0] : 0.f;
          u[3 * aa + 1] = ev ? (float)xs[l + 1] : 0.f;
          u[3 * aa + 2] = ev ? (float)xs[l + 2] : 0.f;
        }
        f32x4 d0, d1;
        mfma_tile_bf16(ka, u, q4, d0, d1);
        if (!ev) return;
        const float ce = (float)coef[ca.ent_elem[n0 + en]];
        for (int qs = 0; qs < (quarters ? 4 : 1); ++qs) {
          if (quarters && q4 != qs) continue;
#pragma unroll
          for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int R = 16 * t + 4 * q4 + r;
              if (R < 24) atomicAdd(&ys[lsm[en * 8 + R / 3] * 3 + R % 3], (double)(ce * (t ? d1[r] : d0[r])));
            }
        }
      };
      if (DET) wave_turns([&]() { tile(true); });
      else tile(false);
    }
  }
  __syncthreads();
  // y_m += w_hm y_h  (P^T of Eq. (7)); deterministic mode: wave 0 alone, in
  // triple order
  for (int i = DET ? (tid < 64 ? tid : nh * 3) : tid; i < nh * 3; i += DET ? 64 : NT) {
    const int k = i / 3, comp = i % 3;
    const uint32_t hm = trip_hm_s[k];
    atomicAdd(&ys[(hm & 0xffff) * 3 + comp], trip_w_s[k] * ys[(hm >> 16) * 3 + comp]);
  }
  __syncthreads();
  double dot = 0.0;
  VT qk[COARSE ? NPT : 1][3];  // q of the owned regular nodes (coarse recurrence)
  // Chebyshev coefficients of this step: rho_s from rho_0 = 1 / sigma
  double ch_a = 0.0, ch_c = 0.0, ch_t = 1.0;
  if (CHEB && a.cheb_mode) {
    double rho = 1.0 / c_sigma;
    for (int s = 0; s < a.cheb_step; ++s) rho = 1.0 / (2.0 * c_sigma - rho);
    const double rho1 = 1.0 / (2.0 * c_sigma - rho);
    ch_a = rho1 * rho;
    ch_c = 2.0 * rho1 / c_delta;
    ch_t = c_theta;
  }
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int t = tid + NT * r;
#pragma unroll
    for (int comp = 0; comp < 3; ++comp)
      if (COARSE) qk[r][comp] = 0;
    const bool own_reg = t < nown, own_hang = t >= nreg && t < nreg + nhown;
    if (!own_reg && !own_hang) continue;
    const long g = 3L * gn[r];
    if (own_hang) {  // identity row; in a solve the hanging entries stay zero
      for (int comp = 0; comp < 3; ++comp) {
        if (FUSED) {
          PN[g + comp] = 0;
          Y[g + comp] = 0;
        } else if (CHEB && a.cheb_mode) {
          if (a.cheb_mode != 2) Y[g + comp] = 0;
        } else {
          Y[g + comp] = X[g + comp];
        }
      }
      continue;
    }
    if (CHEB && a.cheb_mode && a.cheb_binv) {
      // node-block smoothing: the node's three residual components first,
      // then the inverse node block (constrained components have identity
      // rows in it and a zero residual, so they stay zero)
      double q3[3], rv[3], zb[3];
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        q3[comp] = ((fb[r] >> comp) & 1) ? 0.0 : ys[t * 3 + comp];
        rv[comp] = cr[r][comp] - q3[comp];
        a.cheb_r[g + comp] = rv[comp];
      }
      if (a.cheb_mode != 2) {
        double b6[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) b6[k] = cdi[r][k];
        block_apply<double>(b6, rv, zb);
      }
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const double dv = (double)xs[t * 3 + comp];
        if (a.cheb_mode == 3) {
          Y[g + comp] = (VT)(zb[comp] / ch_t);
        } else {
          a.cheb_x[g + comp] = cxo[r][comp] + dv;
          if (a.cheb_mode == 1) Y[g + comp] = (VT)(ch_a * dv + ch_c * zb[comp]);
        }
      }
      continue;
    }
    for (int comp = 0; comp < 3; ++comp) {
      const VT acc = (VT)ys[t * 3 + comp];
      const bool fixed = (fb[r] >> comp) & 1;
      if (FUSED) {
        const VT pn = xs[t * 3 + comp];
        const VT q = fixed ? (VT)0 : acc;
        PN[g + comp] = pn;
        Y[g + comp] = q;
        dot += (double)pn * (double)q;
        if (COARSE) qk[r][comp] = q;
      } else if (CHEB && a.cheb_mode) {
        // constrained-form vectors are zero at supported DOFs: q = 0 there
        const double q = fixed ? 0.0 : (double)acc, dv = (double)xs[t * 3 + comp];
        const double rv = cr[r][comp] - q;
        a.cheb_r[g + comp] = rv;
        if (a.cheb_mode == 3) {
          Y[g + comp] = (VT)(cdi[r][comp] * rv / ch_t);
        } else {
          a.cheb_x[g + comp] = cxo[r][comp] + dv;
          if (a.cheb_mode == 1) Y[g + comp] = (VT)(ch_a * dv + ch_c * cdi[r][comp] * rv);
        }
      } else {
        Y[g + comp] = fixed ? X[g + comp] : acc;
      }
    }
  }
  if (FUSED) {
    dot = block_sum(dot, sh);
    if (tid == 0) cg.part_out[cg.part_base + blockIdx.x] = dot;
  }
  if (COARSE && a.zq_part) {
    // Z^T q over the owned regular nodes.  The first region present (a
    // bitmask; the only one in most chunks) is summed in fixed order: sums
    // per thread in node order, then through LDS (ys is free here) 16 partial
    // sums per column and one final sum per column.  Entries of the other
    // regions (the chunks cut by a region boundary) add their contributions
    // to their columns with LDS atomics, all in one step, as the element
    // contributions to ys are added.  Columns of absent regions are zero.
    __shared__ double zred[12][16];
    static_assert(TAB_MAX * 3 >= 12 * 256, "the Z^T q columns are staged in ys");
    const int R = a.coarse_R, kk = 12 * R;
    for (int j = tid; j < kk; j += NT) czs[j] = 0.0;
    double s[4][3];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int c3 = 0; c3 < 3; ++c3) s[f][c3] = 0.0;
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int w = __float_as_int(gv[r].w);
      if (tid + NT * r < nown && (w & 0xff) == g0) {
        const double d[3] = {(double)gv[r].x, (double)gv[r].y, (double)gv[r].z};
#pragma unroll
        for (int c3 = 0; c3 < 3; ++c3) {
          const double qc = ((w >> (8 + c3)) & 1) ? 0.0 : (double)qk[r][c3];
          s[0][c3] += qc;
          s[1][c3] += qc * d[c3];
          s[2][c3] += qc * d[c3 == 2 ? 0 : c3 + 1];
          s[3][c3] += qc * d[c3 == 0 ? 2 : c3 - 1];
        }
      }
    }
    if (NT > 256) {  // fold the upper threads' sums onto threads 0-255 (fixed order)
      if (tid >= 256)
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
          for (int c3 = 0; c3 < 3; ++c3) ys[(f * 3 + c3) * 256 + tid - 256] = s[f][c3];
      __syncthreads();
      if (tid < 256)
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
          for (int c3 = 0; c3 < 3; ++c3) s[f][c3] += ys[(f * 3 + c3) * 256 + tid];
      __syncthreads();
    }
    if (tid < 256)
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int c3 = 0; c3 < 3; ++c3) ys[(f * 3 + c3) * 256 + tid] = s[f][c3];
    __syncthreads();  // also orders the zeroing of czs before the atomics below
    if (mall & (mall - 1)) {
      auto add = [&]() {
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
          const int w = __float_as_int(gv[r].w), g = w & 0xff;
          if (tid + NT * r < nown && g != g0) {
            const double d[3] = {(double)gv[r].x, (double)gv[r].y, (double)gv[r].z};
#pragma unroll
            for (int c3 = 0; c3 < 3; ++c3) {
              const double qc = ((w >> (8 + c3)) & 1) ? 0.0 : (double)qk[r][c3];
              if (qc == 0.0) continue;
              atomicAdd(&czs[g * 3 + c3], qc);
              atomicAdd(&czs[(R + g) * 3 + c3], qc * d[c3]);
              atomicAdd(&czs[(2 * R + g) * 3 + c3], qc * d[c3 == 2 ? 0 : c3 + 1]);
              atomicAdd(&czs[(3 * R + g) * 3 + c3], qc * d[c3 == 0 ? 2 : c3 - 1]);
            }
          }
        }
      };
      if (DET) wave_turns(add);
      else add();
    }
    if (tid < 192) {
      const int u = tid >> 4, sub = tid & 15;
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) v += ys[u * 256 + i * 16 + sub];
      zred[u][sub] = v;
    }
    __syncthreads();
    if (tid < 12 && g0 >= 0) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) v += zred[tid][i];
      czs[((tid / 3) * R + g0) * 3 + tid % 3] = v;
    }
    __syncthreads();
    // E^-1 Z^T q over the nonzero columns (twelve per region present; E^-1
    // symmetric, so column i serves as row i): those of the first one or two
    // regions are in e0 (for j = tid), the others are loaded two at a time
    for (int j = tid; j < kk; j += NT) {
      double wj = 0.0;
      uint32_t rest = mall;
      if (j == tid) {
#pragma unroll
        for (int u = 0; u < EPF; ++u) {
          const int g = u < 12 ? g0 : g1, v = u % 12;
          if (g >= 0) wj += e0[u] * czs[((v / 3) * R + g) * 3 + v % 3];
        }
        rest &= ~((g0 >= 0 ? 1u << g0 : 0u) | (EPF > 12 && g1 >= 0 ? 1u << g1 : 0u));
      }
      while (rest) {
        const int ga = __ffs((int)rest) - 1;
        rest &= rest - 1;
        const int gb = rest ? __ffs((int)rest) - 1 : -1;
        if (gb >= 0) rest &= rest - 1;
        double e[24];
#pragma unroll
        for (int u = 0; u < 24; ++u) {
          const int g = u < 12 ? ga : gb, v = u % 12;
          e[u] = g >= 0 ? a.einv[(long)(((v / 3) * R + g) * 3 + v % 3) * kk + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 24; ++u) {
          const int g = u < 12 ? ga : gb, v = u % 12;
          if (g >= 0) wj += e[u] * czs[((v / 3) * R + g) * 3 + v % 3];
        }
      }
      a.zq_part[(long)j * gridDim.x + blockIdx.x] = czs[j];
      a.zq_part[(long)(kk + j) * gridDim.x + blockIdx.x] = wj;
    }
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
// create.  Owned rows are inverted and written (identity for supported and
// hanging rows).
__global__ __launch_bounds__(512) void k_diag_chunks(double* __restrict__ dinv, const double* __restrict__ coef,
                                                     const uint8_t* __restrict__ fix, const double* __restrict__ K0,
                                                     ChunkArgs ca) {
  __shared__ double ds[TAB_MAX * 3];
  __shared__ uint32_t trip_hm_s[TRIP_MAX];
  __shared__ double trip_w_s[TRIP_MAX];
  __shared__ int hbeg_s[TAB_MAX];
  __shared__ double K0s[576];
  const int c = blockIdx.x;
  if (c >= ca.n_chunks) return;
  constexpr int DT = 512;
  const int tid = threadIdx.x;
  const ChunkDims cd = chunk_dims(ca, c);
  const int n0 = cd.n0, nent = cd.nent, t0 = cd.t0, nt = cd.nt, h0 = cd.h0, nh = cd.nh;
  const int nown = cd.nown, nreg = cd.nreg, nhown = cd.nhown;
  for (int i = tid; i < nt * 3; i += DT) ds[i] = 0.0;
  // the chunk's hanging triples and per-entry triple ranges, and K0, in LDS
  for (int k = tid; k < nh; k += DT) {
    trip_hm_s[k] = ca.trip_hm[h0 + k];
    trip_w_s[k] = ca.trip_w[h0 + k];
  }
  for (int t = nreg + tid; t < nt; t += DT) hbeg_s[t - nreg] = ca.tab_hbeg[t0 + t];
  for (int i = tid; i < 576; i += DT) K0s[i] = K0[i];
  __syncthreads();
  // vertex aa of an entry maps to the masters [kb, ke) of its hanging table
  // entry, or to itself (kb = -1) when regular
  auto range = [&](int l, int& kb, int& ke) {
    if (l < nreg) {
      kb = -1; ke = 0;
    } else {
      kb = hbeg_s[l - nreg];
      ke = l + 1 < nt ? hbeg_s[l + 1 - nreg] : nh;
    }
  };
  // one work item per (entry, vertex): the few entries that touch hanging
  // nodes carry most of the work, so it is spread over the threads by vertex
  // (deterministic mode: the waves take turns, see wave_turns)
  for (int base = 0; base < nent * 8; base += DT) {
    const int it = base + tid;
    auto item = [&]() {
    if (it >= nent * 8) return;
    const int en = it >> 3, aa = it & 7;
    int loc[8];
    const uint4 lv = *reinterpret_cast<const uint4*>(ca.ent_loc + 8L * (n0 + en));
    loc[0] = lv.x & 0xffff; loc[1] = lv.x >> 16; loc[2] = lv.y & 0xffff; loc[3] = lv.y >> 16;
    loc[4] = lv.z & 0xffff; loc[5] = lv.z >> 16; loc[6] = lv.w & 0xffff; loc[7] = lv.w >> 16;
    const double ce = coef[ca.ent_elem[n0 + en]];
    {
      int ka, kae;
      range(loc[aa], ka, kae);
      for (int k = ka; k < (ka < 0 ? 0 : kae); ++k) {
        const int ma = ka < 0 ? loc[aa] : (int)(trip_hm_s[k] & 0xffff);
        const double wa = ka < 0 ? 1.0 : trip_w_s[k];
        if (ma >= nown) continue;  // only owned rows are written
        double acc[3] = {0.0, 0.0, 0.0};
        for (int bb = 0; bb < 8; ++bb) {
          int kb, kbe;
          range(loc[bb], kb, kbe);
          for (int j = kb; j < (kb < 0 ? 0 : kbe); ++j) {
            const int mb = kb < 0 ? loc[bb] : (int)(trip_hm_s[j] & 0xffff);
            if (mb != ma) continue;
            const double w = wa * (kb < 0 ? 1.0 : trip_w_s[j]);
            for (int cc = 0; cc < 3; ++cc) acc[cc] += w * K0s[(3 * aa + cc) * 24 + 3 * bb + cc];
          }
        }
        for (int cc = 0; cc < 3; ++cc) atomicAdd(&ds[ma * 3 + cc], ce * acc[cc]);
      }
    }
    };
    if (ca.det) wave_turns(item);
    else item();
  }
  __syncthreads();
  for (int i = tid; i < (nown + nhown) * 3; i += DT) {
    int t = i / 3;
    const int comp = i % 3;
    const bool hang = t >= nown;
    if (hang) t = nreg + (t - nown);
    const long g = 3L * ca.tab_node[t0 + t] + comp;
    const bool fixed = (fix[g / 3] >> comp) & 1;
    dinv[g] = (hang || fixed) ? 1.0 : 1.0 / ds[t * 3 + comp];
  }
}

__global__ void k_to_float(const double* __restrict__ a, float* __restrict__ b, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------------ host side
void uniform_grid(const amrto_ctx* ctx, int& tiles_x, int& tiles_y, int& zchunk, int& n_tiles, int& grid) {
  tiles_x = (ctx->nx + 1 + UT - 1) / UT;
  tiles_y = (ctx->ny + 1 + UT - 1) / UT;
  const int layers = ctx->nz + 1;
  // aim for ~4 workgroups per CU (256 CUs) with at least 4 node layers each
  const int want = 1024;
  int nzc = std::max(1, want / std::max(1, tiles_x * tiles_y));
  zchunk = std::max(4, (layers + nzc - 1) / nzc);
  nzc = (layers + zchunk - 1) / zchunk;
  n_tiles = tiles_x * tiles_y * nzc;
  grid = ((n_tiles + 7) / 8) * 8;
}

template <typename VT>
static void brick_grid(const amrto_ctx* ctx, int& tiles_x, int& tiles_y, int& n_tiles) {
  constexpr int BZ = BrickZ<VT>::layers;
  tiles_x = (ctx->nx + 1 + BO - 1) / BO;
  tiles_y = (ctx->ny + 1 + BOY - 1) / BOY;
  n_tiles = tiles_x * tiles_y * ((ctx->nz + 1 + BZ - 1) / BZ);
}

// Both uniform kernels run on one grid (the larger of their tile counts,
// rounded to a multiple of 8), so the partial sums of p.q always fill the
// same slots whatever the precision; surplus workgroups write zeros.
int apply_blocks(const amrto_ctx* ctx) {
  if (ctx->uniform) {
    int tx, ty, zc, nt, grid, nb64, nb32;
    uniform_grid(ctx, tx, ty, zc, nt, grid);
    brick_grid<double>(ctx, tx, ty, nb64);
    brick_grid<float>(ctx, tx, ty, nb32);
    return ((std::max(nt, std::max(nb64, nb32)) + 7) / 8) * 8;
  }
  return ((ctx->n_chunks + 7) / 8) * 8;
}

template <typename VT, int PREC, bool FUSED, int COARSE = 0>
static void launch_chunks(amrto_ctx* ctx, dim3 grid, const UArgs& a, const ChunkArgs& ch, const CgArgs& cg) {
  if (ch.det)
    hipLaunchKernelGGL((k_apply_chunks<VT, PREC, FUSED, COARSE, true>), grid, dim3(chunk_threads(PREC, COARSE)), 0,
                       ctx->stream, a, ch, brick_k<VT>(ctx), cg);
  else
    hipLaunchKernelGGL((k_apply_chunks<VT, PREC, FUSED, COARSE, false>), grid, dim3(chunk_threads(PREC, COARSE)), 0,
                       ctx->stream, a, ch, brick_k<VT>(ctx), cg);
}

template <typename VT, int PREC, bool FUSED>
static int launch_t(amrto_ctx* ctx, const UArgs& ua, const CgArgs& cg) {
  if (ctx->uniform) {
    int tx, ty, zc, nt, grid;
    UArgs a = ua;
    a.nx = ctx->nx; a.ny = ctx->ny; a.nz = ctx->nz;
    if constexpr (PREC == P_BF16) {
      uniform_grid(ctx, tx, ty, zc, nt, grid);
      grid = apply_blocks(ctx);
      a.tiles_x = tx; a.tiles_y = ty; a.zchunk = zc; a.n_tiles = nt;
      hipLaunchKernelGGL((k_apply_uniform_bf16<FUSED>), dim3(grid), dim3(256), 0, ctx->stream, a, cg);
    } else {
      brick_grid<VT>(ctx, tx, ty, nt);
      grid = apply_blocks(ctx);
      a.tiles_x = tx; a.tiles_y = ty; a.zchunk = BrickZ<VT>::layers; a.n_tiles = nt;
      hipLaunchKernelGGL((k_apply_brick<VT, FUSED>), dim3(grid), dim3(BTHREADS), 0, ctx->stream, a, brick_k<VT>(ctx),
                         cg);
    }
  } else {
    launch_chunks<VT, PREC, FUSED>(ctx, dim3(apply_blocks(ctx)), ua, chunk_args(ctx), cg);
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

static UArgs base_args(amrto_ctx* ctx, int prec) {
  UArgs a;
  std::memset(&a, 0, sizeof a);
  a.fix = ctx->d_fix;
  a.coef = prec == AMRTO_FP64 ? (const void*)ctx->d_coef : (const void*)ctx->d_coef_f;
  a.kb = prec == AMRTO_BF16 ? (const void*)ctx->d_K0bf : nullptr;  // FP64/FP32 take the eight block constants
  return a;
}

int apply_stop(amrto_ctx* ctx, const void* x, void* y, int prec, const double* stop) {
  UArgs a = base_args(ctx, prec);
  a.x = x;
  a.y = y;
  a.stop = stop;
  CgArgs cg;
  std::memset(&cg, 0, sizeof cg);
  if (prec == AMRTO_FP64) return launch_t<double, P_F64, false>(ctx, a, cg);
  if (prec == AMRTO_FP32) return launch_t<float, P_F32, false>(ctx, a, cg);
  return launch_t<float, P_BF16, false>(ctx, a, cg);
}

int launch_apply(amrto_ctx* ctx, const void* x, void* y, int prec) { return apply_stop(ctx, x, y, prec, nullptr); }

// the octree FP64 operator pass with the multigrid smoothing epilogue (see UArgs)
int apply_cheb(amrto_ctx* ctx, const double* d, double* dnew, int mode, int step, const double* scal,
               const double* dinv, double* x, double* r, const double* binv) {
  if (ctx->uniform) return ctx->fail(AMRTO_ESTATE, "apply_cheb: octree meshes only");
  if (mode < 1 || mode > 3 || !scal || !dinv || !x || !r || (mode != 2 && (!dnew || dnew == d)))
    return ctx->fail(AMRTO_EINVAL, "apply_cheb: bad arguments");
  UArgs a = base_args(ctx, AMRTO_FP64);
  a.x = d;
  a.y = dnew;
  a.dinv = dinv;
  a.cheb_mode = mode;
  a.cheb_step = step;
  a.cheb_scal = scal;
  a.cheb_x = x;
  a.cheb_r = r;
  a.cheb_binv = binv;
  CgArgs cg;
  std::memset(&cg, 0, sizeof cg);
  return launch_t<double, P_F64, false>(ctx, a, cg);
}

// one fused CG step: p = z + beta p_old, q = A~ p, partial p.q
int apply_fused(amrto_ctx* ctx, const void* z, const void* pold, void* pnew, void* q, int prec, const CgArgs& cg) {
  UArgs a = base_args(ctx, prec);
  a.x = z;
  a.pold = pold;
  a.pnew = pnew;
  a.y = q;
  if (prec == AMRTO_FP64) return launch_t<double, P_F64, true>(ctx, a, cg);
  if (prec == AMRTO_FP32) return launch_t<float, P_F32, true>(ctx, a, cg);
  return launch_t<float, P_BF16, true>(ctx, a, cg);
}

// Fused octree pass with the affine coarse space folded into the staging
// (no separate z pass): p = (M r + Z cz) + beta p_old, q = A~ p, with M the
// Jacobi diagonal D^-1 (minv: 3 per node) or the inverse node blocks (block3:
// 6 per node).
int apply_fused_coarse(amrto_ctx* ctx, const void* r, const void* minv, const void* pold, void* pnew, void* q,
                       int prec, const CgArgs& cg, bool block3, double* zq_part) {
  if (ctx->uniform || !ctx->coarse_affine_only || ctx->coarse_k <= 0)
    return ctx->fail(AMRTO_ESTATE, "apply_fused_coarse: needs an octree mesh and an affine coarse space");
  UArgs a = base_args(ctx, prec);
  a.x = r;
  a.pold = pold;
  a.pnew = pnew;
  a.y = q;
  a.dinv = minv;
  a.geo = ctx->d_cgeo;
  a.cz = ctx->d_cz;
  a.coarse_R = ctx->coarse_R;
  a.zq_part = zq_part;
  a.einv = ctx->d_cinv;
  a.ct = ctx->d_ct;
  const dim3 grid(apply_blocks(ctx));
  const ChunkArgs ch = chunk_args(ctx);
  if (prec == AMRTO_FP64) {
    if (block3)
      launch_chunks<double, P_F64, true, 2>(ctx, grid, a, ch, cg);
    else
      launch_chunks<double, P_F64, true, 1>(ctx, grid, a, ch, cg);
  } else if (prec == AMRTO_FP32) {
    if (block3)
      launch_chunks<float, P_F32, true, 2>(ctx, grid, a, ch, cg);
    else
      launch_chunks<float, P_F32, true, 1>(ctx, grid, a, ch, cg);
  } else {
    if (block3)
      launch_chunks<float, P_BF16, true, 2>(ctx, grid, a, ch, cg);
    else
      launch_chunks<float, P_BF16, true, 1>(ctx, grid, a, ch, cg);
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int launch_diag(amrto_ctx* ctx) {
  const long n3 = 3L * ctx->n_nodes;
  if (ctx->uniform) {
    const long n = ctx->n_nodes;
    hipLaunchKernelGGL(k_diag_uniform, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_coef,
                       ctx->d_fix, ctx->K0[0], ctx->d_dinv, ctx->nx, ctx->ny, ctx->nz);
  } else {
    hipLaunchKernelGGL(k_diag_chunks, dim3(ctx->n_chunks), dim3(512), 0, ctx->stream, ctx->d_dinv, ctx->d_coef,
                       ctx->d_fix, ctx->d_K0, chunk_args(ctx));
  }
  hipLaunchKernelGGL(k_to_float, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_dinv,
                     ctx->d_dinv_f, n3);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

}  // namespace amrto
