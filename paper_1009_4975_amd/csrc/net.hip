// Learned warm start: a small fully convolutional network on a regular grid
// (FP32), trained and evaluated on the GPU by the kernels below, and the
// transfers between the finite-element mesh and that grid.
//
// Network: n_layers 3x3x3 convolutions (stride 1, zero padding 1) with ReLU
// between layers and none after the last.  Activations (B, C, Z, Y, X),
// weights (Cout, Cin, 3, 3, 3).  The convolutions are direct and tiled: a
// workgroup stages a halo tile of its sample in LDS and every thread keeps
// several output channels in registers (forward and data gradient); the weight
// gradient sums per workgroup in registers and then over workgroups in a fixed
// order (deterministic).
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.h"

struct amrto_net {
  int device = 0;
  hipStream_t stream = nullptr;
  int L = 0;
  int skip = -1;           // output += input channels [skip, skip + C_L) (-1: none)
  std::vector<int> ch;     // L + 1 channel counts
  int gx = 0, gy = 0, gz = 0, max_batch = 0, batch = 0;
  std::vector<long> woff;  // parameter offsets: w_l at woff[l], b_l after it
  long n_params = 0;
  float* d_params = nullptr;
  float* d_grads = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  std::vector<float*> acts;  // acts[0] = input copy, acts[l + 1] = output of layer l (post-ReLU except last)
  float* d_tmp0 = nullptr;   // gradient buffers (max activation size)
  float* d_tmp1 = nullptr;
  double* d_red = nullptr;
  float* d_wpart = nullptr;  // weight-gradient partial rows (wrows x the largest layer's parameter count)
  int wrows = 0;
  float* d_wt = nullptr;     // one layer's weights arranged for the tiled convolution
  std::string err;
  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
};

namespace amrto {

__device__ __forceinline__ bool in_grid(int z, int y, int x, int Z, int Y, int X) {
  return z >= 0 && z < Z && y >= 0 && y < Y && x >= 0 && x < X;
}

// ---------------------------------------------------------------- convolutions
// Tiled direct convolutions.  A workgroup of 256 threads owns an 8x8x4 tile
// of output positions (one per thread) of one sample and stages the input
// channels over the tile plus its one-cell halo in LDS, CG channels at a time
// (zero outside the grid: the zero padding).  The weights are the same for
// every thread of the workgroup and are read as uniform values; each thread
// keeps CG output channels in registers, so every staged value feeds CG
// multiply-adds.  Offsets d = (dz, dy, dx) + 1 in 0..2 run as d = 9 dz + 3 dy +
// dx, and off(d) = (dz - 1, dy - 1, dx - 1).
constexpr int CT_X = 8, CT_Y = 8, CT_Z = 4, CT_N = CT_X * CT_Y * CT_Z;  // output tile
constexpr int CH_X = CT_X + 2, CH_Y = CT_Y + 2, CH_Z = CT_Z + 2;
constexpr int CH_N = CH_X * CH_Y * CH_Z;  // staged tile with halo (600)
constexpr int CH_S = CH_N + 1;            // channel stride in LDS (odd: channels fall in different banks)
constexpr int CG = 16;                    // channels staged / outputs per thread at a time
constexpr int CGS = CT_N + 1;             // gradient-tile channel stride in LDS
static_assert(CT_N == 256, "one output position per thread");

struct ConvGrid {
  int Z, Y, X, tx, ty, tz;  // grid and tiles per axis
};

__device__ __forceinline__ int halo_off(int d) { return ((d / 9) * CH_Y + (d / 3) % 3) * CH_X + d % 3; }

// channels [c0, c0 + CG) of src (sample n, C channels) over the halo tile whose
// first cell is (x0 - 1, y0 - 1, z0 - 1) into s; zero outside the grid and for
// c >= C; with mask (same shape as src) values whose mask is not > 0 are zero
// (the ReLU derivative)
// (256 threads: a thread's loads go out in batches of 8 before they are
// stored, so at most 8 wait at once and the registers stay few)
constexpr int STAGE_PER = (CG * CH_N + 255) / 256;
constexpr int STAGE_B = 8;
__device__ __forceinline__ void stage_halo(const float* __restrict__ src, const float* __restrict__ mask, int n,
                                           int C, int c0, const ConvGrid& G, int z0, int y0, int x0, float* s) {
  const long V = (long)G.Z * G.Y * G.X;
#pragma unroll 1
  for (int m0 = 0; m0 < STAGE_PER; m0 += STAGE_B) {
    float v[STAGE_B];
#pragma unroll
    for (int m = 0; m < STAGE_B; ++m) {
      const int k = threadIdx.x + 256 * (m0 + m);
      const int c = k / CH_N, h = k - c * CH_N;
      const int hx = h % CH_X, hy = (h / CH_X) % CH_Y, hz = h / (CH_X * CH_Y);
      const int x = x0 - 1 + hx, y = y0 - 1 + hy, z = z0 - 1 + hz;
      v[m] = 0.f;
      if (k < CG * CH_N && c0 + c < C && in_grid(z, y, x, G.Z, G.Y, G.X)) {
        const long q = ((long)n * C + c0 + c) * V + ((long)z * G.Y + y) * G.X + x;
        v[m] = src[q];
        if (mask && !(mask[q] > 0.f)) v[m] = 0.f;
      }
    }
#pragma unroll
    for (int m = 0; m < STAGE_B; ++m) {
      const int k = threadIdx.x + 256 * (m0 + m);
      if (k < CG * CH_N) s[(k / CH_N) * CH_S + k % CH_N] = v[m];
    }
  }
}

// Weights of one layer rearranged for k_conv_tiled: wt[og][c][d][16] holds, for
// output group og (16 outputs, zero beyond Cd) and staged channel c < Cs,
//   FWD: w[o, c, d]       (o = 16 og + k, Cs = Cin, Cd = Cout)
//   BWD: w[c, i, 26 - d]  (i = 16 og + k, Cs = Cout, Cd = Cin),
// so the 16 weights of a tap are contiguous and every thread of a workgroup
// reads the same ones (uniform loads into scalar registers).
template <bool BWD>
__global__ __launch_bounds__(256) void k_conv_wt(const float* __restrict__ w, float* __restrict__ wt, int Cs, int Cd) {
  const int n_og = (Cd + CG - 1) / CG;
  const long n = (long)n_og * Cs * 27 * CG;
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int k = (int)(j % CG), d = (int)((j / CG) % 27), c = (int)((j / (CG * 27)) % Cs), og = (int)(j / ((long)CG * 27 * Cs));
  const int o = og * CG + k;
  float v = 0.f;
  if (o < Cd) v = BWD ? w[((long)c * Cd + o) * 27 + 26 - d] : w[((long)o * Cs + c) * 27 + d];
  wt[j] = v;
}

// FWD (BWD = false): dst[n, o, p] = bias[o] + sum_{i < Cs, d} w[o, i, d] src[n, i, p + off(d)],
//   then ReLU if relu (Cs = Cin, Cd = Cout).
// BWD: dst[n, i, p] = sum_{o < Cs, d} w[o, i, d] srcm[n, o, p - off(d)]
//   = sum_{o, d} w[o, i, 26 - d] srcm[n, o, p + off(d)], srcm = src masked by mask
//   (Cs = Cout, Cd = Cin): the data gradient through the ReLU of the layer's output.
// wt: the weights as k_conv_tiled<BWD> arranges them.  Grid: (tiles, ceil(Cd / CG), batch).
template <bool BWD>
__global__ __launch_bounds__(256) void k_conv_tiled(const float* __restrict__ src, const float* __restrict__ mask,
                                                    const float* __restrict__ wt, const float* __restrict__ bias,
                                                    float* __restrict__ dst, int Cs, int Cd, ConvGrid G, int relu) {
  __shared__ float s[CG * CH_S];
  const int tile = blockIdx.x, o0 = blockIdx.y * CG, n = blockIdx.z;
  const int x0 = (tile % G.tx) * CT_X, y0 = ((tile / G.tx) % G.ty) * CT_Y, z0 = (tile / (G.tx * G.ty)) * CT_Z;
  const int lx = threadIdx.x % CT_X, ly = (threadIdx.x / CT_X) % CT_Y, lz = threadIdx.x / (CT_X * CT_Y);
  const int hb = (lz * CH_Y + ly) * CH_X + lx;
  const float* __restrict__ wg = wt + (long)blockIdx.y * Cs * 27 * CG;
  float acc[CG];
#pragma unroll
  for (int oo = 0; oo < CG; ++oo) acc[oo] = 0.f;
  for (int c0 = 0; c0 < Cs; c0 += CG) {
    __syncthreads();  // the previous group has been read
    stage_halo(src, BWD ? mask : nullptr, n, Cs, c0, G, z0, y0, x0, s);
    __syncthreads();
    const int cn = min(CG, Cs - c0);
    for (int c = 0; c < cn; ++c) {
      // one z plane of taps (9) per step
#pragma unroll 1
      for (int dz = 0; dz < 3; ++dz) {
        const float* sc = s + c * CH_S + hb + dz * CH_X * CH_Y;
        const float* wc = wg + ((long)(c0 + c) * 27 + dz * 9) * CG;
#pragma unroll
        for (int d = 0; d < 9; ++d) {
          const float v = sc[(d / 3) * CH_X + d % 3];
#pragma unroll
          for (int oo = 0; oo < CG; ++oo) acc[oo] = fmaf(wc[d * CG + oo], v, acc[oo]);
        }
      }
    }
  }
  const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
  if (!in_grid(z, y, x, G.Z, G.Y, G.X)) return;
  const long V = (long)G.Z * G.Y * G.X, p = ((long)z * G.Y + y) * G.X + x;
#pragma unroll
  for (int oo = 0; oo < CG; ++oo)
    if (o0 + oo < Cd) {
      float v = acc[oo] + (BWD ? 0.f : bias[o0 + oo]);
      if (relu) v = fmaxf(v, 0.f);
      dst[((long)n * Cd + o0 + oo) * V + p] = v;
    }
}

// Weight gradient, partial sums per workgroup:
//   dw[o, i, d] = sum_{n, p} gm[n, o, p] in[n, i, p + off(d)],  db[o] = sum gm[n, o, p],
// gm = g masked by the ReLU of the layer's output.  Workgroup (b, combo) walks
// the (sample, tile) pairs b, b + gridDim.x, ... for the channel groups of its
// combo (input group ig, output group og); thread (i, oq, pg) = tid (16, 4, 4)
// keeps 4 outputs x 27 offsets of input channel i over the 64 positions of
// group pg.  The four position groups (one per wave) are folded in wave order
// through LDS, and row b of part receives this workgroup's share of the layer's
// P = Co Ci 27 + Co gradient entries (k_wgrad_reduce sums the rows in order).
__global__ __launch_bounds__(256) void k_conv_wgrad(const float* __restrict__ g, const float* __restrict__ post,
                                                    const float* __restrict__ in, float* __restrict__ part, int B,
                                                    int Ci, int Co, ConvGrid G, long P) {
  __shared__ float s_in[CG * CH_S];
  __shared__ float s_g[CG * CGS];
  static_assert(CG * CH_S >= 64 * 4 * 27 + 64 * 4, "the fold buffer fits in s_in");
  const int n_ig = (Ci + CG - 1) / CG;
  const int ig = blockIdx.y % n_ig, og = blockIdx.y / n_ig;
  const int i0 = ig * CG, o0 = og * CG;
  const int tid = threadIdx.x, i = tid & 15, oq = (tid >> 4) & 3, pg = tid >> 6;
  const int n_tiles = G.tx * G.ty * G.tz;
  const long V = (long)G.Z * G.Y * G.X;
  float acc[4][27], accb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    accb[k] = 0.f;
#pragma unroll
    for (int d = 0; d < 27; ++d) acc[k][d] = 0.f;
  }
  for (int t = blockIdx.x; t < n_tiles * B; t += gridDim.x) {
    const int n = t / n_tiles, tile = t - n * n_tiles;
    const int x0 = (tile % G.tx) * CT_X, y0 = ((tile / G.tx) % G.ty) * CT_Y, z0 = (tile / (G.tx * G.ty)) * CT_Z;
    __syncthreads();
    stage_halo(in, nullptr, n, Ci, i0, G, z0, y0, x0, s_in);
    // the gradient tile: thread tid holds position tid of every channel, so
    // one position's index work serves its CG loads (all requested at once)
    {
      const int x = x0 + tid % CT_X, y = y0 + (tid / CT_X) % CT_Y, z = z0 + tid / (CT_X * CT_Y);
      const bool in = in_grid(z, y, x, G.Z, G.Y, G.X);
      const long p = ((long)z * G.Y + y) * G.X + x;
      float gv_in[CG];
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        gv_in[c] = 0.f;
        if (in && o0 + c < Co) {
          const long gi = ((long)n * Co + o0 + c) * V + p;
          gv_in[c] = g[gi];
          if (post && !(post[gi] > 0.f)) gv_in[c] = 0.f;
        }
      }
#pragma unroll
      for (int c = 0; c < CG; ++c) s_g[c * CGS + tid] = gv_in[c];
    }
    __syncthreads();
    for (int q = pg * 64; q < pg * 64 + 64; ++q) {
      const int hb = ((q / (CT_X * CT_Y)) * CH_Y + (q / CT_X) % CT_Y) * CH_X + q % CT_X;
      float gv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        gv[k] = s_g[(oq * 4 + k) * CGS + q];
        accb[k] += gv[k];
      }
      const float* sc = s_in + i * CH_S + hb;
#pragma unroll
      for (int d = 0; d < 27; ++d) {
        const float v = sc[halo_off(d)];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k][d] = fmaf(gv[k], v, acc[k][d]);
      }
    }
  }
  // fold the four position groups in wave order: slot (i, oq) holds 4 x 27
  // weight sums, then 4 bias sums
  float* red = s_in;
  const int slot = i * 4 + oq;
  for (int wv = 0; wv < 4; ++wv) {
    __syncthreads();
    if (pg == wv) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int d = 0; d < 27; ++d) {
          float* r = red + slot * 108 + k * 27 + d;
          *r = (wv ? *r : 0.f) + acc[k][d];
        }
        float* rb = red + 64 * 108 + slot * 4 + k;
        *rb = (wv ? *rb : 0.f) + accb[k];
      }
    }
  }
  __syncthreads();
  float* row = part + (long)blockIdx.x * P;
  for (int e = tid; e < 64 * 108; e += blockDim.x) {
    const int sl = e / 108, r = e - sl * 108, k = r / 27, d = r - k * 27;
    const int ii = i0 + sl / 4, o = o0 + (sl % 4) * 4 + k;
    if (ii < Ci && o < Co) row[((long)o * Ci + ii) * 27 + d] = red[e];
  }
  if (ig == 0 && tid < 16) {  // bias: the slots of input channel 0 carry the sums of g
    const int o = o0 + tid;
    if (o < Co) row[(long)Co * Ci * 27 + o] = red[64 * 108 + (tid / 4) * 4 + tid % 4];
  }
}

// out[j] = sum over rows b < nrows of part[b P + j], in a fixed order: a
// workgroup takes 64 entries; its four waves sum the rows b = w, w + 4, ...
// (FP64) and the four sums are added in wave order.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int nrows, long P,
                                                      float* __restrict__ out) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long j = blockIdx.x * 64L + lane;
  double s = 0.0;
  if (j < P)
    for (int b = wv; b < nrows; b += 4) s += (double)part[(long)b * P + j];
  sh[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && j < P) out[j] = (float)(((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane]);
}

// masked MSE: partial sums of mask (p - t)^2 and of mask; dpred = 2 mask (p - t) / sum(mask)
__global__ __launch_bounds__(256) void k_mse_part(const float* __restrict__ p, const float* __restrict__ t,
                                                  const uint8_t* __restrict__ m, long n, double* __restrict__ part) {
  __shared__ double sh[8];
  double s = 0.0, c = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (!m || m[i]) {
      const double d = (double)p[i] - (double)t[i];
      s += d * d;
      c += 1.0;
    }
  s = block_sum(s, sh);
  c = block_sum(c, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    part[RED_BLOCKS + blockIdx.x] = c;
  }
}

__global__ __launch_bounds__(256) void k_mse_grad(const float* __restrict__ p, const float* __restrict__ t,
                                                  const uint8_t* __restrict__ m, long n,
                                                  const double* __restrict__ part, float* __restrict__ dp,
                                                  double* __restrict__ out) {
  __shared__ double sh[8];
  const double s = sum_partials(part, RED_BLOCKS, sh);
  const double c = sum_partials(part + RED_BLOCKS, RED_BLOCKS, sh);
  const double inv = c > 0 ? 1.0 / c : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = s * inv;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dp[i] = (!m || m[i]) ? (float)(2.0 * ((double)p[i] - (double)t[i]) * inv) : 0.f;
}

// out[n, oo + c, p] += in[n, io + c, p] for c < C (residual connection around
// the stack; out has Co channels, in has Ci)
__global__ __launch_bounds__(256) void k_add_skip(float* __restrict__ out, int Co, int oo, const float* __restrict__ in,
                                                  int Ci, int io, int C, int B, long V) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)B * C * V) return;
  const long p = idx % V;
  const int c = (int)((idx / V) % C), n = (int)(idx / (V * C));
  out[((long)n * Co + oo + c) * V + p] += in[((long)n * Ci + io + c) * V + p];
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ mesh <-> grid
// rho_grid[g] = sum over the elements overlapping the dual cell of grid node g
// of rho_e times the overlapped fraction of that cell (fixed order: deterministic)
__global__ __launch_bounds__(256) void k_grid_density(const double* __restrict__ rho, const int32_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ elem, const double* __restrict__ w,
                                                      int n_gn, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_gn) return;
  double s = 0.0;
  for (int k = ptr[c]; k < ptr[c + 1]; ++k) s += w[k] * rho[elem[k]];
  out[c] = (float)s;
}

// u_grid[c][g] = scale sum_a w[8 g + a] (u - u_ref)[3 node[8 g + a] + c]
__global__ __launch_bounds__(256) void k_grid_sample(const double* __restrict__ u, const double* __restrict__ uref,
                                                     const int32_t* __restrict__ node, const float* __restrict__ w,
                                                     long n_gn, double scale, float* __restrict__ out) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= 3 * n_gn) return;
  const int c = (int)(i / n_gn);
  const long g = i % n_gn;
  double v = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const long d = 3L * node[8 * g + a] + c;
    v += (double)w[8 * g + a] * (uref ? u[d] - uref[d] : u[d]);
  }
  out[i] = (float)(scale * v);
}

// u[3 n + c] = scale x trilinear interpolation of u_grid[c] at the node's lattice position
__global__ __launch_bounds__(256) void k_grid_interp(const float* __restrict__ ug, const int32_t* __restrict__ xyz,
                                                     int n_nodes, int cell, int gx, int gy, int gz, double scale,
                                                     double* __restrict__ u, int sx, int sy) {
  const int nd = blockIdx.x * blockDim.x + threadIdx.x;
  if (nd >= n_nodes) return;
  int px, py, pz;
  if (xyz) {
    px = xyz[3L * nd]; py = xyz[3L * nd + 1]; pz = xyz[3L * nd + 2];
  } else {
    px = nd % sx; py = (nd / sx) % sy; pz = nd / (sx * sy);
  }
  const int ix = min(px / cell, gx - 1), iy = min(py / cell, gy - 1), iz = min(pz / cell, gz - 1);
  const double tx = (double)(px - ix * cell) / cell, ty = (double)(py - iy * cell) / cell,
               tz = (double)(pz - iz * cell) / cell;
  const long NX = gx + 1, NY = gy + 1, NN = NX * NY * (gz + 1);
  for (int c = 0; c < 3; ++c) {
    double v = 0.0;
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
      const double w = (ax ? tx : 1.0 - tx) * (ay ? ty : 1.0 - ty) * (az ? tz : 1.0 - tz);
      v += w * ug[c * NN + ((iz + az) * NY + iy + ay) * NX + ix + ax];
    }
    u[3L * nd + c] = scale * v;
  }
}

static uint64_t splitmix64(uint64_t x) {
  // SplitMix64 (Steele, Lea, Flood 2014) output function of state x
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

}  // namespace amrto

using namespace amrto;

#define NET_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return net->fail(AMRTO_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

static ConvGrid conv_grid(const amrto_net* net) {
  ConvGrid G;
  G.Z = net->gz; G.Y = net->gy; G.X = net->gx;
  G.tx = (net->gx + CT_X - 1) / CT_X;
  G.ty = (net->gy + CT_Y - 1) / CT_Y;
  G.tz = (net->gz + CT_Z - 1) / CT_Z;
  return G;
}

extern "C" {

int amrto_net_create(amrto_net** out, int device, void* stream, int32_t n_layers, const int32_t* channels,
                     int32_t skip_from, int32_t gx, int32_t gy, int32_t gz, int32_t max_batch, uint64_t seed) {
  if (!out || !channels || n_layers < 1 || n_layers > 16 || gx < 1 || gy < 1 || gz < 1 || max_batch < 1)
    return AMRTO_EINVAL;
  if (skip_from >= 0 && skip_from + channels[n_layers] > channels[0]) return AMRTO_EINVAL;
  for (int l = 0; l <= n_layers; ++l)
    if (channels[l] < 1 || channels[l] > 256) return AMRTO_EINVAL;
  amrto_net* net = new (std::nothrow) amrto_net();
  if (!net) return AMRTO_ENOMEM;
  *out = nullptr;
  net->device = device;
  net->stream = (hipStream_t)stream;
  net->L = n_layers;
  net->skip = skip_from < 0 ? -1 : skip_from;
  net->ch.assign(channels, channels + n_layers + 1);
  net->gx = gx; net->gy = gy; net->gz = gz; net->max_batch = max_batch;
  long off = 0;
  for (int l = 0; l < n_layers; ++l) {
    net->woff.push_back(off);
    off += (long)channels[l + 1] * channels[l] * 27 + channels[l + 1];
  }
  net->n_params = off;
  if (hipSetDevice(device) != hipSuccess) { delete net; return AMRTO_EHIP; }
  const long V = (long)gx * gy * gz;
  int cmax = 0;
  for (int c : net->ch) cmax = std::max(cmax, c);
  bool ok = hipMalloc((void**)&net->d_params, off * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_grads, off * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_m, off * 4) == hipSuccess && hipMalloc((void**)&net->d_v, off * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_tmp0, (long)max_batch * cmax * V * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_tmp1, (long)max_batch * cmax * V * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_red, 4 * RED_BLOCKS * sizeof(double)) == hipSuccess;
  // weight-gradient partials: up to 512 rows, at most 16 M floats in all
  long pmax = 1;
  for (int l = 0; l < n_layers; ++l) pmax = std::max(pmax, (long)channels[l + 1] * channels[l] * 27 + channels[l + 1]);
  net->wrows = (int)std::max(1L, std::min(512L, (16L << 20) / pmax));
  ok = ok && hipMalloc((void**)&net->d_wpart, (long)net->wrows * pmax * 4) == hipSuccess;
  long wtmax = 1;
  for (int l = 0; l < n_layers; ++l) {
    const long a = channels[l], b = channels[l + 1];
    wtmax = std::max(wtmax, std::max((b + 15) / 16 * 16 * a * 27, (a + 15) / 16 * 16 * b * 27));
  }
  ok = ok && hipMalloc((void**)&net->d_wt, wtmax * 4) == hipSuccess;
  for (int l = 0; l <= n_layers && ok; ++l) {
    float* p = nullptr;
    ok = hipMalloc((void**)&p, (long)max_batch * channels[l] * V * 4) == hipSuccess;
    net->acts.push_back(p);
  }
  if (!ok) { amrto_net_destroy(net); return AMRTO_ENOMEM; }
  // He-normal weights from a counter-based generator (SplitMix64 + Box-Muller), zero biases
  std::vector<float> h(off, 0.f);
  for (int l = 0; l < n_layers; ++l) {
    const long nw = (long)channels[l + 1] * channels[l] * 27;
    const double sd = std::sqrt(2.0 / (27.0 * channels[l]));
    for (long k = 0; k < nw; ++k) {
      const uint64_t a = splitmix64(seed ^ (uint64_t)(net->woff[l] + k) * 2ULL);
      const uint64_t b = splitmix64(seed ^ ((uint64_t)(net->woff[l] + k) * 2ULL + 1ULL));
      const double u1 = ((a >> 11) + 1.0) / 9007199254740993.0, u2 = (b >> 11) / 9007199254740992.0;
      h[net->woff[l] + k] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
  }
  if (hipMemcpy(net->d_params, h.data(), off * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(net->d_m, 0, off * 4) != hipSuccess || hipMemset(net->d_v, 0, off * 4) != hipSuccess) {
    amrto_net_destroy(net);
    return AMRTO_EHIP;
  }
  *out = net;
  return AMRTO_OK;
}

int amrto_net_destroy(amrto_net* net) {
  if (!net) return AMRTO_OK;
  (void)hipSetDevice(net->device);
  (void)hipDeviceSynchronize();
  for (float* p : {net->d_params, net->d_grads, net->d_m, net->d_v, net->d_tmp0, net->d_tmp1})
    if (p) (void)hipFree(p);
  for (float* p : net->acts)
    if (p) (void)hipFree(p);
  if (net->d_red) (void)hipFree(net->d_red);
  if (net->d_wpart) (void)hipFree(net->d_wpart);
  if (net->d_wt) (void)hipFree(net->d_wt);
  delete net;
  return AMRTO_OK;
}

const char* amrto_net_last_error(const amrto_net* net) { return net ? net->err.c_str() : "null network"; }

int amrto_net_n_params(const amrto_net* net, int64_t* n) {
  if (!net || !n) return AMRTO_EINVAL;
  *n = net->n_params;
  return AMRTO_OK;
}

int amrto_net_get_params(const amrto_net* net, float* host) {
  if (!net || !host) return AMRTO_EINVAL;
  return hipMemcpy(host, net->d_params, net->n_params * 4, hipMemcpyDeviceToHost) == hipSuccess ? AMRTO_OK : AMRTO_EHIP;
}

int amrto_net_set_params(amrto_net* net, const float* host) {
  if (!net || !host) return AMRTO_EINVAL;
  return hipMemcpy(net->d_params, host, net->n_params * 4, hipMemcpyHostToDevice) == hipSuccess ? AMRTO_OK : AMRTO_EHIP;
}

int amrto_net_get_grads(const amrto_net* net, float* host) {
  if (!net || !host) return AMRTO_EINVAL;
  return hipMemcpy(host, net->d_grads, net->n_params * 4, hipMemcpyDeviceToHost) == hipSuccess ? AMRTO_OK : AMRTO_EHIP;
}

int amrto_net_get_adam(const amrto_net* net, float* m_host, float* v_host) {
  if (!net || !m_host || !v_host) return AMRTO_EINVAL;
  const size_t bytes = net->n_params * 4;
  return hipMemcpy(m_host, net->d_m, bytes, hipMemcpyDeviceToHost) == hipSuccess &&
                 hipMemcpy(v_host, net->d_v, bytes, hipMemcpyDeviceToHost) == hipSuccess
             ? AMRTO_OK
             : AMRTO_EHIP;
}

int amrto_net_set_adam(amrto_net* net, const float* m_host, const float* v_host) {
  if (!net || !m_host || !v_host) return AMRTO_EINVAL;
  for (int64_t i = 0; i < net->n_params; ++i)
    if (!std::isfinite(m_host[i]) || !std::isfinite(v_host[i]) || v_host[i] < 0.f)
      return net->fail(AMRTO_EINVAL, "amrto_net_set_adam: moments must be finite, second moments >= 0");
  const size_t bytes = net->n_params * 4;
  return hipMemcpy(net->d_m, m_host, bytes, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(net->d_v, v_host, bytes, hipMemcpyHostToDevice) == hipSuccess
             ? AMRTO_OK
             : AMRTO_EHIP;
}

int amrto_net_forward(amrto_net* net, const float* in, int32_t batch, float* out) {
  if (!net || !in || batch < 1 || batch > net->max_batch) return net ? net->fail(AMRTO_EINVAL, "amrto_net_forward: bad arguments") : AMRTO_EINVAL;
  NET_HIP(hipSetDevice(net->device));
  const long V = (long)net->gx * net->gy * net->gz;
  net->batch = batch;
  NET_HIP(hipMemcpyAsync(net->acts[0], in, (long)batch * net->ch[0] * V * 4, hipMemcpyDeviceToDevice, net->stream));
  for (int l = 0; l < net->L; ++l) {
    const float* w = net->d_params + net->woff[l];
    const float* b = w + (long)net->ch[l + 1] * net->ch[l] * 27;
    const ConvGrid G = conv_grid(net);
    const int Ci = net->ch[l], Co = net->ch[l + 1], n_og = (Co + CG - 1) / CG;
    const long nwt = (long)n_og * CG * Ci * 27;
    hipLaunchKernelGGL(k_conv_wt<false>, dim3((unsigned)((nwt + 255) / 256)), dim3(256), 0, net->stream, w, net->d_wt,
                       Ci, Co);
    hipLaunchKernelGGL(k_conv_tiled<false>, dim3(G.tx * G.ty * G.tz, n_og, batch), dim3(256), 0, net->stream,
                       net->acts[l], nullptr, net->d_wt, b, net->acts[l + 1], Ci, Co, G, l + 1 < net->L ? 1 : 0);
  }
  if (net->skip >= 0) {
    const long n = (long)batch * net->ch[net->L] * V;
    hipLaunchKernelGGL(k_add_skip, dim3((n + 255) / 256), dim3(256), 0, net->stream, net->acts[net->L],
                       net->ch[net->L], 0, net->acts[0], net->ch[0], net->skip, net->ch[net->L], batch, V);
  }
  if (out)
    NET_HIP(hipMemcpyAsync(out, net->acts[net->L], (long)batch * net->ch[net->L] * V * 4, hipMemcpyDeviceToDevice,
                           net->stream));
  NET_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_net_backward(amrto_net* net, const float* dout, float* din) {
  if (!net || !dout || net->batch < 1) return net ? net->fail(AMRTO_ESTATE, "amrto_net_backward: no forward pass") : AMRTO_EINVAL;
  NET_HIP(hipSetDevice(net->device));
  const int B = net->batch;
  const long V = (long)net->gx * net->gy * net->gz;
  const float* g = dout;
  float* bufs[2] = {net->d_tmp0, net->d_tmp1};
  for (int l = net->L - 1; l >= 0; --l) {
    const int Ci = net->ch[l], Co = net->ch[l + 1];
    const float* post = l + 1 < net->L ? net->acts[l + 1] : nullptr;  // ReLU mask of this layer's output
    float* w = net->d_params + net->woff[l];
    float* dw = net->d_grads + net->woff[l];
    const ConvGrid G = conv_grid(net);
    const long P = (long)Co * Ci * 27 + Co;
    const int rows = (int)std::min<long>(net->wrows, (long)G.tx * G.ty * G.tz * B);
    const int combos = ((Ci + CG - 1) / CG) * ((Co + CG - 1) / CG);
    hipLaunchKernelGGL(k_conv_wgrad, dim3(rows, combos), dim3(256), 0, net->stream, g, post, net->acts[l],
                       net->d_wpart, B, Ci, Co, G, P);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((P + 63) / 64)), dim3(256), 0, net->stream, net->d_wpart,
                       rows, P, dw);
    if (l > 0 || din) {
      float* dst = l > 0 ? bufs[l & 1] : din;
      const int n_ig = (Ci + CG - 1) / CG;
      const long nwt = (long)n_ig * CG * Co * 27;
      hipLaunchKernelGGL(k_conv_wt<true>, dim3((unsigned)((nwt + 255) / 256)), dim3(256), 0, net->stream, w,
                         net->d_wt, Co, Ci);
      hipLaunchKernelGGL(k_conv_tiled<true>, dim3(G.tx * G.ty * G.tz, n_ig, B), dim3(256), 0, net->stream, g, post,
                         net->d_wt, nullptr, dst, Co, Ci, G, 0);
      g = dst;
    }
  }
  if (din && net->skip >= 0) {
    const long n = (long)B * net->ch[net->L] * V;
    hipLaunchKernelGGL(k_add_skip, dim3((n + 255) / 256), dim3(256), 0, net->stream, din, net->ch[0], net->skip, dout,
                       net->ch[net->L], 0, net->ch[net->L], B, V);
  }
  NET_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_net_mse(amrto_net* net, const float* pred, const float* tgt, const uint8_t* mask, int64_t n, float* dpred,
                  double* loss_host) {
  if (!net || !pred || !tgt || !dpred || n < 1) return AMRTO_EINVAL;
  NET_HIP(hipSetDevice(net->device));
  hipLaunchKernelGGL(k_mse_part, dim3(RED_BLOCKS), dim3(256), 0, net->stream, pred, tgt, mask, (long)n, net->d_red);
  hipLaunchKernelGGL(k_mse_grad, dim3(RED_BLOCKS), dim3(256), 0, net->stream, pred, tgt, mask, (long)n, net->d_red,
                     dpred, net->d_red + 2 * RED_BLOCKS);
  NET_HIP(hipGetLastError());
  if (loss_host) {
    NET_HIP(hipMemcpyAsync(loss_host, net->d_red + 2 * RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, net->stream));
    NET_HIP(hipStreamSynchronize(net->stream));
  }
  return AMRTO_OK;
}

int amrto_net_adam(amrto_net* net, float lr, float b1, float b2, float eps, int32_t t) {
  if (!net || t < 1) return AMRTO_EINVAL;
  NET_HIP(hipSetDevice(net->device));
  const long n = net->n_params;
  const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, net->stream, net->d_params, net->d_grads, net->d_m,
                     net->d_v, n, lr, b1, b2, eps, c1, c2);
  NET_HIP(hipGetLastError());
  return AMRTO_OK;
}

// ------------------------------------------------------------------ mesh <-> grid
// Host tables of the transfers for grid cells of edge `cell` lattice units:
// the elements overlapping each cell with their overlap fractions, and for
// each grid node the element containing it with the trilinear weights of that
// element's vertices (exact at mesh nodes; at a hanging node it equals the
// constrained value of Eq. (6)).
static int grid_maps(amrto_ctx* ctx, int cell) {
  if (ctx->grid_cell == cell) return AMRTO_OK;
  if (cell < 1 || ctx->nx % cell || ctx->ny % cell || ctx->nz % cell)
    return ctx->fail(AMRTO_EINVAL, "grid: cell must divide the domain");
  const int gx = ctx->nx / cell, gy = ctx->ny / cell, gz = ctx->nz / cell;
  const long NX = gx + 1, NY = gy + 1, n_gn = NX * NY * (gz + 1);
  const int ne = ctx->n_elems;
  std::vector<int32_t> celem, fill;
  std::vector<double> cw;
  auto elem_geom = [&](int e, int* p, int* vert) -> int {
    if (ctx->uniform) {
      const int ex = e % ctx->nx, ey = (e / ctx->nx) % ctx->ny, ez = e / (ctx->nx * ctx->ny);
      p[0] = ex; p[1] = ey; p[2] = ez;
      for (int a = 0; a < 8; ++a)
        vert[a] = (ex + (a & 1)) + (ctx->nx + 1) * ((ey + ((a >> 1) & 1)) + (ctx->ny + 1) * (ez + (a >> 2)));
      return 1;
    }
    for (int a = 0; a < 8; ++a) vert[a] = ctx->h_elem_nodes[8L * e + a];
    const int* q = &ctx->h_node_xyz[3L * vert[0]];
    p[0] = q[0]; p[1] = q[1]; p[2] = q[2];
    return 1 << (ctx->max_level - ctx->h_level[e]);
  };
  // grid node -> elements overlapping its dual cell (the box of edge `cell`
  // centred at the node, clipped to the domain); doubled coordinates keep the
  // half-cell offsets integral.  Counting pass, then fill in element order.
  const int dims[3] = {ctx->nx, ctx->ny, ctx->nz};
  const int gdim[3] = {gx, gy, gz};
  int p[3], vert[8];
  auto node_range = [&](int ax, int lo, int h, int& n0, int& n1) {
    n0 = std::max(0, (2 * lo - cell) / (2 * cell) - 1);
    n1 = std::min(gdim[ax], (2 * (lo + h) + cell) / (2 * cell) + 1);
  };
  auto overlap2 = [&](int ax, int i, int lo, int h) -> long {
    const long b0 = std::max(0L, 2L * i * cell - cell), b1 = std::min(2L * dims[ax], 2L * i * cell + cell);
    return std::max(0L, std::min(b1, 2L * (lo + h)) - std::max(b0, 2L * lo));
  };
  auto box2 = [&](int ax, int i) -> long {
    return std::min(2L * dims[ax], 2L * i * cell + cell) - std::max(0L, 2L * i * cell - cell);
  };
  std::vector<int32_t> cnt(n_gn + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
    for (int e = 0; e < ne; ++e) {
      const int h = elem_geom(e, p, vert);
      int r[3][2];
      for (int ax = 0; ax < 3; ++ax) node_range(ax, p[ax], h, r[ax][0], r[ax][1]);
      for (int k = r[2][0]; k <= r[2][1]; ++k)
        for (int j = r[1][0]; j <= r[1][1]; ++j)
          for (int i = r[0][0]; i <= r[0][1]; ++i) {
            const long o = overlap2(0, i, p[0], h) * overlap2(1, j, p[1], h) * overlap2(2, k, p[2], h);
            if (o == 0) continue;
            const long g = ((long)k * NY + j) * NX + i;
            if (pass == 0) {
              ++cnt[g + 1];
            } else {
              celem[fill[g]] = e;
              cw[fill[g]++] = (double)o / ((double)box2(0, i) * box2(1, j) * box2(2, k));
            }
          }
    }
    if (pass == 0) {
      for (long g = 0; g < n_gn; ++g) cnt[g + 1] += cnt[g];
      celem.resize(cnt[n_gn]);
      cw.resize(cnt[n_gn]);
      fill.assign(cnt.begin(), cnt.end() - 1);
    }
  }
  // each grid node: the first element whose closed box holds it
  std::vector<int32_t> gnode(8 * n_gn, -1);
  std::vector<float> gw(8 * n_gn, 0.f);
  for (int e = 0; e < ne; ++e) {
    const int h = elem_geom(e, p, vert);
    const int gi0 = (p[0] + cell - 1) / cell, gi1 = (p[0] + h) / cell;
    const int gj0 = (p[1] + cell - 1) / cell, gj1 = (p[1] + h) / cell;
    const int gk0 = (p[2] + cell - 1) / cell, gk1 = (p[2] + h) / cell;
    for (int k = gk0; k <= gk1; ++k)
      for (int j = gj0; j <= gj1; ++j)
        for (int i = gi0; i <= gi1; ++i) {
          const long g = ((long)k * NY + j) * NX + i;
          if (gnode[8 * g] >= 0) continue;
          const double tx = (double)(i * cell - p[0]) / h, ty = (double)(j * cell - p[1]) / h,
                       tz = (double)(k * cell - p[2]) / h;
          for (int a = 0; a < 8; ++a) {
            gnode[8 * g + a] = vert[a];
            gw[8 * g + a] = (float)(((a & 1) ? tx : 1.0 - tx) * (((a >> 1) & 1) ? ty : 1.0 - ty) *
                                    ((a >> 2) ? tz : 1.0 - tz));
          }
        }
  }
  for (long g = 0; g < n_gn; ++g)
    if (gnode[8 * g] < 0) return ctx->fail(AMRTO_EINVAL, "grid: a grid node lies outside the mesh");
  auto up = [&](auto*& dst, const auto& v) -> hipError_t {
    if (dst) (void)hipFree(dst);
    dst = nullptr;
    const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(v[0]);
    hipError_t err = hipMalloc((void**)&dst, bytes);
    if (err == hipSuccess && !v.empty()) err = hipMemcpy(dst, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice);
    return err;
  };
  ctx->grid_cell = 0;
  AMRTO_HIP(up(ctx->d_cell_ptr, cnt));
  AMRTO_HIP(up(ctx->d_cell_elem, celem));
  AMRTO_HIP(up(ctx->d_cell_w, cw));
  AMRTO_HIP(up(ctx->d_gn_node, gnode));
  AMRTO_HIP(up(ctx->d_gn_w, gw));
  if (!ctx->uniform && !ctx->d_node_xyz) AMRTO_HIP(up(ctx->d_node_xyz, ctx->h_node_xyz));
  ctx->grid_cell = cell;
  return AMRTO_OK;
}

int amrto_grid_from_mesh(amrto_ctx* ctx, int32_t cell, const double* rho, const double* u, const double* u_ref,
                         double u_scale, float* rho_grid, float* u_grid) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_grid_from_mesh: no mesh");
  AMRTO_HIP(hipSetDevice(ctx->device));
  int rc = grid_maps(ctx, cell);
  if (rc) return rc;
  const long ngn = (long)(ctx->nx / cell + 1) * (ctx->ny / cell + 1) * (ctx->nz / cell + 1);
  if (rho && rho_grid)
    hipLaunchKernelGGL(k_grid_density, dim3((ngn + 255) / 256), dim3(256), 0, ctx->stream, rho, ctx->d_cell_ptr,
                       ctx->d_cell_elem, ctx->d_cell_w, (int)ngn, rho_grid);
  if (u && u_grid)
    hipLaunchKernelGGL(k_grid_sample, dim3((3 * ngn + 255) / 256), dim3(256), 0, ctx->stream, u, u_ref,
                       ctx->d_gn_node, ctx->d_gn_w, ngn, u_scale, u_grid);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_grid_to_mesh(amrto_ctx* ctx, int32_t cell, const float* u_grid, double scale, double* u) {
  if (!ctx || !u_grid || !u) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_grid_to_mesh: no mesh");
  AMRTO_HIP(hipSetDevice(ctx->device));
  int rc = grid_maps(ctx, cell);
  if (rc) return rc;
  hipLaunchKernelGGL(k_grid_interp, dim3((ctx->n_nodes + 255) / 256), dim3(256), 0, ctx->stream, u_grid,
                     ctx->uniform ? nullptr : ctx->d_node_xyz, ctx->n_nodes, cell, ctx->nx / cell, ctx->ny / cell,
                     ctx->nz / cell, scale, u, ctx->nx + 1, ctx->ny + 1);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

}  // extern "C"
