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
#include <algorithm>
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

// ------------------------------------------------------------------ Gram matrix, octree + affine space
// Regions met by a chunk: mask[2c] = regions of its regular table nodes (the
// columns whose field is nonzero somewhere in the chunk's node table),
// mask[2c + 1] = regions of its owned regular nodes (the rows it adds to).
__global__ __launch_bounds__(256) void k_gram_masks(ChunkArgs ca, const float4* __restrict__ geo,
                                                    uint32_t* __restrict__ mask) {
  __shared__ uint32_t m[2];
  const int c = blockIdx.x;
  if (c >= ca.n_chunks) return;
  if (threadIdx.x == 0) m[0] = m[1] = 0u;
  __syncthreads();
  const ChunkDims cd = chunk_dims(ca, c);
  const int t0 = cd.t0, nreg = cd.nreg, nown = cd.nown;
  uint32_t mt = 0, mo = 0;
  for (int t = threadIdx.x; t < nreg; t += blockDim.x) {
    const uint32_t bit = 1u << (__float_as_int(geo[ca.tab_node[t0 + t]].w) & 31);
    mt |= bit;
    if (t < nown) mo |= bit;
  }
  atomicOr(&m[0], mt);
  atomicOr(&m[1], mo);
  __syncthreads();
  if (threadIdx.x == 0) {
    mask[2 * c] = m[0];
    mask[2 * c + 1] = m[1];
  }
}

// value of affine field f (1, d_c, d_{c+1}, d_{c+2}) at offsets d for component c
__device__ __forceinline__ double affine_value(int f, int c, const double (&d)[3]) {
  return f == 0 ? 1.0 : d[(c + f - 1) % 3];
}

// E = Z^T A~ Z with one chunk per block.  For every column z_j (field f,
// region gj, component cc) whose region meets the chunk's node table, the
// block forms A~ z_j on its owned nodes exactly as the operator pass does
// (z_j generated from the node descriptors, hanging values interpolated,
// element products, P^T), then reduces Z^T (A~ z_j) over its owned regular
// nodes per row region (fixed order: per-thread sums, 16 partials per row,
// one sum per row).  The results go to 12 x 12 tiles (row region, column
// region) at the chunk's tile offset, rows i = f' 3 + c', columns f 3 + cc.
// The twelve columns of a region are split over `split` blocks per chunk
// (block b: chunk b mod n_chunks, columns (b / n_chunks) + split m), so that
// chunks met by many regions do not set the launch's length alone.
__global__ __launch_bounds__(256) void k_gram_chunks(ChunkArgs ca, BrickK<double> kc, const double* __restrict__ coef,
                                                     const uint8_t* __restrict__ fix, const float4* __restrict__ geo,
                                                     const uint32_t* __restrict__ mask,
                                                     const int32_t* __restrict__ tile_off, double* __restrict__ tiles,
                                                     int split) {
  __shared__ double xs[TAB_MAX * 3];
  __shared__ double ys[TAB_MAX * 3];
  __shared__ uint32_t trip_hm_s[TRIP_MAX];
  __shared__ double trip_w_s[TRIP_MAX];
  __shared__ int hbeg_s[TAB_MAX];
  __shared__ double zred[12][16];
  static_assert(TAB_MAX * 3 >= 12 * 256, "the row sums are staged in xs");
  const int tid = threadIdx.x, c = blockIdx.x % ca.n_chunks, col0 = blockIdx.x / ca.n_chunks;
  if (col0 >= split) return;
  const ChunkDims cd = chunk_dims(ca, c);
  const int n0 = cd.n0, nent = cd.nent, t0 = cd.t0, nt = cd.nt, h0 = cd.h0, nh = cd.nh;
  const int nown = cd.nown, nreg = cd.nreg;
  const uint32_t mt = mask[2 * c], mo = mask[2 * c + 1];
  if (!mt || !mo) return;  // no tiles
  const int nct = __popc(mt);
  double* tb = tiles + 144L * tile_off[c];
  constexpr int NPT = TAB_MAX / 256, EPT = ENT_MAX / 256;
  float4 gv[NPT];
  uint8_t fb[NPT];
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int t = tid + 256 * r;
    gv[r] = make_float4(0.f, 0.f, 0.f, 0.f);
    fb[r] = 0;
    if (t < nreg) {
      const int g = ca.tab_node[t0 + t];
      gv[r] = geo[g];
      fb[r] = fix[g];
    }
  }
  uint4 lvp[EPT];
  double cep[EPT];
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const int en = tid + 256 * r;
    lvp[r] = en < nent ? *reinterpret_cast<const uint4*>(ca.ent_loc + 8L * (n0 + en)) : make_uint4(0, 0, 0, 0);
    cep[r] = en < nent ? coef[ca.ent_elem[n0 + en]] : 0.0;
  }
  for (int k = tid; k < nh; k += 256) {
    trip_hm_s[k] = ca.trip_hm[h0 + k];
    trip_w_s[k] = ca.trip_w[h0 + k];
  }
  for (int t = nreg + tid; t < nt; t += 256) hbeg_s[t - nreg] = ca.tab_hbeg[t0 + t];
  int jc = 0;  // column region rank
  for (uint32_t mj = mt; mj; mj &= mj - 1, ++jc) {
    const int gj = __ffs((int)mj) - 1;
    for (int col = col0; col < 12; col += split) {
      const int f = col / 3, cc = col % 3;
      // z_j on the regular table nodes (zero on supported components)
#pragma unroll
      for (int r = 0; r < NPT; ++r) {
        const int t = tid + 256 * r;
        if (t < nreg) {
          const int w = __float_as_int(gv[r].w);
          const double d[3] = {(double)gv[r].x, (double)gv[r].y, (double)gv[r].z};
          const bool on = (w & 0xff) == gj && !((w >> (8 + cc)) & 1);
#pragma unroll
          for (int c3 = 0; c3 < 3; ++c3) xs[3 * t + c3] = (on && c3 == cc) ? affine_value(f, cc, d) : 0.0;
        }
      }
      for (int i = tid; i < nt * 3; i += 256) ys[i] = 0.0;
      __syncthreads();
      for (int i = tid; i < (nt - nreg) * 3; i += 256) {  // hanging values from their masters
        const int t = nreg + i / 3, comp = i % 3;
        const int kb = hbeg_s[t - nreg], ke = t + 1 < nt ? hbeg_s[t + 1 - nreg] : nh;
        double v = 0.0;
        for (int k = kb; k < ke; ++k) v += trip_w_s[k] * xs[(trip_hm_s[k] & 0xffff) * 3 + comp];
        xs[t * 3 + comp] = v;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < EPT; ++r) {
        const int en = tid + 256 * r;
        const bool ev = en < nent;
        if (!ev && !ca.det) break;  // deterministic mode: the waves take turns over whole elements
        auto elem = [&]() {
          if (!ev) return;
          int loc[8];
          const uint4 lv = lvp[r];
          loc[0] = lv.x & 0xffff; loc[1] = lv.x >> 16; loc[2] = lv.y & 0xffff; loc[3] = lv.y >> 16;
          loc[4] = lv.z & 0xffff; loc[5] = lv.z >> 16; loc[6] = lv.w & 0xffff; loc[7] = lv.w >> 16;
          double u[24], out[24], ks[8];
#pragma unroll
          for (int aa = 0; aa < 8; ++aa) {
            u[3 * aa + 0] = xs[loc[aa] * 3 + 0];
            u[3 * aa + 1] = xs[loc[aa] * 3 + 1];
            u[3 * aa + 2] = xs[loc[aa] * 3 + 2];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) ks[q] = cep[r] * kc.c[q];
          contract_brick<double>(ks, u, out);
#pragma unroll
          for (int aa = 0; aa < 8; ++aa) {
            atomicAdd(&ys[loc[aa] * 3 + 0], out[3 * aa + 0]);
            atomicAdd(&ys[loc[aa] * 3 + 1], out[3 * aa + 1]);
            atomicAdd(&ys[loc[aa] * 3 + 2], out[3 * aa + 2]);
          }
        };
        if (ca.det) wave_turns(elem);
        else elem();
      }
      __syncthreads();
      // y_m += w_hm y_h; deterministic mode: wave 0 alone
      for (int i = ca.det ? (tid < 64 ? tid : nh * 3) : tid; i < nh * 3; i += ca.det ? 64 : 256) {
        const int k = i / 3, comp = i % 3;
        const uint32_t hm = trip_hm_s[k];
        atomicAdd(&ys[(hm & 0xffff) * 3 + comp], trip_w_s[k] * ys[(hm >> 16) * 3 + comp]);
      }
      __syncthreads();
      // rows: Z^T y over the owned regular nodes, one row region at a time
      int ic = 0;
      for (uint32_t mi = mo; mi; mi &= mi - 1, ++ic) {
        const int gi = __ffs((int)mi) - 1;
        double s[12];
#pragma unroll
        for (int u = 0; u < 12; ++u) s[u] = 0.0;
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
          const int t = tid + 256 * r;
          const int w = __float_as_int(gv[r].w);
          if (t < nown && (w & 0xff) == gi) {
            const double d[3] = {(double)gv[r].x, (double)gv[r].y, (double)gv[r].z};
#pragma unroll
            for (int c3 = 0; c3 < 3; ++c3) {
              const double y = ((w >> (8 + c3)) & 1) ? 0.0 : ys[t * 3 + c3];
#pragma unroll
              for (int f2 = 0; f2 < 4; ++f2) s[f2 * 3 + c3] += affine_value(f2, c3, d) * y;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < 12; ++u) xs[u * 256 + tid] = s[u];
        __syncthreads();
        if (tid < 192) {
          const int u = tid >> 4, sub = tid & 15;
          double v = 0.0;
#pragma unroll
          for (int i = 0; i < 16; ++i) v += xs[u * 256 + i * 16 + sub];
          zred[u][sub] = v;
        }
        __syncthreads();
        if (tid < 12) {
          double v = 0.0;
#pragma unroll
          for (int i = 0; i < 16; ++i) v += zred[tid][i];
          tb[(long)(ic * nct + jc) * 144 + tid * 12 + col] = v;
        }
      }
      __syncthreads();  // xs and zred are rewritten by the next column
    }
  }
}

// E tile of region pair p = gi R + gj: the sum of its block tiles in block
// order (pair_tile lists tile indices per pair), or zero.  144 threads.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ tiles,
                                                     const int32_t* __restrict__ pair_ptr,
                                                     const int32_t* __restrict__ pair_tile, int R,
                                                     double* __restrict__ E) {
  const int p = blockIdx.x, gi = p / R, gj = p % R, u = threadIdx.x;
  if (u >= 144) return;
  double v = 0.0;
  for (int q = pair_ptr[p]; q < pair_ptr[p + 1]; ++q) v += tiles[144L * pair_tile[q] + u];
  const int row = u / 12, col = u % 12;
  const int i = ((row / 3) * R + gi) * 3 + row % 3, j = ((col / 3) * R + gj) * 3 + col % 3;
  E[(long)i * (12 * R) + j] = v;
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
  // inverse of the active block as Li^T Li with Li = L^-1, both built by
  // rows (contiguous inner loops): row i of Li is (e_i - sum_{l<i} L_il Li_l) / L_ii
  std::vector<double> Li((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) {
    double* ri = Li.data() + (size_t)i * m;
    ri[i] = 1.0;
    for (int l = 0; l < i; ++l) {
      const double a = L[(size_t)i * k + l];
      if (a == 0.0) continue;
      const double* rl = Li.data() + (size_t)l * m;
      for (int j = 0; j <= l; ++j) ri[j] -= a * rl[j];
    }
    const double d = 1.0 / L[(size_t)i * k + i];
    for (int j = 0; j <= i; ++j) ri[j] *= d;
  }
  // (Li^T Li)_ab = sum_{l >= max(a, b)} Li_la Li_lb: lower triangle by rank-one
  // updates with row l, then mirrored
  std::vector<double> S((size_t)m * m, 0.0);
  for (int l = 0; l < m; ++l) {
    const double* rl = Li.data() + (size_t)l * m;
    for (int a = 0; a <= l; ++a) {
      const double ra = rl[a];
      if (ra == 0.0) continue;
      double* sa = S.data() + (size_t)a * m;
      for (int b = 0; b <= a; ++b) sa[b] += ra * rl[b];
    }
  }
  for (int a = 0; a < m; ++a)
    for (int b = 0; b <= a; ++b) {
      const double v = S[(size_t)a * m + b];
      inv[(size_t)act[a] * k + act[b]] = v;
      inv[(size_t)act[b] * k + act[a]] = v;
    }
  return m;
}

// E = Z^T A~ Z for the affine space on an octree mesh (k = 12 R) into E_dev:
// region masks per chunk, tile offsets and per-pair tile lists on the host,
// then k_gram_chunks and k_gram_reduce.
static int gram_chunks(amrto_ctx* ctx, int R, double* E_dev) {
  const int nc = ctx->n_chunks;
  if ((long)2 * nc > ctx->gram_mask_cap) {
    if (ctx->d_gram_mask) (void)hipFree(ctx->d_gram_mask);
    ctx->d_gram_mask = nullptr;
    ctx->gram_mask_cap = 0;
    AMRTO_HIP(hipMalloc((void**)&ctx->d_gram_mask, 2L * nc * sizeof(uint32_t)));
    ctx->gram_mask_cap = 2L * nc;
  }
  hipLaunchKernelGGL(k_gram_masks, dim3(nc), dim3(256), 0, ctx->stream, chunk_args(ctx),
                     (const float4*)ctx->d_cgeo, ctx->d_gram_mask);
  std::vector<uint32_t> mask(2L * nc);
  AMRTO_HIP(hipMemcpyAsync(mask.data(), ctx->d_gram_mask, mask.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                           ctx->stream));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  // tiles of chunk c: (row region, column region) over its owned-row and
  // column regions, row-region major, both ascending
  std::vector<int32_t> toff(nc + 1, 0), cnt(R * R, 0);
  for (int c = 0; c < nc; ++c) {
    const uint32_t mt = mask[2 * c], mo = mask[2 * c + 1];
    const int n = (mt && mo) ? __builtin_popcount(mt) * __builtin_popcount(mo) : 0;
    toff[c + 1] = toff[c] + n;
    if (!n) continue;
    for (uint32_t mi = mo; mi; mi &= mi - 1)
      for (uint32_t mj = mt; mj; mj &= mj - 1) ++cnt[__builtin_ctz(mi) * R + __builtin_ctz(mj)];
  }
  const int ntile = toff[nc];
  std::vector<int32_t> pptr(R * R + 1, 0), ptile(ntile);
  for (int p = 0; p < R * R; ++p) pptr[p + 1] = pptr[p] + cnt[p];
  std::vector<int32_t> fill(pptr.begin(), pptr.end() - 1);
  for (int c = 0; c < nc; ++c) {
    const uint32_t mt = mask[2 * c], mo = mask[2 * c + 1];
    if (!mt || !mo) continue;
    const int nct = __builtin_popcount(mt);
    int ic = 0;
    for (uint32_t mi = mo; mi; mi &= mi - 1, ++ic) {
      int jc = 0;
      for (uint32_t mj = mt; mj; mj &= mj - 1, ++jc)
        ptile[fill[__builtin_ctz(mi) * R + __builtin_ctz(mj)]++] = toff[c] + ic * nct + jc;
    }
  }
  // one scratch buffer: tiles (doubles), then tile offsets and pair lists
  const size_t n_int = (size_t)(nc + 1) + (R * R + 1) + ntile;
  const size_t bytes = 144 * sizeof(double) * (size_t)ntile + n_int * sizeof(int32_t);
  if (bytes > ctx->gram_cap) {
    if (ctx->d_gram) (void)hipFree(ctx->d_gram);
    ctx->d_gram = nullptr;
    ctx->gram_cap = 0;
    AMRTO_HIP(hipMalloc(&ctx->d_gram, bytes));
    ctx->gram_cap = bytes;
  }
  double* tiles = (double*)ctx->d_gram;
  int32_t* d_toff = (int32_t*)(tiles + 144L * ntile);
  int32_t* d_pptr = d_toff + nc + 1;
  int32_t* d_ptile = d_pptr + R * R + 1;
  AMRTO_HIP(hipMemcpyAsync(d_toff, toff.data(), toff.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  AMRTO_HIP(hipMemcpyAsync(d_pptr, pptr.data(), pptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  if (ntile)
    AMRTO_HIP(hipMemcpyAsync(d_ptile, ptile.data(), ptile.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                             ctx->stream));
  constexpr int GRAM_SPLIT = 12;  // one column of each region per block
  hipLaunchKernelGGL(k_gram_chunks, dim3(nc * GRAM_SPLIT), dim3(256), 0, ctx->stream, chunk_args(ctx),
                     brick_k<double>(ctx), (const double*)ctx->d_coef, (const uint8_t*)ctx->d_fix,
                     (const float4*)ctx->d_cgeo, (const uint32_t*)ctx->d_gram_mask, (const int32_t*)d_toff, tiles,
                     GRAM_SPLIT);
  hipLaunchKernelGGL(k_gram_reduce, dim3(R * R), dim3(256), 0, ctx->stream, (const double*)tiles,
                     (const int32_t*)d_pptr, (const int32_t*)d_ptile, R, E_dev);
  AMRTO_HIP(hipGetLastError());
  // the host vectors above are read by the copies: wait before they go
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  return AMRTO_OK;
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
  if (!ctx->uniform && ctx->coarse_affine_only) {
    int rc = gram_chunks(ctx, R, ctx->d_cinv);
    if (rc) return rc;
  }
  for (int j = 0; !(!ctx->uniform && ctx->coarse_affine_only) && j < k; ++j) {
    const int c = j % 3, g = (j / 3) % R, f = j / (3 * R);
    hipLaunchKernelGGL(k_make_column, dim3(g1), dim3(256), 0, ctx->stream, ctx->d_cf, n3, ctx->d_region, f, g, c,
                       ctx->d_z);
    int rc = apply_stop(ctx, ctx->d_z, ctx->d_q, AMRTO_FP64, nullptr);
    if (rc) return rc;
    rc = launch_zt(ctx, ctx->d_q);
    if (rc) return rc;
    hipLaunchKernelGGL(k_gram_column, dim3(k), dim3(256), 0, ctx->stream, ctx->d_cpart, k, j, ctx->d_cinv);
  }
  std::vector<double>& E = ctx->h_gram;
  E.assign((long)k * k, 0.0);
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

int amrto_coarse_gram(amrto_ctx* ctx, double* E_host, int64_t cap, int32_t* k) {
  if (!ctx) return AMRTO_EINVAL;
  if (ctx->coarse_k <= 0) return ctx->fail(AMRTO_ESTATE, "amrto_coarse_gram: no coarse space set");
  const long kk = ctx->coarse_k;
  if (!E_host || !k || cap < kk * kk) return ctx->fail(AMRTO_EINVAL, "amrto_coarse_gram: need a k x k buffer");
  std::copy(ctx->h_gram.begin(), ctx->h_gram.begin() + kk * kk, E_host);
  *k = (int32_t)kk;
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
