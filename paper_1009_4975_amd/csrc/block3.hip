// Block-Jacobi preconditioner: the 3x3 node blocks of A~ (all three
// displacement components of a node), inverted per node.  The diagonal
// rescaling of the paper (Sec. 5) is its scalar special case; the blocks also
// capture the coupling of a node's components, which the scalar form drops.
//
// Block of node n: sum over its elements of c_e K0[a, a] (the 3x3 block of
// the element's local vertex a), with hanging vertices expanded through their
// masters as in the exact diagonal (pairs of expansions that share the
// master n).  Rows and columns of supported components are replaced by the
// identity (A~ = F T^T K T F + I - F), hanging nodes get the identity block.
// Stored per node as the six entries of the symmetric inverse
// (xx, yy, zz, xy, xz, yz).
#include <cmath>
#include <type_traits>

#include "kernels.h"

namespace amrto {

// identity rows/columns of supported components, then the symmetric inverse
// (cofactors, FP64); out: 9 entries of the masked block (INV false) or the 6
// entries of its inverse (INV true)
template <bool INV>
__device__ __forceinline__ void finish_block(double (&B)[3][3], uint32_t fixbits, double* __restrict__ out) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if ((fixbits >> c) & 1) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        B[c][d] = 0.0;
        B[d][c] = 0.0;
      }
      B[c][c] = 1.0;
    }
  if (!INV) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) out[3 * c + d] = B[c][d];
    return;
  }
  const double a = B[0][0], b = B[1][1], c = B[2][2];
  const double d = 0.5 * (B[0][1] + B[1][0]), e = 0.5 * (B[0][2] + B[2][0]), f = 0.5 * (B[1][2] + B[2][1]);
  const double ca = b * c - f * f, cb = a * c - e * e, cc = a * b - d * d;
  const double cd = e * f - d * c, ce = d * f - e * b, cf = d * e - a * f;
  const double det = a * ca + d * cd + e * ce;
  const double s = 1.0 / det;
  out[0] = ca * s;
  out[1] = cb * s;
  out[2] = cc * s;
  out[3] = cd * s;
  out[4] = ce * s;
  out[5] = cf * s;
}

// uniform brick: one thread per node, the (up to) eight elements around it
template <bool INV>
__global__ __launch_bounds__(256) void k_block_uniform(const double* __restrict__ coef,
                                                       const uint8_t* __restrict__ fix,
                                                       const double* __restrict__ K0, double* __restrict__ out,
                                                       int nx, int ny, int nz) {
  const long n = (long)(nx + 1) * (ny + 1) * (nz + 1);
  const long node = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (node >= n) return;
  const int gx = node % (nx + 1);
  const int gy = (node / (nx + 1)) % (ny + 1);
  const int gz = node / ((long)(nx + 1) * (ny + 1));
  double B[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int dz = -1; dz <= 0; ++dz)
    for (int dy = -1; dy <= 0; ++dy)
      for (int dx = -1; dx <= 0; ++dx) {
        const int ex = gx + dx, ey = gy + dy, ez = gz + dz;
        if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
        const double ce = coef[ex + (long)nx * (ey + (long)ny * ez)];
        const int a = -dx + 2 * (-dy) + 4 * (-dz);  // local vertex of this node
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int d = 0; d < 3; ++d) B[c][d] += ce * K0[(3 * a + c) * 24 + 3 * a + d];
      }
  finish_block<INV>(B, fix[node], out + (INV ? 6 : 9) * node);
}

// octree: per chunk, as the exact diagonal (k_diag_chunks) with the six
// component pairs of the symmetric block (00, 11, 22, 01, 02, 12); owned rows
// are finished and written
template <bool INV>
__global__ __launch_bounds__(512) void k_block_chunks(const double* __restrict__ coef,
                                                      const uint8_t* __restrict__ fix,
                                                      const double* __restrict__ K0, double* __restrict__ out,
                                                      ChunkArgs ca) {
  __shared__ double ds[TAB_MAX * 6];
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
  for (int i = tid; i < nt * 6; i += DT) ds[i] = 0.0;
  // the chunk's hanging triples and per-entry triple ranges, and K0, in LDS
  for (int k = tid; k < nh; k += DT) {
    trip_hm_s[k] = ca.trip_hm[h0 + k];
    trip_w_s[k] = ca.trip_w[h0 + k];
  }
  for (int t = nreg + tid; t < nt; t += DT) hbeg_s[t - nreg] = ca.tab_hbeg[t0 + t];
  for (int i = tid; i < 576; i += DT) K0s[i] = K0[i];
  __syncthreads();
  auto range = [&](int l, int& kb, int& ke) {
    if (l < nreg) {
      kb = -1;
      ke = 0;
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
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int bb = 0; bb < 8; ++bb) {
          int kb, kbe;
          range(loc[bb], kb, kbe);
          for (int j = kb; j < (kb < 0 ? 0 : kbe); ++j) {
            const int mb = kb < 0 ? loc[bb] : (int)(trip_hm_s[j] & 0xffff);
            if (mb != ma) continue;
            const double w = wa * (kb < 0 ? 1.0 : trip_w_s[j]);
            const double* kr = K0s + 3 * aa * 24 + 3 * bb;
            acc[0] += w * kr[0];
            acc[1] += w * kr[24 + 1];
            acc[2] += w * kr[48 + 2];
            acc[3] += w * kr[1];
            acc[4] += w * kr[2];
            acc[5] += w * kr[24 + 2];
          }
        }
        for (int q = 0; q < 6; ++q) atomicAdd(&ds[ma * 6 + q], ce * acc[q]);
      }
    }
    };
    if (ca.det) wave_turns(item);
    else item();
  }
  __syncthreads();
  for (int t = tid; t < nown + nhown; t += DT) {
    const bool hang = t >= nown;
    const int tt = hang ? nreg + (t - nown) : t;
    const long node = ca.tab_node[t0 + tt];
    double B[3][3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) {
        // pair (cc, dd) in the order 00, 11, 22, 01, 02, 12
        const int q = cc == dd ? cc : (cc + dd + 2);
        B[cc][dd] = hang ? (cc == dd ? 1.0 : 0.0) : ds[tt * 6 + q];
      }
    finish_block<INV>(B, hang ? 0u : (uint32_t)fix[node], out + (INV ? 6 : 9) * node);
  }
}

// r = b - q (q may be NULL), z = B^-1 r; partials r.z, r.r, b.b (one thread per node)
template <typename VT, typename BT>
__global__ __launch_bounds__(256) void k_init_b3(const BT* __restrict__ b, const BT* __restrict__ q,
                                                 VT* __restrict__ r, VT* __restrict__ z,
                                                 const VT* __restrict__ binv, long nn, double* __restrict__ part) {
  __shared__ double sh[16];
  double rz = 0, rr = 0, bb = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
    VT rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const BT bi = b[3 * i + c];
      rv[c] = (VT)(q ? (BT)(bi - q[3 * i + c]) : bi);
      bb += (double)bi * (double)bi;
    }
    block_apply<VT>(binv + 6 * i, rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[3 * i + c] = rv[c];
      z[3 * i + c] = zv[c];
      rz += (double)rv[c] * (double)zv[c];
      rr += (double)rv[c] * (double)rv[c];
    }
  }
  block_sum2(rz, rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rz;
    part[RED_BLOCKS + blockIdx.x] = rr;
    part[2 * RED_BLOCKS + blockIdx.x] = bb;
  }
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; z = B^-1 r; partials r.z, r.r
template <typename VT>
__global__ __launch_bounds__(256) void k_cg_update_b3(VT* __restrict__ x, VT* __restrict__ r,
                                                      const VT* __restrict__ p, const VT* __restrict__ q,
                                                      const VT* __restrict__ binv, VT* __restrict__ z, long nn,
                                                      const double* __restrict__ part_pq, int n_pq,
                                                      double* __restrict__ scal, int it,
                                                      double* __restrict__ part) {
  if (scal[S_DONE] != 0.0) return;
  __shared__ double sh[16];
  const double pq = sum_partials(part_pq, n_pq, sh);
  const double rz0 = scal[S_RZ0 + (it & 1)];
  if (!(pq > 0.0) || !(pq < 1e300) || !(rz0 == rz0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_DONE] = 2.0;
    return;
  }
  const VT alpha = (VT)(rz0 / pq);
  double srz = 0.0, srr = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nn; i += (long)gridDim.x * blockDim.x) {
    VT rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[3 * i + c] += alpha * p[3 * i + c];
      rv[c] = r[3 * i + c] - alpha * q[3 * i + c];
    }
    block_apply<VT>(binv + 6 * i, rv, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[3 * i + c] = rv[c];
      z[3 * i + c] = zv[c];
      srz += (double)rv[c] * (double)zv[c];
      srr += (double)rv[c] * (double)rv[c];
    }
  }
  block_sum2(srz, srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[RED_BLOCKS + blockIdx.x] = srr;
  }
}

// ------------------------------------------------------------------ host
template <bool INV>
static int launch_blocks(amrto_ctx* ctx, double* out) {
  if (ctx->uniform) {
    const long n = ctx->n_nodes;
    hipLaunchKernelGGL(k_block_uniform<INV>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_coef,
                       ctx->d_fix, ctx->d_K0, out, ctx->nx, ctx->ny, ctx->nz);
  } else {
    hipLaunchKernelGGL(k_block_chunks<INV>, dim3(ctx->n_chunks), dim3(512), 0, ctx->stream, ctx->d_coef, ctx->d_fix,
                       ctx->d_K0, out, chunk_args(ctx));
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

__global__ void k_to_float6(const double* __restrict__ a, float* __restrict__ b, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// inverse node blocks for the current density (computed once per density),
// with the FP32 copy used by mixed-precision recurrences
int block3_setup(amrto_ctx* ctx) {
  if (ctx->binv_valid) return AMRTO_OK;
  int rc = launch_blocks<true>(ctx, ctx->d_binv);
  if (rc) return rc;
  const long n6 = 6L * ctx->n_nodes;
  hipLaunchKernelGGL(k_to_float6, dim3((n6 + 255) / 256), dim3(256), 0, ctx->stream, (const double*)ctx->d_binv,
                     ctx->d_binv_f, n6);
  AMRTO_HIP(hipGetLastError());
  ctx->binv_valid = true;
  return AMRTO_OK;
}

template <typename VT, typename BT>
int block3_init(amrto_ctx* ctx, const BT* b, const BT* q, VT* r, VT* z) {
  const VT* binv;
  if constexpr (std::is_same<VT, double>::value) binv = ctx->d_binv;
  else binv = ctx->d_binv_f;
  hipLaunchKernelGGL((k_init_b3<VT, BT>), dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, b, q, r, z, binv,
                     (long)ctx->n_nodes, ctx->d_part);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}
template int block3_init<double, double>(amrto_ctx*, const double*, const double*, double*, double*);
template int block3_init<float, double>(amrto_ctx*, const double*, const double*, float*, float*);

template <typename VT>
int block3_update(amrto_ctx* ctx, VT* x, VT* r, const VT* p, const VT* q, VT* z, int it) {
  const VT* binv;
  if constexpr (std::is_same<VT, double>::value) binv = ctx->d_binv;
  else binv = ctx->d_binv_f;
  hipLaunchKernelGGL(k_cg_update_b3<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, x, r, p, q, binv, z,
                     (long)ctx->n_nodes, (const double*)ctx->d_partpq, ctx->n_partpq, ctx->d_scal, it,
                     ctx->d_part);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}
template int block3_update<double>(amrto_ctx*, double*, double*, const double*, const double*, double*, int);
template int block3_update<float>(amrto_ctx*, float*, float*, const float*, const float*, float*, int);

}  // namespace amrto

using namespace amrto;

extern "C" int amrto_get_block_diag(amrto_ctx* ctx, double* blocks) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, "amrto_get_block_diag: density not set");
  if (!blocks) return ctx->fail(AMRTO_EINVAL, "amrto_get_block_diag: NULL buffer");
  AMRTO_HIP(hipSetDevice(ctx->device));
  return launch_blocks<false>(ctx, blocks);
}
