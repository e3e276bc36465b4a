// Jacobi-preconditioned conjugate gradients with one global reduction per
// iteration on octree meshes (the recurrences of Chronopoulos and Gear for
// CG, applied to A~ with M = D^-1):
//
//   u_j = M r_j,  w_j = A~ u_j,  gamma_j = r_j.u_j,  delta_j = w_j.u_j
//   beta_j  = gamma_j / gamma_{j-1}                       (beta_0 = 0)
//   alpha_j = gamma_j / (delta_j - beta_j gamma_j / alpha_{j-1})
//   p_j = u_j + beta_j p_{j-1},  s_j = w_j + beta_j s_{j-1}   (= A~ p_j)
//   x_{j+1} = x_j + alpha_j p_j,  r_{j+1} = r_j - alpha_j s_j
//
// In exact arithmetic these are the iterates of the two-reduction form in
// pcg.hip.  One pass per iteration: every chunk computes u_{j+1} for all its
// table nodes (owned and halo) from r_j, w_j, s_{j-1} of the previous pass,
// applies the operator, and writes x, p, s, r, w of its owned nodes plus the
// partial sums of gamma_{j+1}, delta_{j+1} and r.r.  r, w and s alternate
// between two buffers (halo reads of the old values never meet the new ones).
#include "kernels.h"

namespace amrto {

template <typename VT>
struct Cg1Vecs {
  VT* x;
  VT* p;
  const VT* r_in;
  const VT* w_in;
  const VT* s_in;
  VT* r_out;
  VT* w_out;
  VT* s_out;
  const VT* dinv;
  const VT* coef;
  const uint8_t* fix;
};

struct Cg1Args {
  double* scal;
  const double* part_in;  // gamma, delta, r.r partials of the previous pass (stride n_part)
  double* part_out;       // this pass's partials (stride n_part)
  int n_part;             // partials per quantity (the pass's grid size)
  int it;
  double tol2;
};

__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  if (lane == 0) {
    sh[w] = a;
    sh[nw + w] = b;
    sh[2 * nw + w] = c;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0, sc = 0.0;
  for (int i = 0; i < nw; ++i) {
    sa += sh[i];
    sb += sh[nw + i];
    sc += sh[2 * nw + i];
  }
  __syncthreads();
  a = sa;
  b = sb;
  c = sc;
}

// gamma_0 = r.u, delta_0 = w.u, r.r with the pass layout (n_part blocks)
template <typename VT>
__global__ __launch_bounds__(256) void k_cg1_dots(const VT* __restrict__ r, const VT* __restrict__ u,
                                                  const VT* __restrict__ w, long n, double* __restrict__ part) {
  __shared__ double sh[16];
  double g = 0.0, d = 0.0, rr = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double ri = r[i], ui = u[i];
    g += ri * ui;
    d += (double)w[i] * ui;
    rr += ri * ri;
  }
  block_sum3(g, d, rr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = g;
    part[gridDim.x + blockIdx.x] = d;
    part[2 * gridDim.x + blockIdx.x] = rr;
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_cg1_chunks(Cg1Vecs<VT> v, ChunkArgs ca, BrickK<VT> kc, Cg1Args g) {
  __shared__ VT xs[TAB_MAX * 3];
  __shared__ double ys[TAB_MAX * 3];
  __shared__ double sh[16];
  __shared__ uint32_t trip_hm_s[TRIP_MAX];
  __shared__ double trip_w_s[TRIP_MAX];
  __shared__ int hbeg_s[TAB_MAX];
  const int tid = threadIdx.x;
  const int c = xcd_remap(blockIdx.x, gridDim.x);
  const bool have = c < ca.n_chunks;
  const int cc = have ? c : 0;
  const ChunkDims cd = chunk_dims(ca, cc, have);
  const int n0 = cd.n0, nent = cd.nent, t0 = cd.t0, nt = cd.nt, h0 = cd.h0, nh = cd.nh;
  const int nown = cd.nown, nreg = cd.nreg, nhown = cd.nhown;
  const bool first = g.it == 0;
  // every index and vector value is requested before the reduction of the
  // previous pass's partials (which waits on memory), as in k_apply_chunks
  constexpr int NPT = TAB_MAX / 256;
  int gn[NPT];
  uint8_t fb[NPT];
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int t = tid + 256 * q;
    gn[q] = t < nt ? ca.tab_node[t0 + t] : -1;
  }
  constexpr int EPT = ENT_MAX / 256;
  uint4 lvp[EPT];
  int eel[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int en = tid + 256 * q;
    eel[q] = en < nent ? ca.ent_elem[n0 + en] : 0;
    lvp[q] = en < nent ? *reinterpret_cast<const uint4*>(ca.ent_loc + 8L * (n0 + en)) : make_uint4(0, 0, 0, 0);
  }
  for (int k = tid; k < nh; k += 256) {
    trip_hm_s[k] = ca.trip_hm[h0 + k];
    trip_w_s[k] = ca.trip_w[h0 + k];
  }
  for (int t = nreg + tid; t < nt; t += 256) hbeg_s[t - nreg] = ca.tab_hbeg[t0 + t];
  VT rv[NPT][3], wv[NPT][3], sv[NPT][3], dv[NPT][3], xv[NPT][3], pv[NPT][3];
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int t = tid + 256 * q;
    fb[q] = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      rv[q][k] = 0;
      wv[q][k] = 0;
      sv[q][k] = 0;
      dv[q][k] = 0;
      xv[q][k] = 0;
      pv[q][k] = 0;
    }
    if (t < nreg && gn[q] >= 0) {
      const long gi = 3L * gn[q];
      fb[q] = v.fix[gn[q]];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        rv[q][k] = v.r_in[gi + k];
        wv[q][k] = v.w_in[gi + k];
        if (!first) sv[q][k] = v.s_in[gi + k];
        dv[q][k] = v.dinv[gi + k];
      }
      if (t < nown) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          xv[q][k] = v.x[gi + k];
          if (!first) pv[q][k] = v.p[gi + k];
        }
      }
    }
  }
  VT cep[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) cep[q] = v.coef[eel[q]];
  // scalars of iteration j from the partials of the previous pass
  if (g.scal[S_DONE] != 0.0) return;
  double gam = 0.0, del = 0.0, rho = 0.0;
  for (int i = tid; i < g.n_part; i += 256) {
    gam += g.part_in[i];
    del += g.part_in[g.n_part + i];
    rho += g.part_in[2 * g.n_part + i];
  }
  block_sum3(gam, del, rho, sh);
  const bool lead = blockIdx.x == 0 && tid == 0;
  if (!(gam == gam) || !(del == del) || !(rho == rho) || rho > 1e300 || gam > 1e300) {
    if (lead) g.scal[S_DONE] = 2.0;
    return;
  }
  if (rho <= g.tol2 * g.scal[S_BB]) {
    if (lead) {
      g.scal[S_RR] = rho;
      g.scal[S_ITERS] = g.it;
      g.scal[S_DONE] = 1.0;
    }
    return;
  }
  double beta = 0.0, den = del;
  if (!first) {
    beta = gam / g.scal[S_RZ0 + ((g.it - 1) & 1)];
    den = del - beta * gam / g.scal[S_AL0 + ((g.it - 1) & 1)];
  }
  if (!(den > 0.0) || !(gam > 0.0)) {
    if (lead) g.scal[S_DONE] = 2.0;
    return;
  }
  const double alpha = gam / den;
  if (lead) {
    g.scal[S_RZ0 + (g.it & 1)] = gam;
    g.scal[S_AL0 + (g.it & 1)] = alpha;
    g.scal[S_RR] = rho;
    g.scal[S_ITERS] = g.it;
  }
  if (!have) {
    if (tid == 0) {
      g.part_out[blockIdx.x] = 0.0;
      g.part_out[g.n_part + blockIdx.x] = 0.0;
      g.part_out[2 * g.n_part + blockIdx.x] = 0.0;
    }
    return;
  }
  const VT va = (VT)alpha, vb = (VT)beta;
  // s_j, r_{j+1} and u_{j+1} = M r_{j+1} on every regular table node
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int t = tid + 256 * q;
    if (t < nreg) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const VT s = wv[q][k] + vb * sv[q][k];
        const VT r = rv[q][k] - va * s;
        sv[q][k] = s;
        wv[q][k] = r;  // wv now holds r_{j+1}
        xs[3 * t + k] = ((fb[q] >> k) & 1) ? (VT)0 : dv[q][k] * r;
      }
    }
  }
  for (int i = tid; i < nt * 3; i += 256) ys[i] = 0.0;
  __syncthreads();
  for (int i = tid; i < (nt - nreg) * 3; i += 256) {  // u_h = sum_m w_hm u_m  (Eq. (6))
    const int t = nreg + i / 3, comp = i % 3;
    const int kb = hbeg_s[t - nreg], ke = t + 1 < nt ? hbeg_s[t + 1 - nreg] : nh;
    double acc = 0.0;
    for (int k = kb; k < ke; ++k) acc += trip_w_s[k] * (double)xs[(trip_hm_s[k] & 0xffff) * 3 + comp];
    xs[t * 3 + comp] = (VT)acc;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int en = tid + 256 * q;
    const bool ev = en < nent;
    if (!ev && !ca.det) break;  // deterministic mode: the waves take turns over whole elements
    auto elem = [&]() {
      if (!ev) return;
      int loc[8];
      const uint4 lv = lvp[q];
      loc[0] = lv.x & 0xffff; loc[1] = lv.x >> 16; loc[2] = lv.y & 0xffff; loc[3] = lv.y >> 16;
      loc[4] = lv.z & 0xffff; loc[5] = lv.z >> 16; loc[6] = lv.w & 0xffff; loc[7] = lv.w >> 16;
      VT u[24], out[24];
#pragma unroll
      for (int aa = 0; aa < 8; ++aa) {
        u[3 * aa + 0] = xs[loc[aa] * 3 + 0];
        u[3 * aa + 1] = xs[loc[aa] * 3 + 1];
        u[3 * aa + 2] = xs[loc[aa] * 3 + 2];
      }
      VT ks[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) ks[k] = cep[q] * kc.c[k];
      contract_brick<VT>(ks, u, out);
#pragma unroll
      for (int aa = 0; aa < 8; ++aa) {
        atomicAdd(&ys[loc[aa] * 3 + 0], (double)out[3 * aa + 0]);
        atomicAdd(&ys[loc[aa] * 3 + 1], (double)out[3 * aa + 1]);
        atomicAdd(&ys[loc[aa] * 3 + 2], (double)out[3 * aa + 2]);
      }
    };
    if (ca.det) wave_turns(elem);
    else elem();
  }
  __syncthreads();
  // y_m += w_hm y_h  (P^T of Eq. (7)); deterministic mode: wave 0 alone
  for (int i = ca.det ? (tid < 64 ? tid : nh * 3) : tid; i < nh * 3; i += ca.det ? 64 : 256) {
    const int k = i / 3, comp = i % 3;
    const uint32_t hm = trip_hm_s[k];
    atomicAdd(&ys[(hm & 0xffff) * 3 + comp], trip_w_s[k] * ys[(hm >> 16) * 3 + comp]);
  }
  __syncthreads();
  double sg = 0.0, sd = 0.0, sr = 0.0;
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int t = tid + 256 * q;
    const bool own_reg = t < nown, own_hang = t >= nreg && t < nreg + nhown;
    if (!own_reg && !own_hang) continue;
    const long gi = 3L * gn[q];
    if (own_hang) {  // identity rows with zero right-hand side
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        v.p[gi + k] = 0;
        v.s_out[gi + k] = 0;
        v.r_out[gi + k] = 0;
        v.w_out[gi + k] = 0;
      }
      continue;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const bool fixed = (fb[q] >> k) & 1;
      const VT u1 = xs[t * 3 + k];
      const VT w1 = fixed ? (VT)0 : (VT)ys[t * 3 + k];
      const VT r1 = wv[q][k];
      const VT p = dv[q][k] * rv[q][k] + vb * pv[q][k];  // p_j = u_j + beta p_{j-1}
      v.x[gi + k] = xv[q][k] + va * p;
      v.p[gi + k] = p;
      v.s_out[gi + k] = sv[q][k];
      v.r_out[gi + k] = r1;
      v.w_out[gi + k] = w1;
      sg += (double)r1 * (double)u1;
      sd += (double)w1 * (double)u1;
      sr += (double)r1 * (double)r1;
    }
  }
  block_sum3(sg, sd, sr, sh);
  if (tid == 0) {
    g.part_out[blockIdx.x] = sg;
    g.part_out[g.n_part + blockIdx.x] = sd;
    g.part_out[2 * g.n_part + blockIdx.x] = sr;
  }
}

// ------------------------------------------------------------------ host
// the single-reduction form runs on octree meshes (chunk kernels)
bool cg1_available(const amrto_ctx* ctx) { return !ctx->uniform && ctx->d_cg1_r2 != nullptr; }

int cg1_parts(const amrto_ctx* ctx) { return ((ctx->n_chunks + 7) / 8) * 8; }

static Cg1Vecs<double> cg1_vecs(amrto_ctx* ctx, double* x, int it) {
  double* R[2] = {ctx->d_r, ctx->d_cg1_r2};
  double* W[2] = {ctx->d_cg1_w, ctx->d_cg1_w2};
  double* S[2] = {ctx->d_cg1_s, ctx->d_cg1_s2};
  const int a = it & 1, b = a ^ 1;
  return Cg1Vecs<double>{x, ctx->d_p, R[a], W[a], S[a], R[b], W[b], S[b], ctx->d_dinv, ctx->d_coef, ctx->d_fix};
}

// set-up after r_0 (in d_r) and u_0 (in d_z) are formed: w_0 = A~ u_0 and the
// partials of gamma_0, delta_0 and r_0.r_0
int cg1_init(amrto_ctx* ctx) {
  int rc = apply_stop(ctx, ctx->d_z, ctx->d_cg1_w, AMRTO_FP64, nullptr);
  if (rc) return rc;
  hipLaunchKernelGGL(k_cg1_dots<double>, dim3(cg1_parts(ctx)), dim3(256), 0, ctx->stream, (const double*)ctx->d_r,
                     (const double*)ctx->d_z, (const double*)ctx->d_cg1_w, 3L * ctx->n_nodes, ctx->d_cg1_part);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int cg1_enqueue(amrto_ctx* ctx, double* x, double tol2, int it0, int count) {
  const int np = cg1_parts(ctx);
  for (int it = it0; it < it0 + count; ++it) {
    Cg1Args g{ctx->d_scal, ctx->d_cg1_part + 3L * np * (it & 1), ctx->d_cg1_part + 3L * np * ((it & 1) ^ 1), np,
              it, tol2};
    hipLaunchKernelGGL(k_cg1_chunks<double>, dim3(np), dim3(256), 0, ctx->stream, cg1_vecs(ctx, x, it),
                       chunk_args(ctx), brick_k<double>(ctx), g);
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

}  // namespace amrto
