// Krylov subspace recycling across the systems of a design sequence (paper
// Sec. 5: an approximate invariant subspace for the smallest eigenvalues is
// taken from one solve's Krylov space and carried to the next system).
//
// A recorded PCG solve keeps its first m residuals r_j and the products
// r_j^T z_j, p_j^T A~ p_j (z_j = M^-1 r_j); it runs its usual kernels, the
// recording adds one copy per iteration.  Those coefficients give the
// Lanczos matrix T of the preconditioned operator (the CG/Lanczos
// correspondence; Lanczos vectors v_j = (-1)^j z_j / sqrt(r_j^T z_j)), whose
// smallest eigenpairs give Ritz vectors u = V y = M^-1 (sum_j c_j r_j): one
// preconditioner application per Ritz vector.  Before the next solve the
// Ritz vectors start it (the initial error's Galerkin projection onto them,
// amrto_energy_combine) or, combined with carried vectors by Rayleigh-Ritz
// for the pencil (A~, D) of the new system (D = diag A~), enter the coarse
// space of the two-level preconditioner.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.h"

namespace amrto {

constexpr int REC_MMAX = 256;   // recorded vectors
constexpr int COMB_MAX = 4096;  // coefficients of one combination (sources x outputs)
constexpr int RR_NMAX = 16;     // vectors of a Rayleigh-Ritz step
constexpr int GRAM_BLOCKS = 64;

struct VecSet {
  const double* base;  // contiguous: source j at base + j * stride
  long stride;
  const double* p[RR_NMAX];  // or explicit pointers (base == nullptr)
};
struct OutSet {
  double* p[RR_NMAX];
};

__device__ __forceinline__ const double* vs_get(const VecSet& s, int j) {
  return s.base ? s.base + (long)j * s.stride : s.p[j];
}

// After the update pass of CG iteration it (it = -1: after the start),
// store r_{it+1} into slot it + 1 and, for it >= 0, the pair (r_it^T z_it,
// p_it^T A~ p_it): r.z from the scalar slot the operator pass of iteration
// it wrote (its coarse part included), p.q from that pass's partials.
// Nothing is stored once the solve has stopped (its flag raised).
template <typename VT>
__global__ __launch_bounds__(256) void k_rec_store(const VT* __restrict__ r, double* __restrict__ slot, long n3,
                                                   const double* __restrict__ part_pq, int n_pq,
                                                   const double* __restrict__ scal, double* __restrict__ coef,
                                                   int it) {
  if (scal[S_DONE] != 0.0) return;
  if (slot)
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n3; i += (long)gridDim.x * blockDim.x)
      slot[i] = (double)r[i];
  if (blockIdx.x == 0) {
    __shared__ double sh[8];
    double pq = 0.0;
    if (it >= 0) pq = sum_partials(part_pq, n_pq, sh);
    if (threadIdx.x == 0) {
      if (it >= 0) {
        coef[2 * it] = scal[S_RZ0 + (it & 1)];
        coef[2 * it + 1] = pq;
        coef[2 * REC_MMAX + 1] = (double)(it + 1);  // coefficient pairs
      }
      if (slot) coef[2 * REC_MMAX] = (double)(it + 2);  // stored vectors
    }
  }
}

// out_o = sum_j C[j * nout + o] src_j, o < nout (C staged in LDS)
__global__ __launch_bounds__(256) void k_combine(VecSet src, int nsrc, const double* __restrict__ C, int nout,
                                                 OutSet dst, long n) {
  __shared__ double sC[COMB_MAX];
  for (int t = threadIdx.x; t < nsrc * nout; t += blockDim.x) sC[t] = C[t];
  __syncthreads();
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double acc[RR_NMAX];
#pragma unroll
    for (int o = 0; o < RR_NMAX; ++o) acc[o] = 0.0;
    for (int j = 0; j < nsrc; ++j) {
      const double v = vs_get(src, j)[i];
#pragma unroll
      for (int o = 0; o < RR_NMAX; ++o)
        if (o < nout) acc[o] = fma(sC[j * nout + o], v, acc[o]);
    }
#pragma unroll
    for (int o = 0; o < RR_NMAX; ++o)
      if (o < nout) dst.p[o][i] = acc[o];
  }
}

// Partial sums of s_a^T t_b (pair index = blockIdx.y over a < b... all n x n
// pairs a, b with a <= b) and s_a^T D s_b with D = 1 / dinv.
__global__ __launch_bounds__(256) void k_rr_gram(VecSet S, VecSet T, int n, const double* __restrict__ dinv, long n3,
                                                 double* __restrict__ part) {
  __shared__ double sh[8];
  int a = 0, b = blockIdx.y;
  while (b >= n - a) { b -= n - a; ++a; }
  b += a;
  const double* sa = vs_get(S, a);
  const double* sb = vs_get(S, b);
  const double* tb = vs_get(T, b);
  double g = 0.0, m = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n3; i += (long)gridDim.x * blockDim.x) {
    const double x = sa[i];
    g = fma(x, tb[i], g);
    m = fma(x, sb[i] / dinv[i], m);
  }
  g = block_sum(g, sh);
  m = block_sum(m, sh);
  if (threadIdx.x == 0) {
    part[(2L * blockIdx.y) * gridDim.x + blockIdx.x] = g;
    part[(2L * blockIdx.y + 1) * gridDim.x + blockIdx.x] = m;
  }
}

// ------------------------------------------------------------------ host linear algebra
// Eigenpairs of a symmetric tridiagonal matrix (diagonal d, off-diagonal e,
// e[i] couples i and i + 1) by the implicit QL method with Wilkinson shifts;
// Z receives the eigenvectors as columns (row-major n x n), d the
// eigenvalues, both sorted ascending.  Returns false if an eigenvalue did not
// converge in 60 sweeps.
static bool tridiag_eig(int n, std::vector<double>& d, std::vector<double> e, std::vector<double>& Z) {
  Z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  e.resize(n, 0.0);
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-15 * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) return false;
      // Wilkinson shift from the leading 2x2 block at l
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      for (; i >= l; --i) {
        double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          double* zk = &Z[(size_t)k * n];
          f = zk[i + 1];
          zk[i + 1] = s * zk[i] + c * f;
          zk[i] = c * zk[i] - s * f;
        }
      }
      if (r == 0.0 && i >= l) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  // sort ascending
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] < d[b]; });
  std::vector<double> d2(n), Z2((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    d2[j] = d[ord[j]];
    for (int k = 0; k < n; ++k) Z2[(size_t)k * n + j] = Z[(size_t)k * n + ord[j]];
  }
  d = d2;
  Z = Z2;
  return true;
}

// Eigenpairs of a dense symmetric matrix A (row-major n x n, overwritten) by
// cyclic Jacobi rotations; V receives eigenvectors as columns, w eigenvalues,
// sorted ascending.
static void jacobi_eig(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) (i == j ? tot : off) += a(i, j) * a(i, j);
    if (off <= 1e-30 * (tot + off)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (a(p, q) == 0.0) continue;
        const double theta = (a(q, q) - a(p, p)) / (2.0 * a(p, q));
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
  std::vector<double> V2((size_t)n * n);
  w.resize(n);
  for (int j = 0; j < n; ++j) {
    w[j] = a(ord[j], ord[j]);
    for (int k = 0; k < n; ++k) V2[(size_t)k * n + j] = V[(size_t)k * n + ord[j]];
  }
  V = V2;
}

// ------------------------------------------------------------------ recording (called by the solve)
template <typename VT>
int recycle_store(amrto_ctx* ctx, const VT* r, int it) {
  if (!ctx->rec_active || it >= ctx->rec_m) return AMRTO_OK;
  const long n3 = 3L * ctx->n_nodes;
  double* slot = it + 1 < ctx->rec_m ? ctx->d_rec_store + (long)(it + 1) * n3 : nullptr;
  hipLaunchKernelGGL(k_rec_store<VT>, dim3(slot ? grid_for(n3, 256, 1024) : 1), dim3(256), 0, ctx->stream, r, slot,
                     n3, (const double*)ctx->d_partpq, ctx->n_partpq, (const double*)ctx->d_scal, ctx->d_rec_coef,
                     it);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}
template int recycle_store<double>(amrto_ctx*, const double*, int);
template int recycle_store<float>(amrto_ctx*, const float*, int);

__global__ void k_zero(double* __restrict__ x, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = 0.0;
}

int recycle_begin(amrto_ctx* ctx, bool block3) {
  if (!ctx->rec_active) return AMRTO_OK;
  ctx->rec_block3 = block3;
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, ctx->stream, ctx->d_rec_coef, 2 * REC_MMAX + 2);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

static int combine(amrto_ctx* ctx, const VecSet& src, int nsrc, const std::vector<double>& C, int nout,
                   double* const* out) {
  if (nsrc * nout > COMB_MAX || nout > RR_NMAX) return ctx->fail(AMRTO_EINVAL, "recycling: combination too large");
  OutSet o{};
  for (int i = 0; i < nout; ++i) o.p[i] = out[i];
  AMRTO_HIP(hipMemcpyAsync(ctx->d_rec_C, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  const long n3 = 3L * ctx->n_nodes;
  hipLaunchKernelGGL(k_combine, dim3(grid_for(n3, 256, 2048)), dim3(256), 0, ctx->stream, src, nsrc,
                     (const double*)ctx->d_rec_C, nout, o, n3);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

}  // namespace amrto

using namespace amrto;

extern "C" {

int amrto_recycle_setup(amrto_ctx* ctx, int32_t m) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_recycle_setup: no mesh");
  if (m < 2 || m > REC_MMAX) return ctx->fail(AMRTO_EINVAL, "amrto_recycle_setup: m must be in [2, 256]");
  AMRTO_HIP(hipSetDevice(ctx->device));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  const long n3 = 3L * ctx->n_nodes;
  auto re = [&](double*& p, size_t count) -> hipError_t {
    if (p) (void)hipFree(p);
    p = nullptr;
    return hipMalloc((void**)&p, std::max<size_t>(1, count) * sizeof(double));
  };
  AMRTO_HIP(re(ctx->d_rec_store, (size_t)m * n3));
  AMRTO_HIP(re(ctx->d_rec_coef, 2 * REC_MMAX + 2));
  AMRTO_HIP(re(ctx->d_rec_C, COMB_MAX));
  AMRTO_HIP(re(ctx->d_rr_aw, (size_t)RR_NMAX * n3));
  AMRTO_HIP(re(ctx->d_rr_part, (size_t)2 * GRAM_BLOCKS * RR_NMAX * (RR_NMAX + 1) / 2));
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, ctx->stream, ctx->d_rec_coef, 2 * REC_MMAX + 2);
  AMRTO_HIP(hipGetLastError());
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  ctx->rec_m = m;
  return AMRTO_OK;
}

int amrto_recycle_harvest(amrto_ctx* ctx, int32_t k, double* const* u_host, double* theta_host, double* resid_host,
                          int32_t* m_used) {
  if (!ctx) return AMRTO_EINVAL;
  if (ctx->rec_m <= 0) return ctx->fail(AMRTO_ESTATE, "amrto_recycle_harvest: no amrto_recycle_setup");
  if (k < 1 || k > RR_NMAX || !u_host) return ctx->fail(AMRTO_EINVAL, "amrto_recycle_harvest: need 1 <= k <= 16 outputs");
  for (int i = 0; i < k; ++i)
    if (!u_host[i]) return ctx->fail(AMRTO_EINVAL, "amrto_recycle_harvest: NULL output");
  AMRTO_HIP(hipSetDevice(ctx->device));
  std::vector<double> coef(2 * REC_MMAX + 2);
  AMRTO_HIP(hipMemcpyAsync(coef.data(), ctx->d_rec_coef, coef.size() * sizeof(double), hipMemcpyDeviceToHost,
                           ctx->stream));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  const int nvec = (int)coef[2 * REC_MMAX], npair = (int)coef[2 * REC_MMAX + 1];
  const int m = std::min(npair - 1, nvec);  // Lanczos steps with known alpha, beta and the next r.z
  if (m < k) return ctx->fail(AMRTO_ESTATE, "amrto_recycle_harvest: the recorded solve is shorter than k + 1 steps");
  std::vector<double> rz(m + 1), pq(m);
  for (int j = 0; j <= m; ++j) rz[j] = coef[2 * j];
  for (int j = 0; j < m; ++j) pq[j] = coef[2 * j + 1];
  for (int j = 0; j < m; ++j)
    if (!(rz[j] > 0.0) || !(pq[j] > 0.0) || !std::isfinite(rz[j]) || !std::isfinite(pq[j]))
      return ctx->fail(AMRTO_EBREAKDOWN, "amrto_recycle_harvest: non-positive recorded coefficient");
  std::vector<double> d(m), e(m, 0.0), Y;
  for (int j = 0; j < m; ++j) {
    const double alpha = rz[j] / pq[j];
    d[j] = 1.0 / alpha;
    if (j > 0) d[j] += (rz[j] / rz[j - 1]) / (rz[j - 1] / pq[j - 1]);
    if (j + 1 < m) e[j] = std::sqrt(rz[j + 1] / rz[j]) / alpha;
  }
  if (!tridiag_eig(m, d, e, Y)) return ctx->fail(AMRTO_EBREAKDOWN, "amrto_recycle_harvest: eigenvalues did not converge");
  const double off = std::sqrt(rz[m] / rz[m - 1]) / (rz[m - 1] / pq[m - 1]);
  std::vector<double> C((size_t)m * k);
  for (int j = 0; j < m; ++j) {
    const double s = ((j & 1) ? -1.0 : 1.0) / std::sqrt(rz[j]);
    for (int i = 0; i < k; ++i) C[(size_t)j * k + i] = s * Y[(size_t)j * m + i];
  }
  for (int i = 0; i < k; ++i) {
    if (theta_host) theta_host[i] = d[i];
    if (resid_host) resid_host[i] = std::fabs(off * Y[(size_t)(m - 1) * m + i]);
  }
  if (m_used) *m_used = m;
  VecSet src{};
  src.base = ctx->d_rec_store;
  src.stride = 3L * ctx->n_nodes;
  if ((long)m * k > COMB_MAX) return ctx->fail(AMRTO_EINVAL, "amrto_recycle_harvest: m k above 4096");
  // u_i = M^-1 (sum_j c_ij r_j): the stored residuals are combined first, the
  // recorded solve's preconditioner is applied once per Ritz vector
  const long n3 = 3L * ctx->n_nodes;
  double* tmp[RR_NMAX];
  for (int i = 0; i < k; ++i) tmp[i] = ctx->d_rr_aw + i * n3;
  int rc = combine(ctx, src, m, C, k, tmp);
  for (int i = 0; i < k && !rc; ++i) rc = apply_precond(ctx, tmp[i], u_host[i], ctx->rec_block3, ctx->rec_coarse);
  if (rc) return rc;
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  return AMRTO_OK;
}

int amrto_rayleigh_ritz(amrto_ctx* ctx, const double* const* s_host, int32_t n, int32_t k, double* const* w_host,
                        double* theta_host, int32_t* rank) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, "amrto_rayleigh_ritz: density not set");
  if (ctx->rec_m <= 0) return ctx->fail(AMRTO_ESTATE, "amrto_rayleigh_ritz: no amrto_recycle_setup");
  if (n < 1 || n > RR_NMAX || k < 1 || k > n || !s_host || !w_host)
    return ctx->fail(AMRTO_EINVAL, "amrto_rayleigh_ritz: need 1 <= k <= n <= 16");
  for (int i = 0; i < n; ++i)
    if (!s_host[i]) return ctx->fail(AMRTO_EINVAL, "amrto_rayleigh_ritz: NULL input");
  for (int i = 0; i < k; ++i) {
    if (!w_host[i]) return ctx->fail(AMRTO_EINVAL, "amrto_rayleigh_ritz: NULL output");
    for (int j = 0; j < n; ++j)
      if (w_host[i] == s_host[j]) return ctx->fail(AMRTO_EINVAL, "amrto_rayleigh_ritz: outputs alias inputs");
  }
  AMRTO_HIP(hipSetDevice(ctx->device));
  const long n3 = 3L * ctx->n_nodes;
  VecSet S{}, AS{};
  for (int j = 0; j < n; ++j) {
    S.p[j] = s_host[j];
    AS.p[j] = ctx->d_rr_aw + j * n3;
    int rc = launch_apply(ctx, s_host[j], ctx->d_rr_aw + j * n3, AMRTO_FP64);
    if (rc) return rc;
  }
  const int npair = n * (n + 1) / 2;
  hipLaunchKernelGGL(k_rr_gram, dim3(GRAM_BLOCKS, npair), dim3(256), 0, ctx->stream, S, AS, n,
                     (const double*)ctx->d_dinv, n3, ctx->d_rr_part);
  AMRTO_HIP(hipGetLastError());
  std::vector<double> part((size_t)2 * npair * GRAM_BLOCKS);
  AMRTO_HIP(hipMemcpyAsync(part.data(), ctx->d_rr_part, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                           ctx->stream));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<double> G((size_t)n * n), B((size_t)n * n);
  for (int a = 0, pidx = 0; a < n; ++a)
    for (int b = a; b < n; ++b, ++pidx) {
      double g = 0.0, m = 0.0;
      for (int t = 0; t < GRAM_BLOCKS; ++t) {
        g += part[(size_t)(2 * pidx) * GRAM_BLOCKS + t];
        m += part[(size_t)(2 * pidx + 1) * GRAM_BLOCKS + t];
      }
      G[(size_t)a * n + b] = G[(size_t)b * n + a] = g;
      B[(size_t)a * n + b] = B[(size_t)b * n + a] = m;
    }
  // B = U L L^T U^T restricted to its numerically independent directions:
  // eigen-decompose B, keep eigenvalues above 1e-12 of the largest, and
  // solve the reduced standard problem in the basis X = V_B Lambda^-1/2.
  std::vector<double> Bw, BV, Bc = B;
  jacobi_eig(n, Bc, Bw, BV);
  const double bmax = Bw[n - 1];
  if (!(bmax > 0.0) || !std::isfinite(bmax)) return ctx->fail(AMRTO_EINVAL, "amrto_rayleigh_ritz: zero or non-finite inputs");
  std::vector<int> keep;
  for (int i = 0; i < n; ++i)
    if (Bw[i] > 1e-12 * bmax) keep.push_back(i);
  const int r = (int)keep.size();
  if (r < k) return ctx->fail(AMRTO_EINVAL, "amrto_rayleigh_ritz: inputs span fewer than k directions");
  std::vector<double> X((size_t)n * r);
  for (int c = 0; c < r; ++c)
    for (int i = 0; i < n; ++i) X[(size_t)i * r + c] = BV[(size_t)i * n + keep[c]] / std::sqrt(Bw[keep[c]]);
  std::vector<double> H((size_t)r * r, 0.0);  // X^T G X
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) {
      double s = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) s += X[(size_t)i * r + a] * G[(size_t)i * n + j] * X[(size_t)j * r + b];
      H[(size_t)a * r + b] = s;
    }
  for (int a = 0; a < r; ++a)
    for (int b = a + 1; b < r; ++b) H[(size_t)a * r + b] = H[(size_t)b * r + a] = 0.5 * (H[(size_t)a * r + b] + H[(size_t)b * r + a]);
  std::vector<double> hw, HV;
  jacobi_eig(r, H, hw, HV);
  std::vector<double> C((size_t)n * k, 0.0);  // Y = X HV[:, :k]
  for (int i = 0; i < n; ++i)
    for (int o = 0; o < k; ++o) {
      double s = 0.0;
      for (int c = 0; c < r; ++c) s += X[(size_t)i * r + c] * HV[(size_t)c * r + o];
      C[(size_t)i * k + o] = s;
    }
  for (int o = 0; o < k; ++o)
    if (theta_host) theta_host[o] = hw[o];
  if (rank) *rank = r;
  int rc = combine(ctx, S, n, C, k, w_host);
  if (rc) return rc;
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  return AMRTO_OK;
}

}  // extern "C"
