// Element coefficients (SIMP law), right-hand-side projection and hanging
// recovery (paper Sec. 3 Eq. (2), Sec. 6 Eq. (7) and (9)).
#include <cmath>

#include "internal.h"

namespace amrto {

// c_e = (Emin + rho^p (E0 - Emin)) h_e with h_e = 2^(max_level - level_e):
// the element matrix of an edge-h cube is h K0 (strain ~ 1/h, volume ~ h^3).
__global__ __launch_bounds__(256) void k_set_density(
    const double* __restrict__ rho, const int8_t* __restrict__ level, double* __restrict__ coef,
    float* __restrict__ coef_f, int n, int max_level, double E0, double Emin, double p) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double h = (double)(1 << (max_level - level[e]));
  const double E = Emin + pow(rho[e], p) * (E0 - Emin);
  coef[e] = E * h;
  coef_f[e] = (float)(E * h);
}

// b = F T^T f.  Regular DOFs copy f, then receive the hanging loads of the
// hanging nodes they interpolate (gathered per hanging node in fixed order),
// then supported and hanging DOFs are zeroed.
__global__ __launch_bounds__(256) void k_rhs_copy(const double* __restrict__ f, double* __restrict__ b,
                                                  const uint8_t* __restrict__ fix, long n3) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n3) return;
  b[i] = ((fix[i / 3] >> (i % 3)) & 1) ? 0.0 : f[i];
}

__global__ __launch_bounds__(256) void k_rhs_hanging(
    const double* __restrict__ f, double* __restrict__ b, const uint8_t* __restrict__ fix,
    const int32_t* __restrict__ mt_node, const int32_t* __restrict__ mt_ptr,
    const int32_t* __restrict__ mt_h, const double* __restrict__ mt_w, int n_mt) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= 3L * n_mt) return;
  const int s = (int)(i / 3), c = (int)(i % 3);
  const int m = mt_node[s];
  if ((fix[m] >> c) & 1) return;
  double v = 0.0;
  for (int k = mt_ptr[s]; k < mt_ptr[s + 1]; ++k) v += mt_w[k] * f[3L * mt_h[k] + c];
  b[3L * m + c] += v;
}

__global__ __launch_bounds__(256) void k_zero_hanging(double* __restrict__ b, const int32_t* __restrict__ hang_node,
                                                      int n_hang) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= 3L * n_hang) return;
  b[3L * hang_node[i / 3] + i % 3] = 0.0;
}

// u = T u~: copy, then u_h = sum_m w_hm u~_m (masters are never hanging).
__global__ __launch_bounds__(256) void k_copy(const double* __restrict__ a, double* __restrict__ b, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_recover_hanging(
    const double* __restrict__ ut, double* __restrict__ u, const int32_t* __restrict__ hang_node,
    const int32_t* __restrict__ hang_ptr, const int32_t* __restrict__ hang_master,
    const double* __restrict__ hang_w, int n_hang) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= 3L * n_hang) return;
  const int h = (int)(i / 3), c = (int)(i % 3);
  double v = 0.0;
  for (int k = hang_ptr[h]; k < hang_ptr[h + 1]; ++k) v += hang_w[k] * ut[3L * hang_master[k] + c];
  u[3L * hang_node[h] + c] = v;
}

int launch_set_density(amrto_ctx* ctx, const double* rho) {
  const int n = ctx->n_elems;
  hipLaunchKernelGGL(k_set_density, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, rho, ctx->d_level,
                     ctx->d_coef, ctx->d_coef_f, n, ctx->max_level, ctx->E0, ctx->Emin, ctx->p);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int launch_project_rhs(amrto_ctx* ctx, const double* f, double* b) {
  const long n3 = 3L * ctx->n_nodes;
  hipLaunchKernelGGL(k_rhs_copy, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, f, b, ctx->d_fix, n3);
  if (ctx->n_hang > 0) {
    const long nm = 3L * ctx->n_mt;
    if (nm > 0)
      hipLaunchKernelGGL(k_rhs_hanging, dim3((nm + 255) / 256), dim3(256), 0, ctx->stream, f, b, ctx->d_fix,
                         ctx->d_mt_node, ctx->d_mt_ptr, ctx->d_mt_h, ctx->d_mt_w, ctx->n_mt);
    const long nh = 3L * ctx->n_hang;
    hipLaunchKernelGGL(k_zero_hanging, dim3((nh + 255) / 256), dim3(256), 0, ctx->stream, b,
                       ctx->d_hang_node, ctx->n_hang);
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int launch_recover(amrto_ctx* ctx, const double* ut, double* u) {
  const long n3 = 3L * ctx->n_nodes;
  if (ut != u)
    hipLaunchKernelGGL(k_copy, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, ut, u, n3);
  if (ctx->n_hang > 0) {
    const long nh = 3L * ctx->n_hang;
    hipLaunchKernelGGL(k_recover_hanging, dim3((nh + 255) / 256), dim3(256), 0, ctx->stream, ut, u,
                       ctx->d_hang_node, ctx->d_hang_ptr, ctx->d_hang_master, ctx->d_hang_w, ctx->n_hang);
  }
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

__global__ __launch_bounds__(256) void k_recip(const double* __restrict__ a, double* __restrict__ b, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = 1.0 / a[i];
}

int launch_recip(amrto_ctx* ctx, const double* a, double* b, long n) {
  hipLaunchKernelGGL(k_recip, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, a, b, n);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

}  // namespace amrto
