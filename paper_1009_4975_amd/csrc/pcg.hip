// Jacobi-preconditioned conjugate gradients on A~ (paper Sec. 5: symmetric
// diagonal rescaling; warm start from the previous solution) and FP64
// iterative refinement around FP32 / BF16 inner solves.
//
// All scalars live on the device.  Reductions write RED_BLOCKS partial sums;
// every consumer block re-adds them in the same order, so every block takes
// the same decision (alpha, beta, convergence, breakdown) without a separate
// finalize launch.  Convergence raises a flag that makes every later kernel
// of the batch return at once, so the host can enqueue several iterations
// between checks without running past the converged iterate.
#include <chrono>
#include <cmath>

#include "internal.h"

namespace amrto {

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double sum_partials(const double* __restrict__ part, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += blockDim.x) v += part[i];
  return block_sum(v, sh);
}

// zero the supported and hanging entries of a vector (their rows are identity
// with zero right-hand side, so the iterate keeps them at zero)
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

template <typename VT>
__global__ __launch_bounds__(256) void k_fill(VT* __restrict__ x, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

// r = b - q (q may be NULL: r = b), z = D^-1 r, p = z; partials of r.z, r.r, b.b
template <typename VT>
__global__ __launch_bounds__(256) void k_init(const VT* __restrict__ b, const VT* __restrict__ q,
                                              VT* __restrict__ r, VT* __restrict__ z, VT* __restrict__ p,
                                              const VT* __restrict__ dinv, long n, double* __restrict__ part) {
  __shared__ double sh[16];
  double rz = 0, rr = 0, bb = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const VT bi = b[i];
    const VT ri = q ? (VT)(bi - q[i]) : bi;
    const VT zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    p[i] = zi;
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

__global__ __launch_bounds__(256) void k_init_scalars(const double* __restrict__ part, double* __restrict__ scal,
                                                      double tol2) {
  __shared__ double sh[16];
  const double rz = sum_partials(part, sh);
  const double rr = sum_partials(part + RED_BLOCKS, sh);
  const double bb = sum_partials(part + 2 * RED_BLOCKS, sh);
  if (threadIdx.x == 0) {
    scal[S_RZ0] = rz;
    scal[S_RZ1] = rz;
    scal[S_BB] = bb;
    scal[S_RR] = rr;
    scal[S_ITERS] = 0.0;
    scal[S_DONE] = (rr <= tol2 * bb) ? 1.0 : (std::isfinite(rr) ? 0.0 : 2.0);
  }
}

// partial sums of a.b
template <typename VT>
__global__ __launch_bounds__(256) void k_dot(const VT* __restrict__ a, const VT* __restrict__ b, long n,
                                             double* __restrict__ part, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double sh[16];
  double s = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    s += (double)a[i] * (double)b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// alpha = rz / p.q; x += alpha p; r -= alpha q; z = D^-1 r; partials of r.z, r.r
template <typename VT>
__global__ __launch_bounds__(256) void k_update(VT* __restrict__ x, VT* __restrict__ r, const VT* __restrict__ p,
                                                const VT* __restrict__ q, const VT* __restrict__ dinv,
                                                VT* __restrict__ z, long n, const double* __restrict__ part_pq,
                                                double* __restrict__ part, double* __restrict__ scal, int rz_slot) {
  if (scal[S_DONE] != 0.0) return;
  __shared__ double sh[16];
  const double pq = sum_partials(part_pq, sh);
  const double rz = scal[rz_slot];
  if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_DONE] = 2.0;
    return;
  }
  const VT alpha = (VT)(rz / pq);
  double srz = 0.0, srr = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const VT ri = r[i] - alpha * q[i];
    const VT zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    srz += (double)ri * (double)zi;
    srr += (double)ri * (double)ri;
  }
  srz = block_sum(srz, sh);
  srr = block_sum(srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[RED_BLOCKS + blockIdx.x] = srr;
  }
}

// beta = rz_new / rz; p = z + beta p; convergence when r.r <= tol^2 b.b
template <typename VT>
__global__ __launch_bounds__(256) void k_direction(VT* __restrict__ p, const VT* __restrict__ z, long n,
                                                   const double* __restrict__ part, double* __restrict__ scal,
                                                   int rz_cur, int rz_next, double tol2, int it) {
  if (scal[S_DONE] != 0.0) return;
  __shared__ double sh[16];
  const double rz_new = sum_partials(part, sh);
  const double rr = sum_partials(part + RED_BLOCKS, sh);
  if (!std::isfinite(rr) || !std::isfinite(rz_new)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_DONE] = 2.0;
    return;
  }
  if (rr <= tol2 * scal[S_BB]) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      scal[S_RR] = rr;
      scal[S_ITERS] = it + 1;
      scal[S_DONE] = 1.0;
    }
    return;
  }
  const VT beta = (VT)(rz_new / scal[rz_cur]);
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[rz_next] = rz_new;
    scal[S_RR] = rr;
    scal[S_ITERS] = it + 1;
  }
}

// r = b - q and partial r.r (FP64), for true residuals and refinement steps
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ b, const double* __restrict__ q,
                                                  double* __restrict__ r, long n, double* __restrict__ part) {
  __shared__ double sh[16];
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

__global__ __launch_bounds__(256) void k_residual_scalars(const double* __restrict__ part, double* __restrict__ scal) {
  __shared__ double sh[16];
  const double rr = sum_partials(part, sh);
  const double bb = sum_partials(part + RED_BLOCKS, sh);
  if (threadIdx.x == 0) {
    scal[S_RR] = rr;
    scal[S_BB] = bb;
  }
}

// inner right-hand side: b32 = r / ||r||
__global__ __launch_bounds__(256) void k_scale_to_float(const double* __restrict__ r, float* __restrict__ b32,
                                                        const double* __restrict__ scal, long n) {
  const double s = 1.0 / sqrt(scal[S_RR]);
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) b32[i] = (float)(r[i] * s);
}

// x += ||r|| * d32
__global__ __launch_bounds__(256) void k_correct(double* __restrict__ x, const float* __restrict__ d32,
                                                 const double* __restrict__ scal_outer, long n) {
  const double s = sqrt(scal_outer[0]);
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) x[i] += s * (double)d32[i];
}

__global__ void k_copy_scalar(const double* __restrict__ a, double* __restrict__ b) { *b = *a; }

// ------------------------------------------------------------------ host
struct Work {
  void* r; void* z; void* p; void* q; const void* dinv;
};

template <typename VT>
static Work work_for(amrto_ctx* ctx);
template <>
Work work_for<double>(amrto_ctx* ctx) { return {ctx->d_r, ctx->d_z, ctx->d_p, ctx->d_q, ctx->d_dinv}; }
template <>
Work work_for<float>(amrto_ctx* ctx) { return {ctx->f_r, ctx->f_z, ctx->f_p, ctx->f_q, ctx->d_dinv_f}; }

// One CG run on A~ (contraction precision `prec`) from x (x0_zero: x = 0).
// Returns AMRTO_OK, AMRTO_NOT_CONVERGED or AMRTO_EBREAKDOWN; *iters counts
// the iterations performed.
template <typename VT>
static int cg_core(amrto_ctx* ctx, const VT* b, VT* x, int prec, double rtol, int max_it, int check_every,
                   bool x0_zero, int* iters) {
  const long n3 = 3L * ctx->n_nodes;
  const int g1 = (int)((n3 + 255) / 256);
  Work w = work_for<VT>(ctx);
  VT* r = (VT*)w.r; VT* z = (VT*)w.z; VT* p = (VT*)w.p; VT* q = (VT*)w.q;
  const VT* dinv = (const VT*)w.dinv;
  double* part = ctx->d_part;
  double* scal = ctx->d_scal;
  const double tol2 = rtol * rtol;
  if (x0_zero) {
    hipLaunchKernelGGL(k_fill<VT>, dim3(g1), dim3(256), 0, ctx->stream, x, n3);
  } else {
    hipLaunchKernelGGL(k_mask<VT>, dim3(g1), dim3(256), 0, ctx->stream, x, ctx->d_fix, n3);
    if (ctx->n_hang)
      hipLaunchKernelGGL(k_mask_hanging<VT>, dim3((3L * ctx->n_hang + 255) / 256), dim3(256), 0, ctx->stream, x,
                         ctx->d_hang_node, ctx->n_hang);
    int rc = apply_stop(ctx, x, q, prec, nullptr);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_init<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, b, x0_zero ? nullptr : q, r, z, p,
                     dinv, n3, part);
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(256), 0, ctx->stream, part, scal, tol2);
  AMRTO_HIP(hipGetLastError());
  int it = 0;
  int status = AMRTO_NOT_CONVERGED;
  double* stop = scal + S_DONE;
  while (true) {
    AMRTO_HIP(hipMemcpyAsync(ctx->h_scal, scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    AMRTO_HIP(hipStreamSynchronize(ctx->stream));
    const double done = ctx->h_scal[S_DONE];
    if (done == 1.0) { status = AMRTO_OK; break; }
    if (done == 2.0) { status = AMRTO_EBREAKDOWN; break; }
    if (it >= max_it) break;
    const int batch = std::min(check_every, max_it - it);
    for (int k = 0; k < batch; ++k, ++it) {
      int rc = apply_stop(ctx, p, q, prec, stop);
      if (rc) return rc;
      hipLaunchKernelGGL(k_dot<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, p, q, n3, part, stop);
      hipLaunchKernelGGL(k_update<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, x, r, p, q, dinv, z, n3, part,
                         part + 2 * RED_BLOCKS, scal, (it & 1) ? S_RZ1 : S_RZ0);
      hipLaunchKernelGGL(k_direction<VT>, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, p, z, n3,
                         part + 2 * RED_BLOCKS, scal, (it & 1) ? S_RZ1 : S_RZ0, (it & 1) ? S_RZ0 : S_RZ1, tol2, it);
    }
    AMRTO_HIP(hipGetLastError());
  }
  *iters = (int)ctx->h_scal[S_ITERS];
  return status;
}

// true FP64 residual of A~ x = b: *rel = ||b - A~ x|| / ||b||; leaves r in d_r
static int true_residual(amrto_ctx* ctx, const double* b, const double* x, double* rel, double* rr_out,
                         double* bb_out) {
  const long n3 = 3L * ctx->n_nodes;
  int rc = apply_stop(ctx, x, ctx->d_q, AMRTO_FP64, nullptr);
  if (rc) return rc;
  hipLaunchKernelGGL(k_residual, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, b, ctx->d_q, ctx->d_r, n3,
                     ctx->d_part);
  hipLaunchKernelGGL(k_residual_scalars, dim3(1), dim3(256), 0, ctx->stream, ctx->d_part, ctx->d_scal);
  AMRTO_HIP(hipGetLastError());
  AMRTO_HIP(hipMemcpyAsync(ctx->h_scal, ctx->d_scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  const double rr = ctx->h_scal[S_RR], bb = ctx->h_scal[S_BB];
  *rel = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
  if (rr_out) *rr_out = rr;
  if (bb_out) *bb_out = bb;
  return AMRTO_OK;
}

}  // namespace amrto

using namespace amrto;

extern "C" {

void amrto_solve_opts_default(amrto_solve_opts* o) {
  if (!o) return;
  o->rtol = 1e-8;
  o->max_it = 20000;
  o->precond = AMRTO_PRECOND_JACOBI;
  o->inner_prec = AMRTO_FP64;
  o->inner_rtol = 1e-3;
  o->max_outer = 50;
  o->check_every = 16;
  o->Z_dev = nullptr;
  o->k = 0;
}

int amrto_pcg(amrto_ctx* ctx, const double* b, double* u, const amrto_solve_opts* opts_in,
              amrto_solve_stats* stats) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, "amrto_pcg: density not set");
  if (!b || !u || b == u) return ctx->fail(AMRTO_EINVAL, "amrto_pcg: b and u must be distinct device buffers");
  amrto_solve_opts o;
  amrto_solve_opts_default(&o);
  if (opts_in) o = *opts_in;
  if (!(o.rtol > 0.0) || o.max_it < 0 || o.check_every < 1 || o.max_outer < 1 || !(o.inner_rtol > 0.0))
    return ctx->fail(AMRTO_EINVAL, "amrto_pcg: bad options");
  if (o.inner_prec != AMRTO_FP64 && o.inner_prec != AMRTO_FP32 && o.inner_prec != AMRTO_BF16)
    return ctx->fail(AMRTO_EINVAL, "amrto_pcg: unknown inner precision");
  if (o.precond != AMRTO_PRECOND_JACOBI) return ctx->fail(AMRTO_EINVAL, "amrto_pcg: unknown preconditioner");
  AMRTO_HIP(hipSetDevice(ctx->device));
  const auto t0 = std::chrono::steady_clock::now();
  const long n3 = 3L * ctx->n_nodes;
  int iters = 0, outer = 0, status;
  double rel = 0.0;
  if (o.inner_prec == AMRTO_FP64) {
    status = cg_core<double>(ctx, b, u, AMRTO_FP64, o.rtol, o.max_it, o.check_every, false, &iters);
    if (status < 0 && status != AMRTO_EBREAKDOWN) return status;
    int rc = true_residual(ctx, b, u, &rel, nullptr, nullptr);
    if (rc) return rc;
  } else {
    // FP64 outer loop: r = b - A~64 x, inner CG on A~lo d = r / ||r|| in FP32
    // vectors, x += ||r|| d.  Residual, norms and dots stay in FP64.
    hipLaunchKernelGGL(k_mask<double>, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, u, ctx->d_fix, n3);
    if (ctx->n_hang)
      hipLaunchKernelGGL(k_mask_hanging<double>, dim3((3L * ctx->n_hang + 255) / 256), dim3(256), 0, ctx->stream, u,
                         ctx->d_hang_node, ctx->n_hang);
    status = AMRTO_NOT_CONVERGED;
    double rr = 0, bb = 0;
    for (outer = 0; outer <= o.max_outer; ++outer) {
      int rc = true_residual(ctx, b, u, &rel, &rr, &bb);
      if (rc) return rc;
      if (!std::isfinite(rel)) { status = AMRTO_EBREAKDOWN; break; }
      if (rel <= o.rtol) { status = AMRTO_OK; break; }
      if (outer == o.max_outer || iters >= o.max_it) break;
      hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, ctx->stream, ctx->d_scal + S_RR, ctx->d_oc);
      hipLaunchKernelGGL(k_scale_to_float, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_r, ctx->f_b,
                         ctx->d_scal, n3);
      int it_in = 0;
      rc = cg_core<float>(ctx, ctx->f_b, ctx->f_x, o.inner_prec, o.inner_rtol, o.max_it - iters, o.check_every,
                          true, &it_in);
      if (rc < 0 && rc != AMRTO_EBREAKDOWN) return rc;
      iters += it_in;
      hipLaunchKernelGGL(k_correct, dim3((n3 + 255) / 256), dim3(256), 0, ctx->stream, u, ctx->f_x, ctx->d_oc, n3);
      AMRTO_HIP(hipGetLastError());
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
  }
  if (status == AMRTO_EBREAKDOWN) return ctx->fail(AMRTO_EBREAKDOWN, "amrto_pcg: breakdown (p^T A p <= 0 or non-finite)");
  if (status == AMRTO_NOT_CONVERGED) ctx->err = "amrto_pcg: iteration cap reached";
  return status;
}

}  // extern "C"
