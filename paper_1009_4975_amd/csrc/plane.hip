// The 2-D variant of the hot path (paper Sec. 6-7, Test 1): Q4 plane-stress
// elements on a quadtree mesh with hanging nodes.  Per design iteration:
// matrix-free constrained operator A~ = F T^T K T F + (I - F), Jacobi-PCG in
// FP64 with device-resident scalars, compliance and sensitivities, the Eq. (5)
// filter with area weights, and the OC update.
//
// The operator runs in three passes without atomics: (1) per node, the
// masked vector with hanging values interpolated from their masters (in a CG
// step also p = z + beta p_old); (2) per element, y_e = c_e K0 u_e into an
// element-output array; (3) per node, the sum over the node's incidences
// (element vertex, weight: 1 for its own vertices, the interpolation weight
// for vertices that hang on it) in a fixed order, identity rows for supported
// and hanging DOFs.  The incidence lists are built once at mesh upload.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"

namespace amrto {

constexpr int P_RED = 256;    // partial sums of the plane kernels
constexpr int P_OCK = 256;    // OC candidates per pass
constexpr int P_OCB = 256;    // OC blocks
enum { PS_RZ0 = 0, PS_RZ1 = 1, PS_BB = 2, PS_DONE = 3, PS_ITERS = 4, PS_RR = 5, PS_C = 6, PS_COUNT = 8 };

}  // namespace amrto

using namespace amrto;

struct amrto_plane {
  int device = 0;
  hipStream_t stream = nullptr;
  double E0 = 1.0, Emin = 1e-9, nu = 0.3, p = 3.0;
  double K0[64];
  std::string err;
  bool has_mesh = false, has_density = false;
  int n_nodes = 0, n_elems = 0, max_level = 0, nx = 0, ny = 0, hmax = 1;
  std::vector<int8_t> h_level;
  double* d_K0 = nullptr;
  int32_t* d_elem = nullptr;      // [4 ne]
  uint8_t* d_fix = nullptr;       // per node: bits 0, 1 supported DOFs, bit 2 hanging
  int32_t* d_hang_of = nullptr;   // per node: its row of the hanging CSR, or -1
  int32_t* d_hang_node = nullptr; // hanging CSR rows: node, masters, weights
  int32_t* d_hang_ptr = nullptr;
  int32_t* d_hang_master = nullptr;
  double* d_hang_w = nullptr;
  int32_t* d_rhs_ptr = nullptr;   // per node: the hanging nodes it masters, with weights
  int32_t* d_rhs_h = nullptr;
  double* d_rhs_w = nullptr;
  int n_hang = 0;
  int32_t* d_inc_ptr = nullptr;   // [nn + 1] incidences per node
  int32_t* d_inc_slot = nullptr;  // 4 e + a
  double* d_inc_w = nullptr;
  double* d_area = nullptr;
  int32_t* d_edesc = nullptr;     // [3 ne] anchor x, y, edge
  int32_t* d_cmap = nullptr;      // [nx ny] leaf per lattice cell, bit 31 on its anchor cell
  double* d_coef = nullptr;
  double* d_dinv = nullptr;
  double* d_E = nullptr;          // [8 ne] element outputs
  double* d_xe = nullptr;         // expanded vector
  double *d_r = nullptr, *d_z = nullptr, *d_p = nullptr, *d_p2 = nullptr, *d_q = nullptr;  // p ping-pongs
  double* d_part = nullptr;       // 4 x P_RED partial sums
  double* d_scal = nullptr;
  double* h_scal = nullptr;
  double* d_oc = nullptr;         // OC search: bracket, P_OCK x P_OCB partials, P_OCK volumes
  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
};

#define PL_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) return pl->fail(AMRTO_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace amrto {

// unit-square Q4 plane-stress matrix from exact one-dimensional integrals of
// the bilinear shape functions (local node a = i + 2 j, DOF 2 a + c)
static void k0_unit_square(double nu, double* K) {
  const double d11 = 1.0 / (1.0 - nu * nu), d12 = nu / (1.0 - nu * nu), g = 0.5 * (1.0 - nu) / (1.0 - nu * nu);
  auto one_d = [](int ia, int ib, bool da, bool db) -> double {
    if (da && db) return ia == ib ? 1.0 : -1.0;
    if (da) return ia ? 0.5 : -0.5;
    if (db) return ib ? 0.5 : -0.5;
    return ia == ib ? 1.0 / 3.0 : 1.0 / 6.0;
  };
  auto I = [&](int a, int b, int pd, int qd) {
    return one_d(a & 1, b & 1, pd == 0, qd == 0) * one_d(a >> 1, b >> 1, pd == 1, qd == 1);
  };
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      K[(2 * a) * 8 + 2 * b] = d11 * I(a, b, 0, 0) + g * I(a, b, 1, 1);
      K[(2 * a + 1) * 8 + 2 * b + 1] = d11 * I(a, b, 1, 1) + g * I(a, b, 0, 0);
      K[(2 * a) * 8 + 2 * b + 1] = d12 * I(a, b, 0, 1) + g * I(a, b, 1, 0);
      K[(2 * a + 1) * 8 + 2 * b] = d12 * I(a, b, 1, 0) + g * I(a, b, 0, 1);
    }
}

__global__ __launch_bounds__(256) void k2_coef(const double* __restrict__ rho, double* __restrict__ coef, int n,
                                               double E0, double Emin, double p) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) coef[e] = Emin + pow(rho[e], p) * (E0 - Emin);
}

// value of DOF (v, c) of the masked vector with hanging values interpolated;
// in a CG step the vector is p = z + beta p_old, formed here for the node and
// for the masters of a hanging node
__device__ __forceinline__ double masked(const double* __restrict__ z, const double* __restrict__ pold, double beta,
                                         const uint8_t* __restrict__ fix, int v, int c) {
  if ((fix[v] >> c) & 1) return 0.0;
  double x = z[2 * v + c];
  if (pold) x += beta * pold[2 * v + c];
  return x;
}

// pass 1: xe (and, in a CG step, p for the unconstrained DOFs)
__global__ __launch_bounds__(256) void k2_expand(const double* __restrict__ z, const double* __restrict__ pold,
                                                 double* __restrict__ pnew, double* __restrict__ xe,
                                                 const uint8_t* __restrict__ fix, const int32_t* __restrict__ hang_of,
                                                 const int32_t* __restrict__ hptr, const int32_t* __restrict__ hm,
                                                 const double* __restrict__ hw, int nn, const double* __restrict__ part,
                                                 double* __restrict__ scal, int it) {
  __shared__ double sh[8];
  double beta = 0.0;
  if (scal) {  // CG step: beta from the r.z partials of the previous update
    const double done = scal[PS_DONE];
    const double rz = sum_partials(part, P_RED, sh);
    if (done != 0.0) return;
    beta = it == 0 ? 0.0 : rz / scal[PS_RZ0 + ((it - 1) & 1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[PS_RZ0 + (it & 1)] = rz;
  }
  const double* po = scal && it > 0 ? pold : nullptr;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += gridDim.x * blockDim.x) {
    const int h = hang_of[v];
    for (int c = 0; c < 2; ++c) {
      double x;
      if (h < 0) {
        x = masked(z, po, beta, fix, v, c);
        if (pnew) pnew[2 * v + c] = x;
      } else {
        x = 0.0;
        for (int k = hptr[h]; k < hptr[h + 1]; ++k) x += hw[k] * masked(z, po, beta, fix, hm[k], c);
        if (pnew) pnew[2 * v + c] = 0.0;
      }
      xe[2 * v + c] = x;
    }
  }
}

// pass 2: element outputs y_e = c_e K0 u_e
__global__ __launch_bounds__(256) void k2_elem(const double* __restrict__ xe, const int32_t* __restrict__ elem,
                                               const double* __restrict__ coef, const double* __restrict__ K0g,
                                               double* __restrict__ E, int ne, const double* __restrict__ scal) {
  __shared__ double K0[64];
  if (threadIdx.x < 64) K0[threadIdx.x] = K0g[threadIdx.x];
  __syncthreads();
  if (scal && scal[PS_DONE] != 0.0) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double u[8];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int v = elem[4 * e + a];
    u[2 * a] = xe[2 * v];
    u[2 * a + 1] = xe[2 * v + 1];
  }
  const double ce = coef[e];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s = fma(K0[r * 8 + k], u[k], s);
    E[8 * e + r] = ce * s;
  }
}

// pass 3: y = A~ x per node, fixed order over the incidences; with pq,
// q = A~ p (p in x) and the p.q partials
__global__ __launch_bounds__(256) void k2_gather(const double* __restrict__ E, const int32_t* __restrict__ iptr,
                                                 const int32_t* __restrict__ islot, const double* __restrict__ iw,
                                                 const uint8_t* __restrict__ fix, const double* __restrict__ x,
                                                 double* __restrict__ y, int nn, double* __restrict__ part_pq,
                                                 const double* __restrict__ scal) {
  __shared__ double sh[8];
  if (scal && scal[PS_DONE] != 0.0) return;
  double pq = 0.0;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += gridDim.x * blockDim.x) {
    double s0 = 0.0, s1 = 0.0;
    for (int k = iptr[v]; k < iptr[v + 1]; ++k) {
      const int sl = islot[k];
      const double w = iw[k];
      s0 = fma(w, E[2 * sl], s0);
      s1 = fma(w, E[2 * sl + 1], s1);
    }
    const uint8_t f = fix[v];
    const bool hang = (f >> 2) & 1;
    const double y0 = (hang || (f & 1)) ? (part_pq ? 0.0 : x[2 * v]) : s0;
    const double y1 = (hang || (f & 2)) ? (part_pq ? 0.0 : x[2 * v + 1]) : s1;
    y[2 * v] = y0;
    y[2 * v + 1] = y1;
    if (part_pq) pq += x[2 * v] * y0 + x[2 * v + 1] * y1;
  }
  if (part_pq) {
    pq = block_sum(pq, sh);
    if (threadIdx.x == 0) part_pq[blockIdx.x] = pq;
  }
}

// exact diagonal of A~: per node and component, sum over the node's
// incidences grouped by element of c_e t_a t_b K0[2a+c][2b+c]
__global__ __launch_bounds__(256) void k2_diag(const int32_t* __restrict__ iptr, const int32_t* __restrict__ islot,
                                               const double* __restrict__ iw, const double* __restrict__ coef,
                                               const double* __restrict__ K0g, const uint8_t* __restrict__ fix,
                                               double* __restrict__ dinv, int nn) {
  __shared__ double K0[64];
  if (threadIdx.x < 64) K0[threadIdx.x] = K0g[threadIdx.x];
  __syncthreads();
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  double d[2] = {0.0, 0.0};
  const int k1 = iptr[v + 1];
  for (int k = iptr[v]; k < k1;) {
    const int e = islot[k] >> 2;
    int kk = k;
    double t[4] = {0, 0, 0, 0};
    while (kk < k1 && (islot[kk] >> 2) == e) {
      t[islot[kk] & 3] += iw[kk];
      ++kk;
    }
    const double ce = coef[e];
    for (int c = 0; c < 2; ++c) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) s += t[a] * t[b] * K0[(2 * a + c) * 8 + 2 * b + c];
      d[c] += ce * s;
    }
    k = kk;
  }
  const uint8_t f = fix[v];
  for (int c = 0; c < 2; ++c) dinv[2 * v + c] = (((f >> 2) & 1) || ((f >> c) & 1)) ? 1.0 : 1.0 / d[c];
}

__device__ __forceinline__ bool constrained(const uint8_t* __restrict__ fix, long i) {
  const uint8_t f = fix[i >> 1];
  return ((f >> 2) & 1) || ((f >> (i & 1)) & 1);
}

// r = b - q with supported and hanging rows zero, z = D^-1 r; partials r.z, r.r, b.b
__global__ __launch_bounds__(256) void k2_init(const double* __restrict__ b, const double* __restrict__ q,
                                               const double* __restrict__ dinv, const uint8_t* __restrict__ fix,
                                               double* __restrict__ r, double* __restrict__ z, long n,
                                               double* __restrict__ part) {
  __shared__ double sh[8];
  double rz = 0, rr = 0, bb = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const bool cs = constrained(fix, i);
    const double bi = cs ? 0.0 : b[i];
    const double ri = cs ? 0.0 : bi - q[i], zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    rz += ri * zi;
    rr += ri * ri;
    bb += bi * bi;
  }
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rz;
    part[P_RED + blockIdx.x] = rr;
    part[2 * P_RED + blockIdx.x] = bb;
  }
}

__global__ __launch_bounds__(256) void k2_init_scalars(const double* __restrict__ part, double* __restrict__ scal,
                                                       double tol2) {
  __shared__ double sh[8];
  const double rz = sum_partials(part, P_RED, sh), rr = sum_partials(part + P_RED, P_RED, sh), bb = sum_partials(part + 2 * P_RED, P_RED, sh);
  if (threadIdx.x == 0) {
    scal[PS_BB] = bb;
    scal[PS_RZ0] = scal[PS_RZ1] = rz;
    scal[PS_RR] = rr;
    scal[PS_ITERS] = 0.0;
    scal[PS_DONE] = (rr <= tol2 * bb) ? 1.0 : ((rr == rr && rr < 1e300) ? 0.0 : 2.0);
  }
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; z = D^-1 r; partials r.z, r.r
__global__ __launch_bounds__(256) void k2_update(double* __restrict__ x, double* __restrict__ r,
                                                 const double* __restrict__ p, const double* __restrict__ q,
                                                 const double* __restrict__ dinv, double* __restrict__ z, long n,
                                                 const double* __restrict__ part_pq, double* __restrict__ part,
                                                 double* __restrict__ scal, int it) {
  __shared__ double sh[8];
  const double done = scal[PS_DONE];
  const double pq = sum_partials(part_pq, P_RED, sh);
  if (done != 0.0) return;
  const double rz = scal[PS_RZ0 + (it & 1)];
  if (!(pq > 0.0) || !(pq < 1e300)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[PS_DONE] = 2.0;
    return;
  }
  const double alpha = rz / pq;
  double srz = 0, srr = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i], zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    srz += ri * zi;
    srr += ri * ri;
  }
  srz = block_sum(srz, sh);
  srr = block_sum(srr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[P_RED + blockIdx.x] = srr;
  }
}

// convergence test on r.r of the update just finished (one block)
__global__ __launch_bounds__(256) void k2_check(const double* __restrict__ part, double* __restrict__ scal, int it,
                                                double tol2) {
  __shared__ double sh[8];
  const double rr = sum_partials(part + P_RED, P_RED, sh);
  if (threadIdx.x != 0 || scal[PS_DONE] != 0.0) return;
  scal[PS_RR] = rr;
  scal[PS_ITERS] = it + 1;
  if (!(rr == rr) || rr > 1e300) scal[PS_DONE] = 2.0;
  else if (rr <= tol2 * scal[PS_BB]) scal[PS_DONE] = 1.0;
}

// true residual partials r.r and b.b of b - A~ x (q = A~ x) over the unconstrained rows
__global__ __launch_bounds__(256) void k2_resid(const double* __restrict__ b, const double* __restrict__ q,
                                                const uint8_t* __restrict__ fix, long n, double* __restrict__ part) {
  __shared__ double sh[8];
  double rr = 0, bb = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    if (constrained(fix, i)) continue;
    const double ri = b[i] - q[i];
    rr += ri * ri;
    bb += b[i] * b[i];
  }
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[P_RED + blockIdx.x] = rr;
    part[2 * P_RED + blockIdx.x] = bb;
  }
}

__global__ __launch_bounds__(256) void k2_sums(const double* __restrict__ part, int off, double* __restrict__ out) {
  __shared__ double sh[8];
  const double a = sum_partials(part + off, P_RED, sh), b = sum_partials(part + off + P_RED, P_RED, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

// b = F T^T f: condense hanging loads onto masters (each hanging node adds to
// its masters through the incidence-free hanging CSR), zero constrained rows
__global__ __launch_bounds__(256) void k2_rhs(const double* __restrict__ f, double* __restrict__ b,
                                              const uint8_t* __restrict__ fix, const int32_t* __restrict__ mptr,
                                              const int32_t* __restrict__ mh, const double* __restrict__ mw, int nn) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  const uint8_t fl = fix[v];
  for (int c = 0; c < 2; ++c) {
    double s = f[2 * v + c];
    for (int k = mptr[v]; k < mptr[v + 1]; ++k) s += mw[k] * f[2 * mh[k] + c];
    b[2 * v + c] = (((fl >> 2) & 1) || ((fl >> c) & 1)) ? 0.0 : s;
  }
}

// u_h = sum w u_m at hanging nodes (Eq. (9)), in place
__global__ __launch_bounds__(256) void k2_recover(double* __restrict__ u, const int32_t* __restrict__ hang_node,
                                                  const int32_t* __restrict__ hptr, const int32_t* __restrict__ hm,
                                                  const double* __restrict__ hw, int nh) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nh) return;
  for (int c = 0; c < 2; ++c) {
    double s = 0.0;
    for (int k = hptr[h]; k < hptr[h + 1]; ++k) s += hw[k] * u[2 * hm[k] + c];
    u[2 * hang_node[h] + c] = s;
  }
}

// dc_e = -p rho^(p-1) (E0 - Emin) u_e^T K0 u_e (element mean removed first)
__global__ __launch_bounds__(256) void k2_sens(const double* __restrict__ u, const double* __restrict__ rho,
                                               const int32_t* __restrict__ elem, const double* __restrict__ K0g,
                                               double* __restrict__ dc, int ne, double dE, double p) {
  __shared__ double K0[64];
  if (threadIdx.x < 64) K0[threadIdx.x] = K0g[threadIdx.x];
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double ue[8];
  for (int a = 0; a < 4; ++a) {
    const int v = elem[4 * e + a];
    ue[2 * a] = u[2 * v];
    ue[2 * a + 1] = u[2 * v + 1];
  }
  for (int c = 0; c < 2; ++c) {
    const double m = 0.25 * (ue[c] + ue[2 + c] + ue[4 + c] + ue[6 + c]);
    for (int a = 0; a < 4; ++a) ue[2 * a + c] -= m;
  }
  double w = 0.0;
  for (int r = 0; r < 8; ++r) {
    double s = 0.0;
    for (int k = 0; k < 8; ++k) s = fma(K0[r * 8 + k], ue[k], s);
    w = fma(ue[r], s, w);
  }
  dc[e] = -p * pow(rho[e], p - 1.0) * dE * w;
}

__global__ __launch_bounds__(256) void k2_dot(const double* __restrict__ a, const double* __restrict__ b, long n,
                                              double* __restrict__ part) {
  __shared__ double sh[8];
  double s = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) s += a[i] * b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Eq. (5) filter with area weights: per leaf size, the aligned anchors a
// neighbour of that size can have (|2 a + h - c| < 2 rmin per axis) are
// probed in the lattice map; each leaf counts once, at its anchor cell
__global__ __launch_bounds__(256) void k2_filter(const double* __restrict__ in, const double* __restrict__ rho,
                                                 double* __restrict__ out, const int32_t* __restrict__ desc,
                                                 const int32_t* __restrict__ cmap, int n, int nx, int ny, int hmax,
                                                 double rmin, int mode) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int cx = 2 * desc[3 * e] + desc[3 * e + 2], cy = 2 * desc[3 * e + 1] + desc[3 * e + 2];
  const double r2 = 2.0 * rmin, lim2 = r2 * r2;
  double num = 0.0, den = 0.0;
  for (int h = 1; h <= hmax; h <<= 1) {
    auto lo = [&](int c) { return max(0, (int)ceil(0.5 * ((double)(c - h) - r2) / h) * h); };
    auto hi = [&](int c, int m) { return min(m - h, (int)floor(0.5 * ((double)(c - h) + r2) / h) * h); };
    const int x0 = lo(cx), x1 = hi(cx, nx), y0 = lo(cy), y1 = hi(cy, ny);
    for (int y = y0; y <= y1; y += h)
      for (int x = x0; x <= x1; x += h) {
        const int v = cmap[(long)nx * y + x];
        if (v >= 0) continue;
        const int d = v & 0x7fffffff;
        if (desc[3 * d + 2] != h) continue;
        const double dx = (double)(2 * desc[3 * d] + h - cx), dy = (double)(2 * desc[3 * d + 1] + h - cy);
        const double D2 = dx * dx + dy * dy;
        if (D2 >= lim2) continue;
        const double H = rmin - 0.5 * sqrt(D2);
        if (H <= 0.0) continue;
        const double w = H * (double)h * h;
        num += w * (mode == AMRTO_FILTER_SENSITIVITY ? rho[d] * in[d] : in[d]);
        den += w;
      }
  }
  out[e] = mode == AMRTO_FILTER_SENSITIVITY ? num / (fmax(rho[e], 1e-3) * den) : num / den;
}

__global__ __launch_bounds__(256) void k2_cmap(const int32_t* __restrict__ desc, int n, int nx,
                                               int32_t* __restrict__ cmap) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int ax = desc[3 * e], ay = desc[3 * e + 1], h = desc[3 * e + 2];
    for (int j = 0; j < h; ++j)
      for (int i = 0; i < h; ++i)
        cmap[(long)nx * (ay + j) + ax + i] = (i | j) ? e : (int32_t)((uint32_t)e | 0x80000000u);
  }
}

// OC: volume of P_OCK candidate multipliers per pass (log-spaced in the
// bracket), one bracket update per pass, then the update at the bracket's
// midpoint; rho (g / lam)^eta = (rho g^eta) lam^-eta
__global__ __launch_bounds__(P_OCK) void k2_oc_vol(const double* __restrict__ rho, const double* __restrict__ dc,
                                                   const double* __restrict__ area, int n, double eta, double move,
                                                   double rmin, double* __restrict__ ws) {
  __shared__ double srg[64], slo[64], shi[64], sv[64];
  const double llo = ws[0], lhi = ws[1];
  const int j = threadIdx.x;
  const double lam = exp(llo + (lhi - llo) * (double)j / (double)(P_OCK - 1));
  const double il = pow(lam, -eta);
  double acc = 0.0;
  for (int base = blockIdx.x * 64; base < n; base += gridDim.x * 64) {
    __syncthreads();
    if (j < 64 && base + j < n) {
      const int e = base + j;
      const double r = rho[e], g = fmax(-dc[e], 0.0) / area[e];
      srg[j] = r * pow(g, eta);
      slo[j] = fmax(rmin, r - move);
      shi[j] = fmin(1.0, r + move);
      sv[j] = area[e];
    }
    __syncthreads();
    const int m = min(64, n - base);
    for (int t = 0; t < m; ++t) acc += fmin(fmax(srg[t] * il, slo[t]), shi[t]) * sv[t];
  }
  ws[2 + (long)j * gridDim.x + blockIdx.x] = acc;
}

__global__ __launch_bounds__(P_OCK) void k2_oc_bracket(double* __restrict__ ws, int nb, double v0) {
  __shared__ double sv[P_OCK];
  const int j = threadIdx.x;
  double v = 0.0;
  for (int b = 0; b < nb; ++b) v += ws[2 + (long)j * nb + b];
  sv[j] = v;
  __syncthreads();
  if (j == 0) {
    const double llo = ws[0], lhi = ws[1];
    int jl = -1;
    for (int t = 0; t < P_OCK; ++t)
      if (sv[t] > v0) jl = t;
    if (jl < 0) ws[1] = llo;
    else if (jl == P_OCK - 1) ws[0] = lhi;
    else {
      ws[0] = llo + (lhi - llo) * (double)jl / (double)(P_OCK - 1);
      ws[1] = llo + (lhi - llo) * (double)(jl + 1) / (double)(P_OCK - 1);
    }
  }
}

__global__ __launch_bounds__(256) void k2_oc_apply(const double* __restrict__ rho, const double* __restrict__ dc,
                                                   const double* __restrict__ area, int n, double eta, double move,
                                                   double rmin, double* __restrict__ out, double* __restrict__ ws) {
  __shared__ double sh[8];
  const double lam = exp(0.5 * (ws[0] + ws[1]));
  double ch = 0.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const double g = fmax(-dc[e], 0.0) / area[e];
    const double r = fmin(fmax(rho[e] * pow(g / lam, eta), fmax(rmin, rho[e] - move)), fmin(1.0, rho[e] + move));
    ch = fmax(ch, fabs(r - rho[e]));
    out[e] = r;
  }
  // block maximum (all threads take part)
  for (int off = 32; off > 0; off >>= 1) ch = fmax(ch, __shfl_down(ch, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ch;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, sh[w]);
    ws[2 + blockIdx.x] = m;
  }
}

__global__ void k2_oc_finish(double* __restrict__ ws, int nb) {
  double m = 0.0;
  for (int b = 0; b < nb; ++b) m = fmax(m, ws[2 + b]);
  ws[2] = m;
  ws[3] = exp(0.5 * (ws[0] + ws[1]));
}

__global__ void k2_bracket_init(double* ws, double lo, double hi) {
  ws[0] = lo;
  ws[1] = hi;
}

template <typename T>
static hipError_t pl_alloc(T*& p, size_t n) {
  if (p) (void)hipFree(p);
  p = nullptr;
  return hipMalloc((void**)&p, std::max<size_t>(1, n) * sizeof(T));
}
template <typename T>
static void pl_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

static void free_mesh(amrto_plane* pl) {
  pl_free(pl->d_elem); pl_free(pl->d_fix); pl_free(pl->d_hang_of); pl_free(pl->d_hang_ptr);
  pl_free(pl->d_hang_master); pl_free(pl->d_hang_w); pl_free(pl->d_inc_ptr); pl_free(pl->d_inc_slot);
  pl_free(pl->d_inc_w); pl_free(pl->d_area); pl_free(pl->d_edesc); pl_free(pl->d_cmap); pl_free(pl->d_coef);
  pl_free(pl->d_dinv); pl_free(pl->d_E); pl_free(pl->d_xe); pl_free(pl->d_r); pl_free(pl->d_z); pl_free(pl->d_p);
  pl_free(pl->d_p2); pl_free(pl->d_q); pl_free(pl->d_hang_node); pl_free(pl->d_rhs_ptr); pl_free(pl->d_rhs_h);
  pl_free(pl->d_rhs_w);
  pl->n_hang = 0;
  pl->has_mesh = pl->has_density = false;
}

// y = A~ x (three passes)
static int plane_apply(amrto_plane* pl, const double* x, double* y) {
  const int nn = pl->n_nodes, ne = pl->n_elems;
  hipLaunchKernelGGL(k2_expand, dim3(grid_for(nn, 256, 4096)), dim3(256), 0, pl->stream, x, (const double*)nullptr,
                     (double*)nullptr, pl->d_xe, pl->d_fix, pl->d_hang_of, pl->d_hang_ptr, pl->d_hang_master,
                     pl->d_hang_w, nn, (const double*)nullptr, (double*)nullptr, 0);
  hipLaunchKernelGGL(k2_elem, dim3((ne + 255) / 256), dim3(256), 0, pl->stream, pl->d_xe, pl->d_elem, pl->d_coef,
                     pl->d_K0, pl->d_E, ne, (const double*)nullptr);
  hipLaunchKernelGGL(k2_gather, dim3(grid_for(nn, 256, 4096)), dim3(256), 0, pl->stream, pl->d_E, pl->d_inc_ptr,
                     pl->d_inc_slot, pl->d_inc_w, pl->d_fix, x, y, nn, (double*)nullptr, (const double*)nullptr);
  PL_HIP(hipGetLastError());
  return AMRTO_OK;
}

}  // namespace amrto

extern "C" {

int amrto_plane_create(amrto_plane** out, int device, void* stream) {
  if (!out) return AMRTO_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return AMRTO_EINVAL;
  amrto_plane* pl = new (std::nothrow) amrto_plane();
  if (!pl) return AMRTO_ENOMEM;
  pl->device = device;
  pl->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess || hipMalloc((void**)&pl->d_K0, 64 * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&pl->d_part, 4 * P_RED * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&pl->d_scal, PS_COUNT * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&pl->d_oc, (2 + P_OCK * P_OCB + 64) * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&pl->h_scal, PS_COUNT * sizeof(double)) != hipSuccess) {
    amrto_plane_destroy(pl);
    return AMRTO_ENOMEM;
  }
  k0_unit_square(pl->nu, pl->K0);
  if (hipMemcpy(pl->d_K0, pl->K0, sizeof(pl->K0), hipMemcpyHostToDevice) != hipSuccess) {
    amrto_plane_destroy(pl);
    return AMRTO_EHIP;
  }
  *out = pl;
  return AMRTO_OK;
}

int amrto_plane_destroy(amrto_plane* pl) {
  if (!pl) return AMRTO_OK;
  (void)hipSetDevice(pl->device);
  (void)hipStreamSynchronize(pl->stream);
  free_mesh(pl);
  pl_free(pl->d_K0); pl_free(pl->d_part); pl_free(pl->d_scal); pl_free(pl->d_oc);
  if (pl->h_scal) (void)hipHostFree(pl->h_scal);
  delete pl;
  return AMRTO_OK;
}

const char* amrto_plane_last_error(const amrto_plane* pl) { return pl ? pl->err.c_str() : "null context"; }

int amrto_plane_set_material(amrto_plane* pl, double E0, double Emin, double nu, double p) {
  if (!pl) return AMRTO_EINVAL;
  if (!(E0 > Emin) || !(Emin >= 0.0) || !(nu > -1.0 && nu < 0.5) || !(p >= 1.0))
    return pl->fail(AMRTO_EINVAL, "amrto_plane_set_material: need E0 > Emin >= 0, -1 < nu < 0.5, p >= 1");
  PL_HIP(hipSetDevice(pl->device));
  pl->E0 = E0; pl->Emin = Emin; pl->nu = nu; pl->p = p;
  k0_unit_square(nu, pl->K0);
  PL_HIP(hipMemcpyAsync(pl->d_K0, pl->K0, sizeof(pl->K0), hipMemcpyHostToDevice, pl->stream));
  PL_HIP(hipStreamSynchronize(pl->stream));
  pl->has_density = false;
  return AMRTO_OK;
}

int amrto_plane_upload_mesh(amrto_plane* pl, const amrto_mesh2d* m) {
  if (!pl) return AMRTO_EINVAL;
  if (!m || m->n_nodes <= 0 || m->n_elems <= 0 || !m->node_xy || !m->elem_nodes || !m->dof_fixed ||
      m->dims[0] <= 0 || m->dims[1] <= 0 || m->max_level < 0 || m->max_level > 20 || m->n_hang < 0 ||
      (m->n_hang > 0 && (!m->hang_node || !m->hang_ptr || !m->hang_master || !m->hang_w)))
    return pl->fail(AMRTO_EINVAL, "amrto_plane_upload_mesh: bad mesh");
  if (2L * m->n_nodes > 2147483647L || 8L * m->n_elems > 2147483647L || (long)m->dims[0] * m->dims[1] > (1L << 30))
    return pl->fail(AMRTO_EINVAL, "amrto_plane_upload_mesh: mesh too large");
  const int nn = m->n_nodes, ne = m->n_elems;
  for (long i = 0; i < 4L * ne; ++i)
    if (m->elem_nodes[i] < 0 || m->elem_nodes[i] >= nn)
      return pl->fail(AMRTO_EINVAL, "amrto_plane_upload_mesh: element node index out of range");
  std::vector<int8_t> lev(ne, (int8_t)m->max_level);
  if (m->elem_level) std::memcpy(lev.data(), m->elem_level, ne);
  for (int8_t l : lev)
    if (l < 0 || l > m->max_level) return pl->fail(AMRTO_EINVAL, "amrto_plane_upload_mesh: element level out of range");
  std::vector<int32_t> hang_of(nn, -1);
  for (int h = 0; h < m->n_hang; ++h) {
    const int v = m->hang_node[h];
    if (v < 0 || v >= nn || m->hang_ptr[h] > m->hang_ptr[h + 1])
      return pl->fail(AMRTO_EINVAL, "amrto_plane_upload_mesh: bad hanging table");
    hang_of[v] = h;
  }
  const int nent = m->n_hang ? m->hang_ptr[m->n_hang] : 0;
  for (int k = 0; k < nent; ++k)
    if (m->hang_master[k] < 0 || m->hang_master[k] >= nn || hang_of[m->hang_master[k]] >= 0)
      return pl->fail(AMRTO_EINVAL, "amrto_plane_upload_mesh: a hanging master is out of range or hanging");
  PL_HIP(hipSetDevice(pl->device));
  PL_HIP(hipStreamSynchronize(pl->stream));
  free_mesh(pl);
  pl->n_nodes = nn; pl->n_elems = ne; pl->max_level = m->max_level; pl->nx = m->dims[0]; pl->ny = m->dims[1];
  pl->h_level = lev;
  std::vector<uint8_t> fix(nn, 0);
  for (int v = 0; v < nn; ++v)
    fix[v] = (uint8_t)((m->dof_fixed[2 * v] ? 1 : 0) | (m->dof_fixed[2 * v + 1] ? 2 : 0) | (hang_of[v] >= 0 ? 4 : 0));
  // incidences: own vertices (weight 1) and vertices hanging on the node
  std::vector<std::vector<std::pair<int32_t, double>>> inc(nn);
  std::vector<int32_t> desc(3L * ne);
  std::vector<double> area(ne);
  int hmax = 1;
  for (int e = 0; e < ne; ++e) {
    const int h = 1 << (m->max_level - lev[e]);
    hmax = std::max(hmax, h);
    area[e] = (double)h * h;
    const int n0 = m->elem_nodes[4L * e];
    desc[3L * e] = m->node_xy[2L * n0];
    desc[3L * e + 1] = m->node_xy[2L * n0 + 1];
    desc[3L * e + 2] = h;
    if (desc[3L * e] < 0 || desc[3L * e + 1] < 0 || desc[3L * e] + h > m->dims[0] || desc[3L * e + 1] + h > m->dims[1])
      return pl->fail(AMRTO_EINVAL, "amrto_plane_upload_mesh: element outside the lattice box");
    for (int a = 0; a < 4; ++a) {
      const int v = m->elem_nodes[4L * e + a];
      const int32_t slot = 4 * e + a;
      if (hang_of[v] < 0) {
        inc[v].push_back({slot, 1.0});
      } else {
        const int hh = hang_of[v];
        for (int k = m->hang_ptr[hh]; k < m->hang_ptr[hh + 1]; ++k) inc[m->hang_master[k]].push_back({slot, m->hang_w[k]});
      }
    }
  }
  pl->hmax = hmax;
  std::vector<int32_t> iptr(nn + 1, 0), islot;
  std::vector<double> iw;
  for (int v = 0; v < nn; ++v) {
    std::sort(inc[v].begin(), inc[v].end());
    for (const auto& sw : inc[v]) {
      islot.push_back(sw.first);
      iw.push_back(sw.second);
    }
    iptr[v + 1] = (int32_t)islot.size();
  }
  // masters' view of the hanging loads for the right-hand side: per node the
  // hanging nodes it masters with their weights
  std::vector<std::vector<std::pair<int32_t, double>>> mastered(nn);
  for (int h = 0; h < m->n_hang; ++h)
    for (int k = m->hang_ptr[h]; k < m->hang_ptr[h + 1]; ++k)
      mastered[m->hang_master[k]].push_back({m->hang_node[h], m->hang_w[k]});
  std::vector<int32_t> mptr(nn + 1, 0), mh;
  std::vector<double> mw;
  for (int v = 0; v < nn; ++v) {
    for (const auto& hw : mastered[v]) {
      mh.push_back(hw.first);
      mw.push_back(hw.second);
    }
    mptr[v + 1] = (int32_t)mh.size();
  }
  auto up = [&](auto*& dst, const auto& v) -> hipError_t {
    using T = typename std::remove_reference<decltype(v)>::type::value_type;
    hipError_t er = pl_alloc(dst, v.size());
    if (er == hipSuccess && !v.empty()) er = hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return er;
  };
  std::vector<int32_t> elem(m->elem_nodes, m->elem_nodes + 4L * ne);
  std::vector<int32_t> hptr(m->hang_ptr ? m->hang_ptr : nullptr, m->hang_ptr ? m->hang_ptr + m->n_hang + 1 : nullptr);
  if (hptr.empty()) hptr.push_back(0);
  std::vector<int32_t> hmv(m->hang_master ? m->hang_master : nullptr, m->hang_master ? m->hang_master + nent : nullptr);
  std::vector<double> hwv(m->hang_w ? m->hang_w : nullptr, m->hang_w ? m->hang_w + nent : nullptr);
  std::vector<int32_t> hnode(m->hang_node ? m->hang_node : nullptr, m->hang_node ? m->hang_node + m->n_hang : nullptr);
  PL_HIP(up(pl->d_elem, elem));
  PL_HIP(up(pl->d_fix, fix));
  PL_HIP(up(pl->d_hang_of, hang_of));
  PL_HIP(up(pl->d_hang_ptr, hptr));
  PL_HIP(up(pl->d_hang_master, hmv));
  PL_HIP(up(pl->d_hang_w, hwv));
  PL_HIP(up(pl->d_inc_ptr, iptr));
  PL_HIP(up(pl->d_inc_slot, islot));
  PL_HIP(up(pl->d_inc_w, iw));
  PL_HIP(up(pl->d_area, area));
  PL_HIP(up(pl->d_edesc, desc));
  PL_HIP(up(pl->d_rhs_ptr, mptr));
  PL_HIP(up(pl->d_rhs_h, mh));
  PL_HIP(up(pl->d_rhs_w, mw));
  PL_HIP(up(pl->d_hang_node, hnode));
  pl->n_hang = m->n_hang;
  PL_HIP(pl_alloc(pl->d_cmap, (size_t)pl->nx * pl->ny));
  hipLaunchKernelGGL(k2_cmap, dim3(grid_for(ne, 256, 4096)), dim3(256), 0, pl->stream, (const int32_t*)pl->d_edesc, ne,
                     pl->nx, pl->d_cmap);
  PL_HIP(hipGetLastError());
  PL_HIP(pl_alloc(pl->d_coef, ne));
  PL_HIP(pl_alloc(pl->d_dinv, 2L * nn));
  PL_HIP(pl_alloc(pl->d_E, 8L * ne));
  PL_HIP(pl_alloc(pl->d_xe, 2L * nn));
  PL_HIP(pl_alloc(pl->d_r, 2L * nn)); PL_HIP(pl_alloc(pl->d_z, 2L * nn));
  PL_HIP(pl_alloc(pl->d_p, 2L * nn)); PL_HIP(pl_alloc(pl->d_p2, 2L * nn)); PL_HIP(pl_alloc(pl->d_q, 2L * nn));
  PL_HIP(hipStreamSynchronize(pl->stream));
  pl->has_mesh = true;
  return AMRTO_OK;
}

int amrto_plane_set_density(amrto_plane* pl, const double* rho) {
  if (!pl) return AMRTO_EINVAL;
  if (!pl->has_mesh) return pl->fail(AMRTO_ESTATE, "amrto_plane_set_density: no mesh");
  if (!rho) return pl->fail(AMRTO_EINVAL, "amrto_plane_set_density: NULL rho");
  PL_HIP(hipSetDevice(pl->device));
  hipLaunchKernelGGL(k2_coef, dim3((pl->n_elems + 255) / 256), dim3(256), 0, pl->stream, rho, pl->d_coef, pl->n_elems,
                     pl->E0, pl->Emin, pl->p);
  hipLaunchKernelGGL(k2_diag, dim3((pl->n_nodes + 255) / 256), dim3(256), 0, pl->stream, pl->d_inc_ptr, pl->d_inc_slot,
                     pl->d_inc_w, pl->d_coef, pl->d_K0, pl->d_fix, pl->d_dinv, pl->n_nodes);
  PL_HIP(hipGetLastError());
  pl->has_density = true;
  return AMRTO_OK;
}

int amrto_plane_apply(amrto_plane* pl, const double* x, double* y) {
  if (!pl) return AMRTO_EINVAL;
  if (!pl->has_density) return pl->fail(AMRTO_ESTATE, "amrto_plane_apply: density not set");
  if (!x || !y || x == y) return pl->fail(AMRTO_EINVAL, "amrto_plane_apply: x and y must be distinct");
  PL_HIP(hipSetDevice(pl->device));
  return plane_apply(pl, x, y);
}

int amrto_plane_project_rhs(amrto_plane* pl, const double* f, double* b) {
  if (!pl) return AMRTO_EINVAL;
  if (!pl->has_mesh) return pl->fail(AMRTO_ESTATE, "amrto_plane_project_rhs: no mesh");
  if (!f || !b || f == b) return pl->fail(AMRTO_EINVAL, "amrto_plane_project_rhs: f and b must be distinct");
  PL_HIP(hipSetDevice(pl->device));
  hipLaunchKernelGGL(k2_rhs, dim3((pl->n_nodes + 255) / 256), dim3(256), 0, pl->stream, f, b, pl->d_fix, pl->d_rhs_ptr,
                     pl->d_rhs_h, pl->d_rhs_w, pl->n_nodes);
  PL_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_plane_pcg(amrto_plane* pl, const double* b, double* u, double rtol, int32_t max_it, int32_t check_every,
                    amrto_solve_stats* stats) {
  if (!pl) return AMRTO_EINVAL;
  if (!pl->has_density) return pl->fail(AMRTO_ESTATE, "amrto_plane_pcg: density not set");
  if (!b || !u || b == u || !(rtol > 0.0) || max_it < 0 || check_every < 1)
    return pl->fail(AMRTO_EINVAL, "amrto_plane_pcg: bad arguments");
  PL_HIP(hipSetDevice(pl->device));
  const auto t0 = std::chrono::steady_clock::now();
  const int nn = pl->n_nodes, ne = pl->n_elems;
  const long n2 = 2L * nn;
  const double tol2 = rtol * rtol;
  // Each pass starts from the current iterate with r = b - A~ u recomputed
  // (residual replacement); a pass whose recurrence reports convergence is
  // judged by the true residual and, above rtol, restarted (at most 8 times).
  int total = 0, outer = 0, status = AMRTO_NOT_CONVERGED;
  double rel = 0.0;
  while (true) {
    // the iterate is u with supported and hanging entries zeroed (A~ keeps
    // them as identity rows of a zero right-hand side)
    hipLaunchKernelGGL(k2_expand, dim3(grid_for(nn, 256, 4096)), dim3(256), 0, pl->stream, u, (const double*)nullptr,
                       pl->d_p, pl->d_xe, pl->d_fix, pl->d_hang_of, pl->d_hang_ptr, pl->d_hang_master, pl->d_hang_w,
                       nn, (const double*)nullptr, (double*)nullptr, 0);
    PL_HIP(hipMemcpyAsync(u, pl->d_p, n2 * sizeof(double), hipMemcpyDeviceToDevice, pl->stream));
    int rc = plane_apply(pl, u, pl->d_q);
    if (rc) return rc;
    hipLaunchKernelGGL(k2_init, dim3(P_RED), dim3(256), 0, pl->stream, b, pl->d_q, pl->d_dinv, pl->d_fix, pl->d_r,
                       pl->d_z, n2, pl->d_part);
    hipLaunchKernelGGL(k2_init_scalars, dim3(1), dim3(256), 0, pl->stream, pl->d_part, pl->d_scal, tol2);
    int it = 0;
    double done = 0.0;
    while (true) {
      PL_HIP(hipMemcpyAsync(pl->h_scal, pl->d_scal, PS_COUNT * sizeof(double), hipMemcpyDeviceToHost, pl->stream));
      PL_HIP(hipStreamSynchronize(pl->stream));
      done = pl->h_scal[PS_DONE];
      if (done != 0.0) {
        it = (int)pl->h_scal[PS_ITERS];
        break;
      }
      if (total + it >= max_it) break;
      const int batch = std::min(check_every, max_it - total - it);
      for (int k = it; k < it + batch; ++k) {
        // p = z + beta p_old into the other buffer, xe = expanded p; q = A~ p; update
        double* pc = (k & 1) ? pl->d_p2 : pl->d_p;
        const double* po = (k & 1) ? pl->d_p : pl->d_p2;
        hipLaunchKernelGGL(k2_expand, dim3(grid_for(nn, 256, 4096)), dim3(256), 0, pl->stream, pl->d_z, po, pc,
                           pl->d_xe, pl->d_fix, pl->d_hang_of, pl->d_hang_ptr, pl->d_hang_master, pl->d_hang_w, nn,
                           pl->d_part, pl->d_scal, k);
        hipLaunchKernelGGL(k2_elem, dim3((ne + 255) / 256), dim3(256), 0, pl->stream, pl->d_xe, pl->d_elem,
                           pl->d_coef, pl->d_K0, pl->d_E, ne, pl->d_scal);
        hipLaunchKernelGGL(k2_gather, dim3(P_RED), dim3(256), 0, pl->stream, pl->d_E, pl->d_inc_ptr, pl->d_inc_slot,
                           pl->d_inc_w, pl->d_fix, pc, pl->d_q, nn, pl->d_part + 3 * P_RED, pl->d_scal);
        hipLaunchKernelGGL(k2_update, dim3(P_RED), dim3(256), 0, pl->stream, u, pl->d_r, pc, pl->d_q, pl->d_dinv,
                           pl->d_z, n2, pl->d_part + 3 * P_RED, pl->d_part, pl->d_scal, k);
        hipLaunchKernelGGL(k2_check, dim3(1), dim3(256), 0, pl->stream, pl->d_part, pl->d_scal, k, tol2);
      }
      PL_HIP(hipGetLastError());
      it += batch;
    }
    total += it;
    // true residual over the unconstrained rows
    rc = plane_apply(pl, u, pl->d_q);
    if (rc) return rc;
    hipLaunchKernelGGL(k2_resid, dim3(P_RED), dim3(256), 0, pl->stream, b, pl->d_q, pl->d_fix, n2, pl->d_part);
    hipLaunchKernelGGL(k2_sums, dim3(1), dim3(256), 0, pl->stream, pl->d_part, P_RED, pl->d_scal + PS_C);
    PL_HIP(hipGetLastError());
    PL_HIP(hipMemcpyAsync(pl->h_scal, pl->d_scal, PS_COUNT * sizeof(double), hipMemcpyDeviceToHost, pl->stream));
    PL_HIP(hipStreamSynchronize(pl->stream));
    rel = pl->h_scal[PS_C + 1] > 0 ? std::sqrt(pl->h_scal[PS_C] / pl->h_scal[PS_C + 1]) : 0.0;
    if (done == 2.0) {
      status = AMRTO_EBREAKDOWN;
      break;
    }
    if (rel <= rtol) {
      status = AMRTO_OK;
      break;
    }
    if (done != 1.0 || total >= max_it || outer >= 8) break;
    ++outer;
  }
  // hanging values from their masters (Eq. (9))
  if (pl->n_hang)
    hipLaunchKernelGGL(k2_recover, dim3((pl->n_hang + 255) / 256), dim3(256), 0, pl->stream, u, pl->d_hang_node,
                       pl->d_hang_ptr, pl->d_hang_master, pl->d_hang_w, pl->n_hang);
  PL_HIP(hipGetLastError());
  if (stats) {
    stats->iters = total;
    stats->outer = outer;
    stats->rel_res = rel;
    stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stats->fell_back = 0;
  }
  if (status == AMRTO_EBREAKDOWN) return pl->fail(AMRTO_EBREAKDOWN, "amrto_plane_pcg: breakdown");
  if (status == AMRTO_NOT_CONVERGED) pl->err = "amrto_plane_pcg: not converged";
  return status;
}

int amrto_plane_compliance(amrto_plane* pl, const double* u, const double* f, const double* rho, double* c_host,
                           double* dc) {
  if (!pl) return AMRTO_EINVAL;
  if (!pl->has_mesh) return pl->fail(AMRTO_ESTATE, "amrto_plane_compliance: no mesh");
  if (!u || (c_host && !f) || (dc && !rho)) return pl->fail(AMRTO_EINVAL, "amrto_plane_compliance: NULL buffer");
  PL_HIP(hipSetDevice(pl->device));
  if (dc)
    hipLaunchKernelGGL(k2_sens, dim3((pl->n_elems + 255) / 256), dim3(256), 0, pl->stream, u, rho, pl->d_elem, pl->d_K0,
                       dc, pl->n_elems, pl->E0 - pl->Emin, pl->p);
  if (c_host) {
    hipLaunchKernelGGL(k2_dot, dim3(P_RED), dim3(256), 0, pl->stream, f, u, 2L * pl->n_nodes, pl->d_part);
    hipLaunchKernelGGL(k2_sums, dim3(1), dim3(256), 0, pl->stream, pl->d_part, 0, pl->d_scal + PS_C);
    PL_HIP(hipMemcpyAsync(pl->h_scal, pl->d_scal, PS_COUNT * sizeof(double), hipMemcpyDeviceToHost, pl->stream));
    PL_HIP(hipStreamSynchronize(pl->stream));
    *c_host = pl->h_scal[PS_C];
  }
  PL_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_plane_filter(amrto_plane* pl, int mode, double rmin, const double* in, const double* rho, double* out) {
  if (!pl) return AMRTO_EINVAL;
  if (!pl->has_mesh) return pl->fail(AMRTO_ESTATE, "amrto_plane_filter: no mesh");
  if ((mode != AMRTO_FILTER_SENSITIVITY && mode != AMRTO_FILTER_DENSITY) || !(rmin > 0.0) || rmin > 16.0 || !in ||
      !out || in == out || (mode == AMRTO_FILTER_SENSITIVITY && !rho))
    return pl->fail(AMRTO_EINVAL, "amrto_plane_filter: bad arguments");
  PL_HIP(hipSetDevice(pl->device));
  hipLaunchKernelGGL(k2_filter, dim3((pl->n_elems + 255) / 256), dim3(256), 0, pl->stream, in, rho, out, pl->d_edesc,
                     pl->d_cmap, pl->n_elems, pl->nx, pl->ny, pl->hmax, rmin, mode);
  PL_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_plane_oc_update(amrto_plane* pl, const double* rho, const double* dc, double volfrac, double move, double eta,
                          double rho_min, double* rho_new, double* change_host, double* lam_host) {
  if (!pl) return AMRTO_EINVAL;
  if (!pl->has_mesh) return pl->fail(AMRTO_ESTATE, "amrto_plane_oc_update: no mesh");
  if (!rho || !dc || !rho_new || rho_new == rho || !(volfrac > 0.0 && volfrac <= 1.0) || !(move > 0.0) ||
      !(eta > 0.0) || !(rho_min >= 0.0 && rho_min < 1.0))
    return pl->fail(AMRTO_EINVAL, "amrto_plane_oc_update: bad arguments");
  PL_HIP(hipSetDevice(pl->device));
  const int ne = pl->n_elems;
  double atot = 0.0;
  for (int e = 0; e < ne; ++e) {
    const double h = (double)(1 << (pl->max_level - pl->h_level[e]));
    atot += h * h;
  }
  const int nb = std::min(P_OCB, (ne + 63) / 64);
  hipLaunchKernelGGL(k2_bracket_init, dim3(1), dim3(1), 0, pl->stream, pl->d_oc, std::log(1e-300), std::log(1e300));
  double width = std::log(1e300) - std::log(1e-300);
  while (width > 1e-14) {
    hipLaunchKernelGGL(k2_oc_vol, dim3(nb), dim3(P_OCK), 0, pl->stream, rho, dc, pl->d_area, ne, eta, move, rho_min,
                       pl->d_oc);
    hipLaunchKernelGGL(k2_oc_bracket, dim3(1), dim3(P_OCK), 0, pl->stream, pl->d_oc, nb, volfrac * atot);
    width /= (P_OCK - 1);
  }
  const int g = std::min(256, (ne + 255) / 256);
  hipLaunchKernelGGL(k2_oc_apply, dim3(g), dim3(256), 0, pl->stream, rho, dc, pl->d_area, ne, eta, move, rho_min,
                     rho_new, pl->d_oc);
  hipLaunchKernelGGL(k2_oc_finish, dim3(1), dim3(1), 0, pl->stream, pl->d_oc, g);
  PL_HIP(hipGetLastError());
  if (change_host || lam_host) {
    PL_HIP(hipMemcpyAsync(pl->h_scal, pl->d_oc, 4 * sizeof(double), hipMemcpyDeviceToHost, pl->stream));
    PL_HIP(hipStreamSynchronize(pl->stream));
    if (change_host) *change_host = pl->h_scal[2];
    if (lam_host) *lam_host = pl->h_scal[3];
  }
  return AMRTO_OK;
}

}  // extern "C"
