// Geometric multigrid on the octree hierarchy as the preconditioner of CG.
//
// The paper (Sec. 5) needs a strong preconditioner at the p = 3 stiffness
// contrast and uses IC(0) on the rescaled system; its triangular solves are
// sequential, so this library uses a V-cycle built from the mesh hierarchy
// the octree already has:
//
// * level 0 is the analysis mesh; level k <= L merges every leaf finer than
//   level L - k into its ancestor, levels k > L coarsen the uniform base grid
//   by two per axis (levels.h); levels are added until one has at most
//   coarse_dofs DOFs and is a uniform grid (no hanging nodes);
// * the prolongation evaluates the continuous level-k field (hanging values
//   from their masters) at the level k - 1 nodes, P = F_{k-1} I T_k F_k, and
//   the restriction is its transpose;
// * coarse operators are exactly Galerkin, A_k = P^T A_{k-1} P + (I - F_k),
//   assembled element by element: a level-k element that is a single level-0
//   leaf keeps c_e K0, every merged element stores the dense 24 x 24 sum
//   of its children's matrices mapped through the trilinear interpolation
//   from its corners to theirs;
// * smoothing is the Chebyshev iteration for D^-1 A on [hi / ratio, hi], hi
//   from power iteration, fused into the per-node pass that sums element
//   outputs (no atomics, fixed order); the coarsest level is solved with its
//   dense inverse (Gauss-Jordan, one workgroup).
//
// Vectors of every level are in the constrained form (zero at hanging and
// supported DOFs), 3 doubles per node.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "kernels.h"
#include "levels.h"

namespace amrto {

constexpr int MG_LMAX = 16;
constexpr int MG_COARSE_MAX = 1024;
constexpr int MG_RED = 256;  // partial sums of the multigrid kernels
// PCG scalars
enum { MC_RZ = 0, MC_BB = 1, MC_DONE = 2, MC_ITERS = 3, MC_RR = 4, MC_RES = 5, MC_COUNT = 8 };
enum MgMode { MG_APPLY = 0, MG_CHEB = 1, MG_CHEB_LAST = 2, MG_CORR = 3, MG_POWER = 4, MG_RAYLEIGH = 5 };

struct MgLevel {
  int nn = 0, ne = 0, nd = 0, nh = 0;  // nodes, elements, dense elements (first nd), hanging nodes
  int32_t* pure_src = nullptr;   // [ne - nd] index into the context's c_e
  double* Kd = nullptr;          // [576 nd] per element, column-major: entry (i, j) at 576 e + 24 j + i
  uint8_t* flag = nullptr;       // per node: bits 0-2 supported components, bit 3 hanging
  // assembled Galerkin operator: 3 x 3 block rows (supported columns zeroed;
  // hanging rows empty), rebuilt per density from contribution lists
  int nnzb = 0;
  int32_t* bptr = nullptr; int32_t* bcol = nullptr; int32_t* bdiag = nullptr; double* bval = nullptr;
  int32_t* kptr = nullptr; int32_t* ke = nullptr; uint8_t* kab = nullptr; double* kw = nullptr;
  int lanes = 4;                 // lanes per node in the block-row pass
  int rlanes = 4;                // lanes per node in the restriction to this level
  double* dinv = nullptr;        // owned except on level 0
  const double* binv = nullptr;  // level 0 with node-block smoothing: the inverse node blocks (6 per node)
  double *x = nullptr, *r = nullptr, *d = nullptr, *q = nullptr, *b = nullptr;
  double* scal = nullptr;        // MS_COUNT
  // coarse side of the transfer to the next finer level (this level k >= 1):
  int32_t* pptr = nullptr; int32_t* pcol = nullptr; double* pw = nullptr;  // rows: level k-1 nodes
  int32_t* rptr = nullptr; int32_t* rcol = nullptr; double* rw = nullptr;  // rows: level k nodes
  int32_t* cptr = nullptr; int32_t* celem = nullptr; uint8_t* coct = nullptr;  // children of dense elements
  double* Ainv = nullptr;        // coarsest level: dense inverse of A~ (3 nn x 3 nn)
  std::vector<void*> owned;
};

struct MgData {
  int nlev = 0;
  MgLevel lv[MG_LMAX];
  int degree = 2, coarse_degree = 2, power_its = 20;
  double ratio = 10.0, hi_factor = 1.1;
  bool blocks0 = false;          // level 0 smooths with the inverse node blocks
  bool user_bounds = false;
  double lam_user[MG_LMAX] = {};
  double* part = nullptr;   // 4 x MG_RED
  double* cg = nullptr;     // MC_COUNT
  double* h_cg = nullptr;   // pinned, S_COUNT >= MC_COUNT
  double *z = nullptr, *p = nullptr, *z2 = nullptr, *qv = nullptr;  // PCG vectors (p and z2: direction pair)
  double* cpart = nullptr;  // 2 x RED_BLOCKS partials of the fused CG
  double* cs = nullptr;     // S_COUNT scalars of the fused CG
  // P_o^T K0 P_o for every placement code o (256 x 576, row-major), the
  // Galerkin matrix of a unit-coefficient leaf placed by o; built for the
  // Poisson ratio in G_nu
  double* G = nullptr;
  double G_nu = -2.0;
  // the coarsest inverse runs beside the power iterations: a second stream
  // (default priority) forked from and joined to the context's by events
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<void*> owned;
};

void mg_free(amrto_ctx* ctx);

}  // namespace amrto

using namespace amrto;

namespace {

template <typename T>
hipError_t mg_alloc(std::vector<void*>& own, T*& p, size_t n) {
  p = nullptr;
  hipError_t e = hipMalloc((void**)&p, std::max<size_t>(n, 1) * sizeof(T));
  if (e == hipSuccess) own.push_back(p);
  return e;
}
template <typename T>
hipError_t mg_upload(std::vector<void*>& own, T*& p, const std::vector<T>& v) {
  hipError_t e = mg_alloc(own, p, v.size());
  if (e == hipSuccess && !v.empty()) e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

__device__ __forceinline__ bool mg_cons(uint8_t f, int c) { return ((f >> 3) & 1) || ((f >> c) & 1); }

// s[c] = sum over k in [k0, k1) of w[k] src[3 col[k] + c], in order, four
// entries' loads issued together
__device__ __forceinline__ void csr_gather3(const double* __restrict__ src, int k0, int k1,
                                            const int32_t* __restrict__ col, const double* __restrict__ w,
                                            double* s) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  int k = k0;
  for (; k + 4 <= k1; k += 4) {
    long c[4];
    double ww[4], v[12];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c[j] = col[k + j];
      ww[j] = w[k + j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) v[3 * j + q] = src[3 * c[j] + q];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      s0 = fma(ww[j], v[3 * j], s0);
      s1 = fma(ww[j], v[3 * j + 1], s1);
      s2 = fma(ww[j], v[3 * j + 2], s2);
    }
  }
  for (; k < k1; ++k) {
    const long c = col[k];
    const double ww = w[k];
    s0 = fma(ww, src[3 * c], s0);
    s1 = fma(ww, src[3 * c + 1], s1);
    s2 = fma(ww, src[3 * c + 2], s2);
  }
  s[0] = s0;
  s[1] = s1;
  s[2] = s2;
}

// LANES lanes per row: lane q sums entries k0 + q, k0 + q + LANES, ... in
// order; the lane sums are combined with xor shuffles in a fixed tree, so
// every lane of the row gets the same deterministic value
template <int LANES>
__device__ __forceinline__ void row_gather(const double* __restrict__ src, int k0, int k1,
                                           const int32_t* __restrict__ col, const double* __restrict__ w, int q,
                                           double& a0, double& a1, double& a2) {
  a0 = a1 = a2 = 0.0;
  for (int k = k0 + q; k < k1; k += LANES) {
    const long c = col[k];
    const double ww = w[k];
    a0 = fma(ww, src[3 * c], a0);
    a1 = fma(ww, src[3 * c + 1], a1);
    a2 = fma(ww, src[3 * c + 2], a2);
  }
#pragma unroll
  for (int o = 1; o < LANES; o <<= 1) {
    a0 += __shfl_xor(a0, o, 64);
    a1 += __shfl_xor(a1, o, 64);
    a2 += __shfl_xor(a2, o, 64);
  }
}

__device__ __forceinline__ void row_gather4(const double* __restrict__ src, int k0, int k1,
                                            const int32_t* __restrict__ col, const double* __restrict__ w, int q,
                                            double& a0, double& a1, double& a2) {
  row_gather<4>(src, k0, k1, col, w, q, a0, a1, a2);
}

__device__ __forceinline__ double pick3(int c, double a0, double a1, double a2) {
  return c == 0 ? a0 : (c == 1 ? a1 : a2);
}

struct MgUpd {
  int mode;
  int step;                 // Chebyshev step (MG_CHEB)
  const double* scal;       // MS_* of the level
  const double* dinv;
  const double* binv;       // set: node-block smoothing (level 0)
  double *x, *r, *d;
  double* dn;               // where the next direction goes (MG_CHEB, MG_CORR): d itself only
                            // when no thread of the pass reads other nodes' d
  const double* xin;        // MG_APPLY: identity rows; MG_POWER / MG_RAYLEIGH: iterate
  double* y;                // MG_APPLY / MG_POWER output
};

// per-DOF update after q = (A d)_i; returns the two Rayleigh terms in MG_RAYLEIGH
__device__ __forceinline__ void mg_update(const MgUpd& u, long i, bool cons, double q, double& t1, double& t2) {
  switch (u.mode) {
    case MG_APPLY:
      u.y[i] = cons ? u.xin[i] : q;
      break;
    case MG_CHEB: {
      const double sigma = u.scal[MS_SIGMA], delta = u.scal[MS_DELTA];
      double rho = 1.0 / sigma;
      for (int s = 0; s < u.step; ++s) rho = 1.0 / (2.0 * sigma - rho);
      const double rho1 = 1.0 / (2.0 * sigma - rho);
      if (cons) {
        u.x[i] = 0.0; u.r[i] = 0.0; u.dn[i] = 0.0;
      } else {
        const double dd = u.d[i];
        u.x[i] += dd;
        const double rr = u.r[i] - q;
        u.r[i] = rr;
        u.dn[i] = rho1 * rho * dd + (2.0 * rho1 / delta) * u.dinv[i] * rr;
      }
      break;
    }
    case MG_CHEB_LAST:
      if (cons) {
        u.x[i] = 0.0; u.r[i] = 0.0;
      } else {
        u.x[i] += u.d[i];
        u.r[i] -= q;
      }
      break;
    case MG_CORR: {
      const double rr = cons ? 0.0 : u.r[i] - q;
      u.r[i] = rr;
      u.dn[i] = u.dinv[i] * rr / u.scal[MS_THETA];
      break;
    }
    case MG_POWER:
      u.y[i] = cons ? 0.0 : u.dinv[i] * q;
      break;
    case MG_RAYLEIGH:
      if (!cons) {
        const double xi = u.xin[i];
        t1 += xi * q;
        t2 += xi * xi / u.dinv[i];
      }
      break;
  }
}

// z = M^-1 r at node v: the diagonal inverse, or with binv the inverse node
// block (six entries xx, yy, zz, xy, xz, yz)
__device__ __forceinline__ void mg_minv(const double* __restrict__ dinv, const double* __restrict__ binv, long v,
                                        const double (&r)[3], double (&z)[3]) {
  if (binv) {
    block_apply<double>(binv + 6 * v, r, z);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) z[c] = dinv[3 * v + c] * r[c];
  }
}

// y = B x at node v, B the node block itself (the inverse of the stored
// inverse, symmetric: cofactors over the determinant)
__device__ __forceinline__ void mg_bnode(const double* __restrict__ binv, long v, const double (&x)[3],
                                         double (&y)[3]) {
  const double* b = binv + 6 * v;
  const double a0 = b[0], a1 = b[1], a2 = b[2], a3 = b[3], a4 = b[4], a5 = b[5];
  const double c00 = a1 * a2 - a5 * a5, c01 = a4 * a5 - a3 * a2, c02 = a3 * a5 - a1 * a4;
  const double c11 = a0 * a2 - a4 * a4, c12 = a3 * a4 - a0 * a5, c22 = a0 * a1 - a3 * a3;
  const double inv_det = 1.0 / (a0 * c00 + a3 * c01 + a4 * c02);
  y[0] = (c00 * x[0] + c01 * x[1] + c02 * x[2]) * inv_det;
  y[1] = (c01 * x[0] + c11 * x[1] + c12 * x[2]) * inv_det;
  y[2] = (c02 * x[0] + c12 * x[1] + c22 * x[2]) * inv_det;
}

// the update of mode u.mode for the three components of node v after q = (A d)_v;
// with node blocks (u.binv) the modes that apply M^-1 work on the node at once
__device__ __forceinline__ void mg_update_node(const MgUpd& u, long v, uint8_t f, const double (&q)[3], double& t1,
                                               double& t2) {
  const bool blk = u.binv != nullptr &&
                   (u.mode == MG_CHEB || u.mode == MG_CORR || u.mode == MG_POWER || u.mode == MG_RAYLEIGH);
  if (!blk) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool cs = mg_cons(f, c);
      mg_update(u, 3 * v + c, cs, cs ? 0.0 : q[c], t1, t2);
    }
    return;
  }
  bool cs[3];
  double w[3], z[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) cs[c] = mg_cons(f, c);
  switch (u.mode) {
    case MG_CHEB: {
      const double sigma = u.scal[MS_SIGMA], delta = u.scal[MS_DELTA];
      double rho = 1.0 / sigma;
      for (int s = 0; s < u.step; ++s) rho = 1.0 / (2.0 * sigma - rho);
      const double rho1 = 1.0 / (2.0 * sigma - rho);
#pragma unroll
      for (int c = 0; c < 3; ++c) w[c] = cs[c] ? 0.0 : u.r[3 * v + c] - q[c];
      mg_minv(u.dinv, u.binv, v, w, z);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long i = 3 * v + c;
        const double dd = cs[c] ? 0.0 : u.d[i];
        u.x[i] = cs[c] ? 0.0 : u.x[i] + dd;
        u.r[i] = w[c];
        u.dn[i] = cs[c] ? 0.0 : rho1 * rho * dd + (2.0 * rho1 / delta) * z[c];
      }
      break;
    }
    case MG_CORR:
#pragma unroll
      for (int c = 0; c < 3; ++c) w[c] = cs[c] ? 0.0 : u.r[3 * v + c] - q[c];
      mg_minv(u.dinv, u.binv, v, w, z);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        u.r[3 * v + c] = w[c];
        u.dn[3 * v + c] = cs[c] ? 0.0 : z[c] / u.scal[MS_THETA];
      }
      break;
    case MG_POWER:
#pragma unroll
      for (int c = 0; c < 3; ++c) w[c] = cs[c] ? 0.0 : q[c];
      mg_minv(u.dinv, u.binv, v, w, z);
#pragma unroll
      for (int c = 0; c < 3; ++c) u.y[3 * v + c] = cs[c] ? 0.0 : z[c];
      break;
    default: {  // MG_RAYLEIGH: x.q and x.(B x) over the free components
#pragma unroll
      for (int c = 0; c < 3; ++c) w[c] = cs[c] ? 0.0 : u.xin[3 * v + c];
      mg_bnode(u.binv, v, w, z);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        t1 += w[c] * (cs[c] ? 0.0 : q[c]);
        t2 += w[c] * z[c];
      }
    }
  }
}

// per node: q = (A_k in)_v from the level's block rows (3 x 3 blocks of the
// assembled Galerkin operator, supported columns zeroed), then the update of
// mode u.mode; LANES lanes per node (lane c < 3 updates component c)
template <int LANES>
__global__ __launch_bounds__(256) void k_mg_spmv(const double* __restrict__ in, const int32_t* __restrict__ bptr,
                                                 const int32_t* __restrict__ bcol, const double* __restrict__ bval,
                                                 const uint8_t* __restrict__ flag, int nn, MgUpd u,
                                                 double* __restrict__ part) {
  __shared__ double sh[16];
  double t1 = 0.0, t2 = 0.0;
  const int q = threadIdx.x & (LANES - 1);
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)LANES * nn;
       t += (long)gridDim.x * blockDim.x) {
    const int v = (int)(t / LANES);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k = bptr[v] + q; k < bptr[v + 1]; k += LANES) {
      const long c = bcol[k];
      const double x0 = in[3 * c], x1 = in[3 * c + 1], x2 = in[3 * c + 2];
      const double* __restrict__ B = bval + 9L * k;
      a0 = fma(B[0], x0, fma(B[1], x1, fma(B[2], x2, a0)));
      a1 = fma(B[3], x0, fma(B[4], x1, fma(B[5], x2, a1)));
      a2 = fma(B[6], x0, fma(B[7], x1, fma(B[8], x2, a2)));
    }
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) {
      a0 += __shfl_xor(a0, o, 64);
      a1 += __shfl_xor(a1, o, 64);
      a2 += __shfl_xor(a2, o, 64);
    }
    if (q < 3) {
      const bool cs = mg_cons(flag[v], q);
      mg_update(u, 3L * v + q, cs, cs ? 0.0 : pick3(q, a0, a1, a2), t1, t2);
    }
  }
  if (u.mode == MG_RAYLEIGH) {
    block_sum2(t1, t2, sh);
    if (threadIdx.x == 0) {
      part[blockIdx.x] = t1;
      part[MG_RED + blockIdx.x] = t2;
    }
  }
}

// level 0: the same updates with q from the context's operator
__global__ __launch_bounds__(256) void k_mg_vec0(const double* __restrict__ q, const uint8_t* __restrict__ flag,
                                                 int nn, MgUpd u, double* __restrict__ part) {
  __shared__ double sh[16];
  double t1 = 0.0, t2 = 0.0;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += gridDim.x * blockDim.x) {
    const double qv[3] = {q[3L * v], q[3L * v + 1], q[3L * v + 2]};
    mg_update_node(u, v, flag[v], qv, t1, t2);
  }
  if (u.mode == MG_RAYLEIGH) {
    block_sum2(t1, t2, sh);
    if (threadIdx.x == 0) {
      part[blockIdx.x] = t1;
      part[MG_RED + blockIdx.x] = t2;
    }
  }
}

// b_c = R r_f on the coarse level; with init, the smoother starts there:
// x = 0, r = b, d = D^-1 b / theta.  LANES lanes per coarse node (rows of R
// grow with the coarsening ratio: 27 fine nodes per coarse node at ratio 2,
// up to 343 at ratio 4).
template <int LANES>
__global__ __launch_bounds__(256) void k_mg_restrict(const double* __restrict__ rf, const int32_t* __restrict__ rptr,
                                                     const int32_t* __restrict__ rcol, const double* __restrict__ rw,
                                                     const uint8_t* __restrict__ flag, int nn, double* __restrict__ b,
                                                     int init, double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ d, const double* __restrict__ dinv,
                                                     const double* __restrict__ scal) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int v = (int)(t / LANES), q = threadIdx.x & (LANES - 1);
  if (v >= nn) return;  // the lanes of a node leave together
  double a0, a1, a2;
  row_gather<LANES>(rf, rptr[v], rptr[v + 1], rcol, rw, q, a0, a1, a2);
  if (q >= 3) return;
  const long i = 3L * v + q;
  const double bi = mg_cons(flag[v], q) ? 0.0 : pick3(q, a0, a1, a2);
  b[i] = bi;
  if (init) {
    x[i] = 0.0;
    r[i] = bi;
    d[i] = dinv[i] * bi / scal[MS_THETA];
  }
}

// t = P (xc + dc) at the fine nodes; df = t, xf += t.  Four lanes per node;
// dc (the coarse level's last smoothing correction) may be null.
__global__ __launch_bounds__(256) void k_mg_prolong(const double* __restrict__ xc, const double* __restrict__ dc,
                                                    const int32_t* __restrict__ pptr, const int32_t* __restrict__ pcol,
                                                    const double* __restrict__ pw, const uint8_t* __restrict__ flag,
                                                    int nn, double* __restrict__ xf, double* __restrict__ df) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int v = (int)(t >> 2), q = threadIdx.x & 3;
  if (v >= nn) return;
  double a0, a1, a2, e0 = 0.0, e1 = 0.0, e2 = 0.0;
  row_gather4(xc, pptr[v], pptr[v + 1], pcol, pw, q, a0, a1, a2);
  if (dc) row_gather4(dc, pptr[v], pptr[v + 1], pcol, pw, q, e0, e1, e2);
  if (q == 3) return;
  const long i = 3L * v + q;
  const double tv = mg_cons(flag[v], q) ? 0.0 : pick3(q, a0, a1, a2) + pick3(q, e0, e1, e2);
  df[i] = tv;
  xf[i] += tv;
}

// plain prolongation (tests): xf = P xc
__global__ __launch_bounds__(256) void k_mg_prolong_plain(const double* __restrict__ xc,
                                                          const int32_t* __restrict__ pptr,
                                                          const int32_t* __restrict__ pcol,
                                                          const double* __restrict__ pw,
                                                          const uint8_t* __restrict__ flag, int nn,
                                                          double* __restrict__ xf) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  double s[3] = {0.0, 0.0, 0.0};
  for (int k = pptr[v]; k < pptr[v + 1]; ++k)
    for (int c = 0; c < 3; ++c) s[c] = fma(pw[k], xc[3L * pcol[k] + c], s[c]);
  for (int c = 0; c < 3; ++c) xf[3L * v + c] = mg_cons(flag[v], c) ? 0.0 : s[c];
}

// coarsest level: x = A~^-1 b, one workgroup per row (every thread requests
// its few entries at once; fixed-order block sum)
__global__ __launch_bounds__(256) void k_mg_coarse_solve(const double* __restrict__ Ainv,
                                                         const double* __restrict__ b, double* __restrict__ x, int n) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) s = fma(Ainv[(long)i * n + j], b[j], s);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) x[i] = s;
}

// ---------------------------------------------------------------- set-up kernels
// placement of a child in its parent: bits 0-1 log2 of the size ratio r
// (1, 2 or 4), bits 2 + 2 ax the child's offset along axis ax in child edges
// (0 .. r - 1).  Weight of parent corner a at child corner a2 (trilinear).
__device__ __forceinline__ double mg_pw(int code, int a2, int a) {
  const double inv_r = 1.0 / (double)(1 << (code & 3));
  double w = 1.0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double t = (double)(((code >> (2 + 2 * ax)) & 3) + ((a2 >> ax) & 1)) * inv_r;
    w *= ((a >> ax) & 1) ? t : 1.0 - t;
  }
  return w;
}

// (P_o (x) I3)^T K0 (P_o (x) I3) for the placement code o = blockIdx.x (codes
// that place no child, a ratio field of 3 or an offset beyond the ratio, give
// zeros); the same two products as k_mg_galerkin
__global__ __launch_bounds__(256) void k_mg_gtable(const double* __restrict__ K0, double* __restrict__ G) {
  __shared__ double Kc[576], T1[576], Pw[64];
  const int o = blockIdx.x, r = 1 << (o & 3);
  bool valid = (o & 3) != 3;
  for (int ax = 0; ax < 3; ++ax) valid = valid && ((o >> (2 + 2 * ax)) & 3) < r;
  for (int i = threadIdx.x; i < 576; i += blockDim.x) Kc[i] = K0[i];
  if (threadIdx.x < 64) Pw[threadIdx.x] = mg_pw(o, threadIdx.x >> 3, threadIdx.x & 7);
  __syncthreads();
  for (int i = threadIdx.x; i < 576; i += blockDim.x) {
    const int row = i / 24, col = i % 24, b = col / 3, dd = col % 3;
    double s = 0.0;
    for (int b2 = 0; b2 < 8; ++b2) s = fma(Kc[row * 24 + 3 * b2 + dd], Pw[b2 * 8 + b], s);
    T1[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 576; i += blockDim.x) {
    const int row = i / 24, col = i % 24, a = row / 3, c = row % 3;
    double s = 0.0;
    for (int a2 = 0; a2 < 8; ++a2) s = fma(Pw[a2 * 8 + a], T1[(3 * a2 + c) * 24 + col], s);
    G[576L * o + i] = valid ? s : 0.0;
  }
}

// dense Galerkin matrix of each merged element: sum over children j of
// (P_j (x) I3)^T K_j (P_j (x) I3); K_j dense (previous level) or, for a leaf
// of the finer level, c_j K0, whose product is c_j times the tabulated
// P^T K0 P of its placement
__global__ __launch_bounds__(256) void k_mg_galerkin(const int32_t* __restrict__ cptr,
                                                     const int32_t* __restrict__ celem,
                                                     const uint8_t* __restrict__ coct, int nd,
                                                     const double* __restrict__ Kd_f, int nd_f,
                                                     const int32_t* __restrict__ pure_f,
                                                     const double* __restrict__ coef, const double* __restrict__ G,
                                                     double* __restrict__ Kd) {
  __shared__ double Kc[576], T1[576], Pw[64];
  const int e = blockIdx.x;
  if (e >= nd) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int k = cptr[e]; k < cptr[e + 1]; ++k) {
    const int ch = celem[k], o = coct[k];
    if (ch >= nd_f) {  // a leaf: no shared memory, the same for every thread
      const double c = coef[pure_f[ch - nd_f]];
      for (int i = threadIdx.x, t = 0; i < 576; i += blockDim.x, ++t) acc[t] += c * G[576L * o + i];
      continue;
    }
    __syncthreads();
    // the child's matrix (stored transposed: read in order, placed by the
    // transpose) and its 8 x 8 corner weights Pw[a2][a] = mg_pw(o, a2, a)
    for (int j = threadIdx.x; j < 576; j += blockDim.x) Kc[(j % 24) * 24 + j / 24] = Kd_f[576L * ch + j];
    if (o != 0 && threadIdx.x < 64) Pw[threadIdx.x] = mg_pw(o, threadIdx.x >> 3, threadIdx.x & 7);
    __syncthreads();
    if (o == 0) {  // the same box
      for (int i = threadIdx.x, t = 0; i < 576; i += blockDim.x, ++t) acc[t] += Kc[i];
      continue;
    }
    // T1[(a2,c),(b,d)] = sum_b2 Kc[(a2,c),(b2,d)] P[b2][b]
    for (int i = threadIdx.x; i < 576; i += blockDim.x) {
      const int row = i / 24, col = i % 24, b = col / 3, dd = col % 3;
      double s = 0.0;
      for (int b2 = 0; b2 < 8; ++b2) s = fma(Kc[row * 24 + 3 * b2 + dd], Pw[b2 * 8 + b], s);
      T1[i] = s;
    }
    __syncthreads();
    // acc[(a,c),(b,d)] += sum_a2 P[a2][a] T1[(a2,c),(b,d)]
    for (int i = threadIdx.x, t = 0; i < 576; i += blockDim.x, ++t) {
      const int row = i / 24, col = i % 24, a = row / 3, c = row % 3;
      double s = 0.0;
      for (int a2 = 0; a2 < 8; ++a2) s = fma(Pw[a2 * 8 + a], T1[(3 * a2 + c) * 24 + col], s);
      acc[t] += s;
    }
  }
  for (int i = threadIdx.x, t = 0; i < 576; i += blockDim.x, ++t) Kd[576L * e + (i % 24) * 24 + i / 24] = acc[t];
}

// block rows of A_k after a density change: each block sums its
// contributions w K_e[(a, .), (b, .)] (w the product of the two vertices'
// interpolation weights) in the stored order, then zeroes the columns of
// supported DOFs
__global__ __launch_bounds__(256) void k_mg_bsr_values(const int32_t* __restrict__ kptr,
                                                       const int32_t* __restrict__ ke,
                                                       const uint8_t* __restrict__ kab,
                                                       const double* __restrict__ kw,
                                                       const int32_t* __restrict__ bcol,
                                                       const uint8_t* __restrict__ flag,
                                                       const double* __restrict__ Kd, int nd,
                                                       const int32_t* __restrict__ pure_src,
                                                       const double* __restrict__ coef,
                                                       const double* __restrict__ K0, double* __restrict__ bval,
                                                       int nnzb) {
  const int blk = blockIdx.x * blockDim.x + threadIdx.x;
  if (blk >= nnzb) return;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = kptr[blk]; k < kptr[blk + 1]; ++k) {
    const int e = ke[k], a = kab[k] >> 3, b = kab[k] & 7;
    const double w = kw[k];
    if (e < nd) {
      const double* __restrict__ Ke = Kd + 576L * e;  // column-major
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[3 * i + j] = fma(w, Ke[(3 * b + j) * 24 + 3 * a + i], acc[3 * i + j]);
    } else {
      const double wc = w * coef[pure_src[e - nd]];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[3 * i + j] = fma(wc, K0[(3 * a + i) * 24 + 3 * b + j], acc[3 * i + j]);
    }
  }
  const uint8_t fc = flag[bcol[blk]];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) bval[9L * blk + 3 * i + j] = ((fc >> j) & 1) ? 0.0 : acc[3 * i + j];
}

// diagonal inverse of A~ on a level from its diagonal blocks
__global__ __launch_bounds__(256) void k_mg_bsr_diag(const int32_t* __restrict__ bdiag,
                                                     const double* __restrict__ bval,
                                                     const uint8_t* __restrict__ flag, double* __restrict__ dinv,
                                                     int nn) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  const int blk = bdiag[v];
  for (int c = 0; c < 3; ++c)
    dinv[3L * v + c] = (mg_cons(flag[v], c) || blk < 0) ? 1.0 : 1.0 / bval[9L * blk + 4 * c];
}

// power-iteration start: +-1 from a counter hash (SplitMix64 finaliser), zero at constrained DOFs
__global__ __launch_bounds__(256) void k_mg_power_init(double* __restrict__ x, const uint8_t* __restrict__ flag,
                                                       int nn) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= 3L * nn) return;
  uint64_t z = (uint64_t)i + 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  z ^= z >> 31;
  x[i] = mg_cons(flag[i / 3], (int)(i % 3)) ? 0.0 : ((z >> 63) ? 1.0 : -1.0);
}

// lambda = (x.Ax)/(x.Dx) from the partials, or the caller's value; smoothing interval
__global__ void k_mg_lambda(const double* __restrict__ part, double* __restrict__ scal, double user, double hi_factor,
                            double ratio) {
  __shared__ double sh[16];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < MG_RED; i += blockDim.x) {
    a += part[i];
    b += part[MG_RED + i];
  }
  block_sum2(a, b, sh);
  if (threadIdx.x == 0) {
    const double lam = user > 0.0 ? user : (b > 0.0 ? a / b : 1.0);
    const double hi = hi_factor * lam, lo = hi / ratio;
    scal[MS_LAM] = lam;
    scal[MS_THETA] = 0.5 * (hi + lo);
    scal[MS_DELTA] = 0.5 * (hi - lo);
    scal[MS_SIGMA] = (hi + lo) / (hi - lo);
  }
}

// coarsest level: dense A~ from its block rows, identity rows and columns
// for constrained DOFs; one workgroup per node row (its three DOF rows)
__global__ __launch_bounds__(256) void k_mg_coarse_assemble(const int32_t* __restrict__ bptr,
                                                            const int32_t* __restrict__ bcol,
                                                            const double* __restrict__ bval,
                                                            const uint8_t* __restrict__ flag, int nn,
                                                            double* __restrict__ A) {
  const int n = 3 * nn, v = blockIdx.x;
  for (int e = threadIdx.x; e < 3 * n; e += blockDim.x) {
    const int I = 3 * v + e / n, J = e % n;
    A[(long)I * n + J] = (I == J && mg_cons(flag[v], I - 3 * v)) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int k0 = bptr[v], nk = bptr[v + 1] - k0;
  for (int e = threadIdx.x; e < 9 * nk; e += blockDim.x) {
    const int k = k0 + e / 9, i = (e % 9) / 3, j = e % 3, w = bcol[k];
    if (!mg_cons(flag[v], i) && !mg_cons(flag[w], j)) A[(long)(3 * v + i) * n + 3 * w + j] = bval[9L * k + 3 * i + j];
  }
}

// In-place inverse of the SPD coarsest matrix (row-major, n x n) by blocked
// Gauss-Jordan elimination without pivoting (the pivot blocks of an SPD
// matrix are SPD Schur complements).  For each block k of BGJ rows (the last
// one may be shorter), with P the inverse of the pivot block A_kk:
//   A_kk = P;  A_kj = P A_kj (j != k);  A_ij -= A_ik A_kj (i, j != k);
//   A_ik = -A_ik P (i != k),
// the block form of the scalar steps a_kk = 1 / a_kk, a_kj /= a_kk,
// a_ij -= a_ik a_kj, a_ik = -a_ik / a_kk.  One step is four launches (pivot
// block, row panel, trailing update, column panel), the last three over
// 64-wide tiles in parallel workgroups.
constexpr int BGJ = 64;
constexpr int BGJ_S = BGJ + 1;  // LDS row stride

// pivot block k0: scalar Gauss-Jordan in registers, one workgroup of 256
// threads; thread (rg, J) = (t / 64, t % 64) holds column J, rows rg + 4 m
// (m < 16).  Per step s the pivot row and column go through LDS (two buffers
// alternating by step, so one barrier per step suffices).
__global__ __launch_bounds__(256) void k_bgj_pivot(double* __restrict__ A, int n, int k0) {
  __shared__ double rowv[2][BGJ], colv[2][BGJ];
  const int bs = min(BGJ, n - k0), t = threadIdx.x, J = t & 63, rg = t >> 6;
  double p[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int I = rg + 4 * m;
    p[m] = (I < bs && J < bs) ? A[(long)(k0 + I) * n + k0 + J] : 0.0;
  }
  // selects rather than branches: every thread runs the same straight code
  for (int s = 0; s < bs; ++s) {
    const int b = s & 1, ms = s >> 2;
    double ps = 0.0;
#pragma unroll
    for (int m = 0; m < 16; ++m) ps = (m == ms) ? p[m] : ps;
    if (rg == (s & 3)) rowv[b][J] = ps;
    if (J == s)
#pragma unroll
      for (int m = 0; m < 16; ++m) colv[b][rg + 4 * m] = p[m];
    __syncthreads();
    const double piv = 1.0 / rowv[b][s];
    const double rj = (J == s ? 1.0 : rowv[b][J]) * piv;
    const bool js = J == s;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const double c = colv[b][rg + 4 * m];
      const double u = fma(-c, rj, js ? 0.0 : p[m]);
      p[m] = (rg + 4 * m == s) ? rj : u;
    }
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int I = rg + 4 * m;
    if (I < bs && J < bs) A[(long)(k0 + I) * n + k0 + J] = p[m];
  }
}

// C (rows x cols, at most 64 x 64) = X (rows x m) Y (m x cols) from LDS
// (strides BGJ_S); each of the 256 threads owns a 4 x 4 patch
__device__ __forceinline__ void bgj_patch(const double* X, const double* Y, int m, double (&c)[4][4]) {
  const int r0 = (threadIdx.x >> 4) * 4, c0 = (threadIdx.x & 15) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) c[a][b] = 0.0;
  for (int q = 0; q < m; ++q) {
    double x[4], y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = X[(r0 + a) * BGJ_S + q];
#pragma unroll
    for (int b = 0; b < 4; ++b) y[b] = Y[q * BGJ_S + c0 + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) c[a][b] = fma(x[a], y[b], c[a][b]);
  }
}

// load the tile of A at (r0, c0) with rows x cols (zero outside) into S; a
// thread's 16 loads are all requested before the first is stored (256 threads)
constexpr int BGJ_PER = BGJ * BGJ / 256;
__device__ __forceinline__ void bgj_load(const double* __restrict__ A, int n, int r0, int c0, int rows, int cols,
                                         double* S) {
  double v[BGJ_PER];
#pragma unroll
  for (int m = 0; m < BGJ_PER; ++m) {
    const int e = threadIdx.x + 256 * m, I = e / BGJ, J = e % BGJ;
    v[m] = (I < rows && J < cols) ? A[(long)(r0 + I) * n + c0 + J] : 0.0;
  }
#pragma unroll
  for (int m = 0; m < BGJ_PER; ++m) {
    const int e = threadIdx.x + 256 * m, I = e / BGJ, J = e % BGJ;
    S[I * BGJ_S + J] = v[m];
  }
}

// row panel: A_kj = P A_kj for the column tiles j != k (grid: one tile each)
__global__ __launch_bounds__(256) void k_bgj_row(double* __restrict__ A, int n, int k0) {
  __shared__ double Ps[BGJ * BGJ_S], T[BGJ * BGJ_S];
  const int j0 = blockIdx.x * BGJ;
  if (j0 == k0) return;
  const int bs = min(BGJ, n - k0), w = min(BGJ, n - j0);
  bgj_load(A, n, k0, k0, bs, bs, Ps);
  bgj_load(A, n, k0, j0, bs, w, T);
  __syncthreads();
  double c[4][4];
  bgj_patch(Ps, T, bs, c);
  const int r0 = (threadIdx.x >> 4) * 4, cc0 = (threadIdx.x & 15) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (r0 + a < bs && cc0 + b < w) A[(long)(k0 + r0 + a) * n + j0 + cc0 + b] = c[a][b];
}

// trailing update: A_ij -= A_ik A_kj for the tiles i, j != k (grid: nb x nb)
__global__ __launch_bounds__(256) void k_bgj_trail(double* __restrict__ A, int n, int k0) {
  __shared__ double X[BGJ * BGJ_S], Y[BGJ * BGJ_S];
  const int i0 = blockIdx.y * BGJ, j0 = blockIdx.x * BGJ;
  if (i0 == k0 || j0 == k0) return;
  const int bs = min(BGJ, n - k0), h = min(BGJ, n - i0), w = min(BGJ, n - j0);
  // the patch of A_ij this thread updates is requested with the tiles
  const int r0 = (threadIdx.x >> 4) * 4, cc0 = (threadIdx.x & 15) * 4;
  double old[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      old[a][b] = (r0 + a < h && cc0 + b < w) ? A[(long)(i0 + r0 + a) * n + j0 + cc0 + b] : 0.0;
  bgj_load(A, n, i0, k0, h, bs, X);
  bgj_load(A, n, k0, j0, bs, w, Y);
  __syncthreads();
  double c[4][4];
  bgj_patch(X, Y, bs, c);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (r0 + a < h && cc0 + b < w) A[(long)(i0 + r0 + a) * n + j0 + cc0 + b] = old[a][b] - c[a][b];
}

// column panel: A_ik = -A_ik P for the row tiles i != k (after the trailing
// update, which read the old A_ik)
__global__ __launch_bounds__(256) void k_bgj_col(double* __restrict__ A, int n, int k0) {
  __shared__ double X[BGJ * BGJ_S], Ps[BGJ * BGJ_S];
  const int i0 = blockIdx.x * BGJ;
  if (i0 == k0) return;
  const int bs = min(BGJ, n - k0), h = min(BGJ, n - i0);
  bgj_load(A, n, i0, k0, h, bs, X);
  bgj_load(A, n, k0, k0, bs, bs, Ps);
  __syncthreads();
  double c[4][4];
  bgj_patch(X, Ps, bs, c);
  const int r0 = (threadIdx.x >> 4) * 4, cc0 = (threadIdx.x & 15) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (r0 + a < h && cc0 + b < bs) A[(long)(i0 + r0 + a) * n + k0 + cc0 + b] = -c[a][b];
}

static void bgj_invert(hipStream_t st, double* A, int n) {
  const int nb = (n + BGJ - 1) / BGJ;
  for (int k = 0; k < nb; ++k) {
    const int k0 = k * BGJ;
    hipLaunchKernelGGL(k_bgj_pivot, dim3(1), dim3(256), 0, st, A, n, k0);
    if (nb == 1) break;
    hipLaunchKernelGGL(k_bgj_row, dim3(nb), dim3(256), 0, st, A, n, k0);
    hipLaunchKernelGGL(k_bgj_trail, dim3(nb, nb), dim3(256), 0, st, A, n, k0);
    hipLaunchKernelGGL(k_bgj_col, dim3(nb), dim3(256), 0, st, A, n, k0);
  }
}

// ---------------------------------------------------------------- PCG kernels


// z = x0 + d0 (the V-cycle's last correction folded in); partials of r.z
__global__ __launch_bounds__(256) void k_mgcg_rz(const double* __restrict__ x0, const double* __restrict__ d0,
                                                 const double* __restrict__ r, double* __restrict__ z, long n,
                                                 double* __restrict__ part, const double* __restrict__ cg) {
  __shared__ double sh[16];
  if (cg && cg[MC_DONE] != 0.0) return;
  double s = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double zi = x0[i] + d0[i];
    z[i] = zi;
    s += r[i] * zi;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = z + beta p with beta = r.z / (r.z)_old (beta = 0 on the first iteration)




__global__ __launch_bounds__(256) void k_mgcg_resid(const double* __restrict__ b, const double* __restrict__ q,
                                                    const uint8_t* __restrict__ flag, long n,
                                                    double* __restrict__ part) {
  __shared__ double sh[16];
  double rr = 0.0, bb = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    if (mg_cons(flag[i / 3], (int)(i % 3))) continue;
    const double ri = b[i] - q[i];
    rr += ri * ri;
    bb += b[i] * b[i];
  }
  block_sum2(rr, bb, sh);
  if (threadIdx.x == 0) {
    part[2 * MG_RED + blockIdx.x] = rr;
    part[3 * MG_RED + blockIdx.x] = bb;
  }
}

__global__ void k_mgcg_resid_scal(const double* __restrict__ part, double* __restrict__ cg) {
  __shared__ double sh[16];
  double rr = 0.0, bb = 0.0;
  for (int i = threadIdx.x; i < MG_RED; i += blockDim.x) {
    rr += part[2 * MG_RED + i];
    bb += part[3 * MG_RED + i];
  }
  block_sum2(rr, bb, sh);
  if (threadIdx.x == 0) cg[MC_RES] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
}

__global__ __launch_bounds__(256) void k_mg_mask_copy(const double* __restrict__ src, double* __restrict__ dst,
                                                      const uint8_t* __restrict__ flag, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = mg_cons(flag[i / 3], (int)(i % 3)) ? 0.0 : src[i];
}

// CG on the fused operator pass (S_* scalar slots, RED_BLOCKS partials):
// r = b - q masked, the level-0 smoother started from r, partials r.r and b.b
__global__ __launch_bounds__(256) void k_mgcg_start(const double* __restrict__ b, const double* __restrict__ q,
                                                    const uint8_t* __restrict__ flag, double* __restrict__ r,
                                                    long nn, const double* __restrict__ dinv,
                                                    const double* __restrict__ binv,
                                                    const double* __restrict__ s0, double* __restrict__ x0,
                                                    double* __restrict__ r0, double* __restrict__ d0,
                                                    double* __restrict__ part) {
  __shared__ double sh[16];
  double rr = 0.0, bb = 0.0;
  const double th = s0[MS_THETA];
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < nn; v += (long)gridDim.x * blockDim.x) {
    double rv[3], z[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long i = 3 * v + c;
      const bool cs = mg_cons(flag[v], c);
      const double bi = cs ? 0.0 : b[i];
      rv[c] = cs ? 0.0 : bi - q[i];
      r[i] = rv[c];
      x0[i] = 0.0;
      r0[i] = rv[c];
      rr += rv[c] * rv[c];
      bb += bi * bi;
    }
    mg_minv(dinv, binv, v, rv, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) d0[3 * v + c] = z[c] / th;
  }
  block_sum2(rr, bb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rr;
    part[RED_BLOCKS + blockIdx.x] = bb;
  }
}

__global__ void k_mgcg_start_scal(const double* __restrict__ part, double* __restrict__ scal, double tol2) {
  __shared__ double sh[16];
  double rr = 0.0, bb = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += blockDim.x) {
    rr += part[i];
    bb += part[RED_BLOCKS + i];
  }
  block_sum2(rr, bb, sh);
  if (threadIdx.x == 0) {
    scal[S_BB] = bb;
    scal[S_RR] = rr;
    scal[S_ITERS] = 0.0;
    scal[S_RZ0] = scal[S_RZ1] = 0.0;
    scal[S_DONE] = (rr <= tol2 * bb) ? 1.0 : ((rr == rr && rr < 1e300) ? 0.0 : 2.0);
  }
}

// z = x0 + d0 (the V-cycle's output with its last correction); partials r.z, r.r
__global__ __launch_bounds__(256) void k_mgcg_z(const double* __restrict__ x0, const double* __restrict__ d0,
                                                const double* __restrict__ r, double* __restrict__ z, long n,
                                                double* __restrict__ part, const double* __restrict__ scal) {
  __shared__ double sh[16];
  if (scal[S_DONE] != 0.0) return;
  double rz = 0.0, rr = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double zi = x0[i] + d0[i], ri = r[i];
    z[i] = zi;
    rz += ri * zi;
    rr += ri * ri;
  }
  block_sum2(rz, rr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rz;
    part[RED_BLOCKS + blockIdx.x] = rr;
  }
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; the level-0 smoother starts from r
__global__ __launch_bounds__(256) void k_mgcg_step(double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   long n, const double* __restrict__ part_pq, int n_pq,
                                                   double* __restrict__ scal, int it,
                                                   const double* __restrict__ dinv, const double* __restrict__ binv,
                                                   const double* __restrict__ s0,
                                                   double* __restrict__ x0, double* __restrict__ r0,
                                                   double* __restrict__ d0) {
  __shared__ double sh[16];
  const double done = scal[S_DONE];
  const double pq = sum_partials(part_pq, n_pq, sh);
  if (done != 0.0) return;
  const double rz = scal[S_RZ0 + (it & 1)];
  if (!(pq > 0.0) || !(pq < 1e300) || !(rz == rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_DONE] = 2.0;
    return;
  }
  const double alpha = rz / pq, th = s0[MS_THETA];
  // per node (n = 3 nn): the smoother's start needs the node's three residual
  // components together when it smooths with node blocks
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < n / 3; v += (long)gridDim.x * blockDim.x) {
    double rv[3], z[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long i = 3 * v + c;
      x[i] += alpha * p[i];
      rv[c] = r[i] - alpha * q[i];
      r[i] = rv[c];
      x0[i] = 0.0;
      r0[i] = rv[c];
    }
    mg_minv(dinv, binv, v, rv, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) d0[3 * v + c] = z[c] / th;
  }
}

__global__ __launch_bounds__(256) void k_mg_zero(double* __restrict__ a, double* __restrict__ b, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) {
    a[i] = 0.0;
    b[i] = 0.0;
  }
}

// ---------------------------------------------------------------- host side
int blocks_for(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 1L << 20)); }

// b_c = R r_f (with the coarse smoother's start when init), lanes by row length
void launch_restrict(hipStream_t st, MgLevel& C, const double* rf, double* b, int init) {
  const double *dinv = init ? C.dinv : nullptr, *scal = init ? C.scal : nullptr;
  double *x = init ? C.x : nullptr, *r = init ? C.r : nullptr, *d = init ? C.d : nullptr;
  switch (C.rlanes) {
    case 32:
      hipLaunchKernelGGL(k_mg_restrict<32>, dim3(blocks_for(32L * C.nn)), dim3(256), 0, st, rf, C.rptr, C.rcol, C.rw,
                         C.flag, C.nn, b, init, x, r, d, dinv, scal);
      break;
    case 16:
      hipLaunchKernelGGL(k_mg_restrict<16>, dim3(blocks_for(16L * C.nn)), dim3(256), 0, st, rf, C.rptr, C.rcol, C.rw,
                         C.flag, C.nn, b, init, x, r, d, dinv, scal);
      break;
    case 8:
      hipLaunchKernelGGL(k_mg_restrict<8>, dim3(blocks_for(8L * C.nn)), dim3(256), 0, st, rf, C.rptr, C.rcol, C.rw,
                         C.flag, C.nn, b, init, x, r, d, dinv, scal);
      break;
    default:
      hipLaunchKernelGGL(k_mg_restrict<4>, dim3(blocks_for(4L * C.nn)), dim3(256), 0, st, rf, C.rptr, C.rcol, C.rw,
                         C.flag, C.nn, b, init, x, r, d, dinv, scal);
  }
}

// q = A_k in on level k >= 1 from its block rows, fused with the update u
int level_pass(amrto_ctx* ctx, MgLevel& L, const double* in, const MgUpd& u, double* part) {
  // the Rayleigh partials fill exactly MG_RED slots
  const int grid = u.mode == MG_RAYLEIGH ? MG_RED : blocks_for((long)L.lanes * L.nn);
  switch (L.lanes) {
    case 32:
      hipLaunchKernelGGL(k_mg_spmv<32>, dim3(grid), dim3(256), 0, ctx->stream, in, L.bptr, L.bcol, L.bval, L.flag,
                         L.nn, u, part);
      break;
    case 16:
      hipLaunchKernelGGL(k_mg_spmv<16>, dim3(grid), dim3(256), 0, ctx->stream, in, L.bptr, L.bcol, L.bval, L.flag,
                         L.nn, u, part);
      break;
    case 8:
      hipLaunchKernelGGL(k_mg_spmv<8>, dim3(grid), dim3(256), 0, ctx->stream, in, L.bptr, L.bcol, L.bval, L.flag,
                         L.nn, u, part);
      break;
    default:
      hipLaunchKernelGGL(k_mg_spmv<4>, dim3(grid), dim3(256), 0, ctx->stream, in, L.bptr, L.bcol, L.bval, L.flag,
                         L.nn, u, part);
  }
  return hipGetLastError() == hipSuccess ? AMRTO_OK : ctx->fail(AMRTO_EHIP, "multigrid level pass");
}

// level 0: q = A~ d through the context's operator, then the vector update
int level0_pass(amrto_ctx* ctx, MgLevel& L, const double* in, const MgUpd& u, double* part) {
  int rc = launch_apply(ctx, in, L.q, AMRTO_FP64);
  if (rc) return rc;
  const int grid = u.mode == MG_RAYLEIGH ? MG_RED : blocks_for(L.nn);
  hipLaunchKernelGGL(k_mg_vec0, dim3(grid), dim3(256), 0, ctx->stream, L.q, L.flag,
                     L.nn, u, part);
  return hipGetLastError() == hipSuccess ? AMRTO_OK : ctx->fail(AMRTO_EHIP, "multigrid level-0 pass");
}

int pass(amrto_ctx* ctx, int k, const double* in, const MgUpd& u) {
  MgData* g = ctx->mg;
  MgLevel& L = g->lv[k];
  if (k == 0 && !ctx->uniform && in == L.d &&
      (u.mode == MG_CHEB || u.mode == MG_CHEB_LAST || u.mode == MG_CORR)) {
    // octree level 0: the smoothing update runs in the operator pass itself;
    // the next direction goes to the other buffer of the pair (d, q)
    const int mode = u.mode == MG_CHEB ? 1 : (u.mode == MG_CHEB_LAST ? 2 : 3);
    const int rc = apply_cheb(ctx, L.d, L.q, mode, u.step, L.scal, L.dinv, L.x, L.r, L.binv);
    if (rc) return rc;
    if (mode != 2) std::swap(L.d, L.q);
    return AMRTO_OK;
  }
  if (k == 0) return level0_pass(ctx, L, in, u, g->part);  // pointwise update: d in place
  // the block-row pass reads neighbours' d: the next direction goes to the
  // other buffer of the pair (d, q)
  const bool newdir = u.mode == MG_CHEB || u.mode == MG_CORR;
  MgUpd v = u;
  if (newdir) v.dn = L.q;
  const int rc = level_pass(ctx, L, in, v, g->part);
  if (rc == AMRTO_OK && newdir) std::swap(L.d, L.q);
  return rc;
}

MgUpd upd(MgLevel& L, int mode, int step = 0) {
  MgUpd u{};
  u.mode = mode;
  u.step = step;
  u.scal = L.scal;
  u.dinv = L.dinv;
  u.binv = L.binv;
  u.x = L.x;
  u.r = L.r;
  u.d = L.d;
  u.dn = L.d;
  return u;
}

// one V-cycle below level k; level k's b holds the right-hand side and, for
// k < coarsest, its smoother state was initialised by the restriction
int vcycle_from(amrto_ctx* ctx, int k) {
  MgData* g = ctx->mg;
  MgLevel& L = g->lv[k];
  int rc;
  if (k == g->nlev - 1) {
    const int n = 3 * L.nn;
    hipLaunchKernelGGL(k_mg_coarse_solve, dim3(n), dim3(256), 0, ctx->stream, L.Ainv, L.b, L.x, n);
    return hipGetLastError() == hipSuccess ? AMRTO_OK : ctx->fail(AMRTO_EHIP, "multigrid coarse solve");
  }
  const int m = k == 0 ? g->degree : g->coarse_degree;
  for (int s = 0; s < m; ++s)
    if ((rc = pass(ctx, k, L.d, upd(L, s == m - 1 ? MG_CHEB_LAST : MG_CHEB, s)))) return rc;
  MgLevel& C = g->lv[k + 1];
  const bool coarsest = k + 1 == g->nlev - 1;
  launch_restrict(ctx->stream, C, L.r, C.b, coarsest ? 0 : 1);
  if ((rc = vcycle_from(ctx, k + 1))) return rc;
  // x += P x_c (the coarse level's last correction d folded in), d = that correction
  hipLaunchKernelGGL(k_mg_prolong, dim3(blocks_for(4L * L.nn)), dim3(256), 0, ctx->stream, C.x,
                     coarsest ? (const double*)nullptr : C.d, C.pptr, C.pcol, C.pw, L.flag, L.nn, L.x, L.d);
  if ((rc = pass(ctx, k, L.d, upd(L, MG_CORR)))) return rc;
  // post-smoothing: m - 1 passes; the last correction stays in d (added by the consumer)
  for (int s = 0; s < m - 1; ++s)
    if ((rc = pass(ctx, k, L.d, upd(L, MG_CHEB, s)))) return rc;
  return hipGetLastError() == hipSuccess ? AMRTO_OK : ctx->fail(AMRTO_EHIP, "multigrid V-cycle");
}

// level-0 smoother start from the right-hand side b (device): x = 0, r = b, d = M^-1 b / theta
__global__ __launch_bounds__(256) void k_mg_start0(const double* __restrict__ b, const uint8_t* __restrict__ flag,
                                                   const double* __restrict__ dinv, const double* __restrict__ binv,
                                                   const double* __restrict__ scal, double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ d, long nn) {
  const long v = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (v >= nn) return;
  double bv[3], z[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    bv[c] = mg_cons(flag[v], c) ? 0.0 : b[3 * v + c];
    x[3 * v + c] = 0.0;
    r[3 * v + c] = bv[c];
  }
  mg_minv(dinv, binv, v, bv, z);
#pragma unroll
  for (int c = 0; c < 3; ++c) d[3 * v + c] = z[c] / scal[MS_THETA];
}

int vcycle(amrto_ctx* ctx, const double* b) {
  MgData* g = ctx->mg;
  MgLevel& L = g->lv[0];
  const long n = 3L * L.nn;
  (void)n;
  hipLaunchKernelGGL(k_mg_start0, dim3(blocks_for(L.nn)), dim3(256), 0, ctx->stream, b, L.flag, L.dinv, L.binv,
                     L.scal, L.x, L.r, L.d, (long)L.nn);
  return vcycle_from(ctx, 0);
}

// numeric set-up after a density change: Galerkin matrices, diagonals,
// smoothing intervals, coarsest inverse
int mg_numeric(amrto_ctx* ctx) {
  MgData* g = ctx->mg;
  g->lv[0].dinv = ctx->d_dinv;
  g->lv[0].binv = nullptr;
  if (g->blocks0) {  // the inverse node blocks of the current density
    const int rc = block3_setup(ctx);
    if (rc) return rc;
    g->lv[0].binv = ctx->d_binv;
  }
  if (g->G_nu != ctx->nu) {  // K0 changes with the Poisson ratio only
    hipLaunchKernelGGL(k_mg_gtable, dim3(256), dim3(256), 0, ctx->stream, ctx->d_K0, g->G);
    g->G_nu = ctx->nu;
  }
  for (int k = 1; k < g->nlev; ++k) {
    MgLevel& L = g->lv[k];
    MgLevel& F = g->lv[k - 1];
    if (L.nd > 0)
      hipLaunchKernelGGL(k_mg_galerkin, dim3(L.nd), dim3(256), 0, ctx->stream, L.cptr, L.celem, L.coct, L.nd, F.Kd,
                         F.nd, F.pure_src, ctx->d_coef, g->G, L.Kd);
    hipLaunchKernelGGL(k_mg_bsr_values, dim3(blocks_for(L.nnzb)), dim3(256), 0, ctx->stream, L.kptr, L.ke, L.kab,
                       L.kw, L.bcol, L.flag, L.Kd, L.nd, L.pure_src, ctx->d_coef, ctx->d_K0, L.bval, L.nnzb);
    hipLaunchKernelGGL(k_mg_bsr_diag, dim3(blocks_for(L.nn)), dim3(256), 0, ctx->stream, L.bdiag, L.bval, L.flag,
                       L.dinv, L.nn);
  }
  if (hipGetLastError() != hipSuccess) return ctx->fail(AMRTO_EHIP, "multigrid Galerkin set-up");
  // the coarsest level's dense matrix and its inverse need only its block
  // rows: they run on the second stream while the power iterations below
  // (smoothed levels only) run on the context's
  MgLevel& C = g->lv[g->nlev - 1];
  const int n = 3 * C.nn;
  AMRTO_HIP(hipEventRecord(g->ev_fork, ctx->stream));
  AMRTO_HIP(hipStreamWaitEvent(g->aux, g->ev_fork, 0));
  hipLaunchKernelGGL(k_mg_coarse_assemble, dim3(C.nn), dim3(256), 0, g->aux, C.bptr, C.bcol, C.bval, C.flag,
                     C.nn, C.Ainv);
  bgj_invert(g->aux, C.Ainv, n);
  AMRTO_HIP(hipEventRecord(g->ev_join, g->aux));
  // lambda_max of D^-1 A on every smoothed level by power iteration
  for (int k = 0; k < g->nlev - 1; ++k) {
    MgLevel& L = g->lv[k];
    const long n = 3L * L.nn;
    int rc;
    if (!g->user_bounds) {
      hipLaunchKernelGGL(k_mg_power_init, dim3(blocks_for(n)), dim3(256), 0, ctx->stream, L.x, L.flag, L.nn);
      for (int it = 0; it < g->power_its; ++it) {
        MgUpd u = upd(L, MG_POWER);
        u.y = (it & 1) ? L.x : L.r;
        if ((rc = pass(ctx, k, (it & 1) ? L.r : L.x, u))) return rc;
      }
      const double* xl = (g->power_its & 1) ? L.r : L.x;
      MgUpd u = upd(L, MG_RAYLEIGH);
      u.xin = xl;
      if ((rc = pass(ctx, k, xl, u))) return rc;
    }
    hipLaunchKernelGGL(k_mg_lambda, dim3(1), dim3(256), 0, ctx->stream, g->part, L.scal,
                       g->user_bounds ? g->lam_user[k] : 0.0, g->hi_factor, g->ratio);
  }
  AMRTO_HIP(hipStreamWaitEvent(ctx->stream, g->ev_join, 0));
  if (hipGetLastError() != hipSuccess) return ctx->fail(AMRTO_EHIP, "multigrid coarse set-up");
  ctx->mg_valid = true;
  return AMRTO_OK;
}

}  // namespace

namespace amrto {

void mg_free(amrto_ctx* ctx) {
  if (!ctx->mg) return;
  MgData* g = ctx->mg;
  for (int k = 0; k < g->nlev; ++k)
    for (void* p : g->lv[k].owned) (void)hipFree(p);
  for (void* p : g->owned) (void)hipFree(p);
  if (g->h_cg) (void)hipHostFree(g->h_cg);
  if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
  if (g->ev_join) (void)hipEventDestroy(g->ev_join);
  if (g->aux) (void)hipStreamDestroy(g->aux);
  delete g;
  ctx->mg = nullptr;
  ctx->mg_valid = false;
}

}  // namespace amrto

// ---------------------------------------------------------------- hierarchy (host)
namespace {

struct HostLevel {
  LevelMesh m;
  std::vector<int32_t> perm;      // original element -> device order
  std::vector<int32_t> parent;    // original element -> parent on the next level (original order there)
  std::vector<uint8_t> oct;       // placement within the parent (see mg_pw), 0 = the same box
  std::vector<uint8_t> pure;      // per original element
  std::vector<int32_t> src;       // per original element: coefficient index when pure
  int nd = 0;
};

// lattice coordinates stay below 2^20 (octree limits); a point is the anchor
// of at most one leaf of a level
inline uint64_t anchor_key(int64_t x, int64_t y, int64_t z) {
  return ((uint64_t)z << 40) | ((uint64_t)y << 20) | (uint64_t)x;
}

int build_hierarchy(amrto_ctx* ctx, const amrto_octree* tree, int coarse_dofs, int first, std::vector<HostLevel>& H) {
  H.clear();
  H.emplace_back();
  if (!octree_level_mesh(tree, 0, &H[0].m)) return ctx->fail(AMRTO_ESTATE, "amrto_mg_setup: the tree has no mesh");
  if (H[0].m.n_nodes != ctx->n_nodes || H[0].m.n_elems != ctx->n_elems)
    return ctx->fail(AMRTO_EINVAL, "amrto_mg_setup: the tree's mesh is not the uploaded mesh");
  const int L = H[0].m.L;
  // depths 0, first, first + 1, ...; depths >= L are uniform grids
  for (int k = first, prev = 0;; prev = k, ++k) {
    if (prev >= L && 3 * H.back().m.n_nodes <= coarse_dofs) break;
    if ((int)H.size() >= MG_LMAX) break;
    LevelMesh lm;
    if (!octree_level_mesh(tree, k, &lm)) break;
    H.emplace_back();
    H.back().m = std::move(lm);
  }
  const HostLevel& C = H.back();
  if (!C.m.hang_node.empty() || 3 * C.m.n_nodes > MG_COARSE_MAX || H.size() < 2)
    return ctx->fail(AMRTO_EINVAL, "amrto_mg_setup: no coarsest uniform level with at most 1024 DOFs "
                                   "(base extents must allow coarsening)");
  // level 0: every element is its own coefficient
  HostLevel& F0 = H[0];
  const int ne0 = F0.m.n_elems;
  F0.pure.assign(ne0, 1);
  F0.src.resize(ne0);
  for (int e = 0; e < ne0; ++e) {
    if (ctx->uniform) {
      const int32_t* a = &F0.m.anchor[3L * e];
      F0.src[e] = a[0] + ctx->nx * (a[1] + ctx->ny * a[2]);
    } else {
      F0.src[e] = e;
    }
  }
  F0.nd = 0;
  F0.perm.resize(ne0);
  for (int e = 0; e < ne0; ++e) F0.perm[e] = e;
  // parents, purity and device element order level by level
  for (size_t k = 1; k < H.size(); ++k) {
    HostLevel& F = H[k - 1];
    HostLevel& Cl = H[k];
    const int ne = Cl.m.n_elems;
    std::unordered_map<uint64_t, int> box;
    box.reserve(2L * ne);
    for (int e = 0; e < ne; ++e)
      box.emplace(anchor_key(Cl.m.anchor[3L * e], Cl.m.anchor[3L * e + 1], Cl.m.anchor[3L * e + 2]), e);
    std::vector<int> nchild(ne, 0), only(ne, -1);
    F.parent.resize(F.m.n_elems);
    F.oct.resize(F.m.n_elems);
    for (int e = 0; e < F.m.n_elems; ++e) {
      const int64_t s = 1L << (F.m.L - F.m.level[e]);
      const int32_t* a = &F.m.anchor[3L * e];
      int found = -1, o = 0;
      for (int lr = 0; lr <= 2 && found < 0; ++lr) {
        const int64_t S = s << lr;
        auto it = box.find(anchor_key(a[0] / S * S, a[1] / S * S, a[2] / S * S));
        if (it != box.end() && (1L << (Cl.m.L - Cl.m.level[it->second])) == S) {
          found = it->second;
          o = lr;
          for (int ax = 0; ax < 3; ++ax) o |= (int)(((a[ax] % S) / s) << (2 + 2 * ax));
        }
      }
      if (found < 0) return ctx->fail(AMRTO_EINVAL, "amrto_mg_setup: a leaf has no parent on the next level");
      F.parent[e] = found;
      F.oct[e] = (uint8_t)o;
      nchild[found]++;
      only[found] = e;
    }
    Cl.pure.assign(ne, 0);
    Cl.src.assign(ne, -1);
    for (int e = 0; e < ne; ++e)
      if (nchild[e] == 1 && F.oct[only[e]] == 0 && F.pure[only[e]]) {
        Cl.pure[e] = 1;
        Cl.src[e] = F.src[only[e]];
      }
    Cl.perm.assign(ne, -1);
    int nd = 0;
    for (int e = 0; e < ne; ++e)
      if (!Cl.pure[e]) Cl.perm[e] = nd++;
    int np = nd;
    for (int e = 0; e < ne; ++e)
      if (Cl.pure[e]) Cl.perm[e] = np++;
    Cl.nd = nd;
  }
  return AMRTO_OK;
}

int upload_level(amrto_ctx* ctx, MgData* g, std::vector<HostLevel>& H, int k) {
  MgLevel& L = g->lv[k];
  HostLevel& h = H[k];
  const LevelMesh& m = h.m;
  auto& own = L.owned;
  L.nn = m.n_nodes;
  L.ne = m.n_elems;
  L.nd = h.nd;
  L.nh = (int)m.hang_node.size();
  const int nn = m.n_nodes, ne = m.n_elems;
  std::vector<int32_t> hang_of(nn, -1);
  for (int i = 0; i < L.nh; ++i) hang_of[m.hang_node[i]] = i;
  std::vector<uint8_t> flag(nn, 0);
  for (int v = 0; v < nn; ++v) {
    for (int c = 0; c < 3; ++c)
      if (m.fixed[3L * v + c]) flag[v] |= (uint8_t)(1 << c);
    if (hang_of[v] >= 0) flag[v] |= 8;
  }
  AMRTO_HIP(mg_upload(own, L.flag, flag));
  const long n3 = 3L * nn;
  AMRTO_HIP(mg_alloc(own, L.x, n3));
  AMRTO_HIP(mg_alloc(own, L.r, n3));
  AMRTO_HIP(mg_alloc(own, L.d, n3));
  AMRTO_HIP(mg_alloc(own, L.q, n3));
  AMRTO_HIP(mg_alloc(own, L.b, n3));
  AMRTO_HIP(mg_alloc(own, L.scal, MS_COUNT));
  if (k == 0) {
    // every level-0 element is a leaf with its own coefficient (read by the
    // level-1 Galerkin pass)
    for (int32_t i : h.src)
      if (i < 0 || i >= ctx->n_elems) return ctx->fail(AMRTO_EINVAL, "amrto_mg_setup: bad level-0 element");
    AMRTO_HIP(mg_upload(own, L.pure_src, h.src));
    return AMRTO_OK;
  }
  AMRTO_HIP(mg_alloc(own, L.dinv, n3));
  // coefficient index of the single-leaf elements (device order)
  std::vector<int32_t> psrc(ne - h.nd);
  for (int e = 0; e < ne; ++e)
    if (h.pure[e]) psrc[h.perm[e] - h.nd] = h.src[e];
  AMRTO_HIP(mg_upload(own, L.pure_src, psrc));
  AMRTO_HIP(mg_alloc(own, L.Kd, 576L * h.nd));
  // assembled operator: every element vertex pair (a, b) contributes
  // w_a w_b K_e[(a, .), (b, .)] to the block (m_a, m_b) for each master m_a
  // of a (a itself when it does not hang) and m_b of b; contributions are
  // kept per block in (element, a, b, master) order
  struct Contrib {
    int32_t col, e;
    uint8_t ab;
    double w;
  };
  std::vector<std::vector<Contrib>> rows(nn);
  auto expand = [&](int v, int32_t* mm, double* ww) -> int {
    if (hang_of[v] < 0) {
      mm[0] = v;
      ww[0] = 1.0;
      return 1;
    }
    const int hh = hang_of[v], k0 = m.hang_ptr[hh], cnt = m.hang_ptr[hh + 1] - k0;
    for (int j = 0; j < cnt && j < 8; ++j) {
      mm[j] = m.hang_master[k0 + j];
      ww[j] = m.hang_w[k0 + j];
    }
    return std::min(cnt, 8);
  };
  for (int e = 0; e < ne; ++e) {
    const int32_t de = h.perm[e];
    int32_t mm[8][8];
    double ww[8][8];
    int cnt[8];
    for (int a = 0; a < 8; ++a) {
      const int v = m.elem_nodes[8L * e + a];
      if (hang_of[v] >= 0 && m.hang_ptr[hang_of[v] + 1] - m.hang_ptr[hang_of[v]] > 8)
        return ctx->fail(AMRTO_EINVAL, "amrto_mg_setup: a hanging node with more than eight masters");
      cnt[a] = expand(v, mm[a], ww[a]);
    }
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b)
        for (int i = 0; i < cnt[a]; ++i)
          for (int j = 0; j < cnt[b]; ++j)
            rows[mm[a][i]].push_back({mm[b][j], de, (uint8_t)(8 * a + b), ww[a][i] * ww[b][j]});
  }
  std::vector<int32_t> bptr(nn + 1, 0), bcol, bdiag(nn, -1), kptr(1, 0), ke;
  std::vector<uint8_t> kab;
  std::vector<double> kw;
  for (int v = 0; v < nn; ++v) {
    auto& R = rows[v];
    std::stable_sort(R.begin(), R.end(), [](const Contrib& x, const Contrib& y) {
      if (x.col != y.col) return x.col < y.col;
      if (x.e != y.e) return x.e < y.e;
      return x.ab < y.ab;
    });
    for (size_t i = 0; i < R.size(); ++i) {
      if (i == 0 || R[i].col != R[i - 1].col) {
        if (R[i].col == v) bdiag[v] = (int32_t)bcol.size();
        bcol.push_back(R[i].col);
        if (bcol.size() > 1) kptr.push_back((int32_t)ke.size());
      }
      ke.push_back(R[i].e);
      kab.push_back(R[i].ab);
      kw.push_back(R[i].w);
    }
    bptr[v + 1] = (int32_t)bcol.size();
    std::vector<Contrib>().swap(R);
  }
  kptr.push_back((int32_t)ke.size());
  if (bcol.empty()) kptr.assign(1, 0);
  L.nnzb = (int)bcol.size();
  AMRTO_HIP(mg_upload(own, L.bptr, bptr));
  AMRTO_HIP(mg_upload(own, L.bcol, bcol));
  AMRTO_HIP(mg_upload(own, L.bdiag, bdiag));
  AMRTO_HIP(mg_upload(own, L.kptr, kptr));
  AMRTO_HIP(mg_upload(own, L.ke, ke));
  AMRTO_HIP(mg_upload(own, L.kab, kab));
  AMRTO_HIP(mg_upload(own, L.kw, kw));
  AMRTO_HIP(mg_alloc(own, L.bval, 9L * std::max(1, L.nnzb)));
  // long block rows: more lanes per node, so a row's blocks are requested at
  // once (C2's coarse levels, ~22 blocks per row: 8 lanes 5.6 / 4.7 us per
  // pass, 16 lanes 5.3 / 3.8, 32 lanes 6.0 / 3.7)
  L.lanes = (long)bcol.size() > 12L * nn ? 16 : 4;
  // children of the dense elements (previous level, its device order)
  HostLevel& F = H[k - 1];
  std::vector<std::vector<std::pair<int32_t, uint8_t>>> ch(h.nd);
  for (int e = 0; e < F.m.n_elems; ++e) {
    const int de = h.perm[F.parent[e]];
    if (de < h.nd) ch[de].push_back({F.perm[e], F.oct[e]});
  }
  std::vector<int32_t> cptr(h.nd + 1, 0), celem;
  std::vector<uint8_t> coct;
  for (int e = 0; e < h.nd; ++e) {
    std::sort(ch[e].begin(), ch[e].end());
    for (auto& c : ch[e]) {
      celem.push_back(c.first);
      coct.push_back(c.second);
    }
    cptr[e + 1] = (int32_t)celem.size();
  }
  AMRTO_HIP(mg_upload(own, L.cptr, cptr));
  AMRTO_HIP(mg_upload(own, L.celem, celem));
  AMRTO_HIP(mg_upload(own, L.coct, coct));
  // prolongation rows (previous level's nodes) from this level's masters
  const LevelMesh& fm = F.m;
  std::vector<std::vector<std::pair<int32_t, double>>> prow(fm.n_nodes);
  std::vector<uint8_t> done(fm.n_nodes, 0);
  std::vector<int32_t> fh(fm.n_nodes, -1);
  for (size_t i = 0; i < fm.hang_node.size(); ++i) fh[fm.hang_node[i]] = (int32_t)i;
  for (int e = 0; e < fm.n_elems; ++e) {
    const int C = F.parent[e];
    const double S = (double)(1L << (m.L - m.level[C]));
    const int32_t* ca = &m.anchor[3L * C];
    for (int a = 0; a < 8; ++a) {
      const int v = fm.elem_nodes[8L * e + a];
      if (done[v] || fh[v] >= 0) continue;
      done[v] = 1;
      double xi[3];
      for (int ax = 0; ax < 3; ++ax) xi[ax] = (fm.xyz[3L * v + ax] - ca[ax]) / S;
      std::unordered_map<int32_t, double> acc;
      for (int b = 0; b < 8; ++b) {
        double w = 1.0;
        for (int ax = 0; ax < 3; ++ax) w *= ((b >> ax) & 1) ? xi[ax] : 1.0 - xi[ax];
        if (w == 0.0) continue;
        const int cn = m.elem_nodes[8L * C + b];
        if (hang_of[cn] < 0) {
          acc[cn] += w;
        } else {
          const int hh = hang_of[cn];
          for (int j = m.hang_ptr[hh]; j < m.hang_ptr[hh + 1]; ++j) acc[m.hang_master[j]] += w * m.hang_w[j];
        }
      }
      for (auto& kv : acc) prow[v].push_back(kv);
      std::sort(prow[v].begin(), prow[v].end());
    }
  }
  std::vector<int32_t> pptr(fm.n_nodes + 1, 0), pcol;
  std::vector<double> pw;
  std::vector<std::vector<std::pair<int32_t, double>>> rrow(nn);
  for (int v = 0; v < fm.n_nodes; ++v) {
    for (auto& cw : prow[v]) {
      pcol.push_back(cw.first);
      pw.push_back(cw.second);
      rrow[cw.first].push_back({v, cw.second});
    }
    pptr[v + 1] = (int32_t)pcol.size();
  }
  std::vector<int32_t> rptr(nn + 1, 0), rcol;
  std::vector<double> rw;
  for (int v = 0; v < nn; ++v) {
    for (auto& fw : rrow[v]) {  // already in fine-node order
      rcol.push_back(fw.first);
      rw.push_back(fw.second);
    }
    rptr[v + 1] = (int32_t)rcol.size();
  }
  // every index a kernel follows must stay inside its target array
  auto in_range = [](const std::vector<int32_t>& v, long lim) {
    for (int32_t i : v)
      if (i < 0 || i >= lim) return false;
    return true;
  };
  if (!in_range(psrc, ctx->n_elems) || !in_range(bcol, nn) || !in_range(ke, ne) || !in_range(celem, F.m.n_elems) ||
      !in_range(pcol, nn) || !in_range(rcol, fm.n_nodes) || (long)bptr.back() != (long)bcol.size() ||
      (long)kptr.size() != (long)bcol.size() + 1 || (long)kptr.back() != (long)ke.size() ||
      (long)pptr.back() != (long)pcol.size() || (long)rptr.back() != (long)rcol.size() ||
      (long)cptr.back() != (long)celem.size())
    return ctx->fail(AMRTO_EINVAL, "amrto_mg_setup: inconsistent level tables");
  for (size_t i = 0; i < celem.size(); ++i) {
    const int lr = coct[i] & 3;
    for (int ax = 0; ax < 3; ++ax)
      if (lr > 2 || ((coct[i] >> (2 + 2 * ax)) & 3) >= (1 << lr))
        return ctx->fail(AMRTO_EINVAL, "amrto_mg_setup: bad child placement");
  }
  AMRTO_HIP(mg_upload(own, L.pptr, pptr));
  AMRTO_HIP(mg_upload(own, L.pcol, pcol));
  AMRTO_HIP(mg_upload(own, L.pw, pw));
  long rmax = 0;
  for (int v = 0; v < nn; ++v) rmax = std::max<long>(rmax, rptr[v + 1] - rptr[v]);
  L.rlanes = rmax > 128 ? 32 : (rmax > 48 ? 16 : (rmax > 16 ? 8 : 4));  // the longest rows set the pace
  AMRTO_HIP(mg_upload(own, L.rptr, rptr));
  AMRTO_HIP(mg_upload(own, L.rcol, rcol));
  AMRTO_HIP(mg_upload(own, L.rw, rw));
  if (k == g->nlev - 1) AMRTO_HIP(mg_alloc(own, L.Ainv, (size_t)n3 * n3));
  return AMRTO_OK;
}

int check_mg(amrto_ctx* ctx, const char* name) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->mg) return ctx->fail(AMRTO_ESTATE, std::string(name) + ": no multigrid hierarchy (amrto_mg_setup)");
  if (!ctx->has_density) return ctx->fail(AMRTO_ESTATE, std::string(name) + ": density not set");
  return AMRTO_OK;
}

int ensure_numeric(amrto_ctx* ctx) { return ctx->mg_valid ? AMRTO_OK : mg_numeric(ctx); }

}  // namespace

extern "C" {

int amrto_mg_setup(amrto_ctx* ctx, const amrto_octree* tree, const amrto_mg_opts* opts) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_mg_setup: no mesh uploaded");
  if (!tree) return ctx->fail(AMRTO_EINVAL, "amrto_mg_setup: NULL tree");
  amrto_mg_opts o{2, 10.0, 20, 1.1, 200, 1, 0, 0};
  if (opts) o = *opts;
  if (o.degree < 1 || o.degree > 8 || o.coarse_degree < 0 || o.coarse_degree > 8 || !(o.ratio > 1.0) ||
      o.power_its < 1 || o.power_its > 200 || !(o.hi_factor >= 1.0) || o.coarse_dofs < 3 || o.first < 1 ||
      o.first > 2 || o.blocks0 < 0 || o.blocks0 > 1)
    return ctx->fail(AMRTO_EINVAL, "amrto_mg_setup: bad options");
  AMRTO_HIP(hipSetDevice(ctx->device));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  mg_free(ctx);
  std::vector<HostLevel> H;
  int rc = build_hierarchy(ctx, tree, o.coarse_dofs, o.first, H);
  if (rc) return rc;
  MgData* g = new (std::nothrow) MgData();
  if (!g) return ctx->fail(AMRTO_ENOMEM, "amrto_mg_setup: out of host memory");
  ctx->mg = g;
  g->nlev = (int)H.size();
  g->degree = o.degree;
  g->coarse_degree = o.coarse_degree > 0 ? o.coarse_degree : o.degree;
  g->ratio = o.ratio;
  g->power_its = o.power_its;
  g->hi_factor = o.hi_factor;
  g->blocks0 = o.blocks0 != 0;
  for (int k = 0; k < g->nlev; ++k)
    if ((rc = upload_level(ctx, g, H, k))) {
      mg_free(ctx);
      return rc;
    }
  const long n0 = 3L * ctx->n_nodes;
  if (mg_alloc(g->owned, g->part, 4 * MG_RED) != hipSuccess || mg_alloc(g->owned, g->cg, MC_COUNT) != hipSuccess ||
      mg_alloc(g->owned, g->z, n0) != hipSuccess || mg_alloc(g->owned, g->p, n0) != hipSuccess ||
      mg_alloc(g->owned, g->qv, n0) != hipSuccess || mg_alloc(g->owned, g->z2, n0) != hipSuccess ||
      mg_alloc(g->owned, g->cpart, 2 * RED_BLOCKS) != hipSuccess || mg_alloc(g->owned, g->cs, S_COUNT) != hipSuccess ||
      mg_alloc(g->owned, g->G, 256L * 576) != hipSuccess ||
      hipStreamCreateWithFlags(&g->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&g->h_cg, std::max<int>(MC_COUNT, S_COUNT) * sizeof(double)) != hipSuccess) {
    mg_free(ctx);
    return ctx->fail(AMRTO_ENOMEM, "amrto_mg_setup: out of device memory");
  }
  ctx->mg_valid = false;
  return AMRTO_OK;
}

int amrto_mg_info(amrto_ctx* ctx, int32_t* n_levels, int32_t* dofs, int32_t* dense, int64_t* blocks) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->mg) return ctx->fail(AMRTO_ESTATE, "amrto_mg_info: no multigrid hierarchy");
  MgData* g = ctx->mg;
  if (n_levels) *n_levels = g->nlev;
  for (int k = 0; k < g->nlev; ++k) {
    if (dofs) dofs[k] = 3 * g->lv[k].nn;
    if (dense) dense[k] = g->lv[k].nd;
    if (blocks) blocks[k] = k == 0 ? 0 : g->lv[k].nnzb;
  }
  return AMRTO_OK;
}

int amrto_mg_set_bounds(amrto_ctx* ctx, const double* lam) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->mg) return ctx->fail(AMRTO_ESTATE, "amrto_mg_set_bounds: no multigrid hierarchy");
  MgData* g = ctx->mg;
  if (lam) {
    for (int k = 0; k < g->nlev - 1; ++k)
      if (!(lam[k] > 0.0)) return ctx->fail(AMRTO_EINVAL, "amrto_mg_set_bounds: lambda must be positive");
    for (int k = 0; k < g->nlev - 1; ++k) g->lam_user[k] = lam[k];
  }
  g->user_bounds = lam != nullptr;
  ctx->mg_valid = false;
  return AMRTO_OK;
}

int amrto_mg_get_bounds(amrto_ctx* ctx, double* lam) {
  int rc = check_mg(ctx, "amrto_mg_get_bounds");
  if (rc) return rc;
  if (!lam) return ctx->fail(AMRTO_EINVAL, "amrto_mg_get_bounds: NULL output");
  AMRTO_HIP(hipSetDevice(ctx->device));
  if ((rc = ensure_numeric(ctx))) return rc;
  MgData* g = ctx->mg;
  for (int k = 0; k < g->nlev - 1; ++k)
    AMRTO_HIP(hipMemcpyAsync(&lam[k], g->lv[k].scal + MS_LAM, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  return AMRTO_OK;
}

int amrto_mg_vcycle(amrto_ctx* ctx, const double* r, double* z) {
  int rc = check_mg(ctx, "amrto_mg_vcycle");
  if (rc) return rc;
  if (!r || !z || r == z) return ctx->fail(AMRTO_EINVAL, "amrto_mg_vcycle: r and z must be distinct device buffers");
  AMRTO_HIP(hipSetDevice(ctx->device));
  if ((rc = ensure_numeric(ctx))) return rc;
  if ((rc = vcycle(ctx, r))) return rc;
  MgLevel& L = ctx->mg->lv[0];
  const long n = 3L * L.nn;
  // z = x0 + d0 (the level-0 smoother's last correction); the r.z partials are unused here
  hipLaunchKernelGGL(k_mgcg_rz, dim3(MG_RED), dim3(256), 0, ctx->stream, L.x, L.d, r, z, n, ctx->mg->part,
                     (const double*)nullptr);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_mg_level_apply(amrto_ctx* ctx, int32_t k, const double* x, double* y) {
  int rc = check_mg(ctx, "amrto_mg_level_apply");
  if (rc) return rc;
  MgData* g = ctx->mg;
  if (k < 1 || k >= g->nlev || !x || !y || x == y)
    return ctx->fail(AMRTO_EINVAL, "amrto_mg_level_apply: level out of range or bad buffers");
  AMRTO_HIP(hipSetDevice(ctx->device));
  if ((rc = ensure_numeric(ctx))) return rc;
  MgUpd u = upd(g->lv[k], MG_APPLY);
  u.xin = x;
  u.y = y;
  return level_pass(ctx, g->lv[k], x, u, g->part);
}

int amrto_mg_level_diag(amrto_ctx* ctx, int32_t k, double* dinv) {
  int rc = check_mg(ctx, "amrto_mg_level_diag");
  if (rc) return rc;
  MgData* g = ctx->mg;
  if (k < 1 || k >= g->nlev || !dinv) return ctx->fail(AMRTO_EINVAL, "amrto_mg_level_diag: bad arguments");
  AMRTO_HIP(hipSetDevice(ctx->device));
  if ((rc = ensure_numeric(ctx))) return rc;
  AMRTO_HIP(hipMemcpyAsync(dinv, g->lv[k].dinv, 3L * g->lv[k].nn * sizeof(double), hipMemcpyDeviceToDevice,
                           ctx->stream));
  return AMRTO_OK;
}

int amrto_mg_prolong(amrto_ctx* ctx, int32_t k, const double* xc, double* xf) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->mg) return ctx->fail(AMRTO_ESTATE, "amrto_mg_prolong: no multigrid hierarchy");
  MgData* g = ctx->mg;
  if (k < 1 || k >= g->nlev || !xc || !xf || xc == xf)
    return ctx->fail(AMRTO_EINVAL, "amrto_mg_prolong: level out of range or bad buffers");
  AMRTO_HIP(hipSetDevice(ctx->device));
  MgLevel& C = g->lv[k];
  MgLevel& F = g->lv[k - 1];
  hipLaunchKernelGGL(k_mg_prolong_plain, dim3(blocks_for(F.nn)), dim3(256), 0, ctx->stream, xc, C.pptr, C.pcol, C.pw,
                     F.flag, F.nn, xf);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_mg_restrict(amrto_ctx* ctx, int32_t k, const double* rf, double* rc_out) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->mg) return ctx->fail(AMRTO_ESTATE, "amrto_mg_restrict: no multigrid hierarchy");
  MgData* g = ctx->mg;
  if (k < 1 || k >= g->nlev || !rf || !rc_out || rf == rc_out)
    return ctx->fail(AMRTO_EINVAL, "amrto_mg_restrict: level out of range or bad buffers");
  AMRTO_HIP(hipSetDevice(ctx->device));
  MgLevel& C = g->lv[k];
  launch_restrict(ctx->stream, C, rf, rc_out, 0);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_mg_pass_times(amrto_ctx* ctx, int32_t reps, double* us) {
  int rc = check_mg(ctx, "amrto_mg_pass_times");
  if (rc) return rc;
  if (reps < 1 || !us) return ctx->fail(AMRTO_EINVAL, "amrto_mg_pass_times: bad arguments");
  AMRTO_HIP(hipSetDevice(ctx->device));
  if ((rc = ensure_numeric(ctx))) return rc;
  MgData* g = ctx->mg;
  hipEvent_t e0, e1;
  AMRTO_HIP(hipEventCreate(&e0));
  AMRTO_HIP(hipEventCreate(&e1));
  for (int k = 0; k < g->nlev - 1 && rc == AMRTO_OK; ++k) {
    MgLevel& L = g->lv[k];
    const long n = 3L * L.nn;
    // zero vectors: every pass keeps them zero, so repetitions stay finite
    hipLaunchKernelGGL(k_mg_zero, dim3(blocks_for(n)), dim3(256), 0, ctx->stream, L.x, L.r, n);
    hipLaunchKernelGGL(k_mg_zero, dim3(blocks_for(n)), dim3(256), 0, ctx->stream, L.d, L.q, n);
    if ((rc = pass(ctx, k, L.d, upd(L, MG_CHEB, 0)))) break;  // warm-up
    if (hipEventRecord(e0, ctx->stream) != hipSuccess) { rc = ctx->fail(AMRTO_EHIP, "event"); break; }
    for (int i = 0; i < reps && rc == AMRTO_OK; ++i) rc = pass(ctx, k, L.d, upd(L, MG_CHEB, 0));
    if (rc) break;
    if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = ctx->fail(AMRTO_EHIP, "event");
      break;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    us[k] = 1e3 * (double)ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int amrto_mg_pcg(amrto_ctx* ctx, const double* b, double* u, double rtol, int32_t max_it, int32_t check_every,
                 amrto_solve_stats* stats) {
  int rc = check_mg(ctx, "amrto_mg_pcg");
  if (rc) return rc;
  if (!b || !u || b == u || !(rtol > 0.0) || max_it < 0 || check_every < 1)
    return ctx->fail(AMRTO_EINVAL, "amrto_mg_pcg: bad arguments");
  AMRTO_HIP(hipSetDevice(ctx->device));
  const auto t0 = std::chrono::steady_clock::now();
  if ((rc = ensure_numeric(ctx))) return rc;
  MgData* g = ctx->mg;
  MgLevel& L0 = g->lv[0];
  const long n = 3L * ctx->n_nodes;
  const double tol2 = rtol * rtol;
  double* r = L0.b;  // the CG residual (the level-0 smoother keeps its own in L0.r)
  double* p0 = g->p;
  double* p1 = g->z2;
  // x = u masked; r = b - A~ x; the level-0 smoother starts from r
  hipLaunchKernelGGL(k_mg_mask_copy, dim3(blocks_for(n)), dim3(256), 0, ctx->stream, u, g->qv, L0.flag, n);
  AMRTO_HIP(hipMemcpyAsync(u, g->qv, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  hipLaunchKernelGGL(k_mg_zero, dim3(blocks_for(n)), dim3(256), 0, ctx->stream, p0, p1, n);
  if ((rc = launch_apply(ctx, u, g->qv, AMRTO_FP64))) return rc;
  hipLaunchKernelGGL(k_mgcg_start, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, b, g->qv, L0.flag, r, (long)L0.nn,
                     L0.dinv, L0.binv, L0.scal, L0.x, L0.r, L0.d, g->cpart);
  hipLaunchKernelGGL(k_mgcg_start_scal, dim3(1), dim3(256), 0, ctx->stream, g->cpart, g->cs, tol2);
  AMRTO_HIP(hipGetLastError());
  // every check drains the stream, so runs between checks grow with the
  // predicted distance to the target (next_batch); iterations queued past
  // convergence still run their V-cycle but leave u and the CG state as they
  // are (the CG kernels test the device's finished flag)
  int it = 0, last = 0, status = AMRTO_NOT_CONVERGED;
  double rr0 = 0.0, rr_prev = 0.0;
  while (true) {
    AMRTO_HIP(hipMemcpyAsync(g->h_cg, g->cs, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    AMRTO_HIP(hipStreamSynchronize(ctx->stream));
    const double done = g->h_cg[S_DONE];
    if (done == 1.0) {
      status = AMRTO_OK;
      it = (int)g->h_cg[S_ITERS];
      break;
    }
    if (done == 2.0) {
      status = AMRTO_EBREAKDOWN;
      it = (int)g->h_cg[S_ITERS];
      break;
    }
    if (it >= max_it) break;
    const double rr = g->h_cg[S_RR];
    if (it == 0) rr0 = rr;
    const int batch = next_batch(rr0, rr_prev, rr, it, last, tol2 * g->h_cg[S_BB], check_every, max_it - it);
    rr_prev = rr;
    last = batch;
    for (int k = it; k < it + batch; ++k) {
      // z = V-cycle(r); p = z + beta p_old, q = A~ p and p.q in one fused pass; update
      if ((rc = vcycle_from(ctx, 0))) return rc;
      hipLaunchKernelGGL(k_mgcg_z, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, L0.x, L0.d, r, g->z, n, g->cpart,
                         g->cs);
      double* pnew = (k & 1) ? p1 : p0;
      double* pold = (k & 1) ? p0 : p1;
      CgArgs cg{g->cs, g->cpart, ctx->d_partpq, 0, k, tol2, 0};
      if ((rc = apply_fused(ctx, g->z, pold, pnew, g->qv, AMRTO_FP64, cg))) return rc;
      hipLaunchKernelGGL(k_mgcg_step, dim3(RED_BLOCKS), dim3(256), 0, ctx->stream, u, r, pnew, g->qv, n,
                         ctx->d_partpq, ctx->n_partpq, g->cs, k, L0.dinv, L0.binv, L0.scal, L0.x, L0.r, L0.d);
    }
    AMRTO_HIP(hipGetLastError());
    it += batch;
  }
  // true residual, then u = T u~ (hanging values from their masters, Eq. (9))
  if ((rc = launch_apply(ctx, u, g->qv, AMRTO_FP64))) return rc;
  hipLaunchKernelGGL(k_mgcg_resid, dim3(MG_RED), dim3(256), 0, ctx->stream, b, g->qv, L0.flag, n, g->part);
  hipLaunchKernelGGL(k_mgcg_resid_scal, dim3(1), dim3(256), 0, ctx->stream, g->part, g->cg);
  AMRTO_HIP(hipGetLastError());
  if ((rc = launch_recover(ctx, u, u))) return rc;
  AMRTO_HIP(hipMemcpyAsync(g->h_cg, g->cg, MC_COUNT * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  AMRTO_HIP(hipStreamSynchronize(ctx->stream));
  const double rel = g->h_cg[MC_RES];
  if (status == AMRTO_OK && rel > rtol) status = AMRTO_NOT_CONVERGED;
  if (stats) {
    stats->iters = it;
    stats->outer = 0;
    stats->rel_res = rel;
    stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stats->fell_back = 0;
  }
  if (status == AMRTO_EBREAKDOWN) return ctx->fail(AMRTO_EBREAKDOWN, "amrto_mg_pcg: breakdown");
  if (status == AMRTO_NOT_CONVERGED) ctx->err = "amrto_mg_pcg: not converged";
  return status;
}

}  // extern "C"
