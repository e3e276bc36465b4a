// Internal declarations of the amrto HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "amrto.h"

namespace amrto {
struct MgData;
}

#define AMRTO_HIP(call)                                                          \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      return ctx->fail(AMRTO_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    }                                                                            \
  } while (0)

namespace amrto {

// Uniform-brick apply tile: each workgroup owns UT x UT node columns and a
// range of node layers; it computes the (UT+1)^2 element columns around them
// (one element per thread) and marches upwards one element layer at a time.
constexpr int UT = 15;
constexpr int UE = UT + 1;  // element columns per tile edge
constexpr int UN = UT + 2;  // node columns per tile edge (with halo)
// Brick kernel tile: 16 x BTY node columns per workgroup (one per thread),
// 15 x (BTY - 1) element columns, 14 x (BTY - 2) owned node columns.
#ifndef AMRTO_BRICK_TY
#define AMRTO_BRICK_TY 16
#endif
constexpr int BT = 16;
constexpr int BO = BT - 2;
constexpr int BTY = AMRTO_BRICK_TY;
constexpr int BOY = BTY - 2;
constexpr int BTHREADS = BT * BTY;

// Octree operator chunk: a run of at most CH_MAX consecutive elements plus
// the halo elements around its owned nodes (at most ENT_MAX in all); its node
// table (at most TAB_MAX entries) and hanging triples (at most TRIP_MAX) are
// staged in LDS.
#ifndef AMRTO_CH_MAX
#define AMRTO_CH_MAX 128
#endif
constexpr int CH_MAX = AMRTO_CH_MAX;
constexpr int ENT_MAX = 4 * CH_MAX;
constexpr int TAB_MAX = 8 * CH_MAX;
constexpr int TRIP_MAX = 8 * CH_MAX;  // hanging (node, master, weight) triples per chunk

// Reductions: fixed grid of partial sums; every consumer re-adds them in the
// same order, so results are deterministic without a separate finalize pass.
constexpr int RED_BLOCKS = 512;
constexpr int RED_THREADS = 256;
constexpr int OC_WS = 2 + 1024 * 256 + 256 + 64;  // OC search: bracket, 1024 blocks x 256 partial
                                                   // volumes, 256 candidate volumes
constexpr int COARSE_KMAX = 384;  // coarse-space columns
constexpr int COARSE_NFMAX = 8;  // coarse-space fields (4 affine + caller fields)

template <typename T>
struct DevArray {
  T* p = nullptr;
  size_t n = 0;
};

// Smoothing interval of a multigrid level (device resident): lambda_max
// estimate, theta, delta and sigma = theta / delta of the Chebyshev iteration.
enum { MS_LAM = 0, MS_THETA = 1, MS_DELTA = 2, MS_SIGMA = 3, MS_COUNT = 4 };

// Scalars of a running Krylov solve (device resident).
enum ScalarSlot {
  S_RZ0 = 0,   // r.z, double buffered on iteration parity
  S_RZ1 = 1,
  S_BB = 2,    // b.b
  S_DONE = 3,  // 0 running, 1 converged, 2 breakdown
  S_ITERS = 4, // iterations completed when the flag was raised
  S_RR = 5,    // last r.r
  // 6, 7: true residual r.r and b.b
  S_CTZ = 8,   // coarse space: ct^T E^-1 ct, the coarse part of r.z
  S_AL0 = 9,   // single-reduction CG: alpha, double buffered on iteration parity
  S_AL1 = 10,
  S_COUNT = 12
};

// Arguments of a fused conjugate-gradient step (see kernels.h).
struct CgArgs {
  double* scal;
  const double* part_in;  // r.z and r.r partials of the previous update
  double* part_out;       // p.q partials written by this pass
  int part_base;          // first slot of this kernel in part_out
  int it;
  double tol2;
  int coarse = 0;         // r.z = partial sums + scal[S_CTZ]
  // coarse space in recurrence form: r.z = partial sums + ct^T cz, formed
  // from the ck entries of ct and cz by every block
  const double* cct = nullptr;
  const double* ccz = nullptr;
  int ck = 0;
};

}  // namespace amrto

struct amrto_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  double E0 = 1.0, Emin = 1e-9, nu = 0.3, p = 3.0;
  double K0[576];
  // the eight distinct entries of the mirror-symmetry blocks (brick kernel):
  // a - b, b, d, e, f, g, h - i, i (see k_apply_brick)
  double bk[8];
  std::string err;
  // deterministic mode: LDS accumulations of the octree passes in a fixed order
  bool deterministic = false;

  // mesh
  bool has_mesh = false, uniform = false, has_density = false;
  int n_nodes = 0, n_elems = 0, max_level = 0;
  int nx = 0, ny = 0, nz = 0;
  int n_chunks = 0, n_hang = 0;
  std::vector<int32_t> h_node_xyz;   // octree: lattice coordinates (host copy)
  std::vector<int8_t> h_level;
  std::vector<int32_t> h_elem_nodes;

  // device: material
  double* d_K0 = nullptr;      // 576
  float* d_K0f = nullptr;      // 576
  uint16_t* d_K0bf = nullptr;  // 2 x 576 (hi, lo) bf16 bit patterns
  // device: mesh
  uint8_t* d_fix = nullptr;        // per node, bit c = DOF c supported
  int8_t* d_level = nullptr;       // per element
  int32_t* d_elem_nodes = nullptr; // octree only
  // octree node-owner chunks (chunks.hip)
  int n_entries = 0;                 // chunk elements including halo elements
  int32_t* d_chunk_cnt = nullptr;    // [8 n_chunks] entries, table, triples, owned regular, regular, owned hanging
  // per chunk at fixed strides (ENT_MAX, TAB_MAX, TRIP_MAX), zero padded:
  int32_t* d_ent_elem = nullptr;     // element of each entry
  uint16_t* d_ent_loc = nullptr;     // [8 per entry] table index per local vertex
  int32_t* d_tab_node = nullptr;     // global node per table entry
  uint32_t* d_trip_hm = nullptr;     // (h_loc << 16) | m_loc
  double* d_trip_w = nullptr;
  int32_t* d_tab_hbeg = nullptr;     // per table entry: first triple of a hanging entry
  int32_t* d_hang_node = nullptr;    // [n_hang]
  int32_t* d_hang_ptr = nullptr;     // [n_hang + 1]
  int32_t* d_hang_master = nullptr;
  double* d_hang_w = nullptr;
  int n_mt = 0;                      // masters that receive hanging loads
  int32_t* d_mt_node = nullptr;      // [n_mt]
  int32_t* d_mt_ptr = nullptr;       // [n_mt + 1]
  int32_t* d_mt_h = nullptr;         // hanging node per entry
  double* d_mt_w = nullptr;          // weight per entry
  // octree filter (built at upload): element descriptors (anchor, edge) and
  // the finest-lattice cell map (leaf per cell, bit 31 on its anchor cell)
  int filt_hmax = 1;
  int32_t* d_edesc = nullptr;   // [4 n_elems]
  int32_t* d_cmap = nullptr;    // [nx ny nz]

  // device: density dependent
  double* d_coef = nullptr;   // c_e
  float* d_coef_f = nullptr;
  double* d_dinv = nullptr;   // 1 / diag(A~)
  float* d_dinv_f = nullptr;
  double* d_vol = nullptr;    // V_e

  // device: solver workspace
  double* d_r = nullptr; double* d_z = nullptr; double* d_p = nullptr; double* d_q = nullptr;
  double* d_p2 = nullptr; float* f_p2 = nullptr;
  double* d_partpq = nullptr; // p.q partials of the fused operator passes
  // single-reduction CG on octree meshes: second r buffer, w and s pairs, and
  // the gamma / delta / r.r partials of two passes
  double* d_cg1_r2 = nullptr; double* d_cg1_w = nullptr; double* d_cg1_w2 = nullptr;
  double* d_cg1_s = nullptr; double* d_cg1_s2 = nullptr; double* d_cg1_part = nullptr;
  // block-Jacobi: inverse 3x3 node blocks (6 entries per node), computed on
  // the first block-Jacobi solve after a density change
  double* d_binv = nullptr;
  float* d_binv_f = nullptr;
  bool binv_valid = false;
  int n_partpq = 0;
  float* f_b = nullptr; float* f_x = nullptr; float* f_r = nullptr; float* f_z = nullptr; float* f_p = nullptr; float* f_q = nullptr;
  double* d_part = nullptr;   // reduction partials (4 x RED_BLOCKS)
  double* d_scal = nullptr;   // scalar slots
  double* h_scal = nullptr;   // pinned mirror
  double* d_oc = nullptr;     // OC search workspace
  double* d_oc_scratch = nullptr;  // device address of the file-scope OC scratch on this device
  // coarse space (coarse.hip)
  int coarse_k = 0, coarse_nf = 0, coarse_R = 0, coarse_cap = 0;
  int coarse_affine_only = 0;   // fields generated on the fly by the solve kernels
  uint8_t* d_cmask = nullptr;   // per node: bit c = DOF c supported or hanging
  float4* d_cgeo = nullptr;     // affine space: per node (dx, dy, dz, region | mask << 8)
  double* d_cf = nullptr;      // n_fields x 3n fields (masked)
  uint8_t* d_region = nullptr; // region of each node
  double* d_cpart = nullptr;   // RED_BLOCKS x COARSE_KMAX partials (block-major)
  double* d_cinv = nullptr;    // E^-1 (k x k)
  std::vector<double> h_gram;  // E as formed (host copy)
  double* d_ct = nullptr;      // Z^T r of the current iteration
  double* d_cz = nullptr;      // E^-1 Z^T r
  // recurrence form (octree, affine space): per operator-pass block, the
  // partials of Z^T q and E^-1 Z^T q (2 k x blocks, column-major)
  double* d_cqpart = nullptr;
  long cq_cap = 0;
  // Gram matrix on octree meshes (coarse.hip): region masks per chunk, and
  // tiles + tile offsets + per-pair tile lists
  uint32_t* d_gram_mask = nullptr;
  long gram_mask_cap = 0;
  void* d_gram = nullptr;
  size_t gram_cap = 0;
  int coarse_exact_it = 0;      // iteration at which ct, cz were last formed from r
  bool coarse_fresh = false;    // ct, cz were just formed from r (coarse_init)
  // Krylov recycling (recycle.hip): recorded residuals of one solve
  // (rec_m x 3n, FP64), their coefficients (r.z at 2j, p.q at 2j + 1, the
  // counts of stored vectors and coefficient pairs at 2 REC_MMAX and
  // 2 REC_MMAX + 1), combination coefficients, and the Rayleigh-Ritz
  // workspace (A~ s_j for up to 16 vectors, partials)
  int rec_m = 0;
  bool rec_active = false;      // the running solve records
  bool rec_block3 = false, rec_coarse = false;  // its preconditioner
  double* d_rec_store = nullptr;
  double* d_rec_coef = nullptr;
  double* d_rec_C = nullptr;
  double* d_rr_aw = nullptr;
  double* d_rr_part = nullptr;
  // mesh <-> grid transfers (net.hip)
  int grid_cell = 0;
  int32_t* d_node_xyz = nullptr;
  int32_t* d_cell_ptr = nullptr;   // [cells + 1] elements overlapping each grid cell
  int32_t* d_cell_elem = nullptr;
  double* d_cell_w = nullptr;      // overlap volume / cell volume
  int32_t* d_gn_node = nullptr;    // [8 grid nodes] mesh nodes interpolated at each grid node
  float* d_gn_w = nullptr;         // [8 grid nodes] their trilinear weights

  // geometric multigrid (mg.hip): hierarchy of the uploaded mesh; its
  // numeric part (Galerkin matrices, smoothing intervals, coarsest inverse)
  // is rebuilt on first use after a density or material change
  amrto::MgData* mg = nullptr;
  bool mg_valid = false;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
};

namespace amrto {

// apply.hip
int launch_apply(amrto_ctx* ctx, const void* x, void* y, int prec);
int launch_diag(amrto_ctx* ctx);
int build_chunks(amrto_ctx* ctx, const amrto_mesh* m);
// recycle.hip
int recycle_begin(amrto_ctx* ctx, bool block3);
template <typename VT>
int recycle_store(amrto_ctx* ctx, const VT* r, int it);
// pcg.hip
int apply_precond(amrto_ctx* ctx, const double* s, double* u, bool block3, bool coarse);
// mg.hip
void mg_free(amrto_ctx* ctx);
// topopt.hip
int build_cell_map(amrto_ctx* ctx);
int oc_scratch_attach(amrto_ctx* ctx);
// vec.hip
int launch_set_density(amrto_ctx* ctx, const double* rho);
int launch_project_rhs(amrto_ctx* ctx, const double* f, double* b);
int launch_recover(amrto_ctx* ctx, const double* ut, double* u);
int launch_recip(amrto_ctx* ctx, const double* a, double* b, long n);
int mask_vector(amrto_ctx* ctx, double* x);
int mask_vector_n(amrto_ctx* ctx, double* x, int count);
int launch_zt(amrto_ctx* ctx, const double* v);
int apply_stop(amrto_ctx* ctx, const void* x, void* y, int prec, const double* stop);
int apply_cheb(amrto_ctx* ctx, const double* d, double* dnew, int mode, int step, const double* scal,
               const double* dinv, double* x, double* r, const double* binv = nullptr);
int apply_fused(amrto_ctx* ctx, const void* z, const void* pold, void* pnew, void* q, int prec, const CgArgs& cg);
int block3_setup(amrto_ctx* ctx);
template <typename VT, typename BT>
int block3_init(amrto_ctx* ctx, const BT* b, const BT* q, VT* r, VT* z);
template <typename VT>
int block3_update(amrto_ctx* ctx, VT* x, VT* r, const VT* p, const VT* q, VT* z, int it);
bool cg1_available(const amrto_ctx* ctx);
int cg1_parts(const amrto_ctx* ctx);
int cg1_init(amrto_ctx* ctx);
int cg1_enqueue(amrto_ctx* ctx, double* x, double tol2, int it0, int count);
int apply_fused_coarse(amrto_ctx* ctx, const void* r, const void* minv, const void* pold, void* pnew, void* q,
                       int prec, const CgArgs& cg, bool block3 = false, double* zq_part = nullptr);
int apply_blocks(const amrto_ctx* ctx);
void uniform_grid(const amrto_ctx* ctx, int& tiles_x, int& tiles_y, int& zchunk, int& n_tiles, int& grid);
// iterations a Krylov solve enqueues before its next host convergence check,
// from r.r at the start (rr0), at the previous check (rr_prev, last
// iterations ago) and now (rr, its iterations in): check_every while nothing
// is known, then 3/4 of the iterations the residual still needs to reach
// target, between check_every and 8 check_every, at most left
int next_batch(double rr0, double rr_prev, double rr, int its, int last, double target, int check_every, int left);

// helpers
void k0_unit_cube(double nu, double* K);  // 24 x 24, E = 1
uint16_t f32_to_bf16_rne(float f);
float bf16_to_f32(uint16_t h);
int grid_for(long n, int threads, int cap);

}  // namespace amrto
