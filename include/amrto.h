/*
 * amrto.h - C ABI of the MI355X (gfx950) hot path for dynamic-AMR SIMP
 * topology optimisation (Wang, de Sturler, Paulino, "Dynamic Adaptive Mesh
 * Refinement for Topology Optimization", arXiv:1009.4975).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every function returns int.  0 = AMRTO_OK; negative values are
 *   errors; AMRTO_NOT_CONVERGED (+1) is a warning whose outputs hold the last
 *   iterate.  No exception crosses the ABI.  amrto_last_error() returns a
 *   per-context message for the most recent failure.
 * - Memory: pointers named *_dev are device pointers owned by the caller
 *   (for example torch tensors); pointers named *_host or inside mesh structs
 *   are host pointers, read during the call only.  The context owns its copies
 *   of mesh data, its coefficient arrays and its solver workspace.  Hot calls
 *   (apply, pcg, compliance, filter, oc) allocate nothing.
 * - Streams: all device work is enqueued on the stream given to
 *   amrto_create().  Calls are asynchronous except those that return host
 *   scalars (c_host, change_host, stats), which synchronise the stream.
 * - Mesh: nodes sit on the finest integer lattice (finest element edge 1; an
 *   element of level l in a tree with max_level L has edge h = 2^(L-l)).
 *   DOF vectors are node-major interleaved: dof = 3*node + c (c = x, y, z).
 *   Element local node a = i + 2j + 4k is the vertex at offset (i, j, k).
 * - Operator (paper Sec. 6, Eq. (6)-(8), supports handled as identity rows):
 *       A~ = F T^T K T F + (I - F)
 *   K = sum_e c_e G_e^T K0 G_e with c_e = (Emin + rho_e^p (E0 - Emin)) h_e
 *   (Sec. 3, Eq. (2)); T interpolates hanging DOFs from their masters
 *   (Eq. (6)); F masks out hanging and supported DOFs.  Rows of hanging and
 *   supported DOFs are the identity.
 */
#ifndef AMRTO_H
#define AMRTO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  AMRTO_OK = 0,
  AMRTO_NOT_CONVERGED = 1,
  AMRTO_EINVAL = -1,     /* bad argument, size or mesh table */
  AMRTO_EHIP = -2,       /* a HIP runtime call failed */
  AMRTO_ENOMEM = -3,     /* device or host allocation failed */
  AMRTO_EBREAKDOWN = -4, /* p^T A p <= 0, NaN or Inf inside a Krylov solve */
  AMRTO_ESTATE = -5      /* call out of order (no mesh, no density, ...) */
};

/* Precision of the element contraction and of the vectors it reads/writes. */
enum {
  AMRTO_FP64 = 0, /* FP64 vectors, FP64 contraction */
  AMRTO_FP32 = 1, /* FP32 vectors, FP32 contraction */
  AMRTO_BF16 = 2  /* FP32 vectors, BF16 operands with FP32 accumulation */
};

/* Preconditioners of amrto_pcg: JACOBI = the exact diagonal of A~ (the
 * diagonal rescaling of Sec. 5); BLOCK3 = the 3x3 node blocks of A~ (all
 * components of a node), alone or, on an octree mesh, added to the affine
 * coarse space (M^-1 = B^-1 + Z E^-1 Z^T). */
enum { AMRTO_PRECOND_JACOBI = 0, AMRTO_PRECOND_BLOCK3 = 1 };
enum { AMRTO_FILTER_SENSITIVITY = 0, AMRTO_FILTER_DENSITY = 1 };

typedef struct amrto_ctx amrto_ctx;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`; `hip_stream` (hipStream_t, may be
 * NULL for the null stream) is used by every later call.  *ctx receives the
 * handle.  Errors: EINVAL (ctx NULL, bad device), EHIP. */
int amrto_create(amrto_ctx** ctx, int device, void* hip_stream);
/* Free all device memory owned by the context.  NULL is accepted. */
int amrto_destroy(amrto_ctx* ctx);
/* Message of the most recent error on this context ("" if none).  The string
 * is owned by the context and valid until the next call on it. */
const char* amrto_last_error(const amrto_ctx* ctx);
/* Replace the stream used by later calls. */
int amrto_set_stream(amrto_ctx* ctx, void* hip_stream);
/* Deterministic mode (on != 0).  The octree passes sum element contributions
 * in workgroup-local FP64 accumulators; by default the waves of a workgroup
 * add to them in the order they happen to run, so the last bits of y = A~ x,
 * of the diagonal and of the coarse-space sums, and with them iteration
 * counts, can vary from run to run.  In deterministic mode the waves take
 * turns in a fixed order and hanging-node condensation runs in one wave, so
 * every result depends only on the inputs (same device, same build).  It
 * covers the operator passes of every precision and solver form, the Jacobi
 * diagonal and node blocks, the coarse-space passes and the multigrid; the
 * uniform-brick passes are deterministic in both modes.  Costs time on the
 * octree passes.  Switching recomputes the diagonal now and the node-block
 * inverses and multigrid operators when next used; a coarse space formed
 * before the switch keeps its Gram matrix until amrto_coarse_setup runs
 * again.  Default off.  Errors: none beyond a HIP failure of the diagonal. */
int amrto_set_deterministic(amrto_ctx* ctx, int32_t on);

/* SIMP material law E(rho) = Emin + rho^p (E0 - Emin) (Sec. 3, Eq. (2);
 * Emin plays the role of the density floor rho_o^p) and Poisson ratio nu,
 * which fixes the unit-cube element matrix K0.  Defaults: 1, 1e-9, 0.3, 3.
 * Errors: EINVAL (E0 <= Emin, Emin < 0, nu outside (-1, 0.5), p < 1). */
int amrto_set_material(amrto_ctx* ctx, double E0, double Emin, double nu, double p);

/* ------------------------------------------------------------------ mesh */

/* A mesh as host arrays (copied by amrto_upload_mesh).
 * Uniform brick: elem_nodes == NULL; dims gives the element counts, nodes and
 * elements are numbered lexicographically with x fastest, every element has
 * h = 1 and there are no hanging nodes (n_hang must be 0).
 * Octree: elem_nodes[8*e + a] gives the node of local vertex a; elem_level
 * gives levels (h_e = 2^(max_level - level)); node_xyz gives lattice
 * coordinates; elements should be in space-filling-curve order for locality.
 * Hanging nodes (Eq. (6)): hang_node[i] is interpolated as
 *   u[hang_node[i]] = sum_{k in [hang_ptr[i], hang_ptr[i+1])} hang_w[k] u[hang_master[k]],
 * masters must not be hanging themselves (chains resolved by the caller).
 * dof_fixed[3*n + c] != 0 marks a supported DOF (u = 0 there, Eq. (1)). */
typedef struct {
  int32_t n_nodes;
  int32_t n_elems;
  int32_t dims[3];            /* finest-lattice extents in elements */
  int32_t max_level;          /* 0 for a uniform brick */
  const int32_t* node_xyz;    /* [3*n_nodes] or NULL for a uniform brick */
  const int32_t* elem_nodes;  /* [8*n_elems] or NULL for a uniform brick */
  const int8_t* elem_level;   /* [n_elems] or NULL (all max_level) */
  int32_t n_hang;
  const int32_t* hang_node;   /* [n_hang] */
  const int32_t* hang_ptr;    /* [n_hang + 1] */
  const int32_t* hang_master; /* [hang_ptr[n_hang]] */
  const double* hang_w;       /* [hang_ptr[n_hang]] */
  const uint8_t* dof_fixed;   /* [3*n_nodes] */
} amrto_mesh;

/* Copy a mesh to the device, build the element chunks, node tables, the
 * hanging-node tables and the solver workspace.  Replaces any earlier mesh
 * (densities must be set again).  Errors: EINVAL (inconsistent sizes, node
 * indices out of range, a hanging master that is hanging, a chunk whose node
 * table cannot fit, 3 n_nodes or 8 n_elems not below 2^31, an octree whose
 * finest lattice has more than 2^30 cells: the filter's cell map holds one
 * int32 per cell), ENOMEM, EHIP. */
int amrto_upload_mesh(amrto_ctx* ctx, const amrto_mesh* mesh);

/* Sizes of the uploaded mesh. */
int amrto_mesh_info(const amrto_ctx* ctx, int32_t* n_nodes, int32_t* n_elems, int32_t* n_chunks);

/* Element densities rho_dev[n_elems] (FP64, caller-owned, read only): computes
 * c_e (Eq. (2) scaled by h_e), the exact diagonal of A~ (Jacobi, the diagonal
 * rescaling of Sec. 5) and the FP32 copies used by mixed precision.
 * Errors: ESTATE (no mesh), EHIP. */
int amrto_set_density(amrto_ctx* ctx, const double* rho_dev);

/* ------------------------------------------------------------------ operator */

/* y = A~ x over all 3*n_nodes DOFs (Sec. 6, Eq. (8)).  prec = AMRTO_FP64:
 * x_dev, y_dev are double; AMRTO_FP32 / AMRTO_BF16: float.  x and y must not
 * alias.  Errors: ESTATE, EINVAL (prec). */
int amrto_apply(amrto_ctx* ctx, const void* x_dev, void* y_dev, int prec);

/* b = F T^T f: condense a consistent load on all nodes onto unconstrained
 * DOFs (right-hand side of Eq. (7)) and zero supported/hanging entries. */
int amrto_project_rhs(amrto_ctx* ctx, const double* f_dev, double* b_dev);

/* u = T u~: recover hanging DOFs from their masters (Eq. (9)); unconstrained
 * entries are copied.  u_dev and ut_dev may alias. */
int amrto_recover(amrto_ctx* ctx, const double* ut_dev, double* u_dev);

/* Diagonal of A~ (as used by the Jacobi preconditioner) into diag_dev[3n]. */
int amrto_get_diag(amrto_ctx* ctx, double* diag_dev);

/* The 3x3 node blocks of A~ (as used by the block-Jacobi preconditioner,
 * before inversion) into blocks_dev[9n], row-major per node: supported
 * components carry identity rows and columns, hanging nodes the identity.
 * Errors: ESTATE (no density), EINVAL. */
int amrto_get_block_diag(amrto_ctx* ctx, double* blocks_dev);

/* ------------------------------------------------------------------ solve */

typedef struct {
  double rtol;        /* stop when ||b - A~ u||_2 <= rtol ||b||_2 (default 1e-8) */
  int32_t max_it;     /* iteration cap of the (inner) CG (default 20000) */
  int32_t precond;    /* AMRTO_PRECOND_JACOBI (default) or AMRTO_PRECOND_BLOCK3
                         (any precision, two-pass form; with a coarse space
                         only the affine one on an octree mesh: EINVAL
                         otherwise) */
  int32_t inner_prec; /* AMRTO_FP64: plain PCG; FP32/BF16: mixed precision with
                         FP64 reliable updates (FP32 vectors, FP32/BF16 operator) */
  double inner_rtol;  /* mixed precision: factor by which the FP32 recurrence
                         residual falls between two FP64 reliable updates
                         (default 0.1; a recurrence that levels off above its
                         target for 2048 iterations is updated anyway) */
  int32_t check_every;/* shortest run of iterations between host convergence
                          checks (default 16); runs grow to at most 8x this
                          while the residual's convergence rate says the
                          target is further away */
  int32_t use_coarse; /* 1 (default): add the coarse correction set by
                         amrto_coarse_setup, when one is set; 0: Jacobi only */
  int32_t fallback_fp64; /* 1 (default): a mixed solve that breaks down or
                         stalls above rtol continues as plain FP64 PCG from
                         its iterate (from zero if that is not finite) */
  int32_t single_reduction; /* 1: plain FP64 Jacobi-PCG on an octree mesh runs
                         the one-reduction recurrences of Chronopoulos and
                         Gear (one pass per iteration, same iterates in exact
                         arithmetic); 0 (default): two passes, which measured
                         faster on the octree cantilever (the one pass carries
                         the update's gathers and is as long as both) */
  int32_t record;     /* 1: keep the first m residuals and the CG
                         coefficients of this solve for amrto_recycle_harvest
                         (needs amrto_recycle_setup; any precision and
                         preconditioner of the two-pass form; only the first
                         CG run of a solve, or the first cycle of a mixed
                         solve, is recorded).  0 (default): nothing recorded */
} amrto_solve_opts;

typedef struct {
  int32_t iters;       /* total CG iterations (inner iterations summed) */
  int32_t outer;       /* FP64 reliable updates (mixed) or residual-replacement
                          restarts (plain FP64) */
  double rel_res;      /* true FP64 ||b - A~ u|| / ||b|| at exit */
  double ms;           /* wall time of the call */
  int32_t fell_back;   /* 1 if a mixed solve was finished by plain FP64 PCG */
} amrto_solve_stats;

/* Fill opts with the defaults above. */
void amrto_solve_opts_default(amrto_solve_opts* opts);

/* Solve A~ u~ = b by Jacobi-preconditioned conjugate gradients (FP64; when the
 * recurrence residual converges but the true residual does not, CG restarts
 * from the iterate with r = b - A~ u, up to 8 times while each restart halves
 * the true residual), or by
 * the same recurrence in FP32 vectors with an FP32 or BF16 element contraction
 * whose iterate is folded into an FP64 solution with an FP64 true residual
 * whenever the recurrence residual has fallen by inner_rtol (reliable
 * updates); convergence is always judged on the FP64 true residual.
 * u_dev: in = initial guess (its hanging and supported entries are ignored),
 * out = u = T u~ with hanging DOFs recovered (Eq. (9)).  b_dev = F T^T f.
 * With a coarse space, M^-1 = D^-1 + Z (Z^T A~ Z)^-1 Z^T (an SPD two-level
 * preconditioner).  Returns NOT_CONVERGED when the cap is reached; EBREAKDOWN
 * on p^T A p <= 0 or non-finite values. */
int amrto_pcg(amrto_ctx* ctx, const double* b_dev, double* u_dev,
              const amrto_solve_opts* opts, amrto_solve_stats* stats);

/* Measurement of the solver's two passes per iteration: the variant named by
 * opts (precision, preconditioner, coarse space in use) is started from
 * u_dev as amrto_pcg starts it, run for two iterations, then its operator
 * pass (stiffness apply fused with the preconditioner and the search
 * direction update) is launched reps times back to back, then its update
 * side (vector updates, preconditioner, reductions, coarse-space recurrences)
 * reps times; *op_us and *update_us receive the mean device time of one
 * launch of each from HIP events on the context stream.  u_dev is left
 * masked and otherwise unchanged (FP64 variants use it as the iterate and
 * leave it overwritten); nothing else computed is a result, and the next
 * amrto_pcg starts afresh.  Synchronises.  Errors as amrto_pcg; EINVAL for
 * reps outside [1, 100000]. */
int amrto_pcg_pass_times(amrto_ctx* ctx, const double* b_dev, double* u_dev, const amrto_solve_opts* opts,
                         int32_t reps, double* op_us, double* update_us);

/* ------------------------------------------------------------------ recycling
 * Krylov subspace recycling across the systems of a design sequence (Sec. 5:
 * an approximate invariant subspace for the smallest eigenvalues, taken from
 * one solve's Krylov space, is carried to the next system).  A recorded solve
 * keeps its first m residuals r_j with r_j^T z_j and p_j^T A~ p_j (z_j =
 * M^-1 r_j); their Lanczos matrix T (T[j][j] = 1/alpha_j +
 * beta_{j-1}/alpha_{j-1}, T[j][j+1] = sqrt(beta_j)/alpha_j, Lanczos vectors
 * (-1)^j z_j / sqrt(r_j^T z_j)) gives Ritz pairs of the solve's preconditioned
 * operator.  The caller starts the next solve from the Galerkin projection of
 * its initial error onto them (amrto_energy_combine), or passes them to
 * amrto_coarse_setup as fields after Rayleigh-Ritz for the pencil (A~, D),
 * D = diag(A~), has picked the best k directions for the current system. */

/* Allocate the recording store (m x 3 n_nodes doubles plus Rayleigh-Ritz
 * workspace of 16 x 3 n_nodes) for the uploaded mesh; 2 <= m <= 256.  A new
 * mesh drops it.  Errors: EINVAL, ESTATE (no mesh), ENOMEM, EHIP. */
int amrto_recycle_setup(amrto_ctx* ctx, int32_t m);
/* From the last recorded solve, with the coarse space (if it used one) and
 * density it ran with still set: the k (1..16) smallest Ritz values
 * (theta_host, may be NULL), their Lanczos residual norms
 * |T[m-1][m] y_{m-1}| = ||A~ u - theta M u||_{M^-1} (resid_host, may be NULL),
 * the Ritz vectors u_i = V y_i into the k device vectors u_host[i] (3 n FP64,
 * M-normalised, zero on supported and hanging DOFs; the solve's FP64
 * preconditioner is applied once per vector) and the number of Lanczos steps
 * used (*m_used, may be NULL: the recorded steps minus one).  Synchronises.
 * Errors: ESTATE (nothing recorded, or fewer than k + 1 steps), EINVAL,
 * EBREAKDOWN (a non-positive recorded coefficient). */
int amrto_recycle_harvest(amrto_ctx* ctx, int32_t k, double* const* u_host, double* theta_host,
                          double* resid_host, int32_t* m_used);
/* Rayleigh-Ritz: the k smallest pairs of S^T A~ S y = theta S^T D S y over
 * the span of the n (1..16) device vectors s_host[i] (3 n FP64, masked),
 * D = diag(A~) of the current density; w_host[i] (k outputs, distinct from
 * the inputs) receive W = S Y with W^T D W = I, theta_host (may be NULL) the
 * values, *rank (may be NULL) the number of independent input directions
 * kept (eigenvalues of S^T D S above 1e-12 of the largest).  Synchronises.
 * Errors: ESTATE (no density or no amrto_recycle_setup), EINVAL (sizes,
 * aliasing, inputs spanning fewer than k directions). */
int amrto_rayleigh_ritz(amrto_ctx* ctx, const double* const* s_host, int32_t n, int32_t k,
                        double* const* w_host, double* theta_host, int32_t* rank);

/* ------------------------------------------------------------------ design */

/* Compliance c = f^T u (Eq. (1)) into *c_host (may be NULL) and, if dc_dev is
 * not NULL, dc_e = -p rho_e^(p-1) (E0 - Emin) h_e u_e^T K0 u_e (the
 * self-adjoint sensitivity; Sec. 3).  u_dev: all DOFs, hanging recovered. */
int amrto_compliance(amrto_ctx* ctx, const double* u_dev, const double* f_dev,
                     const double* rho_dev, double* c_host, double* dc_dev);

/* Filters of Sec. 6 with H_de = max(rmin - |x_d - x_e|, 0) between element
 * centres (Eq. (4)) and volume weights (Eq. (5)):
 *  SENSITIVITY: out_e = sum_d rho_d H V_d in_d / (max(rho_e, 1e-3) sum_d H V_d)
 *  DENSITY:     out_e = sum_d H V_d in_d / sum_d H V_d
 * rho_dev is ignored in DENSITY mode.  in/out must not alias.  Any rmin in
 * (0, 16] (finest-lattice units) works on the same mesh: neighbours are found
 * on the device from the lattice cell map built by amrto_upload_mesh, so the
 * call builds, copies and allocates nothing.  Errors: EINVAL (mode, rmin,
 * NULL or aliased buffers), ESTATE (no mesh). */
int amrto_filter(amrto_ctx* ctx, int mode, double rmin, const double* in_dev,
                 const double* rho_dev, double* out_dev);

/* Optimality Criteria step (Sec. 3): rho_new = clamp(rho (-dc/(lam V_e))^eta,
 * max(rho_min, rho - move), min(1, rho + move)) with lam such that
 * sum rho_new V_e = volfrac * sum V_e (k-ary search on log lam to relative
 * width 1e-13).  *change_host (may be NULL) = max |rho_new - rho|;
 * *lam_host (may be NULL) = lam. */
int amrto_oc_update(amrto_ctx* ctx, const double* rho_dev, const double* dc_dev,
                    double volfrac, double move, double eta, double rho_min,
                    double* rho_new_dev, double* change_host, double* lam_host);

/* amrto_oc_update for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, kernels and results, but its search workspace is a
 * file-scope device array of the library (262,466 doubles, 2.1 MB,
 * one copy per GPU, held until the process ends; its address is looked up at
 * amrto_create) instead of the context's buffer, and the host results come
 * back through the context's pinned scalar buffer.  The call allocates and
 * frees nothing.  The workspace does not grow with the mesh (the search uses
 * at most 1024 blocks of partial volumes whatever n_elems), so every mesh the
 * context accepts fits; a layout that would not fit is rejected with EINVAL.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (each call writes every entry it reads before reading it):
 * overlapping calls on one GPU, from any context or stream, race.
 * Errors as amrto_oc_update; ESTATE if the scratch address is unknown. */
int amrto_oc_update_noalloc(amrto_ctx* ctx, const double* rho_dev, const double* dc_dev,
                            double volfrac, double move, double eta, double rho_min,
                            double* rho_new_dev, double* change_host, double* lam_host);

/* Relative difference of two designs (Sec. 7, Eq. (10)):
 *   D = int |rho_a - rho_b| dOmega / int rho_a dOmega,
 * evaluated on the finest lattice after carrying both designs to the finest
 * level everywhere (each cell takes its covering leaf's density; a uniform
 * brick's elements are the cells).  rho_a_dev / rho_b_dev: per-element
 * densities of the meshes uploaded to contexts a and b, which must be on one
 * device and cover the same lattice box.  The work runs on a's stream; b's
 * densities must be ready.  Synchronises a's stream.  Errors: EINVAL
 * (different boxes or devices, NULL), ESTATE (no mesh). */
int amrto_design_difference(amrto_ctx* a, const double* rho_a_dev, const amrto_ctx* b,
                            const double* rho_b_dev, double* D_host);

/* Zero the supported and hanging entries of a DOF vector x_dev[3n] in place
 * (the entries whose rows of A~ are the identity with zero right-hand side). */
int amrto_mask(amrto_ctx* ctx, double* x_dev);

/* ------------------------------------------------------------------ learned warm start
 * (not in the paper, whose solves start from the previous displacement,
 * Sec. 5: a network's prediction of the displacement change refines that
 * start, and a Galerkin coarse space accelerates the Jacobi-PCG; the plain
 * solve judges every result) */

/* Two-level preconditioner M^-1 = D^-1 + Z (Z^T A~ Z)^-1 Z^T used by
 * amrto_pcg while set (SPD for any Z, so CG stays valid).  The lattice box is
 * split into rx x ry x rz equal regions; column (f, g, c) of Z is component
 * c of field f on the nodes of region g, zero elsewhere.  The fields are, in
 * this order: with affine != 0, the four affine fields (1,1,1), (x,y,z),
 * (y,z,x), (z,x,y) (centred coordinates; per region they span the rigid
 * motions and the constant strains), then the n_fields caller fields
 * (fields_host: host array of device pointers to 3n FP64 vectors; copied).
 * Every field is masked (zero on supported and hanging DOFs).  At most 8
 * fields in all, and k = 3 rx ry rz (4 affine + n_fields) <= 384.  Z^T A~ Z is
 * formed on the device (for the affine space alone on an octree mesh in one
 * pass over the chunks: each forms A~ z_j for the columns whose region meets
 * it; otherwise by k operator applications) and factorised on the host,
 * dropping columns whose pivot falls below 1e-12 of the largest (*k_kept
 * receives the rank kept; may be NULL).  Needs the density set;
 * amrto_set_density drops the coarse space.
 * Errors: EINVAL (bad sizes, k > 384, a field with non-finite values; the
 * solve then runs without a coarse space), ESTATE, EHIP. */
int amrto_coarse_setup(amrto_ctx* ctx, int32_t affine, const double* const* fields_host, int32_t n_fields,
                       int32_t rx, int32_t ry, int32_t rz, int32_t* k_kept);
/* Stop using the coarse space (plain Jacobi again). */
int amrto_coarse_clear(amrto_ctx* ctx);
/* The Gram matrix E = Z^T A~ Z of the current coarse space as formed (before
 * factorisation) into E_host (row-major k x k; cap = its length in doubles),
 * *k = the coarse dimension.  Errors: ESTATE (no coarse space), EINVAL
 * (cap < k^2 or NULL arguments). */
int amrto_coarse_gram(amrto_ctx* ctx, double* E_host, int64_t cap, int32_t* k);
/* x0 = base + sum_j a_j v_j with a minimising the energy 1/2 x^T A~ x - b^T x
 * (base_dev may be NULL: zero), so x0 is never worse in the energy norm than
 * base or any single v_j.  vecs_host: host array of n (1..8) device pointers;
 * base and the vectors should be masked.  coef_host (may be NULL) receives a.
 * x0_dev must not alias base or the vectors.  EINVAL if a vector or the base
 * residual is not finite (x0 is then left untouched). */
int amrto_energy_combine(amrto_ctx* ctx, const double* b_dev, const double* base_dev,
                         const double* const* vecs_host, int32_t n, double* x0_dev, double* coef_host);

/* Mesh -> regular grid with nodes every `cell` lattice units (cell divides
 * every extent; gx = nx / cell etc.), node-major arrays (z, y, x) of
 * (gz+1)(gy+1)(gx+1) values, FP32:
 *   rho_grid = exact volume average of rho over each grid node's dual cell
 *              (the box of edge `cell` centred at the node, clipped to the domain);
 *   u_grid (3 components one after the other) = u_scale times the FE
 *              displacement u - u_ref (u_ref may be NULL), trilinear on the
 *              element holding the grid node.
 * Either output may be NULL.  The transfer tables are built on the first call
 * for a given cell (host work, then cached with the mesh). */
int amrto_grid_from_mesh(amrto_ctx* ctx, int32_t cell, const double* rho_dev, const double* u_dev,
                         const double* u_ref_dev, double u_scale, float* rho_grid_dev, float* u_grid_dev);
/* u_dev[3n] = scale times the trilinear interpolation of u_grid (layout as
 * above) at every mesh node (hanging nodes included; a solve ignores them). */
int amrto_grid_to_mesh(amrto_ctx* ctx, int32_t cell, const float* u_grid_dev, double scale, double* u_dev);

/* A fully convolutional network on a gx x gy x gz grid: n_layers 3x3x3
 * convolutions (stride 1, zero padding), channels[0..n_layers], ReLU between
 * layers, FP32; with skip_from >= 0 the output adds the input channels
 * [skip_from, skip_from + channels[n_layers]) (a residual connection).
 * Parameters are stored layer by layer as w (Cout, Cin, 3, 3, 3) then b
 * (Cout); initial weights are He-normal, N(0, 2 / (27 Cin)), drawn as
 * Box-Muller pairs of SplitMix64 outputs of (seed XOR counter); biases zero.
 * Work is enqueued on hip_stream.  Buffers are allocated here only. */
typedef struct amrto_net amrto_net;
int amrto_net_create(amrto_net** net, int device, void* hip_stream, int32_t n_layers, const int32_t* channels,
                     int32_t skip_from, int32_t gx, int32_t gy, int32_t gz, int32_t max_batch, uint64_t seed);
int amrto_net_destroy(amrto_net* net);
const char* amrto_net_last_error(const amrto_net* net);
int amrto_net_n_params(const amrto_net* net, int64_t* n);
/* host copies of all parameters / of the gradients of the last backward */
int amrto_net_get_params(const amrto_net* net, float* host);
int amrto_net_set_params(amrto_net* net, const float* host);
int amrto_net_get_grads(const amrto_net* net, float* host);
/* host copies of the Adam first and second moments (n_params each), for a
 * checkpoint; set rejects non-finite moments and negative second moments */
int amrto_net_get_adam(const amrto_net* net, float* m_host, float* v_host);
int amrto_net_set_adam(amrto_net* net, const float* m_host, const float* v_host);
/* in_dev (batch, C0, gz, gy, gx) -> out_dev (batch, C_last, gz, gy, gx) (out may be NULL);
 * activations are kept for the next backward */
int amrto_net_forward(amrto_net* net, const float* in_dev, int32_t batch, float* out_dev);
/* gradients of all parameters (overwritten) from dL/dout of the last forward;
 * din_dev (may be NULL) receives dL/din */
int amrto_net_backward(amrto_net* net, const float* dout_dev, float* din_dev);
/* masked mean squared error over n values (mask_dev may be NULL): *loss_host
 * (may be NULL) and dpred_dev = dL/dpred */
int amrto_net_mse(amrto_net* net, const float* pred_dev, const float* target_dev, const uint8_t* mask_dev,
                  int64_t n, float* dpred_dev, double* loss_host);
/* one Adam step (step t >= 1, bias-corrected) on all parameters */
int amrto_net_adam(amrto_net* net, float lr, float beta1, float beta2, float eps, int32_t t);

/* ------------------------------------------------------------------ octree (host) */

typedef struct amrto_octree amrto_octree;

/* Plane or line of the lattice: axis a is pinned to at[a] when has[a] != 0. */
typedef struct {
  int32_t has[3];
  int32_t at[3];
} amrto_region;

/* A tree of base[0] x base[1] x base[2] level-0 leaves, max_level levels. */
int amrto_octree_create(amrto_octree** t, const int32_t base[3], int32_t max_level);
int amrto_octree_destroy(amrto_octree* t);
/* Leaves in Morton order (the order every per-leaf array uses). */
int32_t amrto_octree_n_leaves(const amrto_octree* t);
int amrto_octree_leaves(const amrto_octree* t, int8_t* level, int32_t* anchor /*[3n]*/);
/* Split every leaf with marks[i] != 0 (below max_level) into 8 children. */
int amrto_octree_refine(amrto_octree* t, const uint8_t* marks);
/* Level-one closure (Sec. 6): refine leaves that share a face or an edge
 * with a leaf two or more levels finer, until none remain. */
int amrto_octree_balance(amrto_octree* t);
/* One adaptation of Sec. 4 with rho per current leaf: marking (solid if
 * rho >= rho_s; refine if solid or a solid centre lies within r_amr),
 * sweep 1 (whole families only), refinement plus closure, sweep 2 (no
 * level-two incompatibility from a derefinement), derefinement.  *n_new
 * receives the new leaf count; amrto_octree_adapt_result then fills rho_new
 * (caller buffer of n_new values) with transferred densities: children
 * inherit, parents average.  src_first and src_count are not filled (pass
 * NULL): displacements move through amrto_octree_transfer_nodal. */
int amrto_octree_adapt(amrto_octree* t, const double* rho, double rho_s, double r_amr,
                       int32_t* n_new);
int amrto_octree_adapt_result(const amrto_octree* t, double* rho_new, int32_t* src_first,
                              int32_t* src_count);
/* Build the finite-element mesh of the current leaves: nodes (Morton or
 * lexicographic order), connectivity, hanging-node interpolation with chains
 * resolved (Eq. (6)), supported DOFs from `fixed` regions, and the consistent
 * load on all nodes: kind 0 = line (edge length / 2 per end), kind 1 = face
 * (area / 4 per corner), scaled to `total` on component `comp`.
 * lexicographic != 0 numbers nodes with x fastest (required for a uniform
 * brick upload). */
int amrto_octree_build_mesh(amrto_octree* t, int32_t n_fixed, const amrto_region* fixed,
                            const amrto_region* load_region, int32_t load_kind,
                            int32_t load_comp, double load_total, int32_t lexicographic);
int amrto_octree_mesh_sizes(const amrto_octree* t, int32_t* n_nodes, int32_t* n_elems,
                            int32_t* n_hang, int32_t* n_hang_entries);
int amrto_octree_mesh_export(const amrto_octree* t, int32_t* node_xyz, int32_t* elem_nodes,
                             int8_t* elem_level, int32_t* hang_node, int32_t* hang_ptr,
                             int32_t* hang_master, double* hang_w, uint8_t* dof_fixed,
                             double* f_load);
/* Evaluate a nodal field of the previous mesh (kept by adapt) at the nodes
 * of the current mesh: u_new = trilinear interpolation on the old leaves. */
int amrto_octree_transfer_nodal(const amrto_octree* t, const double* u_old, double* u_new);

/* ------------------------------------------------------------------ multigrid preconditioner */
/* A geometric multigrid V-cycle on the octree hierarchy as the preconditioner
 * of FP64 CG: a stronger preconditioner than Jacobi for the p = 3 contrast
 * (the paper's own choice, Sec. 5, is IC(0) on the rescaled system).
 * Level 0 is the uploaded mesh; a level of depth k <= L merges every leaf
 * finer than level L - k into its ancestor; depths k > L coarsen the uniform
 * base grid by two per axis; the coarse levels have depths first, first + 1,
 * ... and are added until a uniform level has at most coarse_dofs DOFs (it
 * must have at most 1024).  Coarse operators are exactly
 * Galerkin (P^T A P, element by element), the prolongation evaluates the
 * continuous coarse field at the fine nodes, smoothing is Chebyshev on
 * D^-1 A over [hi / ratio, hi] with hi = hi_factor * lambda_max estimated by
 * power_its power iterations, and the coarsest level is solved with its
 * dense inverse.  Vectors are in the constrained form (zero at hanging and
 * supported DOFs). */
typedef struct {
  int32_t degree;       /* Chebyshev degree per smoothing on level 0 (default 2) */
  double ratio;         /* smoothing interval [hi / ratio, hi] (default 10) */
  int32_t power_its;    /* power iterations for lambda_max (default 20) */
  double hi_factor;     /* hi = hi_factor * estimate (default 1.1) */
  int32_t coarse_dofs;  /* target size of the coarsest level (default 200) */
  int32_t first;        /* octree levels merged by the first coarsening, 1 or 2 (default 1) */
  int32_t coarse_degree; /* Chebyshev degree on the coarse levels (0: the same as degree) */
  int32_t blocks0;      /* level 0 smooths with the inverse 3x3 node blocks of A~ (point-block
                           Jacobi inside the Chebyshev iteration) instead of D^-1 (default 0) */
} amrto_mg_opts;

/* Build the hierarchy of the uploaded mesh from the host tree it was built
 * from (its last amrto_octree_build_mesh; uniform meshes: the one-level tree
 * with lexicographic numbering).  Per mesh; allocates the level data.
 * opts may be NULL.  AMRTO_EINVAL when the tree's mesh is not the uploaded
 * one or no small uniform coarsest level exists. */
int amrto_mg_setup(amrto_ctx* ctx, const amrto_octree* tree, const amrto_mg_opts* opts);
/* Level count, DOFs per level, dense (merged) elements per level and 3x3
 * blocks of each coarse level's assembled operator (0 on level 0, which runs
 * the octree operator pass) (host arrays of at least 16 entries, any may be
 * NULL). */
int amrto_mg_info(amrto_ctx* ctx, int32_t* n_levels, int32_t* dofs, int32_t* dense, int64_t* blocks);
/* Replace the power-iteration estimates of lambda_max(D^-1 A) by the given
 * values (one per smoothed level, host), or restore them (lam == NULL). */
int amrto_mg_set_bounds(amrto_ctx* ctx, const double* lam);
/* The lambda_max in use per smoothed level (host output). */
int amrto_mg_get_bounds(amrto_ctx* ctx, double* lam);
/* z = one V-cycle applied to r (device, 3 n_nodes each, distinct). */
int amrto_mg_vcycle(amrto_ctx* ctx, const double* r, double* z);
/* y = A_k x on level k >= 1 (identity rows for constrained DOFs), the
 * diagonal inverse of A_k, x_f = P_k x_c and r_c = P_k^T r_f (device). */
int amrto_mg_level_apply(amrto_ctx* ctx, int32_t k, const double* x, double* y);
int amrto_mg_level_diag(amrto_ctx* ctx, int32_t k, double* dinv);
int amrto_mg_prolong(amrto_ctx* ctx, int32_t k, const double* xc, double* xf);
int amrto_mg_restrict(amrto_ctx* ctx, int32_t k, const double* rf, double* rc);
/* Mean device time (microseconds, HIP events on the context stream) of one
 * smoothing pass per smoothed level, over reps passes on zeroed vectors:
 * us[0] the level-0 operator pass with its Chebyshev update, us[k] level k's
 * block-row pass (host array of n_levels - 1 entries). */
int amrto_mg_pass_times(amrto_ctx* ctx, int32_t reps, double* us);
/* CG in FP64 on A~ u~ = b preconditioned by one V-cycle per iteration, from
 * the initial guess in u (constrained entries ignored), to ||r|| <= rtol
 * ||b||; the numeric set-up runs first after a density change.  check_every
 * (>= 1) is the shortest run of iterations between host convergence checks;
 * runs grow to at most 8x this while the residual's convergence rate says
 * the target is further away (iterations queued past convergence leave u,
 * the iteration count and the residual as they were).  On exit u = T u~
 * with hanging DOFs recovered (Eq. (9)), as from amrto_pcg.
 * Returns AMRTO_OK, AMRTO_NOT_CONVERGED or AMRTO_EBREAKDOWN. */
int amrto_mg_pcg(amrto_ctx* ctx, const double* b, double* u, double rtol, int32_t max_it,
                 int32_t check_every, amrto_solve_stats* stats);

/* ------------------------------------------------------------------ 2-D variant (Sec. 6-7, Test 1) */
/* Q4 plane-stress elements (unit thickness) on a quadtree mesh with hanging
 * nodes, FP64 throughout.  K0 is the unit square's matrix (the stiffness of
 * a square does not depend on its size in 2-D), K_e = (Emin + rho^p (E0 -
 * Emin)) K0; local node a = i + 2 j at (i, j), local DOF 2 a + c.  The
 * constrained operator is A~ = F T^T K T F + (I - F) (Eq. (7)-(8)) with
 * hanging nodes interpolated from their masters (Eq. (6)) and supported DOFs
 * as identity rows.  Vectors hold 2 doubles per node (x, y); element arrays
 * hold one double per element.  All device pointers are on the context's
 * device and stream; calls are asynchronous unless they return a host value.
 * Errors: AMRTO_EINVAL for bad arguments, AMRTO_ESTATE when a required step
 * (mesh, density) is missing, AMRTO_EHIP for runtime failures;
 * amrto_plane_last_error() describes the last one. */
typedef struct amrto_plane amrto_plane;

typedef struct {
  int32_t n_nodes, n_elems;
  int32_t dims[2];            /* finest-lattice box (cells per axis) */
  int32_t max_level;          /* a level-l element has edge 2^(max_level - l) */
  const int32_t* node_xy;     /* [2 n_nodes] lattice coordinates */
  const int32_t* elem_nodes;  /* [4 n_elems], local a = i + 2 j; node 0 is the anchor */
  const int8_t* elem_level;   /* [n_elems], NULL = all at max_level */
  int32_t n_hang;             /* hanging nodes and their master lists (CSR) */
  const int32_t* hang_node;   /* [n_hang] */
  const int32_t* hang_ptr;    /* [n_hang + 1] */
  const int32_t* hang_master; /* [hang_ptr[n_hang]], never hanging themselves */
  const double* hang_w;       /* [hang_ptr[n_hang]] */
  const uint8_t* dof_fixed;   /* [2 n_nodes] supported DOFs */
} amrto_mesh2d;

int amrto_plane_create(amrto_plane** pl, int device, void* stream);
int amrto_plane_destroy(amrto_plane* pl);
const char* amrto_plane_last_error(const amrto_plane* pl);
/* E0 > Emin >= 0, -1 < nu < 0.5, p >= 1 (defaults 1, 1e-9, 0.3, 3). */
int amrto_plane_set_material(amrto_plane* pl, double E0, double Emin, double nu, double p);
/* Copies the (host) mesh; builds the per-node incidence lists (element
 * vertex, weight) through which the operator sums element outputs in a
 * fixed order, and the lattice cell map of the filter. */
int amrto_plane_upload_mesh(amrto_plane* pl, const amrto_mesh2d* mesh);
/* Element Young's moduli and the exact diagonal of A~ from rho (device). */
int amrto_plane_set_density(amrto_plane* pl, const double* rho);
/* y = A~ x (device, distinct). */
int amrto_plane_apply(amrto_plane* pl, const double* x, double* y);
/* b = F T^T f (device, distinct): hanging loads moved onto their masters,
 * supported and hanging rows zero. */
int amrto_plane_project_rhs(amrto_plane* pl, const double* f, double* b);
/* Jacobi-preconditioned CG on A~ u = b in FP64 from the initial guess in u
 * (its supported and hanging entries are ignored), to ||r|| <= rtol ||b||
 * over the unconstrained rows; the host reads the convergence flag every
 * check_every iterations.  On exit the hanging entries of u hold their
 * interpolated values (Eq. (9)).  A pass whose recurrence converges is checked
 * against the true residual and restarted from the current iterate when it
 * is above rtol (at most 8 restarts, counted in stats->outer).  Returns
 * AMRTO_OK, AMRTO_NOT_CONVERGED or
 * AMRTO_EBREAKDOWN; stats may be NULL. */
int amrto_plane_pcg(amrto_plane* pl, const double* b, double* u, double rtol, int32_t max_it,
                    int32_t check_every, amrto_solve_stats* stats);
/* Compliance c = f . u to *c_host (when c_host != NULL) and the Eq. (4)
 * sensitivities dc_e = -p rho^(p-1) (E0 - Emin) u_e^T K0 u_e into dc (device,
 * when dc != NULL; needs rho). */
int amrto_plane_compliance(amrto_plane* pl, const double* u, const double* f, const double* rho,
                           double* c_host, double* dc);
/* The Eq. (5) filter with area weights H_ed = max(0, rmin - |x_e - x_d|)
 * h_d^2 over element centres (lattice units, 0 < rmin <= 16):
 * sensitivity mode out_e = sum H rho_d in_d / (max(rho_e, 1e-3) sum H),
 * density mode out_e = sum H in_d / sum H.  Allocates nothing. */
int amrto_plane_filter(amrto_plane* pl, int32_t mode, double rmin, const double* in, const double* rho,
                       double* out);
/* OC step: rho_new = clamp(rho (max(-dc, 0) / (lam h_e^2))^eta, max(rho_min,
 * rho - move), min(1, rho + move)) with lam such that sum rho_new h_e^2 =
 * volfrac sum h_e^2 (log-spaced candidate multipliers narrowed to a relative
 * width below 1e-14).  change_host = max |rho_new - rho|, lam_host = lam;
 * either may be NULL. */
int amrto_plane_oc_update(amrto_plane* pl, const double* rho, const double* dc, double volfrac, double move,
                          double eta, double rho_min, double* rho_new, double* change_host, double* lam_host);

/* ------------------------------------------------------------------ quadtree (host) */
/* The 2-D tree of base[0] x base[1] level-0 leaves with max_level levels;
 * leaves are kept in Morton order.  Regions use has[0..1] / at[0..1]. */
typedef struct amrto_quadtree amrto_quadtree;

int amrto_quadtree_create(amrto_quadtree** t, const int32_t base[2], int32_t max_level);
int amrto_quadtree_destroy(amrto_quadtree* t);
int32_t amrto_quadtree_n_leaves(const amrto_quadtree* t);
int amrto_quadtree_leaves(const amrto_quadtree* t, int8_t* level, int32_t* anchor /*[2n]*/);
/* Split every leaf with marks[i] != 0 (below max_level) into 4 children. */
int amrto_quadtree_refine(amrto_quadtree* t, const uint8_t* marks);
/* Refine until leaves sharing an edge segment differ by at most one level. */
int amrto_quadtree_balance(amrto_quadtree* t);
/* Sec. 4 adaptation in 2-D: mark (refine solid leaves and leaves whose
 * centre lies within r_amr of a solid centre, derefine the rest), keep only
 * complete families of four, refine with closure, drop families whose
 * parent would break the edge rule, derefine.  Densities: children inherit,
 * parents average (amrto_quadtree_adapt_result). */
int amrto_quadtree_adapt(amrto_quadtree* t, const double* rho, double rho_s, double r_amr, int32_t* n_new);
int amrto_quadtree_adapt_result(const amrto_quadtree* t, double* rho_new);
/* The Q4 mesh of the current leaves: nodes numbered with x fastest, element
 * connectivity (a = i + 2 j), hanging edge midpoints on their edge ends
 * (1/2, 1/2) with chains resolved, both DOFs supported at nodes matching a
 * fixed region, and a point load of load_total on component load_comp at the
 * node (load_x, load_y), which must exist and not hang. */
int amrto_quadtree_build_mesh(amrto_quadtree* t, int32_t n_fixed, const amrto_region* fixed, int32_t load_x,
                              int32_t load_y, int32_t load_comp, double load_total);
int amrto_quadtree_mesh_sizes(const amrto_quadtree* t, int32_t* n_nodes, int32_t* n_elems, int32_t* n_hang,
                              int32_t* n_hang_entries);
int amrto_quadtree_mesh_export(const amrto_quadtree* t, int32_t* node_xy, int32_t* elem_nodes, int8_t* elem_level,
                               int32_t* hang_node, int32_t* hang_ptr, int32_t* hang_master, double* hang_w,
                               uint8_t* dof_fixed, double* f_load);
/* Bilinear interpolation of a nodal field of the mesh before the last adapt
 * at the nodes of the current mesh. */
int amrto_quadtree_transfer_nodal(const amrto_quadtree* t, const double* u_old, double* u_new);

#ifdef __cplusplus
}
#endif
#endif /* AMRTO_H */
