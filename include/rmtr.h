/*
 * librmtr: matrix-free evaluation of the pressure-induced phase-field
 * fracture energy on uniform Q1 grids, the operators of the recursive
 * multilevel trust-region method (RMTR) around it, and the RMTR load step,
 * for AMD Instinct MI355X (gfx950).
 *
 * Reference: P. Zulian et al., "Large scale simulation of pressure induced
 * phase-field fracture propagation using Utopia", arXiv 2007.12908.
 *
 * Problem (Sec. 2, eq. (min_problem_pf)): find (u, c) in V_u^t x V_c
 * minimising E(u, c, p) of eq. (pressurized) on the unit square / cube with
 *   W = g(c) psi+(eps) + psi-(eps) + Gc/2 (c^2/l + l |grad c|^2) + gp(c) div(p u),
 *   g(c) = (1-k)(1-c)^2 + k,  gp(c) = (1-c)^2,  AT2 crack density (Sec. 2.1),
 *   psi+ = K/2 <tr eps>+^2 + mu dev(eps):dev(eps),  psi- = K/2 <tr eps>-^2
 *   (volumetric-deviatoric split; 2D is plane strain), the unsplit
 *   psi+ = lambda/2 (tr eps)^2 + mu eps:eps, psi- = 0 (Sec. 2, first paragraph),
 *   or the spectral split on the principal strains eps_a (Sec. 4.2.1 lists
 *   principal strains among the precomputed quantities):
 *   psi+- = lambda/2 <tr eps>+-^2 + mu sum_a <eps_a>+-^2.
 * Discretisation: first-order Lagrange (Q1) elements (Sec. 2.2), N^d cells,
 * 2^d Gauss points per cell.  Feasible set V_c: c_lower <= c <= 1
 * (eq. (space_pf)); displacements fixed on the Dirichlet set (V_u^t).
 *
 * Conventions shared by every entry point
 *   - Levels are numbered as in Sec. 3: 1 = coarsest ... L = finest.  Level l
 *     has N_l = N_L / 2^(L-l) cells per side and (N_l + 1)^d nodes.
 *   - Node n = i + (N+1) (j + (N+1) k); vectors are node-major interleaved:
 *     v[(d+1) n + comp], comp = (u_x, u_y[, u_z], c).  Scalar nodal fields
 *     (pressure p, c_lower) hold one value per node.
 *   - Every array argument is a DEVICE pointer owned by the caller unless the
 *     comment says "host".  Arrays must not alias unless stated.
 *   - precision: RMTR_FP64 -> the void* arrays are double; RMTR_FP32 -> float
 *     (the mixed-precision form's Hessian and smoother arithmetic).
 *   - dirichlet: per-node uint8 bit mask (bit comp set = that component is
 *     fixed), device pointer, or NULL for the default set: every displacement
 *     component on the boundary.  Gradients have zero rows and Hessians zero
 *     rows and columns at fixed dofs.
 *   - stream: a hipStream_t (passed as void*); work is enqueued on it.  Calls
 *     that return host values synchronise that stream.
 *   - Errors: no exception crosses this interface.  A negative status means
 *     the outputs are undefined; rmtr_last_error() describes the failure.
 *   - Device workspace: by default the library allocates its buffers on
 *     first use of an operation on a level and frees them in rmtr_destroy().
 *     A caller that owns the memory binds one buffer instead
 *     (rmtr_workspace_bytes, rmtr_bind_workspace) and the library then makes
 *     no device allocation.  A context is not thread safe, and its calls must
 *     not overlap in time on different streams: they share its scratch
 *     buffers (reduction partials; in 3D the ring partials that carry the
 *     FP64 gradient's and Hv's tile-border sums from the element kernel to
 *     the kernel that adds them).
 */
#ifndef RMTR_H
#define RMTR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmtr_ctx rmtr_ctx;
typedef int32_t rmtr_status;

#define RMTR_OK 0
#define RMTR_NOT_CONVERGED 1 /* warning: outputs valid, tolerance not met */
#define RMTR_E_ARG (-1)
#define RMTR_E_HIP (-2)
#define RMTR_E_WORKSPACE (-3) /* the bound workspace is too small for the call */
#define RMTR_E_NONFINITE (-4)

#define RMTR_FP64 0
#define RMTR_FP32 1

/* Restriction modes for rmtr_restrict (Sec. 3: R = I^T, projection P). */
#define RMTR_R_DUAL 0   /* R = I^T, for gradients (dual quantities)        */
#define RMTR_R_INJECT 1 /* P: fine node (2i,2j,2k) -> coarse node (i,j,k)  */
#define RMTR_R_BOX_LO 2 /* max over the support of each coarse basis fn    */
#define RMTR_R_BOX_HI 3 /* min over the support of each coarse basis fn    */

/* Model (Sec. 2): material and grid.  ls = l_s (the paper uses 2h, Sec. 5). */
typedef struct {
  int32_t dim;      /* 2 or 3 */
  int32_t n_cells;  /* N_L, cells per side on the finest level */
  int32_t n_levels; /* L >= 1; N_L must be divisible by 2^(L-1) */
  int32_t split;    /* 0: unsplit density, 1: volumetric-deviatoric split,
                       2: spectral split (principal strains); other values
                       make rmtr_create return RMTR_E_ARG */
  double lambda, mu, Gc, ls, k;
} rmtr_model;

/* Solver constants (Alg. 1-3, Sec. 3.2.1, Sec. 4.2.1). */
/* A trained proposal network (see the learned-proposal section below);
   every pointer is device memory owned by the caller. */
typedef struct {
  const uint16_t* w;    /* RMTR_NN_WEIGHTS BF16 weights, layer by layer      */
  const float* bias;    /* RMTR_NN_BIASES FP32 biases, layer by layer        */
  const float* scales;  /* 12 FP32: input scales (x: 4, g: 4), output (4)   */
} rmtr_nn;

typedef struct {
  double eta1, eta2;       /* 0 < eta1 <= eta2 <= 1 (Alg. 3)            */
  double gamma1, gamma2;   /* 0 < gamma1 <= 1 <= gamma2 (Alg. 3)        */
  double delta0, delta_max; /* initial and largest TR radius             */
  double rtol;             /* stop when chi <= rtol chi(x_initial)      */
  double coarse_qp_rtol;   /* MPRGP relative tolerance                  */
  double guard;            /* TR ratio round-off level: |pred| <= tol = guard |f(x_in)| /
                              sqrt(elements of the level) counts as rho = 1 unless
                              ared < -tol (eq. (rho_tr), (rho_ml) in finite precision) */
  int32_t mu1, mu2;        /* pre-/post-smoothing TR steps (Alg. 1)     */
  int32_t pgs_sweeps;      /* symmetric PGS sweeps per TR subproblem    */
  int32_t coarse_tr_its;   /* TR steps on the coarsest level (mu^1)     */
  int32_t coarse_qp_its;   /* MPRGP iteration cap                       */
  int32_t fallback_sweeps; /* PGS sweeps after MPRGP meets p^T A p <= 0 */
  int32_t max_vcycles;
  int32_t precision;       /* RMTR_FP64 or RMTR_FP32 (fine Hv + PGS)    */
  int32_t coarse_model;    /* f~^l of the coarse models (eq. (second_order_consistency)):
                              0: the same functional on the level-l grid,
                              1: f~ = 0 (the pure Galerkin quadratic),
                              2: f~^l(x) = f(I_{l->L} x), the finest functional
                              of the prolongated iterate */
  int32_t use_learned;     /* 1: learned proposal before the first finest-level
                              pre-smoothing step of each V-cycle (3D; needs nn) */
  const rmtr_nn* nn;       /* host pointer, read during the call         */
  int32_t nn_patience;     /* stop proposing after this many consecutive
                              rejections in a load step (0: never stop)  */
  int32_t shrink_to_step;  /* 0: Alg. 3 as printed, delta <- gamma1 delta on
                              rejection; 1: delta <- gamma1 min(delta,
                              |s|_inf) (the radius follows the rejected step) */
  int32_t gs_mode;         /* Gauss-Seidel order of the smoother (Sec. 3.2.1,
                              Sec. 4.2.2): 0 = global 2^d node colours (the
                              sequential order within a colour); 1 = the
                              hybrid Jacobi/Gauss-Seidel over tiles, not built
                              (RMTR_E_ARG) */
  int32_t first_order;     /* 1: first-order coarse models (ablation): no dH
                              term, each coarse level smooths with its own
                              lagged Hessian grad^2 f~^l(x0) instead of the
                              Galerkin product; needs coarse_model 0 */
} rmtr_params;

typedef struct {
  int32_t vcycles, tr_accepted, tr_rejected, status;
  double chi0, chi, energy, seconds;
  int32_t nn_proposed, nn_accepted; /* learned proposals made / accepted */
  double delta;                     /* finest-level TR radius at the end */
} rmtr_stats;

/* Fills p with the defaults used throughout: eta = (0.1, 0.75),
   gamma = (0.5, 2), delta0 = 1, delta_max = 10, rtol = 1e-8, mu1 = mu2 = 1,
   3 PGS sweeps, 5 coarse TR steps, MPRGP 500 its / 1e-10, 50 fallback sweeps,
   200 V-cycles, FP64, f~ = f, no learned proposal (patience 3), Alg. 3's
   radius update as printed. */
void rmtr_default_params(rmtr_params* p);

/* Create a context for the hierarchy of `model`.  Returns RMTR_E_ARG on an
   invalid model (dim, N not divisible by 2^(L-1), non-positive material). */
rmtr_status rmtr_create(const rmtr_model* model, rmtr_ctx** out);
void rmtr_destroy(rmtr_ctx* ctx);
const char* rmtr_last_error(const rmtr_ctx* ctx);
/* Nodes of level `level` ((N_l+1)^d), or -1 for an invalid level. */
int64_t rmtr_level_nodes(const rmtr_ctx* ctx, int32_t level);

/* Caller-owned device workspace (host-only computation, no GPU call).
   rmtr_workspace_bytes(ctx, params): bytes of device memory that
   rmtr_solve_loadstep with these parameters needs on a fresh context
   (precision and use_learned matter), which also covers every later
   rmtr_energy, rmtr_energy_diff, rmtr_gradient, rmtr_hessvec,
   rmtr_diag_blocks, rmtr_restrict, rmtr_prolong, rmtr_dot and rmtr_chi
   call; params == NULL: the bytes those calls alone need.  The other entry
   points (rmtr_smooth, rmtr_coarse_hessvec, rmtr_mprgp, rmtr_step_box,
   rmtr_init_fields, the rmtr_nn_* calls) carve their scratch from what is
   left and return RMTR_E_WORKSPACE when it does not fit.
   rmtr_bind_workspace: from now on every device buffer of the context is
   carved, in call order, from [dev, dev + bytes) (256-byte aligned, device
   memory owned by the caller, kept alive until rmtr_destroy); the library
   makes no device allocation.  Bind once, before the context's first device
   call (RMTR_E_ARG otherwise).  A few hundred bytes of pinned host memory for
   returned scalars are still allocated on first use.
   rmtr_workspace_used: bytes carved so far. */
size_t rmtr_workspace_bytes(const rmtr_ctx* ctx, const rmtr_params* params);
rmtr_status rmtr_bind_workspace(rmtr_ctx* ctx, void* dev, size_t bytes);
size_t rmtr_workspace_used(const rmtr_ctx* ctx);

/* Nodal inclusion initialisation (Sec. 5, first paragraph; Sec. 5.2):
   c0[n] = 1 if node n lies inside a fracture's volumetric description
   (3D: within distance `band` of a disc; 2D: inside a rectangle), else 0.
   table (host, row-major): 3D rows (cx cy cz nx ny nz radius pressure),
   2D rows (cx cy tx ty half_length half_width pressure).
   p_mode 0: p[n] = p_value everywhere; 1 (3D): p[n] = max pressure of the
   discs within distance p_band of the node, else 0.  p may be NULL. */
rmtr_status rmtr_init_fields(rmtr_ctx* ctx, int32_t level, const double* table, int32_t n_frac, double band,
                             int32_t p_mode, double p_value, double p_band, double* c0, double* p, void* stream);

/* Energy f(x) = sum_e sum_q w_q W (eq. (pressurized), discretised), FP64.
   x: (d+1) per node; p: nodal pressure; out: ONE double in device memory. */
rmtr_status rmtr_energy(rmtr_ctx* ctx, int32_t level, const double* x, const double* p, double* out,
                        void* stream);

/* rmtr_energy for callers that cannot allocate memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the same
   kernels and result, with the reduction's partial sums in a fixed device
   array of 4096 doubles held by the library on each GPU it runs on, instead
   of context memory.  Allocates nothing (host or device).  Calls that overlap
   on one GPU share that array and race; a level that would need more
   partial sums than it holds is refused with RMTR_E_ARG. */
rmtr_status rmtr_energy_noalloc(rmtr_ctx* ctx, int32_t level, const double* x, const double* p, double* out,
                                void* stream);

/* f(x + s) - f(x), accumulated element by element (numerator of eq. (rho_tr)
   and (rho_ml)); s is double (s_precision RMTR_FP64) or float (RMTR_FP32). */
rmtr_status rmtr_energy_diff(rmtr_ctx* ctx, int32_t level, const double* x, const void* s, int32_t s_precision,
                             const double* p, double* out, void* stream);

/* Gradient of f at x (first variation of W), Dirichlet rows zero. */
rmtr_status rmtr_gradient(rmtr_ctx* ctx, int32_t level, const double* x, const double* p,
                          const uint8_t* dirichlet, double* g, void* stream);

/* Hv = grad^2 f(x_lin) v on the free dofs (second variation of W; Sec. 4.2.1:
   the Hessian is taken at a lagged linearisation point).  FP32: x_lin, p,
   v and Hv are float. */
rmtr_status rmtr_hessvec(rmtr_ctx* ctx, int32_t level, const void* x_lin, const void* p,
                         const uint8_t* dirichlet, const void* v, void* Hv, int32_t precision, void* stream);

/* Node diagonal blocks of grad^2 f(x_lin): (d+1)^2 values per node,
   row-major, Dirichlet rows and columns zero (Sec. 4.2.2, the diagonal-block
   copy used by the Gauss-Seidel smoother). */
rmtr_status rmtr_diag_blocks(rmtr_ctx* ctx, int32_t level, const void* x_lin, const void* p,
                             const uint8_t* dirichlet, void* D, int32_t precision, void* stream);

/* Symmetric projected Gauss-Seidel (Sec. 3.2.1) on the TR subproblem
   eq. (model_qp) with the Hessian at x_lin:
     min g^T s + 1/2 s^T H s,  lo <= s <= hi;
   n_sweeps sweeps (forward then backward over the 2^d node colours; the
   components of a node in order, then reversed), starting from s_inout.
   The Hessian at x_lin (FP64 x_lin and p) is first assembled into a block
   stencil held by the library (Sec. 4.2.2: the diagonal blocks are kept
   apart); g, lo, hi and s_inout, the stencil and the sweeps are in
   `precision`. */
rmtr_status rmtr_smooth(rmtr_ctx* ctx, int32_t level, const double* x_lin, const double* p,
                        const uint8_t* dirichlet, const void* g, const void* lo, const void* hi,
                        void* s_inout, int32_t n_sweeps, int32_t precision, void* stream);

/* Level transfers (Sec. 3): fine (level fine_level) -> coarse (fine_level-1). */
rmtr_status rmtr_restrict(rmtr_ctx* ctx, int32_t fine_level, int32_t mode, const void* fine, void* coarse,
                          int32_t precision, void* stream);
/* Prolongation I: coarse (coarse_level) -> fine (coarse_level + 1). */
rmtr_status rmtr_prolong(rmtr_ctx* ctx, int32_t coarse_level, const void* coarse, void* fine, int32_t precision,
                         void* stream);

/* Hv with the Galerkin coarse Hessian of `level` < L as the load step
   builds it (eq. (delta_terms), Alg. 1, lagged at x_lin): the finest-level
   Hessian at x_lin (FP64 x_lin and p; stored FP64, or FP32 if precision is
   RMTR_FP32) assembled into a block stencil (finest Dirichlet mask
   `dirichlet`) and coarsened level by level, H_l = D_l R H_{l+1} I D_l with
   D_l the default Dirichlet set of level l, in FP64.  v, Hv: FP64 on
   `level`. */
rmtr_status rmtr_coarse_hessvec(rmtr_ctx* ctx, int32_t level, const double* x_lin, const double* p,
                                const uint8_t* dirichlet, const double* v, double* Hv, int32_t precision,
                                void* stream);

/* MPRGP (Sec. 3.2.1, coarsest level) for min g^T s + 1/2 s^T K s,
   lo <= s <= hi, from s = 0.  iterations/status (host, may be NULL):
   status 0 converged, 1 iteration cap, 2 non-positive curvature (then
   fallback_sweeps PGS sweeps were applied).  Synchronises the stream. */
rmtr_status rmtr_mprgp(rmtr_ctx* ctx, int32_t level, const double* K, const double* g, const double* lo,
                       const double* hi, double* s, int32_t max_it, double rtol, int32_t fallback_sweeps,
                       int32_t* iterations, int32_t* status, void* stream);

/* Reductions on FP64 vectors (device scalar result). */
rmtr_status rmtr_dot(rmtr_ctx* ctx, int64_t n, const double* a, const double* b, double* out, void* stream);
/* chi = || P_F(x - g) - x ||_2 over the free dofs, F: c_lower <= c <= 1. */
rmtr_status rmtr_chi(rmtr_ctx* ctx, int32_t level, const double* x, const double* g, const double* c_lower,
                     const uint8_t* dirichlet, double* out, void* stream);

/* One load step (Sec. 4.1 workflow step 7b): RMTR V-cycles (Alg. 1-3 with
   Hessian lagging, Sec. 4.2.1) from x_inout until chi <= rtol chi(x_in) or
   max_vcycles.  With params->use_learned, each V-cycle first tries the
   learned proposal on the finest level: it is projected onto the step box,
   scaled by the model minimiser beta in (0, 1] along it (it must be a
   descent direction of the model, with beta >= 1/2), judged by the FP64
   ratio of eq. (rho_tr) against the lagged model (rho > eta1), required to
   predict at least the decrease of a Cauchy step (d = P(-t g),
   t = g^T g / g^T H g, projected onto the box, scaled by the exact model
   minimiser alpha in [0, 1]), and taken in place of the first PGS
   pre-smoothing step only if it lowers the energy at least as much as
   that PGS step from the same state would (or the PGS step would fail its
   ratio test); otherwise the PGS step runs.  A rejected proposal leaves x
   and delta unchanged.  p: fine nodal pressure; c_lower: c^{t-1} per fine node;
   x_inout must be feasible; its Dirichlet values (the data g^t of V_u^t,
   e.g. a prescribed displacement for displacement-driven loading) are kept.
   f_ext (device, may be NULL): external load on the finest level (the
   Neumann terms, rmtr_neumann_load); the functional minimised is then
   f(x) - f_ext . x, and stats->energy reports it.  chi_history (host, may be
   NULL) receives chi after each V-cycle (max_vcycles entries).  Returns
   RMTR_OK, RMTR_NOT_CONVERGED (x still feasible) or an error.  Synchronises. */
rmtr_status rmtr_solve_loadstep(rmtr_ctx* ctx, const double* p, const double* c_lower, const uint8_t* dirichlet,
                                const double* f_ext, const rmtr_params* params, double* x_inout,
                                rmtr_stats* stats, double* chi_history, void* stream);

/* External load of the Neumann terms of eq. (pressurized) (Sec. 2.1, the
   boundary part Gamma_N where the displacement is free):
     b[(d+1) n + i] = int_{Gamma_N} (tbar_i + p n_i) N_n ds,  b[(d+1) n + d] = 0,
   over the faces in face_mask (bit f = face f = 2 axis + side: x = 0, x = 1,
   y = 0, y = 1[, z = 0, z = 1]), n the outward normal.  traction (host,
   2d x d doubles, row f = the constant traction tbar of face f).  With the
   pressure work of the density written as + gp(c) div(p u), the boundary
   term of the divergence theorem enters the energy as - int p n . u, so
   the functional with these terms is f(x) - b . x (pass b as f_ext).  Face
   cells by the (d-1)-dimensional 2-point Gauss rule (exact). */
rmtr_status rmtr_neumann_load(rmtr_ctx* ctx, int32_t level, int32_t face_mask, const double* traction,
                              const double* p, double* b, void* stream);

/* Trust-region step box of Alg. 3 on the finest level (Sec. 3, the
   constraints of eq. (model_qp)): lo = max(-delta, L - x), hi = min(delta,
   U - x) with L = (-inf, c_lower) and U = (+inf, 1) per node (u, c); zero at
   Dirichlet dofs.  level must be the finest level. */
rmtr_status rmtr_step_box(rmtr_ctx* ctx, int32_t level, const double* x, const double* c_lower, double delta,
                          const uint8_t* dirichlet, double* lo, double* hi, void* stream);

/* ------------------------------------------------------------------------
   Learned proposal (not part of the paper's method: a learned form of the
   finest-level smoother, gated by the unchanged trust-region ratio test of
   eq. (rho_tr), a Cauchy sufficient-decrease check, a comparison with the
   smoother step's energy decrease and the bound projection, with the PGS
   smoother of Sec. 3.2.1 as fallback).

   Network: six 3x3x3 convolutions with zero padding on the node grid,
   channels 8 -> 32 -> 32 -> 32 -> 32 -> 32 -> 4, ReLU after the first five:
     y[v][co] = b[co] + sum_k sum_ci W[k][ci][co] x[v + off(k)][ci],
   off(k) = (k%3 - 1, (k/3)%3 - 1, k/9 - 1) in (x, y, z).  Tensors are
   channels-last FP32 on nx*ny*nz voxels, voxel v = i + nx (j + ny k).
   Weights are BF16 (round-to-nearest-even of FP32 masters), [27][Cin][Cout]
   per layer, layers concatenated.  Every convolution runs on the BF16
   matrix cores: layer inputs, output gradients and weights rounded to BF16
   (round-to-nearest-even), products summed in FP32.
   Input channels: (u, c) of x times scales[0..3], then g_k / rms(g_k) times
   scales[4..7], rms(g_k) the root mean square of component k of g over the
   level's nodes (the input is 0 where it vanishes); output channel k times
   scales[8+k] rms(g_k) is the proposed step of component k (3D only).  The
   network is thus first-order homogeneous in g: its step scales with the
   gradient as a Newton-type correction does. */
#define RMTR_NN_WEIGHTS 120960
#define RMTR_NN_BIASES 164

/* Sizes in floats: what 0 = weights, 1 = biases, 2 = activation buffer of
   rmtr_nn_forward (all 7 layer tensors: 172 floats per voxel), 3 = work
   buffer of rmtr_nn_backward.  -1 on a bad argument. */
int64_t rmtr_nn_size(int32_t what, int32_t nx, int32_t ny, int32_t nz);

/* Forward pass.  act: rmtr_nn_size(2) floats; its first 8 nx ny nz floats
   are the input (caller-filled); the layer outputs follow in order, the
   4-channel result last (offset 168 nx ny nz). */
rmtr_status rmtr_nn_forward(rmtr_ctx* ctx, const uint16_t* w, const float* bias, float* act, int32_t nx,
                            int32_t ny, int32_t nz, void* stream);

/* Backward pass of L(result) given dL/d(result) = dout (4 floats per voxel)
   on the activations of a forward pass: grad (RMTR_NN_WEIGHTS +
   RMTR_NN_BIASES floats) receives dL/dW then dL/db, summed over voxels in a
   fixed order (deterministic).  work: rmtr_nn_size(3) floats. */
rmtr_status rmtr_nn_backward(rmtr_ctx* ctx, const uint16_t* w, const float* act, const float* dout, float* grad,
                             float* work, int32_t nx, int32_t ny, int32_t nz, void* stream);

/* Mean squared error over the window [window[0], window[1]) x [window[2],
   window[3]) x [window[4], window[5]) (host int32, voxel indices in x, y, z)
   and the 4 channels: loss (one device double) and dout = dL/d(out). */
rmtr_status rmtr_nn_mse(rmtr_ctx* ctx, const float* out, const float* target, const int32_t* window, float* dout,
                        double* loss, int32_t nx, int32_t ny, int32_t nz, void* stream);

/* One Adam step (Kingma and Ba, beta = (0.9, 0.999), eps = 1e-8, bias
   correction with step number t >= 1) on n FP32 masters; the first n_bf16
   of them are also written to w_bf16 (may be NULL). */
rmtr_status rmtr_nn_adam_step(rmtr_ctx* ctx, int64_t n, int64_t n_bf16, float lr, int32_t t, const float* grad,
                              float* master, float* m, float* v, uint16_t* w_bf16, void* stream);

/* w_bf16[i] = round-to-nearest-even BF16 of master[i], i < n. */
rmtr_status rmtr_nn_to_bf16(rmtr_ctx* ctx, int64_t n, const float* master, uint16_t* w_bf16, void* stream);

/* Network input from a state of `level`: in8[8 n + k] = x[4 n + k] *
   scales[k] (k < 4), g[4 n + k - 4] / rms(g_{k-4}) * scales[k] (k >= 4). */
rmtr_status rmtr_nn_features(rmtr_ctx* ctx, int32_t level, const double* x, const double* g, const float* scales,
                             float* in8, void* stream);

/* rms[k] = root mean square of component k of the nodal 4-vector v over
   the level's nodes (4 device doubles; 3D levels). */
rmtr_status rmtr_nn_channel_rms(rmtr_ctx* ctx, int32_t level, const double* v, double* rms, void* stream);

/* Training target of a harvested step s at gradient g (the inverse of the
   proposal's output scaling): t[4 n + k] = s[4 n + k] / (scales[8+k]
   rms(g_k)), 0 where the denominator vanishes; t FP32. */
rmtr_status rmtr_nn_target(rmtr_ctx* ctx, int32_t level, const double* g, const double* s, const float* scales,
                           float* t, void* stream);

/* Normalisation constants of the network from n_samples harvested (x, g, s)
   triples of `level` (x, g, s: host arrays of n_samples device pointers):
   scales[k] = 1 / mean rms(x_k), scales[4+k] = 1 (g enters divided by its
   own RMS), scales[8+k] = mean over samples of rms(s_k) / rms(g_k) (0 for a
   sample with rms(g_k) = 0); a constant that comes out 0 is set to 1. */
rmtr_status rmtr_nn_fit_scales(rmtr_ctx* ctx, int32_t level, int32_t n_samples, const double* const* x,
                               const double* const* g, const double* const* s, float* scales, void* stream);

/* Proposed step of `level` (3D): features of (x, g), forward pass, output
   channel k times scales[8+k] rms(g_k), projected onto [lo, hi] (non-finite
   values become 0 before the projection); s: FP64, (d+1) per node. */
rmtr_status rmtr_nn_propose(rmtr_ctx* ctx, int32_t level, const rmtr_nn* net, const double* x, const double* g,
                            const double* lo, const double* hi, double* s, void* stream);

/* Floating-point additions, subtractions, multiplications and divisions that
   the library's element operators perform on data for ONE element (the
   executed arithmetic, a multiply-add counting two; host-only, no GPU call).
   kind: 0 energy, 1 energy difference, 2 gradient, 3 Hessian-vector product
   (3D: kinds 0, 2 and 3 as the quarter-wise FP64 kernels evaluate them, the
   volumetric-deviatoric form; kind 1 all eight Gauss points at once), 4 one
   element's contribution to one node's rows in a Gauss-Seidel colour pass.
   In 2D, kinds 2 and 3 are per element and node (node-centric kernels).
   Returns -1 for a bad argument. */
int64_t rmtr_element_flops(int32_t dim, int32_t kind);

#ifdef __cplusplus
}
#endif
#endif /* RMTR_H */
