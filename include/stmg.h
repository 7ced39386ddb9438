/*
 * stmg.h - C ABI of libstmg, a space-time multigrid (STMG) solver for 1D transient
 * heat conduction on MI355X (gfx950), after Appel & Alexandersen, "Space-Time
 * Multigrid Methods Suitable for Topology Optimisation of Transient Heat
 * Conduction" (arXiv 2505.10168).
 *
 * Problem (Section 2): c dT/dt - d/dx(k dT/dx) = q on [0,L] x [0,t_T], T = 0 at t = 0
 * and at x = 0, dT/dx = 0 at x = L.  Linear finite elements in space (N_el elements),
 * backward Euler in time (N_t steps), element-wise constant k, c, q (Section 2.2),
 * giving the all-at-once system J u = b with the Dirichlet treatment of Appendix A.
 * Materials follow the SIMP maps of Section 2.1 applied to element densities rho_e.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Space-time vectors are DEVICE pointers to compact, time-major FP64 arrays of
 *   shape [(N_t+1)][(N_el+1)] for the grid they belong to: element (n, i) at
 *   offset n*(N_el+1) + i, time level n = 0..N_t, node i = 0..N_el.
 * - Per-element arrays (densities, gradients) are DEVICE pointers to N_el FP64 values.
 * - The caller owns every pointer it passes and keeps it valid until the call
 *   returns; the library never retains a caller pointer after a call.
 * - All device work runs on the stream given at creation (a hipStream_t passed as
 *   void*, NULL = the default stream).  Calls return after their work is complete
 *   on that stream.
 * - A handle is not thread-safe; use one handle per host thread.  Distinct handles
 *   may be used concurrently from different threads on different streams.
 * - Return values: 0 = OK; > 0 = outcome of an iterative solve (outputs and stats
 *   are written); < 0 = error (outputs untouched, stmg_last_error() describes it).
 */
#ifndef STMG_H
#define STMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------ */
#define STMG_OK               0
#define STMG_NOT_CONVERGED    1   /* cycle cap reached before the tolerance        */
#define STMG_DIVERGED         2   /* residual above the divergence bound, or NaN   */
#define STMG_EINVAL          -1   /* invalid argument                               */
#define STMG_ENOMEM          -2   /* device allocation failed                       */
#define STMG_EHIP            -3   /* HIP runtime error                              */
#define STMG_EUNSUPPORTED    -4   /* valid request the library does not implement   */

/* reassembly methods of the coarse levels (Section 5.1) */
#define STMG_REASSEMBLE_R     0   /* average thermal resistivity 1/k (default)     */
#define STMG_REASSEMBLE_K     1   /* average conductivity                           */
#define STMG_REASSEMBLE_D     2   /* average the design field, then apply SIMP      */
#define STMG_REASSEMBLE_P     3   /* Galerkin: J^(l+1) = R J^(l) P (K-averaged k, c
                                     still steer the coarsening decision); in mixed
                                     precision the FP32 cycles use an FP32 copy of the
                                     FP64 products and the coarsest solve stays FP64;
                                     with bilinear interpolation the coarsest level
                                     must have at most 16384 DOFs                     */

/* precision of the solve */
#define STMG_FP64             0   /* everything in FP64                             */
#define STMG_MIXED            1   /* FP64 outer defect correction around FP32 cycles */

/* interpolation in time (Section 5.1) */
#define STMG_INTERP_C         0   /* causal: coarse level J to fine levels 2J and 2J+1 */
#define STMG_INTERP_B         1   /* bilinear: fine 2J <- 1, fine 2J +- 1 <- 1/2      */

#define STMG_MAX_HISTORY   1024   /* longest residual history kept in the stats     */

/* kind of the per-element field a handle is built from (Section 2: k(x), c(x)) */
#define STMG_FIELD_DENSITY       0   /* design densities rho_e in [0, 1] through SIMP      */
#define STMG_FIELD_CONDUCTIVITY  1   /* conductivities k_e > 0 given directly; c_e = c_con */

/* Physical problem.  With field_kind = STMG_FIELD_DENSITY the materials are
 * k(rho) = k_ins + (k_con - k_ins) rho^p_k and c(rho) = c_ins + (c_con - c_ins) rho^p_c
 * (Section 2.1, eqs. SIMP k / SIMP c); with STMG_FIELD_CONDUCTIVITY the field is k
 * itself, the heat capacity is c_con everywhere (so the diffusivity D_e = k_e / c_con
 * of Section 3.3 is the field over c_con), k_ins and the SIMP exponents are unused, and
 * gradients are dTheta/dk_e.  theta_ref normalises the objective (Section 7.1).
 * q_uniform is the heat source used when no element-wise load is given at creation. */
typedef struct {
    int32_t n_el;          /* elements, >= 1                                        */
    int32_t n_t;           /* backward-Euler steps, >= 1                            */
    double  length;        /* L > 0                                                 */
    double  t_final;       /* t_T > 0                                               */
    double  k_ins, k_con;  /* conductivities of insulator / conductor, > 0          */
    double  c_ins, c_con;  /* heat capacities, > 0                                  */
    double  p_k, p_c;      /* SIMP penalties (paper: 3 and 2)                       */
    double  theta_ref;     /* > 0                                                   */
    double  q_uniform;     /* uniform heat source                                   */
    int32_t field_kind;    /* STMG_FIELD_DENSITY (0) or STMG_FIELD_CONDUCTIVITY (1)  */
} stmg_problem;

/* Solver options.  stmg_default_options() fills: nu = 2, omega = 0.5,
 * lambda_crit = 0.25, max_levels = 0, min_coarse_dofs = 1024, M_min_elems = 0,
 * reassembly = R, deff_mode = 0, tol = 1e-10, diverge = 1e9, max_cycles = 100,
 * precision = FP64, w_diri_override = 0, fused = 1, time_kernels = 0, interp = C,
 * debug_poison = 0, inner_cycles = 4, time_levels = 0. */
typedef struct {
    int32_t nu;               /* smoothing steps before and after the coarse correction (Algorithm 1) */
    double  omega;            /* Jacobi damping (Section 3.1 uses 1/2)                       */
    double  lambda_crit;      /* threshold of Algorithms 2-4                                 */
    int32_t max_levels;       /* N_l; 0 = coarsen while a level has > min_coarse_dofs DOFs    */
    int64_t min_coarse_dofs;  /* used when max_levels == 0                                    */
    int32_t M_min_elems;      /* Algorithm 4 guard: t-coarsen when N_el/2 < M (0 = off)       */
    int32_t reassembly;       /* STMG_REASSEMBLE_*                                           */
    int32_t deff_mode;        /* 0: D_eff from the field (Algorithm 3);
                                 1: sqrt(D_SIMP(0) D_SIMP(1)) (Section 7.2), path independent of rho */
    double  tol;              /* stop when r_n < tol (Section 3.1 termination rule)          */
    double  diverge;          /* stop when r_n > diverge                                      */
    int32_t max_cycles;       /* stop after this many cycles (<= STMG_MAX_HISTORY)           */
    int32_t precision;        /* STMG_FP64 or STMG_MIXED                                      */
    double  w_diri_override;  /* > 0: use this W_Diri on every level; otherwise Appendix A    */
    int32_t fused;            /* 1: fused streaming kernels, and the smallest levels in one
                                    single-workgroup launch with u, b in LDS; 2: fused streaming
                                    kernels on every level; 0: one kernel per method step.
                                    All three give bit-identical iterates.                     */
    int32_t time_kernels;     /* k > 0: time the fine-level fused passes of every k-th V-cycle
                                    with HIP events (1: all of them); 0: no timing            */
    int32_t interp;           /* STMG_INTERP_C or STMG_INTERP_B: prolongation P in time, and
                                    R = P^T / 2.  With B the t transfers run as separate
                                    one-thread-per-DOF kernels beside the fused smoothing
                                    passes, and no single-workgroup tail is used              */
    int32_t debug_poison;     /* 1: the per-level entry points fill the library's internal
                                    output vectors (nodes 0..N_el of every time level) with
                                    NaN before computing them, so an entry a kernel fails to
                                    write shows in the result; a testing aid, 0 by default  */
    int32_t inner_cycles;     /* MIXED: FP32 V-cycles per FP64 defect correction (1..8).  Each
                                    correction u += e solves J e = r approximately by that many
                                    cycles from e = 0; the history and `cycles` count
                                    corrections.                                              */
    int32_t time_levels;      /* k > 0: time every k-th cycle of a solve (the first included)
                                    level by level with HIP events recorded on the stream at
                                    the level boundaries; the means land in
                                    stmg_stats.level_ms.  The events sit between the passes,
                                    so they add a little to the solve time; 0: off          */
} stmg_options;

typedef struct {
    int32_t status;                  /* same value as the call's return               */
    int32_t cycles;                  /* V-cycles (FP64) or outer corrections (mixed)  */
    int32_t n_levels;
    double  rel_residual;            /* final ||J u - b|| / ||b|| (FP64)               */
    double  conv_factor;             /* (r_N / r_0)^(1/N) (Section 3.1)               */
    double  solve_ms;                /* wall time of the solve call                    */
    double  dof_updates;             /* sum over cycles of sum_{l < N_l} 2 nu n_l      */
    double  fine_kernel_ms;          /* time_kernels: summed time of fine fused passes */
    double  fine_kernel_bytes;       /* their algorithmic bytes                         */
    int64_t fine_kernel_launches;
    int64_t fine_passes;             /* fused passes launched on the finest level      */
    double  setup_ms;                /* wall time of the handle's last hierarchy build or
                                        re-assembly (stmg_create / stmg_set_field)     */
    char    path[128];               /* coarsening directions, 'x' / 't' per step       */
    int32_t level_cycles;            /* time_levels: cycles that were timed level by level */
    double  level_ms[64];            /* time_levels: mean device ms per cycle (V-cycle, or
                                        outer correction of MIXED with all its inner
                                        cycles) spent on level l: its smoothing passes,
                                        transfers and norms; on the last level the
                                        coarsest solve; with fused = 1 the
                                        single-workgroup tail counts on its first level
                                        (stmg_info.tail_level).  Finest level of the
                                        cross-cycle form: one pass per cycle, the
                                        post-smoothing of this cycle with the
                                        pre-smoothing of the next.                      */
    double  history[STMG_MAX_HISTORY + 1];   /* r_0 .. r_cycles                       */
} stmg_stats;

/* Hierarchy description (read-only copy). */
typedef struct {
    int32_t n_levels;
    int32_t n_el[64], n_t[64];
    double  h[64], tau[64], w_diri[64];
    double  lambda_eff[64];          /* value that chose the direction leaving level l */
    char    path[64];                /* 'x' / 't' per coarsening step, NUL terminated  */
    size_t  device_bytes;            /* device memory held by the handle               */
    int32_t tail_level;              /* first level of the single-workgroup V-cycle tail
                                        (fused = 1), -1 when every level runs on its own */
} stmg_info;

typedef struct stmg_ctx* stmg_t;

/* Fill *o with the defaults listed above.  Returns STMG_EINVAL if o is NULL. */
int stmg_default_options(stmg_options* o);

/* Device bytes of one request for (p, o), without allocating: what a handle
 * allocates plus the request's compact FP64 outputs, the solution u and, with
 * with_adjoint != 0, the adjoint solution and the N_el gradient.  The handle part is
 * exact for the path that field-independent D_eff (deff_mode = 1) yields and an upper
 * bound (each level as large as any coarsening path can make it) otherwise. */
int stmg_footprint(const stmg_problem* p, const stmg_options* o, int with_adjoint,
                   size_t* bytes);

/* Build the level hierarchy (Algorithms 3/4 with the reassembly method of
 * Section 5.1) and the fine load vector (Section 2.2) on the device.
 *   d_rho : the N_el values of the field of kind p->field_kind (device): densities in
 *           [0, 1], or conductivities > 0.  The call starts by copying it, so it may be
 *           released once the call returns.
 *   d_q   : optional element load, [(N_t+1)][N_el] FP64 (device), row n = q at t_n,
 *           row 0 ignored; NULL = q_uniform everywhere.
 *   stream: hipStream_t used by every call on this handle (NULL = default stream).
 * N_el and N_t need not be powers of two; a direction that cannot halve is
 * replaced by the other one and coarsening stops when neither can.
 * Errors: EINVAL (bad sizes or values, a conductivity field that is not positive,
 * field_kind = CONDUCTIVITY with reassembly D or deff_mode 1, which need densities),
 * ENOMEM, EHIP. */
int stmg_create(stmg_t* handle, const stmg_problem* p, const stmg_options* o,
                const double* d_rho, const double* d_q, void* stream);

/* Re-assemble every level from a new field of the handle's field_kind (Section 7.2:
 * with deff_mode = 1 the path and memory stay fixed across designs).  With
 * deff_mode = 0 the path is recomputed; if it changes, EUNSUPPORTED is returned and
 * the handle is unchanged (create a new handle instead).  EINVAL for a conductivity
 * field that is not positive (the handle then keeps its previous field). */
int stmg_set_field(stmg_t h, const double* d_field);
/* The same call under the name of the design loop (densities). */
int stmg_set_design(stmg_t h, const double* d_rho);

/* Solve J u = b by V-cycles (Algorithm 1) from u0, stopping by the rule of
 * Section 3.1 with the tol / diverge / max_cycles options.
 *   d_rhs : right-hand side on the fine grid, or NULL for the assembled load b.
 *   d_u0  : initial guess, or NULL for u = 0 (the paper's choice).
 *   d_u   : output (may alias d_u0).
 *   st    : optional statistics.
 * Returns OK, NOT_CONVERGED or DIVERGED (d_u holds the last iterate in all three).
 * In FP64 with fused != 0 the residual of cycle k is tested while cycle k+1 already
 * runs; a cycle run past the stopping point is discarded, so iterates, history and
 * cycle count are those of the plain loop (the fine level keeps one more vector for
 * this; stmg_footprint counts it). */
int stmg_solve_forward(stmg_t h, const double* d_rhs, const double* d_u0,
                       double* d_u, stmg_stats* st);

/* Solve the adjoint J^T Lambda = b dt / Theta_ref (Section 7.2) with (J^(l))^T on
 * every level and the same forward-causal transfers.  d_rhs = NULL selects
 * b dt / Theta_ref; otherwise as stmg_solve_forward. */
int stmg_solve_adjoint(stmg_t h, const double* d_rhs, const double* d_l0,
                       double* d_lambda, stmg_stats* st);

/* Theta = b^T u dt / Theta_ref (Section 7.1) with the assembled load b, written to
 * *theta (host). */
int stmg_objective(stmg_t h, const double* d_u, double* theta);

/* dTheta/dfield_e for all elements by the discrete adjoint method (Section 7.2):
 * g_e = -Lambda^T (dJ/dfield_e) u with Dirichlet entries of u and Lambda removed; the
 * field is the densities or the conductivities (field_kind).  d_grad: N_el FP64
 * (device). */
int stmg_gradient(stmg_t h, const double* d_u, const double* d_lambda, double* d_grad);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): the gradient of stmg_gradient
 * without a handle and without any allocation.  The problem p supplies N_el, N_t, L,
 * t_T, the field kind and the SIMP maps; d_rho (the N_el field values), d_u and
 * d_lambda (compact [(N_t+1)][(N_el+1)])
 * are device inputs, d_grad (N_el, device) the output, bit-identical to stmg_gradient
 * of a handle built from the same p and d_rho.  Work runs on `stream` (a hipStream_t
 * of the current device, NULL = default stream); the call returns when it is done.
 * Temporaries live in a fixed device array of 8 Mi doubles (64 MiB) that each device
 * holds from the library's first use until the process ends: N_el * (ceil(N_t/128)
 * capped to 1024, + 2) doubles must fit, else EINVAL.  The array is shared by every
 * call on a device, so calls that overlap on one device (several host threads or
 * streams) race; serialise them.  Nothing needs to start at zero (every temporary is
 * written before it is read).  The first call on a device resolves the array's
 * address (hipGetSymbolAddress); no call allocates, frees or calls an allocating
 * library routine.  Errors: EINVAL (null pointer, bad size, too large), EHIP. */
int stmg_gradient_noalloc(const stmg_problem* p, const double* d_rho, const double* d_u,
                          const double* d_lambda, double* d_grad, void* stream);

/* One design update for the optimisation problem of Section 7.1: minimise Theta
 * subject to 0 <= rho_e <= 1 and the volume bound mean(rho) <= volume (the paper's
 * bound is volume = 1/2).  The paper moves the design with MMA, which it only cites;
 * this is the optimality-criteria step for one volume constraint (Bendsoe 1995):
 *   D_e = max(-grad_e, 0),  lo_e = max(rho_min, rho_e - move),  hi_e = min(1, rho_e + move),
 *   rho_new_e = min(max(rho_e (D_e / lam)^eta, lo_e), hi_e),
 * with the multiplier lam from 96 halvings of [1e-40, 1e40] max_e D_e in log space
 * (midpoint sqrt(a) sqrt(b), stepping up while mean(rho_new) > volume), so that
 * mean(rho_new) = volume to rounding when the bound is active; when it is not, every
 * element with D_e > 0 moves to hi_e.  Elements with D_e = 0 move to lo_e.
 *   d_rho     : N_el FP64 (device), the current design.
 *   d_grad    : N_el FP64 (device), dTheta/drho (e.g. from stmg_gradient).
 *   d_rho_new : N_el FP64 (device) output; may alias d_rho.
 * The handle supplies N_el and the stream; its hierarchy is not touched (load the new
 * design with stmg_set_design).  Returns after the update has finished.
 * Errors: EINVAL unless 0 < volume <= 1, move > 0, 0 < eta <= 1, 0 <= rho_min < 1. */
int stmg_oc_update(stmg_t h, const double* d_rho, const double* d_grad, double volume,
                   double move, double eta, double rho_min, double* d_rho_new);

int stmg_get_info(stmg_t h, stmg_info* info);
int stmg_destroy(stmg_t h);

/* ---- per-level components (each level's own grid, compact layout) -------------
 * Entry points for testing one step of Algorithm 1 at a time.  `level` is 0-based
 * (0 = finest); `transpose` selects J^T.  Level vectors have the shape of that
 * level from stmg_get_info and are FP64 at the interface.  On an FP64 handle the FP64
 * kernels run; on a MIXED handle the FP32 kernels of its inner cycles run on FP32
 * copies of the inputs (the coarsest solve keeps FP64 arithmetic on FP32 vectors, as
 * in those cycles) and the results are widened to FP64 (stmg_vcycle needs FP64). */

/* y = J x  (Appendix A form of the BE-FE operator of Section 2.2). */
int stmg_level_apply(stmg_t h, int level, int transpose, const double* d_x, double* d_y);

/* nu damped-Jacobi steps u <- u + omega D^-1 (b - J u) in place (Section 3.1),
 * through the fused kernels when the handle has fused = 1 or 2. */
int stmg_level_smooth(stmg_t h, int level, int transpose, int nu, const double* d_b, double* d_u);

/* b_c = R (b - J u) after nu pre-smoothing steps, i.e. lines "smooth" and
 * "restrict" of Algorithm 1 on `level` (level < n_levels - 1).  d_u is updated in
 * place; d_bc has the shape of level + 1. */
int stmg_level_presmooth_restrict(stmg_t h, int level, int transpose, int nu,
                                  const double* d_b, double* d_u, double* d_bc);

/* u <- u + P z, then nu post-smoothing steps (the last two steps of Algorithm 1). */
int stmg_level_prolong_postsmooth(stmg_t h, int level, int transpose, int nu,
                                  const double* d_b, const double* d_z, double* d_u);

/* Exact solve of J z = b on the coarsest level (Algorithm 1, first branch). */
int stmg_level_coarsest_solve(stmg_t h, int transpose, const double* d_b, double* d_z);

/* One V-cycle in place on the fine grid; *rel_res (host, optional) receives
 * ||J u - b|| / ||b|| after the cycle.  FP64 handles only (EUNSUPPORTED otherwise). */
int stmg_vcycle(stmg_t h, int transpose, const double* d_b, double* d_u, double* rel_res);

/* Streaming-rate calibration (a measurement aid): y = a (d_b == NULL) or y = a + s b
 * over n FP64 values with the access pattern of the fused passes (16-byte loads and
 * stores, non-temporal stores when nontemporal != 0).  Device pointers, 16-byte
 * aligned, n even.  Unlike every other call this one returns as soon as the kernel is
 * queued on `stream`, so that events around it time the kernel alone.
 * Errors: EINVAL (null or misaligned pointer, odd n), EHIP. */
int stmg_stream_calibrate(const double* d_a, const double* d_b, double s, double* d_y, int64_t n,
                          int nontemporal, void* stream);

/* Launch geometry of one fused streaming pass of `sweeps` Jacobi steps (0..6) on an
 * n_el x n_t level (fp32: the FP32 kernels; fine: the finest level's kernels): each
 * wavefront owns a strip of *strip_cols columns and a segment of *seg_rows time levels
 * (*strips strips along x, *waves wavefronts).  This is the geometry of passes that end
 * with a t restriction, and of every pass on a level whose segments are longer than two
 * time levels; other passes on small levels (2-row segments giving at most 640
 * wavefronts) take 1-row segments.  Host-only; a testing aid, so that sampled checks can
 * be placed across the boundaries between wavefronts. */
int stmg_pass_geometry(int n_el, int n_t, int sweeps, int fp32, int fine, int* strip_cols,
                       int* strips, int* seg_rows, int* waves);

const char* stmg_status_string(int status);
/* Message of the last error on the calling thread (empty if none). */
const char* stmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STMG_H */
