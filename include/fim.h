/*
 * fim.h -- C ABI of the localized fully implicit Newton library for
 * fractured reservoirs on MI355X (gfx950).
 *
 * The library advances a discrete reservoir model by fully implicit
 * timesteps.  Jiang (2020), Section 4.1, states the problem: given the
 * state u^n and a timestep dt, find u^{n+1} with F(u^{n+1}) = 0 by Newton
 * iterates J(u^nu) du^nu = -F(u^nu); Section 4.3 (Algorithm 1, localized
 * Newton) and Section 4.4 (Algorithm 2, adaptive nonlinear domain
 * decomposition) restrict each iteration to an a-priori active set; the
 * residual-based localization that Sections 1 and 4.2 describe as the
 * prior method is a fourth mode.  F is the finite-volume two-point-flux
 * residual with phase-potential upwinding of Appendix A.
 *
 * Conventions
 *  - SI units everywhere (Pa, m, m^2, m^3, s, kg, Pa s).
 *  - Cells are numbered 0..n-1.  A state is b planes of n doubles:
 *    plane 0 pressure, plane 1 water saturation (b >= 2), plane 2 the
 *    black-oil variable X (b = 3): gas saturation where status = 1
 *    (saturated), dissolved-gas ratio R_s where status = 0.
 *  - Every call is stream-ordered on the stream given at creation
 *    (NULL: the library creates its own).  Calls that return host data
 *    synchronise that stream.
 *  - Return codes: FIM_OK = 0; negative = hard error (the message is in
 *    fim_last_error; the model keeps its last valid state only where the
 *    call says so); positive = soft failure, state rolled back.
 *  - One host thread per handle.  Different handles may be driven from
 *    different threads on different streams.
 */
#ifndef FIM_H
#define FIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fim_status {
    FIM_OK = 0,
    FIM_NOT_CONVERGED = 1,   /* Newton failed; state rolled back to u^n   */
    FIM_E_ARG = -1,          /* invalid argument or model description     */
    FIM_E_NOMEM = -2,        /* device allocation failed                  */
    FIM_E_HIP = -3,          /* HIP runtime error                         */
    FIM_E_STATE = -4,        /* call not valid in the current step state  */
    FIM_E_NONFINITE = -5     /* non-finite input                          */
} fim_status;

/* Solver modes.  FIM_DD_ADD is Algorithm 2 with the additive form of its
 * phase 2 (Section 4.4 names the additive Schwarz form; the combination rule
 * for the adaptive, overlapping subdomains is this library's): phase 1 is
 * as in FIM_DD; each later fim_newton_step is one sweep that solves every
 * subdomain whose latest update on V_A^k or its outer layer is at least
 * eps_loc, all from the same state and in one batched linear solve, and
 * each cell takes the update of the first subdomain (in build order) that
 * contains it.  Its iteration statistics report the sweep: n_active = the
 * sum of the solved subdomains' sizes, subdomain = how many were solved.
 * The first sweep of a model allocates one subdomain workspace (about the
 * model's local-system memory) per subdomain solved at once, kept until the
 * model is destroyed.  FIM_RESID is the residual-based localization that
 * Sections 1 and 4.2 describe as the prior method (Lu and Beckner): the
 * first iteration of a timestep takes every cell, each later one the cells
 * whose residual error measure e_i = dt max_c |R_{i,c}| / (V_i rho_c)
 * (V_i the reference pore volume, rho_c the reference density of component
 * c: rho_ref; rho_w, rho_o; rho_wsc, rho_osc, rho_gsc) is at least eps_res,
 * inflated by res_layers neighbour layers.  Its step ends when the update
 * meets the convergence test or no cell is at or above eps_res. */
enum { FIM_FULL = 0, FIM_LOCAL = 1, FIM_DD = 2, FIM_RESID = 3, FIM_DD_ADD = 4 };
enum { FIM_FP64 = 0, FIM_MIXED = 1 };                     /* Krylov precision */
enum { FIM_HOST = 0, FIM_DEVICE = 1 };                    /* pointer kind */
enum { FIM_FLUID_SINGLE = 1, FIM_FLUID_DEADOIL = 2, FIM_FLUID_BLACKOIL = 3 };

/* Fluid description (Section 2 and Appendix A leave the fluid open; these
 * are the three closed families the library implements).  Unused fields
 * are ignored.
 *  single  : rho = rho_ref exp(c (p - p_ref)), viscosity mu, b = 1.
 *  deadoil : rho_w = rho_w exp(c_w (p - p_ref)), rho_o likewise with c_o;
 *            Corey exponent 2, S_wn = clamp((S_w - swc)/(1 - swc - sor)),
 *            k_rw = S_wn^2, k_ro = (1 - S_wn)^2; b = 2 (water, oil).
 *  blackoil: R_s,sat = rs_b p / p_b, B_o = (1 + bo_slope R_s)
 *            exp(-c_o (p - p_b R_s / rs_b)), B_g = bg_c / p,
 *            B_w = exp(-c_w (p - p_ref)); surface densities rho_*sc;
 *            k_rw = ((S_w - swc)/span)^2, k_rg = (S_g/span)^2,
 *            k_ro = (S_o/span)^2 (clamped); b = 3 (water, oil, gas). */
typedef struct fim_fluid {
    int32_t kind;
    double p_ref;
    double rho_ref, c, mu;                                       /* single */
    double rho_w, c_w, mu_w, rho_o, c_o, mu_o, swc, sor;         /* dead oil */
    double rs_b, p_b, bo_slope, bg_c, rho_osc, rho_gsc, rho_wsc, /* black oil */
           mu_g, span;
} fim_fluid;

/* The discrete problem (host pointers; the library copies everything and
 * the caller keeps ownership).  Connections need conn_i < conn_j, no
 * duplicates, T >= 0; pore volumes > 0; at most one perforation per cell.
 * Pore volume is pv_ref (1 + c_r (p - p_ref_rock)).  always_active may be
 * NULL (no cell always active); the paper keeps fracture cells active.
 * frac_id may be NULL; else the fracture (>= 0) each cell belongs to, -1
 * for matrix cells: the linear solver's fracture-block preconditioner
 * groups cells of one fracture that are consecutive in the cell order. */
typedef struct fim_model_desc {
    int32_t n_cells, n_conn, n_perf;
    const double*  pv_ref;        /* [n] m^3                               */
    const double*  depth;         /* [n] m, positive downward              */
    const uint8_t* always_active; /* [n] or NULL                           */
    const int32_t* conn_i;        /* [n_conn]                              */
    const int32_t* conn_j;        /* [n_conn]                              */
    const double*  conn_T;        /* [n_conn] m^3                          */
    const int32_t* perf_cell;     /* [n_perf]                              */
    const double*  perf_wi;       /* [n_perf] m^3                          */
    const double*  perf_bhp;      /* [n_perf] Pa                           */
    double c_r, p_ref_rock, gravity;
    fim_fluid fluid;
    const int32_t* frac_id;       /* [n] or NULL                           */
} fim_model_desc;

/* Preconditioners of the local linear solve (the paper names none).  A
 * fracture block is a run of consecutive rows of one fracture inside a
 * 256-row tile, cut at the fracture's units (fim_inspect_pc_blocks); on
 * top of the b x b block-Jacobi scaling A~ = D^{-1} J, M^{-1} is applied
 * on the left. */
enum {
    FIM_PC_JACOBI = 0,            /* block Jacobi over the b x b cell blocks   */
    FIM_PC_FRACTURE = 1,          /* plus, per fracture block and unknown c,
                                     the exact inverse of A~ restricted to
                                     unknown c of the block's cells (the
                                     unknowns decoupled inside the block;
                                     b = 1: the block's exact inverse)        */
    FIM_PC_FRACTURE_COUPLED = 2   /* plus the exact inverse of A~ restricted
                                     to all unknowns of the block's cells     */
};

/* Solver options.  fim_default_options fills the paper's settings
 * (Section 5: eps_p = 0.3 psi cutoff and convergence, m = 2 for
 * Algorithm 1, m = 4 for Algorithm 2) and a linear tolerance of 1e-4
 * (inexact Newton; the paper does not state one). */
typedef struct fim_options {
    double  eps_conv;        /* Newton convergence: ||dp||_inf < eps_conv (Pa) */
    double  eps_loc;         /* active/boundary cutoff |dp_i| >= eps_loc (Pa)  */
    double  eps_s;           /* tight mode: ||dS||_inf < eps_s                 */
    int32_t tight;           /* 1: also require ||dS|| < eps_s and no switch   */
    int32_t m_layers;        /* neighbour layers, Algorithm 1                  */
    int32_t m_layers_dd;     /* neighbour layers, Algorithm 2                  */
    int32_t max_newton;      /* Newton iteration cap per timestep              */
    int32_t max_sweeps;      /* Algorithm 2 outer sweep cap                    */
    int32_t auto_cut;        /* solve_timestep halves dt on failure            */
    int32_t max_cuts;
    double  ds_max;          /* saturation chop per iteration                  */
    int32_t precision;       /* FIM_FP64 or FIM_MIXED (FP32 Krylov + FP64 IR)  */
    double  lin_rtol;        /* ||J x + F|| <= lin_rtol ||F||                  */
    double  inner_rtol;      /* FP32 inner reduction per refinement pass       */
    int32_t krylov_maxit;    /* BiCGStab iterations per refinement pass        */
    int32_t max_refine;      /* refinement passes                              */
    int32_t check_every;     /* BiCGStab iterations between host checks        */
    int32_t precond;         /* FIM_PC_JACOBI, FIM_PC_FRACTURE (default) or
                                FIM_PC_FRACTURE_COUPLED (both Jacobi when the
                                model has no frac_id); others: FIM_E_ARG      */
    double  eps_res;         /* FIM_RESID: unconverged when e_i >= eps_res
                                (default 1e-6)                                 */
    int32_t res_layers;      /* FIM_RESID: neighbour layers added (default 1,
                                at most 8)                                     */
    double  forcing_max;     /* > lin_rtol (default 0.1): inexact Newton
                                forcing term of Eisenstat and Walker (1996,
                                choice 2: eta = 0.9 (|F_k| / |F_k-1|)^a,
                                a = (1 + sqrt 5) / 2, safeguarded by
                                0.9 eta_k-1^a when that exceeds 0.1) within
                                [lin_rtol, forcing_max],
                                forcing_max on a timestep's first iteration;
                                |F| is the iteration's local residual
                                (FIM_FULL, FIM_LOCAL; FIM_RESID after a
                                first iteration at lin_rtol; the sweeps of
                                FIM_DD and FIM_DD_ADD with one sequence per
                                subdomain).  Algorithm 2's subdomain-building
                                phase, tight mode and forcing_max <=
                                lin_rtol solve every iteration to lin_rtol.
                                Negative or non-finite: FIM_E_ARG            */
} fim_options;

typedef struct fim_iter_stats {
    int32_t n_active;        /* n_A of this iteration                     */
    int32_t n_boundary;      /* |V_B| of this iteration                   */
    int32_t is_expand;       /* mode after this iteration                 */
    int32_t converged;       /* timestep converged and committed          */
    int32_t krylov_iters;
    int32_t refine_passes;
    int32_t n_switch;
    int32_t nonfinite;
    int32_t phase;           /* Algorithm 2: 1 build, 2 sweep; else 0     */
    int32_t subdomain;       /* Algorithm 2 subdomain index               */
    double  dp_max;          /* ||dp||_inf over the active cells (Pa)     */
    double  ds_max;
    double  lin_relres;      /* ||J x + F|| / ||F||                       */
    int32_t fp64_fallback;   /* mixed precision: FP32 passes stalled and the
                                solve finished with the FP64 Krylov        */
} fim_iter_stats;

typedef struct fim_step_stats {
    int32_t iterations;      /* Newton (or Algorithm 2 inner) iterations  */
    int32_t converged;
    int32_t cuts;            /* dt halvings used                          */
    int32_t krylov_iters;
    double  sum_active;      /* sum of n_A over the iterations            */
    int32_t max_active;
    int32_t subdomains;      /* Algorithm 2: N                            */
} fim_step_stats;

typedef struct fim_model fim_model;

void fim_default_options(fim_options* o);

/* Uploads the model (Section 4.3, the index set V and the connection
 * graph).  hip_stream: a hipStream_t or NULL.  Errors: FIM_E_ARG on an
 * invalid description or when the Jacobian blocks of the whole grid would
 * pass 4 GiB (64 (max degree + 1) ceil(n/64) b^2 8 bytes; about 40 M
 * cells at b = 3 and degree 10), FIM_E_NOMEM / FIM_E_HIP on device
 * failures; *out is NULL then. */
fim_status fim_create_model(const fim_model_desc* d, const fim_options* o,
                            void* hip_stream, fim_model** out);

/* Replaces the state (b planes of n doubles, status may be NULL for
 * b < 3) and ends any timestep in progress; the next Newton call starts a
 * new timestep from this state with a fresh history (first-step initial
 * active set).  mem: FIM_HOST or FIM_DEVICE.  Non-finite input returns
 * FIM_E_NONFINITE and leaves the previous state. */
fim_status fim_set_state(fim_model* m, const double* u, const int8_t* status, int mem);

/* Copies the current state (mid-step: the current Newton iterate). */
fim_status fim_get_state(fim_model* m, double* u_out, int8_t* status_out, int mem);

/* Checkpoints between timesteps.  A timestep maps u^n to u^{n+1}
 * (Section 4.1), but Algorithm 1 (Section 4.3) and Algorithm 2 (Section
 * 4.4) seed a step's first active set from the previous step's support
 * (the cells whose update reached the cutoff), so a run resumed from u and
 * the phase status alone starts its next step from the first-step seed set
 * instead.  A checkpoint carries both: a host byte blob of
 * fim_checkpoint_bytes(m) bytes (a header with the model's n and b, the
 * state as b planes of n doubles, the phase status, the support set).
 * After fim_set_checkpoint the model's next timesteps run bit for bit as
 * they ran after fim_get_checkpoint in the run that wrote it (same model
 * description and options).
 * fim_checkpoint_bytes: -1 for a NULL model.
 * fim_get_checkpoint: buf is host memory the caller owns, of at least
 * that size (FIM_E_ARG otherwise); FIM_E_STATE inside a timestep.
 * fim_set_checkpoint: ends any timestep in progress; FIM_E_ARG on a blob
 * that is shorter than the model's size, not a checkpoint of this library
 * or of another n or b; FIM_E_NONFINITE on a non-finite state (the
 * previous state is kept in both cases). */
int64_t    fim_checkpoint_bytes(const fim_model* m);
fim_status fim_get_checkpoint(fim_model* m, void* buf, int64_t cap);
fim_status fim_set_checkpoint(fim_model* m, const void* buf, int64_t len);

/* One Newton iteration (Algorithm 1 in FIM_LOCAL, the standard iteration
 * in FIM_FULL, one subdomain solve of Algorithm 2 in FIM_DD, one
 * residual-localized iteration in FIM_RESID).  The first
 * call of a timestep stores u^n and the initial active set.  When the
 * stopping test of the algorithm holds the step is committed and
 * st->converged = 1.  Calling with a different dt or mode inside a step
 * returns FIM_E_STATE.  Hitting max_newton rolls back and returns
 * FIM_NOT_CONVERGED.  st may be NULL. */
fim_status fim_newton_step(fim_model* m, double dt, int mode, fim_iter_stats* st);

/* Loops fim_newton_step to convergence (Section 4.1).  On failure rolls
 * back to u^n and returns FIM_NOT_CONVERGED.  With auto_cut a failed step
 * is replaced by two substeps of half the size, each cut again on failure
 * (at most max_cuts halvings); substeps that converge are committed as
 * they go, and when a substep fails at the halving limit the model is
 * restored to the state, phase status and previous-step support it had
 * on entry before FIM_NOT_CONVERGED returns. */
fim_status fim_solve_timestep(fim_model* m, double dt, int mode, fim_step_stats* st);

/* For callers that cannot allocate memory (code that must not call
 * hipMalloc: HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): fim_newton_step with the same arguments, results (bit for
 * bit) and return codes, but no device or pinned memory is allocated or
 * freed by the call.  The kernels' partial sums, Krylov scalars,
 * compaction tile counts and launch descriptors come from one static
 * device array per GPU (about 0.65 MB, held until the process ends)
 * instead of the model's own buffers; everything else is the model's
 * memory, allocated by fim_create_model.  Limits: models of at most
 * 4,194,304 cells (FIM_E_ARG beyond), modes FIM_FULL, FIM_LOCAL and
 * FIM_RESID (FIM_DD returns FIM_E_ARG: its subdomain lists grow), the
 * event profiler off (FIM_E_STATE).  All models on one GPU share that
 * GPU's array and it keeps the last call's contents: calls that overlap
 * in time on one GPU (different streams or threads) race and must be
 * serialised by the caller.  It may be mixed with fim_newton_step on the
 * same model and timestep. */
fim_status fim_newton_step_noalloc(fim_model* m, double dt, int mode, fim_iter_stats* st);

/* Frees all device memory after synchronising the stream. */
fim_status fim_destroy_model(fim_model* m);

/* Last error message of the handle (never NULL); with m = NULL, the
 * reason the calling thread's last fim_create_model failed. */
const char* fim_last_error(const fim_model* m);

int32_t fim_num_cells(const fim_model* m);
int32_t fim_block_size(const fim_model* m);

/* ---------------- device footprint -------------------------------------- */

/* Device bytes a model holds, and the bytes fim_create_model would
 * allocate for a description (computed without allocating; -1 on an
 * invalid description).  Used for admission by HBM footprint. */
int64_t fim_model_bytes(const fim_model* m);
int64_t fim_estimate_bytes(const fim_model_desc* d, const fim_options* o);

/* ---------------- batches of models ------------------------------------ */

/* A batch advances several independent models together: each call runs
 * one Newton iteration (Algorithm 1, full Newton or the residual-based
 * mode; Algorithm 2 members: see below) of every member with one launch
 * per kernel for all members (the
 * timestep starts, assembly, the local linear systems' Krylov solves, the
 * updates, active sets and structure; per-member reductions and
 * convergence) and one synchronisation for the members' status words, plus
 * one when some member starts a timestep.  A member's result is the same
 * alone and in any batch.  Members keep their
 * own state and may be in different phases of their own timesteps; a
 * member whose step converged starts its next step at its next call.
 * Members need the same block size and Krylov precision; the batch does
 * not own them.  Membership can change between calls (fim_batch_set), which
 * is how a serving loop admits and retires requests.  hip_stream: stream of
 * the batch's launches (NULL: own stream); members' own streams are
 * ordered before and after each call with events. */
typedef struct fim_batch fim_batch;

fim_status fim_batch_create(fim_model* const* models, int32_t k, void* hip_stream,
                            fim_batch** out);
fim_status fim_batch_set(fim_batch* b, fim_model* const* models, int32_t k);

/* dts[k], modes[k] (FIM_FULL, FIM_LOCAL, FIM_RESID, or FIM_DD /
 * FIM_DD_ADD) per member; Algorithm 2 members run one inner iteration
 * each with their own launches on the batch stream (their subdomain
 * phases are host-driven), the others share the batched launches; stats (nullable)
 * and codes receive each member's statistics and status (FIM_OK,
 * FIM_NOT_CONVERGED after a rollback, or a negative error).  The call
 * itself returns FIM_OK unless the batch as a whole failed. */
fim_status fim_batch_newton_step(fim_batch* b, const double* dts, const int32_t* modes,
                                 fim_iter_stats* stats, int32_t* codes);
fim_status fim_batch_destroy(fim_batch* b);
const char* fim_batch_last_error(const fim_batch* b);

/* ---------------- cell classes of an iteration ------------------------- */

/* Section 5.2.1 plots four cell sets per Newton iteration: active cells,
 * boundary cells, active cells with a non-negligible update and boundary
 * cells with a non-negligible update.  When enabled, every iteration
 * records per cell: bit 0 = active, bit 1 = boundary (V_B; never set in
 * FIM_FULL), bit 2 = |dp| >= eps_loc; inactive cells read 0.  out: host
 * u8[n], the classes of the last iteration run. */
fim_status fim_flags_enable(fim_model* m, int32_t on);
fim_status fim_get_flags(fim_model* m, uint8_t* out);

/* ---------------- profiling ------------------------------------------- */

/* Per-kernel timing with hipEvents recorded on the model's stream around
 * each launch (kernel classes: assemble, precond, ir_residual,
 * bicg_spmv_p, bicg_spmv_s, update, sets_compact, step_setup,
 * frac_invert).  BiCGStab launches queued after the solve converged return
 * at once and are not counted.  rows = sum over launches of the active
 * rows the launch processed, nnzb = sum of the blocks (diagonal included)
 * of the local matrix for the kernels that read or write it, aux = sum of
 * the fracture-block inverse entries that the product kernels applied
 * (zero without fracture blocks).  Profiling adds event records and one
 * extra synchronisation per linear solve and is off by default. */
typedef struct fim_kernel_profile {
    char    name[32];
    int64_t launches;
    double  total_ms;
    double  rows;
    double  nnzb;
    double  aux;
} fim_kernel_profile;

/* on != 0 clears the counters and starts recording; 0 stops. */
fim_status fim_profile_enable(fim_model* m, int32_t on);

/* Fills up to cap records; returns the number written. */
int32_t fim_profile_read(fim_model* m, fim_kernel_profile* out, int32_t cap);

/* ---------------- inspection entry points (used by parity tests) -------- */

/* Assembles F_A and J_A = R_A J R_A^T (Section 4.3) at iterate u_iter with
 * old-time state u_old, on the active set act (host u8[n], NULL = all
 * cells), without solving.  Outputs (host, caller-allocated): n_active,
 * l2g[n] (first n_active used), F[n_active b], and the matrix in block
 * CSR form: row_ptr[n_active+1], col[cap_blocks], val[cap_blocks b b]
 * (row-major blocks, diagonal block first in each row, then active
 * neighbours ascending).  FIM_E_ARG if cap_blocks is too small.  Ends any
 * timestep in progress and leaves u_iter as the current state. */
fim_status fim_inspect_assemble(fim_model* m, const double* u_old,
                                const double* u_iter, const int8_t* status,
                                double dt, const uint8_t* act,
                                int32_t* n_active, int32_t* l2g, double* F,
                                int32_t* row_ptr, int32_t* col, double* val,
                                int64_t cap_blocks);

/* Runs one active-set update of Algorithm 1 (expand or shrink) on given
 * inputs: act_in and dp_abs (host, [n]); writes act_out, bnd_out (host
 * u8[n], boundary of the new set), l2g_out (host i32[n]; first *n_active
 * entries), *is_expand.  bnd of the input set is computed by the library. */
fim_status fim_inspect_sets(fim_model* m, const uint8_t* act_in,
                            const double* dp_abs, double eps, int32_t layers,
                            uint8_t* act_out, uint8_t* bnd_out,
                            int32_t* l2g_out, int32_t* n_active,
                            int32_t* is_expand);

/* The error measure of FIM_RESID (see the solver modes) at state u_iter
 * with old-time state u_old and step dt, on every cell: err_out (host,
 * [n]).  status may be NULL (all 0).  Ends any timestep in progress and
 * leaves u_iter as the current state. */
fim_status fim_inspect_resid_error(fim_model* m, const double* u_old,
                                   const double* u_iter, const int8_t* status,
                                   double dt, double* err_out);

/* The FIM_RESID active set from a given error array err (host, [n]): the
 * cells with err_i >= tol and their layers-layer neighbourhood (layers in
 * [0, 8], else FIM_E_ARG).  Writes act_out (host u8[n]), l2g_out (host
 * i32[n]; first *n_active entries, ascending) and *n_unconverged (cells
 * with err_i >= tol).  Ends any timestep in progress. */
fim_status fim_inspect_resid_sets(fim_model* m, const double* err, double tol,
                                  int32_t layers, uint8_t* act_out,
                                  int32_t* l2g_out, int32_t* n_active,
                                  int32_t* n_unconverged);

/* The fracture-block layout of the preconditioner (FIM_PC_FRACTURE) for
 * the active set act (host u8[n], NULL = all cells): *n_active, l2g (host
 * i32[n], first *n_active entries, ascending) and, per active row r,
 * blk_start[r] = the first row of r's block and blk_rows[r] = its rows
 * (1 for matrix rows and one-row blocks).  Each run of consecutive rows of
 * one fracture inside a 256-row tile is cut into blocks of whole units of
 * the fracture (its cells in index order, u at a time, u = the largest
 * index-order distance of a connection inside the fracture when that is at
 * most c cells, else 1), at most c cells each (c = 64, 20, 21 for b = 1, 2,
 * 3), in about equal parts.  FIM_E_STATE without fracture blocks.  Ends any timestep in
 * progress. */
fim_status fim_inspect_pc_blocks(fim_model* m, const uint8_t* act,
                                 int32_t* n_active, int32_t* l2g,
                                 int32_t* blk_start, int32_t* blk_rows);

/* Solves J_A x = -F_A for the system of the last fim_inspect_assemble with
 * the library's Krylov solver (precision as in the options); x (host,
 * [n_active b]).  *iters receives BiCGStab iterations, *relres the final
 * ||J x + F|| / ||F||. */
fim_status fim_inspect_solve(fim_model* m, double* x, int32_t* iters,
                             double* relres);

/* Algorithm 2 (Section 4.4, Step 1), the set logic that follows the local
 * solve on subdomain V_A^k, on given inputs (host u8[n] flags and
 * dp_abs[n] = |dp_i|): vt_in = V_T so far, act_in = V_A^k, bnd_in = V_B^k
 * (read on the cells of act_in only).  The layers-layer neighbourhoods of
 * the cells of V_B^k with dp_abs >= eps join V_T and form V_A^{k+1}; then
 * V_B^{k+1} = boundary(V_T) ^ V_A^{k+1} (boundary: cells of the set with a
 * neighbour outside it) and dB^{k+1} = the cells outside V_A^{k+1}
 * adjacent to it.  Outputs (host u8[n]): vt_out = updated V_T, act_out =
 * V_A^{k+1}, bnd_out = V_B^{k+1}, outer_out = dB^{k+1}; *n_active =
 * |V_A^{k+1}|; *is_expand = whether any cell of V_B^k qualified (when 0,
 * the three next-set outputs are all zero).  layers in [0, 8], else
 * FIM_E_ARG.  Ends any timestep in progress. */
fim_status fim_inspect_dd_expand(fim_model* m, const uint8_t* vt_in,
                                 const uint8_t* act_in, const uint8_t* bnd_in,
                                 const double* dp_abs, double eps, int32_t layers,
                                 uint8_t* vt_out, uint8_t* act_out,
                                 uint8_t* bnd_out, uint8_t* outer_out,
                                 int32_t* n_active, int32_t* is_expand);

/* Algorithm 2 (Section 4.4, Step 2), the choice of the next subdomain to
 * solve.  n_sub subdomains (1..64) given as host lists: subdomain k has
 * the cells cells[cells_ptr[k] .. cells_ptr[k+1]) and the outer-layer
 * cells outer[outer_ptr[k] .. outer_ptr[k+1]) (offsets start at 0 and do
 * not decrease; indices in [0, n)).  last_dp (host, [n]) holds each cell's
 * |dp| from the latest solve that touched it.  sub_max[k] (host, [n_sub])
 * receives the largest last_dp over subdomain k and its outer layer;
 * *pick the first k, searching cyclically from position next (0..n_sub:
 * one past the subdomain solved last), with sub_max[k] >= eps, or -1;
 * *new_sweep = 1 when that search passed the end of the list (the pick
 * opens the next sweep).  Ends any timestep in progress. */
fim_status fim_inspect_dd_pick(fim_model* m, int32_t n_sub,
                               const int32_t* cells_ptr, const int32_t* cells,
                               const int32_t* outer_ptr, const int32_t* outer,
                               const double* last_dp, double eps, int32_t next,
                               double* sub_max, int32_t* pick,
                               int32_t* new_sweep);

/* V_T (Section 4.4: the union of the subdomains) of the most recent
 * Algorithm 2 timestep (in progress or committed): vt_out host u8[n];
 * *n_sub = the number of subdomains built.  FIM_E_STATE when no Algorithm
 * 2 step has run since the model was created or an Algorithm 2
 * inspection call ran. */
fim_status fim_get_dd_total(fim_model* m, uint8_t* vt_out, int32_t* n_sub);

#ifdef __cplusplus
}
#endif

#endif /* FIM_H */
