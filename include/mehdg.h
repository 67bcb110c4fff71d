/*
 * mehdg.h -- C ABI of the MI355X library for the per-macro-element local
 * work of one Newton step of the entropy-variable macro-element HDG method
 * (arXiv 2507.22195).
 *
 * Discretisation.  Every macro-element is an axis-aligned box split into
 * 2x2x2 hexahedral sub-elements carrying a C0-continuous tensor Q_p space on
 * Gauss-Lobatto nodes (Sec. 3.1, local space W_p(K)); macro-elements are
 * coupled only through the trace unknowns on their six faces.  Volume
 * integrals use p+1 Gauss points per sub-element and axis, face integrals
 * the matching 2-D rule (Sec. 3.1 eq. C31, C32).
 *
 * Unknowns and layouts (device memory, float64, row-major, per macro m):
 *   n1d = 2p+1, n = n1d^3, nf = n1d^2
 *   v      [m][5][n]        entropy variables (eq. s222), node a = i + n1d*(j + n1d*k)
 *   q      [m][5][3][n]     gradient unknown q_{kj} ~ d v_k / d x_j
 *   vhat   [m][6][5][nf]    trace, gathered per macro; faces (-x,+x,-y,+y,-z,+z);
 *                           face node c = c1 + n1d*c2 over the two tangential axes
 *                           in increasing axis order
 *   N_V = 5n, N_Q = 15n, N_VH = 30 nf
 *   V index  k*n + a,  Q index (k*3 + j)*n + a,  Vhat index (f*5 + k)*nf + c.
 *
 * Ownership.  The caller owns every array passed in or out.  The context
 * owns its tables and workspaces: pointwise Jacobian coefficients, the
 * bordered matrix [[S, -Y, r_V], [X, A', r_hat]] of every macro, and after
 * mehdg_condense its factors (U of S, L^-1 P(-Y), L^-1 P r_V), which
 * mehdg_recover reads.  mehdg_assemble(want_blocks = 1) overwrites the
 * bordered matrices; mehdg_condense overwrites them with factors.
 *
 * Errors.  Argument errors are detected on the host before anything is
 * enqueued and return MEHDG_EINVAL / MEHDG_ESTATE.  Device-side conditions
 * (non-physical state, non-finite values, zero pivot) never abort a kernel:
 * the kernel records a per-macro status code, and at the end of every
 * compute call the outputs of each macro whose code is set (codes persist
 * until mehdg_status clears them) are overwritten with NaN: R_q, R_v,
 * R_vhat, entropy after mehdg_assemble; Ahat, bhat after mehdg_condense;
 * dv, dq after mehdg_recover.  mehdg_status returns the codes.
 *
 * Asynchrony.  Every compute call only enqueues work on the given stream
 * (NULL = default stream) and returns.  mehdg_create and mehdg_status
 * synchronise.  Calls on one context must not overlap on different streams.
 */
#ifndef MEHDG_H
#define MEHDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mehdg_ctx mehdg_ctx;
typedef struct ihipStream_t* mehdg_stream; /* a hipStream_t */

typedef enum {
    MEHDG_OK = 0,
    MEHDG_EINVAL = 1,        /* bad argument */
    MEHDG_ENOMEM = 2,        /* device allocation failed */
    MEHDG_EHIP = 3,          /* HIP runtime error (launch, copy) */
    MEHDG_ESTATE = 4,        /* call out of order (recover before condense) */
    MEHDG_ENONPHYSICAL = 5,  /* per macro: beta = -v5 <= 0 or rho, P not positive */
    MEHDG_ENONFINITE = 6,    /* per macro: NaN / Inf met in inputs or results */
    MEHDG_ESINGULAR = 7,     /* per macro: zero pivot in the LU of S */
    MEHDG_EIRNOCONV = 8      /* per macro: iterative refinement of a mixed-precision
                                condensation did not reach ir_tol in ir_maxit steps */
} mehdg_err;

/* Arithmetic of the condensation (mehdg_condense). */
typedef enum {
    MEHDG_FP64 = 0,          /* blocked LU of S and Schur product in FP64 (MFMA) */
    MEHDG_FP32_IR = 1,       /* LU of S and its solves in FP32 (MFMA, FP32 accumulation),
                                refined with FP64 residuals; Schur product in FP64 */
    MEHDG_BF16_IR = 2        /* as FP32_IR with the LU's trailing updates on BF16 MFMA
                                (operands rounded to BF16, FP32 accumulation) */
} mehdg_prec;

typedef enum {
    MEHDG_FLUX_EC = 0,       /* entropy-conservative KEP flux, eq. (EC) */
    MEHDG_FLUX_ES = 1,       /* entropy-stable flux, eq. (Flux_En_Inv) */
    MEHDG_FLUX_KEPES = 2     /* KEP + entropy-stable flux, eq. (ES) */
} mehdg_flux;

/* Physical and numerical parameters (acoustic scaling: rho0 = c0 = 1). */
typedef struct {
    double gamma;          /* ratio of specific heats */
    double mu;             /* mu / Re_c, viscous stress coefficient (eq. C6) */
    double kappa;          /* heat flux phi = -kappa grad T, T = gamma P / rho */
    double lam;            /* bulk viscosity ratio lambda (eq. C6), -2/3 Stokes */
    double sigma_vis[5];   /* diagonal viscous trace penalty (eq. Flux_En_Vis) */
    double alpha_t;        /* time term alpha_t (u(v) - u(v_old), w) (eq. C242) */
    double alpha_ps;       /* pseudo-time term alpha_ps (A0 dv, w): Jacobian only */
    double logmean_eps;    /* series branch of the log mean when ((a-b)/(a+b))^2 < eps */
    double T_wall;         /* wall temperature T = gamma P / rho of isothermal wall faces (> 0 if any) */
    int32_t flux;          /* mehdg_flux */
    int32_t viscous;       /* 0: Euler (G = 0), 1: Navier-Stokes */
    double ir_tol;         /* mixed precision: stop refining when the estimated relative
                              forward error of S^-1 [-Y | r_V] is below ir_tol (> 0) */
    int32_t ir_maxit;      /* mixed precision: at most this many refinement steps (>= 1) */
    int32_t pad_;
} mehdg_params;

/* Macro-element mesh.  All pointers are host memory, copied at create. */
typedef struct {
    int64_t n_macro;
    int32_t p;             /* polynomial degree of the sub-elements, 1..4 (4: see below) */
    int32_t pad_;
    const double* h;       /* [n_macro][3] sub-element edge lengths (macro = 2h) */
    const uint8_t* face_bc;/* [n_macro][6] or NULL: 1 = isothermal no-slip wall, 0 = interior/periodic */
} mehdg_mesh;

/* Sizes of one macro-element at degree p = 1..4 (n, nf, N_V, N_Q, N_VH), the
 * degrees mehdg_create accepts; other degrees are MEHDG_EINVAL.
 * Degree 4 (N_V 3645, N_VH 2430, a 295 MB bordered matrix per macro) takes
 * the FP64 Newton step: mehdg_assemble with want_blocks 0 or 1,
 * mehdg_condense(MEHDG_FP64), mehdg_recover and the diagnostics.  The other
 * entry points (products, stored-factor solves, the trace system, the
 * mixed-precision modes, want_blocks 2) return MEHDG_EINVAL at degree 4. */
mehdg_err mehdg_sizes(int32_t p, int64_t out[5]);

/* Builds the reference tables, copies the mesh and allocates workspaces.
 * Synchronises.  On error *out is NULL.  face_bc entries other than 0 and 1,
 * or wall faces with T_wall <= 0, are MEHDG_EINVAL. */
mehdg_err mehdg_create(const mehdg_mesh* mesh, const mehdg_params* prm, mehdg_ctx** out);

mehdg_err mehdg_destroy(mehdg_ctx* ctx);

/* Residual of eq. (s32a)-(s32c) with the stage time term of eq. (C242), per
 * macro-element (the trace residual is this macro's local contribution; the
 * caller sums the two sides of each face), plus the face entropy production
 * sum_s w ([[v]]^T Fhat - [[Psi_n]]) of Thm. (EC_ES) with the inviscid trace
 * flux.  On a wall face (mesh face_bc = 1) the trace equations take the
 * boundary operator [(Fhat + Ghat)_1, vhat_2, vhat_3, vhat_4, vhat_5 + gamma/T_wall]
 * (no mass flux, zero velocity, T = T_wall; a reading: the paper gives no
 * wall operator) tested against the trace basis; the element equations keep
 * Fhat + Ghat.  q may be NULL: then q is the weak gradient of (v, vhat), i.e. the
 * solution of R_Q = 0.  With want_blocks = 1 also assembles, per macro, the
 * Jacobian blocks of Sec. 6.2 with Q eliminated (eq. R1-R3): the bordered
 * matrix [[S, -Y, r_V], [X, A', r_hat]] in the context workspace.  With
 * want_blocks = 2 only the pointwise Jacobian coefficients that mehdg_jvp and
 * mehdg_vjp read are stored (no bordered matrix; a preceding condensation's
 * factors stay valid).  Both 1 and 2 set the state those products linearise at.
 *   v, v_old [n_macro][5][n]; vhat [n_macro][6][5][nf]; q NULL or [n_macro][5][3][n];
 *   R_q [n_macro][5][3][n]; R_v [n_macro][5][n]; R_vhat [n_macro][6][5][nf];
 *   entropy [n_macro].  All device pointers. */
mehdg_err mehdg_assemble(mehdg_ctx* ctx, const double* v, const double* vhat, const double* q,
                         const double* v_old, double* R_q, double* R_v, double* R_vhat,
                         double* entropy, int32_t want_blocks, mehdg_stream stream);

/* Static condensation (Sec. 6.2 eq. R4-R5): partial-pivoted LU of S and the
 * trace Schur complement Ahat = A' + X S^-1 Y and right-hand side
 * bhat = r_hat - X S^-1 r_V of every macro.  Requires a preceding assemble
 * with want_blocks = 1.  Ahat [n_macro][N_VH][N_VH] may be NULL (only bhat is
 * formed); bhat [n_macro][N_VH].  Device pointers.
 *   prec = MEHDG_FP64: the FP64 blocked LU over the bordered matrix.
 *   prec = MEHDG_FP32_IR / MEHDG_BF16_IR: S is factored in low precision;
 *   Z = S^-1 [-Y | r_V] is solved with those factors and refined with FP64
 *   residuals [-Y | r_V] - S Z until the estimated relative forward error of
 *   Z (the size of the last correction times the observed contraction
 *   rho / (1 - rho)) is at most params.ir_tol, in at most params.ir_maxit
 *   steps; a macro that does not get there is flagged MEHDG_EIRNOCONV (its
 *   outputs are NaN like any flagged macro's).  Then Ahat = A' + X S^-1 Y and
 *   bhat in FP64.  The residual, u(v), the log means and the entropy sums are
 *   FP64 in every mode.  The low-precision workspace holds a wave of macros
 *   (at most 32 GiB; the batch is processed wave by wave), allocated at the
 *   first mixed call.  After a mixed condensation, mehdg_recover works as
 *   after FP64, mehdg_condense_rhs returns MEHDG_ESTATE (the factors of S are
 *   not kept), and mehdg_copy_bordered shows Z (its Y part transposed in the
 *   X rows, its r_V part in the r_V column) in place of the factors.  Invalid
 *   prec, or a mixed prec with ir_tol <= 0 or ir_maxit < 1: MEHDG_EINVAL. */
mehdg_err mehdg_condense(mehdg_ctx* ctx, int32_t prec, double* Ahat, double* bhat, mehdg_stream stream);

/* Refinement steps of the last mixed-precision mehdg_condense (the most any
 * wave of macros needed; 0 after an FP64 condensation). */
int32_t mehdg_ir_iterations(const mehdg_ctx* ctx);

/* The stored condensation applied to a new right-hand side (Sec. 6.2 eq. R4,
 * R5b): with r_V [n_macro][N_V] (V ordering) and r_hat [n_macro][N_VH]
 * (NULL: zero) in place of the assembled -R_V + A_vq A_qq^-1 R_Q and
 * -R_Vhat + A_vhatq A_qq^-1 R_Q, writes bhat = r_hat - X S^-1 r_V and makes
 * the next mehdg_recover return dV = S^-1 (r_V + Y dVhat) (dQ from its R_q
 * argument as before).  Requires a preceding mehdg_condense (else
 * MEHDG_ESTATE); the factors are kept.  This solves the assembled Newton
 * system for any right-hand side, e.g. as the preconditioner of a
 * Jacobian-free Newton-Krylov iteration.  Device pointers. */
mehdg_err mehdg_condense_rhs(mehdg_ctx* ctx, const double* r_v, const double* r_hat, double* bhat,
                             mehdg_stream stream);

/* Back-substitution once the trace update is known (eq. R2 then R6):
 * dV = S^-1 (r_V + Y dVhat), dQ = A_qq^-1 (-R_Q - A_qv dV - A_qvhat dVhat).
 * R_q is the residual returned by the assemble that preceded the condense.
 *   dvhat [n_macro][6][5][nf]; dv [n_macro][5][n]; dq [n_macro][5][3][n]. */
mehdg_err mehdg_recover(mehdg_ctx* ctx, const double* R_q, const double* dvhat, double* dv,
                        double* dq, mehdg_stream stream);

/* Jacobian-vector product of the residual of mehdg_assemble (Sec. 4.1
 * eq. s32a-c with the time term of eq. C242; the Jacobian of Sec. 6.2 eq. R1,
 * with the pseudo-time term alpha_ps (A0 dv, w) included as in the assembled
 * blocks), at the state of the last mehdg_assemble with want_blocks 1 or 2
 * (else MEHDG_ESTATE):
 *   [JR_q; JR_v; JR_vhat] = J [dq; dv; dvhat].
 * dq may be NULL: then dq is the weak gradient of (dv, dvhat), which is the
 * derivative of the residual computed with q = NULL (JR_q is then zero up to
 * rounding).  Layouts as in mehdg_assemble: dv, JR_v [n_macro][5][n];
 * dvhat, JR_vhat [n_macro][6][5][nf]; dq, JR_q [n_macro][5][3][n].  Device
 * pointers; outputs of macros with a status code set are NaN. */
mehdg_err mehdg_jvp(mehdg_ctx* ctx, const double* dv, const double* dvhat, const double* dq, double* JR_q,
                    double* JR_v, double* JR_vhat, mehdg_stream stream);

/* Vector-Jacobian product, the transpose of mehdg_jvp at the same state.
 * With w_q and g_q given: [g_q; g_v; g_vhat] = J^T [w_q; w_v; w_vhat], the
 * gradient of w_q.R_Q + w_v.R_V + w_vhat.R_Vhat in (q, v, vhat).  With
 * w_q = g_q = NULL: the gradient of w_v.R_V + w_vhat.R_Vhat in (v, vhat) with
 * q the weak gradient of (v, vhat) (the transpose of mehdg_jvp with
 * dq = NULL).  Exactly one of w_q, g_q NULL is MEHDG_EINVAL.  Layouts as in
 * mehdg_jvp; device pointers; outputs of flagged macros are NaN. */
mehdg_err mehdg_vjp(mehdg_ctx* ctx, const double* w_q, const double* w_v, const double* w_vhat, double* g_q,
                    double* g_v, double* g_vhat, mehdg_stream stream);

/* Copies the per-macro status codes (mehdg_err values, 0 = fine) of the
 * calls since the last mehdg_status into host memory status[n_macro] and
 * clears them.  Per macro the most basic condition met is kept (the smallest
 * code: MEHDG_ENONPHYSICAL before MEHDG_ENONFINITE before MEHDG_ESINGULAR).
 * Synchronises the stream.  Returns the first non-zero code in macro order,
 * or MEHDG_OK. */
mehdg_err mehdg_status(mehdg_ctx* ctx, int32_t* status, mehdg_stream stream);

/* Diagnostics.  Copies the bordered matrix of macro m (after an assemble
 * with want_blocks = 1; after mehdg_condense it holds the factors instead)
 * into host memory out[rows][ld], row-major with columns
 * [V (N_V) | Vhat (N_VH) | rhs | padding].  With out = NULL only *rows and
 * *ld are set.  Synchronises the device. */
mehdg_err mehdg_copy_bordered(mehdg_ctx* ctx, int64_t m, double* out, int64_t* rows, int64_t* ld);

/* Tests.  Replaces the bordered matrix of macro m with host memory
 * in[rows][ld] (layout of mehdg_copy_bordered), so that a test can hand the
 * condensation a matrix the assembly would not produce (e.g. a singular S:
 * MEHDG_ESINGULAR).  Requires the block workspace of an assemble with
 * want_blocks = 1 (else MEHDG_ESTATE); the context returns to the assembled
 * state (stored factors are invalid).  Synchronises the device. */
mehdg_err mehdg_load_bordered(mehdg_ctx* ctx, int64_t m, const double* in);

/* Kernel timing.  While enabled, every kernel launch of the context is
 * bracketed by HIP events recorded on the launch's own stream.
 * mehdg_profile_read synchronises the device, then returns and clears, per
 * kernel slot i < n (at most MEHDG_NPROF), the summed milliseconds ms[i] and
 * the number of launches calls[i] since the last read.  Host arrays. */
enum {
    MEHDG_PROF_RESIDUAL = 0,   /* residual (+ pointwise Jacobian coefficients) */
    MEHDG_PROF_MINV_RQ = 1,    /* M^-1 R_Q */
    MEHDG_PROF_ROWS_V = 2,     /* bordered rows of the interior equations */
    MEHDG_PROF_ROWS_H = 3,     /* bordered rows of the trace equations */
    MEHDG_PROF_PANEL = 4,      /* panel factorisation */
    MEHDG_PROF_ROWBLOCK = 5,   /* L^-1 applied to the columns right of a panel / block */
    MEHDG_PROF_UPDATE = 6,     /* trailing MFMA update */
    MEHDG_PROF_SCHUR = 7,      /* Ahat = A' - L21 U12 on MFMA */
    MEHDG_PROF_RECOVER = 8,    /* back-substitution */
    MEHDG_PROF_TRSM = 9,       /* L21 = X U^-1 of the trace rows */
    MEHDG_PROF_JVP = 10,       /* Jacobian-vector product */
    MEHDG_PROF_VJP = 11,       /* vector-Jacobian product */
    MEHDG_PROF_FSOLVE = 12,    /* stored factors applied to a new right-hand side */
    MEHDG_PROF_LP_PANEL = 13,  /* mixed precision: FP32 panel of the LU of S */
    MEHDG_PROF_LP_UPDATE = 14, /* mixed precision: FP32 / BF16 MFMA trailing update */
    MEHDG_PROF_LP_SOLVE = 15,  /* mixed precision: solves with the low-precision factors */
    MEHDG_PROF_IR_RESID = 16,  /* mixed precision: FP64 refinement residual */
    MEHDG_PROF_LP_MOVE = 17,   /* mixed precision: conversion in, Z out */
    MEHDG_NPROF = 18
};
mehdg_err mehdg_profile_enable(mehdg_ctx* ctx, int32_t enable);
mehdg_err mehdg_profile_read(mehdg_ctx* ctx, double* ms, int64_t* calls, int32_t n);

/* Bytes of device workspace the context holds. */
int64_t mehdg_workspace_bytes(const mehdg_ctx* ctx);

/* Tile shapes of the batched FP64 MFMA products of the condensation (the
 * trailing updates of the LU of S and the Schur product, Sec. 6.2).  The
 * library carries a fixed list of variants; variant i is a workgroup of
 * shapes[6i] x shapes[6i+1] waves, each owning shapes[6i+2] x shapes[6i+3]
 * blocks of 16 x 16, K staged in chunks of shapes[6i+4], shapes[6i+5] waves
 * per SIMD asked for.  Every variant adds the products of one output element
 * in the same order, so the choice changes the time and never the bits.  A
 * context starts with the variant of the table compiled into the library
 * for its degree (written by the package's autotuner from a sweep that
 * times every variant on the device); mehdg_set_tile overrides it for one
 * call site (variant -1 restores the table's).  Host calls, no device work. */
typedef enum {
    MEHDG_TILE_UPDATE = 0,   /* trailing updates of the LU of S */
    MEHDG_TILE_SCHUR = 1,    /* [Ahat | bhat] = [A' | r_hat] - L21 [U12 | y], and the
                                products of the mixed-precision refinement */
    MEHDG_NTILE_SITES = 2
} mehdg_tile_site;
/* *count variants; shapes (host, 6 * count entries, or NULL) as above. */
mehdg_err mehdg_tile_variants(int32_t* count, int32_t* shapes);
mehdg_err mehdg_set_tile(mehdg_ctx* ctx, int32_t site, int32_t variant);
mehdg_err mehdg_get_tile(const mehdg_ctx* ctx, int32_t site, int32_t* variant);

/* Depth of the delayed trailing updates of the LU of S (Sec. 6.2).  The
 * columns of S are eliminated in outer blocks of 128, taken in groups of
 * `depth` blocks: inside a group the update of the S rows below waits until
 * the group's last block (each block first takes the pending update of its
 * own columns and rows), so the trailing part of the bordered matrix is read
 * and written once per group.  Depth 1 updates after every block; a depth of
 * at least the number of blocks makes the factorisation left-looking.  The
 * depth changes the time and the rounding order, never the factors beyond
 * rounding.  A context starts with the library's default for its degree;
 * mehdg_set_lu_depth(ctx, 0) restores it.  A new depth takes effect at the
 * next FP64 mehdg_condense; mehdg_condense_rhs always follows the depth of
 * the condensation whose factors it applies.  mehdg_get_lu_depth gives the
 * depth the next condensation will use.  Host calls, no device work;
 * MEHDG_EINVAL for depth < 0 or > 1024. */
mehdg_err mehdg_set_lu_depth(mehdg_ctx* ctx, int32_t depth);
mehdg_err mehdg_get_lu_depth(const mehdg_ctx* ctx, int32_t* depth);

/* ---------------------------------------------------------------------------
 * Batches of macro-elements of mixed degree (p = 1..4) and boundary type in
 * one call per phase of the Newton step.
 * The batch orders its macros by degree (stable) and keeps one context per
 * degree present; every per-macro array of a batch call is one flat device
 * array in that order, each macro's block of the size its degree gives:
 *   MEHDG_KEY_V      5n doubles   (v, v_old, R_v, dv)
 *   MEHDG_KEY_Q      15n          (R_q, dq)
 *   MEHDG_KEY_VHAT   30nf         (vhat, R_vhat, dvhat)
 *   MEHDG_KEY_ENTROPY 1, MEHDG_KEY_AHAT N_VH^2, MEHDG_KEY_BHAT N_VH
 * (n, nf, N_VH of the macro's degree, as mehdg_sizes), each block laid out
 * as in the single-degree calls.  Each degree's work runs on a stream of the
 * batch (default priority) forked from the caller's stream and joined back to
 * it, so the calls are asynchronous on that stream, and an FP64 step is
 * capturable in a HIP graph once the contexts' workspaces exist (after the
 * first step).  The residual pass (residual, entropy production, pointwise
 * Jacobian coefficients) of all groups that are not streamed is one
 * persistent launch: its workgroups take the macros from a device queue in
 * descending degree and run each with its degree's code.
 * Device memory: when the contexts of all groups would need more than
 * max_workspace_bytes, the groups with the largest macros are streamed in
 * waves (their context holds one wave and works through the group wave by
 * wave); mehdg_batch_groups reports the wave of every group.  The factors of
 * a streamed group are not kept, so mehdg_batch_recover assembles and
 * condenses each of its waves again from v, vhat, v_old (the same values,
 * bit for bit) before the back-substitution. */
typedef struct mehdg_batch mehdg_batch;
typedef struct {
    int64_t n_macro;
    const int32_t* p;        /* [n_macro] degree of every macro, 1..4 */
    const double* h;         /* [n_macro][3] sub-element edge lengths */
    const uint8_t* face_bc;  /* [n_macro][6] or NULL: 1 = isothermal no-slip wall */
    int64_t max_workspace_bytes;   /* device workspace of the contexts; 0: 60% of the free
                                      device memory at creation */
    int32_t residual_per_degree;   /* 0: the residual pass of all groups that are not streamed
                                      in one persistent launch over a degree-sorted queue;
                                      1: one residual launch per degree (same results) */
    int32_t pad_;
} mehdg_batch_mesh;
typedef enum {
    MEHDG_KEY_V = 0,
    MEHDG_KEY_Q = 1,
    MEHDG_KEY_VHAT = 2,
    MEHDG_KEY_ENTROPY = 3,
    MEHDG_KEY_AHAT = 4,
    MEHDG_KEY_BHAT = 5,
    MEHDG_NKEYS = 6
} mehdg_batch_key;

/* Creates the per-degree contexts (host mesh arrays, copied) and streams.
 * A degree outside 1..4 or invalid mesh data: MEHDG_EINVAL (as mehdg_create). */
mehdg_err mehdg_batch_create(const mehdg_batch_mesh* mesh, const mehdg_params* prm, mehdg_batch** out);
mehdg_err mehdg_batch_destroy(mehdg_batch* batch);

/* Flat layout of arrays of kind key: order[n_macro] (host) the macro at each
 * batch position, offsets[n_macro + 1] (host) the first double of each
 * position's block and the total; either may be NULL. */
mehdg_err mehdg_batch_layout(const mehdg_batch* batch, int32_t key, int64_t* order, int64_t* offsets);

/* Degree groups: *n_groups, and per group (arrays of at least 4 entries, or
 * NULL) its degree, first batch position, number of macros and wave (the
 * macros its context holds; equal to the number unless streamed). */
mehdg_err mehdg_batch_groups(const mehdg_batch* batch, int32_t* n_groups, int32_t* degree, int64_t* first,
                             int64_t* count, int64_t* wave);

/* mehdg_assemble (want_blocks = 1) then mehdg_condense(prec) on every degree
 * group, flat arrays as above (Ahat may be NULL).  Device pointers.  The
 * mixed-precision modes take degrees 1..3. */
mehdg_err mehdg_batch_assemble_condense(mehdg_batch* batch, int32_t prec, const double* v, const double* vhat,
                                        const double* v_old, double* R_q, double* R_v, double* R_vhat,
                                        double* entropy, double* Ahat, double* bhat, mehdg_stream stream);

/* mehdg_recover on every degree group, after mehdg_batch_assemble_condense.
 * v, vhat, v_old: the inputs of that call, read by streamed groups only (NULL
 * allowed when no group is streamed).  Device pointers. */
mehdg_err mehdg_batch_recover(mehdg_batch* batch, const double* v, const double* vhat, const double* v_old,
                              const double* R_q, const double* dvhat, double* dv, double* dq, mehdg_stream stream);

/* Status codes of every macro (host status[n_macro], macro order, not batch
 * order) since the last call, cleared; returns the first non-zero code in
 * macro order.  Synchronises the batch's streams (stream is not used). */
mehdg_err mehdg_batch_status(mehdg_batch* batch, int32_t* status, mehdg_stream stream);

/* ---------------------------------------------------------------------------
 * Global trace system of one Newton step (Sec. 6.2, Algorithm 1): with the
 * trace single-valued per global face,
 *   K dVhat = F,  K = sum_m P_m^T Ahat_m P_m,  F = sum_m P_m^T bhat_m,
 * the linearisation of sum_m R_Vhat,m = 0 (conservation on every face); P_m
 * gathers the six faces of macro m.  Global traces are [n_faces][5][nf]
 * (float64, device), a face's nodes ordered as on either of its two sides
 * (axis-aligned boxes of one orientation).  Ahat, bhat as returned by
 * mehdg_condense.
 *
 * Builds the face map: face_ids [n_macro][6] (host) gives the global face of
 * every local face; every face in [0, n_faces) must occur exactly twice
 * (periodic or interior faces) unless it is a wall face of the mesh's face_bc,
 * which belongs to its macro alone (a domain boundary: exactly one side, the
 * boundary operator's trace equations); anything else is MEHDG_EINVAL.
 * Synchronises. */
mehdg_err mehdg_trace_setup(mehdg_ctx* ctx, const int64_t* face_ids, int64_t n_faces);

/* F = sum_m P_m^T bhat_m. */
mehdg_err mehdg_trace_rhs(mehdg_ctx* ctx, const double* bhat, double* F, mehdg_stream stream);

/* y = K x (x, y global traces) from the per-macro Ahat.  Ahat may be NULL
 * after an FP64 mehdg_condense (else MEHDG_ESTATE): then K is applied without
 * Ahat, from the factors the condensation left in the context (Algorithm 1,
 * its four local stages): Ahat_m x_m = A' x_m + X S^-1 Y x_m
 * = A' x_m - L21 (U12 x_m), with U12 = L^-1 P (-Y) and L21 = X U^-1, two
 * products per macro and no triangular solve.  The same NULL convention holds
 * for mehdg_trace_precond_setup, mehdg_trace_solve and
 * mehdg_trace_solve_fgmres, so that a Newton step can call mehdg_condense
 * with Ahat = NULL and never store Ahat. */
mehdg_err mehdg_trace_apply(mehdg_ctx* ctx, const double* Ahat, const double* x, double* y,
                            mehdg_stream stream);

/* Per-macro trace xl [n_macro][6][5][nf] (the layout of vhat / dvhat) of a
 * global one xg. */
mehdg_err mehdg_trace_gather(mehdg_ctx* ctx, const double* xg, double* xl, mehdg_stream stream);

/* Block-Jacobi preconditioner of K (Sec. 6.4): inverts every diagonal face
 * block of K (5nf x 5nf: Ahat_m1[f1,f1] + Ahat_m2[f2,f2], plus the cross blocks
 * when both sides are faces of one macro) by Gauss-Jordan elimination with
 * partial pivoting; kept in the context.  For p <= 2 the block is eliminated
 * in LDS; the p = 3 block (245 x 245) in place in the context's workspace
 * (correct, bandwidth-bound). */
mehdg_err mehdg_trace_precond_setup(mehdg_ctx* ctx, const double* Ahat, mehdg_stream stream);

/* z = D^-1 r per face with the blocks of the last mehdg_trace_precond_setup. */
mehdg_err mehdg_trace_precond_apply(mehdg_ctx* ctx, const double* r, double* z, mehdg_stream stream);

/* Solves K x = F by restarted GMRES(restart) with the block-Jacobi
 * preconditioner on the right (set up here), classical Gram-Schmidt applied
 * twice; x holds the initial guess and returns the solution.  Stops when the
 * residual estimate reaches rtol ||F|| or after maxit iterations; *iters and
 * *relres (final true residual / ||F||) on return.  The tiny Hessenberg
 * least-squares problem is solved on the host: synchronises the stream in
 * every iteration.  restart in [1, 60]. */
mehdg_err mehdg_trace_solve(mehdg_ctx* ctx, const double* Ahat, const double* F, double* x, double rtol,
                            int32_t maxit, int32_t restart, int32_t* iters, double* relres,
                            mehdg_stream stream);

/* Sec. 6.4's solver: flexible GMRES(restart) on K x = F whose preconditioner
 * for every outer direction is `inner` iterations of GMRES (from zero, no
 * restart, right-preconditioned by the block Jacobi of
 * mehdg_trace_precond_setup, set up here); inner = 0 is plain block Jacobi.
 * Stops at rtol ||F|| (residual estimate) or after maxit outer iterations;
 * *iters outer iterations, *inner_iters inner iterations in total, *relres
 * the final true residual / ||F||.  restart and inner in [1, 60] and [0, 60].
 * Ahat NULL: matrix-free (see mehdg_trace_apply).  Synchronises the stream in
 * every iteration. */
mehdg_err mehdg_trace_solve_fgmres(mehdg_ctx* ctx, const double* Ahat, const double* F, double* x, double rtol,
                                   int32_t maxit, int32_t restart, int32_t inner, int32_t* iters,
                                   int32_t* inner_iters, double* relres, mehdg_stream stream);

/* Precision of the factors Algorithm 1's product reads inside the inner
 * iterations of mehdg_trace_solve_fgmres with Ahat NULL: MEHDG_FP64 (default)
 * or MEHDG_FP32_IR, single-precision copies of U12, L21 and A' (n_macro
 * (2 N_V N_VH + N_VH^2) floats, made once per FP64 condensation, on the first
 * such solve after it).  The product sums in FP64 either way; the outer
 * iterations and every other product keep the FP64 factors, so the solution
 * still meets rtol for the FP64 operator (the inner solve is only FGMRES's
 * preconditioner).  Other values: MEHDG_EINVAL.  Host call. */
mehdg_err mehdg_trace_set_inner_precision(mehdg_ctx* ctx, int32_t prec);

/* Constant source of a DIRK stage (Sec. 5.3): adds s [n_macro][5][n] to the
 * interior residual R_v and subtracts it from the right-hand side r_V of the
 * bordered matrix.  With v_old = v^n, stage i of a DIRK method with a_ii = a
 * for all i (alpha_t = 1/(a dt)) has the residual of mehdg_assemble plus
 * s_i = alpha_t dt sum_{j<i} a_ij R_sp(V_j), R_sp the residual without time
 * term.  Call between mehdg_assemble(want_blocks = 1) and mehdg_condense;
 * else MEHDG_ESTATE. */
mehdg_err mehdg_add_source(mehdg_ctx* ctx, const double* s, double* R_v, mehdg_stream stream);

/* Pseudo-transient continuation (Sec. 6.1): sets the pseudo-time coefficient
 * alpha_ps = 1/tau of the Jacobian term alpha_ps (A0 dv, w) for the following
 * mehdg_assemble calls (and the JVP / VJP of the state they store), so that a
 * Newton loop can adapt tau between iterations; the residual does not depend
 * on it.  alpha_ps < 0 or not finite: MEHDG_EINVAL. */
mehdg_err mehdg_set_pseudo_time(mehdg_ctx* ctx, double alpha_ps);

/* y = a x + b y for device vectors of n doubles.  A zero coefficient drops its
 * term without reading the vector (a = 0: x is not read; b = 0: y is not read),
 * so NaN or Inf left in unread memory does not propagate. */
mehdg_err mehdg_axpby(int64_t n, double a, const double* x, double b, double* y, mehdg_stream stream);

/* *out = x . y for device vectors of n doubles (partial sums on the device,
 * summed on the host in a fixed order).  Synchronises the stream. */
mehdg_err mehdg_dot(mehdg_ctx* ctx, int64_t n, const double* x, const double* y, double* out,
                    mehdg_stream stream);

/* mehdg_dot for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * context, no allocation.  The partial sums (256 doubles, whatever n) live in
 * a file-scope device array that each GPU holds for the life of the process;
 * its address is looked up once per device (hipGetSymbolAddress) on the first
 * call with that device current.  Same kernel and the same host summation
 * order as mehdg_dot, so the result is identical.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race.  Synchronises the stream.  n < 0, a NULL output,
 * or NULL vectors with n > 0: MEHDG_EINVAL; no usable device: MEHDG_EHIP. */
mehdg_err mehdg_dot_noalloc(int64_t n, const double* x, const double* y, double* out, mehdg_stream stream);

/* ------------------------------------------------------------------------
 * Tetrahedral macro-elements (Sec. 3.1: K a tetrahedron resolved by eight
 * P_p sub-tetrahedra, continuous inside K; the paper's own discretisation).
 *
 * The submesh is the red refinement of K: four corner tetrahedra at the edge
 * midpoints and the inner octahedron split along the diagonal joining the
 * midpoints of reference edges 0-2 and 1-3.  Equispaced Lagrange nodes of
 * degree p on every sub-tetrahedron make the macro nodes the degree-2p
 * lattice of K.  Reference tetrahedron (0,0,0), e_x, e_y, e_z; a macro is its
 * affine image x = X0 + sum_i xi_i (X_i - X0).
 *   n  = (2p+1)(2p+2)(2p+3)/6, node a at xi = (i,j,k)/(2p), i+j+k <= 2p,
 *        i fastest, then j, then k;
 *   nf = (2p+1)(2p+2)/2 per face; face f is opposite vertex f, with vertices
 *        (P0,P1,P2) the other three in increasing order, node c at
 *        P0 + (i (P1-P0) + j (P2-P0))/(2p), i+j <= 2p, i fastest;
 *   v [m][5][n], q [m][5][3][n], vhat [m][4][5][nf];
 *   N_V = 5n, N_Q = 15n, N_VH = 20 nf.
 * Quadrature: the collapsed Gauss-Jacobi rule with p+1 points per direction
 * on every sub-tetrahedron, the matching rule on every face sub-triangle.
 * ------------------------------------------------------------------------ */
typedef struct mehdg_tet_ctx mehdg_tet_ctx;

/* Tetrahedral mesh.  Host memory, copied at create. */
typedef struct {
    int64_t n_macro;
    int32_t p;               /* 1..3 */
    int32_t pad_;
    const double* X;         /* [n_macro][4][3] vertex coordinates (non-degenerate) */
    const uint8_t* face_bc;  /* [n_macro][4] or NULL: 1 = isothermal no-slip wall (T_wall > 0 required) */
} mehdg_tet_mesh;

/* Sizes at degree p (n, nf, N_V, N_Q, N_VH); EINVAL for p outside 1..3. */
mehdg_err mehdg_tet_sizes(int32_t p, int64_t out[5]);

/* Builds the reference tables (host) and the per-macro geometry (J^-1,
 * |det J|, outward face normals, face areas).  EINVAL for a bad degree,
 * parameter set, wall flag or a degenerate macro; ENOMEM if device memory
 * runs out.  The parameters mean what they mean for mehdg_create. */
mehdg_err mehdg_tet_create(const mehdg_tet_mesh* mesh, const mehdg_params* params, mehdg_tet_ctx** ctx);
mehdg_err mehdg_tet_destroy(mehdg_tet_ctx* ctx);

/* Residual of every macro (Sec. 4.1 eq. s32a-c, time term of eq. C242):
 *   R_Q[k,j,a] = (q_kj, phi_a) + (v_k, d_j phi_a) - <vhat_k, phi_a n_j>,
 *   R_V[k,a]   = alpha_t (u_k(v) - u_k(v_old), phi_a) - (F_kj + G_kj, d_j phi_a)
 *                + <Fhat_k + Ghat_k, phi_a>,
 *   R_Vhat[f,k,c] = <Fhat_k + Ghat_k, psi_c>_f  (wall faces: rows 2..5 are
 *                <vhat_k (+ gamma/T_wall for k = 5), psi_c>_f, as for mehdg_assemble),
 * and entropy[m], the face entropy production sum over face points of
 * w ([[v]]^T Fhat - [[rho V.n]]).  q NULL: q is the weak gradient, the q that
 * makes R_Q vanish.  Device pointers, layouts above; asynchronous on
 * ``stream``.  A macro with a non-physical state (beta <= 0, rho or P not
 * positive) or a non-finite result gets NaN outputs and a status code
 * (mehdg_tet_status); EINVAL for a NULL argument, EHIP for a launch error. */
mehdg_err mehdg_tet_residual(mehdg_tet_ctx* ctx, const double* v, const double* vhat, const double* q,
                             const double* v_old, double* R_q, double* R_v, double* R_vhat,
                             double* entropy, mehdg_stream stream);

/* Jacobian-vector product of mehdg_tet_residual at the state (q, v, vhat),
 * with the pseudo-time term alpha_ps (A0 dv, w) added as in the assembled
 * Jacobian of the hexahedral path (Sec. 6.2 eq. R1):
 *   [JR_q; JR_v; JR_vhat] = J [dq; dv; dvhat].
 * q NULL: q is the weak gradient of (v, vhat).  dq NULL: dq is the weak
 * gradient of (dv, dvhat), the derivative of the residual computed with
 * q = NULL (JR_q then vanishes up to rounding).  The pointwise physics is
 * differentiated exactly (dual numbers).  Layouts as for mehdg_tet_residual;
 * device pointers; asynchronous on ``stream``; flagged macros get NaN
 * outputs and a status code; EINVAL for a NULL required argument. */
mehdg_err mehdg_tet_jvp(mehdg_tet_ctx* ctx, const double* v, const double* vhat, const double* q,
                        const double* dv, const double* dvhat, const double* dq, double* JR_q, double* JR_v,
                        double* JR_vhat, mehdg_stream stream);

/* Local work of one Newton step on tetrahedral macros (Sec. 6.2 eq. R1-R6),
 * with q the weak gradient of (v, vhat) (so R_Q = 0 up to rounding):
 *
 * mehdg_tet_assemble writes the residual (as mehdg_tet_residual with q NULL)
 * and the bordered matrix [[S, -Y, r_V], [X, A', r_hat]] of every macro into
 * the context.  With R_Q = 0 that matrix is [J_r | -R], J_r the reduced
 * Jacobian of (R_V, R_Vhat) in (v, vhat) through the weak gradient
 * (S = A_vv - A_vq A_qq^-1 A_qv, -Y = A_vvh - A_vq A_qq^-1 A_qvh,
 * X = A_hv - A_hq A_qq^-1 A_qv, A' = A_hh - A_hq A_qq^-1 A_qvh; the
 * pseudo-time term alpha_ps (A0 dv, w) is in S), built column by column with
 * the JVP kernel.  The first call allocates the workspace, about
 * (N_V + N_VH)^2 doubles per macro (7.7 MB at p = 3); ENOMEM if it does not fit.
 *
 * mehdg_tet_condense factors it (pivoted LU of S) and writes
 * Ahat = A' + X S^-1 Y [n_macro][N_VH][N_VH] and bhat = r_hat - X S^-1 r_V
 * [n_macro][N_VH] (eq. R5a-b); ESTATE before an assemble.
 *
 * mehdg_tet_recover, after a condense (else ESTATE): dV = S^-1 (r_V + Y dVhat)
 * and dQ = A_qq^-1 (-R_Q - A_qv dV - A_qvh dVhat) (eq. R2, R6) for a trace
 * update dvhat [n_macro][4][5][nf]; dv [n_macro][5][n], dq [n_macro][5][3][n];
 * R_q as returned by the assemble.
 *
 * Device pointers, asynchronous on ``stream``; flagged macros (non-physical
 * state, non-finite values, zero pivot: mehdg_tet_status) get NaN outputs. */
mehdg_err mehdg_tet_assemble(mehdg_tet_ctx* ctx, const double* v, const double* vhat, const double* v_old,
                             double* R_q, double* R_v, double* R_vhat, double* entropy, mehdg_stream stream);
/* Reduced vector-Jacobian product at the state of the last mehdg_tet_assemble,
 * before mehdg_tet_condense (else ESTATE): [g_v; g_vhat] = J_r^T [w_v; w_vhat],
 * the gradient of w_v.R_V + w_vhat.R_Vhat in (v, vhat) with q the weak
 * gradient (the transpose of mehdg_tet_jvp with dq = NULL, pseudo-time term
 * included), read from the assembled bordered matrices.  w_v, g_v
 * [n_macro][5][n]; w_vhat, g_vhat [n_macro][4][5][nf]; device pointers;
 * asynchronous on ``stream``. */
mehdg_err mehdg_tet_vjp(mehdg_tet_ctx* ctx, const double* w_v, const double* w_vhat, double* g_v,
                        double* g_vhat, mehdg_stream stream);
mehdg_err mehdg_tet_condense(mehdg_tet_ctx* ctx, double* Ahat, double* bhat, mehdg_stream stream);
/* The stored tetrahedral condensation applied to a new right-hand side, as
 * mehdg_condense_rhs: r_V [n_macro][N_V] and r_hat [n_macro][N_VH] (NULL:
 * zero) in place of -R_V and -R_Vhat; writes bhat = r_hat - X S^-1 r_V and
 * makes the next mehdg_tet_recover return dV = S^-1 (r_V + Y dVhat).  After
 * mehdg_tet_condense (else ESTATE); the factors are kept. */
mehdg_err mehdg_tet_condense_rhs(mehdg_tet_ctx* ctx, const double* r_v, const double* r_hat, double* bhat,
                                 mehdg_stream stream);
mehdg_err mehdg_tet_recover(mehdg_tet_ctx* ctx, const double* R_q, const double* dvhat, double* dv,
                            double* dq, mehdg_stream stream);

/* Per-macro status of the calls since the last mehdg_tet_residual,
 * mehdg_tet_jvp or mehdg_tet_assemble (0, ENONPHYSICAL, ENONFINITE, or
 * ESINGULAR from a condense) into host memory; returns the first non-zero
 * code or OK.
 * Synchronises the stream. */
mehdg_err mehdg_tet_status(mehdg_tet_ctx* ctx, int32_t* status, mehdg_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* MEHDG_H */
