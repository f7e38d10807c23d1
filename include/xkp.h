/*
 * xkp.h -- C ABI of the MI355X (gfx950) cross-matrix Krylov projection library (libxkp.so).
 *
 * The library solves, for many images at one timestep, the implicit linearised log-density
 * Fokker-Planck systems A u = b of Lau, Na and Wan, "Efficient Score Pre-computation for
 * Diffusion Models via Cross-Matrix Krylov Projection" (arXiv 2511.17634):
 *   - the operator A is the five-point stencil of Section 2.3 (coefficients C_diag, C_north,
 *     C_south, C_east, C_west built from the lagged log-density m~ and the drift f), kept
 *     matrix-free;
 *   - xkp_seed_build solves a seed system by restarted GMRES and keeps the orthonormal basis of
 *     its first cycle, which spans the Krylov subspace K_k(A_seed, r0) (Section 3, Phase 1);
 *   - xkp_target_project_solve projects each target system onto that basis, solves the small
 *     k x k system and polishes the result with GMRES to the tolerance (Section 3, Phase 2);
 *   - xkp_residual returns ||b - A x||_2 / ||b||_2 in FP64 for any batch of systems.
 *
 * Conventions shared by every call
 *   - Grids are square: H x H, n = H*H, h = 1/H (Section 2.3 takes dx = dy = h).  Unknown p of
 *     a grid vector is p = i*H + j, i the x (width) index, j the y (height) index: the y index
 *     runs fastest, as in the paper's vector definition.  Values outside the grid are zero.
 *   - Every array pointer inside a descriptor, and every descriptor array passed to a batched
 *     call, is a DEVICE pointer owned by the caller; the library never frees them.  Scalars and
 *     xkp_params are host values.
 *   - Calls are asynchronous on the context's stream: they return after enqueuing work and can
 *     be captured into a HIP graph.  Argument errors detectable on the host (null pointers,
 *     sizes beyond the context limits) are returned synchronously before anything is enqueued.
 *     Per-system outcomes (convergence, breakdown, singular projection, bad descriptor) are
 *     written to the caller's device xkp_info array.
 *   - A context is used from one host thread at a time.  Calls on one context run in stream
 *     order; they share the context's workspace, so two contexts are needed for overlap.
 *   - All solver arithmetic is FP64 in XKP_FP64 mode.  In XKP_MIXED mode the operator inside
 *     the targets' GMRES cycles is applied in FP32 (FP32 coefficients, operands rounded to FP32,
 *     FP32 row sums) and their (discarded) Krylov basis is stored in FP32 (each vector rounded
 *     once when formed); the Gram-Schmidt products, rotations and updates run in FP64 on those
 *     values, every restart recomputes the true residual b - A x with the FP64 operator, and
 *     convergence is judged on it, so results meet params->tol in FP64.  A cycle ends early
 *     once its residual estimate has fallen by 1e-5 (the reduction the FP32 operator can
 *     deliver).  Seeds keep the FP64 operator (a seed is one system per timestep on the
 *     chain's critical path, where the cycle limit would cost it restarts) and write a BF16
 *     copy of the kept basis; the target-Galerkin projection forms A'V_k with the FP32
 *     operator, rounds it to BF16 and contracts V_k^T (A'V_k) on BF16 matrix cores with FP32
 *     accumulation; V_k^T r_base, the k x k solve and x0 = x_base + V_k alpha stay FP64.
 */
#ifndef XKP_H
#define XKP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XKP_OK = 0,            /* success / system converged                                   */
    XKP_EINVAL = 1,        /* invalid argument or descriptor; per system also data that
                              are not finite (NaN or Inf in m~, f, b or x0)               */
    XKP_ENOMEM = 2,        /* device allocation failed                                    */
    XKP_EDEVICE = 3,       /* HIP runtime error                                           */
    XKP_ENOCONV = 4,       /* GMRES hit max_restarts; x holds the last iterate            */
    XKP_ESINGULAR = 5,     /* projected k x k system had a zero pivot; x0 = x_base used   */
    XKP_EUNSUPPORTED = 6   /* valid but not supported by this library (e.g. m > 64)      */
} xkp_status;

typedef enum { XKP_FP64 = 0, XKP_MIXED = 1 } xkp_precision;

/* How a target is projected onto the seed basis V_k (Section 3, Phase 2). */
typedef enum {
    XKP_PROJ_TARGET_GALERKIN = 0, /* A_p = V_k^T A' V_k, the target's own operator          */
    XKP_PROJ_SEED_GALERKIN = 1,   /* A_p = H_k = V_k^T A_seed V_k, the seed operator the
                                     paper substitutes to avoid forming V^T A_i V per target */
    XKP_PROJ_SEED_LSQ = 2,        /* alpha minimises ||V_{k+1}^T r_base - Hbar_k alpha||_2    */
    XKP_PROJ_NONE = 3             /* no projection: plain GMRES from x_base                  */
} xkp_proj_mode;

/*
 * Gram-Schmidt passes per Arnoldi step.  A basis that is kept (the first cycle of a seed,
 * Section 3, Phase 1) must be orthonormal to working precision for the projection, which two
 * modified Gram-Schmidt passes give; a GMRES cycle whose basis is discarded (target polish, plain
 * GMRES, the seed's later cycles) converges as well with one pass, GMRES with modified
 * Gram-Schmidt being backward stable (Paige, Rozloznik and Strakos, SIAM J. Matrix Anal. Appl.
 * 28, 2006), at half the basis traffic and half the sequential reductions.  In a seed call whose
 * largest system (params->batch_max_n, or the context's max_n) has at most 4096 unknowns the
 * kept cycle gets its two passes by delayed classical Gram-Schmidt with re-orthogonalisation
 * (DCGS2, Bielich et al., Parallel Computing 112, 2022): the same basis and Hessenberg matrix to
 * rounding, with one workgroup reduction per Arnoldi step instead of one per basis column;
 * larger calls use two modified Gram-Schmidt passes.
 */
/* Discarded cycles whose basis fits the registers of a workgroup (grids of at most 4096
 * unknowns: up to 6 steps per cycle at 64x64 with 8-wave workgroups, 9 with 4-wave ones; up to 8
 * / 15 at 32x32) keep it there and orthogonalise by two classical Gram-Schmidt passes, each one
 * workgroup reduction for all the step's inner products (CGS2, an orthonormal basis to working
 * precision like two modified passes); longer cycles use the single modified pass above. */
typedef enum {
    XKP_REORTH_AUTO = 0,   /* two passes while a basis is kept, one pass elsewhere          */
    XKP_REORTH_ALWAYS = 1  /* two passes in every Arnoldi step                              */
} xkp_reorth;

/* One linear system of one image channel at one timestep (device-resident array element). */
typedef struct {
    int32_t H;            /* grid side; n = H*H unknowns                                    */
    int32_t basis_id;     /* targets: index into the bases array of the seed basis to use  */
    double dt;            /* time step (1/T)                                                 */
    double g;             /* diffusion coefficient g                                         */
    const double *mt;     /* [n] lagged log-density m~ defining the coefficients            */
    const double *fx;     /* [n] drift x component, or NULL for f = 0                       */
    const double *fy;     /* [n] drift y component, or NULL for f = 0                       */
    const double *b;      /* [n] right-hand side                                            */
    const double *x0;     /* [n] initial guess (seed) / base vector x_base (target), or NULL */
    double *x;            /* [n] solution (output); may alias x0                            */
} xkp_system;

typedef struct {
    int32_t m;            /* GMRES restart length = seed basis dimension, 1 <= m <= 64      */
    int32_t max_restarts; /* restarts allowed after the first cycle                         */
    double tol;           /* converged when ||b - A x||_2 <= tol ||b||_2 (FP64, true residual) */
    int32_t precision;    /* xkp_precision                                                  */
    int32_t mode;         /* xkp_proj_mode (targets)                                        */
    int32_t batch_max_n;  /* largest n among this call's systems, or 0 for the context's
                             max_n; smaller values select leaner kernels.  A system with more
                             unknowns than this gets status XKP_EINVAL.                    */
    int32_t polish_m;     /* restart length of every GMRES cycle whose basis is not kept:
                             the polish, plain GMRES and a seed's cycles after its kept first
                             one; 1..64, or 0 for m.  The seed basis dimension stays m.     */
    int32_t reorth;       /* xkp_reorth                                                     */
} xkp_params;

/* Per-system outcome, device-resident. */
typedef struct {
    int32_t status;       /* xkp_status of this system                                      */
    int32_t iters;        /* Arnoldi steps (operator applications in the Krylov loop)        */
    int32_t restarts;     /* restarts after the first cycle                                 */
    int32_t basis_dim;    /* seed: k kept in the basis; target: k used by the projection    */
    double res_est;       /* last Givens residual estimate, relative                        */
    double res_true;      /* final ||b - A x||_2 / ||b||_2 computed in FP64                  */
    double guess_res;     /* target: relative residual of the starting guess x0            */
    int32_t guess_source; /* target: 0 x_base, 1 projection onto the seed basis, 2 learned,
                             3 projection corrected by the learned prediction; seed: 0, or 4
                             when a spread-out solve gave up and one workgroup solved it again */
    int32_t pad;
} xkp_info;

/*
 * Seed basis buffer, caller-allocated device memory of xkp_basis_bytes(n, m) bytes, 256-byte
 * aligned.  Layout (all offsets in bytes from the start):
 *   [0, 256)         xkp_basis_header
 *   [256, ...)       V: (m+1) columns of ldv = roundup(n + 1, 8) doubles, column c at
 *                    256 + 8*c*ldv: the orthonormal Arnoldi vectors v_0..v_k of the seed's
 *                    first GMRES cycle in rows 0..n-1, zeros in rows n..ldv-1 (column k is
 *                    zero after a breakdown)
 *   then             Hbar: m columns of (m+1) doubles (column-major, leading dimension m+1),
 *                    the unrotated Hessenberg matrix of that cycle
 *   then             Vb: (m+1) columns of ldv bf16 values (XKP_MIXED copies of V, 256-aligned;
 *                    header field bf16 = 1 when written).  A mixed-precision target-Galerkin
 *                    projection on a basis without it gives that target XKP_EINVAL.
 * An accumulated basis (xkp_basis_accumulate) has the same layout with k orthonormal columns,
 * no Hessenberg matrix and kind = XKP_BASIS_ACCUMULATED.
 */
typedef enum {
    XKP_BASIS_ARNOLDI = 0,     /* a seed's first GMRES cycle: V_{k+1} and Hbar_k             */
    XKP_BASIS_ACCUMULATED = 1  /* orthonormal columns gathered from several seeds, no Hbar   */
} xkp_basis_kind;

typedef struct {
    int32_t n, m, k, status;
    double beta;          /* ||r0|| of the seed's first cycle                               */
    int32_t ldv;          /* leading dimension of V in doubles                              */
    int32_t bf16;         /* 1 if the BF16 copy Vb was written (seed built with XKP_MIXED)  */
    int32_t kind;         /* xkp_basis_kind                                                 */
    int32_t pad[55];
} xkp_basis_header;

typedef struct xkp_ctx xkp_ctx;

/* Create a context on `device` bound to `hip_stream` (a hipStream_t, or NULL for the null
 * stream).  Workspace for up to `max_batch` concurrently solved systems of at most max_n
 * unknowns and restart length max_m is allocated here; no later solve call allocates (the
 * setup calls xkp_ctx_set_seed_width and xkp_ctx_set_projection_split allocate their own
 * buffers when first switched on). */
xkp_status xkp_ctx_create(xkp_ctx **ctx, int device, void *hip_stream, int32_t max_n,
                          int32_t max_m, int32_t max_batch);
xkp_status xkp_ctx_destroy(xkp_ctx *ctx);

/* Launch shape of the context's later solve calls: workgroups of `waves` wave64s (8, 16 or 4;
 * 16 needs max_n <= 16384, 4 needs max_n <= 4096) and up to wg_per_cu workgroups per compute
 * unit.  Results do not depend on it (up to rounding: the row-to-thread mapping and the
 * reduction trees change).  XKP_EUNSUPPORTED if no kernel variant of that size covers max_n. */
xkp_status xkp_ctx_set_launch(xkp_ctx *ctx, int32_t waves, int32_t wg_per_cu);

/*
 * Seed solves spread over several workgroups (Section 3, Phase 1: the seed of a timestep gates
 * every target of that timestep, so its single solve is the chain's critical path).  With
 * rows_per_thread = 1, later xkp_seed_build calls of this context (of at most 64 seeds, default
 * Gram-Schmidt setting) solve each seed with ceil(n / 256) workgroups of 256 threads, each owning
 * 256 consecutive rows and keeping its rows of the cycle's basis in LDS; a seed's workgroups share
 * one XCD when there are at most 32 of them.  The operator's neighbour rows of adjacent blocks
 * are exchanged through device memory, and each Arnoldi step takes two classical Gram-Schmidt
 * passes whose inner products are summed over the blocks in a fixed order (an orthonormal basis
 * to working precision, as the two modified passes of the one-workgroup solve give); results are
 * those of the one-workgroup solve to rounding.  The exchange areas are uncached device memory
 * (workgroups of one seed may sit on different XCDs), taken from a per-device pool that keeps
 * them until the process ends.  The workgroups of a seed must be resident together: each wait
 * for the others gives up after a time limit (100 ms unless xkp_ctx_set_seed_wait says
 * otherwise; no hang), and a seed whose solve gave up is solved again in the same call by one
 * workgroup (info.guess_source = 4), so every seed ends with the one-workgroup solve's result.  Requires grids of at most 128 x 128 and
 * max_m <= 64 (XKP_EUNSUPPORTED otherwise); allocates the exchange buffers (a setup call, like
 * xkp_ctx_create).  0 returns to one workgroup per seed.
 */
xkp_status xkp_ctx_set_seed_width(xkp_ctx *ctx, int32_t rows_per_thread);

/*
 * The time after which a wait of a spread-out seed (xkp_ctx_set_seed_width) gives up, in
 * microseconds (0 .. 60e6; default 1e5).  0 gives up at the first wait whose data has not yet
 * arrived: the seed is then solved again by one workgroup in the same call (info.guess_source
 * = 4).  XKP_EINVAL outside the range.
 */
xkp_status xkp_ctx_set_seed_wait(xkp_ctx *ctx, int64_t microseconds);

/*
 * Target projection in launches of its own (Section 3, Phase 2).  With max_tiles >= 0, later
 * xkp_target_project_solve calls of this context (projection modes other than XKP_PROJ_NONE)
 * first project every target over the whole chip, then polish in the solve launch:
 *   1. each target's rows are split into at most T row tiles of a multiple of 256 rows
 *      (T = max_tiles, or when 0 about as many tiles in all as the chip runs Gram workgroups
 *      at once, two per compute unit; never more than one tile per 256 rows nor more tiles than
 *      the context's partial slots, 2048 at most); one workgroup per tile forms its rows of
 *      A' V_k and its share of V_k^T [A' V_k | r_base] (FP64 matrix cores, or BF16 ones for the
 *      mixed-precision Gram matrix, z in FP64), and the target's last tile adds the shares in
 *      tile order and solves the small system (LU with partial pivoting, or Givens rotations for
 *      XKP_PROJ_SEED_LSQ)
 *   2. x0 = x_base + V_k alpha by tiles
 *   3. the solve launch polishes from x0.
 * Batches of more than the context's max_batch targets project inside the solve launch.
 * Statuses, basis_dim, guess_res and the iterate are those of the in-launch projection up to
 * rounding (the order of the row sums differs).  Calls stay free of allocation and host
 * synchronisation (graph-capturable).  The first call with max_tiles >= 0 allocates the partial
 * slots (at most 2048 of (max_m + 1)^2 doubles, in uncached device memory, since a target's
 * tiles on different XCDs exchange them within one launch; like the spread-out seeds' exchange
 * areas they return to a per-device pool on xkp_ctx_destroy and are never freed while the
 * process runs) and per-target buffers (a setup call);
 * max_tiles = -1 returns to the projection inside the solve launch (the default).  XKP_EINVAL
 * for max_tiles < -1.
 */
xkp_status xkp_ctx_set_projection_split(xkp_ctx *ctx, int32_t max_tiles);

/*
 * Phase timing of target calls.  With on = 1, each later xkp_target_project_solve of this
 * context records three HIP events on its stream: before the projection launches, before the
 * solve launch, after it (the first two coincide when the projection runs inside the solve
 * launch).  The first call with on = 1 creates the events (a setup call).  Recording events
 * stays graph-capturable but adds event nodes: keep timing off in captured chains.
 * xkp_ctx_last_timing waits for the last recorded call and returns its projection launches'
 * and solve launch's durations in milliseconds; XKP_EINVAL if timing is off or no call has
 * been recorded since it was switched on.
 */
xkp_status xkp_ctx_set_timing(xkp_ctx *ctx, int32_t on);
xkp_status xkp_ctx_last_timing(xkp_ctx *ctx, float *ms_projection, float *ms_solve);

/* Size in bytes of one seed basis buffer for n unknowns and restart length m. */
size_t xkp_basis_bytes(int32_t n, int32_t m);

/*
 * Batches.  Each of xkp_seed_build and xkp_target_project_solve is ONE persistent kernel launch
 * over its whole batch.  Systems of different sizes may share a batch (params->batch_max_n, or
 * the context's max_n, bounds them); each runs the code path compiled for its own size.
 * Workgroups take systems from a work queue in array order, so ordering a batch largest first
 * balances it (longest-processing-time first).  Results do not depend on the order or on which
 * workgroup solved a system.  Calls enqueue work on the context's stream without host
 * synchronisation and allocate nothing, so a sequence of them can be captured in a HIP graph
 * and replayed; calls on one context must not run concurrently (they share its workspace and
 * work-queue counters).
 */

/*
 * Phase 1 (Section 3): solve each of the n_seeds seed systems by restarted GMRES(m) from
 * seeds[i].x0 (NULL: zero) to params->tol, write the solution to seeds[i].x and the first
 * cycle's basis V, Hessenberg matrix and header into the buffer bases[i].
 *   seeds: device array of n_seeds descriptors; bases: device array of n_seeds device
 *   pointers to buffers of xkp_basis_bytes(n, params->m); infos: device array of n_seeds.
 * In XKP_MIXED mode a BF16 copy of V is also written (the seed itself is solved in FP64).
 */
xkp_status xkp_seed_build(xkp_ctx *ctx, int32_t n_seeds, const xkp_system *seeds,
                          void *const *bases, const xkp_params *params, xkp_info *infos);

/*
 * Phase 2 (Section 3): for each target i, r_base = b - A' x_base (x_base = targets[i].x0,
 * NULL: zero); alpha solves the projected system selected by params->mode on the basis
 * bases[targets[i].basis_id]; x0 = x_base + V_k alpha; then GMRES(m) from x0 to params->tol.
 * The result goes to targets[i].x.  Mode XKP_PROJ_NONE skips the projection (plain GMRES from
 * x_base) and ignores `bases` (may be NULL).  A basis with a different n than the target, or
 * a basis_id outside [0, n_bases), sets that target's status to XKP_EINVAL; so does a seed mode
 * (XKP_PROJ_SEED_GALERKIN, XKP_PROJ_SEED_LSQ) on an accumulated basis, which has no Hessenberg
 * matrix.
 */
xkp_status xkp_target_project_solve(xkp_ctx *ctx, int32_t n_targets, const xkp_system *targets,
                                    int32_t n_bases, const void *const *bases,
                                    const xkp_params *params, xkp_info *infos);

/*
 * Target solve starting from a learned guess.  alpha[i*alpha_ld + r], r <= k (FP32 device array,
 * e.g. xkp_cnn_forward's output; alpha_ld >= k+1) is the network's prediction of target i's
 * residual coordinates zeta = Hbar_k (V_k^T x*) / beta on its seed basis
 * bases[targets[i].basis_id] (Hbar_k and beta = ||r0|| of the seed's kept cycle, see
 * xkp_basis_coeffs kind 1).  The guess is x0_L = x_base + V_k a with
 * a = argmin || beta * alpha_scale * zeta - Hbar_k a || (Givens least squares).  If
 * ||b - A x0_L|| / ||b|| (FP64) <= gate the polish starts from x0_L (info.guess_source = 2);
 * otherwise the target falls back to xkp_target_project_solve's path for params->mode
 * (projection then polish, or plain GMRES from x_base for XKP_PROJ_NONE); so does a target on
 * an accumulated basis (no Hessenberg matrix).  One persistent launch, as
 * xkp_target_project_solve.
 */
xkp_status xkp_learned_solve(xkp_ctx *ctx, int32_t n_targets, const xkp_system *targets,
                             int32_t n_bases, const void *const *bases, const xkp_params *params,
                             const float *alpha, int32_t alpha_ld, double alpha_scale,
                             double gate, xkp_info *infos);

/*
 * Learned correction of the projection: each target is first projected as in xkp_target_project_solve (params->mode, which must not be
 * XKP_PROJ_NONE: XKP_EINVAL), giving x0_P = x_base + V_k a_P; the prediction alpha + i*alpha_ld
 * (k+1 FP32 values) is then read as a correction of the projected guess's residual
 * coordinates: x0_C = x0_P + V_k d with d = argmin || beta * alpha_scale * alpha - Hbar_k d ||
 * (Givens least squares; train it on basis coordinates of x* minus those of x0_P, kind 1 of
 * xkp_basis_coeffs).  The polish starts from x0_C (info.guess_source = 3) when its FP64
 * relative residual is <= gate and below x0_P's, else from x0_P (guess_source 1): the
 * correction never starts the polish from a worse guess than the projection.  A projected
 * system that is singular (XKP_ESINGULAR) keeps x_base uncorrected.  One persistent launch.
 */
xkp_status xkp_learned_correction_solve(xkp_ctx *ctx, int32_t n_targets,
                                        const xkp_system *targets, int32_t n_bases,
                                        const void *const *bases, const xkp_params *params,
                                        const float *alpha, int32_t alpha_ld, double alpha_scale,
                                        double gate, xkp_info *infos);

/* kind 0: alpha[i][c] = v_c . x_i (FP64) for c < k of the basis bases[systems[i].basis_id], 0
 * for k <= c < m_out (1 <= m_out <= 64): the coordinates of systems[i].x in the seed subspace.
 * kind 1: alpha[i][r] = (Hbar_k (V_k^T x_i))_r / beta for r <= k, 0 past (m_out <= 65): the
 * residual coordinates a learned guess predicts (xkp_learned_solve; an Arnoldi basis only).
 * A descriptor or basis that does not fit writes NaN. */
xkp_status xkp_basis_coeffs(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems,
                            int32_t n_bases, const void *const *bases, int32_t m_out,
                            int32_t kind, double *alpha);

/* rel_res[i] = ||b_i - A_i x_i||_2 / ||b_i||_2 in FP64 (||r||_2 when b_i = 0), for a device
 * array of n_sys descriptors; rel_res is a device array of n_sys doubles. */
xkp_status xkp_residual(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems, double *rel_res);

/* Right-hand side of each system at the new timestep (Section 2.3):
 *   b = m^{n-1}/dt - [(f_x)_{i+1,j} - (f_x)_{i-1,j} + (f_y)_{i,j+1} - (f_y)_{i,j-1}] / (2h)
 * with m^{n-1} = systems[i].mt (one linearisation pass, m~ = m^{n-1}), written to the memory
 * that systems[i].b points to (the one call that writes through b). */
xkp_status xkp_build_rhs(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems);

/* y_i = A_i u_i for a batch (the stencil operator alone): u = systems[i].x0, y = systems[i].x. */
xkp_status xkp_apply(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems);

/*
 * Learned starting guess: a small network maps a target's initial image (64 x 64, FP64, index
 * [i][j] = unknown p = 64 i + j) and the timestep index n to k coefficients alpha_L in the seed
 * subspace (x0_L = x_base + V_k alpha_L, see xkp_learned_solve).  Layers: 2x2 average pool to
 * 32 x 32; three 3x3 stride-2 padding-1 convolutions (1 -> 16 -> 32 -> 64 channels), each with
 * bias and GELU; mean over the 4 x 4 positions concatenated with a 32-wide sinusoidal embedding
 * of n (sin / cos of n * 10000^(-i/16), i < 16); linear 96 -> k.  Parameters are one FP32
 * device array of xkp_cnn_param_count(k) values: conv1.W[16][9], conv1.b[16], conv2.W[32][144],
 * conv2.b[32], conv3.W[64][288], conv3.b[64], lin.W[k][96], lin.b[k] (weight column
 * ci*9 + ky*3 + kx).  The convolutions run on BF16 matrix cores with FP32 accumulation; the rest
 * is FP32.  `work` is a caller-allocated device buffer of xkp_cnn_workspace_bytes(batch, k).
 * All arrays are device arrays; 1 <= k <= 64, batch >= 1.
 */
size_t xkp_cnn_param_count(int32_t k);
size_t xkp_cnn_workspace_bytes(int32_t batch, int32_t k);

/* alpha[b][0..k) (FP32) for sample b = image images + 4096 * image_idx[b] (image_idx NULL:
 * image b; FP64 images) at timestep steps[b]. */
xkp_status xkp_cnn_forward(xkp_ctx *ctx, int32_t batch, int32_t k, const float *params,
                           const double *images, const int32_t *image_idx, const int32_t *steps,
                           float *alpha, void *work);

/* Forward pass, then the mean squared error against the targets t[b][o] =
 * target_scale * target[target_idx[b] * target_ld + o] (FP64 rows; target_idx NULL: row b) into
 * *loss (one device float) and its gradient with respect to every parameter into grad
 * (param_count floats, overwritten).  alpha receives the forward outputs. */
xkp_status xkp_cnn_backward(xkp_ctx *ctx, int32_t batch, int32_t k, const float *params,
                            const double *images, const int32_t *image_idx, const int32_t *steps,
                            const double *target, int32_t target_ld, const int32_t *target_idx,
                            double target_scale, float *alpha, float *grad, float *loss,
                            void *work);

/* One Adam step on `count` FP32 parameters: m, v are the moment buffers (zero before step 1),
 * t >= 1 the step number (bias correction). */
xkp_status xkp_cnn_adam(xkp_ctx *ctx, int32_t count, float *params, const float *grad, float *m,
                        float *v, int32_t t, float lr, float beta1, float beta2, float eps);

/*
 * Krylov subspace accumulation over an image cycle (Section 3: the seed basis V^n of each
 * timestep is reused for the targets; Experiment 2: a new seed every 50 images expands the
 * subspace, capped at a vectors).  For j = 0..n_src-1, out_bases[j] receives the orthonormal
 * basis gathered from the first-cycle bases src_bases[0..j], in that order: each source's
 * columns v_0, v_1, ... (its Krylov order) are orthogonalised by two passes of modified
 * Gram-Schmidt against the columns gathered so far and appended, normalised, when the norm
 * left exceeds 1e-8; at most per_source columns are appended per source and cap in total.
 *   n:          unknowns of every source (grid H x H); sources with another n, a missing basis
 *               or an accumulated kind give out_k[j] = -1 and leave out_bases[j] unset
 *   src_bases:  device array of n_src pointers to seed bases (xkp_seed_build results)
 *   out_bases:  device array of n_src pointers to caller buffers of xkp_basis_bytes(n, cap)
 *               bytes; header n, m = cap, k = columns gathered, ldv, bf16 = 1 (the BF16 copy is
 *               written), kind = XKP_BASIS_ACCUMULATED.  Only the target-Galerkin projection
 *               (FP64 or mixed, with params->m = cap) and xkp_basis_coeffs kind 0 accept it.
 *   out_k:      device array of n_src int32 (columns gathered), or NULL
 * Returns XKP_EINVAL for null arrays, n_src < 1, per_source < 1, cap < 1, cap above the
 * context's max_m or n above its max_n.  Enqueued on the context's stream; out_j is computed
 * from scratch by workgroup j (the sources are read, never written).
 */
xkp_status xkp_basis_accumulate(xkp_ctx *ctx, int32_t n, int32_t n_src,
                                const void *const *src_bases, void *const *out_bases,
                                int32_t per_source, int32_t cap, int32_t *out_k);

/*
 * Score and probability-flow embedding (the step after the solves).  For each system i and grid
 * point p = i_x*H + j, with h = 1/H and the log-density m taken as zero outside the grid:
 *   s_x = (m[i_x+1, j] - m[i_x-1, j]) / (2h),   s_y = (m[i_x, j+1] - m[i_x, j-1]) / (2h)
 * (Section 2.3's central difference of the solution; the 2h divisor is the one of the PDE's
 * discrete gradient), and one explicit step of the probability-flow ODE that embeds the score
 * into the image (Section 4, x^n = x^{n-1} + (f - g^2/2 grad m^{n-1}) dt), applied per grid point
 * to a two-component displacement:  d_x += (f_x - g^2/2 s_x) dt,  d_y += (f_y - g^2/2 s_y) dt.
 *   field:   XKP_FIELD_MT takes m = systems[i].mt (m^{n-1}, the state before the step's solve:
 *            the embedding's argument), XKP_FIELD_X takes m = systems[i].x (the solution m^n)
 *   score:   device array of n_sys pointers to 2n doubles (s_x then s_y), or NULL; a NULL entry
 *            skips that system's score
 *   disp:    device array of n_sys pointers to 2n doubles updated in place, or NULL / NULL entry
 * g, dt, fx, fy (NULL: 0) come from the descriptor.  A descriptor with H < 1, H*H above the
 * context's max_n, dt <= 0 or a NULL field is skipped.  n_sys <= 65535.  One launch, on the
 * context's stream; 16-byte aligned outputs of even-sided grids take the faster paired path.
 */
typedef enum { XKP_FIELD_MT = 0, XKP_FIELD_X = 1 } xkp_field;

xkp_status xkp_score_flow(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems, int32_t field,
                          double *const *score, double *const *disp);

/*
 * Clustered seed selection (the paper's remedy for diverse datasets: one seed per group of
 * similar images).  k-means on block-mean features: each image (H x H, p = i*H + j) averaged
 * over pool x pool blocks; farthest-first start (centroid 0 = image 0, centroid k = the image
 * farthest, in squared distance, from its nearest chosen centroid, lowest index on ties); Lloyd
 * iterations (nearest centroid, lowest cluster on ties; centroids = member means, an empty
 * cluster keeps its centroid) until no assignment changes or max_iters assignments; a final
 * assignment; the seed of cluster c is its member nearest to centroid c (lowest index on ties),
 * -1 for an empty cluster.
 *   images:  device, n_img x H x H doubles (the initial log-densities m^0)
 *   assign:  device, n_img int32 (cluster of each image);  seeds: device, K int32
 *   iters:   host int32, assignments made (may be NULL)
 * Requires 1 <= K <= min(64, n_img), pool >= 1 dividing H, max_iters >= 1, H*H <= the
 * context's max_n.  Host-synchronous (it reads distances back between steps) and allocates its
 * temporary device memory (features, centroids, distances), freed before it returns: not
 * capturable.  Distances are summed in a fixed order, so results do not depend on scheduling.
 */
xkp_status xkp_cluster_seeds(xkp_ctx *ctx, int32_t n_img, int32_t H, const double *images,
                             int32_t pool, int32_t K, int32_t max_iters, int32_t *assign,
                             int32_t *seeds, int32_t *iters);

/* Outcome of xkp_autotune. */
typedef struct {
    int32_t polish_m;     /* fastest restart length of the polish (for params->polish_m)    */
    int32_t wg_per_cu;    /* fastest workgroups per compute unit (now set in the context)    */
    float ms_best;        /* time of one call with the chosen values, milliseconds           */
    float ms_default;     /* time with polish_m = m, 8-wave workgroups, the most per CU     */
    int32_t n_tried;      /* candidates timed                                               */
    int32_t waves;        /* fastest workgroup size in wave64s (now set in the context)     */
    int32_t seed_rows;    /* xkp_autotune_seeds: 1 if spreading each seed over several
                             workgroups was chosen (xkp_ctx_set_seed_width), else 0           */
    int32_t split;        /* xkp_autotune: the tile cap of the projection in launches of its
                             own if that was chosen (xkp_ctx_set_projection_split, now set in
                             the context), -1 for the projection inside the solve launch    */
} xkp_tuning;

/*
 * Launch autotuner for target calls: times xkp_target_project_solve on the given batch (one
 * representative timestep) for each kernel variant covering the batch (workgroups of 8, 16 or 4
 * wave64s), each candidate restart length of the polish (6, 8, 9, then m/4 (at least 8), m/2, 3m/4
 * and m, at most m; the short ones let the cycle's basis stay in registers) and each
 * workgroup count per compute unit the kernels can hold (1..occupancy), two timed calls each
 * after one untimed call, and keeps the fastest candidate whose every target converged.  For
 * projected batches of at most max_batch targets every candidate is timed twice: with the
 * projection inside the solve launch and in launches of its own (xkp_ctx_set_projection_split,
 * with the context's tile cap if one was set, else 0).  The chosen variant, workgroup count
 * and projection placement are stored in the context and apply to its later seed and target
 * calls; the chosen restart length is returned for the caller's params.
 * Side effects: targets[i].x and infos hold the last candidate's results.  Unlike the other
 * calls this one synchronises the stream (it reads timings and statuses back), so it must not
 * be captured in a graph.  Returns XKP_ENOCONV if no candidate converged everywhere.
 */
xkp_status xkp_autotune(xkp_ctx *ctx, int32_t n_targets, const xkp_system *targets,
                        int32_t n_bases, const void *const *bases, const xkp_params *params,
                        xkp_info *infos, xkp_tuning *out);

/*
 * Launch autotuner for seed calls: times xkp_seed_build on the given seeds (one representative
 * timestep) for each kernel variant covering them and each workgroup count per compute unit,
 * then each seed spread over several workgroups (xkp_ctx_set_seed_width 1, where that gives a
 * seed at least two workgroups), five timed calls each after one
 * untimed call, and keeps the fastest candidate whose every seed converged; the choice is stored
 * in the context (meant for a context
 * that serves seed calls only: a seed is one workgroup on the chain's critical path, whose best
 * workgroup size can differ from the targets').  out->polish_m is params->m.
 * Side effects: the bases, seeds[i].x and infos hold the last candidate's results.  Synchronises
 * the stream; must not be captured.  Returns XKP_ENOCONV if no candidate converged everywhere.
 */
xkp_status xkp_autotune_seeds(xkp_ctx *ctx, int32_t n_seeds, const xkp_system *seeds,
                              void *const *bases, const xkp_params *params, xkp_info *infos,
                              xkp_tuning *out);

/*
 * Target solve that allocates nothing, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as xkp_target_project_solve with the default 8-wave launch, without a
 * context.  Its workspace (per-workgroup Krylov basis, coefficient arrays, projection block) and
 * work-queue counters live in a fixed device array of XKP_NOALLOC_SCRATCH_MIB MiB inside the
 * library, one per GPU it runs on, held until the process ends; the call itself calls no
 * allocator.  The array holds as many workgroup slots as fit for the call's size (n at most
 * params->batch_max_n, or XKP_NOALLOC_MAX_N when 0; restart length the larger of m and
 * polish_m), so larger systems run on fewer workgroups; a size of which not even one slot fits
 * returns XKP_EINVAL.  `device` is the GPU (made current by the call), `hip_stream` a stream on
 * it (NULL: the null stream); the other arguments are those of xkp_target_project_solve, whose
 * checks apply (with m, polish_m <= 64 and batch_max_n <= XKP_NOALLOC_MAX_N).  Argument errors
 * return before any device call.  Every call on one GPU uses the same array and leaves its last
 * contents there (the queue counters are cleared by a small kernel at the start of each call):
 * calls that overlap in time on one GPU race, so callers serialise them, e.g. on one stream.
 */
#define XKP_NOALLOC_SCRATCH_MIB 64
#define XKP_NOALLOC_MAX_N 16384

xkp_status xkp_target_project_solve_noalloc(int device, void *hip_stream, int32_t n_targets,
                                            const xkp_system *targets, int32_t n_bases,
                                            const void *const *bases, const xkp_params *params,
                                            xkp_info *infos);

/* Static description of a status code. */
const char *xkp_status_string(xkp_status s);

#ifdef __cplusplus
}
#endif
#endif /* XKP_H */
