/*
 * rbns.h -- C ABI of the MI355X (gfx950) online solver for the velocity-only reduced-basis
 * Navier-Stokes method (Fonn, van Brummelen, Kvamsdal, Rasheed: "Fast divergence-conforming
 * reduced basis methods for steady Navier-Stokes flow").
 *
 * The online stage, per parameter mu (Sections 2.2, 2.4, 3.4, 3.5, 4.1 of the paper):
 *   solve  F(u) = A(mu) u + C(mu)(u, u) - f(mu) = 0   (velocity-only system, eqn velonly)
 *   with   A(mu) = sum_q theta^a_q(mu) A_q,
 *          C(mu)(v, w)_i = sum_q theta^c_q(mu) sum_jk C_q[i][j][k] v_j w_k,
 *          f(mu) = sum_q theta^f_q(mu) f_q                (affine representation, eqns split-*)
 *   by Newton's method with the Jacobian assembled from the precomputed third-order tensors
 *          J = A(mu) + sum_q theta^c_q sum_k (C_q[:, :, k] + C_q[:, k, :]) u_k    (Section 3.5)
 *   and a dense pivoted LU solve per step; then recover the pressure a posteriori
 *          B(mu) p = f_s(mu) - A_sv(mu) u - C_sv(mu)(u, u)          (eqns sup-vvar, blocksolve-2).
 *
 * Conventions for every entry point:
 *   - All matrices are row-major (C order), FP64 on the host side of rb_load_tensors.
 *   - Per-request arrays are DEVICE pointers owned by the caller; calls enqueue work on the
 *     given HIP stream (hipStream_t passed as void*, NULL = the null stream) and return
 *     without synchronising. Outputs are valid once that stream has completed.
 *   - Calls on one context that share a stream are ordered by it; the library keeps one
 *     workspace per stream, so calls on different streams may overlap.
 *   - Return value: RB_OK, or a negative call-level error, in which case nothing was
 *     enqueued and rb_last_error() describes the failure (thread-local message).
 *   - Per-request outcomes are reported in status arrays (RB_ST_*), never as call errors.
 */
#ifndef RBNS_H
#define RBNS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* call-level return codes */
#define RB_OK             0
#define RB_E_INVAL       -1   /* bad argument: NULL pointer, size out of range, unknown set  */
#define RB_E_NOMEM       -2   /* the request exceeds the context's HBM budget, or hipMalloc */
#define RB_E_DEVICE      -3   /* a HIP runtime call failed                                   */
#define RB_E_STATE       -4   /* context not usable (destroyed, wrong device)                */
#define RB_E_UNSUPPORTED -5   /* valid request this build does not implement                 */

/* per-request status codes */
#define RB_ST_CONVERGED  0    /* update below tolerance                                      */
#define RB_ST_MAXIT      1    /* iteration limit reached; the last iterate is returned       */
#define RB_ST_SINGULAR   2    /* zero pivot in the Newton (or pressure) system               */
#define RB_ST_NONFINITE  3    /* NaN or Inf in an operand, update or iterate                 */
#define RB_ST_BADN       4    /* basis size out of range for the loaded set                  */
#define RB_ST_REFINED    6    /* mixed precisions: the refinement steps ran out while every
                                 refinement update after the first was at most half the one
                                 before it: the error is of the order of the last update times
                                 that contraction; a refinement that stagnates or grows ends
                                 RB_ST_MAXIT instead                                          */

/* arithmetic of the Newton iteration */
#define RB_PREC_F64      0    /* FP64 tensors, FP64 MFMA contraction, FP64 LU                */
#define RB_PREC_F32      1    /* FP32 tensors + FP32 MFMA contraction, FP32 LU, FP64 iterates,
                                 then FP64-residual refinement steps                          */
#define RB_PREC_BF16     2    /* as RB_PREC_F32 with BF16 tensors on BF16 MFMA (FP32 accum.) */
#define RB_PREC_BF16X3   3    /* as RB_PREC_BF16 with tensors and iterate terms each split into
                                 a BF16 high and low part, three BF16 MFMAs per product (about
                                 16 mantissa bits), so one refinement step reaches ~1e-9       */

typedef struct rb_ctx rb_ctx;

/*
 * Reduced operators of one parameterised model (host pointers, FP64, copied on load).
 * Sizes are the stored maxima; bases are nested, so a solve at basis size n <= N uses the
 * leading n x n (x n) blocks. Index meaning (row index = test function, as in a Galerkin
 * matrix; paper eqn tensor writes C^i_{jkl} = c_i(u_j, u_k, u_l), i.e. C_q[l][j][k] here):
 *   A   [Q][N][N]        A_q[i][j]      = a_q(phi_j, phi_i)
 *   C   [Qc][N][N][N]    C_q[i][j][k]   = c_q(phi_j, phi_k, phi_i)   (j advects, k advected)
 *   F   [Qf][N]          f_q[i]         = d_q(phi_i)
 *   H   [N][N] or NULL   Gram matrix of the norm used by the stopping test (the paper uses the
 *                        H^1 seminorm, Section 6); NULL selects the Euclidean norm.
 * Optional pressure recovery data (Np = 0 disables it):
 *   Bp  [Qb][Np][Np]     B_q[i][j]      = b_q(p_j, s_i)   (s_i = supremizers, Section 3.4)
 *   Asv [Q][Np][N]       A_sv,q[i][j]   = a_q(phi_j, s_i)
 *   Csv [Qc][Np][N][N]   C_sv,q[i][j][k]= c_q(phi_j, phi_k, s_i)
 *   Fs  [Qf][Np]         f_s,q[i]       = d_q(s_i)
 */
typedef struct {
    int N, Q, Qc, Qf;
    const double *A, *C, *F, *H;
    int Np, Qb;
    const double *Bp, *Asv, *Csv, *Fs;
} rb_tensors_desc;

typedef struct {
    double tol;          /* stop when ||delta|| <= tol * ||u|| (norm given by H)           */
    int max_iter;        /* Newton iteration limit (>= 1); for the mixed precisions, the
                            limit of the low-precision phase                                 */
    int precision;       /* RB_PREC_*                                                        */
    int refine_steps;    /* mixed precisions only (0..100): at most this many refinement
                            steps after the low-precision phase; each evaluates the residual
                            F(u) from the FP64 tensors, solves with the low-precision
                            Jacobian of the last low-precision step and adds the correction
                            to the FP64 iterate                                              */
} rb_solve_opts;

/* Size limits of this build. The LU keeps one system row per lane: one 64-wide wavefront per
 * system up to 64 unknowns, a workgroup of ceil(N/64) wavefronts beyond. */
#define RB_MAX_N      152   /* basis size, mixed precisions (FP32 LU)                   */
#define RB_MAX_N_F64   96   /* basis size, RB_PREC_F64 (FP64 LU rows in registers)      */
#define RB_MAX_NP      64   /* pressure basis size                                      */
#define RB_MAX_Q   64   /* affine terms of a (the paper's Piola expansion: 4n + 2 = 50)  */
#define RB_MAX_QC  64   /* affine terms of c (4n + 1 = 49); mixed precisions: Q <= 12,
                           Qc <= 4                                                       */
#define RB_MAX_QF   2
#define RB_MAX_QB   2

/* Variants of the FP64 dense solve of the Newton and pressure systems (one system per
 * wavefront up to 64 unknowns): one row per lane with the pivot row broadcast by readlane or
 * through LDS, or the system in matrix-core tiles with panel updates on MFMA (N <=
 * RB_LU_MFMA_MAX_N; larger systems fall back to readlane). RB_LU_AUTO (the default) takes the
 * matrix-core solve up to RB_LU_AUTO_MFMA_N unknowns and readlane beyond, the faster of the
 * two on MI355X at 4096 systems (N = 30: 39 vs 53 us per launch; N = 50: 129 vs 97 us). The
 * environment variable RB_LU=auto|readlane|lds|mfma sets it for a new context, and the
 * autotuner times the variants per batch shape. */
#define RB_LU_READLANE   0
#define RB_LU_LDS        1
#define RB_LU_MFMA       2
#define RB_LU_AUTO       3
#define RB_LU_MFMA_MAX_N 63
#define RB_LU_AUTO_MFMA_N 31

/*
 * rb_create: make a context on HIP device `device`. hbm_budget_bytes caps the device memory
 * the context may hold (resident tensors + workspaces); 0 means no cap.
 * Errors: RB_E_INVAL (out == NULL, bad device), RB_E_DEVICE.
 */
int rb_create(int device, size_t hbm_budget_bytes, rb_ctx **out);

/* rb_destroy: free every device buffer of the context. Pending work must have completed. */
int rb_destroy(rb_ctx *ctx);

/* rb_last_error: message for the last failing call on this thread ("" if none). */
const char *rb_last_error(void);

/* rb_hbm_used: bytes of device memory the context currently holds. */
size_t rb_hbm_used(const rb_ctx *ctx);

/*
 * rb_load_tensors: copy a model's reduced operators (the affine matrices of Section 3.4, the
 * third-order convection tensors of eqn tensor in Section 3.5, and the supremizer-tested
 * pressure operators of Section 4.1) to the device (FP64, plus the packed contraction
 * operands built from them) and return its set id. Low-precision copies (FP32, BF16) are
 * built from the FP64 tensors on the device the first time a precision is used, so the
 * descriptor carries no storage type. The caller may free the host
 * arrays on return. Synchronous.
 * Errors: RB_E_INVAL (NULL pointer, sizes out of range), RB_E_NOMEM (over budget),
 * RB_E_DEVICE.
 */
int rb_load_tensors(rb_ctx *ctx, const rb_tensors_desc *desc, int *set_id_out);

/*
 * rb_theta: evaluate the parameter functions of the loaded model's affine expansion (eqns
 * split-a .. split-d1 of Section 2.4; the functions are a reading, see below) for B
 * parameters mu[b] = (alpha [rad], Re) (device, [B][2]). Writes theta_a [B][Q],
 * theta_c [B][Qc], theta_f [B][Qf] and, if the set has pressure data and theta_b != NULL,
 * theta_b [B][Qb] (all device). Families (trigonometric / polynomial in alpha, viscous 1/Re):
 *   theta_a = first Q of (1/Re, cos a, sin a, a, a^2, a^3, cos 2a, sin 2a, 1 - cos a, a^4,
 *             a cos a, a sin a);  theta_c = first Qc of (1, cos a, sin a, a);
 *   longer expansions (Q > 12, Qc > 4) are the Piola-mapped forms' truncated power series in
 *   the angle (Section 5): theta_a[q] = a^q / Re, theta_c[q] = a^q;
 *   theta_f = (1) if Qf = 1, else (cos a, sin a);  theta_b = (1) if Qb = 1, else (1, a).
 * Errors: RB_E_INVAL.
 */
int rb_theta(rb_ctx *ctx, int set, int B, const double *mu, double *theta_a, double *theta_c,
             double *theta_f, double *theta_b, void *hip_stream);

/*
 * rb_solve_batch: B independent reduced Newton solves of the velocity-only system (eqn
 * velonly, Section 2.2), the Jacobian assembled from the tensors (Section 3.5), at one basis
 * size N (1 <= N <= the set's N; per-request sizes: rb_solve_uneven). Device inputs: theta_a [B][Q], theta_c [B][Qc], and either theta_f [B][Qf] or
 * f_override [B][ldu] (right-hand sides replacing f(mu), e.g. for manufactured solutions);
 * u0 [B][ldu] initial iterates or NULL (zero: the first step is then the Stokes solve, whose
 * Jacobian A(mu) is summed from the Q affine operators alone, at every precision).
 * Device outputs: u [B][ldu] (entries >= N are set to 0), iters [B] (Newton updates applied),
 * status [B] (RB_ST_*). ldu >= N is the row stride of u0 / f_override / u.
 * opts == NULL selects tol 1e-12, max_iter 10, RB_PREC_F64.
 * Mixed precisions (RB_PREC_F32 / RB_PREC_BF16 / RB_PREC_BF16X3): the low-precision phase stops
 * a request when its update is below tol or has stagnated (update <= 5e-2 ||u|| for BF16,
 * 1e-3 ||u|| for the others, and no longer halving), or at max_iter. RB_PREC_BF16X3 needs
 * Qc*N <= 640, RB_PREC_BF16 likewise; the mixed precisions need Q <= 12 and Qc <= 4
 * (RB_E_UNSUPPORTED otherwise: long expansions run in FP64). Then every request without a failure status takes
 * up to refine_steps refinement steps (FP64 residual, the Jacobian of its last low-precision
 * step) until an update is below tol (status RB_ST_CONVERGED, else RB_ST_REFINED or
 * RB_ST_MAXIT, see RB_ST_REFINED). iters
 * counts both kinds of updates.
 * Schedule (FP64, N <= 64 with the readlane LU): the first K Newton iterations run as launch
 * pairs over the whole batch and the remaining max_iter - K in one launch that steps each
 * 64-request tile until its requests are done; K is the largest iteration count of the last
 * finished call with the same set and N (read back without blocking; max_iter at first), or
 * RB_NEWTON_K in the environment of rb_create (0: all max_iter iterations as launch pairs,
 * n > 0: K = n). Results do not depend on K, bit for bit. Under stream capture the schedule
 * keeps all max_iter pairs.
 * Errors: RB_E_INVAL (NULL, B < 0, N or ldu out of range, bad opts), RB_E_NOMEM,
 * RB_E_UNSUPPORTED (RB_PREC_F64 with N > RB_MAX_N_F64), RB_E_DEVICE. B == 0 is a no-op.
 */
int rb_solve_batch(rb_ctx *ctx, int set, int B, int N, int ldu, const double *theta_a,
                   const double *theta_c, const double *theta_f, const double *f_override,
                   const double *u0, const rb_solve_opts *opts, double *u, int *iters,
                   int *status, void *hip_stream);

/*
 * rb_solve_batch_noalloc: rb_solve_batch for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * arguments, same kernels and tile shapes, same results as rb_solve_batch (it runs all
 * max_iter Newton iterations as launch pairs: the iteration history would need an
 * allocation). The Newton state
 * (Jacobians, iterates, partial sums, flags) lives in one static device array of
 * RB_NOALLOC_SCRATCH_BYTES per device, held from library load to process exit, instead of a
 * per-stream workspace; the call allocates nothing (no hipMalloc / hipFree / library
 * allocation, no kernel-timing events). The state is initialised by the call's first kernel,
 * so nothing carries over between calls.
 * Every call on one device shares that device's array: calls that overlap on a device (other
 * streams, other contexts, other threads) race and corrupt each other's results. Serialise
 * them (one stream, or events) and leave this entry point out of concurrent use.
 * Preconditions: the packed contraction operands for (N, precision) exist; rb_load_tensors
 * builds them for the set's own N in FP64, and any earlier rb_solve_batch or rb_autotune call
 * at (N, precision) builds the others.
 * Errors: as rb_solve_batch; RB_E_NOMEM when the batch's state exceeds the array (about 24 KB
 * per request at N = 50 in FP64, so B <= 2700 there; 64-request tiles), RB_E_STATE when the
 * packed operands are missing.
 */
#define RB_NOALLOC_SCRATCH_BYTES (64ull << 20)
int rb_solve_batch_noalloc(rb_ctx *ctx, int set, int B, int N, int ldu, const double *theta_a,
                           const double *theta_c, const double *theta_f,
                           const double *f_override, const double *u0,
                           const rb_solve_opts *opts, double *u, int *iters, int *status,
                           void *hip_stream);

/*
 * rb_solve_uneven: like rb_solve_batch, but each request b has its own basis size N[b]
 * (device int [B]; the nested basis of size N[b] is the leading block of the set's tensors);
 * rows of u0 / f_override / u have stride ldu >= the set's N. Not part of the paper: a
 * batching form for mixed basis sizes.
 * The call copies N to the host (it waits for the work already queued on hip_stream), groups
 * the requests by N (largest first, each group padded to whole 64-request tiles), gathers
 * their inputs into library staging, runs the groups' Newton chains and scatters the results
 * back in the caller's order. The group chains are captured into one HIP graph the second time
 * the same shape (group sizes in tiles, options, tile shapes) occurs and replayed from then on
 * (one graph launch per call, up to 4 group chains running concurrently); a shape seen for the
 * first time runs as plain launches. The first time a (set, N, precision, batch size class)
 * occurs, the autotuner times the candidate tile shapes on that group (synchronously) and
 * keeps the fastest (environment RB_AUTOTUNE=0 disables it; RB_UNEVEN_GRAPHS=0 keeps every
 * call on plain launches, so that the kernel timing of rb_timing_* sees each launch).
 * Requests with N[b] outside [1, set N] get status RB_ST_BADN, iters 0 and u = 0.
 * Errors: as rb_solve_batch (RB_E_INVAL also for ldu < the set's N).
 */
int rb_solve_uneven(rb_ctx *ctx, int set, int B, const int *N, int ldu, const double *theta_a,
                    const double *theta_c, const double *theta_f, const double *f_override,
                    const double *u0, const rb_solve_opts *opts, double *u, int *iters,
                    int *status, void *hip_stream);

/*
 * rb_recover_pressure_uneven: like rb_recover_pressure, but each request b has its own
 * velocity basis size N[b] (device int [B]; pressure size Np for all); rows of u have stride
 * ldu >= the set's N, rows of p stride ldp >= Np. The call copies N to the host (it waits for
 * the work already queued on hip_stream), groups the requests by N, recovers each group's
 * pressure and scatters p and status back in the caller's order. Requests with N[b] outside
 * [1, set N] get status RB_ST_BADN and p = 0.
 * Errors: as rb_recover_pressure.
 */
int rb_recover_pressure_uneven(rb_ctx *ctx, int set, int B, const int *N, int Np, int ldu,
                               int ldp, const double *theta_a, const double *theta_c,
                               const double *theta_f, const double *theta_b, const double *u,
                               double *p, int *status, void *hip_stream);

/*
 * rb_autotune: time the candidate tile shapes of a batch of B requests at basis size N with
 * these coefficients (device theta_a [B][Q], theta_c [B][Qc], theta_f [B][Qf]) and keep the
 * fastest for (set, N, opts->precision, batch size class ceil(log2(B/64))); later
 * rb_solve_batch / rb_solve_uneven calls of that class use it. Candidates: 2, 4, 8, 16 and
 * the default number of row splits per 64-request tile of the contraction, and (FP64,
 * N <= 64) the pivot-row broadcast of the LU (readlane or LDS). Synchronous; produces no
 * solution.
 * rb_tuned_config: the shape in use for such a batch, lu_variant one of RB_LU_*.
 * Defaults when never tuned: readlane, and 8 row splits (one per XCD) for batches that fill
 * the chip, up to 64 for small ones (about 512 workgroups, at least 4 row blocks a split).
 * Errors: RB_E_INVAL, RB_E_UNSUPPORTED (FP64 beyond RB_MAX_N_F64), RB_E_DEVICE.
 */
int rb_autotune(rb_ctx *ctx, int set, int B, int N, const double *theta_a,
                const double *theta_c, const double *theta_f, const rb_solve_opts *opts,
                void *hip_stream);
int rb_tuned_config(rb_ctx *ctx, int set, int N, int precision, int B, int *nsplit,
                    int *lu_variant);

/*
 * rb_recover_pressure: a posteriori pressure for B velocity solutions at basis size N and
 * pressure size Np (<= the set's Np), from eqn sup-vvar with the supremizers as test space:
 *   B(mu) p = f_s(mu) - A_sv(mu) u - C_sv(mu)(u, u),   B(mu) = sum_q theta^b_q B_q.
 * Device inputs: theta_a, theta_c, theta_f as for rb_solve_batch, theta_b [B][Qb], u [B][ldu].
 * Device outputs: p [B][ldp] (entries >= Np set to 0), status [B] (RB_ST_CONVERGED on
 * success, RB_ST_SINGULAR / RB_ST_NONFINITE otherwise).
 * Errors: RB_E_INVAL (no pressure data, sizes), RB_E_NOMEM, RB_E_DEVICE.
 */
int rb_recover_pressure(rb_ctx *ctx, int set, int B, int N, int Np, int ldu, int ldp,
                        const double *theta_a, const double *theta_c, const double *theta_f,
                        const double *theta_b, const double *u, double *p, int *status,
                        void *hip_stream);

/*
 * rb_reconstruct_pressure: pressure from a combined velocity-pressure basis (Section 4.2, the
 * second construction after eqn z_c): each reduced velocity function carries a pressure part
 * made of the same snapshot combination, so p = Pc u for every request,
 *   p[b][i] = sum_{j < N} Pc[i][j] u[b][j],  i < Np   (entries Np <= i < ldp set to 0).
 * Device inputs: Pc [Np][ldpc] (pressure-basis coefficients of the pressure parts of the
 * first N velocity functions; nested bases use its leading columns), u [B][ldu]. Device
 * output: p [B][ldp]. Unlike rb_recover_pressure this presumes that the pressure depends
 * linearly on the velocity (the paper's remark on linearity); it needs no tensor set.
 * Errors: RB_E_INVAL (NULL, sizes: 1 <= N <= RB_MAX_N, 1 <= Np <= RB_MAX_NP, ldpc, ldu >= N,
 * ldp >= Np), RB_E_DEVICE. B == 0 is a no-op.
 */
int rb_reconstruct_pressure(rb_ctx *ctx, int B, int N, int Np, const double *Pc, int ldpc,
                            const double *u, int ldu, double *p, int ldp, void *hip_stream);

/*
 * rb_assemble_convection: offline assembly of the convection tensors by quadrature on the
 * device (eqn tensor, Section 3.5; the offline step, not the online solve): for the affine
 * terms c_q(u, v, t) = int ((u . grad) v) . (M_q t),
 *   out[q][i][j][k] = w * sum_x sum_{b,c} M_q[b][c] ((phi_j . grad) phi_k)^b(x) t_i^c(x),
 * i < R (test functions), j, k < N (velocity functions), x < X (quadrature points, weight w).
 * With t = phi this is C_q[i][j][k] of rb_tensors_desc; with t = the supremizers, C_sv.
 * The Qc tensors are formed from four base contractions (R x X x N^2 each) on MFMA-F64.
 * Device inputs, point-major: phiT [X][2][N] (phi_j^a(x) at (x*2 + a)*N + j), dphiT
 * [X][2][2][N] (d_a phi_k^b(x) at ((x*2 + a)*2 + b)*N + k), testT [X][2][R]. Host input:
 * M [Qc][2][2]. Device output: out [Qc][R][N][N]. Synchronous (returns when out is written);
 * uses the stream's workspace (8 * 4 * R * N^2 bytes per quadrature split, at most 16).
 * Errors: RB_E_INVAL (NULL, N or R outside [1, RB_MAX_N], Qc outside [1, RB_MAX_QC],
 * X < 1), RB_E_NOMEM, RB_E_DEVICE.
 */
int rb_assemble_convection(rb_ctx *ctx, int N, int R, int X, int Qc, const double *phiT,
                           const double *dphiT, const double *testT, const double *M, double w,
                           double *out, void *hip_stream);

/* ------------------------------------------------------------------ serving --------- */
/*
 * Continuous-batching server on top of one context and tensor set (not part of the paper: a
 * serving form of the online stage). rb_server_submit queues requests (mu, N) and returns at
 * once; a worker thread forms a batch whenever one of its `lanes` (HIP streams, each with its
 * own device buffers) is free, so requests that arrive while others are on the GPU are
 * admitted as soon as a lane and the HBM budget allow, and the batches of different lanes
 * overlap on the device. Requests fall into size classes (N rounded up to a multiple of 16,
 * at most the set's N); a free lane takes the class of the oldest waiting request, every
 * queued request of that class up to max_batch, so small bases do not wait for the large ones
 * and no request waits behind younger ones of its class. A batch is solved as one batch of its
 * class size (theta(mu) on the device, Newton, optionally the pressure), every request as the
 * leading N x N block of the class system with its other unknowns held at zero; the tile
 * shapes depend on the class only, so a request's result does not depend on the other
 * requests of its batch (a class's row splits are fixed by its N alone, never by the batch
 * size or the tuning table). rb_server_poll hands back finished
 * results (with the latency from submission to the moment the worker saw the batch finish).
 * The tensor set stays resident; each lane keeps its buffers and workspace between batches.
 * Stop every server of a context before rb_destroy.
 */
#define RB_ST_FAILED 5   /* server: the batch could not be run (see rb_server_counters.error) */

typedef struct rb_server rb_server;

typedef struct {
    int precision;            /* RB_PREC_*                                                  */
    int refine_steps;         /* mixed precisions: refinement steps                         */
    int max_iter;             /* Newton iteration limit                                     */
    double tol;               /* Newton tolerance                                           */
    int max_batch;            /* requests per batch (1..65536)                              */
    int lanes;                /* batches in flight at once (1..16), each one size class on
                                 its own stream; lanes beyond the device's hardware queues
                                 (HIP's default: 4) share queues and wait on each other       */
    size_t hbm_budget_bytes;  /* workspace of the batches in flight (0: no limit): a batch is
                                 cut (halved until it fits) beside the batches in flight, or
                                 waits for them to finish; alone it runs at any size        */
    int pressure;             /* 1: also recover the pressure (set must have pressure data) */
} rb_server_opts;

typedef struct {
    double alpha, re;         /* mu = (angle of attack [rad], Reynolds number)              */
    int N;                    /* basis size, 1 <= N <= set N (else status RB_ST_BADN)       */
    long long tag;            /* caller's label, returned with the result                   */
} rb_request;

typedef struct {
    long long ticket, tag;
    int N, status, iters, pstatus;
    double latency_ms;        /* submission -> batch completion seen by the worker          */
    double queue_ms;          /* submission -> launch of its batch (the rest of latency_ms is
                                 the batch on the GPU plus the copy back)                     */
    double u[RB_MAX_N];       /* velocity coefficients (first N valid, rest 0)              */
    double p[RB_MAX_NP];      /* pressure coefficients (first Np valid) if opts.pressure    */
} rb_result;

typedef struct {
    long long submitted, completed, batches;
    double p50_ms, p99_ms, max_ms;   /* latency quantiles over the completed requests
                                        (log-spaced histogram: within 0.5 %; max exact)     */
    double p50_queue_ms, p99_queue_ms;   /* same for the wait before the batch launch       */
    double mean_batch;               /* requests per batch                                  */
    double first_submit_s, last_done_s;   /* on the server's clock (seconds since start)   */
    size_t hbm_inflight_peak;        /* largest workspace estimate of batches in flight    */
    char error[256];                 /* last batch failure, empty if none                  */
} rb_server_counters;

/* Errors: RB_E_INVAL (bad set / opts), RB_E_NOMEM (lane buffers), RB_E_DEVICE. */
int rb_server_start(rb_ctx *ctx, int set, const rb_server_opts *opts, rb_server **out);
/* Queue n requests; tickets[i] receives the ticket of reqs[i] (may be NULL). */
int rb_server_submit(rb_server *srv, const rb_request *reqs, int n, long long *tickets);
/* Move up to max finished results into out; *n_out = how many. Never blocks. */
int rb_server_poll(rb_server *srv, rb_result *out, int max, int *n_out);
/* Latency / throughput counters so far. */
int rb_server_stats(rb_server *srv, rb_server_counters *out);
/* Finish every queued request, stop the worker and free the lanes (results not yet polled
 * are dropped). */
int rb_server_stop(rb_server *srv);

/*
 * Kernel timing for measurement (used by the benchmark): while enabled, every launch of the
 * kernel families "jacobian" (MFMA Jacobian + residual contraction), "lu" (pivoted LU solve +
 * update) and "pressure" (pressure recovery) is bracketed by HIP events recorded on the
 * stream it is launched on. rb_timing_read waits for the recorded events of one family,
 * returns their summed duration (ms) and launch count, and forgets them.
 * Errors: RB_E_INVAL (unknown family), RB_E_DEVICE.
 */
int rb_timing_enable(rb_ctx *ctx, int enable);
/* (family "residual": the FP64 residual contraction of the mixed-precision refinement;
 *  family "reconstruct": rb_reconstruct_pressure; family "stokes": the first Jacobian of a
 *  solve without initial iterates, A(mu) assembled from the affine operators, at every
 *  precision) */
int rb_timing_read(rb_ctx *ctx, const char *family, double *total_ms, int *launches);

#ifdef __cplusplus
}
#endif

#endif /* RBNS_H */
