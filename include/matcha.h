/*
 * matcha.h -- C ABI of libmatcha, the MI355X (gfx950) implementation of the
 * rotational-alignment path of "Matcha: Fast Volume Alignment by
 * Frequency-Marched Newton Method":
 *
 *   coefficient assembly  (Sec. 2.1, eq. sigmalmm)
 *   -> low-bandwidth SOFFT search keeping the strongest local maxima (Sec. 2.3)
 *   -> frequency-marched Newton refinement and final selection (Sec. 2.2, 2.4, Alg. 1)
 *   and the adjoint of the selected objective value with respect to the inputs.
 *
 * Problem statement (Sec. 1): given a particle f and a template h, both real functions,
 * return the rotation g maximising <f, g o h>; the inputs of Alg. 1 are the band schedule
 * {L_j}, the Newton steps per level M_iter and the number of SOFFT candidates (the paper's P,
 * Kc here).
 *
 * Conventions (App. A.3-A.5).  Rotations use the ZYZ chart
 * g(a, b, c) = r_z(a) r_y(b) r_z(c) (eq. Euler), angles in radians, a and c in
 * [0, 2pi), b in [0, pi].  D^l_mn(a, b, c) = e^{-ima} d^l_mn(b) e^{-inc}
 * (eq. wigner-D) with d^l_mn(b) = <l m| exp(-i b J_y) |l n>.  The objective is
 *   C_L(g) = Re sum_{l<=L} sum_{m,n} C^l_mn conj(D^l_mn(g)),
 *   C^l_mn = sum_r w_r f_lm(r) conj(h_ln(r)),
 * i.e. <f, g o h> with (g o h)_l = D^l(g) h_l; the conjugation of D is the
 * "conjugation absorbed into the coefficients" of App. A.5.
 *
 * Memory.  Every pointer is a device pointer unless its comment says (host).  The caller
 * allocates every input, output and workspace buffer; the library allocates nothing on the
 * caller's behalf and keeps no pointer after the enqueued work completes.  A context owns only
 * read-only tables: the Wigner-d recurrence coefficients for every degree up to MATCHA_MAX_L
 * (built by matcha_create), the SOFFT node tables of each (B, n_grid) passed to matcha_prepare,
 * and the launch shapes chosen by matcha_autotune.  Tables are freed only by matcha_destroy, so
 * a captured graph never refers to freed tables while its context lives.
 *
 * Calls.  matcha_create, matcha_prepare, matcha_autotune and the graph calls are synchronous
 * set-up calls and may allocate.  The enqueue calls (matcha_coeff_assemble, matcha_soft_search,
 * matcha_march_newton, matcha_evaluate, matcha_grad_template) validate their arguments on the
 * host and enqueue kernels on `stream` (a hipStream_t passed as void*); they never allocate,
 * free or wait on the device, so they can be captured into a HIP graph.  A context is not
 * thread-safe; calls that share a workspace must be ordered (one stream).
 *
 * Errors.  Invalid arguments return MATCHA_ERR_INVALID_ARG and enqueue nothing; a workspace
 * below the call's need returns MATCHA_ERR_WORKSPACE; a SOFFT shape not passed to
 * matcha_prepare returns MATCHA_ERR_NOT_PREPARED.  The enqueue calls check, in this order, the
 * batch, the configuration and buffer arguments, the workspace and then the context (a NULL ctx
 * gives MATCHA_ERR_INVALID_ARG only once everything else has passed; device pointers are checked
 * for NULL and alignment only, never read on the host).  Launch failures return MATCHA_ERR_HIP.
 * Numerical conditions never fail a call; they set per-particle status bits (MATCHA_ST_*).
 * No C++ exception crosses the ABI.
 *
 * Layouts.
 *   complex      : interleaved (re, im), float32 unless stated.
 *   f (particle) : particle p at element offset f_offset[p]: [R_p][(L_p+1)^2],
 *                  lm = l*l + l + m.  h (template): [R_h][(L_h+1)^2].  Inputs must be
 *                  Hermitian-symmetric, c_{l,-m} = (-1)^m conj(c_lm) (real volumes);
 *                  kernels read only the m >= 0 half.
 *   C (wedge)    : particle p at element offset C_offset[p], matcha_c_elems(L_p)
 *                  complex values.  For l = 0..L_p, for every "wedge pair"
 *                  (m, n) with 0 <= |n| <= m <= l, in the order q = m*m + m + n,
 *                  two values: C^l_mn and C^l_{m'n'} of its partner
 *                  (m', n') = (n, m) if n >= 0, (-n, -m) if n < 0.
 *                  Row l starts at 2 * l(l+1)(2l+1)/6 complex values, so the rows l <= L' of a
 *                  band-L_p block are the band-L' block.  The wedge and its partners cover
 *                  {m > 0} and {m = 0, n >= 0}; the other half follows from
 *                  C^l_{-m,-n} = (-1)^{m-n} conj(C^l_mn).  matcha_c_unpack converts to the
 *                  packed-by-l layout.
 *   C (by l)     : block l at l(4l^2-1)/3 complex values, (2l+1)^2 values row-major in
 *                  (m, n), m, n = -l..l.
 *   candidates   : float4 (a, b, c, value) per candidate, [P][Kc].
 */
#ifndef MATCHA_H
#define MATCHA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MATCHA_OK = 0,
    MATCHA_ERR_INVALID_ARG = -1,
    MATCHA_ERR_UNSUPPORTED = -2,
    MATCHA_ERR_HIP = -3,
    MATCHA_ERR_WORKSPACE = -4,
    MATCHA_ERR_NOT_PREPARED = -5
} matcha_status;

typedef enum {
    MATCHA_FP32 = 0,        /* FP32 storage and arithmetic                                  */
    MATCHA_BF16_FP32ACC = 1 /* BF16 f/h storage, MFMA products with FP32 accumulation      */
} matcha_precision;

/* per-particle status bits (numerical conditions; never an error) */
#define MATCHA_ST_NONFINITE 1u   /* a non-finite objective value or derivative was met   */
#define MATCHA_ST_INDEFINITE 2u  /* a Newton step was taken with H not negative definite */
#define MATCHA_ST_SINGULAR 4u    /* |det H| <= 1e-30 max|H|^3: the step was skipped       */
#define MATCHA_ST_NEAR_POLE 8u   /* sin b < 1e-3 after a step (chart singular at b = 0, pi) */
#define MATCHA_ST_FEW_MAXIMA 16u /* the SOFFT grid had fewer than Kc local maxima         */
#define MATCHA_ST_EARLY_STOP 32u /* early stopping ended a level before M_iter steps      */

/* Limits of the library. */
#define MATCHA_MAX_L 64
#define MATCHA_MAX_KC 64
#define MATCHA_MAX_LEVELS 16

typedef struct matcha_ctx matcha_ctx;

/* A batch of particles.  Per-particle band limits L_p <= L_max and shell counts
 * R_p <= R_h are given twice: on the host (validation, launch sizing) and on the
 * device (kernels).  Particle p uses template shells 0..R_p-1 and degrees l <= L_p. */
typedef struct {
    int32_t n_particles;
    int32_t L_max;              /* max_p L_p                                    */
    const int32_t *L_host;      /* (host) [P]                                   */
    const int32_t *R_host;      /* (host) [P]                                   */
    const int32_t *L_dev;       /* [P]                                          */
    const int32_t *R_dev;       /* [P]                                          */
    const int64_t *f_offset;    /* [P] complex-element offsets of particles in f (any layout
                                   that keeps particles apart; need not be packed) */
    const int64_t *C_offset;    /* [P] complex-element offsets in C (even)       */
    int32_t L_h, R_h;           /* template extents: h is [R_h][(L_h+1)^2]       */
    const int32_t *order;       /* [P] nullable: processing order of the particles for the
                                   march (e.g. longest first from matcha_lpt_order); the
                                   hardware starts workgroups in this order as slots free up */
} matcha_batch;

/* SOFFT search (Sec. 2.3): grid of n_grid^3 rotations a_j = 2 pi j/n,
 * b_i = pi (2i+1)/(2n), c_k = 2 pi k/n; band B = L0 (the paper's oversampling K
 * gives n_grid = 2 K B); keep the Kc strongest local maxima (the paper's P). */
typedef struct {
    int32_t B;
    int32_t n_grid;
    int32_t Kc;
} matcha_soft_cfg;

/* Frequency march (Alg. 1).  levels (host) is the global schedule; particle p
 * runs every level < L_p and then L_p.  steps = M_iter Newton steps per level (gradient ascent
 * steps when gd_rate > 0).
 * max_step > 0 clips the largest component of a Newton step (0: pure Newton, as
 * in the paper).  early_stop enables the Sec. 2.4 tests: a level ends once
 * |grad| <= tol_grad |F|, |F - F_prev| <= tol_rel |F| (from its second step on) or the last
 * step's largest component <= tol_step. */
typedef struct {
    const int32_t *levels; /* (host) strictly increasing, levels[0] >= 1 */
    int32_t n_levels;
    int32_t steps;
    double max_step;
    int32_t early_stop;
    double tol_grad, tol_step, tol_rel;
    int32_t fp64_above;    /* levels above this degree run the Wigner-d recurrence in FP64 (FP64
                              coefficient table; the l-sums stay FP32); 0 or >= MATCHA_MAX_L: FP32 only */
    const float *C_final;  /* nullable: coefficients (same layout and offsets as C) for each
                              particle's final level L_p and the final values; NULL: C.  The BF16
                              path marches the lower levels on BF16-assembled C and the final level
                              on FP32-assembled C_final. */
    double gd_rate;        /* 0: Newton steps (the method).  > 0: gradient ascent steps instead, the
                              first-order comparator of Sec. 4.1 (Fig. newton_v_gd): theta += t grad,
                              t = gd_rate / ((1 + L_j)^2 |C_{L_j}(theta)|), i.e. the Bernstein bound
                              of App. A.7 on the Hessian as smoothness constant with gd_rate for
                              1 / B2; max_step and early_stop apply as for Newton, and the
                              INDEFINITE / SINGULAR flags are never set. */
} matcha_march_cfg;

/* Launch shapes and tile shapes.  Zero fields mean "library default".  Results never depend on
 * them (every output is computed by the same arithmetic in the same order).
 *   march_nc: candidates per wavefront of the march kernel (1, 2, 4 or 8; a workgroup holds
 *     ceil(Kc / march_nc) <= 8 waves).
 *   soft_threads: threads per workgroup of the SOFFT ranking kernel (256 or 512; each particle's
 *     maxima list holds twice as many keys).
 *   asm_tiles: 16-row output tiles per wave and workgroup of the assembly (1, 2, 4 or 8;
 *     default 4).
 *   grid_nodes: polar nodes per wave of the register-resident SOFFT grid kernel (8, 16, 32, 48 or 64;
 *     default 16).
 *   march_persistent: 1 launches the march as a persistent grid (as many workgroups as are resident
 *     at once, each taking the next particle from a counter in the workspace); 0 (default): one
 *     workgroup per particle, started by the hardware in batch order. */
typedef struct {
    int32_t march_nc;
    int32_t soft_threads;
    int32_t asm_tiles;
    int32_t grid_nodes;
    int32_t march_persistent;
} matcha_tuning;

/* ---- context ---------------------------------------------------------- */
/* Creates a context on HIP device `device` and builds its recurrence tables for every degree up
 * to MATCHA_MAX_L (synchronous).  tune_cache (host, nullable): path of a text file of autotune
 * results, read now if it exists; matcha_autotune looks results up there before timing anything
 * and adds what it measures.  out receives the handle. */
matcha_status matcha_create(int device, const char *tune_cache, matcha_ctx **out);
/* Waits for the device, then frees the context's tables.  Graphs made on it must be destroyed
 * first. */
matcha_status matcha_destroy(matcha_ctx *ctx);
/* Builds the SOFFT node tables of band B on an n_grid^3 grid (1 <= B <= 32, 4 <= n_grid <= 96),
 * kept until matcha_destroy; searches with a (B, n_grid) not prepared return
 * MATCHA_ERR_NOT_PREPARED.  Synchronous; repeated calls with a prepared shape do nothing. */
matcha_status matcha_prepare(matcha_ctx *ctx, int32_t B, int32_t n_grid);
const char *matcha_status_string(matcha_status s);
/* Sets / reads the launch shapes used by later calls on this context. */
matcha_status matcha_set_tuning(matcha_ctx *ctx, const matcha_tuning *t);
matcha_status matcha_get_tuning(const matcha_ctx *ctx, matcha_tuning *t);

/* ---- sizes -------------------------------------------------------------- */
/* Complex values of one particle's wedge-layout C for band limit L:
 * 2 * (L+1)(L+2)(2L+3)/6.  Returns -1 if L is outside [0, MATCHA_MAX_L]. */
int64_t matcha_c_elems(int32_t L);
/* Complex values of one particle's f: R (L+1)^2. */
int64_t matcha_f_elems(int32_t L, int32_t R);
/* Bytes of workspace with which the forward path's calls on this batch run in one pass: the
 * maximum of
 *   matcha_coeff_assemble: P int32 (the particle order by L_p) when the L_p differ, else 0;
 *   matcha_soft_search (soft non-NULL): per particle n^3 floats of grid, n (B+1)(2B+1) complex
 *     node transforms and 1024 maxima keys (575 KB at B = 12, n_grid = 48), for as many particles
 *     as fit in 4 GiB;
 *   matcha_march_newton: 256 bytes (the work counter of the persistent launch);
 *   matcha_evaluate: none.
 * Returns 0 for an empty or invalid batch.  ctx and march may be NULL. */
size_t matcha_workspace_size(const matcha_ctx *ctx, const matcha_batch *batch, const matcha_soft_cfg *soft,
                             const matcha_march_cfg *march);
/* Bytes of workspace of matcha_grad_template with grad_h requested: P int64 offsets (256-byte
 * aligned), S partial template gradients of R_h (L_h+1)^2 complex float32 (256-byte aligned; the
 * particles are summed in S consecutive segments, S = min(64, P, ceil(2048 / ceil(R_h (L_h+1)^2 /
 * 256)))), and one template-gradient term of R_p (L_p+1)^2 complex float32 per particle.  0 for an
 * empty or invalid batch. */
size_t matcha_grad_workspace_size(const matcha_batch *batch);

/* Longest-processing-time order (host): particle indices sorted by decreasing march cost
 * Kc * steps * sum over the particle's schedule of (L_j+1)(L_j+2)(2L_j+3)/6, ties by index. */
matcha_status matcha_lpt_order(const matcha_batch *batch, const matcha_march_cfg *cfg, int32_t *order_host);

/* Wedge layout -> packed-by-l layout (host, for callers that want C^l as full matrices):
 * C_wedge [matcha_c_elems(L)] complex float32 of one particle, C_byl [sum_{l<=L} (2l+1)^2]
 * complex float32; the half not stored is filled from C^l_{-m,-n} = (-1)^{m-n} conj(C^l_mn). */
matcha_status matcha_c_unpack(int32_t L, const float *C_wedge_host, float *C_byl_host);

/* ---- the path ------------------------------------------------------------ */
/* Coefficient assembly, eq. sigmalmm (Sec. 2.1, App. A.5) with shells in place of
 * the radial index:  C^l_mn = sum_{r < R_p} w_r f_lm(r) conj(h_ln(r)), l <= L_p.
 * f, h: complex float32 (MATCHA_FP32) or complex bfloat16 (MATCHA_BF16_FP32ACC,
 * interleaved (re, im) bf16 pairs); w: float32 [R_h]; C: complex float32, wedge
 * layout.  Accumulation is FP32 in both modes.  The template's degree-L_max row over
 * R_max = max_p R_p shells is staged in one workgroup's LDS: MATCHA_ERR_UNSUPPORTED when
 * 8 R_max 16 ceil((2 L_max + 1) / 16) bytes (FP32; BF16: 4 (2 R_max rounded up to 32, + 8)
 * 16 ceil((2 L_max + 1) / 16)) exceed 160 KB, e.g. R_max > 142 at L_max = 64 in FP32.
 * When the L_p differ, a first kernel orders the particles by decreasing L_p into the head of
 * ws (P int32; MATCHA_ERR_WORKSPACE if ws_bytes is smaller), so that the rows of degree l cover
 * only the particles with L_p >= l; results do not depend on that order.  With equal L_p, ws
 * may be NULL. */
matcha_status matcha_coeff_assemble(matcha_ctx *ctx, const matcha_batch *batch, const void *f, const void *h,
                                    const float *w, float *C, matcha_precision prec, void *ws, size_t ws_bytes,
                                    void *stream);

/* SOFFT search at band B (Sec. 2.3; the search step of Alg. 1): evaluates C_B on the
 * n_grid^3 grid (Wigner-d transform over l, then a 2-D inverse DFT over (a, c)),
 * finds the nodes that beat all 26 neighbours (a, c periodic; b neighbours outside
 * the grid absent; equal values: the smaller linear index i n^2 + j n + k wins),
 * ranks them by (value desc, index asc) and writes the first Kc to cand
 * [P][Kc] float4 (a_j, b_i, c_k, value).  With fewer than Kc maxima the list is
 * filled with the best remaining nodes and MATCHA_ST_FEW_MAXIMA is set.
 * status [P] is overwritten.  Requires 1 <= B <= min_p L_p, 1 <= Kc <= MATCHA_MAX_KC and
 * (B, n_grid) prepared (MATCHA_ERR_UNSUPPORTED if the shape does not fit a workgroup's LDS).
 * The node transforms, the grid and the maxima lists of each particle pass through ws; the
 * batch runs in chunks of as many particles as ws holds (MATCHA_ERR_WORKSPACE below one
 * particle's share, see matcha_workspace_size). */
matcha_status matcha_soft_search(matcha_ctx *ctx, const matcha_batch *batch, const float *C,
                                 const matcha_soft_cfg *cfg, float *cand, uint32_t *status, void *ws, size_t ws_bytes,
                                 void *stream);

/* Frequency-marched Newton refinement and selection (the march and selection steps of
 * Alg. 1, Sec. 2.2):
 * for every candidate, M_iter Newton steps theta <- theta - H^{-1} grad C_L on
 * each level of the particle's schedule, the 3x3 system inverted explicitly in
 * FP64; then C_{L_p} at each final point, and the candidate with the largest value
 * (ties: lowest index; non-finite values never win).
 * cand [P][Kc] float4 in/out: in = start points, out = (final angles, C_{L_p}).
 * best [P] float4 (a, b, c, C_{L_p}) of the selected candidate; best_idx [P];
 * status [P] in/out: the selected candidate's bits are OR-ed into it.  The persistent launch
 * (matcha_tuning.march_persistent) keeps its work counter in the first 4 bytes of ws
 * (MATCHA_ERR_WORKSPACE below 256 bytes); otherwise ws may be NULL. */
matcha_status matcha_march_newton(matcha_ctx *ctx, const matcha_batch *batch, const float *C,
                                  const matcha_march_cfg *cfg, int32_t Kc, float *cand, float *best,
                                  int32_t *best_idx, uint32_t *status, void *ws, size_t ws_bytes, void *stream);

/* Objective only: value, gradient and Hessian of C_{L_eval} at one rotation per
 * particle.  theta [P] float4 (a, b, c, unused); out [P][10] float:
 * F, F_a, F_b, F_c, F_aa, F_ab, F_ac, F_bb, F_bc, F_cc (Sec. 2.2, App. A.4).
 * 1 <= L_eval <= L_p for every particle, or L_eval = 0 for each particle's own L_p. */
matcha_status matcha_evaluate(matcha_ctx *ctx, const matcha_batch *batch, const float *C, int32_t L_eval,
                              int32_t fp64_above, const float *theta, float *out, void *stream);

/* Adjoint of sum_p g_p C_{L_p}(R_p*) at fixed rotations R_p* = best[p]
 * (envelope theorem), as d/dRe + i d/dIm of the full complex arrays:
 *   grad_h[r][l,n] = sum_p g_p w_r sum_m f_p,lm(r) conj(D^l_mn(R_p*))
 *   grad_f_p[r][l,m] = g_p w_r sum_n D^l_mn(R_p*) h_ln(r)
 * grad_h: complex float32 [R_h][(L_h+1)^2] (entries outside every particle's
 * range are zeroed); grad_f: same layout as f; either may be NULL.  prec: MATCHA_FP32 only
 * (MATCHA_ERR_UNSUPPORTED otherwise).  The sum over particles is deterministic (within each of S
 * consecutive segments of particles in index order, then the segments in order; no floating-point
 * atomics); each particle's term passes through ws (packed in the
 * library's own order, whatever f_offset is; MATCHA_ERR_WORKSPACE if ws_bytes is below
 * matcha_grad_workspace_size when grad_h is requested). */
matcha_status matcha_grad_template(matcha_ctx *ctx, const matcha_batch *batch, const float *f, const float *h,
                                   const float *w, const float *best, const float *g, float *grad_h, float *grad_f,
                                   matcha_precision prec, void *ws, size_t ws_bytes, void *stream);

/* SOFFT search for callers that cannot allocate (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): the kernels and results of matcha_soft_search, with its
 * workspace taken from a static device array of MATCHA_NOALLOC_SCRATCH_BYTES that each device the
 * library runs on holds from library load until the process ends (its address is looked up once per
 * device by matcha_create).  The caller still passes C, cand and status.  The batch runs in chunks
 * of as many particles as the array holds; a shape whose one-particle share exceeds it returns
 * MATCHA_ERR_WORKSPACE (the largest shape the search accepts, B = 32 on a 96^3 grid, needs
 * 5.2 MB).  Every call on a device shares that device's array and leaves its contents behind
 * (each call writes what it reads before reading it): calls that overlap in time on one device
 * (other streams, other contexts, other threads) race, so the caller must order them.  Calls
 * no hipMalloc, hipFree or allocating routine. */
#define MATCHA_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
matcha_status matcha_soft_search_noalloc(matcha_ctx *ctx, const matcha_batch *batch, const float *C,
                                         const matcha_soft_cfg *cfg, float *cand, uint32_t *status, void *stream);

/* ---- low-rank structure of the correlation blocks ------------------------- */
/* App. A.6 and B.1: per particle and degree l <= L_p the singular values of the block
 * C^l = sum_r w_r f_l(r) h_l(r)^H (eq. Alpha_l_factorization with shells for the radial index: rank at
 * most R_p, eq. rank_bound, and unchanged by rotating h) and its effective rank
 *     r_eff(l) = min { k >= 1 : s_{k+1} / s_k < rho }
 * (the paper uses rho = 0.2; the number of values min(2l+1, R_p) when no ratio falls below rho; 0
 * for a zero block).  Computed in FP64 from the R_p x R_p Gram matrices of the shells (pivoted
 * Cholesky factors X_F, X_H; the singular values of X_F^H X_H by one-sided Jacobi), one wave per
 * (particle, degree).  f, h, w as for matcha_coeff_assemble in FP32.  Outputs (device):
 * sv [P][L_max+1][n_sv] float64, descending, zero-padded (entries beyond min(2l+1, R_p) and
 * degrees above L_p are 0); r_eff [P][L_max+1] int32.  1 <= n_sv <= 64, 0 < rho < 1.
 * MATCHA_ERR_UNSUPPORTED when max R_p > MATCHA_LOWRANK_MAX_SHELLS (the LDS holds three
 * R_p x R_p complex FP64 matrices). */
#define MATCHA_LOWRANK_MAX_SHELLS 48
matcha_status matcha_lowrank_spectrum(matcha_ctx *ctx, const matcha_batch *batch, const float *f, const float *h,
                                      const float *w, double rho, int32_t n_sv, double *sv, int32_t *r_eff,
                                      void *stream);

/* ---- translation search and the rotation-translation alternation (App. C) --- */
/* The 6-D problem maximises <f, g o S_tau h> over rotations g and shifts tau, (S_tau h)(x) = h(x - tau),
 * by alternating the path (rotations at a fixed shift) with an FFT cross-correlation (shifts at a
 * fixed rotation), T times from zero shift.  Written with s = g tau, the pose is f = S_s (g o h):
 * the rotation step aligns f(x + s) to h (so the template, shared by the batch, never moves), and
 * the translation step maximises c(s) = sum_x f(x) (g o h)(x - s), (g o h)(x) = h(R_g^T x), the
 * rotated template resampled by trilinear interpolation.  c is evaluated on the integer shifts by
 * inverse FFT of F conj(U), the best one within a window is refined by an upsampled DFT around it
 * (+-0.75 voxel at 1/upsample steps: the efficient upsampled correlation the paper cites), and the
 * shift is returned in voxels along (x, y, z).  tau = R_g^T s.
 * Volumes: float32 [n][N][N][N], x fastest; spectra: the unnormalised forward transform's half
 * plane, complex float32 [n][N][N][N/2+1]; shifts and rotations: float4 per volume, (x, y, z, .) and
 * (a, b, c, .) (the march's best has this layout).  FFTs are hipFFT plans made by matcha_fft_prepare
 * for one (N, n) and kept until matcha_destroy; their work area comes from the caller's workspace.
 * Calls on one context share those plans and must be ordered. */
#define MATCHA_TRANSLATE_MAX_N 256
#define MATCHA_TRANSLATE_MAX_UPSAMPLE 40

/* Plans for n_volumes N^3 volumes (N even, 4 <= N <= MATCHA_TRANSLATE_MAX_N); idempotent. */
matcha_status matcha_fft_prepare(matcha_ctx *ctx, int32_t N, int32_t n_volumes);
/* Workspace bytes of the translation calls for a prepared (N, n_volumes) and an upsampling factor
 * (1 for matcha_volume_spectrum and matcha_shift_volumes); 0 if not prepared. */
size_t matcha_translate_workspace_size(const matcha_ctx *ctx, int32_t N, int32_t n_volumes, int32_t upsample);
/* spec = the forward transforms of vol (device). */
matcha_status matcha_volume_spectrum(matcha_ctx *ctx, int32_t N, int32_t n_volumes, const float *vol, float *spec,
                                     void *ws, size_t ws_bytes, void *stream);
/* out_p(x) = f_p(x + s_p) from f_p's spectrum (cyclic, Nyquist planes dropped): the particles as the
 * rotation step sees them. */
matcha_status matcha_shift_volumes(matcha_ctx *ctx, int32_t N, int32_t n_volumes, const float *spec,
                                   const float *shifts, float *out, void *ws, size_t ws_bytes, void *stream);
/* The translation step: for each volume, the shift s (|s_i| <= window for the integer search, then
 * the upsampled refinement) maximising sum_x f_p(x) h(R_p^T (x - s)); shift_out = (s_x, s_y, s_z, c(s)).
 * spec_f: the particles' spectra; h: device float32 [N^3]; euler: float4 [n] rotations.
 * MATCHA_ERR_UNSUPPORTED when the refinement's tables exceed 64 KB of LDS or n_volumes > 65535. */
matcha_status matcha_translation_search(matcha_ctx *ctx, int32_t N, int32_t n_volumes, const float *spec_f,
                                        const float *h, const float *euler, int32_t window, int32_t upsample,
                                        float *shift_out, void *ws, size_t ws_bytes, void *stream);

/* ---- ball-harmonic front end ---------------------------------------------- */
/* The step before the path (App. A.1): coefficients of real volumes in the ball-harmonic
 * (Fourier-Bessel) basis of the unit ball, psi_klm(x) = c_lk j_l(lam_lk |x|) Y_lm(x / |x|), with
 * lam_lk the k-th positive zero of the spherical Bessel function j_l, c_lk = sqrt(2) / |j_{l+1}(lam_lk)|
 * (orthonormal on the ball), Y_lm orthonormal with the Condon-Shortley phase, and the index set
 * I_Lambda = {(k, l, m): lam_lk <= Lambda}: |K_l| radial indices at degree l, falling with l, up to
 * the largest degree L with a zero <= Lambda.  A volume is N^3 samples at the voxel centres
 * -1 + (2/N)(i + 1/2) per axis (the ball inscribed in the grid), float32 [N][N][N] with x fastest,
 * then y, then z; its coefficients are the voxel-sum inner products
 *     u_klm = (2/N)^3 sum over the voxels with |x_v| < 1 of u(x_v) conj(psi_klm(x_v)),
 * computed exactly (no fast transform; the error against the continuous inner product is the
 * quadrature's, O(1/N) for a volume with a jump at the sphere).  Output layout:
 * [n_volumes][Kmax][(L+1)^2] complex float32 (packed lm = l^2 + l + m), zero where k >= |K_l|:
 * the per-shell layout of f and h with R = Kmax shells, so the path takes it directly with unit
 * shell weights (then C^l_mn is the paper's sigma_lmn summed over K_l). */
#define MATCHA_BALL_MAX_L 63
#define MATCHA_BALL_MAX_LAMBDA 71.0
#define MATCHA_BALL_MAX_N 256
#define MATCHA_BALL_MAX_TABLE_BYTES ((size_t)16 << 30)

/* The index set of Lambda (host only, FP64 zeros by bracketing and bisection): *L, *Kmax = |K_0|;
 * nk_l (optional, >= L + 1 entries) = |K_l|; zeros (optional, [L+1][Kmax], zero-padded) = lam_lk.
 * Pass NULL for both to learn L and Kmax first.  MATCHA_ERR_INVALID_ARG unless
 * pi <= Lambda <= MATCHA_BALL_MAX_LAMBDA (below pi, the first zero of j_0, the set is empty);
 * MATCHA_BALL_MAX_LAMBDA keeps L <= 62, within MATCHA_BALL_MAX_L. */
matcha_status matcha_ball_index(double Lambda, int32_t *L, int32_t *Kmax, int32_t *nk_l, double *zeros);

/* Builds the transform's tables for an N^3 grid and Lambda (host FP64, rounded to FP32) and keeps
 * them on the context's device until matcha_destroy.  The grid's mirrors x -> -x, y -> -y, z -> -z
 * permute the voxels, and every real column function (Re and Im of conj psi_klm) is even or odd
 * under each, so the sum is taken over one octant: the table holds, per column and octant voxel,
 * (2/N)^3 conj psi_klm / (the number of mirrors that fix the voxel), about
 * 4 N^3 / 16 sum_l |K_l| (2l + 1) bytes (Lambda = 38, N = 64: 3476 columns, 0.24 GB).  Idempotent
 * per (N, Lambda).  MATCHA_ERR_INVALID_ARG unless 2 <= N <= MATCHA_BALL_MAX_N and Lambda is accepted
 * by matcha_ball_index; MATCHA_ERR_UNSUPPORTED above MATCHA_BALL_MAX_TABLE_BYTES. */
matcha_status matcha_ball_prepare(matcha_ctx *ctx, int32_t N, double Lambda);

/* Workspace bytes of matcha_ball_transform for n_volumes volumes on a prepared (N, Lambda): the
 * sign-symmetrised volumes (8 x n_volumes x the octant voxel count, float32) and the K-split
 * partial sums (up to 16 x n_volumes x the column count, float32); 0 if (N, Lambda) is not prepared
 * or n_volumes <= 0. */
size_t matcha_ball_workspace_size(const matcha_ctx *ctx, int32_t N, double Lambda, int32_t n_volumes);

/* u: device float32 [n_volumes][N][N][N]; coef: device, [n_volumes][Kmax][(L+1)^2] complex float32
 * (8-byte aligned), every entry written (u_{k,l,-m} = (-1)^m conj(u_klm) for real volumes); ws:
 * device, 16-byte aligned, at least matcha_ball_workspace_size bytes (MATCHA_ERR_WORKSPACE
 * otherwise).  Three kernels on the stream: the 8 sign-symmetrised copies of each volume on the
 * octant, one product per sign class on the matrix cores (rows = volumes, columns = the class's
 * (l, k, m, Re / Im), FP32 inputs and accumulation, in up to 16 partial sums over voxel ranges),
 * and the sum of the partials scattered into the output layout.  The split count depends on
 * n_volumes and the device's compute-unit count only, so results are reproducible bit for bit on
 * one device.  n_volumes = 0 does nothing; MATCHA_ERR_NOT_PREPARED if matcha_ball_prepare(ctx, N,
 * Lambda) has not run. */
matcha_status matcha_ball_transform(matcha_ctx *ctx, int32_t N, double Lambda, int32_t n_volumes, const float *u,
                                    float *coef, void *ws, size_t ws_bytes, void *stream);

/* ---- batching: graphs and tuning ------------------------------------------ */
typedef struct matcha_graph matcha_graph;

/* Buffers of the whole path.  f, h, w, prec: the assembly's inputs, into C.  f32 / h32 (both
 * or neither; FP32, used with prec = MATCHA_BF16_FP32ACC): inputs of an FP32 assembly into C32
 * that the march uses for each particle's final level (matcha_march_cfg.C_final). */
typedef struct {
    const void *f, *h;
    const float *w;
    matcha_precision prec;
    const float *f32, *h32;
    float *C, *C32;
    float *cand, *best;
    int32_t *best_idx;
    uint32_t *status;
} matcha_align_bufs;

/* Records matcha_coeff_assemble (twice with f32 / h32) + matcha_soft_search +
 * matcha_march_newton for these exact buffers and workspace into a HIP graph (captured on a
 * private stream) and instantiates it.  Later replays run the whole path with one launch call
 * and read the buffers' contents at replay time; the buffers and ws must outlive the graph, and
 * the context must outlive it too.  (soft->B, soft->n_grid) must be prepared.  march->C_final is
 * ignored (C32 takes its place).  Synchronous. */
matcha_status matcha_align_graph_create(matcha_ctx *ctx, const matcha_batch *batch, const matcha_align_bufs *bufs,
                                        const matcha_soft_cfg *soft, const matcha_march_cfg *march, void *ws,
                                        size_t ws_bytes, matcha_graph **out);
/* Replays the graph on `stream` (asynchronous). */
matcha_status matcha_graph_launch(matcha_graph *g, void *stream);
matcha_status matcha_graph_destroy(matcha_graph *g);

/* Autotuner: when the context's tune cache holds a result for this device, batch shape and
 * configuration, applies it and returns it without timing.  Otherwise times, on this batch
 * (hipEvents, `reps` repetitions after one warm-up, in two interleaved rounds of which each value
 * keeps its faster), one field of matcha_tuning at a time with
 * the others at their best so far: the assembly's row tiles per wave (bufs->f, h, w, prec into
 * bufs->C), the SOFFT ranking workgroup and grid-kernel nodes per wave, then the march's candidates
 * per wave and launch form (each march trial re-runs the search so that it starts from fresh
 * candidates); keeps the fastest in the context (later calls use it), adds it to the tune cache
 * file and returns it in *best_tuning (host).  bufs->C, cand, best, best_idx and status hold the
 * last trial's (valid) results; bufs->f32 / h32 / C32 are not used.  Synchronous. */
matcha_status matcha_autotune(matcha_ctx *ctx, const matcha_batch *batch, const matcha_align_bufs *bufs,
                              const matcha_soft_cfg *soft, const matcha_march_cfg *march, int32_t reps, void *ws,
                              size_t ws_bytes, matcha_tuning *best_tuning);

#ifdef __cplusplus
}
#endif
#endif /* MATCHA_H */
