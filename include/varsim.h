/*
 * varsim.h -- C ABI of the MI355X (gfx950) steady and transient chip-temperature solve.
 *
 * The solve follows VarSim (Sultan & Sarangi, arXiv 2307.12119):
 *   - the temperature rise is the power map convolved with the die's Green's function
 *     (Sec. II-B, Eq. Green), the die edges handled by mirror-image sources (Sec. IV-F);
 *   - total power is dynamic plus leakage, leakage grows with temperature and is scaled by
 *     the process-variation map (Sec. II-D, Eqs. Ileakmod, Pleak, Pt);
 *   - conductivity follows k = k0 (T/300)^-eta (Sec. II-E, Eq. condsi) and a spatial
 *     conductivity-variation map scales the Green's function as 1/k (Eq. fspvsk);
 *   - leakage and conductivity are iterated against temperature until convergence, the
 *     ground truth of Sec. V-C;
 *   - transients use the single-pole transient Green's function (Eq. tranGreen), or the slab's
 *     multi-pole response, superposed over a piecewise-constant power history (Eq. tranapprox),
 *     whole or truncated after a horizon as in Sec. IV-E;
 *   - optionally: a package stack below the die (Table param), the one-shot leakage-aware
 *     Green's functions (Sec. IV-C, Eqs. detsol, randsol, detrandsol), Anderson(1) mixing of
 *     the fixed point, FP32 transforms with compensated twiddles.
 *
 * Conventions shared by every entry point
 *   - SI units throughout: metres, watts, kelvin, seconds; power maps are densities in W/m^2.
 *   - Maps are DEVICE pointers, row-major [ny][nx], contiguous, element type given by
 *     varsim_options.precision (float for VARSIM_F32, double for VARSIM_F64).
 *   - Outputs are the temperature RISE dT above the ambient temperature, never absolute T.
 *   - The caller owns every map and the workspace; the library never frees caller memory.
 *     The context owns only its caches (Green's-function tables, twiddle tables, timing).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Work is
 *     stream-ordered; calls that return statistics synchronise that stream before returning.
 *   - A context is not thread-safe: use one context per host thread.
 *   - Supported grids: nx and ny powers of two in [16, 1024], ny a multiple of the row pass's
 *     rows per workgroup (which excludes 32 x 16, 64 x 16, 64 x 32 and 128 x 16); the die is
 *     the first layer, optionally above a package stack of up to 8 layers with an isothermal or
 *     convective bottom (steady solves; transients take one square layer over an isothermal
 *     bottom).  Anything else is VARSIM_ERR_UNSUPPORTED.
 *
 * Errors: every entry point returns a varsim_status; on failure varsim_last_error() holds a
 * message.  Device failures (launch or runtime errors) return VARSIM_ERR_DEVICE.
 */
#ifndef VARSIM_H
#define VARSIM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define VARSIM_API __attribute__((visibility("default")))
#else
#define VARSIM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum varsim_status {
  VARSIM_OK = 0,
  VARSIM_ERR_INVALID = 1,        /* NULL required pointer, non-positive size, m <= 0, tol <= 0, ... */
  VARSIM_ERR_UNSUPPORTED = 2,    /* grid, layer stack or boundary outside the supported set */
  VARSIM_ERR_NOT_CONVERGED = 3,  /* max_iter reached; dT_out holds the last iterate, stats valid */
  VARSIM_ERR_RUNAWAY = 4,        /* non-finite iterate, dT above dT_cap_K, or the conductivity law
                                    left its domain: no stable fixed point (thermal runaway) */
  VARSIM_ERR_DEVICE = 5,         /* HIP runtime or launch failure */
  VARSIM_ERR_NO_MEMORY = 6       /* workspace too small, or a context cache allocation failed */
} varsim_status;

enum { VARSIM_LEAK_NONE = 0, VARSIM_LEAK_EXP = 1, VARSIM_LEAK_LINEAR = 2 };
enum { VARSIM_F32 = 0, VARSIM_F64 = 1 };
/* Transient time constants per cosine mode: MOMENT -- one pole with the exact first moment of
 * the slab's response; LUMPED -- one pole with the paper's tau = C F(f_sp0), C = rho c t / 3;
 * MODAL -- the slab's slowest depth modes as separate poles (n_poles - 1 of them) plus one
 * lumped pole keeping the first moment (n_poles = 1 is MOMENT). */
enum { VARSIM_TAU_MOMENT = 0, VARSIM_TAU_LUMPED = 1, VARSIM_TAU_MODAL = 2 };
/* Where the conductivity-variation factor 1/m acts (Eq. fspvsk read as a Hadamard factor):
 *   SOURCE: theta = K (*) (P / m) -- each source's heat spreads with its own cell's conductivity;
 *   TARGET: theta = (K (*) P) / m -- the target cell's conductivity scales its rise.
 * Both are exact for a uniform m.  Against a finite-volume solve of the heat equation with a
 * +-5 % conductivity map the source placement's error is about a quarter of the target's. */
enum { VARSIM_COND_SOURCE = 0, VARSIM_COND_TARGET = 1 };

typedef struct varsim_ctx varsim_ctx;

/* One material layer (Table param gives the paper's stack: silicon, TIM, heat spreader). */
typedef struct varsim_layer {
  double thickness_m;   /* t, > 0 */
  double k0_W_mK;       /* conductivity at 300 K, > 0 (Eq. condsi) */
  double eta;           /* exponent of k = k0 (T/300)^-eta, >= 0 */
  double rho_c_J_m3K;   /* volumetric heat capacity, > 0 (transient only) */
} varsim_layer;

/* Die geometry and boundary (Sec. V-A: a die of lx x ly discretised on an nx x ny grid).
 * Power enters the top face of layer 0 (the silicon); the layers below it (the package of
 * Table param, Sec. II-B's f_sp = f_silic + const) share the die's lateral extent and
 * adiabatic side walls, each with the constant conductivity k0 (T_amb / 300)^-eta.  The stack
 * enters the solve through the exact surface impedance of the layers (Eq. fourier layer by
 * layer) added to the silicon slab's cosine eigenvalues; k(T) (the Kirchhoff inverse) uses
 * layer 0's law, which is exact for one layer over an isothermal bottom and an approximation
 * otherwise. */
typedef struct varsim_geometry {
  double lx_m, ly_m;            /* die size, > 0 */
  int32_t nx, ny;               /* grid (see the supported grids above) */
  int32_t n_layers;             /* 1..8 */
  const varsim_layer* layers;   /* host pointer, n_layers entries, top first */
  int32_t bottom_bc;            /* 0 = bottom face isothermal at t_amb_K; 1 = convective to t_amb_K */
  double h_bottom_W_m2K;        /* heat-transfer coefficient of the convective bottom, > 0 */
  double t_amb_K;               /* ambient temperature, > 0 */
} varsim_geometry;

/* Solver options.  Zero-initialised fields are invalid: fill every field. */
typedef struct varsim_options {
  int32_t leak;                 /* VARSIM_LEAK_EXP: L = exp(beta dT); LINEAR: 1 + beta dT (Eq. Pleak) */
  double beta_per_K;            /* leakage temperature coefficient */
  int32_t sv_radius;            /* shift-variant stencil radius; only 0 (pointwise 1/m) supported */
  int32_t precision;            /* VARSIM_F32 or VARSIM_F64: element type of every map */
  int32_t max_iter;             /* >= 1, <= 1000 */
  double tol_K;                 /* stop at the first iterate with max |dT_k - dT_{k-1}| <= tol, > 0 */
  double dT_cap_K;              /* RUNAWAY when any dT exceeds it, > 0 (1000 K is a sane value) */
  int32_t final_f64_residual;   /* 1: report max |G64(dT) - dT| from one FP64 application */
  int32_t cond_model;           /* VARSIM_COND_SOURCE or VARSIM_COND_TARGET (placement of 1/m) */
  int32_t compensated_twiddles; /* 0 or 1.  1: the FP32 transforms of the fixed-point passes of
                                   varsim_solve_steady / _batch / _batch_noalloc hold every
                                   twiddle and butterfly constant as an FP32 pair hi + lo and add
                                   the product with lo, removing the constants' own rounding from
                                   the result (maps of any size then take the two-pass path).
                                   Ignored by FP64 solves, the one-shot and transient solves. */
  int32_t anderson;             /* 0: plain Picard iteration.  1: Anderson mixing with one stored
                                   difference (a classical acceleration, not from the paper):
                                   x_{k+1} = g_k - gamma_k (g_k - g_{k-1}), g_k = G(x_k),
                                   f_k = g_k - x_k, gamma_k = <f_k - f_{k-1}, f_k> /
                                   |f_k - f_{k-1}|^2 (sums over the map, FP64, fixed order), with
                                   the same stopping rule (max |G(x) - x| <= tol_K, result G(x)).
                                   Two row passes per iteration and three more maps of workspace
                                   per problem; maps of any size take the two-pass path.  Used by
                                   varsim_solve_steady / _batch / _batch_noalloc. */
} varsim_options;

/* One steady problem (all maps device pointers [ny][nx]; see conventions above). */
typedef struct varsim_problem {
  const varsim_geometry* geom;  /* host pointer */
  const void* q_dyn;            /* dynamic power density, W/m^2, required */
  const void* q_leak0;          /* leakage density at T_amb, W/m^2; NULL = no leakage */
  const void* leak_var;         /* variation multiplier v of leakage; NULL = 1 */
  const void* cond_map;         /* conductivity multiplier m (> 0); NULL = 1 */
  const void* dT_init;          /* starting iterate; NULL = 0; a non-finite entry falls back to 0 */
  void* dT_out;                 /* result dT (may alias dT_init) */
} varsim_problem;

/* Per-problem result statistics. */
typedef struct varsim_stats {
  int32_t status;               /* varsim_status of this problem */
  int32_t iterations;           /* applications of the fixed-point map performed */
  double last_increment_K;      /* max |dT_k - dT_{k-1}| of the last iteration */
  double residual_f64_K;        /* max |G64(dT) - dT| in FP64 (NaN when not requested) */
  double dT_max_K;              /* max of dT */
  double dT_mean_K;             /* mean of dT (FP64 accumulation in a fixed order: the same bits
                                   on every run) */
  int64_t hotspot_index;        /* row-major index of the max (lowest index on ties) */
  int32_t warm_start_rejected;  /* 1 when dT_init held a non-finite value and 0 was used */
  int32_t reserved;
} varsim_stats;

/* Transient description (Sec. IV-E, Eq. tranapprox): power held constant over each step. */
typedef struct varsim_transient {
  double dt_s;                  /* step length, > 0 */
  int32_t n_steps;              /* >= 1 */
  int32_t out_every;            /* write dT every out_every steps (>= 1) */
  int32_t n_blocks;             /* >= 1 */
  const int32_t* block_rects;   /* DEVICE [n_blocks][4] = x0, y0, w, h in cells; later blocks
                                   overwrite earlier ones where they overlap */
  const void* trace;            /* DEVICE [n_steps][n_blocks] dynamic power density of each block
                                   held over step n, W/m^2, element type = precision */
  int32_t tau_model;            /* VARSIM_TAU_MOMENT, VARSIM_TAU_LUMPED or VARSIM_TAU_MODAL */
  int32_t n_poles;              /* poles per mode of VARSIM_TAU_MODAL, in [1, 8] (ignored otherwise);
                                   each pole keeps its own spectral state (n_poles maps of
                                   workspace) and moves two more maps of state and coefficients
                                   per step */
  int32_t history_steps;        /* 0: the whole power history enters (exact per-mode recursion).
                                   h in [2, 2^20]: the truncated history of Sec. IV-E (the paper's
                                   5 ms horizon is h = 5 ms / dt_s): the step responses are taken as
                                   saturated from the h-th step on, so the rise at step n is
                                   sum_{j<h} S_j (*) (P_{n-j+1} - P_{n-j}) + S_inf (*) P_{n-h+1} and
                                   a power change is forgotten h steps after it.  Costs h - 1 maps
                                   of workspace (the spectra of the last h - 1 steps) plus
                                   n_poles + 1 coefficient maps, and moves 3 + n_poles more maps
                                   per step (n_poles = 1 but for VARSIM_TAU_MODAL) */
} varsim_transient;

/* ----------------------------------------------------------------------------------------
 * Context.  varsim_create makes `device` current, allocates nothing large, and returns a
 * context; varsim_destroy frees the context's caches.  Errors: INVALID (NULL out), DEVICE.
 */
VARSIM_API varsim_status varsim_create(int device, varsim_ctx** out);
VARSIM_API void varsim_destroy(varsim_ctx* ctx);
VARSIM_API const char* varsim_status_string(varsim_status s);
VARSIM_API const char* varsim_last_error(const varsim_ctx* ctx);

/* ----------------------------------------------------------------------------------------
 * Green's-function table (Sec. II-B Eq. Green; Appendix Theorem I; Sec. IV-F images).
 *
 * Tabulates in FP64 on the device the cell-averaged slab kernel K_per(a, b) of the die
 * (rise at the centre of cell (a, b) per watt spread over the cell at the origin, summed over
 * the mirror images of the side walls), a in [0, nx], b in [0, ny], and its cosine transform
 *     lambda[p][q] = sum_{a, b in (-n, n]} K_per(a, b) cos(pi p b / ny) cos(pi q a / nx)
 * which diagonalises the mirrored convolution.  The conductivity used is k(T_amb).
 *   kernel_out : DEVICE double [ny + 1][nx + 1], or NULL (must be NULL for a package stack,
 *                whose eigenvalues alone are tabulated: UNSUPPORTED otherwise)
 *   lambda_out : DEVICE double [ny][nx], or NULL (a stack's eigenvalues include its layers)
 * The table is also cached in the context for the solves.  Synchronises `stream`.
 * Errors: INVALID, UNSUPPORTED, DEVICE, NO_MEMORY.
 */
VARSIM_API varsim_status varsim_green_table(varsim_ctx* ctx, const varsim_geometry* geom, void* kernel_out,
                                 void* lambda_out, void* stream);

/* ----------------------------------------------------------------------------------------
 * Shift-invariant convolution (Eq. Green with the images of Sec. IV-F): for each of n_maps
 * power maps P (W per cell, DEVICE [n_maps][ny][nx], element type `precision`) writes
 * theta = K_per (*) P with images, computed as DCT-III(lambda . DCT-II(P)).
 * theta_out may alias power.  Synchronises `stream` before returning.
 * Errors: INVALID, UNSUPPORTED, DEVICE, NO_MEMORY.
 */
VARSIM_API varsim_status varsim_conv(varsim_ctx* ctx, const varsim_geometry* geom, int32_t precision,
                          const void* power, void* theta_out, int32_t n_maps, void* stream);

/* ----------------------------------------------------------------------------------------
 * Workspace size in bytes for solving `n` problems with `opts` (steady or batch).  The
 * caller allocates at least that much device memory (alignment 256 B) and passes it in.
 * Errors: INVALID, UNSUPPORTED.
 */
VARSIM_API varsim_status varsim_workspace_size(varsim_ctx* ctx, const varsim_problem* problems, int32_t n,
                                    const varsim_options* opts, size_t* bytes);

/* ----------------------------------------------------------------------------------------
 * Steady solve of one problem: the fixed point dT = G(dT) of
 *   P     = hx hy [q_dyn + q_leak0 v L(dT)]                  (Eqs. Pt, Pleak)
 *   theta = K_per (*) (P / m)  or  (K_per (*) P) / m         (Eqs. Green, fspvsk; cond_model)
 *   G(dT) = Phi^-1(theta), Phi the Kirchhoff transform of k(T) (Eq. condsi)
 * by Picard iteration from dT_init (or 0) to the first increment <= tol_K.
 * Writes dT_out and *stats (host pointer).  Synchronises `stream`; returns stats->status.
 * Errors: INVALID, UNSUPPORTED, NOT_CONVERGED, RUNAWAY, DEVICE, NO_MEMORY.
 */
VARSIM_API varsim_status varsim_solve_steady(varsim_ctx* ctx, const varsim_problem* problem,
                                  const varsim_options* opts, void* workspace, size_t ws_bytes,
                                  varsim_stats* stats, void* stream);

/* ----------------------------------------------------------------------------------------
 * Batched steady solve (Monte Carlo over variation samples, Sec. I): n problems, possibly of
 * different grid sizes and possibly sharing input pointers, solved together; each problem
 * stops at its own convergence.  stats: an array of n entries, in host or device memory.
 *   - Host memory: the call synchronises `stream`, fills stats and returns the worst status.
 *   - Device memory (hipMalloc): the call returns once the last kernels are enqueued (it still
 *     follows the convergence loop on the host); stats is written on `stream`, in the caller's
 *     order, and the return value reports only argument and device errors, not the per-problem
 *     statuses.  The workspace must not be reused by another stream before that point.
 * Consecutive calls of one context may use different streams (calls are made from one host
 * thread at a time); each call in flight needs its own workspace and outputs.  A call waits
 * for the previous call's last convergence counts before reusing the context's count words.
 */
VARSIM_API varsim_status varsim_solve_batch(varsim_ctx* ctx, const varsim_problem* problems, int32_t n,
                                 const varsim_options* opts, void* workspace, size_t ws_bytes,
                                 varsim_stats* stats, void* stream);

/* ----------------------------------------------------------------------------------------
 * Batched steady solve that allocates nothing, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * problems, options, statistics and results as varsim_solve_batch (the same kernels, bitwise
 * equal outputs), with the workspace taken from a static device array of
 * varsim_noalloc_scratch_bytes() bytes (32 MiB) that each GPU holds until the process ends:
 * one 1024 x 1024 map of any precision with both variation maps and the FP64 residual fits.
 * The call makes no hipMalloc / hipFree, so:
 *   - every geometry of the batch must already have its Green's table in the context's cache
 *     (varsim_green_table, or an earlier allocating solve of the same geometry), else INVALID;
 *   - the column strip width is the tuned one if the context has it, else the default (no
 *     timing of candidates); the fixed-point loop is launched directly (no graphs); kernel
 *     timing is suspended for the call.
 * The static array is shared by every call on that GPU and keeps the last call's contents (the
 * call clears what must start at zero).  Calls that overlap on one GPU -- from different streams,
 * threads or contexts -- race on it; calls on one stream are ordered and safe.  With device-side
 * stats the call returns before its last kernels run, so the next call must be on the same stream.
 * Errors: as varsim_solve_batch; NO_MEMORY when the batch's workspace exceeds the static array
 * (nothing is launched); DEVICE if the array's device address could not be looked up.
 */
VARSIM_API varsim_status varsim_solve_batch_noalloc(varsim_ctx* ctx, const varsim_problem* problems, int32_t n,
                                                    const varsim_options* opts, varsim_stats* stats, void* stream);
VARSIM_API varsim_status varsim_noalloc_scratch_bytes(size_t* bytes);

/* ----------------------------------------------------------------------------------------
 * One-shot solve with the paper's leakage-aware modified Green's functions (Sec. IV-C), no
 * iteration.  Leakage is linearised, q_leak0 v (1 + beta theta) (Eq. Pt), and the leakage per
 * unit conductivity multiplier is split into a uniform density mu and a remainder
 * r = q_leak0 v / m - mu (Eq. expanded2):
 *   deterministic part (Eqs. expanded3, detsol with alpha = 0): the operator (I - beta hx hy mu K)
 *     is diagonal in the cosine basis, so theta_det = DCT-III(lambda / (1 - beta hx hy mu lambda)
 *     . DCT-II(g)) with g = hx hy (q_dyn + q_leak0 v) / m;
 *   random part (Eq. randsol, first order in r): theta_rand = the same operator applied to
 *     beta hx hy r theta_det;
 *   total (Eq. detrandsol): dT = Phi^-1(theta_det + theta_rand), the Kirchhoff inverse of k(T)
 *     in place of the paper's empirical alpha (Eq. fspvsT).
 * The result approximates the fixed point of varsim_solve_steady (exactly equal to it for a
 * uniform leakage density, linear leakage and eta = 0); with final_f64_residual the stats report
 * its distance max |G64(dT) - dT| from that fixed point.  It also serves as dT_init of an
 * iterative solve.  The deterministic operator's table is built once per (geometry, beta mu) and
 * cached in the context (the paper's once-per-chip deterministic Green's function).
 *   problems, n, workspace, ws_bytes, stats, stream: as varsim_solve_batch (same workspace size;
 *     dT_init is not read); opts: as for the steady solve, but max_iter and tol_K are not used,
 *     leak NONE means beta = 0, and cond_model must be VARSIM_COND_SOURCE;
 *   stats: iterations = 0, last_increment_K = NaN; max, mean, hotspot and residual as usual.
 * Errors: INVALID, UNSUPPORTED (target-side conductivity), RUNAWAY (beta mu t / k_ref >= 1: the
 * linearised problem has no fixed point, or a non-finite / above-cap rise), DEVICE, NO_MEMORY.
 */
typedef struct varsim_oneshot {
  double mu_W_m2;        /* leakage density (W/m^2, per unit m) the deterministic part treats as uniform, >= 0 */
  int32_t random_part;   /* 1: add the first-order random part; 0: deterministic part only (ignoring f_rand) */
} varsim_oneshot;

VARSIM_API varsim_status varsim_solve_oneshot(varsim_ctx* ctx, const varsim_problem* problems, int32_t n,
                                              const varsim_options* opts, const varsim_oneshot* oneshot,
                                              void* workspace, size_t ws_bytes, varsim_stats* stats, void* stream);

/* ----------------------------------------------------------------------------------------
 * Transient solve (Eqs. Ttran, tranGreen, tranapprox).  Starting from dT = 0 at t = 0, step n
 * holds the block powers trace[n] over (t_{n-1}, t_n]; each spatial cosine mode responds with
 * a single pole, the leakage and conductivity of step n use dT_{n-1}.  Writes dT every
 * out_every steps into dT_steps_out (DEVICE [n_steps / out_every][ny][nx]) and the final
 * step's stats.  problem->q_dyn is ignored (the trace replaces it); problem->dT_out receives
 * the final dT.  Synchronises `stream`.
 * Errors: INVALID, UNSUPPORTED, RUNAWAY, DEVICE, NO_MEMORY.
 */
VARSIM_API varsim_status varsim_solve_transient(varsim_ctx* ctx, const varsim_problem* problem,
                                     const varsim_transient* tr, const varsim_options* opts,
                                     void* dT_steps_out, void* workspace, size_t ws_bytes,
                                     varsim_stats* stats, void* stream);

VARSIM_API varsim_status varsim_transient_workspace_size(varsim_ctx* ctx, const varsim_problem* problem,
                                              const varsim_transient* tr,
                                              const varsim_options* opts, size_t* bytes);

/* ----------------------------------------------------------------------------------------
 * Learned warm start.  The paper has no learned part (it argues against relying on learned
 * thermal models); this network only proposes a starting iterate.  It maps the steady
 * solve's own inputs -- dynamic power q, leakage variation v, conductivity map m and the die
 * conductivity k0 -- to a predicted converged rise, which is passed as varsim_problem.dT_init;
 * the fixed-point solve then decides the result, so a poor prediction costs iterations, not
 * accuracy.  The network: the 4 x 4 patches of the standardized features
 *     f = ((q / 1e6 - shift0) scale0, (ln v - shift1) scale1, (k0 m / 150 - shift2) scale2)
 * enter a 1x1 "stem" convolution on the n/4 grid, then a five-level encoder-decoder of 3x3
 * 'same' convolutions with ReLU (two per encoder level, 2x2 average pooling between levels;
 * one per decoder level on [nearest-2x-upsampled coarser output, encoder skip]), and a 1x1
 * head gives the 16 fine values of each coarse pixel, times out_scale.
 * Parameters (FP32, this order and layout; convolution weights [cout][ky][kx][cin]):
 *   stem.w [w0][48] (input index (py*4 + px)*3 + c), stem.b [w0];
 *   enc<l>a.w [wl][3][3][w(l-1) | w0 for l = 0], enc<l>a.b, enc<l>b.w [wl][3][3][wl], enc<l>b.b,
 *     l = 0..4;
 *   dec<l>.w [wl][3][3][w(l+1) + wl] (upsampled channels first), dec<l>.b, l = 3, 2, 1, 0;
 *   head.w [16][w0] (output (py*4 + px) of a coarse pixel), head.b [16].
 * Arithmetic: BF16 activations and weights on the matrix cores, FP32 accumulation, FP32 master
 * weights and Adam state.
 */
typedef struct varsim_net varsim_net;

typedef struct varsim_net_config {
  int32_t n;          /* input grid: a multiple of 64 in [64, 1024] */
  int32_t width[5];   /* channels of the five levels: multiples of 16 in [16, 256] */
  float shift[3];     /* feature standardisation (see above) */
  float scale[3];
  float out_scale;    /* predicted dT = out_scale * network output, K */
  float k0_W_mK;      /* die conductivity at 300 K */
} varsim_net_config;

/* Creates a network with all parameters zero (set them with varsim_net_set_params). */
VARSIM_API varsim_status varsim_net_create(varsim_ctx* ctx, const varsim_net_config* cfg, varsim_net** out);
VARSIM_API void varsim_net_destroy(varsim_net* net);
VARSIM_API varsim_status varsim_net_param_count(const varsim_net* net, int64_t* count);
/* params: DEVICE float[param_count].  set also resets the Adam state. */
VARSIM_API varsim_status varsim_net_set_params(varsim_net* net, const float* params, void* stream);
VARSIM_API varsim_status varsim_net_get_params(varsim_net* net, float* params, void* stream);
/* Workspace for a batch (training = 1: also the buffers of varsim_net_gradient). */
VARSIM_API varsim_status varsim_net_workspace_size(varsim_net* net, int32_t batch, int32_t training,
                                        size_t* bytes);
/* Predicted rise of `batch` problems.  q_dyn, leak_var, cond_map: DEVICE float [*][n][n]
 * (leak_var / cond_map NULL = 1); problem b reads map index sample_idx[b] (DEVICE int32, NULL =
 * b).  dT_out: DEVICE float [batch][n][n].  Stream-ordered, does not synchronise. */
VARSIM_API varsim_status varsim_net_forward(varsim_net* net, int32_t batch, const float* q_dyn,
                                 const float* leak_var, const float* cond_map,
                                 const int32_t* sample_idx, float* dT_out, void* workspace,
                                 size_t ws_bytes, void* stream);
/* Mean-squared error against target (DEVICE float [*][n][n], indexed like the inputs) and its
 * gradient with respect to every parameter: grad DEVICE float[param_count], loss DEVICE
 * float[1].  Stream-ordered. */
VARSIM_API varsim_status varsim_net_gradient(varsim_net* net, int32_t batch, const float* q_dyn,
                                  const float* leak_var, const float* cond_map,
                                  const int32_t* sample_idx, const float* target, float* grad,
                                  float* loss, void* workspace, size_t ws_bytes, void* stream);
/* One Adam step (bias-corrected) on the FP32 master parameters with gradient grad. */
VARSIM_API varsim_status varsim_net_adam(varsim_net* net, const float* grad, float lr, float beta1,
                              float beta2, float eps, void* stream);

/* One convolution layer on the matrix cores, for testing the kernels the network uses.
 * Tensors are [batch][h][w][c] BF16 bit patterns (channels last); weights [cout][k][k][cin]
 * BF16; cin, cout multiples of 16; k = 1 or 3 ('same' zero padding).
 *   VARSIM_NN_FWD:   a = x, b = weights, bias (FP32 [cout] or NULL), relu -> out BF16 [..][cout]
 *   VARSIM_NN_DGRAD: a = dz [..][cout], b = weights -> out FP32 [..][cin], the gradient of
 *                    sum(dz * conv(x)) with respect to x
 *   VARSIM_NN_WGRAD: a = x, b = dz -> out FP32 [cout][k][k][cin], its gradient with respect to
 *                    the weights
 * The workspace (varsim_nn_conv_workspace) holds transposed weights or partial sums.
 * Synchronises `stream`. */
enum { VARSIM_NN_FWD = 0, VARSIM_NN_DGRAD = 1, VARSIM_NN_WGRAD = 2 };
VARSIM_API varsim_status varsim_nn_conv_workspace(int32_t op, int32_t k, int32_t batch, int32_t h,
                                       int32_t w, int32_t cin, int32_t cout, size_t* bytes);
VARSIM_API varsim_status varsim_nn_conv(varsim_ctx* ctx, int32_t op, int32_t k, int32_t batch,
                             int32_t h, int32_t w, int32_t cin, int32_t cout, const uint16_t* a,
                             const uint16_t* b, const float* bias, int32_t relu, void* out,
                             void* workspace, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------------------
 * Autotuning of launch shapes.  With autotuning on (enable = 1), the first solve of a group of
 * maps with a given (grid size, precision, power-of-two group size) times every column-pass
 * strip width on that group's own workspace arrays (each timed launch right after a row pass
 * over the group, as in the solve, which overwrites the group's spectrum workspace) and keeps
 * the fastest for later solves of the same kind; results do not depend on the choice (the same
 * arithmetic in a different tiling).  enable = 0 stops tuning (kept choices still apply); enable = -1 also forgets them.
 * varsim_autotune_report writes one line per tuned kind into buf (NUL-terminated; returns
 * VARSIM_ERR_NO_MEMORY if truncated).
 */
VARSIM_API varsim_status varsim_set_autotune(varsim_ctx* ctx, int32_t enable);
VARSIM_API varsim_status varsim_autotune_report(varsim_ctx* ctx, char* buf, size_t len);
/* Persisted tuning: varsim_autotune_export writes the context's kept choices as text (a header
 * line "varsim-tuning 1", then one line per choice: "col nx ny precision log2_group variant" and
 * "tr n precision row_variant col_variant"); *needed (if not NULL) receives the size including the
 * terminating NUL, and buf NULL only queries it (VARSIM_ERR_NO_MEMORY if len is smaller).
 * varsim_autotune_import adds the choices of such text to the context, replacing kept choices of
 * the same kinds, so that a later process can skip the timing runs; the text is checked whole
 * first (VARSIM_ERR_INVALID on any malformed or out-of-range line, the context unchanged).  The
 * choices only select among tilings of the same arithmetic, so an imported choice can cost
 * speed, never accuracy; they are specific to the GPU model they were timed on. */
VARSIM_API varsim_status varsim_autotune_export(varsim_ctx* ctx, char* buf, size_t len, size_t* needed);
VARSIM_API varsim_status varsim_autotune_import(varsim_ctx* ctx, const char* text);
/* Small grids: a map with N <= max_n is solved start to finish by one workgroup that keeps its
 * spectrum in LDS (one launch for the whole fixed point, convergence decided on the device);
 * larger maps use two HBM passes per iteration.  The limit is capped at 128 (FP32) / 64 (FP64),
 * the sizes whose working set fits one CU's LDS; max_n = -1 restores that default, 0 turns the
 * path off.  Both paths compute the same iterates. */
VARSIM_API varsim_status varsim_set_small_path(varsim_ctx* ctx, int32_t max_n);
/* Batching (the scope table's persistent-scheduling row; the paper's Monte Carlo use case,
 * Sec. I and Sec. V): with iterations = K > 0 the fixed-point loop of varsim_solve_batch /
 * varsim_solve_steady is launched as HIP graphs of K iterations each (column and row pass of
 * every looping group, then the count of maps still iterating), captured on a private stream and
 * replayed on the caller's stream.  Executable graph j (the j-th chunk of a call) is kept by the
 * context and rewritten for the next call with hipGraphExecUpdate, after its previous launch
 * has finished (re-instantiated when the launch structure differs); the host reads convergence
 * once per chunk, so a chunk may run up to K - 1 iterations past the last needed one, which
 * return at once for maps already converged.  Results are bitwise those of direct launches.
 * iterations = 0 (the default) launches every pass directly; per-kernel timing
 * (varsim_set_timing) also uses direct launches.  VARSIM_ERR_INVALID outside [0, 16];
 * VARSIM_ERR_DEVICE if the capture stream cannot be created. */
VARSIM_API varsim_status varsim_set_graph_iterations(varsim_ctx* ctx, int32_t iterations);
/* Testing / manual tuning: every later column pass (solves and varsim_conv) uses strip-width
 * candidate `variant` (0 = default strip width, 1 = default width with two column pairs per
 * transform group, 2 = half width, 3 / 4 = the wide strip of 128-byte row segments whose
 * transforms use the strip's own tile columns as scratch, one / two pairs per group, 5 / 6 =
 * the pipelined pass on the same 128-byte strips (a few workgroups per CU walk the strips,
 * loading the next strip while transforming the current one), two / four pairs per group,
 * where the strips split evenly over the 8 XCDs (else candidate 0), 7 / 8 = one column per DFT
 * of half the length with lambda applied to its cosine coefficients, default / half strip
 * width (N >= 256 inside solves; elsewhere candidate 0); square maps only, rectangular ones
 * keep 0), and transient solves use row-pass candidate `variant` and column candidate
 * `variant` where N has that candidate (see varsim_force_transient_variant; else their
 * default); -1 returns to the default or tuned choices.  Candidates 0..6 give bitwise equal
 * results, and so do 7 and 8; the two families agree to rounding.  Untuned and tuned choices
 * stay in one family per (N, precision): one column per DFT for FP64 at N >= 512, two columns
 * otherwise.  VARSIM_ERR_INVALID outside [-1, 8]. */
VARSIM_API varsim_status varsim_force_col_variant(varsim_ctx* ctx, int32_t variant);
/* Testing / manual tuning of transient solves: row-pass candidate `row_variant` and column-pass
 * candidate `col_variant`, each in [0, 8): 0..2 transform two rows (columns) per DFT (row: rows
 * per workgroup default / half / one pair; column: strip width default / half / quarter); 3..5
 * transform one row (column) per DFT of half the length (row: 1 / 2 / 4 wavefronts per
 * workgroup; column: widest strip / half / quarter), available for N >= 64; 6..7 spread each
 * row (column) over two wavefronts, the half-length DFT split into two quarter-length DFTs of
 * the even and the odd coefficients (row: 1 / 2 rows per workgroup; column: 4 / 2 columns per
 * strip), available for N = 1024.  A candidate N does not have falls back to candidate 0.
 * Results agree to rounding.  -1 returns to the tuned, forced (varsim_force_col_variant) or
 * default choice (candidate 3 for both passes where N >= 64, else 0; with autotuning on, the
 * (row, column) pairs of the one-sequence families (of the two-sequence family where N < 64)
 * are timed over whole steps on the first solve of each (N, precision) and the fastest pair
 * kept).  VARSIM_ERR_INVALID outside [-1, 8). */
VARSIM_API varsim_status varsim_force_transient_variant(varsim_ctx* ctx, int32_t row_variant,
                                                        int32_t col_variant);

/* ----------------------------------------------------------------------------------------
 * Kernel timing.  When enabled, every kernel launch of the solves is bracketed by HIP events
 * on the launch stream; varsim_kernel_times reports, per kernel class, the launch count and
 * the summed durations (ms) since the last reset.  The events are read when varsim_kernel_times
 * or varsim_reset_timing is called (both wait for the launches recorded so far), not at the end
 * of each solve, so timing adds no host time between calls.  Class names are returned in
 * names[i] (static strings).  n_io: in = capacity, out = number of classes written.
 */
VARSIM_API varsim_status varsim_set_timing(varsim_ctx* ctx, int32_t enable);
VARSIM_API varsim_status varsim_kernel_times(varsim_ctx* ctx, const char** names, int64_t* counts,
                                  double* total_ms, int32_t* n_io);
VARSIM_API varsim_status varsim_reset_timing(varsim_ctx* ctx);
/* Restricts timing to one kernel class (a name varsim_kernel_times reports, e.g. "row_merged"),
 * so that a measurement of that class records two events per launch of it only; NULL or ""
 * times every class again. */
VARSIM_API varsim_status varsim_set_timing_only(varsim_ctx* ctx, const char* kernel_class);

#ifdef __cplusplus
}
#endif

#endif /* VARSIM_H */
