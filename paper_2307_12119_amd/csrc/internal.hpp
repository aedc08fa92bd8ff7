// Host-side declarations shared by the translation units of the varsim library.
#pragma once

#include "common.hpp"

namespace vs {

// Package layers below the first (silicon) layer and the bottom face (Table param).
constexpr int kMaxLayers = 8;
struct StackSpec {
  int n;            // layers including the first (1: a single slab)
  int aliases;      // image aliases per side summed for the eigenvalue correction
  double bottom_h;  // convective bottom coefficient W/m^2K (0: isothermal bottom)
  double t[kMaxLayers], k[kMaxLayers];  // thickness and conductivity (at T_amb) of each layer
};

struct TableSpec {
  int nx, ny;
  double lx, ly, t, k_ref;  // grid, die size, first layer's thickness and conductivity at T_amb
  StackSpec stack;          // zero: a single slab over an isothermal bottom
};

// Green's-function table: K_per [ny+1][nx+1], lambda transposed and scaled (FP64, FP32), the
// column-pass coefficients [nx][ny/2+1][4] (FP64, FP32), and optionally lambda row-major
// unscaled.  scratch: green_table_scratch_doubles(nx, ny) doubles.
hipError_t launch_green_table(const TableSpec& sp, double* kper, double* lam64T, float* lam32T, double* coef64,
                              float* coef32, double* lam_rowmajor, double* scratch, hipStream_t stream);
// Column-pass coefficients of the leakage-aware deterministic operator of the one-shot solve
// (Eq. detsol): lambda / (1 - c lambda) per mode, c = beta hx hy mu (lambda in K/W, unscaled),
// from lam64T of the green table.
hipError_t launch_det_coef(const TableSpec& sp, const double* lam64T, double c, double* coef64, float* coef32,
                           hipStream_t stream);
inline size_t coef_entries(int nx, int ny) { return (size_t)nx * (ny / 2 + 1) * 4; }
size_t green_table_scratch_doubles(int nx, int ny);

// tw32lo / qw32lo: the low parts (exact value - FP32 value, rounded) of tw32 / qw32
hipError_t launch_twiddles(int n, Cx<double>* tw64, Cx<float>* tw32, Cx<double>* qw64, Cx<float>* qw32,
                           Cx<float>* tw32lo, Cx<float>* qw32lo, hipStream_t stream);

// Row-pass variants.
enum RowMode : int {
  ROW_HEAD = 0,       // dT (or 0) -> P -> row DCT-II -> S
  ROW_MERGED = 1,     // S -> row DCT-III -> theta -> dT' (+residual, stats) -> P -> row DCT-II -> S
  ROW_LAST = 2,       // as MERGED without the forward transform
  ROW_RESID = 3,      // S -> theta -> dT'' ; residual max |dT'' - dT| only (no write)
  ROW_CONV_HEAD = 4,  // power map (W per cell) -> row DCT-II -> S
  ROW_CONV_TAIL = 5,  // S -> row DCT-III -> theta written to the output map
  // one-shot solve (Sec. IV-C), after a head pass from dT = 0 and a column pass with the
  // deterministic operator's coefficients:
  ROW_OS_MID = 6,   // S -> theta_det (stored in dT) -> beta hx hy (QL / m - mu) theta_det -> row DCT-II -> S
  ROW_OS_TAIL = 7,  // S -> theta_rand (+ theta_det from dT) -> Phi^-1 -> dT, statistics
  // Anderson(1) mixing, two row passes per iteration:
  ROW_AA_EVAL = 8,  // S -> g = G(x_k) (to dT), f = g - x_k (to af), statistics, dot products
  ROW_AA_MIX = 9,   // x_{k+1} = g - gamma (g - g_prev) (to ax; g to ag) -> P -> row DCT-II -> S
};

struct Twiddles {
  const Cx<double>* tw64;
  const Cx<float>* tw32;
  const Cx<double>* qw64;
  const Cx<float>* qw32;
  const Cx<float>* tw32lo;  // low parts of tw32 and qw32 (compensated twiddles)
  const Cx<float>* qw32lo;
};

struct PassArgs {
  const MapPtrs* maps;  // device array, one entry per map of the group
  int n_maps;
  int n;   // row length nx (the row passes' transform length)
  int ny;  // row count (the column passes' transform length); nx == ny for the LDS-resident solver
  IterState st;
  PointParams pp;
  Twiddles tw;   // twiddles of length nx (row passes)
  Twiddles twc;  // twiddles of length ny (column passes)
  int ct;        // FP32 transforms with compensated twiddles (row modes HEAD / MERGED / LAST, column pass)
  int iter;        // 1-based iteration index of the pass
  int zero_start;  // iteration 1 starts from dT = 0 (no warm start)
  int use_s64;     // operate on MapPtrs::S64 instead of S
  int resid_pass;  // FP64 residual pass: skip only maps flagged invalid / runaway
  // cosine eigenvalues lambda [q][p] of the column transforms (scaled as the column pass applies
  // them) for the one-sequence column pass, or null where the pass applies other coefficients
  const float* lam32 = nullptr;
  const double* lam64 = nullptr;
};

// io: element type of the maps (VARSIM_F32 / VARSIM_F64); compute: type of the transforms.
// With a.ct, FP32 modes HEAD / MERGED / LAST use compensated twiddles (launch_row_pass_ct).
hipError_t launch_row_pass(int mode, int io, int compute, const PassArgs& a, hipStream_t stream);
hipError_t launch_row_pass_ct(int mode, const PassArgs& a, hipStream_t stream);
// coef: the column-pass coefficient table of the compute type; variant: launch-shape candidate
// 0 (default strip width), 1 (default width, two column pairs per transform group), 2 (half
// width), 3 / 4 (wide in-place strip, one / two pairs), 5 / 6 (pipelined 128-byte strips, two /
// four pairs), 7 / 8 (one column per DFT of half the length, default / half strip width: N >= 256
// and a.lam32 / a.lam64 set); col_pass_columns / col_pass_pairs give a candidate's strip width
// and pairs per group, col_pass_pipelined whether it runs as the pipelined pass, col_pass_family
// whether it transforms one column (1) or two columns (0) per DFT
constexpr int kColVariants = 9;
constexpr int kMaxGraphIterations = 16;  // fixed-point iterations one captured graph may hold
hipError_t launch_col_pass(int compute, const PassArgs& a, const void* coef, hipStream_t stream, int variant = 0);
int col_pass_columns(int compute, int n, int variant);
int col_pass_pairs(int compute, int n, int variant);
int col_pass_pipelined(int compute, int n, int variant);
int col_pass_family(int compute, int n, int variant);

// Static inputs: QL = q_leak0 * v, MINV = 1 / m (per map), warm-start screening and copy.
struct PrepArgs {
  const void* q_leak0;
  const void* leak_var;
  const void* cond_map;
  const void* init;
  void* ql_out;    // or null
  void* minv_out;  // or null
  void* dT;
  unsigned* flags;  // this map's flag word
  // source-side inputs of the FP32 passes (MapPtrs::qs, qls), or null: q_dyn / m and
  // q_leak0 v / m (need cond_map; minv_out is then set too)
  const void* q_dyn;
  void* qs_out;
  void* qls_out;
};
// args: device array of n_maps entries; count = cells per map
hipError_t launch_prep(int io, const PrepArgs* args, int n_maps, long count, hipStream_t stream);
hipError_t launch_init_copy(int io, const PrepArgs* args, int n_maps, long count, hipStream_t stream);

hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t stream);

// Convergence count: number of maps not yet finished after iteration `iter`.
// out: one int the kernel overwrites with the count (device or mapped pinned host memory)
hipError_t launch_count_active(const IterState& st, int n_maps, int iter, double tol, int* out, hipStream_t stream);

// The whole fixed point of every map of a group by one LDS-resident workgroup per map
// (n <= small_max_n(io)); coef: the column coefficients of the io type.
int small_max_n(int io);
hipError_t launch_small_solve(int io, const PassArgs& a, int max_iter, const void* coef, hipStream_t stream);

// Final statistics of every map into a device varsim_stats array.
// dst[order[i]] = src[i], i < n (per-problem statistics back into the caller's order)
hipError_t launch_scatter_stats(const varsim_stats* src, const int* order, int n, varsim_stats* dst, hipStream_t s);
// oneshot = 1: statistics of the one-shot solve (iterations 0, no increment)
hipError_t launch_finalize(const IterState& st, const MapPtrs* maps, int n_maps, int io, int nx, int ny, int max_iter,
                           int iters_run, double tol, int residual_done, varsim_stats* out, hipStream_t stream,
                           int oneshot = 0);
// rows one row-pass workgroup transforms for rows of length nx; the workgroups of one map's row
// pass (<= kRowGroupsMax) on an nx x ny grid (0 when ny is not a multiple of row_pass_rows(nx))
int row_pass_rows(int nx);
int row_pass_groups(int nx, int ny);

// Transient solve of one map (element type T = io = compute type).
constexpr int kMaxPoles = 8;  // poles per cosine mode of the multi-pole transient model
constexpr int kMaxHistory = 1 << 20;  // longest truncated transient history, steps
struct TransArgs {
  int n;
  void* S;            // [n][n] transform work array
  void* state;        // [poles][n][n] spectral state theta_hat, layout [q][p] (q: row-transform index)
  const void* ab;     // [poles][n][n][2] per-mode (a, b), layout [q][p]
  int poles;          // poles per mode (1 but for the multi-pole model)
  const int* ids;     // [n][n] block id of each cell, -1 where no block
  const void* trace;  // [n_steps][n_blocks] block power densities
  int n_blocks;
  const void* ql;     // leakage density at ambient times variation, or null
  const void* minv;   // 1 / conductivity multiplier, or null
  void* dT;           // final rise
  void* snaps;        // [n_steps / out_every][n][n], or null
  int out_every;
  // truncated history of hist steps (Eq. tranapprox with saturated step kernels), or ring null:
  // ring [hist - 1][n][n] holds the spectra of the last hist - 1 steps (slot = step mod (hist - 1),
  // layout [q][p]); fir [poles + 1][n][n] the per-pole coefficients -b_j r_j and then the
  // saturated part sum_j c_j r_j, r_j = exp(-(hist - 1) dt / tau_j)
  void* ring;
  const void* fir;
  int hist;
  int slot;
  unsigned* flags;    // runaway flag word
  PointParams pp;
  Twiddles tw;
  // z-order copies (single.hpp) of ids, ql and minv for the one-row passes (null where the
  // natural array is null)
  const int* idz;
  const void* qlz;
  const void* minvz;
};
enum TransMode : int { TR_HEAD = 0, TR_MERGED = 1, TR_LAST = 2 };

// (a, b) per mode from lambda (lam64T, scaled as the column pass uses it), dt and tau_model
// (and, fir non-null, the truncated-history coefficients of hist steps)
hipError_t launch_transient_coef(const TableSpec& sp, const double* lam64T, int io, void* ab, void* fir, int hist,
                                 double alpha, double dt, int tau_model, double rho_c, int poles, hipStream_t stream);
hipError_t launch_block_ids(const int* rects, int n_blocks, int* ids, int nx, int ny, hipStream_t stream);
// TR_HEAD: P_1 -> row spectrum; TR_MERGED (step n): row synthesis -> dT_n -> P_{n+1} -> row
// spectrum; TR_LAST: row synthesis -> dT_n (final)
// variant: launch-shape candidate.  0..2: two sequences per transform (row: rows per workgroup
// default / half / one pair; column: strip width default / half / quarter); 3..5: one sequence
// per transform (row: 1 / 2 / 4 wavefronts per workgroup; column: widest strip / half /
// quarter), available where transient_single_ok(n); 6..7: one sequence over two wavefronts
// (row: 1 / 2 rows per workgroup; column: 4 / 2 columns per strip), where transient_split_ok(n).
constexpr int kTrVariants = 8;
bool transient_single_ok(int n);
bool transient_split_ok(int n);
int transient_variants(int n);
hipError_t launch_transient_row(int mode, int io, const TransArgs& a, int step, hipStream_t stream, int variant = 0);
hipError_t launch_transient_col(int io, const TransArgs& a, hipStream_t stream, int variant = 0);
hipError_t launch_transient_row1(int mode, int io, const TransArgs& a, int step, hipStream_t stream, int variant);
hipError_t launch_transient_col1(int io, const TransArgs& a, hipStream_t stream, int variant);
hipError_t launch_transient_row2(int mode, int io, const TransArgs& a, int step, hipStream_t stream, int variant);
hipError_t launch_transient_col2(int io, const TransArgs& a, hipStream_t stream, int variant);
// dst[row][2j + k] = src[row][z_sample(j, k)] for an n x n array of esz-byte elements
hipError_t launch_zorder(int esz, const void* src, void* dst, int n, hipStream_t stream);
hipError_t launch_map_stats(int io, const void* dT, long cells, const unsigned* flags, int steps, varsim_stats* out,
                            hipStream_t stream);

}  // namespace vs
