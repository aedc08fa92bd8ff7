// C ABI of the varsim library: context, caches, validation, workspace layout and the
// host-side sequencing of the device passes.  No arithmetic of the method runs here: every
// step of the solve is a kernel launch; the host only orders them and reads back per-map
// convergence counts and statistics.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "ctx.hpp"

using namespace vs;

// Workspace of varsim_solve_batch_noalloc: one static device array per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel or copy (on the host the
// name is only a stand-in for the symbol); it uses the device address that varsim_create looks
// up once per device with hipGetSymbolAddress.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> address of `scratch` there (nullptr: lookup failed)

// Called with `device` current.
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    ptr = nullptr;
  }
  g_scratch_addr[device] = ptr;
  return ptr;
}


bool is_pow2_in_range(int n) { return n >= kMinN && n <= kMaxN && (n & (n - 1)) == 0; }

varsim_status check_geometry(varsim_ctx* ctx, const varsim_geometry* g) {
  if (!g) return fail(ctx, VARSIM_ERR_INVALID, "geometry is NULL");
  if (!(g->lx_m > 0) || !(g->ly_m > 0) || !(g->t_amb_K > 0))
    return fail(ctx, VARSIM_ERR_INVALID, "die size and ambient temperature must be positive");
  if (g->nx <= 0 || g->ny <= 0) return fail(ctx, VARSIM_ERR_INVALID, "grid size must be positive");
  if (!is_pow2_in_range(g->nx) || !is_pow2_in_range(g->ny))
    return fail(ctx, VARSIM_ERR_UNSUPPORTED, "grid %dx%d: nx and ny must be powers of two in [16, 1024]", g->nx, g->ny);
  if (row_pass_groups(g->nx, g->ny) < 1)
    return fail(ctx, VARSIM_ERR_UNSUPPORTED, "grid %dx%d: rows of %d cells need ny >= %d", g->nx, g->ny, g->nx,
                row_pass_rows(g->nx));
  if (g->n_layers < 1 || !g->layers) return fail(ctx, VARSIM_ERR_INVALID, "at least one layer is required");
  if (g->n_layers > kMaxLayers) return fail(ctx, VARSIM_ERR_UNSUPPORTED, "at most %d layers", kMaxLayers);
  for (int i = 0; i < g->n_layers; ++i) {
    const varsim_layer& L = g->layers[i];
    if (!(L.thickness_m > 0) || !(L.k0_W_mK > 0) || !(L.eta >= 0) || !std::isfinite(L.thickness_m) ||
        !std::isfinite(L.k0_W_mK) || !std::isfinite(L.eta))
      return fail(ctx, VARSIM_ERR_INVALID, "layer %d: thickness, k0 must be positive and eta >= 0", i);
  }
  if (g->bottom_bc != 0 && g->bottom_bc != 1) return fail(ctx, VARSIM_ERR_INVALID, "bottom_bc must be 0 or 1");
  if (g->bottom_bc == 1 && (!(g->h_bottom_W_m2K > 0) || !std::isfinite(g->h_bottom_W_m2K)))
    return fail(ctx, VARSIM_ERR_INVALID, "a convective bottom needs h_bottom_W_m2K > 0");
  return VARSIM_OK;
}

varsim_status check_options(varsim_ctx* ctx, const varsim_options* o) {
  if (!o) return fail(ctx, VARSIM_ERR_INVALID, "options is NULL");
  if (o->leak < VARSIM_LEAK_NONE || o->leak > VARSIM_LEAK_LINEAR) return fail(ctx, VARSIM_ERR_INVALID, "bad leak law");
  if (o->precision != VARSIM_F32 && o->precision != VARSIM_F64) return fail(ctx, VARSIM_ERR_INVALID, "bad precision");
  if (o->max_iter < 1 || o->max_iter > kMaxIter) return fail(ctx, VARSIM_ERR_INVALID, "max_iter must be in [1, 1000]");
  if (!(o->tol_K > 0)) return fail(ctx, VARSIM_ERR_INVALID, "tol_K must be positive");
  if (!(o->dT_cap_K > 0)) return fail(ctx, VARSIM_ERR_INVALID, "dT_cap_K must be positive");
  if (!std::isfinite(o->beta_per_K)) return fail(ctx, VARSIM_ERR_INVALID, "beta must be finite");
  if (o->sv_radius != 0) return fail(ctx, VARSIM_ERR_UNSUPPORTED, "only sv_radius = 0 is supported");
  if (o->cond_model != VARSIM_COND_SOURCE && o->cond_model != VARSIM_COND_TARGET)
    return fail(ctx, VARSIM_ERR_INVALID, "bad cond_model");
  if (o->compensated_twiddles != 0 && o->compensated_twiddles != 1)
    return fail(ctx, VARSIM_ERR_INVALID, "compensated_twiddles must be 0 or 1");
  if (o->anderson != 0 && o->anderson != 1) return fail(ctx, VARSIM_ERR_INVALID, "anderson must be 0 or 1");
  return VARSIM_OK;
}

double k_ref_of(const varsim_geometry* g, int layer = 0) {
  const varsim_layer& L = g->layers[layer];
  return L.k0_W_mK * std::pow(g->t_amb_K / 300.0, -L.eta);
}

bool is_stack(const varsim_geometry* g) { return g->n_layers > 1 || g->bottom_bc != 0; }

// One-dimensional thermal resistance of the die and package per unit area, sum t_i / k_i (+ 1/h):
// the response of the uniform mode, the largest eigenvalue of the operator times hx hy.
double series_resistance(const varsim_geometry* g) {
  double r = g->bottom_bc ? 1.0 / g->h_bottom_W_m2K : 0.0;
  for (int i = 0; i < g->n_layers; ++i) r += g->layers[i].thickness_m / k_ref_of(g, i);
  return r;
}

TableKey key_of(const varsim_geometry* g) {
  std::vector<double> extra;
  if (is_stack(g)) {
    extra.push_back(g->bottom_bc);
    extra.push_back(g->bottom_bc ? g->h_bottom_W_m2K : 0.0);
    for (int i = 1; i < g->n_layers; ++i) {
      extra.push_back(g->layers[i].thickness_m);
      extra.push_back(k_ref_of(g, i));
    }
  }
  return TableKey(g->nx, g->ny, g->lx_m, g->ly_m, g->layers[0].thickness_m, k_ref_of(g), extra);
}

// The table description of a geometry: grid, first layer, and the package stack if any.
TableSpec spec_of(const varsim_geometry* g) {
  TableSpec sp{g->nx, g->ny, g->lx_m, g->ly_m, g->layers[0].thickness_m, k_ref_of(g), StackSpec{}};
  if (is_stack(g)) {
    StackSpec& st = sp.stack;
    st.n = g->n_layers;
    st.bottom_h = g->bottom_bc ? g->h_bottom_W_m2K : 0.0;
    for (int i = 0; i < g->n_layers; ++i) {
      st.t[i] = g->layers[i].thickness_m;
      st.k[i] = k_ref_of(g, i);
    }
    // aliases until exp(-2 |kappa| t1) < 1e-21: |kappa| >= 2 pi j / h_max
    const double hmax = std::max(g->lx_m / g->nx, g->ly_m / g->ny);
    st.aliases = 1 + (int)std::ceil(25.0 * hmax / (2.0 * M_PI * st.t[0]));
  }
  return sp;
}

varsim_status get_twiddles(varsim_ctx* ctx, int n, hipStream_t s, TwEntry* out) {
  auto it = ctx->twiddles.find(n);
  if (it != ctx->twiddles.end()) {
    *out = it->second;
    return VARSIM_OK;
  }
  TwEntry e;
  if (hipMalloc(&e.tw64, n * sizeof(Cx<double>)) != hipSuccess || hipMalloc(&e.tw32, n * sizeof(Cx<float>)) != hipSuccess ||
      hipMalloc(&e.qw64, n * sizeof(Cx<double>)) != hipSuccess || hipMalloc(&e.qw32, n * sizeof(Cx<float>)) != hipSuccess ||
      hipMalloc(&e.tw32lo, n * sizeof(Cx<float>)) != hipSuccess || hipMalloc(&e.qw32lo, n * sizeof(Cx<float>)) != hipSuccess)
    return fail(ctx, VARSIM_ERR_NO_MEMORY, "twiddle table allocation failed");
  HIP_TRY(launch_twiddles(n, e.tw64, e.tw32, e.qw64, e.qw32, e.tw32lo, e.qw32lo, s));
  HIP_TRY(hipStreamSynchronize(s));
  ctx->twiddles[n] = e;
  *out = e;
  return VARSIM_OK;
}

varsim_status get_table(varsim_ctx* ctx, const varsim_geometry* g, hipStream_t s, TableEntry* out,
                        double* lam_rowmajor = nullptr) {
  const TableKey key = key_of(g);
  auto it = ctx->tables.find(key);
  if (it != ctx->tables.end() && !lam_rowmajor) {
    *out = it->second;
    return VARSIM_OK;
  }
  TableSpec sp = spec_of(g);
  TableEntry e = it != ctx->tables.end() ? it->second : TableEntry{};
  const bool fresh = it == ctx->tables.end();
  if (fresh) {
    if (hipMalloc(&e.kper, (size_t)(sp.nx + 1) * (sp.ny + 1) * sizeof(double)) != hipSuccess ||
        hipMalloc(&e.lam64T, (size_t)sp.nx * sp.ny * sizeof(double)) != hipSuccess ||
        hipMalloc(&e.lam32T, (size_t)sp.nx * sp.ny * sizeof(float)) != hipSuccess ||
        hipMalloc(&e.coef64, coef_entries(sp.nx, sp.ny) * sizeof(double)) != hipSuccess ||
        hipMalloc(&e.coef32, coef_entries(sp.nx, sp.ny) * sizeof(float)) != hipSuccess)
      return fail(ctx, VARSIM_ERR_NO_MEMORY, "table allocation failed");
  }
  double* tab_tmp = nullptr;
  if (hipMalloc(&tab_tmp, green_table_scratch_doubles(sp.nx, sp.ny) * sizeof(double)) != hipSuccess)
    return fail(ctx, VARSIM_ERR_NO_MEMORY, "table scratch allocation failed");
  hipError_t err = timed(ctx, "green_table", s,
                         [&] {
                           return launch_green_table(sp, e.kper, e.lam64T, e.lam32T, e.coef64, e.coef32, lam_rowmajor,
                                                     tab_tmp, s);
                         });
  hipError_t err2 = hipStreamSynchronize(s);
  (void)hipFree(tab_tmp);
  if (err != hipSuccess || err2 != hipSuccess)
    return fail(ctx, VARSIM_ERR_DEVICE, "green table: %s", hipGetErrorString(err != hipSuccess ? err : err2));
  ctx->tables[key] = e;
  *out = e;
  return VARSIM_OK;
}

// Lookup only (no allocation, no kernel): the geometry's Green's table and twiddles, which
// varsim_green_table or an earlier solve of the same geometry put in the context's caches.
varsim_status find_cached(varsim_ctx* ctx, const varsim_geometry* g, TableEntry* tab, TwEntry* tw, TwEntry* twc) {
  auto it = ctx->tables.find(key_of(g));
  auto jt = ctx->twiddles.find(g->nx);
  auto kt = ctx->twiddles.find(g->ny);
  if (it == ctx->tables.end() || jt == ctx->twiddles.end() || kt == ctx->twiddles.end())
    return fail(ctx, VARSIM_ERR_INVALID,
                "no cached Green's table for this %dx%d geometry: build it first with varsim_green_table "
                "(which allocates) or an allocating solve",
                g->nx, g->ny);
  *tab = it->second;
  *tw = jt->second;
  *twc = kt->second;
  return VARSIM_OK;
}

// Column coefficients of the leakage-aware deterministic operator lambda / (1 - c lambda) of
// the one-shot solve (Eq. detsol), cached per (geometry, c); tab: the geometry's green table.
varsim_status get_det_coef(varsim_ctx* ctx, const varsim_geometry* g, const TableEntry& tab, double c, hipStream_t s,
                           DetEntry* out) {
  const auto key = std::make_pair(key_of(g), c);
  auto it = ctx->det_coefs.find(key);
  if (it != ctx->det_coefs.end()) {
    *out = it->second;
    return VARSIM_OK;
  }
  DetEntry e;
  const size_t cnt = coef_entries(g->nx, g->ny);
  if (hipMalloc(&e.coef64, cnt * sizeof(double)) != hipSuccess || hipMalloc(&e.coef32, cnt * sizeof(float)) != hipSuccess) {
    (void)hipFree(e.coef64);
    return fail(ctx, VARSIM_ERR_NO_MEMORY, "deterministic-operator table allocation failed");
  }
  const TableSpec sp = spec_of(g);
  HIP_TRY(timed(ctx, "det_table", s, [&] { return launch_det_coef(sp, tab.lam64T, c, e.coef64, e.coef32, s); }));
  ctx->det_coefs[key] = e;
  *out = e;
  return VARSIM_OK;
}

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Workspace layout of a batch (problems in group-sorted order).
struct Layout {
  int stride = 0;
  size_t resid = 0, sum = 0, maxpack = 0, flags = 0, resid64 = 0, part = 0, aa = 0, state_end = 0;
  size_t stats = 0, maps = 0, prep = 0, order = 0;
  std::vector<size_t> S, QL, MINV, S64, AX, AG, AF, QS, QLS;
  size_t total = 0;
};

size_t esize(int precision) { return precision == VARSIM_F64 ? 8 : 4; }

// The FP32 passes' source-side inputs of map i (MapPtrs::qs, qls: the prep kernel's q_dyn / m and
// QL / m, else q_dyn and QL themselves) and the prep outputs that fill them; m.ql must be set.
void set_source_inputs(MapPtrs& m, PrepArgs& q, const varsim_problem* p, const Layout& L, int i, char* ws) {
  m.qs = L.QS[i] != (size_t)-1 ? (const void*)(ws + L.QS[i]) : p->q_dyn;
  m.qls = L.QLS[i] != (size_t)-1 ? (const void*)(ws + L.QLS[i]) : m.ql;
  q.q_dyn = p->q_dyn;
  q.qs_out = L.QS[i] != (size_t)-1 ? ws + L.QS[i] : nullptr;
  q.qls_out = L.QLS[i] != (size_t)-1 ? ws + L.QLS[i] : nullptr;
}

// true for memory the device owns (hipMalloc / torch tensors), false for host memory
bool is_device_ptr(const void* p) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();  // plain host memory is reported as an error; do not leave it behind
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}

Layout make_layout(const std::vector<const varsim_problem*>& probs, const varsim_options* o) {
  Layout L;
  const size_t n = probs.size();
  L.stride = o->max_iter + 2;
  size_t off = 0;
  L.resid = off;
  off = align_up(off + n * L.stride * 8);
  L.sum = off;
  off = align_up(off + n * L.stride * 8);
  L.maxpack = off;
  off = align_up(off + n * L.stride * 8);
  L.flags = off;
  off = align_up(off + n * 4);
  L.resid64 = off;
  off = align_up(off + n * 8);
  L.state_end = off;  // the words above are zeroed at the start of a call; the partial sums need not be
  L.part = off;
  off = align_up(off + n * kRowGroupsMax * 8);
  L.aa = off;  // Anderson mixing: per-workgroup dot products (written before being read)
  if (o->anderson) off = align_up(off + n * kRowGroupsMax * 2 * 8);
  L.stats = off;
  off = align_up(off + n * sizeof(varsim_stats));
  L.maps = off;
  off = align_up(off + n * sizeof(MapPtrs));
  L.prep = off;
  off = align_up(off + n * sizeof(PrepArgs));
  L.order = off;
  off = align_up(off + n * sizeof(int));
  const size_t es = esize(o->precision);
  for (const varsim_problem* p : probs) {
    const size_t cells = (size_t)p->geom->nx * p->geom->ny;
    L.S.push_back(off);
    off = align_up(off + cells * es);
    if (p->q_leak0 && o->leak != VARSIM_LEAK_NONE && p->leak_var) {
      L.QL.push_back(off);
      off = align_up(off + cells * es);
    } else {
      L.QL.push_back((size_t)-1);
    }
    if (p->cond_map) {
      L.MINV.push_back(off);
      off = align_up(off + cells * es);
    } else {
      L.MINV.push_back((size_t)-1);
    }
    // FP32 with the conductivity factor on the source side: q_dyn / m and QL / m
    const bool pre = p->cond_map && o->precision == VARSIM_F32 && o->cond_model == VARSIM_COND_SOURCE;
    L.QS.push_back(pre ? off : (size_t)-1);
    if (pre) off = align_up(off + cells * es);
    const bool pre_leak = pre && p->q_leak0 && o->leak != VARSIM_LEAK_NONE;
    L.QLS.push_back(pre_leak ? off : (size_t)-1);
    if (pre_leak) off = align_up(off + cells * es);
    if (o->final_f64_residual && o->precision == VARSIM_F32) {
      L.S64.push_back(off);
      off = align_up(off + cells * 8);
    } else {
      L.S64.push_back((size_t)-1);
    }
    for (auto* v : {&L.AX, &L.AG, &L.AF}) {  // Anderson mixing: x_k, G(x_{k-1}), f_{k-1}
      if (o->anderson) {
        v->push_back(off);
        off = align_up(off + cells * es);
      } else {
        v->push_back((size_t)-1);
      }
    }
  }
  L.total = off;
  return L;
}

PointParams point_params(const varsim_geometry* g, const varsim_options* o) {
  PointParams pp{};
  pp.hxhy = (g->lx_m / g->nx) * (g->ly_m / g->ny);
  pp.beta = o->beta_per_K;
  pp.t_amb = g->t_amb_K;
  const double eta = g->layers[0].eta;
  pp.eta_mode = eta == 0.0 ? 0 : (eta == 1.0 ? 1 : 2);
  pp.inv_1m_eta = eta == 1.0 ? 0.0 : 1.0 / (1.0 - eta);
  pp.c_1m_eta = (1.0 - eta) / g->t_amb_K;
  pp.cap = o->dT_cap_K;
  pp.tol = o->tol_K;
  pp.leak = o->leak;
  pp.cond_src = o->cond_model == VARSIM_COND_SOURCE ? 1 : 0;
  // Taylor series of the Kirchhoff inverse in u = u_scale theta:
  //   (1 + u)^a - 1 = sum_k C(a, k) u^k, a = 1/(1 - eta);  exp(u) - 1 = sum_k u^k / k! (eta = 1).
  // The FP32 path uses it where the first dropped term is below 1e-9 of the leading one.
  pp.u_scale = eta == 1.0 ? 1.0 / g->t_amb_K : (1.0 - eta) / g->t_amb_K;
  // The FP64 steady path uses it (more terms) where the first dropped term is below 1e-17.
  double c[kPoly64 + 1];
  double ck = 1.0;
  for (int k = 1; k <= kPoly64 + 1; ++k) {
    ck = eta == 1.0 ? ck / k : ck * (pp.inv_1m_eta - (k - 1)) / k;
    c[k - 1] = ck;
  }
  for (int k = 0; k < kPoly; ++k) pp.polyf[k] = (float)c[k];
  for (int k = 0; k < kPoly64; ++k) pp.polyd[k] = c[k];
  const double lead = std::fabs(c[0]);
  auto umax = [&](int K, double rel) {
    const double drop = std::fabs(c[K]);
    return drop > 0.0 ? std::min(0.1, std::pow(rel * lead / drop, 1.0 / K)) : 0.1;
  };
  pp.poly_umax = umax(kPoly, 1e-9);
  pp.poly_umax64 = umax(kPoly64, 1e-17);
  if (eta == 0.0) pp.poly_umax = pp.poly_umax64 = 0.0;
  return pp;
}

struct Group {
  int first, count;  // range in sorted order
  const varsim_geometry* geom;
  TableEntry table;
  TwEntry tw;   // length nx (row passes)
  TwEntry twc;  // length ny (column passes)
};

varsim_status validate_problem(varsim_ctx* ctx, const varsim_problem* p) {
  if (!p) return fail(ctx, VARSIM_ERR_INVALID, "problem is NULL");
  varsim_status s = check_geometry(ctx, p->geom);
  if (s != VARSIM_OK) return s;
  if (!p->q_dyn || !p->dT_out) return fail(ctx, VARSIM_ERR_INVALID, "q_dyn and dT_out are required");
  return VARSIM_OK;
}

varsim_status sort_into_groups(varsim_ctx* ctx, const varsim_problem* problems, int n,
                               std::vector<int>& order, std::vector<Group>& groups) {
  order.resize(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const varsim_geometry* ga = problems[a].geom;
    const varsim_geometry* gb = problems[b].geom;
    const auto ka = std::make_tuple(key_of(ga), ga->t_amb_K, ga->layers[0].eta);
    const auto kb = std::make_tuple(key_of(gb), gb->t_amb_K, gb->layers[0].eta);
    return ka < kb;
  });
  groups.clear();
  for (int i = 0; i < n; ++i) {
    const varsim_geometry* g = problems[order[i]].geom;
    const auto k = std::make_tuple(key_of(g), g->t_amb_K, g->layers[0].eta);
    if (!groups.empty()) {
      const varsim_geometry* h = groups.back().geom;
      if (std::make_tuple(key_of(h), h->t_amb_K, h->layers[0].eta) == k) {
        groups.back().count++;
        continue;
      }
    }
    groups.push_back(Group{i, 1, g, {}, {}, {}});
  }
  return VARSIM_OK;
}

varsim_status check_transient(varsim_ctx* ctx, const varsim_problem* p, const varsim_transient* tr,
                              const varsim_options* o) {
  if (!p || !tr) return fail(ctx, VARSIM_ERR_INVALID, "problem or transient is NULL");
  varsim_status s = check_geometry(ctx, p->geom);
  if (s != VARSIM_OK) return s;
  if (p->geom->nx != p->geom->ny)
    return fail(ctx, VARSIM_ERR_UNSUPPORTED, "transient solves take square grids (nx == ny)");
  if (is_stack(p->geom))
    return fail(ctx, VARSIM_ERR_UNSUPPORTED, "transient solves take one layer over an isothermal bottom");
  if ((s = check_options(ctx, o)) != VARSIM_OK) return s;
  if (!p->dT_out) return fail(ctx, VARSIM_ERR_INVALID, "dT_out is required");
  if (!(p->geom->layers[0].rho_c_J_m3K > 0) || !std::isfinite(p->geom->layers[0].rho_c_J_m3K))
    return fail(ctx, VARSIM_ERR_INVALID, "rho_c must be positive");
  if (!(tr->dt_s > 0) || !std::isfinite(tr->dt_s)) return fail(ctx, VARSIM_ERR_INVALID, "dt_s must be positive");
  if (tr->n_steps < 1 || tr->out_every < 1 || tr->n_blocks < 1)
    return fail(ctx, VARSIM_ERR_INVALID, "n_steps, out_every and n_blocks must be >= 1");
  if (!tr->block_rects || !tr->trace) return fail(ctx, VARSIM_ERR_INVALID, "block_rects and trace are required");
  if (tr->tau_model != VARSIM_TAU_MOMENT && tr->tau_model != VARSIM_TAU_LUMPED && tr->tau_model != VARSIM_TAU_MODAL)
    return fail(ctx, VARSIM_ERR_INVALID, "bad tau_model");
  if (tr->tau_model == VARSIM_TAU_MODAL && (tr->n_poles < 1 || tr->n_poles > kMaxPoles))
    return fail(ctx, VARSIM_ERR_INVALID, "n_poles must be in [1, %d]", kMaxPoles);
  if (tr->history_steps != 0 && (tr->history_steps < 2 || tr->history_steps > kMaxHistory))
    return fail(ctx, VARSIM_ERR_INVALID, "history_steps must be 0 or in [2, %d]", kMaxHistory);
  return VARSIM_OK;
}

// Workspace of one transient solve.
struct TransLayout {
  size_t flags = 0, state_end = 0, stats = 0, prep = 0, S = 0, state = 0, ab = 0, ring = 0, fir = 0, ids = 0;
  size_t QL = (size_t)-1, MINV = (size_t)-1, IDZ = 0, QLZ = (size_t)-1, MINVZ = (size_t)-1, total = 0;
};

int poles_of(const varsim_transient* tr) { return tr->tau_model == VARSIM_TAU_MODAL ? tr->n_poles : 1; }

TransLayout make_transient_layout(const varsim_problem* p, const varsim_transient* tr, const varsim_options* o) {
  TransLayout L;
  const size_t cells = (size_t)p->geom->nx * p->geom->ny, es = esize(o->precision);
  const size_t poles = (size_t)poles_of(tr);
  size_t off = 0;
  L.flags = off;
  off = align_up(off + 4);
  L.state_end = off;
  L.stats = off;
  off = align_up(off + sizeof(varsim_stats));
  L.prep = off;
  off = align_up(off + sizeof(PrepArgs));
  L.S = off;
  off = align_up(off + cells * es);
  L.state = off;  // one plane per pole
  off = align_up(off + poles * cells * es);
  L.ab = off;
  off = align_up(off + poles * 2 * cells * es);
  if (tr->history_steps >= 2) {  // truncated history: ring of past spectra, coefficient planes
    L.ring = off;
    off = align_up(off + (size_t)(tr->history_steps - 1) * cells * es);
    L.fir = off;
    off = align_up(off + (poles + 1) * cells * es);
  }
  L.ids = off;
  off = align_up(off + cells * 4);
  if (p->q_leak0 && o->leak != VARSIM_LEAK_NONE && p->leak_var) {
    L.QL = off;
    off = align_up(off + cells * es);
  }
  if (p->cond_map) {
    L.MINV = off;
    off = align_up(off + cells * es);
  }
  // z-order copies for the one-row passes
  L.IDZ = off;
  off = align_up(off + cells * 4);
  if (p->q_leak0 && o->leak != VARSIM_LEAK_NONE) {
    L.QLZ = off;
    off = align_up(off + cells * es);
  }
  if (p->cond_map) {
    L.MINVZ = off;
    off = align_up(off + cells * es);
  }
  L.total = off;
  return L;
}

// Column-pass strip width for a group: the tuned choice if the context has one (timing the
// candidates on this group's own arrays first if autotuning is on), else the default.
// The transform family a column pass of this size and precision takes: FP64 at N >= 512 transforms
// one column per DFT of half the length (candidates 7 / 8; the 1024-point pair needs more
// registers than one wavefront per SIMD leaves, and at N = 512 the one-column pass measured
// equal or faster), everything else two columns per DFT (candidates 0..6).  The family is fixed
// per (N, precision) rather than timed, so that the tuner's choice never changes the arithmetic.
int col_family_for(const PassArgs& group, int compute) {
  const bool lam = compute == VARSIM_F32 ? group.lam32 != nullptr : group.lam64 != nullptr;
  return compute == VARSIM_F64 && lam && group.n == group.ny && group.ny >= 512 ? 1 : 0;
}

varsim_status col_variant_for(varsim_ctx* ctx, const PassArgs& group, int io, int compute, const void* coef,
                              hipStream_t s, int* variant, bool may_tune = true) {
  const int family = col_family_for(group, compute);
  *variant = ctx->force_col >= 0 ? ctx->force_col : (family ? 7 : 0);
  if (ctx->force_col >= 0 || group.n != group.ny) return VARSIM_OK;  // rectangular maps: default strip
  const auto key = std::make_tuple(group.n, group.ny, compute, ilog2(group.n_maps));
  auto it = ctx->col_choice.find(key);
  if (it != ctx->col_choice.end()) {
    *variant = it->second;
    return VARSIM_OK;
  }
  if (!ctx->autotune || !may_tune) return VARSIM_OK;
  PassArgs a = group;
  a.iter = -1;  // plain transform: no solver state is read or written
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::vector<float> ms(kColVariants, 0.f);
  int best = *variant;
  for (int v = 0; v < kColVariants; ++v) {
    if (col_pass_family(compute, a.ny, v) != family) {
      ms[v] = -1.f;  // not timed: another transform family
      continue;
    }
    int dup = -1;
    for (int u = 0; u < v; ++u)
      if (col_pass_columns(compute, a.ny, u) == col_pass_columns(compute, a.ny, v) &&
          col_pass_pairs(compute, a.ny, u) == col_pass_pairs(compute, a.ny, v) &&
          col_pass_pipelined(compute, a.ny, u) == col_pass_pipelined(compute, a.ny, v) &&
          col_pass_family(compute, a.ny, u) == col_pass_family(compute, a.ny, v))
        dup = u;
    if (dup >= 0) {
      ms[v] = ms[dup];
      continue;
    }
    // Each timed launch follows a row pass over the same maps, as in the solve: the row pass
    // writes the spectra in reverse map order, so the column pass finds its first maps in the
    // MALL (timed back to back instead, every launch would read what the last one evicted, and
    // the candidates would rank differently).
    constexpr int kReps = 3;
    HIP_TRY(launch_row_pass(ROW_CONV_HEAD, io, compute, a, s));
    HIP_TRY(launch_col_pass(compute, a, coef, s, v));  // warm-up
    float sum = 0.f;
    for (int r = 0; r < kReps; ++r) {
      HIP_TRY(launch_row_pass(ROW_CONV_HEAD, io, compute, a, s));
      HIP_TRY(hipEventRecord(e0, s));
      HIP_TRY(launch_col_pass(compute, a, coef, s, v));
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, e0, e1));
      sum += t;
    }
    ms[v] = sum / kReps;
    if (ms[v] < ms[best]) best = v;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->col_choice[key] = best;
  ctx->col_ms[key] = ms;
  *variant = best;
  return VARSIM_OK;
}

}  // namespace

// =========================================================================================
extern "C" {

varsim_status varsim_create(int device, varsim_ctx** out) {
  if (!out) return VARSIM_ERR_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return VARSIM_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return VARSIM_ERR_DEVICE;
  varsim_ctx* c = new varsim_ctx();
  c->device = device;
  if (hipHostMalloc(&c->active_host, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostGetDevicePointer((void**)&c->active_map, c->active_host, 0) != hipSuccess ||
      hipEventCreateWithFlags(&c->active_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->active_ev[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->desc_ev, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return VARSIM_ERR_NO_MEMORY;
  }
  c->scratch = scratch_address(device);
  *out = c;
  return VARSIM_OK;
}

void varsim_destroy(varsim_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : c->tables) {
    (void)hipFree(kv.second.kper);
    (void)hipFree(kv.second.lam64T);
    (void)hipFree(kv.second.lam32T);
    (void)hipFree(kv.second.coef64);
    (void)hipFree(kv.second.coef32);
  }
  for (auto& kv : c->det_coefs) {
    (void)hipFree(kv.second.coef64);
    (void)hipFree(kv.second.coef32);
  }
  for (auto& kv : c->twiddles) {
    (void)hipFree(kv.second.tw64);
    (void)hipFree(kv.second.tw32);
    (void)hipFree(kv.second.qw64);
    (void)hipFree(kv.second.qw32);
    (void)hipFree(kv.second.tw32lo);
    (void)hipFree(kv.second.qw32lo);
  }
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->desc_ev) (void)hipEventDestroy(c->desc_ev);
  for (hipGraphExec_t g : c->graph_exec)
    if (g) (void)hipGraphExecDestroy(g);
  for (hipEvent_t e : c->graph_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  (void)hipHostFree(c->active_host);
  for (hipEvent_t e : c->active_ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipFree(c->conv_maps);
  delete c;
}

const char* varsim_status_string(varsim_status s) {
  switch (s) {
    case VARSIM_OK: return "ok";
    case VARSIM_ERR_INVALID: return "invalid argument";
    case VARSIM_ERR_UNSUPPORTED: return "unsupported configuration";
    case VARSIM_ERR_NOT_CONVERGED: return "not converged";
    case VARSIM_ERR_RUNAWAY: return "thermal runaway";
    case VARSIM_ERR_DEVICE: return "device error";
    case VARSIM_ERR_NO_MEMORY: return "out of memory";
  }
  return "unknown status";
}

const char* varsim_last_error(const varsim_ctx* c) { return c ? c->err.c_str() : "no context"; }

varsim_status varsim_green_table(varsim_ctx* ctx, const varsim_geometry* geom, void* kernel_out, void* lambda_out,
                                 void* stream) {
  if (!ctx) return VARSIM_ERR_INVALID;
  varsim_status st = check_geometry(ctx, geom);
  if (st != VARSIM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  TableEntry e;
  st = get_table(ctx, geom, s, &e, (double*)lambda_out);
  if (st != VARSIM_OK) return st;
  TwEntry tw;
  if ((st = get_twiddles(ctx, geom->nx, s, &tw)) != VARSIM_OK) return st;
  if ((st = get_twiddles(ctx, geom->ny, s, &tw)) != VARSIM_OK) return st;
  if (kernel_out && is_stack(geom))
    return fail(ctx, VARSIM_ERR_UNSUPPORTED, "K_per is tabulated for a single slab only (lambda_out covers stacks)");
  if (kernel_out)
    HIP_TRY(hipMemcpyAsync(kernel_out, e.kper, (size_t)(geom->nx + 1) * (geom->ny + 1) * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  settle_timing(ctx);
  return VARSIM_OK;
}

varsim_status varsim_conv(varsim_ctx* ctx, const varsim_geometry* geom, int32_t precision, const void* power,
                          void* theta_out, int32_t n_maps, void* stream) {
  if (!ctx) return VARSIM_ERR_INVALID;
  varsim_status st = check_geometry(ctx, geom);
  if (st != VARSIM_OK) return st;
  if (!power || !theta_out || n_maps < 1) return fail(ctx, VARSIM_ERR_INVALID, "power/theta NULL or n_maps < 1");
  if (precision != VARSIM_F32 && precision != VARSIM_F64) return fail(ctx, VARSIM_ERR_INVALID, "bad precision");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  TableEntry tab;
  TwEntry tw, twc;
  if ((st = get_table(ctx, geom, s, &tab)) != VARSIM_OK) return st;
  if ((st = get_twiddles(ctx, geom->nx, s, &tw)) != VARSIM_OK) return st;
  if ((st = get_twiddles(ctx, geom->ny, s, &twc)) != VARSIM_OK) return st;
  const size_t cells = (size_t)geom->nx * geom->ny, es = esize(precision);
  if (ctx->conv_maps_cap < (size_t)n_maps) {
    (void)hipFree(ctx->conv_maps);
    ctx->conv_maps = nullptr;
    ctx->conv_maps_cap = 0;
    if (hipMalloc(&ctx->conv_maps, n_maps * sizeof(MapPtrs)) != hipSuccess)
      return fail(ctx, VARSIM_ERR_NO_MEMORY, "descriptor allocation failed");
    ctx->conv_maps_cap = n_maps;
  }
  wait_descriptors(ctx);
  ctx->h_maps.assign(n_maps, MapPtrs{});
  for (int i = 0; i < n_maps; ++i) {
    ctx->h_maps[i].qd = (const char*)power + i * cells * es;
    ctx->h_maps[i].dT = (char*)theta_out + i * cells * es;
    ctx->h_maps[i].S = ctx->h_maps[i].dT;
  }
  HIP_TRY(hipMemcpyAsync(ctx->conv_maps, ctx->h_maps.data(), n_maps * sizeof(MapPtrs), hipMemcpyHostToDevice, s));
  PassArgs a{};
  a.maps = ctx->conv_maps;
  a.n_maps = n_maps;
  a.n = geom->nx;
  a.ny = geom->ny;
  a.tw = twiddles_of(tw);
  a.twc = twiddles_of(twc);
  a.iter = -1;
  HIP_TRY(timed(ctx, "row_conv_head", s, [&] { return launch_row_pass(ROW_CONV_HEAD, precision, precision, a, s); }));
  HIP_TRY(timed(ctx, "col", s, [&] {
    return launch_col_pass(precision, a, precision == VARSIM_F32 ? (const void*)tab.coef32 : (const void*)tab.coef64, s,
                           ctx->force_col >= 0 ? ctx->force_col : 0);
  }));
  HIP_TRY(timed(ctx, "row_conv_tail", s, [&] { return launch_row_pass(ROW_CONV_TAIL, precision, precision, a, s); }));
  HIP_TRY(hipStreamSynchronize(s));
  settle_timing(ctx);
  return VARSIM_OK;
}

varsim_status varsim_workspace_size(varsim_ctx* ctx, const varsim_problem* problems, int32_t n,
                                    const varsim_options* opts, size_t* bytes) {
  if (!ctx || !problems || n < 1 || !bytes) return fail(ctx, VARSIM_ERR_INVALID, "bad workspace query");
  varsim_status st = check_options(ctx, opts);
  if (st != VARSIM_OK) return st;
  std::vector<const varsim_problem*> ps;
  for (int i = 0; i < n; ++i) {
    if ((st = validate_problem(ctx, &problems[i])) != VARSIM_OK) return st;
    ps.push_back(&problems[i]);
  }
  *bytes = make_layout(ps, opts).total;
  return VARSIM_OK;
}

// The batch solve.  no_alloc: the workspace is the static scratch array and the call allocates
// nothing -- tables and twiddles must be cached, column strip widths are not timed, the loop is
// launched directly (no graphs) and kernel timing is off for the call.
static varsim_status solve_batch_impl(varsim_ctx* ctx, const varsim_problem* problems, int32_t n,
                                      const varsim_options* opts, void* workspace, size_t ws_bytes, varsim_stats* stats,
                                      void* stream, bool no_alloc) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (!problems || n < 1 || !stats || !workspace) return fail(ctx, VARSIM_ERR_INVALID, "NULL argument or n < 1");
  varsim_status st = check_options(ctx, opts);
  if (st != VARSIM_OK) return st;
  for (int i = 0; i < n; ++i)
    if ((st = validate_problem(ctx, &problems[i])) != VARSIM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));

  std::vector<int> order;
  std::vector<Group> groups;
  sort_into_groups(ctx, problems, n, order, groups);
  std::vector<const varsim_problem*> sorted(n);
  for (int i = 0; i < n; ++i) sorted[i] = &problems[order[i]];
  const Layout L = make_layout(sorted, opts);
  if (ws_bytes < L.total) {
    if (no_alloc)
      return fail(ctx, VARSIM_ERR_NO_MEMORY, "batch needs %zu bytes of workspace, more than the %zu-byte static scratch",
                  L.total, ws_bytes);
    return fail(ctx, VARSIM_ERR_NO_MEMORY, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  }
  for (Group& g : groups) {
    if (no_alloc) {
      if ((st = find_cached(ctx, g.geom, &g.table, &g.tw, &g.twc)) != VARSIM_OK) return st;
      continue;
    }
    if ((st = get_table(ctx, g.geom, s, &g.table)) != VARSIM_OK) return st;
    if ((st = get_twiddles(ctx, g.geom->nx, s, &g.tw)) != VARSIM_OK) return st;
    if ((st = get_twiddles(ctx, g.geom->ny, s, &g.twc)) != VARSIM_OK) return st;
  }
  // timing records events from a pool that may grow; a no-allocation call runs untimed
  struct TimingOff {
    varsim_ctx* c;
    bool saved;
    ~TimingOff() { c->timing = saved; }
  } timing_off{ctx, ctx->timing};
  if (no_alloc) ctx->timing = false;

  char* ws = (char*)workspace;
  IterState base{};
  base.resid = (unsigned long long*)(ws + L.resid);
  base.sum = (double*)(ws + L.sum);
  base.maxpack = (unsigned long long*)(ws + L.maxpack);
  base.flags = (unsigned*)(ws + L.flags);
  base.resid64 = (unsigned long long*)(ws + L.resid64);
  base.stride = L.stride;
  base.part = (double*)(ws + L.part);
  base.aa = (double*)(ws + L.aa);
  MapPtrs* d_maps = (MapPtrs*)(ws + L.maps);
  PrepArgs* d_prep = (PrepArgs*)(ws + L.prep);
  int* d_order = (int*)(ws + L.order);
  const bool dev_stats = is_device_ptr(stats);
  varsim_stats* d_stats = (varsim_stats*)(ws + L.stats);
  const int io = opts->precision;
  const bool want_res = opts->final_f64_residual != 0;
  const bool anderson = opts->anderson != 0;

  wait_descriptors(ctx);
  ctx->h_maps.assign(n, MapPtrs{});
  ctx->h_prep.assign(n, PrepArgs{});
  bool any_init = false;
  for (int i = 0; i < n; ++i) {
    const varsim_problem* p = sorted[i];
    MapPtrs& m = ctx->h_maps[i];
    PrepArgs& q = ctx->h_prep[i];
    m.qd = p->q_dyn;
    m.dT = p->dT_out;
    m.S = ws + L.S[i];
    m.S64 = L.S64[i] != (size_t)-1 ? ws + L.S64[i] : nullptr;
    m.init = p->dT_init;
    const bool leak = p->q_leak0 && opts->leak != VARSIM_LEAK_NONE;
    m.ql = leak ? (L.QL[i] != (size_t)-1 ? (const void*)(ws + L.QL[i]) : p->q_leak0) : nullptr;
    m.minv = L.MINV[i] != (size_t)-1 ? ws + L.MINV[i] : nullptr;
    m.ax = L.AX[i] != (size_t)-1 ? ws + L.AX[i] : nullptr;
    m.ag = L.AG[i] != (size_t)-1 ? ws + L.AG[i] : nullptr;
    m.af = L.AF[i] != (size_t)-1 ? ws + L.AF[i] : nullptr;
    q.q_leak0 = p->q_leak0;
    q.leak_var = p->leak_var;
    q.cond_map = p->cond_map;
    q.init = p->dT_init;
    q.ql_out = (leak && L.QL[i] != (size_t)-1) ? ws + L.QL[i] : nullptr;
    q.minv_out = (void*)m.minv;
    q.dT = p->dT_out;
    q.flags = base.flags + i;
    set_source_inputs(m, q, p, L, i, ws);
    any_init = any_init || p->dT_init;
  }

  HIP_TRY(timed(ctx, "setup", s, [&] { return launch_zero_words(ws, L.state_end, s); }));
  HIP_TRY(hipMemcpyAsync(d_maps, ctx->h_maps.data(), n * sizeof(MapPtrs), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_prep, ctx->h_prep.data(), n * sizeof(PrepArgs), hipMemcpyHostToDevice, s));
  if (dev_stats) {
    ctx->h_order = order;
    HIP_TRY(hipMemcpyAsync(d_order, ctx->h_order.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(descriptors_sent(ctx, s));

  auto group_args = [&](const Group& g, int iter) {
    PassArgs a{};
    a.maps = d_maps + g.first;
    a.n_maps = g.count;
    a.n = g.geom->nx;
    a.ny = g.geom->ny;
    a.st = base;
    a.st.resid += (size_t)g.first * L.stride;
    a.st.sum += (size_t)g.first * L.stride;
    a.st.maxpack += (size_t)g.first * L.stride;
    a.st.flags += g.first;
    a.st.resid64 += g.first;
    a.st.part += (size_t)g.first * kRowGroupsMax;
    a.st.aa += (size_t)g.first * kRowGroupsMax * 2;
    a.pp = point_params(g.geom, opts);
    a.tw = twiddles_of(g.tw);
    a.twc = twiddles_of(g.twc);
    a.ct = opts->compensated_twiddles && io == VARSIM_F32 ? 1 : 0;
    a.iter = iter;
    a.zero_start = 0;
    a.lam32 = g.table.lam32T;
    a.lam64 = g.table.lam64T;
    return a;
  };

  // column-pass strip widths (timed on the group's own spectrum arrays before they are used)
  std::vector<int> col_var(groups.size(), 0), col_var64(groups.size(), 0);
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    PassArgs a = group_args(g, 1);
    const void* lam = io == VARSIM_F32 ? (const void*)g.table.coef32 : (const void*)g.table.coef64;
    // the LDS-resident solver has no compensated-twiddle or Anderson variant: such solves take
    // the two-pass path
    const int lim = (opts->compensated_twiddles && io == VARSIM_F32) || opts->anderson
                        ? 0
                        : ctx->small_limit < 0 ? small_max_n(io) : std::min(ctx->small_limit, small_max_n(io));
    if (!(g.geom->nx == g.geom->ny && g.geom->nx <= lim) &&
        (st = col_variant_for(ctx, a, io, io, lam, s, &col_var[gi], !no_alloc)) != VARSIM_OK)
      return st;
    if (want_res) {
      a.use_s64 = io == VARSIM_F32 ? 1 : 0;
      if ((st = col_variant_for(ctx, a, io, VARSIM_F64, g.table.coef64, s, &col_var64[gi], !no_alloc)) != VARSIM_OK)
        return st;
    }
  }

  for (const Group& g : groups) {
    const long cells = (long)g.geom->nx * g.geom->ny;
    HIP_TRY(timed(ctx, "prep", s, [&] { return launch_prep(io, d_prep + g.first, g.count, cells, s); }));
    if (any_init) HIP_TRY(timed(ctx, "prep", s, [&] { return launch_init_copy(io, d_prep + g.first, g.count, cells, s); }));
  }
  // Groups of small maps are solved start to finish by one LDS-resident workgroup per map; the
  // others start with the iteration-1 head P(dT_0) -> row spectrum.  Maps without a warm start
  // use zero_start; in a group mixing warm and cold starts the cold maps get dT_out zeroed.
  std::vector<char> own(groups.size(), 0);
  bool any_loop = false;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    PassArgs a = group_args(g, 1);
    bool all_zero = true;
    for (int i = g.first; i < g.first + g.count; ++i) all_zero = all_zero && !sorted[i]->dT_init;
    a.zero_start = all_zero ? 1 : 0;
    if (!all_zero) {
      for (int i = g.first; i < g.first + g.count; ++i)
        if (!sorted[i]->dT_init)
          HIP_TRY(launch_zero_words(sorted[i]->dT_out, (size_t)g.geom->nx * g.geom->ny * esize(io), s));
    }
    // the LDS-resident solver has no compensated-twiddle or Anderson variant: such solves take
    // the two-pass path
    const int lim = (opts->compensated_twiddles && io == VARSIM_F32) || opts->anderson
                        ? 0
                        : ctx->small_limit < 0 ? small_max_n(io) : std::min(ctx->small_limit, small_max_n(io));
    own[gi] = g.geom->nx == g.geom->ny && g.geom->nx <= lim;  // the LDS-resident solver takes square maps
    if (own[gi]) {
      const void* lam = io == VARSIM_F32 ? (const void*)g.table.coef32 : (const void*)g.table.coef64;
      HIP_TRY(timed(ctx, "small_solve", s, [&] { return launch_small_solve(io, a, opts->max_iter, lam, s); }));
    } else {
      any_loop = true;
      HIP_TRY(timed(ctx, "row_head", s, [&] { return launch_row_pass(ROW_HEAD, io, io, a, s); }));
    }
  }

  // Fixed-point iteration k over every looping group on stream q; slot >= 0 adds the count of
  // maps still iterating after it, written into that pinned host word.
  auto iteration = [&](int k, int slot, hipStream_t q) -> hipError_t {
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      if (own[gi]) continue;
      const Group& g = groups[gi];
      PassArgs a = group_args(g, k);
      bool all_zero = true;
      for (int i = g.first; i < g.first + g.count; ++i) all_zero = all_zero && !sorted[i]->dT_init;
      a.zero_start = all_zero ? 1 : 0;
      const void* lam = io == VARSIM_F32 ? (const void*)g.table.coef32 : (const void*)g.table.coef64;
      hipError_t e = timed(ctx, "col", q, [&] { return launch_col_pass(io, a, lam, q, col_var[gi]); });
      if (e != hipSuccess) return e;
      if (anderson) {  // evaluate G and the residual dot products, then mix the next iterate
        e = timed(ctx, "aa_eval", q, [&] { return launch_row_pass(ROW_AA_EVAL, io, io, a, q); });
        if (e == hipSuccess && k < opts->max_iter)
          e = timed(ctx, "aa_mix", q, [&] { return launch_row_pass(ROW_AA_MIX, io, io, a, q); });
        if (e != hipSuccess) return e;
        continue;
      }
      const int mode = k < opts->max_iter ? ROW_MERGED : ROW_LAST;
      e = timed(ctx, mode == ROW_MERGED ? "row_merged" : "row_last", q,
                [&] { return launch_row_pass(mode, io, io, a, q); });
      if (e != hipSuccess) return e;
    }
    return slot >= 0 ? launch_count_active(base, n, k, opts->tol_K, ctx->active_map + slot, q) : hipSuccess;
  };

  // Convergence is read one step late so that the device never idles: a small kernel behind
  // iteration k (or behind the last iteration of a captured chunk) writes the count of maps still
  // iterating into pinned host memory, and the host waits for the previous step's count only
  // after launching the next step.  Launches past a map's convergence return at once (the map
  // reads its own finished increment), so a chunk may run past the last needed iteration.
  int iters_run = 0;
  const bool graphs = !no_alloc && ctx->graph_chunk > 0 && !ctx->timing && any_loop;
  // A previous call's last counts (possibly queued on another stream, behind iterations the
  // host no longer waited for) land before this call reuses the two words.
  for (int i = 0; any_loop && i < 2; ++i)
    if (ctx->active_live[i]) HIP_TRY(hipEventSynchronize(ctx->active_ev[i]));
  if (!graphs) {
    for (int k = 1; any_loop && k <= opts->max_iter; ++k) {
      const int slot = k & 1;
      HIP_TRY(iteration(k, slot, s));
      HIP_TRY(hipEventRecord(ctx->active_ev[slot], s));
      ctx->active_live[slot] = true;
      iters_run = k;
      if (k >= 2) {
        const int prev = (k - 1) & 1;
        HIP_TRY(hipEventSynchronize(ctx->active_ev[prev]));
        if (ctx->active_host[prev] == 0) break;
      }
    }
  } else {
    const int C = ctx->graph_chunk;
    for (int j = 0, k0 = 1; k0 <= opts->max_iter; ++j, k0 += C) {
      const int k1 = std::min(k0 + C - 1, opts->max_iter);
      const int slot = j & 1;
      if ((int)ctx->graph_exec.size() <= j) {
        ctx->graph_exec.push_back(nullptr);
        ctx->graph_ev.push_back(nullptr);
        ctx->graph_live.push_back(0);
        HIP_TRY(hipEventCreateWithFlags(&ctx->graph_ev[j], hipEventDisableTiming));
      }
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      for (int k = k0; k <= k1 && e == hipSuccess; ++k) e = iteration(k, k == k1 ? slot : -1, ctx->cap_stream);
      const hipError_t e_end = hipStreamEndCapture(ctx->cap_stream, &graph);
      if (e != hipSuccess || e_end != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        HIP_TRY(e);
        HIP_TRY(e_end);
      }
      // the executable graph may still be running from the previous call: its kernel arguments
      // are rewritten only after that launch has finished
      if (ctx->graph_live[j]) HIP_TRY(hipEventSynchronize(ctx->graph_ev[j]));
      bool updated = false;
      if (ctx->graph_exec[j]) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res;
        updated = hipGraphExecUpdate(ctx->graph_exec[j], graph, &bad, &res) == hipSuccess &&
                  res == hipGraphExecUpdateSuccess;
        if (!updated) {
          (void)hipGetLastError();
          (void)hipGraphExecDestroy(ctx->graph_exec[j]);
          ctx->graph_exec[j] = nullptr;
        }
      }
      if (!updated) e = hipGraphInstantiate(&ctx->graph_exec[j], graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) ctx->graph_exec[j] = nullptr;
      HIP_TRY(e);
      HIP_TRY(hipGraphLaunch(ctx->graph_exec[j], s));
      HIP_TRY(hipEventRecord(ctx->graph_ev[j], s));
      ctx->graph_live[j] = 1;
      HIP_TRY(hipEventRecord(ctx->active_ev[slot], s));
      ctx->active_live[slot] = true;
      iters_run = k1;
      if (j >= 1) {
        const int prev = (j - 1) & 1;
        HIP_TRY(hipEventSynchronize(ctx->active_ev[prev]));
        if (ctx->active_host[prev] == 0) break;
      }
    }
  }

  if (want_res) {
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const Group& g = groups[gi];
      PassArgs a = group_args(g, 0);
      a.resid_pass = 1;
      a.use_s64 = io == VARSIM_F32 ? 1 : 0;
      HIP_TRY(timed(ctx, "resid_head", s, [&] { return launch_row_pass(ROW_HEAD, io, VARSIM_F64, a, s); }));
      HIP_TRY(timed(ctx, "resid_col", s,
                    [&] { return launch_col_pass(VARSIM_F64, a, g.table.coef64, s, col_var64[gi]); }));
      HIP_TRY(timed(ctx, "resid_tail", s, [&] { return launch_row_pass(ROW_RESID, io, VARSIM_F64, a, s); }));
    }
  }
  for (const Group& g : groups) {
    PassArgs a = group_args(g, 0);
    HIP_TRY(launch_finalize(a.st, d_maps + g.first, g.count, io, g.geom->nx, g.geom->ny, opts->max_iter, iters_run,
                            opts->tol_K,
                            want_res ? 1 : 0, d_stats + g.first, s));
  }
  if (dev_stats) {  // statistics stay on the device, in the caller's order; no synchronisation
    HIP_TRY(launch_scatter_stats(d_stats, d_order, n, stats, s));
    settle_timing(ctx);
    return VARSIM_OK;
  }
  ctx->h_stats.resize(n);
  HIP_TRY(hipMemcpyAsync(ctx->h_stats.data(), d_stats, n * sizeof(varsim_stats), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  settle_timing(ctx);
  int worst = VARSIM_OK;
  for (int i = 0; i < n; ++i) {
    stats[order[i]] = ctx->h_stats[i];
    const int si = ctx->h_stats[i].status;
    worst = std::max(worst, si);
  }
  if (worst != VARSIM_OK) {
    for (int i = 0; i < n; ++i)
      if (stats[i].status == worst) {
        fail(ctx, (varsim_status)worst, "problem %d: %s", i, varsim_status_string((varsim_status)worst));
        break;
      }
  }
  return (varsim_status)worst;
}

varsim_status varsim_solve_batch(varsim_ctx* ctx, const varsim_problem* problems, int32_t n,
                                 const varsim_options* opts, void* workspace, size_t ws_bytes, varsim_stats* stats,
                                 void* stream) {
  return solve_batch_impl(ctx, problems, n, opts, workspace, ws_bytes, stats, stream, false);
}

varsim_status varsim_solve_batch_noalloc(varsim_ctx* ctx, const varsim_problem* problems, int32_t n,
                                         const varsim_options* opts, varsim_stats* stats, void* stream) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (!ctx->scratch)
    return fail(ctx, VARSIM_ERR_DEVICE, "the static scratch array has no device address on device %d", ctx->device);
  return solve_batch_impl(ctx, problems, n, opts, ctx->scratch, kScratchBytes, stats, stream, true);
}

varsim_status varsim_noalloc_scratch_bytes(size_t* bytes) {
  if (!bytes) return VARSIM_ERR_INVALID;
  *bytes = kScratchBytes;
  return VARSIM_OK;
}

varsim_status varsim_solve_steady(varsim_ctx* ctx, const varsim_problem* problem, const varsim_options* opts,
                                  void* workspace, size_t ws_bytes, varsim_stats* stats, void* stream) {
  return varsim_solve_batch(ctx, problem, 1, opts, workspace, ws_bytes, stats, stream);
}

varsim_status varsim_solve_oneshot(varsim_ctx* ctx, const varsim_problem* problems, int32_t n,
                                   const varsim_options* opts, const varsim_oneshot* os, void* workspace,
                                   size_t ws_bytes, varsim_stats* stats, void* stream) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (!problems || n < 1 || !stats || !workspace || !os)
    return fail(ctx, VARSIM_ERR_INVALID, "NULL argument or n < 1");
  varsim_status st = check_options(ctx, opts);
  if (st != VARSIM_OK) return st;
  if (!(os->mu_W_m2 >= 0) || !std::isfinite(os->mu_W_m2) || (os->random_part != 0 && os->random_part != 1))
    return fail(ctx, VARSIM_ERR_INVALID, "mu_W_m2 must be finite and >= 0, random_part 0 or 1");
  if (opts->cond_model != VARSIM_COND_SOURCE)
    return fail(ctx, VARSIM_ERR_UNSUPPORTED, "the one-shot solve takes the conductivity map on the source side only");
  for (int i = 0; i < n; ++i)
    if ((st = validate_problem(ctx, &problems[i])) != VARSIM_OK) return st;
  const bool leak_on = opts->leak != VARSIM_LEAK_NONE;
  const double beta = leak_on ? opts->beta_per_K : 0.0;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));

  std::vector<int> order;
  std::vector<Group> groups;
  sort_into_groups(ctx, problems, n, order, groups);
  std::vector<const varsim_problem*> sorted(n);
  for (int i = 0; i < n; ++i) sorted[i] = &problems[order[i]];
  const Layout L = make_layout(sorted, opts);
  if (ws_bytes < L.total) return fail(ctx, VARSIM_ERR_NO_MEMORY, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  std::vector<DetEntry> det(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    // the deterministic operator (I - c K) is invertible while c lambda_max = beta mu R < 1
    // (lambda_max = sum of the kernel = R / (hx hy), R the series resistance)
    const double c = beta * (g.geom->lx_m / g.geom->nx) * (g.geom->ly_m / g.geom->ny) * os->mu_W_m2;
    if (beta * os->mu_W_m2 * series_resistance(g.geom) >= 1.0)
      return fail(ctx, VARSIM_ERR_RUNAWAY, "beta mu R >= 1: the linearised leakage has no fixed point");
    if ((st = get_table(ctx, g.geom, s, &g.table)) != VARSIM_OK) return st;
    if ((st = get_twiddles(ctx, g.geom->nx, s, &g.tw)) != VARSIM_OK) return st;
    if ((st = get_twiddles(ctx, g.geom->ny, s, &g.twc)) != VARSIM_OK) return st;
    if ((st = get_det_coef(ctx, g.geom, g.table, c, s, &det[gi])) != VARSIM_OK) return st;
  }

  char* ws = (char*)workspace;
  IterState base{};
  base.resid = (unsigned long long*)(ws + L.resid);
  base.sum = (double*)(ws + L.sum);
  base.maxpack = (unsigned long long*)(ws + L.maxpack);
  base.flags = (unsigned*)(ws + L.flags);
  base.resid64 = (unsigned long long*)(ws + L.resid64);
  base.stride = L.stride;
  base.part = (double*)(ws + L.part);
  MapPtrs* d_maps = (MapPtrs*)(ws + L.maps);
  PrepArgs* d_prep = (PrepArgs*)(ws + L.prep);
  int* d_order = (int*)(ws + L.order);
  varsim_stats* d_stats = (varsim_stats*)(ws + L.stats);
  const bool dev_stats = is_device_ptr(stats);
  const int io = opts->precision;
  const bool want_res = opts->final_f64_residual != 0;

  wait_descriptors(ctx);
  ctx->h_maps.assign(n, MapPtrs{});
  ctx->h_prep.assign(n, PrepArgs{});
  for (int i = 0; i < n; ++i) {
    const varsim_problem* p = sorted[i];
    MapPtrs& m = ctx->h_maps[i];
    PrepArgs& q = ctx->h_prep[i];
    m.qd = p->q_dyn;
    m.dT = p->dT_out;
    m.S = ws + L.S[i];
    m.S64 = L.S64[i] != (size_t)-1 ? ws + L.S64[i] : nullptr;
    const bool leak = p->q_leak0 && leak_on;
    m.ql = leak ? (L.QL[i] != (size_t)-1 ? (const void*)(ws + L.QL[i]) : p->q_leak0) : nullptr;
    m.minv = L.MINV[i] != (size_t)-1 ? ws + L.MINV[i] : nullptr;
    q.q_leak0 = p->q_leak0;
    q.leak_var = p->leak_var;
    q.cond_map = p->cond_map;
    q.ql_out = (leak && L.QL[i] != (size_t)-1) ? ws + L.QL[i] : nullptr;
    q.minv_out = (void*)m.minv;
    q.dT = p->dT_out;
    q.flags = base.flags + i;  // dT_init is not used
    set_source_inputs(m, q, p, L, i, ws);
  }
  HIP_TRY(timed(ctx, "setup", s, [&] { return launch_zero_words(ws, L.state_end, s); }));
  HIP_TRY(hipMemcpyAsync(d_maps, ctx->h_maps.data(), n * sizeof(MapPtrs), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_prep, ctx->h_prep.data(), n * sizeof(PrepArgs), hipMemcpyHostToDevice, s));
  if (dev_stats) {
    ctx->h_order = order;
    HIP_TRY(hipMemcpyAsync(d_order, ctx->h_order.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(descriptors_sent(ctx, s));

  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    const long cells = (long)g.geom->nx * g.geom->ny;
    HIP_TRY(timed(ctx, "prep", s, [&] { return launch_prep(io, d_prep + g.first, g.count, cells, s); }));
    PassArgs a{};
    a.maps = d_maps + g.first;
    a.n_maps = g.count;
    a.n = g.geom->nx;
    a.ny = g.geom->ny;
    a.st = base;
    a.st.resid += (size_t)g.first * L.stride;
    a.st.sum += (size_t)g.first * L.stride;
    a.st.maxpack += (size_t)g.first * L.stride;
    a.st.flags += g.first;
    a.st.resid64 += g.first;
    a.st.part += (size_t)g.first * kRowGroupsMax;
    a.pp = point_params(g.geom, opts);
    a.pp.beta = beta;
    a.pp.os_mu = os->mu_W_m2;
    a.pp.os_rand = os->random_part && leak_on ? 1 : 0;
    a.tw = twiddles_of(g.tw);
    a.twc = twiddles_of(g.twc);
    a.iter = 1;
    a.zero_start = 1;
    const void* dc = io == VARSIM_F32 ? (const void*)det[gi].coef32 : (const void*)det[gi].coef64;
    const auto key = std::make_tuple(a.n, a.ny, io, ilog2(a.n_maps));
    const auto ch = ctx->col_choice.find(key);
    const int var = ctx->force_col >= 0 ? ctx->force_col : (ch != ctx->col_choice.end() ? ch->second : 0);
    // g = hx hy (q_dyn + QL) / m (the head from dT = 0) -> theta_det = DCT-III(lambda_det . DCT-II(g))
    HIP_TRY(timed(ctx, "row_head", s, [&] { return launch_row_pass(ROW_HEAD, io, io, a, s); }));
    HIP_TRY(timed(ctx, "os_col", s, [&] { return launch_col_pass(io, a, dc, s, var); }));
    if (a.pp.os_rand) {  // theta_rand = DCT-III(lambda_det . DCT-II(beta hx hy (QL / m - mu) theta_det))
      HIP_TRY(timed(ctx, "os_mid", s, [&] { return launch_row_pass(ROW_OS_MID, io, io, a, s); }));
      HIP_TRY(timed(ctx, "os_col", s, [&] { return launch_col_pass(io, a, dc, s, var); }));
    }
    HIP_TRY(timed(ctx, "os_tail", s, [&] { return launch_row_pass(ROW_OS_TAIL, io, io, a, s); }));
    if (want_res) {  // distance of the one-shot rise from the fixed point: max |G64(dT) - dT|
      PassArgs r = a;
      r.pp = point_params(g.geom, opts);
      r.iter = 0;
      r.zero_start = 0;
      r.resid_pass = 1;
      r.use_s64 = io == VARSIM_F32 ? 1 : 0;
      HIP_TRY(timed(ctx, "resid_head", s, [&] { return launch_row_pass(ROW_HEAD, io, VARSIM_F64, r, s); }));
      HIP_TRY(timed(ctx, "resid_col", s, [&] { return launch_col_pass(VARSIM_F64, r, g.table.coef64, s, 0); }));
      HIP_TRY(timed(ctx, "resid_tail", s, [&] { return launch_row_pass(ROW_RESID, io, VARSIM_F64, r, s); }));
    }
    HIP_TRY(launch_finalize(a.st, d_maps + g.first, g.count, io, g.geom->nx, g.geom->ny, opts->max_iter, 1, 0.0,
                            want_res ? 1 : 0, d_stats + g.first, s, 1));
  }
  if (dev_stats) {
    HIP_TRY(launch_scatter_stats(d_stats, d_order, n, stats, s));
    settle_timing(ctx);
    return VARSIM_OK;
  }
  ctx->h_stats.resize(n);
  HIP_TRY(hipMemcpyAsync(ctx->h_stats.data(), d_stats, n * sizeof(varsim_stats), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  settle_timing(ctx);
  int worst = VARSIM_OK;
  for (int i = 0; i < n; ++i) {
    stats[order[i]] = ctx->h_stats[i];
    worst = std::max(worst, (int)ctx->h_stats[i].status);
  }
  if (worst != VARSIM_OK)
    fail(ctx, (varsim_status)worst, "one-shot solve: %s", varsim_status_string((varsim_status)worst));
  return (varsim_status)worst;
}

varsim_status varsim_transient_workspace_size(varsim_ctx* ctx, const varsim_problem* problem,
                                              const varsim_transient* tr, const varsim_options* opts, size_t* bytes) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (!bytes) return fail(ctx, VARSIM_ERR_INVALID, "bytes is NULL");
  varsim_status st = check_transient(ctx, problem, tr, opts);
  if (st != VARSIM_OK) return st;
  *bytes = make_transient_layout(problem, tr, opts).total;
  return VARSIM_OK;
}

varsim_status varsim_solve_transient(varsim_ctx* ctx, const varsim_problem* problem, const varsim_transient* tr,
                                     const varsim_options* opts, void* dT_steps_out, void* workspace, size_t ws_bytes,
                                     varsim_stats* stats, void* stream) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (!stats || !workspace) return fail(ctx, VARSIM_ERR_INVALID, "NULL stats or workspace");
  varsim_status st = check_transient(ctx, problem, tr, opts);
  if (st != VARSIM_OK) return st;
  const TransLayout L = make_transient_layout(problem, tr, opts);
  if (ws_bytes < L.total)
    return fail(ctx, VARSIM_ERR_NO_MEMORY, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  const varsim_geometry* g = problem->geom;
  TableEntry tab;
  TwEntry tw;
  if ((st = get_table(ctx, g, s, &tab)) != VARSIM_OK) return st;
  if ((st = get_twiddles(ctx, g->nx, s, &tw)) != VARSIM_OK) return st;

  const int io = opts->precision;
  const long cells = (long)g->nx * g->ny;
  char* ws = (char*)workspace;
  unsigned* d_flags = (unsigned*)(ws + L.flags);
  varsim_stats* d_stats = (varsim_stats*)(ws + L.stats);
  PrepArgs* d_prep = (PrepArgs*)(ws + L.prep);
  const bool leak = problem->q_leak0 && opts->leak != VARSIM_LEAK_NONE;

  TransArgs a{};
  a.n = g->nx;
  a.S = ws + L.S;
  a.state = ws + L.state;
  a.poles = poles_of(tr);
  a.ab = ws + L.ab;
  a.ids = (const int*)(ws + L.ids);
  a.trace = tr->trace;
  a.n_blocks = tr->n_blocks;
  a.ql = leak ? (L.QL != (size_t)-1 ? (const void*)(ws + L.QL) : problem->q_leak0) : nullptr;
  a.minv = L.MINV != (size_t)-1 ? ws + L.MINV : nullptr;
  a.dT = problem->dT_out;
  a.snaps = dT_steps_out;
  a.out_every = tr->out_every;
  a.flags = d_flags;
  a.pp = point_params(g, opts);
  a.tw = twiddles_of(tw);
  a.idz = (const int*)(ws + L.IDZ);
  a.qlz = a.ql ? ws + L.QLZ : nullptr;
  a.minvz = a.minv ? ws + L.MINVZ : nullptr;
  a.hist = tr->history_steps;
  a.ring = a.hist >= 2 ? ws + L.ring : nullptr;
  a.fir = a.hist >= 2 ? ws + L.fir : nullptr;
  a.slot = 0;
  const size_t ring_bytes = a.ring ? (size_t)(a.hist - 1) * cells * esize(io) : 0;

  wait_descriptors(ctx);
  ctx->h_prep.assign(1, PrepArgs{});
  PrepArgs& q = ctx->h_prep[0];
  q.q_leak0 = problem->q_leak0;
  q.leak_var = problem->leak_var;
  q.cond_map = problem->cond_map;
  q.ql_out = (leak && L.QL != (size_t)-1) ? ws + L.QL : nullptr;
  q.minv_out = (void*)a.minv;
  q.dT = problem->dT_out;
  q.flags = d_flags;

  // static inputs: flags, spectral state, QL, 1/m, block ids, per-mode (a, b)
  const TableSpec sp = spec_of(g);
  const double alpha = sp.k_ref / g->layers[0].rho_c_J_m3K;
  HIP_TRY(timed(ctx, "setup", s, [&] { return launch_zero_words(ws, L.state_end, s); }));
  HIP_TRY(timed(ctx, "setup", s, [&] { return launch_zero_words(a.state, (size_t)a.poles * cells * esize(io), s); }));
  if (a.ring) HIP_TRY(timed(ctx, "setup", s, [&] { return launch_zero_words(a.ring, ring_bytes, s); }));
  HIP_TRY(hipMemcpyAsync(d_prep, ctx->h_prep.data(), sizeof(PrepArgs), hipMemcpyHostToDevice, s));
  HIP_TRY(timed(ctx, "prep", s, [&] { return launch_prep(io, d_prep, 1, cells, s); }));
  HIP_TRY(timed(ctx, "setup", s, [&] {
    return launch_block_ids(tr->block_rects, tr->n_blocks, (int*)a.ids, g->nx, g->ny, s);
  }));
  HIP_TRY(timed(ctx, "setup", s, [&] {
    return launch_transient_coef(sp, tab.lam64T, io, (void*)a.ab, (void*)a.fir, a.hist, alpha, tr->dt_s,
                                 tr->tau_model, g->layers[0].rho_c_J_m3K, a.poles, s);
  }));
  if (transient_single_ok(g->nx)) {
    HIP_TRY(timed(ctx, "setup", s, [&] { return launch_zorder(4, a.ids, (void*)a.idz, g->nx, s); }));
    if (a.ql)
      HIP_TRY(timed(ctx, "setup", s, [&] { return launch_zorder((int)esize(io), a.ql, (void*)a.qlz, g->nx, s); }));
    if (a.minv)
      HIP_TRY(timed(ctx, "setup", s, [&] { return launch_zorder((int)esize(io), a.minv, (void*)a.minvz, g->nx, s); }));
  }
  unsigned h_flags = 0;
  HIP_TRY(hipMemcpyAsync(&h_flags, d_flags, sizeof h_flags, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  settle_timing(ctx);
  if (h_flags & kFlagInvalid) {
    varsim_stats bad{};
    bad.status = VARSIM_ERR_INVALID;
    bad.last_increment_K = bad.residual_f64_K = bad.dT_max_K = bad.dT_mean_K = NAN;
    bad.hotspot_index = -1;
    *stats = bad;
    return fail(ctx, VARSIM_ERR_INVALID, "conductivity map must be positive and finite");
  }

  // launch shapes: tuned once per (n, precision) when autotuning is on.  The candidates run on
  // this call's workspace (no snapshots), after which the spectral state and flags are reset.
  const int nv = transient_variants(g->nx);
  int rv = nv > 3 ? 3 : 0, cv = rv;  // untuned default: one-sequence passes where available
  const auto key = std::make_pair(g->nx, io);
  auto it = ctx->tr_choice.find(key);
  if (ctx->force_col >= 0 && ctx->force_col < nv) {
    rv = cv = ctx->force_col;
  } else if (it != ctx->tr_choice.end()) {
    rv = it->second.first;
    cv = it->second.second;
  } else if (ctx->autotune && ctx->force_tr_row < 0 && ctx->force_tr_col < 0) {
    TransArgs t = a;
    t.snaps = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // Candidates are timed inside whole steps (column pass + row pass, as the solve runs them),
    // every (row, column) pair of one pass family, since the best row pass depends on the column
    // pass before it; each pair over 60 steps, two rounds, the faster round kept, after a long
    // untimed burst.  Where the one-sequence passes exist (n >= 64) only their pairs are timed
    // (with the split one-sequence passes where those exist, n = 1024):
    // they were the faster family in every long solve measured, while short timed bursts that
    // follow other GPU work (steady solves in the same process) can rank the two families the
    // other way round (the two-sequence rows measured faster in the bursts and ran 1.18x slower
    // in the solve).
    auto steps = [&](int r, int c, int count) -> hipError_t {
      for (int q = 0; q < count; ++q) {
        hipError_t e = launch_transient_col(io, t, s, c);
        if (e == hipSuccess) e = launch_transient_row(TR_MERGED, io, t, 1, s, r);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    };
    // a burst of 10 untimed steps first: the launches that follow an idle gap (the previous
    // candidate's synchronisation) run slower than those of a long solve and would skew the
    // comparison
    auto time_steps = [&](int r, int c, float* out) -> hipError_t {
      constexpr int kTimed = 60;
      hipError_t e = steps(r, c, 10);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      if (e == hipSuccess) e = steps(r, c, kTimed);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float el = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&el, e0, e1);
      *out = std::min(*out, el / kTimed);
      return e;
    };
    HIP_TRY(steps(rv, cv, 400));
    const int lo = nv > 3 ? 3 : 0, hi = nv > 3 ? nv : 3;  // the family of candidates timed
    std::vector<float> ms(nv * nv, -1.f);  // ms[row * nv + column]; -1: not timed
    for (int r = lo; r < hi; ++r)
      for (int c = lo; c < hi; ++c) ms[r * nv + c] = 1e30f;
    for (int round = 0; round < 2; ++round)
      for (int r = lo; r < hi; ++r)
        for (int c = lo; c < hi; ++c) HIP_TRY(time_steps(r, c, &ms[r * nv + c]));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int best = lo * nv + lo;
    for (int r = lo; r < hi; ++r)
      for (int c = lo; c < hi; ++c)
        if (ms[r * nv + c] < ms[best]) best = r * nv + c;
    rv = best / nv;
    cv = best % nv;
    ctx->tr_choice[key] = {rv, cv};
    ctx->tr_ms[key] = ms;
    HIP_TRY(launch_zero_words(a.state, (size_t)a.poles * cells * esize(io), s));
    if (a.ring) HIP_TRY(launch_zero_words(a.ring, ring_bytes, s));
    HIP_TRY(launch_zero_words(d_flags, sizeof(unsigned), s));
  }
  if (ctx->force_tr_row >= 0) rv = ctx->force_tr_row < nv ? ctx->force_tr_row : 0;
  if (ctx->force_tr_col >= 0) cv = ctx->force_tr_col < nv ? ctx->force_tr_col : 0;

  // step n: column pass (mode update with P_n) then row pass (dT_n, and P_{n+1} unless last)
  HIP_TRY(timed(ctx, "tr_row_head", s, [&] { return launch_transient_row(TR_HEAD, io, a, 0, s, rv); }));
  for (int n = 1; n <= tr->n_steps; ++n) {
    if (a.ring) a.slot = n % (a.hist - 1);  // holds P_hat of step n - (hist - 1) until this step's enters
    HIP_TRY(timed(ctx, "tr_col", s, [&] { return launch_transient_col(io, a, s, cv); }));
    const bool last = n == tr->n_steps;
    HIP_TRY(timed(ctx, last ? "tr_row_last" : "tr_row", s,
                  [&] { return launch_transient_row(last ? TR_LAST : TR_MERGED, io, a, n, s, rv); }));
  }
  HIP_TRY(launch_map_stats(io, problem->dT_out, cells, d_flags, tr->n_steps, d_stats, s));
  HIP_TRY(hipMemcpyAsync(stats, d_stats, sizeof(varsim_stats), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  settle_timing(ctx);
  if (stats->status != VARSIM_OK)
    return fail(ctx, (varsim_status)stats->status, "transient: %s", varsim_status_string((varsim_status)stats->status));
  return VARSIM_OK;
}

varsim_status varsim_set_autotune(varsim_ctx* ctx, int32_t enable) {
  if (!ctx) return VARSIM_ERR_INVALID;
  ctx->autotune = enable != 0;
  if (enable < 0) {
    ctx->col_choice.clear();
    ctx->col_ms.clear();
    ctx->tr_choice.clear();
    ctx->tr_ms.clear();
  }
  return VARSIM_OK;
}

varsim_status varsim_set_small_path(varsim_ctx* ctx, int32_t max_n) {
  if (!ctx) return VARSIM_ERR_INVALID;
  ctx->small_limit = max_n < 0 ? -1 : max_n;
  return VARSIM_OK;
}

varsim_status varsim_force_col_variant(varsim_ctx* ctx, int32_t variant) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (variant < -1 || variant >= kColVariants) return fail(ctx, VARSIM_ERR_INVALID, "variant must be in [-1, %d]", kColVariants - 1);
  ctx->force_col = variant;
  return VARSIM_OK;
}

varsim_status varsim_set_graph_iterations(varsim_ctx* ctx, int32_t iterations) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (iterations < 0 || iterations > kMaxGraphIterations)
    return fail(ctx, VARSIM_ERR_INVALID, "iterations per graph must be in [0, %d]", kMaxGraphIterations);
  if (iterations > 0 && !ctx->cap_stream) {
    if (hipSetDevice(ctx->device) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      ctx->cap_stream = nullptr;
      return fail(ctx, VARSIM_ERR_DEVICE, "capture stream: %s", hipGetErrorString(hipGetLastError()));
    }
  }
  ctx->graph_chunk = iterations;
  return VARSIM_OK;
}

varsim_status varsim_force_transient_variant(varsim_ctx* ctx, int32_t row_variant, int32_t col_variant) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (row_variant < -1 || row_variant >= kTrVariants || col_variant < -1 || col_variant >= kTrVariants)
    return fail(ctx, VARSIM_ERR_INVALID, "transient variants must be in [-1, %d]", kTrVariants - 1);
  ctx->force_tr_row = row_variant;
  ctx->force_tr_col = col_variant;
  return VARSIM_OK;
}

varsim_status varsim_autotune_export(varsim_ctx* ctx, char* buf, size_t len, size_t* needed) {
  if (!ctx) return VARSIM_ERR_INVALID;
  std::string out = "varsim-tuning 1\n";
  char line[128];
  for (const auto& kv : ctx->col_choice) {
    snprintf(line, sizeof line, "col %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first),
             std::get<2>(kv.first), std::get<3>(kv.first), kv.second);
    out += line;
  }
  for (const auto& kv : ctx->tr_choice) {
    snprintf(line, sizeof line, "tr %d %d %d %d\n", kv.first.first, kv.first.second, kv.second.first,
             kv.second.second);
    out += line;
  }
  if (needed) *needed = out.size() + 1;
  if (!buf) return VARSIM_OK;
  if (len < out.size() + 1) return fail(ctx, VARSIM_ERR_NO_MEMORY, "buffer of %zu bytes < %zu", len, out.size() + 1);
  memcpy(buf, out.c_str(), out.size() + 1);
  return VARSIM_OK;
}

varsim_status varsim_autotune_import(varsim_ctx* ctx, const char* text) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (!text) return fail(ctx, VARSIM_ERR_INVALID, "text is NULL");
  // parse everything first; the context changes only if every line is valid
  std::vector<std::pair<std::tuple<int, int, int, int>, int>> cols;
  std::vector<std::pair<std::pair<int, int>, std::pair<int, int>>> trs;
  auto pow2_in = [](int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; };
  auto prec_ok = [](int p) { return p == VARSIM_F32 || p == VARSIM_F64; };
  const char* p = text;
  int lineno = 0;
  bool header = false;
  while (*p) {
    const char* e = strchr(p, '\n');
    const size_t n = e ? (size_t)(e - p) : strlen(p);
    std::string ln(p, n);
    p += n + (e ? 1 : 0);
    ++lineno;
    if (ln.find_first_not_of(" \t\r") == std::string::npos) continue;
    int a0, a1, a2, a3, a4, used = 0;
    if (!header) {
      if (sscanf(ln.c_str(), "varsim-tuning %d %n", &a0, &used) != 1 || a0 != 1 || ln.c_str()[used])
        return fail(ctx, VARSIM_ERR_INVALID, "line %d: expected the header 'varsim-tuning 1'", lineno);
      header = true;
    } else if (sscanf(ln.c_str(), "col %d %d %d %d %d %n", &a0, &a1, &a2, &a3, &a4, &used) == 5 && !ln.c_str()[used]) {
      if (!pow2_in(a0, 16, 1024) || !pow2_in(a1, 16, 1024) || !prec_ok(a2) || a3 < 0 || a3 > 30 || a4 < 0 ||
          a4 >= kColVariants)
        return fail(ctx, VARSIM_ERR_INVALID, "line %d: column choice out of range", lineno);
      cols.push_back({std::make_tuple(a0, a1, a2, a3), a4});
    } else if (sscanf(ln.c_str(), "tr %d %d %d %d %n", &a0, &a1, &a2, &a3, &used) == 4 && !ln.c_str()[used]) {
      if (!pow2_in(a0, 16, 1024) || !prec_ok(a1) || a2 < 0 || a2 >= transient_variants(a0) || a3 < 0 ||
          a3 >= transient_variants(a0))
        return fail(ctx, VARSIM_ERR_INVALID, "line %d: transient choice out of range", lineno);
      trs.push_back({{a0, a1}, {a2, a3}});
    } else {
      return fail(ctx, VARSIM_ERR_INVALID, "line %d: not a tuning record", lineno);
    }
  }
  if (!header) return fail(ctx, VARSIM_ERR_INVALID, "no 'varsim-tuning 1' header");
  for (const auto& c : cols) {
    ctx->col_choice[c.first] = c.second;
    ctx->col_ms.erase(c.first);
  }
  for (const auto& t : trs) {
    ctx->tr_choice[t.first] = t.second;
    ctx->tr_ms.erase(t.first);
  }
  return VARSIM_OK;
}

varsim_status varsim_autotune_report(varsim_ctx* ctx, char* buf, size_t len) {
  if (!ctx || !buf || !len) return VARSIM_ERR_INVALID;
  std::string out;
  char line[256];
  for (const auto& kv : ctx->col_choice) {
    const int nx = std::get<0>(kv.first), n = std::get<1>(kv.first), c = std::get<2>(kv.first),
              b = std::get<3>(kv.first);
    if (nx == n)
      snprintf(line, sizeof line, "col n=%d %s maps>=%d:", n, c == VARSIM_F32 ? "f32" : "f64", 1 << b);
    else
      snprintf(line, sizeof line, "col nx=%d ny=%d %s maps>=%d:", nx, n, c == VARSIM_F32 ? "f32" : "f64", 1 << b);
    out += line;
    const auto found = ctx->col_ms.find(kv.first);
    if (found == ctx->col_ms.end()) {
      snprintf(line, sizeof line, " %d cols x%d%s (imported)\n", col_pass_columns(c, n, kv.second),
               col_pass_pairs(c, n, kv.second),
               col_pass_family(c, n, kv.second) ? " one-column" : col_pass_pipelined(c, n, kv.second) ? " pipelined" : "");
      out += line;
      continue;
    }
    const auto& ms = found->second;
    for (int v = 0; v < (int)ms.size(); ++v) {
      if (ms[v] < 0.f) continue;  // another transform family, not timed
      snprintf(line, sizeof line, " %d cols x%d%s %.4f ms%s", col_pass_columns(c, n, v), col_pass_pairs(c, n, v),
               col_pass_family(c, n, v) ? " one-column" : col_pass_pipelined(c, n, v) ? " pipelined" : "", ms[v],
               v == kv.second ? "*" : "");
      out += line;
    }
    out += "\n";
  }
  for (const auto& kv : ctx->tr_choice) {
    const auto found = ctx->tr_ms.find(kv.first);
    if (found == ctx->tr_ms.end()) {
      snprintf(line, sizeof line, "transient n=%d %s row candidate %d column candidate %d (imported)\n", kv.first.first,
               kv.first.second == VARSIM_F32 ? "f32" : "f64", kv.second.first, kv.second.second);
      out += line;
      continue;
    }
    const auto& ms = found->second;
    int nv = 0;
    while (nv * nv < (int)ms.size()) ++nv;
    snprintf(line, sizeof line, "transient n=%d %s ms per step, row candidate: column candidates", kv.first.first,
             kv.first.second == VARSIM_F32 ? "f32" : "f64");
    out += line;
    for (int r = 0; r < nv; ++r) {
      snprintf(line, sizeof line, "%s r%d:", r ? ";" : "", r);
      out += line;
      for (int c = 0; c < nv; ++c) {
        const bool chosen = r == kv.second.first && c == kv.second.second;
        if (ms[r * nv + c] < 0.f)
          snprintf(line, sizeof line, " -");
        else
          snprintf(line, sizeof line, " %.4f%s", ms[r * nv + c], chosen ? "*" : "");
        out += line;
      }
    }
    out += "\n";
  }
  snprintf(buf, len, "%s", out.c_str());
  return out.size() < len ? VARSIM_OK : VARSIM_ERR_NO_MEMORY;
}

varsim_status varsim_set_timing(varsim_ctx* ctx, int32_t enable) {
  if (!ctx) return VARSIM_ERR_INVALID;
  ctx->timing = enable != 0;
  HIP_TRY(hipSetDevice(ctx->device));
  // events for the launches to come are created now, not between a call's launches
  constexpr size_t kEventStock = 4096;
  while (ctx->timing && ctx->pool.size() + 2 * ctx->pending.size() < kEventStock) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return fail(ctx, VARSIM_ERR_DEVICE, "hipEventCreate failed");
    ctx->pool.push_back(e);
  }
  return VARSIM_OK;
}

varsim_status varsim_set_timing_only(varsim_ctx* ctx, const char* kernel_class) {
  if (!ctx) return VARSIM_ERR_INVALID;
  ctx->timing_only = kernel_class ? kernel_class : "";
  return VARSIM_OK;
}

varsim_status varsim_reset_timing(varsim_ctx* ctx) {
  if (!ctx) return VARSIM_ERR_INVALID;
  flush_timing(ctx);  // launches recorded before the reset do not count after it
  ctx->times.clear();
  ctx->class_names.clear();
  return VARSIM_OK;
}

varsim_status varsim_kernel_times(varsim_ctx* ctx, const char** names, int64_t* counts, double* total_ms,
                                  int32_t* n_io) {
  if (!ctx || !n_io) return VARSIM_ERR_INVALID;
  flush_timing(ctx);  // waits for the recorded launches
  const int cap = *n_io;
  int k = 0;
  for (const char* nm : ctx->class_names) {
    if (k >= cap) break;
    const auto& v = ctx->times[nm];
    if (names) names[k] = nm;
    if (counts) counts[k] = v.first;
    if (total_ms) total_ms[k] = v.second;
    ++k;
  }
  *n_io = k;
  return VARSIM_OK;
}

}  // extern "C"
