// The library context and the helpers every entry point shares: error reporting and
// optional per-kernel-class event timing.
#pragma once

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace vs {

struct TableEntry {
  double* kper = nullptr;
  double* lam64T = nullptr;
  float* lam32T = nullptr;
  double* coef64 = nullptr;
  float* coef32 = nullptr;
};

struct TwEntry {
  Cx<double>* tw64 = nullptr;
  Cx<float>* tw32 = nullptr;
  Cx<double>* qw64 = nullptr;
  Cx<float>* qw32 = nullptr;
  Cx<float>* tw32lo = nullptr;  // low parts of tw32 / qw32 (compensated twiddles)
  Cx<float>* qw32lo = nullptr;
};

inline Twiddles twiddles_of(const TwEntry& e) { return Twiddles{e.tw64, e.tw32, e.qw64, e.qw32, e.tw32lo, e.qw32lo}; }

// (nx, ny, lx, ly, t1, k1_ref, {bottom_bc, h, t2, k2_ref, t3, k3_ref, ...} for a stack)
using TableKey = std::tuple<int, int, double, double, double, double, std::vector<double>>;

// Column coefficients of the one-shot solve's deterministic operator, per (geometry, c).
struct DetEntry {
  double* coef64 = nullptr;
  float* coef32 = nullptr;
};

struct TimedEvent {
  const char* cls;
  hipEvent_t a, b;
};

}  // namespace vs

struct varsim_ctx {
  using TableKey = vs::TableKey;
  using TableEntry = vs::TableEntry;
  using TwEntry = vs::TwEntry;
  using TimedEvent = vs::TimedEvent;
  using MapPtrs = vs::MapPtrs;
  using PrepArgs = vs::PrepArgs;
  int device = 0;
  void* scratch = nullptr;  // device address of the static scratch array on `device`
  std::string err;
  std::map<TableKey, TableEntry> tables;
  std::map<std::pair<TableKey, double>, vs::DetEntry> det_coefs;
  std::map<int, TwEntry> twiddles;
  bool timing = false;
  std::string timing_only;  // non-empty: only this kernel class is timed
  std::vector<TimedEvent> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<long long, double>> times;
  std::vector<const char*> class_names;
  // fixed-point iterations per captured graph (0: direct launches).  Chunk j of a call is
  // captured on the private stream cap_stream and written into executable graph j with
  // hipGraphExecUpdate (instantiated anew when the launch structure changed); graph_ev[j] is
  // recorded after its last launch, and the next update of that graph waits for it
  int graph_chunk = 0;
  hipStream_t cap_stream = nullptr;
  std::vector<hipGraphExec_t> graph_exec;
  std::vector<hipEvent_t> graph_ev;
  std::vector<char> graph_live;  // graph_ev[j] has been recorded
  int* active_host = nullptr;  // [2] pinned host words: counts of maps still iterating
  int* active_map = nullptr;   // the same words as the device addresses them
  hipEvent_t active_ev[2] = {nullptr, nullptr};
  bool active_live[2] = {false, false};  // active_ev[i] has been recorded
  // host staging of per-call descriptor arrays (kept alive until the call returns)
  std::vector<MapPtrs> h_maps;
  std::vector<PrepArgs> h_prep;
  std::vector<varsim_stats> h_stats;
  std::vector<int> h_order;  // caller index of each sorted problem (device-side statistics)
  // recorded after the host descriptor arrays above are copied to the device; a call that
  // returns before its stream finishes (device-side statistics) leaves it pending, and the next
  // call waits on it before refilling the arrays
  hipEvent_t desc_ev = nullptr;
  bool desc_pending = false;
  MapPtrs* conv_maps = nullptr;
  size_t conv_maps_cap = 0;
  // column-pass strip width chosen by timing, per (nx, ny, compute type, log2 of the group size)
  bool autotune = false;
  int force_col = -1;  // >= 0: every column pass uses this strip-width candidate
  int force_tr_row = -1, force_tr_col = -1;  // >= 0: transient passes use these candidates
  int small_limit = -1;  // largest N solved by one LDS-resident workgroup (-1: library default, 0: off)
  std::map<std::tuple<int, int, int, int>, int> col_choice;
  std::map<std::tuple<int, int, int, int>, std::vector<float>> col_ms;
  // transient launch shapes per (n, precision): (row variant, column variant) and their timings
  std::map<std::pair<int, int>, std::pair<int, int>> tr_choice;
  std::map<std::pair<int, int>, std::vector<float>> tr_ms;
};

namespace {

inline varsim_status fail(varsim_ctx* c, varsim_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define HIP_TRY(expr)                                                                            \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return fail(ctx, VARSIM_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

inline void wait_descriptors(varsim_ctx* c) {
  if (c->desc_pending) {
    (void)hipEventSynchronize(c->desc_ev);
    c->desc_pending = false;
  }
}

inline hipError_t descriptors_sent(varsim_ctx* c, hipStream_t s) {
  if (!c->desc_ev) {
    const hipError_t e = hipEventCreateWithFlags(&c->desc_ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  const hipError_t e = hipEventRecord(c->desc_ev, s);
  c->desc_pending = e == hipSuccess;
  return e;
}

inline hipEvent_t take_event(varsim_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

template <class F>
hipError_t timed(varsim_ctx* c, const char* cls, hipStream_t s, F&& f) {
  if (!c->timing || (!c->timing_only.empty() && c->timing_only != cls)) return f();
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  (void)hipEventRecord(a, s);
  const hipError_t e = f();
  (void)hipEventRecord(b, s);
  c->pending.push_back({cls, a, b});
  return e;
}

inline void flush_timing(varsim_ctx* c) {
  for (auto& p : c->pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    auto& slot = c->times[p.cls];
    if (slot.first == 0 &&
        std::find_if(c->class_names.begin(), c->class_names.end(), [&](const char* n) { return !strcmp(n, p.cls); }) ==
            c->class_names.end())
      c->class_names.push_back(p.cls);
    slot.first += 1;
    slot.second += ms;
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
}

// Timing results are read lazily (when the caller asks for them, or when many launches are
// pending), so the event reads add no host time between a call's last kernel and the next call.
inline void settle_timing(varsim_ctx* c) {
  if (c->pending.size() >= 8192) flush_timing(c);
}

}  // namespace
