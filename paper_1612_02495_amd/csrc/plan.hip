// C ABI of the swept library: argument validation, tiling, phase schedule,
// workspace ownership and launch sequencing (declared in include/swept.h).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device_guard.h"
#include "internal.h"
#include "poison.h"
#include "swept.h"

using swept::Consts;
using swept::PhaseArgs;

// Edge slots of swept_run_noalloc: one array per device, in the code object's
// device memory, held by each GPU the library runs on until the process ends.
// Host code never uses its name as an address (on the host it is a stand-in
// symbol): the device address comes from hipGetSymbolAddress, taken once per
// device with that device current.
static constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace

int swept::set_error(int code, const std::string& msg) { return fail(code, msg); }

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(SWEPT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int radius_of(int kind) { return kind == SWEPT_KS_RK2 ? 2 : 1; }

bool valid_kind(int kind) {
  return kind == SWEPT_HEAT_FTCS || kind == SWEPT_KS_RK2 || kind == SWEPT_HEAT_INSULATED;
}

// The stencil a kind runs (the insulated rod is the heat stencil with mirror
// ghosts at its two end nodes).
int stencil_of(int kind) { return kind == SWEPT_KS_RK2 ? swept::kKS : swept::kHeat; }

constexpr int kMinTile = 4;
constexpr int kMinGeneral = 32;  // smallest grid of the uneven tiling
constexpr int kMaxTile = 4096;

// Tile width rules: w = 2s * (tiers of a full triangle); KS phases must end
// on whole timesteps (predictor + final), so w/4 has to be even.
bool tile_ok(int kind, int w, const char** why) {
  const int s = radius_of(kind);
  if (w < kMinTile || w > kMaxTile) {
    *why = "tile_width must lie in [4, 4096]";
    return false;
  }
  if (w % (2 * s) != 0) {
    *why = "tile_width must be a multiple of 2 * stencil radius";
    return false;
  }
  if (kind == SWEPT_KS_RK2 && w % 8 != 0) {
    *why = "KS tile_width must be a multiple of 8 (whole timesteps per phase)";
    return false;
  }
  return true;
}

// Tiers of a full (pure) triangle for this kind and width.
int full_tiers(int kind, int w) {
  const int s = radius_of(kind);
  int h = w / (2 * s);
  if (kind == SWEPT_KS_RK2) h &= ~1;
  return h;
}

int tiers_per_step(int kind) { return kind == SWEPT_KS_RK2 ? 2 : 1; }

bool is_finite(double x) { return std::isfinite(x); }

// Edge-set heights: full phases of h tiers, remainder last.
void make_schedule(int h, int64_t tiers, std::vector<int32_t>* e) {
  e->clear();
  if (tiers <= 0) return;
  const int64_t full = tiers / h;
  const int64_t rem = tiers % h;
  e->reserve((size_t)(full + (rem ? 1 : 0)));
  for (int64_t i = 0; i < full; ++i) e->push_back(h);
  if (rem) e->push_back((int32_t)rem);
}

}  // namespace

struct swept_plan_s {
  int64_t n = 0;
  int kind = 0;
  int dtype = 0;
  int s = 1;
  int w = 0;
  int h = 0;       // tiers per full phase
  int64_t nt = 0;  // tiles
  int engine = SWEPT_ENGINE_AUTO;
  bool general = false;  // uneven tiling: w does not divide n (compacted engine only)
  bool lds_fits = true;  // the LDS engine's tile fits the device's LDS
  int device = 0;
  void* slots = nullptr;
  size_t slots_bytes = 0;
  void* buf = nullptr;  // naive ping-pong / predictor buffer
  size_t buf_bytes = 0;
  bool poison = false;  // SWEPT_DEBUG_POISON: NaN-fill the slots (and the tiles' LDS) before each run
  int checks = 0;       // SWEPT_CHECK_* flags (swept_plan_set_checks)
  int* flag = nullptr;  // device flag of the non-finite check
  Consts<double> kd{};
  Consts<float> kf{};
};

namespace {

size_t elem_size(int dtype) { return dtype == SWEPT_F64 ? sizeof(double) : sizeof(float); }

// The insulated rod has kernels in the compacted engine only.
bool engine_supports(int engine, int kind, int w) {
  const int st = stencil_of(kind);
  if (kind == SWEPT_HEAT_INSULATED)
    return (engine == SWEPT_ENGINE_COMPACT || engine == SWEPT_ENGINE_AUTO) && swept::compact_engine_supports(st, w);
  if (engine == SWEPT_ENGINE_WAVE) return swept::wave_engine_supports(st, w);
  if (engine == SWEPT_ENGINE_COMPACT) return swept::compact_engine_supports(st, w);
  return true;
}

// The engine that runs the phases: the chosen one, or for AUTO the compacted
// engine where it has a kernel, else the register engine, else LDS.
int resolve_engine(int engine, int kind, int w) {
  if (engine != SWEPT_ENGINE_AUTO) return engine;
  const int st = stencil_of(kind);
  if (swept::compact_engine_supports(st, w)) return SWEPT_ENGINE_COMPACT;
  return swept::wave_engine_supports(st, w) ? SWEPT_ENGINE_WAVE : SWEPT_ENGINE_LDS;
}

int resolved_engine(const swept_plan_s* p) { return resolve_engine(p->engine, p->kind, p->w); }

// A phase is one launch of one workgroup per tile, and a dispatch counts its
// work-items in 32 bits: n / w tiles times the engine's work-items per tile
// must stay below 2^32.
bool launch_fits(int engine, int kind, int w, int64_t nt) {
  const int e = resolve_engine(engine, kind, w);
  const int64_t per_tile = e == SWEPT_ENGINE_LDS ? swept::phase_lds_threads(w) : 64;
  return nt * per_tile <= (int64_t)UINT32_MAX;
}

const char* kTooManyTiles = "n / tile_width tiles exceed one launch of this engine (2^32 - 1 work-items)";

template <int KIND, typename T>
hipError_t launch_phase(const swept_plan_s* p, const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  switch (resolved_engine(p)) {
    case SWEPT_ENGINE_WAVE:
      return swept::launch_phase_wave<KIND, T>(a, k, st);
    case SWEPT_ENGINE_COMPACT:
      return swept::launch_phase_compact<KIND, T>(a, k, st);
    default:
      return swept::launch_phase_lds<KIND, T>(a, k, st);
  }
}

template <typename T>
hipError_t dispatch_phase(const swept_plan_s* p, const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  if (p->general)
    return p->kind == SWEPT_KS_RK2 ? swept::launch_phase_general<swept::kKS, T>(a, k, st)
                                   : swept::launch_phase_general<swept::kHeat, T>(a, k, st);
  if (p->kind == SWEPT_HEAT_INSULATED) return swept::launch_phase_compact_insulated<T>(a, k, st);
  if (p->kind == SWEPT_HEAT_FTCS) return launch_phase<swept::kHeat, T>(p, a, k, st);
  return launch_phase<swept::kKS, T>(p, a, k, st);
}

template <typename T>
hipError_t run_naive(const swept_plan_s* p, T* u, int64_t steps, const Consts<T>& k, hipStream_t st) {
  T* buf = static_cast<T*>(p->buf);
  hipError_t e = hipSuccess;
  if (p->kind != SWEPT_KS_RK2) {
    T* cur = u;
    T* nxt = buf;
    for (int64_t m = 0; m < steps; ++m) {
      e = p->kind == SWEPT_HEAT_INSULATED ? swept::launch_naive_heat_insulated<T>(cur, nxt, p->n, k, st)
                                          : swept::launch_naive_heat<T>(cur, nxt, p->n, k, st);
      if (e != hipSuccess) return e;
      T* t = cur;
      cur = nxt;
      nxt = t;
    }
    if (cur != u) e = hipMemcpyAsync(u, cur, (size_t)p->n * sizeof(T), hipMemcpyDeviceToDevice, st);
    return e;
  }
  for (int64_t m = 0; m < steps; ++m) {
    e = swept::launch_naive_ks_predictor<T>(u, buf, p->n, k, st);
    if (e != hipSuccess) return e;
    e = swept::launch_naive_ks_final<T>(u, buf, p->n, k, st);
    if (e != hipSuccess) return e;
  }
  return e;
}

int choose_tile(int kind, int64_t n) {
  // Largest power of two up to 1024 that divides n (the automatic tuner of
  // the benchmark refines this per workload).
  const char* why = "";
  for (int w = 1024; w >= kMinTile; w >>= 1) {
    if (n % w == 0 && n >= w && tile_ok(kind, w, &why) &&
        (kind != SWEPT_HEAT_INSULATED || engine_supports(SWEPT_ENGINE_COMPACT, kind, w)))
      return w;
  }
  return 0;
}

// Validate a plan request and fill in its geometry, constants, engine and
// workspace size, allocating nothing (the device is only queried).  With
// use_tuned, tile_width = 0 and steps_per_cycle = 0 take the autotuner's
// remembered configuration when there is one.
int plan_setup(swept_plan_s* p, int64_t n, int kind, int dtype, double dt, double dx, double alpha, int tile_width,
               int steps_per_cycle, bool use_tuned, size_t max_slot_bytes) {
  if (!valid_kind(kind)) return fail(SWEPT_EINVAL, "unknown stencil kind");
  if (dtype != SWEPT_F32 && dtype != SWEPT_F64) return fail(SWEPT_EINVAL, "unknown dtype");
  if (n < kMinTile) return fail(SWEPT_EINVAL, "n must be >= 4");
  if (!is_finite(dt) || !is_finite(dx) || dx == 0.0) return fail(SWEPT_EINVAL, "dt and dx must be finite, dx != 0");
  if (kind != SWEPT_KS_RK2 && !is_finite(alpha)) return fail(SWEPT_EINVAL, "alpha must be finite");
  if (tile_width < 0) return fail(SWEPT_EINVAL, "tile_width must be >= 0");
  int w = tile_width;
  const char* why = "";
  int tuned_engine = SWEPT_ENGINE_AUTO;
  // The uneven tiling (tile widths 512 and 1024, any n >= 32 of a periodic
  // kind) takes the grids that the width does not divide.
  auto uneven_ok = [&](int width) {
    return kind != SWEPT_HEAT_INSULATED && n >= kMinGeneral && swept::general_engine_supports(width) &&
           n % width != 0;
  };
  auto full_of = [&](int width) {
    return uneven_ok(width) ? swept::general_full_tiers(stencil_of(kind), n, width) : full_tiers(kind, width);
  };
  if (w == 0) {
    // tuned configuration for this (kind, dtype, n) if the autotuner has one
    swept::TuneEntry te;
    if (use_tuned && steps_per_cycle == 0 && swept::tune_lookup(kind, dtype, n, &te) &&
        tile_ok(kind, te.tile_width, &why) && (n % te.tile_width == 0 || uneven_ok(te.tile_width)) &&
        te.steps_per_cycle >= 0 && te.steps_per_cycle * tiers_per_step(kind) <= full_of(te.tile_width) &&
        engine_supports(te.engine, kind, te.tile_width) &&
        (n % te.tile_width == 0 || te.engine == SWEPT_ENGINE_COMPACT || te.engine == SWEPT_ENGINE_AUTO)) {
      w = te.tile_width;
      steps_per_cycle = te.steps_per_cycle;
      tuned_engine = te.engine;
    } else {
      w = choose_tile(kind, n);
      // widths below 256 leave most of each tile's work in its edges: the
      // uneven tiling at 1024 is used instead when it applies
      if (w < 256 && uneven_ok(1024)) w = 1024;
    }
    if (w == 0) return fail(SWEPT_EUNSUPPORTED, "no supported tile width divides n");
  } else if (!tile_ok(kind, w, &why)) {
    return fail(SWEPT_EINVAL, why);
  }
  const bool general = n % w != 0 || n < w;
  if (general && !uneven_ok(w))
    return fail(SWEPT_EUNSUPPORTED,
                "n must be a positive multiple of tile_width, or tile_width 512 or 1024 with n >= 32 (uneven tiles; "
                "not for the insulated rod)");
  if (kind == SWEPT_HEAT_INSULATED && !engine_supports(SWEPT_ENGINE_COMPACT, kind, w))
    return fail(SWEPT_EUNSUPPORTED, "the insulated rod runs on the compacted engine: tile_width 512 or 1024");
  const int hfull = full_of(w);
  const int tps = tiers_per_step(kind);
  if (hfull < tps) return fail(SWEPT_EUNSUPPORTED, "n too small for one timestep per phase");
  if (steps_per_cycle < 0 || steps_per_cycle * tps > hfull)
    return fail(SWEPT_EINVAL, "steps_per_cycle exceeds the triangle height of this tile width");

  *p = swept_plan_s();
  p->n = n;
  p->kind = kind;
  p->dtype = dtype;
  p->s = radius_of(kind);
  p->w = w;
  p->h = steps_per_cycle ? steps_per_cycle * tps : hfull;
  p->general = general;
  p->nt = general ? swept::general_tiles(stencil_of(kind), n, w) : n / w;
  // Discretisation constants in double, rounded once for float (Sec. 4.1, Sec. 5).
  p->kd = swept::make_consts<double>(dt, dx, alpha);
  p->kf = swept::make_consts<float>(dt, dx, alpha);

  p->slots_bytes = (size_t)(2 * p->nt) * (size_t)swept::slot_values(w, p->s) * elem_size(dtype);
  if (max_slot_bytes && p->slots_bytes > max_slot_bytes)
    return fail(SWEPT_EUNSUPPORTED, "the edge slots of this grid need " + std::to_string(p->slots_bytes) +
                                        " bytes; the static workspace holds " + std::to_string(max_slot_bytes));

  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  int max_lds = 0;
  e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  size_t lds = 0;
  if (kind != SWEPT_KS_RK2)
    lds = dtype == SWEPT_F64 ? swept::phase_lds_bytes<swept::kHeat, double>(w)
                             : swept::phase_lds_bytes<swept::kHeat, float>(w);
  else
    lds = dtype == SWEPT_F64 ? swept::phase_lds_bytes<swept::kKS, double>(w)
                             : swept::phase_lds_bytes<swept::kKS, float>(w);
  if (!general && lds > (size_t)max_lds && !swept::wave_engine_supports(stencil_of(kind), w))
    return fail(SWEPT_EUNSUPPORTED, "tile too wide for the LDS of this device");
  p->engine = general ? SWEPT_ENGINE_COMPACT : tuned_engine;
  p->lds_fits = !general && lds <= (size_t)max_lds;
  // a tuned LDS choice that this device's LDS cannot hold falls back to AUTO
  // (a register engine: the width check above guarantees one exists)
  if (!p->lds_fits && p->engine == SWEPT_ENGINE_LDS) p->engine = SWEPT_ENGINE_AUTO;
  if (!launch_fits(p->engine, kind, w, p->nt)) return fail(SWEPT_EUNSUPPORTED, kTooManyTiles);
  return SWEPT_OK;
}

// Enqueue the launches of one swept run of p on st with `slots` as the edge
// slots: an up-triangle phase, the diamond phases and a down-triangle phase;
// full phases of p->h tiers, the remainder last.  Nothing is allocated.
int enqueue_swept(const swept_plan_s* p, void* slots, void* u, int64_t steps, hipStream_t st, bool poison) {
  const int64_t tiers = steps * tiers_per_step(p->kind);
  const int64_t full = tiers / p->h;
  const int rem = (int)(tiers % p->h);
  const int64_t nedge = full + (rem ? 1 : 0);  // edge sets; phases = nedge + 1
  for (int64_t i = 0; i <= nedge; ++i) {
    PhaseArgs a;
    a.u = u;
    a.slots = slots;
    a.n = p->n;
    a.w = p->w;
    a.nt = p->nt;
    a.parity = (int)(i & 1);
    a.hv = i == 0 ? 0 : (i - 1 < full ? p->h : rem);
    a.hl = i == nedge ? 0 : (i < full ? p->h : rem);
    a.poison = poison ? 1 : 0;
    hipError_t err = p->dtype == SWEPT_F64 ? dispatch_phase<double>(p, a, p->kd, st)
                                           : dispatch_phase<float>(p, a, p->kf, st);
    if (err != hipSuccess) return hip_fail(err, "swept phase launch");
  }
  return SWEPT_OK;
}

// With the non-finite check on, scan u after the run, wait for the stream and
// report SWEPT_ENONFINITE if any value is not finite.
int finish_run(const swept_plan_s* p, const void* u, hipStream_t st) {
  if (!(p->checks & SWEPT_CHECK_NONFINITE)) return SWEPT_OK;
  hipError_t e = swept::enqueue_nonfinite_check(u, p->n, (int)elem_size(p->dtype), p->flag, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpy(&bad, p->flag, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "non-finite check");
  return bad ? fail(SWEPT_ENONFINITE, "the grid holds a non-finite value after the run") : SWEPT_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current: looked up
// on the first call for that device, then remembered.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SWEPT_EUNSUPPORTED, "device index beyond the static workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SWEPT_OK;
}

}  // namespace

extern "C" {

const char* swept_last_error(void) { return g_last_error.c_str(); }

int swept_schedule(int kind, int tile_width, int steps_per_cycle, int64_t steps, int32_t* heights,
                   int64_t cap, int64_t* count) {
  if (!valid_kind(kind)) return fail(SWEPT_EINVAL, "unknown stencil kind");
  const char* why = "";
  if (!tile_ok(kind, tile_width, &why)) return fail(SWEPT_EINVAL, why);
  const int hfull = full_tiers(kind, tile_width);
  const int tps = tiers_per_step(kind);
  if (steps_per_cycle < 0 || steps_per_cycle * tps > hfull)
    return fail(SWEPT_EINVAL, "steps_per_cycle exceeds the triangle height of this tile width");
  if (steps < 0) return fail(SWEPT_EINVAL, "steps must be >= 0");
  if (!count) return fail(SWEPT_EINVAL, "count must not be NULL");
  if (cap < 0 || (cap > 0 && !heights)) return fail(SWEPT_EINVAL, "heights must hold cap entries");
  const int h = steps_per_cycle ? steps_per_cycle * tps : hfull;
  std::vector<int32_t> e;
  make_schedule(h, steps * tps, &e);
  for (int64_t i = 0; i < cap && i < (int64_t)e.size(); ++i) heights[i] = e[(size_t)i];
  *count = (int64_t)e.size();
  return SWEPT_OK;
}

int swept_tile_geometry(int kind, int tile_width, int* full_tiers_out, int* row_values,
                        int* edge_slot_values) {
  if (!valid_kind(kind)) return fail(SWEPT_EINVAL, "unknown stencil kind");
  const char* why = "";
  if (!tile_ok(kind, tile_width, &why)) return fail(SWEPT_EINVAL, why);
  const int s = radius_of(kind);
  if (full_tiers_out) *full_tiers_out = full_tiers(kind, tile_width);
  if (row_values) *row_values = tile_width + 2 * s;
  if (edge_slot_values) *edge_slot_values = swept::slot_values(tile_width, s);
  return SWEPT_OK;
}

int swept_plan_create(swept_plan* out, int64_t n, int kind, int dtype, double dt, double dx, double alpha,
                      int tile_width, int steps_per_cycle) {
  if (!out) return fail(SWEPT_EINVAL, "out must not be NULL");
  *out = nullptr;
  swept_plan_s cfg;
  int rc = plan_setup(&cfg, n, kind, dtype, dt, dx, alpha, tile_width, steps_per_cycle, true, 0);
  if (rc != SWEPT_OK) return rc;
  auto* p = new (std::nothrow) swept_plan_s(cfg);
  if (!p) return fail(SWEPT_ENOMEM, "host allocation failed");
  p->poison = swept::debug_poison_requested();
  p->buf_bytes = (size_t)n * elem_size(dtype);
  hipError_t e = hipMalloc(&p->slots, p->slots_bytes);
  if (e != hipSuccess) {
    delete p;
    return fail(SWEPT_ENOMEM, std::string("hipMalloc(edge slots): ") + hipGetErrorString(e));
  }
  e = hipMalloc(&p->buf, p->buf_bytes);
  if (e != hipSuccess) {
    (void)hipFree(p->slots);
    delete p;
    return fail(SWEPT_ENOMEM, std::string("hipMalloc(naive buffer): ") + hipGetErrorString(e));
  }
  *out = p;
  return SWEPT_OK;
}

int swept_plan_set_engine(swept_plan p, int engine) {
  if (!p) return fail(SWEPT_EINVAL, "plan must not be NULL");
  if (engine != SWEPT_ENGINE_AUTO && engine != SWEPT_ENGINE_LDS && engine != SWEPT_ENGINE_WAVE &&
      engine != SWEPT_ENGINE_COMPACT)
    return fail(SWEPT_EINVAL, "unknown engine");
  if (p->general && engine != SWEPT_ENGINE_AUTO && engine != SWEPT_ENGINE_COMPACT)
    return fail(SWEPT_EUNSUPPORTED, "tiles of uneven width (tile_width does not divide n) run on the compacted engine");
  if (!engine_supports(engine, p->kind, p->w))
    return fail(SWEPT_EUNSUPPORTED, engine == SWEPT_ENGINE_WAVE      ? "no wave-resident kernel for this kind and tile width"
                                    : engine == SWEPT_ENGINE_COMPACT ? "no compacted kernel for this kind and tile width"
                                                                     : "no kernel of this engine for this kind");
  if (engine == SWEPT_ENGINE_LDS && !p->lds_fits)
    return fail(SWEPT_EUNSUPPORTED, "tile too wide for the LDS of this device");
  if (!launch_fits(engine, p->kind, p->w, p->nt)) return fail(SWEPT_EUNSUPPORTED, kTooManyTiles);
  p->engine = engine;
  return SWEPT_OK;
}

int swept_plan_info(swept_plan p, int* tile_width, int* steps_per_cycle, size_t* workspace_bytes) {
  if (!p) return fail(SWEPT_EINVAL, "plan must not be NULL");
  if (tile_width) *tile_width = p->w;
  if (steps_per_cycle) *steps_per_cycle = p->h / tiers_per_step(p->kind);
  if (workspace_bytes) *workspace_bytes = p->slots_bytes + p->buf_bytes;
  return SWEPT_OK;
}

void swept_plan_destroy(swept_plan p) {
  if (!p) return;
  swept::DeviceGuard g(p->device);
  if (p->slots) (void)hipFree(p->slots);
  if (p->buf) (void)hipFree(p->buf);
  if (p->flag) (void)hipFree(p->flag);
  delete p;
}

int swept_run(swept_plan p, void* u, int64_t steps, void* stream) {
  if (!p) return fail(SWEPT_EINVAL, "plan must not be NULL");
  if (steps < 0) return fail(SWEPT_EINVAL, "steps must be >= 0");
  if (steps == 0) return SWEPT_OK;
  if (!u) return fail(SWEPT_EINVAL, "u must not be NULL");
  swept::DeviceGuard g(p->device);
  if (!g.ok) return hip_fail(g.err, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->poison) {
    const hipError_t pe = swept::poison_fill(p->slots, p->slots_bytes, (int)elem_size(p->dtype), st);
    if (pe != hipSuccess) return hip_fail(pe, "workspace poison fill");
  }
  const int rc = enqueue_swept(p, p->slots, u, steps, st, p->poison);
  return rc != SWEPT_OK ? rc : finish_run(p, u, st);
}

int swept_run_noalloc(int64_t n, int kind, int dtype, double dt, double dx, double alpha, int tile_width,
                      int steps_per_cycle, void* u, int64_t steps, void* stream) {
  if (steps < 0) return fail(SWEPT_EINVAL, "steps must be >= 0");
  if (steps > 0 && !u) return fail(SWEPT_EINVAL, "u must not be NULL");
  swept_plan_s p;
  int rc = plan_setup(&p, n, kind, dtype, dt, dx, alpha, tile_width, steps_per_cycle, false, kScratchBytes);
  if (rc != SWEPT_OK) return rc;
  if (steps == 0) return SWEPT_OK;
  void* slots = nullptr;
  rc = scratch_address(p.device, &slots);
  if (rc != SWEPT_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool poison = swept::debug_poison_requested();
  if (poison) {
    const hipError_t pe = swept::poison_fill(slots, p.slots_bytes, (int)elem_size(p.dtype), st);
    if (pe != hipSuccess) return hip_fail(pe, "workspace poison fill");
  }
  return enqueue_swept(&p, slots, u, steps, st, poison);
}

int naive_run(swept_plan p, void* u, int64_t steps, void* stream) {
  if (!p) return fail(SWEPT_EINVAL, "plan must not be NULL");
  if (steps < 0) return fail(SWEPT_EINVAL, "steps must be >= 0");
  if (steps == 0) return SWEPT_OK;
  if (!u) return fail(SWEPT_EINVAL, "u must not be NULL");
  swept::DeviceGuard g(p->device);
  if (!g.ok) return hip_fail(g.err, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t err = p->dtype == SWEPT_F64 ? run_naive<double>(p, static_cast<double*>(u), steps, p->kd, st)
                                         : run_naive<float>(p, static_cast<float*>(u), steps, p->kf, st);
  if (err != hipSuccess) return hip_fail(err, "naive launch");
  return finish_run(p, u, st);
}

int swept_plan_set_checks(swept_plan p, int flags) {
  if (!p) return fail(SWEPT_EINVAL, "plan must not be NULL");
  if (flags & ~SWEPT_CHECK_NONFINITE) return fail(SWEPT_EINVAL, "unknown check flags");
  if ((flags & SWEPT_CHECK_NONFINITE) && !p->flag) {
    swept::DeviceGuard g(p->device);
    if (!g.ok) return hip_fail(g.err, "hipSetDevice");
    const hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->flag), sizeof(int));
    if (e != hipSuccess) {
      p->flag = nullptr;
      return fail(SWEPT_ENOMEM, std::string("hipMalloc(check flag): ") + hipGetErrorString(e));
    }
  }
  p->checks = flags;
  return SWEPT_OK;
}

int swept_autotune_lookup(int64_t n, int kind, int dtype, int* tile_width, int* steps_per_cycle, int* engine,
                          double* ns_per_cell_update) {
  if (!valid_kind(kind)) return fail(SWEPT_EINVAL, "unknown stencil kind");
  if (dtype != SWEPT_F32 && dtype != SWEPT_F64) return fail(SWEPT_EINVAL, "unknown dtype");
  swept::TuneEntry te;
  if (!swept::tune_lookup(kind, dtype, n, &te)) return fail(SWEPT_EUNSUPPORTED, "no tuned entry for this problem");
  if (tile_width) *tile_width = te.tile_width;
  if (steps_per_cycle) *steps_per_cycle = te.steps_per_cycle;
  if (engine) *engine = te.engine;
  if (ns_per_cell_update) *ns_per_cell_update = te.ns_per_cell_update;
  return SWEPT_OK;
}

void swept_autotune_forget(void) { swept::tune_forget_all(); }

int swept_autotune(int64_t n, int kind, int dtype, double dt, double dx, double alpha, int64_t steps,
                   swept_tune_result* results, int cap, int* count, int* tile_width, int* steps_per_cycle,
                   int* engine) {
  if (!valid_kind(kind)) return fail(SWEPT_EINVAL, "unknown stencil kind");
  if (dtype != SWEPT_F32 && dtype != SWEPT_F64) return fail(SWEPT_EINVAL, "unknown dtype");
  if (n < kMinTile) return fail(SWEPT_EINVAL, "n must be >= 4");
  if (steps < 0) return fail(SWEPT_EINVAL, "steps must be >= 0");
  if (cap < 0 || (cap > 0 && !results)) return fail(SWEPT_EINVAL, "results must hold cap entries");
  const int tps = tiers_per_step(kind);
  // timed horizon: several full phases of the widest tile
  int64_t T = steps > 0 ? steps : (kind == SWEPT_KS_RK2 ? 512 : 2048);
  if (T > (kind == SWEPT_KS_RK2 ? 1024 : 4096)) T = kind == SWEPT_KS_RK2 ? 1024 : 4096;
  struct Cand {
    int w, spc, engine;
  };
  std::vector<Cand> cands;
  const char* why = "";
  for (int w = 64; w <= 2048; w <<= 1) {
    if (!tile_ok(kind, w, &why)) continue;
    // widths that divide n, and the uneven tiling at 512 and 1024 otherwise
    const bool even = n % w == 0 && n >= w;
    const bool uneven = !even && kind != SWEPT_HEAT_INSULATED && n >= kMinGeneral && swept::general_engine_supports(w);
    if (!even && !uneven) continue;
    const int full_steps =
        (uneven ? swept::general_full_tiers(stencil_of(kind), n, w) : full_tiers(kind, w)) / tps;
    // phase heights: the full triangle, 3/4, 1/2 and 1/4 of it
    const int spcs[4] = {full_steps, full_steps * 3 / 4, full_steps / 2, full_steps / 4};
    for (int eng : {SWEPT_ENGINE_COMPACT, SWEPT_ENGINE_WAVE, SWEPT_ENGINE_LDS}) {
      if (!engine_supports(eng, kind, w) || (uneven && eng != SWEPT_ENGINE_COMPACT)) continue;
      for (int si = 0; si < 4; ++si) {
        bool dup = spcs[si] < 1;
        for (int sj = 0; sj < si; ++sj) dup = dup || spcs[sj] == spcs[si];
        if (!dup) cands.push_back({w, spcs[si], eng});
      }
    }
  }
  if (cands.empty()) return fail(SWEPT_EUNSUPPORTED, "no tile width fits n");

  const size_t es = elem_size(dtype);
  void* u = nullptr;
  hipError_t e = hipMalloc(&u, (size_t)n * es);
  if (e != hipSuccess) return fail(SWEPT_ENOMEM, std::string("hipMalloc(autotune grid): ") + hipGetErrorString(e));
  e = hipMemset(u, 0, (size_t)n * es);
  hipStream_t st = nullptr;
  if (e == hipSuccess) e = hipStreamCreate(&st);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(u);
    return hip_fail(e, "autotune setup");
  }
  int best = -1;
  double best_ns = 0.0;
  int nres = 0;
  int rc = SWEPT_OK;
  for (size_t ci = 0; ci < cands.size(); ++ci) {
    const Cand& c = cands[ci];
    swept_plan p = nullptr;
    int r = swept_plan_create(&p, n, kind, dtype, dt, dx, alpha, c.w, c.spc);
    if (r != SWEPT_OK) continue;  // e.g. LDS too small on this device
    if (swept_plan_set_engine(p, c.engine) != SWEPT_OK) {
      swept_plan_destroy(p);
      continue;
    }
    float ms = 0.0f, best_ms = 0.0f;
    r = swept_run(p, u, T, st);  // warm-up (code object load, caches)
    for (int rep = 0; rep < 3 && r == SWEPT_OK; ++rep) {
      e = hipEventRecord(t0, st);
      if (e == hipSuccess) r = swept_run(p, u, T, st);
      if (r == SWEPT_OK && e == hipSuccess) e = hipEventRecord(t1, st);
      if (r == SWEPT_OK && e == hipSuccess) e = hipEventSynchronize(t1);
      if (r == SWEPT_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e != hipSuccess) r = hip_fail(e, "autotune timing");
      if (r == SWEPT_OK && (rep == 0 || ms < best_ms)) best_ms = ms;
    }
    swept_plan_destroy(p);
    if (r != SWEPT_OK) {
      rc = r;
      break;
    }
    const double ns = 1e6 * (double)best_ms / ((double)n * (double)T);
    if (nres < cap) {
      results[nres].tile_width = c.w;
      results[nres].steps_per_cycle = c.spc;
      results[nres].engine = c.engine;
      results[nres].reserved = 0;
      results[nres].ns_per_cell_update = ns;
    }
    ++nres;
    if (best < 0 || ns < best_ns) {
      best = (int)ci;
      best_ns = ns;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  (void)hipStreamDestroy(st);
  (void)hipFree(u);
  if (rc != SWEPT_OK) return rc;
  if (best < 0) return fail(SWEPT_EUNSUPPORTED, "no candidate configuration could run");
  if (count) *count = nres;
  swept::TuneEntry te;
  te.tile_width = cands[(size_t)best].w;
  te.steps_per_cycle = cands[(size_t)best].spc;
  te.engine = cands[(size_t)best].engine;
  te.ns_per_cell_update = best_ns;
  if (!swept::tune_store(kind, dtype, n, te)) return fail(SWEPT_EDEVICE, "could not write the autotune cache file");
  if (tile_width) *tile_width = te.tile_width;
  if (steps_per_cycle) *steps_per_cycle = te.steps_per_cycle;
  if (engine) *engine = te.engine;
  return SWEPT_OK;
}

}  // extern "C"
