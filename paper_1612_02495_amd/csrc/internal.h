// Internal (non-ABI) declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "stencil.h"

namespace swept {

struct TuneEntry {
  int tile_width = 0;
  int steps_per_cycle = 0;
  int engine = 0;
  double ns_per_cell_update = 0.0;
};

// One swept phase over the whole ring (Sec. 4.2): every tile first fills the
// V between the incoming edge bands (hv tiers; hv == 0 means "read the full
// row from u"), then climbs the triangle/trapezoid Lambda (hl tiers; hl == 0
// means "write the full row to u").  Tiles of phase p start at
// parity * w/2 + j*w; the edge bands live in 2*nt slots of (w + 2s) values.
struct PhaseArgs {
  void* u;       // device grid, n values
  void* slots;   // device edge slots: slot A[j] at j, slot B[j] at nt + j
  int64_t n;
  int w;         // tile width (the widest tile of an uneven tiling)
  int64_t nt;    // tiles: n / w, or those of the uneven tiling
  int parity;    // 0: tiles start at j*w; 1: at j*w + w/2
  int hv;        // V height in tiers (0 = load full row)
  int hl;        // Lambda height in tiers (0 = store full row)
  int poison = 0;  // fill the tile's LDS with NaN first (SWEPT_DEBUG_POISON)
};

// Values per edge slot: (w/2 + s) positions, two tier parities each.
__host__ __device__ inline int slot_values(int w, int s) { return w + 2 * s; }

template <typename T>
hipError_t launch_naive_heat(const T* in, T* out, int64_t n, const Consts<T>& k, hipStream_t st);
template <typename T>
hipError_t launch_naive_ks_predictor(const T* u, T* q, int64_t n, const Consts<T>& k, hipStream_t st);
template <typename T>
hipError_t launch_naive_ks_final(T* u, const T* q, int64_t n, const Consts<T>& k, hipStream_t st);

template <int KIND, typename T>
hipError_t launch_phase_lds(const PhaseArgs& a, const Consts<T>& k, hipStream_t st);
template <int KIND, typename T>
size_t phase_lds_bytes(int w);
// Work-items per tile of the LDS engine (the register engines use one wave64).
int phase_lds_threads(int w);

template <int KIND, typename T>
hipError_t launch_phase_wave(const PhaseArgs& a, const Consts<T>& k, hipStream_t st);
// Whether the wave-resident engine has a kernel for this kind and width.
bool wave_engine_supports(int kind, int w);

template <int KIND, typename T>
hipError_t launch_phase_compact(const PhaseArgs& a, const Consts<T>& k, hipStream_t st);
// Whether the compacted wave engine has a kernel for this kind and width.
bool compact_engine_supports(int kind, int w);
// Uneven tiling of a single grid whose size the tile width w (512 or 1024)
// does not divide: tiles of two halves of at most w / 2 points each, on the
// compacted engine (phase_general.hip).
template <int KIND, typename T>
hipError_t launch_phase_general(const PhaseArgs& a, const Consts<T>& k, hipStream_t st);
bool general_engine_supports(int w);
int64_t general_tiles(int kind, int64_t n, int w);
// Tiers of a full phase of the uneven tiling: the smallest half's triangle.
int general_full_tiers(int kind, int64_t n, int w);
// Heat on a rod with insulated ends (compacted engine; widths as for heat).
template <typename T>
hipError_t launch_phase_compact_insulated(const PhaseArgs& a, const Consts<T>& k, hipStream_t st);

// Naive heat step on a rod with insulated ends (mirror ghosts at nodes 0, n-1).
template <typename T>
hipError_t launch_naive_heat_insulated(const T* in, T* out, int64_t n, const Consts<T>& k, hipStream_t st);

// Record the calling thread's last error (swept_last_error) and return code.
int set_error(int code, const std::string& msg);

// Autotuner table (autotune.hip).
bool tune_lookup(int kind, int dtype, int64_t n, TuneEntry* out);
bool tune_store(int kind, int dtype, int64_t n, const TuneEntry& e);
void tune_forget_all();

}  // namespace swept
