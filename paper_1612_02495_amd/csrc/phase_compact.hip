// Compacted wave engine for one periodic grid (or one insulated rod): one
// wave64 per tile as in the register engine (phase_wave.hip), with each run
// of tiers laid out over the part of the tile it touches (compact_tile.h).
// Tiles, slots and phase parities are those of the other engines, so all
// three can run alternate phases of one run.
#include "compact_tile.h"
#include "poison.h"

namespace swept {
namespace {

// Tile of workgroup b when each XCD is given a contiguous run of tiles.  The
// workgroups of one launch go to the 8 XCDs in turn (b mod 8), so this makes
// the two tiles whose slots a phase reads sit, but for the runs' ends, on the
// XCD that wrote them.  A bijection of [0, nt) for every nt.  Measured on the
// N=2^20, w=1024 diamonds: heat FP64 +2.3%, FP32 +0.6%, KS -2.2% (so KS keeps
// the plain order).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nt) {
  const int64_t q = nt / 8, r = nt % 8, x = b % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

// INS: heat on a rod with insulated ends.  The rod's nodes 0 and n-1 sit at
// the ring seam: at the middle of the last tile of the shifted tiling
// (parity 1), or at the first point of tile 0 and the last of tile nt-1
// (parity 0).  Only those tiles run the tier code with the mirror ghosts.
// POISON: fill the tile's LDS with NaN first (a separate instantiation, so
// that the production kernel carries no branch for it).
template <int KIND, typename T, int P, int ROLE, bool INS, bool POISON>
__global__ void __launch_bounds__(64)
phase_compact_kernel(T* u, T* slots, int64_t n, int64_t nt, int parity, int hv, int hl, Consts<T> k) {
  constexpr int S = Radius<KIND>::value;
  constexpr int W = 64 * P;
  constexpr int HALF = 32 * P;
  constexpr int SLEN = W + 2 * S;
  __shared__ T sb[compact::Lds<KIND, P>::band];
  __shared__ T stg[compact::Lds<KIND, P>::stage];
  if constexpr (POISON) {
    poison_lds(sb, compact::Lds<KIND, P>::band, (int)threadIdx.x, 64);
    poison_lds(stg, compact::Lds<KIND, P>::stage, (int)threadIdx.x, 64);
    compact::wave_sync();
  }
  const int64_t j = KIND == kHeat ? xcd_tile(blockIdx.x, nt) : (int64_t)blockIdx.x;
  const int64_t origin = j * (int64_t)W + (parity ? HALF : 0);
  T* sL = parity ? slots + (nt + j) * SLEN : slots + j * SLEN;
  T* sR = parity ? slots + ((j + 1) % nt) * SLEN : slots + (nt + j) * SLEN;
  if constexpr (INS) {
    compact::Bnd bd;
    bd.seam = parity && j == nt - 1;
    bd.lo = !parity && j == 0;
    bd.hi = !parity && j == nt - 1;
    if (bd.seam || bd.lo || bd.hi) {
      compact::tile_phase<KIND, T, P, ROLE, true>(u, n, origin, sL, sR, hv, hl, k, (int)threadIdx.x, sb, stg, bd);
      return;
    }
  }
  compact::tile_phase<KIND, T, P, ROLE>(u, n, origin, sL, sR, hv, hl, k, (int)threadIdx.x, sb, stg);
}

template <int KIND, typename T, int P, bool INS, bool POISON>
hipError_t launch_pp(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  auto kern = a.hv == 0 ? phase_compact_kernel<KIND, T, P, 0, INS, POISON>
              : (a.hl == 0 ? phase_compact_kernel<KIND, T, P, 2, INS, POISON>
                           : phase_compact_kernel<KIND, T, P, 1, INS, POISON>);
  hipLaunchKernelGGL(kern, dim3((unsigned)a.nt), dim3(64), 0, st, static_cast<T*>(a.u), static_cast<T*>(a.slots),
                     a.n, a.nt, a.parity, a.hv, a.hl, k);
  return hipGetLastError();
}

template <int KIND, typename T, int P, bool INS>
hipError_t launch_p(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  return a.poison ? launch_pp<KIND, T, P, INS, true>(a, k, st) : launch_pp<KIND, T, P, INS, false>(a, k, st);
}

}  // namespace

bool compact_engine_supports(int kind, int w) {
  if (w % 64 != 0) return false;
  const int p = w / 64;
  if (kind == kHeat) return p == 8 || p == 16;
  return p == 8 || p == 16;
}

template <int KIND, typename T>
hipError_t launch_phase_compact(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  if (!compact_engine_supports(KIND, a.w)) return hipErrorInvalidValue;
  switch (a.w / 64) {
    case 8:
      return launch_p<KIND, T, 8, false>(a, k, st);
    case 16:
      return launch_p<KIND, T, 16, false>(a, k, st);
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_phase_compact_insulated(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  if (!compact_engine_supports(kHeat, a.w)) return hipErrorInvalidValue;
  switch (a.w / 64) {
    case 8:
      return launch_p<kHeat, T, 8, true>(a, k, st);
    case 16:
      return launch_p<kHeat, T, 16, true>(a, k, st);
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_phase_compact<kHeat, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_compact<kHeat, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);
template hipError_t launch_phase_compact<kKS, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_compact<kKS, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);
template hipError_t launch_phase_compact_insulated<float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_compact_insulated<double>(const PhaseArgs&, const Consts<double>&, hipStream_t);

}  // namespace swept
