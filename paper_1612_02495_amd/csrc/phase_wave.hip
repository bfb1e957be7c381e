// Wave-resident engine for one periodic grid: one wave64 per tile, the tile
// held in registers, no LDS or barrier in the tier loop.  The per-tile
// algorithm (register layout, DPP halos, lane-masked edge bands, slot layout)
// is in wave_tile.h; here every tile is 64 P points with its seam in the
// middle, tiles start at j*w (even phases) or j*w + w/2 (odd phases), and the
// edge-slot ownership is that of the LDS engine (phase_lds.hip), so the two
// engines can run alternate phases of one run.
#include "wave_tile.h"

namespace swept {
namespace {

// ROLE: 0 up-triangle (hv == 0), 1 diamond, 2 down-triangle (hl == 0).  One
// wave per tile; every tile of the grid has 32 lanes on each side of its seam.
template <int KIND, typename T, int P, int ROLE>
__global__ void __launch_bounds__(64)
phase_wave_kernel(T* u, T* slots, int64_t n, int64_t nt, int parity, int hv, int hl, Consts<T> k) {
  constexpr int S = Radius<KIND>::value;
  constexpr int W = 64 * P;
  constexpr int HALF = 32 * P;
  constexpr int SLEN = W + 2 * S;
  const int64_t j = blockIdx.x;
  wave::Tile<T> g;
  g.origin = j * (int64_t)W + (parity ? HALF : 0);
  g.sL = parity ? slots + (nt + j) * SLEN : slots + j * SLEN;
  g.sR = parity ? slots + ((j + 1) % nt) * SLEN : slots + (nt + j) * SLEN;
  g.kL = 32;
  g.kR = 32;
  wave::tile_phase<KIND, T, P, ROLE>(u, n, g, hv, hl, k, (int)threadIdx.x);
}

template <int KIND, typename T, int P>
hipError_t launch_p(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  auto kern = a.hv == 0 ? phase_wave_kernel<KIND, T, P, 0>
              : (a.hl == 0 ? phase_wave_kernel<KIND, T, P, 2> : phase_wave_kernel<KIND, T, P, 1>);
  hipLaunchKernelGGL(kern, dim3((unsigned)a.nt), dim3(64), 0, st, static_cast<T*>(a.u), static_cast<T*>(a.slots),
                     a.n, a.nt, a.parity, a.hv, a.hl, k);
  return hipGetLastError();
}

}  // namespace

bool wave_engine_supports(int kind, int w) {
  if (w % 64 != 0) return false;
  const int p = w / 64;
  if (kind == kHeat) return p == 2 || p == 4 || p == 8 || p == 16;
  return p == 4 || p == 8 || p == 16;
}

template <int KIND, typename T>
hipError_t launch_phase_wave(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  if (!wave_engine_supports(KIND, a.w)) return hipErrorInvalidValue;
  switch (a.w / 64) {
    case 2:
      if constexpr (KIND == kHeat) return launch_p<KIND, T, 2>(a, k, st);
      break;
    case 4:
      return launch_p<KIND, T, 4>(a, k, st);
    case 8:
      return launch_p<KIND, T, 8>(a, k, st);
    case 16:
      return launch_p<KIND, T, 16>(a, k, st);
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_phase_wave<kHeat, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_wave<kHeat, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);
template hipError_t launch_phase_wave<kKS, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_wave<kKS, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);

}  // namespace swept
