// Swept phases of one periodic grid whose size no tile width divides: the
// uneven tiling of the batched kernel (batch.hip) for a single grid, one
// wave64 per tile on the compacted engine (compact_tile.h, uneven-tile form).
//
// The ring of n points is split into 2 nt halves (compact::uneven_tiling: all
// but the last a multiple of 4 s points, every one at most 32 P points); even
// tile j is halves (2j, 2j+1), odd tile j is halves (2j+1, 2j+2 mod 2nt) --
// the zig-zag of Sec. 4.2 with tiles of uneven width.  Edge
// slot A[j] sits at the left seam of even tile j and B[j] at its centre, as
// for every other engine; the phase height is at most the pure-triangle
// height of the smallest half (Sec. 4.2; flattened tops on the wider halves,
// Sec. 4.3).
#include "compact_tile.h"
#include "poison.h"

namespace swept {
namespace {

// POISON: fill the tile's LDS with NaN first (a separate instantiation).
template <int KIND, typename T, int P, bool POISON>
__global__ void __launch_bounds__(64)
phase_general_kernel(T* u, T* slots, int64_t n, int64_t nt, int parity, int hv, int hl, Consts<T> k) {
  constexpr int S = Radius<KIND>::value;
  constexpr int SLEN = 64 * P + 2 * S;
  __shared__ T sb[compact::Lds<KIND, P>::band];
  __shared__ T stg[compact::Lds<KIND, P>::stage];
  if constexpr (POISON) {
    poison_lds(sb, compact::Lds<KIND, P>::band, (int)threadIdx.x, 64);
    poison_lds(stg, compact::Lds<KIND, P>::stage, (int)threadIdx.x, 64);
    compact::wave_sync();
  }
  const int64_t j = blockIdx.x;
  const compact::Uneven ut = compact::uneven_tiling(n, P, S);
  const int64_t iL = 2 * j + parity;
  const int64_t iR = (iL + 1) % (2 * nt);
  T* sL = parity ? slots + (nt + j) * SLEN : slots + j * SLEN;
  T* sR = parity ? slots + ((j + 1) % nt) * SLEN : slots + (nt + j) * SLEN;
  compact::tile_phase_g<KIND, T, P>(u, n, compact::uneven_origin(ut, iL), sL, sR, compact::uneven_width(ut, iL),
                                    compact::uneven_width(ut, iR), hv, hl, k, (int)threadIdx.x, sb, stg);
}

template <int KIND, typename T, int P>
hipError_t launch_p(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  auto kern = a.poison ? phase_general_kernel<KIND, T, P, true> : phase_general_kernel<KIND, T, P, false>;
  hipLaunchKernelGGL(kern, dim3((unsigned)a.nt), dim3(64), 0, st, static_cast<T*>(a.u), static_cast<T*>(a.slots),
                     a.n, a.nt, a.parity, a.hv, a.hl, k);
  return hipGetLastError();
}

}  // namespace

bool general_engine_supports(int w) { return w == 512 || w == 1024; }

int64_t general_tiles(int kind, int64_t n, int w) {
  return compact::uneven_tiling(n, w / 64, kind == kKS ? 2 : 1).nt;
}

int general_full_tiers(int kind, int64_t n, int w) {
  const int s = kind == kKS ? 2 : 1;
  return compact::uneven_full_tiers(compact::uneven_tiling(n, w / 64, s), s);
}

template <int KIND, typename T>
hipError_t launch_phase_general(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  switch (a.w) {
    case 512:
      return launch_p<KIND, T, 8>(a, k, st);
    case 1024:
      return launch_p<KIND, T, 16>(a, k, st);
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_phase_general<kHeat, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_general<kHeat, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);
template hipError_t launch_phase_general<kKS, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_general<kKS, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);

}  // namespace swept
