// Wave-resident engine (placeholder until the register kernel lands).
#include "internal.h"

namespace swept {

bool wave_engine_supports(int, int) { return false; }

template <int KIND, typename T>
hipError_t launch_phase_wave(const PhaseArgs&, const Consts<T>&, hipStream_t) {
  return hipErrorInvalidValue;
}

template hipError_t launch_phase_wave<kHeat, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_wave<kHeat, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);
template hipError_t launch_phase_wave<kKS, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_wave<kKS, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);

}  // namespace swept
