// cme_wave_f32.hip -- FP32 variants of the two-level wave kernels
// (cme_wave.hpp): FP32 transforms and RK4 state, FP64 time and detuning
// bookkeeping (sigma(t) and omega' - sigma are formed in FP64, then rounded).
#include "cme_wave.hpp"

namespace cme {

static const Variant kWaveVariantsF32[] = {
    wave_variant<float, 128, 2, 1, 1>(),    wave_variant<float, 256, 4, 1, 2>(),
    wave_variant<float, 512, 8, 1, 3>(),    wave_variant<float, 512, 8, 1, 4>(),
    wave_variant<float, 1024, 8, 1, 3>(),   wave_variant<float, 1024, 8, 1, 4>(),
    wave_variant<float, 2048, 8, 1, 3>(),   wave_variant<float, 2048, 8, 1, 4>(),
    wave_variant<float, 4096, 8, 1, 3>(),   wave_variant<float, 4096, 8, 1, 4>(),
    wave_variant<float, 8192, 16, 2, 3>(),
};

const Variant *variants_wave_f32(int *count) {
  *count = (int)(sizeof(kWaveVariantsF32) / sizeof(kWaveVariantsF32[0]));
  return kWaveVariantsF32;
}

}  // namespace cme
