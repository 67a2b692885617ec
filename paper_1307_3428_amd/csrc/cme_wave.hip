// cme_wave.hip -- FP64 variants of the two-level wave kernels (cme_wave.hpp).
#include "cme_wave.hpp"

namespace cme {

// (N, E, V, PS, TP): N modes, E per thread, V sub-transforms per wave, one
// LDS padding element every 2^PS, sub-transform kind TP (0 Stockham through
// LDS; 1 radix-8 passes with the high lane bits exchanged in registers and
// the low ones through LDS).
static const Variant kWaveVariants[] = {
    wave_variant<double, 128, 2, 1, 1>(),     wave_variant<double, 256, 4, 1, 2>(),
    wave_variant<double, 256, 2, 1, 1>(),     wave_variant<double, 512, 8, 1, 3>(),
    wave_variant<double, 512, 4, 1, 2>(),     wave_variant<double, 1024, 8, 1, 3>(),
    wave_variant<double, 1024, 4, 1, 2>(),    wave_variant<double, 2048, 8, 1, 3>(),
    wave_variant<double, 2048, 8, 1, 3, 1>(), wave_variant<double, 4096, 8, 1, 3>(),
    wave_variant<double, 8192, 16, 2, 3>(),   wave_variant<double, 8192, 16, 2, 3, 1>(),
};

// Alias-free truncated sum (CME_FWM_PADDED): instances of N/2 = 128 ... 4096
// modes on N-point transforms.
static const Variant kPadVariants[] = {
    pad_variant<double, 256, 4, 1, 2>(),  pad_variant<double, 512, 8, 1, 3>(),
    pad_variant<double, 1024, 8, 1, 3>(), pad_variant<double, 2048, 8, 1, 3>(),
    pad_variant<double, 4096, 8, 1, 3>(), pad_variant<double, 8192, 16, 2, 3>(),
};

const Variant *variants_pad(int *count) {
  *count = (int)(sizeof(kPadVariants) / sizeof(kPadVariants[0]));
  return kPadVariants;
}

const Variant *variants_wave(int *count) {
  *count = (int)(sizeof(kWaveVariants) / sizeof(kWaveVariants[0]));
  return kWaveVariants;
}

}  // namespace cme
