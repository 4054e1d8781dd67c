// Spectra and plane kernels for detector sizes 40, 45, 48, 50, 54, 60, 64.
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesB[] = {direct_size<40>(), direct_size<45>(), direct_size<48>(), direct_size<50>(), direct_size<54>(), direct_size<60>(), direct_size<64>()};
const int kFftSizesBCount = int(sizeof(kFftSizesB) / sizeof(kFftSizesB[0]));
}  // namespace tomo
