// Spectra and plane kernels for detector sizes 96, 100, 108, 120.
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesD[] = {direct_size<96>(), direct_size<100>(), direct_size<108>(), direct_size<120>()};
const int kFftSizesDCount = int(sizeof(kFftSizesD) / sizeof(kFftSizesD[0]));
}  // namespace tomo
