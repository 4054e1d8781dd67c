// Spectra and plane kernels for detector sizes 125, 128, 135.
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesE[] = {direct_size<125>(), direct_size<128>(), direct_size<135>()};
const int kFftSizesECount = int(sizeof(kFftSizesE) / sizeof(kFftSizesE[0]));
}  // namespace tomo
