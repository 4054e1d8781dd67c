// Spectra and plane kernels for detector sizes 72, 75, 80, 81, 90.
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesC[] = {direct_size<72>(), direct_size<75>(), direct_size<80>(), direct_size<81>(), direct_size<90>()};
const int kFftSizesCCount = int(sizeof(kFftSizesC) / sizeof(kFftSizesC[0]));
}  // namespace tomo
