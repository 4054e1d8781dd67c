// Spectra and plane kernels for detector sizes 162, 180 (as 2 x 2 blocks of 81, 90).
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesG[] = {split_size<81, 2>(), split_size<90, 2>()};
const int kFftSizesGCount = int(sizeof(kFftSizesG) / sizeof(kFftSizesG[0]));
}  // namespace tomo
