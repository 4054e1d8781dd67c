// Spectra and plane kernels for detector sizes 225, 243.
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesJ[] = {split_size<75, 3>(), split_size<81, 3>()};
const int kFftSizesJCount = int(sizeof(kFftSizesJ) / sizeof(kFftSizesJ[0]));
}  // namespace tomo
