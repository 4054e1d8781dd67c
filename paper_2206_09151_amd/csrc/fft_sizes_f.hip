// Spectra and plane kernels for detector sizes 144, 150, 160 (planes as 2 row blocks).
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesF[] = {direct_size<144>(), direct_size<150>(), rows_size<160>()};
const int kFftSizesFCount = int(sizeof(kFftSizesF) / sizeof(kFftSizesF[0]));
}  // namespace tomo
