// Spectra and plane kernels for detector sizes 216, 240, 250, 256 (planes as 2 row blocks).
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesI[] = {split_size<108, 2>(), split_size<120, 2>(), split_size<125, 2>(), split_rows_size<128, 2>()};
const int kFftSizesICount = int(sizeof(kFftSizesI) / sizeof(kFftSizesI[0]));
}  // namespace tomo
