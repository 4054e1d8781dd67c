// Spectra and plane kernels for detector sizes 192 (planes as 4 row blocks), 200 (as 2 x 2 blocks of 100).
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesH[] = {rows_size<192>(), split_size<100, 2>()};
const int kFftSizesHCount = int(sizeof(kFftSizesH) / sizeof(kFftSizesH[0]));
}  // namespace tomo
