// Spectra and plane kernels for detector sizes 16, 18, 20, 24, 25, 27, 30, 32, 36.
#include "fft_sizes.hpp"

namespace tomo {
const FftSize kFftSizesA[] = {direct_size<16>(), direct_size<18>(), direct_size<20>(), direct_size<24>(), direct_size<25>(), direct_size<27>(), direct_size<30>(), direct_size<32>(), direct_size<36>()};
const int kFftSizesACount = int(sizeof(kFftSizesA) / sizeof(kFftSizesA[0]));
}  // namespace tomo
