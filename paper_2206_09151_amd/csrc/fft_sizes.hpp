// Size tables of the spectra / plane kernels: each fft_sizes_<G>.hip instantiates the
// kernels of its sizes (so that the sizes compile in parallel) and lists them here.
#pragma once
#include "fft_kernels.hpp"

namespace tomo {
extern const FftSize kFftSizesA[];
extern const int kFftSizesACount;
extern const FftSize kFftSizesB[];
extern const int kFftSizesBCount;
extern const FftSize kFftSizesC[];
extern const int kFftSizesCCount;
extern const FftSize kFftSizesD[];
extern const int kFftSizesDCount;
extern const FftSize kFftSizesE[];
extern const int kFftSizesECount;
extern const FftSize kFftSizesF[];
extern const int kFftSizesFCount;
extern const FftSize kFftSizesG[];
extern const int kFftSizesGCount;
extern const FftSize kFftSizesH[];
extern const int kFftSizesHCount;
extern const FftSize kFftSizesI[];
extern const int kFftSizesICount;
extern const FftSize kFftSizesJ[];
extern const int kFftSizesJCount;
}  // namespace tomo
