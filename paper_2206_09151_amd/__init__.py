"""MI355X-native reconstruction hot path of the unified CT / phase-contrast CT /
diffraction-tomography method (arXiv:2206.09151): HIP kernels behind the C ABI
of include/tomo.h, with a thin ctypes binding (`tomo`)."""
