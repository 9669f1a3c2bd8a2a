"""MI355X-native hot path of the multi-resolution approximation (MRA) for
Gaussian processes: log-likelihood and kriging through a C-ABI library of
hand-written HIP kernels for gfx950."""
