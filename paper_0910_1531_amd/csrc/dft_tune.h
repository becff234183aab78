// Autotuner of the compiled-length kernels' launch shapes (dft_tune.hip).
#pragma once

#include <cstddef>

#include "dft_kernels.h"

namespace dft {

// Spectral buffers the tuner may overwrite (the context's scratch spectra at setup).
struct TuneBufs {
    void *specA;
    size_t bytesA;
    void *specB;
    size_t bytesB;
};

// Times every launch shape of the tunable passes for the precisions asked for and stores
// the fastest in g.tune (shape choices are cached per process by problem shape).
void autotune(Geo &g, const TuneBufs &b, bool fp64, bool fp32, hipStream_t s);

}  // namespace dft
