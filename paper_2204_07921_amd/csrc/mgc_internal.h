// Internal interface between the host runtime and the kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

namespace mgc {

struct LaunchCtx {
    hipStream_t stream;
    int H, W;
    double alpha;
    int kind;   // 0 mean, 1 Gaussian
    bool f64;   // state dtype
    int M, G;   // samples, bisection steps
};

// b = 1: colour sweep from uin into uout (every pixel of uout is written).
hipError_t launch_sweep_pixels(const LaunchCtx& L, const void* uin, void* uout, const void* f, int colour, int ncolours);
// b >= 2: colour sweep in place.
hipError_t launch_sweep_blocks(const LaunchCtx& L, void* u, const void* f, int b, int colour);
// F(u) into out[0] (device), using partials (energy_partials_count doubles).
hipError_t launch_energy(const LaunchCtx& L, const void* u, const void* f, double* partials, double* out);
int energy_partials_count(int H, int W);

}  // namespace mgc
