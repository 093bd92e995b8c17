// Device evaluation of travelling-wave boundary values (kernels_wave.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "lbmhpde.h"

namespace lbm {

// rows[s * 2 layers + k] = phi*(x_node(k), w.t0 + (s + 1) dt) of wave w for
// s < steps, k < 2 layers (node k for k < layers, else n - 2 layers + k); a
// device array of steps * 2 layers doubles.  The wave must be valid.
hipError_t launch_wave_rows(double* rows, int64_t steps, int layers, int n, double dx, double dt,
                            const lbm_wave& w, hipStream_t s);

}  // namespace lbm
