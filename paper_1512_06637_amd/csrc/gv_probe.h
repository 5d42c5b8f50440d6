// Roof probes: what this device reaches on a plain stream from HBM and on a
// plain chain of FP64 fused multiply-adds, measured beside the kernels whose
// fractions of those roofs are reported.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gv {

// c[i] = a[i] + s b[i] over n doubles (two loads and one store of 16 bytes per
// lane per iteration), grid-stride.  With b NULL it is the copy c[i] = a[i].
__global__ void __launch_bounds__(256) k_probe_triad(const double2* __restrict__ a, const double2* __restrict__ b,
                                                      double2* __restrict__ c, double s, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
    const double2 x = a[i];
    if (b) {
      const double2 y = b[i];
      c[i] = double2{fma(s, y.x, x.x), fma(s, y.y, x.y)};
    } else {
      c[i] = x;
    }
  }
}

// Eight independent chains v = v * m + q per lane, `iters` rounds: 8 iters FP64
// FMAs per lane (v_fma_f64), then one store per lane so nothing is dead.  The
// chains converge to q / (1 - m) and never overflow or go denormal.
__global__ void __launch_bounds__(256) k_probe_fma64(double* __restrict__ out, int iters, double m, double q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v0 = 1e-3 * threadIdx.x, v1 = v0 + 1.0, v2 = v0 + 2.0, v3 = v0 + 3.0;
  double v4 = v0 + 4.0, v5 = v0 + 5.0, v6 = v0 + 6.0, v7 = v0 + 7.0;
  for (int k = 0; k < iters; ++k) {
    v0 = fma(v0, m, q);
    v1 = fma(v1, m, q);
    v2 = fma(v2, m, q);
    v3 = fma(v3, m, q);
    v4 = fma(v4, m, q);
    v5 = fma(v5, m, q);
    v6 = fma(v6, m, q);
    v7 = fma(v7, m, q);
  }
  out[i] = ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7));
}

}  // namespace gv
