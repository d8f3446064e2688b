// Final reduction of the observable sums (one block, fixed order).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_kernels.hpp"

namespace tlbk {

// Final observable reduction: one block sums the per-block partials in a
// fixed order and forms the observables of the header's definitions. The
// fluid-node sum of the central differences of T, with the mirror value
// 2 T_w - T at a solid neighbour, telescopes along every column to the
// wall temperatures above and below each run of fluid nodes; that sum
// (`dtdy_sum`) is formed on the host from the solid map and the wall
// temperatures.
struct ObsArgs {
  const double* partials;   // [nblocks][kObsSums]
  int nblocks;
  double n_fluid, n_top;
  double kappa, dt_nominal, ly;
  double dtdy_sum;
  double* out;   // [6] mass_a, mass_b, sum_t, nu, nu_top, ke
};

__global__ __launch_bounds__(256) void lb_reduce_observables(ObsArgs a) {
  __shared__ double s[kObsSums][256];
  const int tid = threadIdx.x;
  double v[kObsSums] = {0, 0, 0, 0, 0, 0};
  for (int b = tid; b < a.nblocks; b += 256)
    for (int j = 0; j < kObsSums; ++j) v[j] += a.partials[(size_t)b * kObsSums + j];
  for (int j = 0; j < kObsSums; ++j) s[j][tid] = v[j];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h)
      for (int j = 0; j < kObsSums; ++j) s[j][tid] += s[j][tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    const double inv = a.n_fluid > 0 ? 1.0 / a.n_fluid : 0.0;
    a.out[0] = s[0][0];
    a.out[1] = s[1][0];
    a.out[2] = s[2][0];
    a.out[3] = (s[3][0] * inv - a.kappa * a.dtdy_sum * inv) / (a.kappa * a.dt_nominal / a.ly);
    a.out[4] = a.n_top > 0 ? 2.0 * a.ly / a.dt_nominal * (s[5][0] / a.n_top) : 0.0;
    a.out[5] = s[4][0] * inv;
  }
}

// Row averages over fluid nodes (the x-averages of the Couette rheology):
// one block per row sums u^H_x (field plane 2) and the total xy stress
// (plane 5 minus plane 6) in a fixed order. Rows without fluid report 0.
__global__ __launch_bounds__(256) void lb_row_averages(const double* __restrict__ fields,
                                                       const uint8_t* __restrict__ solid, int lx,
                                                       int ly, double* __restrict__ u_av,
                                                       double* __restrict__ pxy_av) {
  __shared__ double su[256], sp[256], sn[256];
  const int tid = threadIdx.x, y = blockIdx.x;
  const size_t nn = (size_t)lx * ly;
  double u = 0, pxy = 0, n = 0;
  for (int x = tid; x < lx; x += 256) {
    const size_t q = (size_t)y * lx + x;
    if (solid[q] != 0) continue;
    u += fields[2 * nn + q];
    pxy += fields[5 * nn + q] - fields[6 * nn + q];
    n += 1.0;
  }
  su[tid] = u;
  sp[tid] = pxy;
  sn[tid] = n;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      su[tid] += su[tid + h];
      sp[tid] += sp[tid + h];
      sn[tid] += sn[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    u_av[y] = sn[0] > 0 ? su[0] / sn[0] : 0.0;
    pxy_av[y] = sn[0] > 0 ? sp[0] / sn[0] : 0.0;
  }
}

}  // namespace tlbk
