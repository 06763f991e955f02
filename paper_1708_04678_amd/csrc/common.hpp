// Generic pieces of the gfx950 kernels shared by the 2-D (D2Q9, triangles) and
// 3-D (D3Q19, tetrahedra) step: launch shape, the XCD-aware block remap,
// wavefront and block reductions, the step's physical constants and the
// deterministic two-pass FP64 reduction of the diagnostics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace felbm {

constexpr int BLOCK = 256;
constexpr double CS2 = 1.0 / 3.0;

struct StepParams {
  double kappa, beta, mobility, rho_l, rho_v, inv_tau_l, inv_tau_v, dt;
};

struct Band {
  double xc, yc, r_lo2, r_hi2, period;  // squared radii of the band, x period (0 = none)
  int enabled;
};

// ----------------------------------------------------------------------------
// launch helpers
// ----------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X; the
// grid is padded to a multiple of 8 and block b is remapped so that every XCD
// walks one contiguous range of nodes (neighbour gathers then hit its own L2).
__device__ __forceinline__ int xcd_block() {
  const int per = gridDim.x >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Deterministic block reduction of NR doubles (sum for all but index imax,
// which is reduced by max); thread 0 writes partials[k * nblk + blk].
template <int NR>
__device__ __forceinline__ void block_reduce_store(double (&v)[NR], int imax, double* partials, int nblk, int blk) {
  __shared__ double red[NR][BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    double r = (k == imax) ? wave_max(v[k]) : wave_sum(v[k]);
    if (lane == 0) red[k][wid] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      double r = red[k][0];
      for (int w = 1; w < BLOCK / 64; ++w) r = (k == imax) ? fmax(r, red[k][w]) : r + red[k][w];
      partials[k * nblk + blk] = r;
    }
  }
}

constexpr int NRED = 6;  // mass, sum rho|u|^2, max|u|, band sum, band count, nonfinite count

// The diagnostics record (mirrors the first members of felbm_diag) and the
// second, fixed-order pass over the block partials.
struct DiagRecord {  // mirrors felbm_diag
  int64_t step;
  double mass, mean_ke, max_u, band_ke;
  int64_t band_nodes;
  int32_t nonfinite, pad_;
};

// Second, fixed-order pass over the block partials (one block of RBLOCK
// threads, four independent accumulators per thread to hide load latency).
constexpr int RBLOCK = 1024;
constexpr int RBLOCK_RES = 256;
template <int UNUSED = 0>
__global__ void __launch_bounds__(RBLOCK) k_reduce_final(const double* __restrict__ partials, int nblk, int N,
                                                          int64_t step, DiagRecord* __restrict__ out,
                                                          int* __restrict__ first_bad) {
  double v[NRED];
#pragma unroll
  for (int k = 0; k < NRED; ++k) {
    const bool mx = (k == 2);
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
    const double* p = partials + (size_t)k * nblk;
    int b = threadIdx.x;
    for (; b + 3 * RBLOCK < nblk; b += 4 * RBLOCK) {
      const double a0 = p[b], a1 = p[b + RBLOCK], a2 = p[b + 2 * RBLOCK], a3 = p[b + 3 * RBLOCK];
      if (mx) { r0 = fmax(r0, a0); r1 = fmax(r1, a1); r2 = fmax(r2, a2); r3 = fmax(r3, a3); }
      else { r0 += a0; r1 += a1; r2 += a2; r3 += a3; }
    }
    for (; b < nblk; b += RBLOCK) r0 = mx ? fmax(r0, p[b]) : r0 + p[b];
    v[k] = mx ? fmax(fmax(r0, r1), fmax(r2, r3)) : (r0 + r1) + (r2 + r3);
  }
  __shared__ double red[NRED][RBLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NRED; ++k) {
    double r = (k == 2) ? wave_max(v[k]) : wave_sum(v[k]);
    if (lane == 0) red[k][wid] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[NRED];
    for (int k = 0; k < NRED; ++k) {
      r[k] = red[k][0];
      for (int w = 1; w < RBLOCK / 64; ++w) r[k] = (k == 2) ? fmax(r[k], red[k][w]) : r[k] + red[k][w];
    }
    DiagRecord d;
    d.step = step;
    d.mass = r[0];
    d.mean_ke = 0.5 * r[1] / (double)N;
    d.max_u = r[2];
    d.band_ke = r[4] > 0 ? r[3] / r[4] : 0.0;
    d.band_nodes = (int64_t)r[4];
    d.nonfinite = r[5] > 0 ? 1 : 0;
    d.pad_ = 0;
    *out = d;
    if (d.nonfinite && *first_bad < 0) *first_bad = (int)step;
  }
}

}  // namespace felbm
