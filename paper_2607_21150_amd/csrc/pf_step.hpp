// Kernels around the operator for a Newton step: Dirichlet face masks, FP64
// Krylov vector operations with deterministic reductions, precision conversions,
// and the device-side pieces of the power iteration (start vector, norms).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf_brick.hpp"

namespace pfmf {

// Fields constrained on each face of the box: bit f of face[k] set means field f
// (u_x, u_y, u_z, phi) is prescribed on face k = x0, x1, y0, y1, z0, z1.
struct DirMask {
  uint32_t face[6];
};

// v[f][i] = 0 for every constrained (node, field) of a [4][n] vector on a lattice. The
// threads run over the nodes of the six boundary faces only (x = 0, x = max, y = 0, ...,
// each face as its own range); a node on an edge or corner is zeroed once per face that
// constrains it (the same zeros, so the result does not depend on the order).
template <typename T>
__global__ void k_mask(T* __restrict__ v, int nx1, int ny1, int nz1, DirMask d) {
  const int64_t n = (int64_t)nx1 * ny1 * nz1;
  const int64_t fx = (int64_t)ny1 * nz1, fy = (int64_t)nx1 * nz1, fz = (int64_t)nx1 * ny1;
  const int64_t total = 2 * (fx + fy + fz);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = t, i;
    int face;
    if (r < 2 * fx) {
      face = (int)(r / fx);
      r -= face * fx;
      const int64_t iy = r % ny1, iz = r / ny1;
      i = (face ? nx1 - 1 : 0) + (int64_t)nx1 * (iy + (int64_t)ny1 * iz);
    } else if ((r -= 2 * fx) < 2 * fy) {
      face = 2 + (int)(r / fy);
      r -= (face - 2) * fy;
      const int64_t ix = r % nx1, iz = r / nx1;
      i = ix + (int64_t)nx1 * ((face == 3 ? ny1 - 1 : 0) + (int64_t)ny1 * iz);
    } else {
      r -= 2 * fy;
      face = 4 + (int)(r / fz);
      r -= (face - 4) * fz;
      i = r + (face == 5 ? (int64_t)(nz1 - 1) * fz : 0);
    }
    const uint32_t f = d.face[face];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if ((f >> k) & 1u) v[k * n + i] = T(0);
  }
}

// Start vector of the power iteration: uniform values in [-1, 1) from a
// counter-based mix (SplitMix64 finaliser) of (seed, index).
static __global__ void k_hash_fill(float* __restrict__ x, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (float)((double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0);
  }
}

// Sum of the first n partials (one block of NT threads, fixed strided order and a
// fixed tree): out[0] = sqrt(sum), inv[0] = 1 / sqrt(sum) (0 when the sum vanishes).
static __global__ void k_norm_finish(const double* __restrict__ part, int n, double* __restrict__ out,
                              float* __restrict__ inv) {
  __shared__ double red[NT];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r = sqrt(red[0]);
    out[0] = r;
    inv[0] = r > 0.0 ? (float)(1.0 / r) : 0.f;
  }
}

// b = s[0] * a (scale held in device memory)
static __global__ void k_vec_axs_dev(const float* __restrict__ a, float* __restrict__ b, const float* __restrict__ s,
                              int64_t n) {
  const float f = s[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = f * a[i];
}

// ---------------------------------------------------------------------------
// FP64 Krylov vectors. Reductions are per-block partials in a fixed order,
// summed on the host in index order, so every result is bitwise reproducible.
// ---------------------------------------------------------------------------

// part[j * gridDim.x + b] = block b's share of <V_j, w>, j = 0..k-1, V_j = V + j * ld.
static __global__ void k_mdot(const double* __restrict__ V, int64_t ld, int k, const double* __restrict__ w, int64_t n,
                       double* __restrict__ part) {
  __shared__ double red[NT];
  const int j = blockIdx.y;
  if (j >= k) return;
  const double* v = V + (int64_t)j * ld;
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += v[i] * w[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
}

// w += sum_j c[j] V_j  (c in device memory, k <= 64)
static __global__ void k_maxpy(const double* __restrict__ V, int64_t ld, int k, const double* __restrict__ c,
                        double* __restrict__ w, int64_t n) {
  __shared__ double cs[64];
  if ((int)threadIdx.x < k) cs[threadIdx.x] = c[threadIdx.x];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double acc = w[i];
    for (int j = 0; j < k; ++j) acc += cs[j] * V[(int64_t)j * ld + i];
    w[i] = acc;
  }
}

// ---- Gram-Schmidt passes that read each basis vector once (k <= GS_MAX vectors) ----
constexpr int GS_MAX = 32;

// Sum each of the k per-thread values acc[0..k) over the block (wave butterflies, then
// the 4 wave sums in wave order) and store block b's share as part[j * gridDim.x + b].
template <int KM>
__device__ __forceinline__ void block_partials(const double* acc, int k, double* __restrict__ part) {
  __shared__ double red[(NT / 64) * KM];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (j < k) {  // uniform: the whole block takes the same branch
      double v = acc[j];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (l == 0) red[wv * KM + j] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w * KM + threadIdx.x];
    part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

// part: block shares of <V_j, w>, j = 0..k-1, with w read once (k <= GS_MAX).
static __global__ __launch_bounds__(NT) void k_mdot_multi(const double* __restrict__ V, int64_t ld, int k,
                                                   const double* __restrict__ w, int64_t n,
                                                   double* __restrict__ part) {
  double acc[GS_MAX];
#pragma unroll
  for (int j = 0; j < GS_MAX; ++j) acc[j] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = w[i];
#pragma unroll
    for (int j = 0; j < GS_MAX; ++j)
      if (j < k) acc[j] += V[(int64_t)j * ld + i] * wi;
  }
  block_partials<GS_MAX>(acc, k, part);
}

// One Gram-Schmidt correction and, in the same pass, the next one's projections or the
// new norm: w += sum_j c[j] V_j (c in device memory), then
//   DOTS: part = block shares of <V_j, w_new>, j < k (the refinement's projections);
//   otherwise part = block shares of ||w_new||^2 (one value per block).
template <bool DOTS>
__global__ __launch_bounds__(NT) void k_maxpy_fused(const double* __restrict__ V, int64_t ld, int k,
                                                    const double* __restrict__ c, double* __restrict__ w, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double cs[GS_MAX];
  if ((int)threadIdx.x < k) cs[threadIdx.x] = c[threadIdx.x];
  __syncthreads();
  double acc[DOTS ? GS_MAX : 1];
#pragma unroll
  for (int j = 0; j < (DOTS ? GS_MAX : 1); ++j) acc[j] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double x = w[i];
    for (int j = 0; j < k; ++j) x += cs[j] * V[(int64_t)j * ld + i];
    w[i] = x;
    if (DOTS) {
#pragma unroll
      for (int j = 0; j < GS_MAX; ++j)
        if (j < k) acc[j] += V[(int64_t)j * ld + i] * x;
    } else {
      acc[0] += x * x;
    }
  }
  block_partials<DOTS ? GS_MAX : 1>(acc, DOTS ? k : 1, part);
}

// y = a x (+ y when accumulate); x may be y
static __global__ void k_daxpy(double a, const double* x, double* y, int64_t n, int accumulate) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (accumulate ? y[i] : 0.0);
}

static __global__ void k_dzero(double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = 0.0;
}

static __global__ void k_d2f(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

static __global__ void k_f2d(const float* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

}  // namespace pfmf
