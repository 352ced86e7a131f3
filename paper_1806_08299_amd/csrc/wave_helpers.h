// wave_helpers.h -- small utility kernels (one translation unit only: wave_api.cpp).
#pragma once
#include "wave_device.h"

namespace wavett {

// --------------------------------------------------------------- helpers

// b = dt^2 / m, evaluated in FP64 and rounded once.
__global__ void k_compute_b(const float* m, float* b, int64_t n, double dt2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)(dt2 / (double)m[i]);
}

// table[n][p] = scale * sum_e w[e] * q[n][src[e]] over e in [ptr[p], ptr[p+1]).
__global__ void k_forcing_table(const float* q, int nq, int nt, const int32_t* ptr, const int32_t* src,
                                const float* w, int npts, float scale, float* table) {
  const int64_t total = (int64_t)nt * npts;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(e / npts), p = (int)(e % npts);
    float s = 0.0f;
    for (int k = ptr[p]; k < ptr[p + 1]; ++k) s = __builtin_fmaf(w[k], q[(int64_t)n * nq + src[k]], s);
    table[e] = s * scale;
  }
}

// out[n][r] = scale * sum over corners c of position r of w[c] * samp[n][pt[c]].
__global__ void k_reduce_samples(const float* samp, int npts, int nt, const int32_t* ptr, const int32_t* pt,
                                 const float* w, int npos, float scale, float* out) {
  const int64_t total = (int64_t)nt * npos;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(e / npos), r = (int)(e % npos);
    float s = 0.0f;
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) s = __builtin_fmaf(w[k], samp[(int64_t)n * npts + pt[k]], s);
    out[e] = s * scale;
  }
}

__global__ void k_fill(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_copy(const float* __restrict__ s, float* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) d[i] = s[i];
}

// out = a - b (the residual of modelled against observed traces).
__global__ void k_sub(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

}  // namespace wavett
