// Device twin of the seeded input generator in csynth.c (same definition:
// counter-based SplitMix64 draws, Box-Muller normals, scaled per auxiliary
// index or per (occupied, auxiliary) pair).  Input harness only: it holds
// none of the MP2 arithmetic.  Device log/cos may differ from the host's in
// the last bit, so values agree with the host generator to ~1e-15 relative,
// not bitwise; checks against the CPU oracle read the device arrays back.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#define GOLDEN 0x9E3779B97F4A7C15ULL

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t n) { return mix64(key + (n + 1) * GOLDEN); }
__device__ __forceinline__ double uniform01(uint64_t x) { return ((double)(x >> 11) + 0.5) * 0x1.0p-53; }

// Grid-stride loop: a dispatch's grid size counts work-items in 32 bits, so
// the grid is capped and each thread covers several elements.
__global__ void three_index_kernel(uint64_t key, int64_t i0, int64_t nrows, int64_t nvir, int64_t naux,
                                   const double* scale, int per_i, double* out) {
  const int64_t total = nrows * naux, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const int64_t r = idx / naux, P = idx - r * naux;       // r: row within [i0*nvir, ...)
    const int64_t i = i0 + r / nvir;
    const uint64_t e = (uint64_t)((i0 * nvir + r) * naux + P);
    const double u1 = uniform01(draw(key, 2 * e)), u2 = uniform01(draw(key, 2 * e + 1));
    const double n = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    out[idx] = n * scale[(per_i ? i * naux : 0) + P];
  }
}

extern "C" int dsynth_three_index(uint64_t key, int64_t i0, int64_t i1, int64_t nvir, int64_t naux,
                                  const double* scale_dev, int per_i, double* out_dev, void* stream) {
  const int64_t rows = (i1 - i0) * nvir, total = rows * naux;
  if (total <= 0) return 0;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(three_index_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, key, i0, rows,
                     nvir, naux, scale_dev, per_i, out_dev);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
