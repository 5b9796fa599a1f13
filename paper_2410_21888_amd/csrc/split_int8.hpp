// Split-precision (Ozaki-style) products on gfx950 INT8 MFMA.
//
// A row (or column) x of an FP64 operand is scaled by 2^-e with
// e = ilogb(max |x|) + 1, so |x| 2^-e < 1, and written as S balanced base-128
// digits:  x = 2^e / 64 * sum_{s=1..S} d_s 128^(1-s),  |d_s| <= 64,  extracted
// exactly in FP64 with round-to-nearest (y = x 2^(6-e); d = rint(y);
// y = (y - d) * 128; ...).  The dropped remainder is at most 2^-7S relative
// to the row maximum.
//
// C = A B^T is then
//   C[m,n] = 2^(ea[m] + eb[n] - 12) * sum_{L=2..S+1} 128^(2-L) * sum_{s+t=L} D_s(A) D_t(B)^T
// (the products with s + t > S + 1 are below the digit truncation and are
// dropped: S(S+1)/2 integer products).  Each level is summed exactly in INT32
// by v_mfma_i32_16x16x64_i8; to rule out overflow the levels are moved into
// FP64 accumulators every kFlushK reduction steps (S * kFlushK * 64 * 64 < 2^31).
//
// MFMA lane layout (measured on gfx950): lane l supplies A[l%16][16(l/16)+b]
// and B[16(l/16)+b][l%16] for byte b; accumulator register r of lane l holds
// D[4(l/16)+r][l%16].  A and B digits are read with the same lane/byte -> k
// map, so the reduction index needs no particular order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rimp2 {

typedef int v4i __attribute__((ext_vector_type(4)));
constexpr int64_t kFlushK = 65536;

// Row-scaled digits of a K-contiguous FP64 matrix X[rows][K] (row stride ld):
// D[s][row][kp] (kp = K rounded up to 64, zero padded) and exps[row].
// One workgroup per row.
template <int S>
__device__ __forceinline__ void split_row(const double* X, int64_t rows, int64_t K, int64_t ld, int8_t* D,
                                          int64_t kp, int32_t* exps, int64_t row) {
  const double* x = X + row * ld;
  __shared__ double sm[256];
  double mx = 0.0;
  for (int64_t k = threadIdx.x; k < K; k += 256) mx = fmax(mx, fabs(x[k]));
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  mx = sm[0];
  const int e = (mx > 0.0) ? ilogb(mx) + 1 : 0;
  if (threadIdx.x == 0) exps[row] = e;
  for (int64_t k = threadIdx.x; k < kp; k += 256) {
    double y = (k < K) ? ldexp(x[k], 6 - e) : 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double d = rint(y);
      D[((int64_t)s * rows + row) * kp + k] = (int8_t)d;
      y = (y - d) * 128.0;
    }
  }
}

template <int S>
__global__ __launch_bounds__(256) void split_rows_kernel(const double* X, int64_t rows, int64_t K, int64_t ld,
                                                         int8_t* D, int64_t kp, int32_t* exps, const int32_t* status) {
  if (status != nullptr && *status != 0) return;
  split_row<S>(X, rows, K, ld, D, kp, exps, blockIdx.x);
}

// Column maxima of X[K][N] (row stride ld) as IEEE bit patterns (non-negative
// doubles order like their bit patterns, so an integer max is exact and
// order-independent).  cmax must start at zero.
__device__ __forceinline__ void colmax_block(const double* X, int64_t K, int64_t N, int64_t ld,
                                             unsigned long long* cmax, int64_t bx, int64_t by) {
  const int64_t n = bx * 256 + threadIdx.x;
  if (n >= N) return;
  const int64_t k0 = by * 1024, k1 = min(K, k0 + 1024);
  double mx = 0.0;
  for (int64_t k = k0; k < k1; ++k) mx = fmax(mx, fabs(X[k * ld + n]));
  atomicMax(cmax + n, (unsigned long long)__double_as_longlong(mx));
}

__global__ __launch_bounds__(256) void colmax_kernel(const double* X, int64_t K, int64_t N, int64_t ld,
                                                     unsigned long long* cmax, const int32_t* status) {
  if (status != nullptr && *status != 0) return;
  colmax_block(X, K, N, ld, cmax, blockIdx.x, blockIdx.y);
}

// Column-scaled digits of X[K][N], written transposed: D[s][n][kp], exps[n].
// 32 x 32 tiles through LDS so both the read and the write are coalesced.
template <int S>
__device__ __forceinline__ void split_cols_tile(const double* X, int64_t K, int64_t N, int64_t ld,
                                                const unsigned long long* cmax, int8_t* D, int64_t kp,
                                                int32_t* exps, int64_t bx, int64_t by) {
  __shared__ double tile[32][33];
  const int64_t k0 = bx * 32, n0 = by * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows per pass
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t k = k0 + ty + 8 * r, n = n0 + tx;
    tile[ty + 8 * r][tx] = (k < K && n < N) ? X[k * ld + n] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t n = n0 + ty + 8 * r, k = k0 + tx;
    if (n >= N || k >= kp) continue;
    const double mx = __longlong_as_double((long long)cmax[n]);
    const int e = (mx > 0.0) ? ilogb(mx) + 1 : 0;
    if (k == 0) exps[n] = e;
    double y = ldexp(tile[tx][ty + 8 * r], 6 - e);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double d = rint(y);
      D[((int64_t)s * N + n) * kp + k] = (int8_t)d;
      y = (y - d) * 128.0;
    }
  }
}

template <int S>
__global__ __launch_bounds__(256) void split_cols_kernel(const double* X, int64_t K, int64_t N, int64_t ld,
                                                         const unsigned long long* cmax, int8_t* D, int64_t kp,
                                                         int32_t* exps, const int32_t* status) {
  if (status != nullptr && *status != 0) return;
  split_cols_tile<S>(X, K, N, ld, cmax, D, kp, exps, blockIdx.x, blockIdx.y);
}

struct OzParams {
  int64_t M, N, kp;            // kp: padded reduction length (multiple of 64), also the digit row stride
  int64_t k0, kc;              // this launch reduces over [k0, k0 + kc) (multiples of 64)
  int32_t accumulate;          // 0: C = the window's sum; 1: C += it
  const int8_t* A;             // digits [S][a_rows][kp]; output rows m use A row a_row0 + m
  int64_t a_slice, a_row0;
  const int8_t* B;             // digits [S][b_rows][kp]
  int64_t b_slice;
  const int32_t* ea;           // exponents of A rows (indexed like A rows)
  const int32_t* eb;
  double* C;
  int64_t ldc;
  int32_t tiles_m, tiles_n, group_m;
  int32_t pair_nvir;           // > 0: skip tiles below the pair-block diagonal (see oz8_tile_skipped)
  const int32_t* status;
};

// 256 threads = 4 waves in 2 x 2; workgroup tile 64 x 64, wave tile 32 x 32
// (2 x 2 MFMA blocks).  All S digit slices of a 64-wide reduction step are
// staged in LDS (S * 8 KB): wave w moves row block w (16 rows x 64 bytes,
// 1 KB) of every (slice, operand).  Within a 1 KB block lane l writes bytes
// [16 l, 16 l + 16), and it loads row r = l / 4, 16-byte chunk
// (l % 4) ^ ((r / 4) % 4): an XOR swizzle that makes the MFMA fragment reads
// (16 lanes reading 16 rows of one chunk) free of bank conflicts.
// NBUF = 2 double-buffers the stage (the next step's copy runs under this
// step's MFMAs); NBUF = 1 keeps one stage, copied after the step's MFMAs, so
// that two workgroups share a CU at any S (measured the faster of the two).
template <int S>
struct OzLds {
  static constexpr int STAGE = S * 2 * 4 * 1024;   // S slices x (A, B) x 4 row blocks x 1 KB
};

// Tiles entirely below the pair-block diagonal (every column block j before
// every row block k) are skipped when p.pair_nvir > 0: the amplitude pass
// forms those blocks from their mirror.
__device__ __forceinline__ bool oz8_tile_skipped(const OzParams& p, int64_t m0, int64_t n0) {
  if (p.pair_nvir <= 0) return false;
  const int64_t last_j = min(n0 + 63, p.N - 1) / p.pair_nvir, first_k = (p.a_row0 + m0) / p.pair_nvir;
  return last_j < first_k;
}

// One 64 x 64 output tile at (m0, n0) over the reduction window [k0, k0 + kc).
template <int S, int NBUF>
__device__ __forceinline__ void oz8_tile(const OzParams& p, int64_t m0, int64_t n0,
                                         int8_t (*lds)[OzLds<S>::STAGE]) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int wm = wv >> 1, wn = wv & 1;

  // copy: rows past the end read the last row (their outputs are not stored)
  const int dr = lane >> 2, dc = (lane & 3) ^ ((dr >> 2) & 3);
  const int64_t rowA = p.a_row0 + min(m0 + 16 * wv + dr, p.M - 1), rowB = min(n0 + 16 * wv + dr, p.N - 1);
  const int8_t* srcA = p.A + rowA * p.kp + 16 * dc;
  const int8_t* srcB = p.B + rowB * p.kp + 16 * dc;
  auto copy = [&](int buf, int64_t k) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      __builtin_amdgcn_global_load_lds((const void*)(srcA + s * p.a_slice + k),
                                       (void*)(lds[buf] + ((s * 2 + 0) * 4 + wv) * 1024), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(srcB + s * p.b_slice + k),
                                       (void*)(lds[buf] + ((s * 2 + 1) * 4 + wv) * 1024), 16, 0, 0);
    }
  };
  // fragment of lane (g, l16): row l16 of a row block, data chunk g
  const int fpos = (l16 * 4 + (g ^ ((l16 >> 2) & 3))) * 16;

  v4i acc[S][2][2];
  auto zero_acc = [&]() {
#pragma unroll
    for (int L = 0; L < S; ++L)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[L][i][j] = v4i{0, 0, 0, 0};
  };
  // flush: the levels of each output are combined in FP64, scaled by the
  // output's exponents (a power of two: exact) and added to C; the first flush
  // of a launch that does not accumulate stores.  C holds the running sum
  // between flushes, so no FP64 accumulators stay live in the loop.
  bool first_flush = p.accumulate == 0;
  auto flush = [&]() {
    int xa[2][4], xb[2];   // exponents of this lane's output rows and columns
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 32 + 16 * i + 4 * g + r;
        xa[i][r] = m < p.M ? p.ea[p.a_row0 + m] : 0;
      }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t n = n0 + wn * 32 + 16 * j + l16;
      xb[j] = n < p.N ? p.eb[n] : 0;
    }
    double w[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double v = 0.0;
#pragma unroll
          for (int L = S - 1; L >= 0; --L) v = v * (1.0 / 128.0) + (double)acc[L][i][j][r];
          w[i][j][r] = ldexp(v, xa[i][r] + xb[j] - 12);
        }
    zero_acc();
    // per row block i: the C reads (clamped: always in bounds and without a
    // branch, so the 8 loads go out together; what an out-of-range output
    // reads is never stored), then the stores
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (!first_flush) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t m = min(m0 + wm * 32 + 16 * i + 4 * g + r, p.M - 1);
            const int64_t n = min(n0 + wn * 32 + 16 * j + l16, p.N - 1);
            w[i][j][r] += p.C[m * p.ldc + n];
          }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = m0 + wm * 32 + 16 * i + 4 * g + r, n = n0 + wn * 32 + 16 * j + l16;
          if (m < p.M && n < p.N) p.C[m * p.ldc + n] = w[i][j][r];
        }
    }
    first_flush = false;
  };
  zero_acc();

  const int nsteps = (int)(p.kc / 64);
  const int flush_every = (int)(kFlushK / 64);
  if (nsteps > 0) copy(0, p.k0);
  for (int st = 0; st < nsteps; ++st) {
    const int b = (NBUF == 2) ? (st & 1) : 0;
    // LDS copies count in vmcnt: wait for this wave's, then the barrier makes
    // every wave's visible (and frees the other buffer)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (NBUF == 2 && st + 1 < nsteps) copy(b ^ 1, p.k0 + (int64_t)(st + 1) * 64);
    const int8_t* L0 = lds[b];
    v4i fb[S][2];
#pragma unroll
    for (int t = 0; t < S; ++t)
#pragma unroll
      for (int j = 0; j < 2; ++j) fb[t][j] = *(const v4i*)(L0 + ((t * 2 + 1) * 4 + 2 * wn + j) * 1024 + fpos);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      v4i fa[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[i] = *(const v4i*)(L0 + ((s * 2 + 0) * 4 + 2 * wm + i) * 1024 + fpos);
#pragma unroll
      for (int t = 0; t < S - s; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[s + t][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[i], fb[t][j], acc[s + t][i][j], 0, 0, 0);
    }
    if (NBUF == 1 && st + 1 < nsteps) {
      __syncthreads();   // every wave is done reading the stage
      copy(0, p.k0 + (int64_t)(st + 1) * 64);
    }
    if ((st + 1) % flush_every == 0) flush();
  }
  flush();
}

template <int S, int NBUF>
__global__ __launch_bounds__(256, 2) void gemm_oz8_kernel(OzParams p) {
  if (p.status != nullptr && *p.status != 0) return;
  __shared__ __attribute__((aligned(1024))) int8_t lds[NBUF][OzLds<S>::STAGE];
  const int wl = xcd_remap(blockIdx.x, gridDim.x);
  const int gsz = p.group_m * p.tiles_n, grp = wl / gsz, first_m = grp * p.group_m;
  const int gm = min(p.group_m, p.tiles_m - first_m), tin = wl - grp * gsz;
  const int64_t m0 = (int64_t)(first_m + tin % gm) * 64, n0 = (int64_t)(tin / gm) * 64;
  if (oz8_tile_skipped(p, m0, n0)) return;
  oz8_tile<S, NBUF>(p, m0, n0, lds);
}

// Persistent grouped launch over the split products of many fragments:
// problem f owns work items [prefix[f], prefix[f+1]) = its tiles, problems
// ordered largest first.  Each workgroup takes items from *counter (zero at
// launch) until all are taken, so every workgroup exits.  window >= 0 runs
// reduction window `window` of every problem (k0 = window * wlen, the first
// window stores and later ones add into C; problems with fewer windows skip
// their items); window < 0 runs each problem's whole reduction.
struct OzGroup {
  const OzParams* probs;
  const int64_t* prefix;   // [nprob + 1]
  int32_t nprob;
  unsigned long long* counter;
};

template <int S, int NBUF>
__global__ __launch_bounds__(256, 2) void gemm_oz8_grouped(OzGroup G, int64_t window, int64_t wlen) {
  __shared__ __attribute__((aligned(1024))) int8_t lds[NBUF][OzLds<S>::STAGE];
  __shared__ long long item;
  const long long total = G.prefix[G.nprob];
  for (;;) {
    if (threadIdx.x == 0) item = (long long)atomicAdd(G.counter, 1ull);
    __syncthreads();
    const long long t = item;
    __syncthreads();
    if (t >= total) break;
    int lo = 0, hi = G.nprob - 1;   // last f with prefix[f] <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (G.prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    OzParams p = G.probs[lo];
    if (p.status != nullptr && *p.status != 0) continue;
    if (window >= 0) {
      p.k0 = window * wlen;
      if (p.k0 >= p.kp && window > 0) continue;
      p.kc = min(wlen, p.kp - p.k0);
      p.accumulate = window > 0;
    }
    const int64_t u = t - G.prefix[lo];
    const int64_t m0 = (u % p.tiles_m) * 64, n0 = (u / p.tiles_m) * 64;
    if (oz8_tile_skipped(p, m0, n0)) continue;
    oz8_tile<S, NBUF>(p, m0, n0, lds);
  }
}

}  // namespace rimp2
