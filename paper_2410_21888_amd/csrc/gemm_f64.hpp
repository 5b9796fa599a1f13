// FP64 MFMA GEMM for gfx950 (CDNA4): C[m, n] = sum_k A(m, k) B(k, n).
//
// Every dense contraction of the RI-MP2 fragment kernel is one of these:
//   (ia|jb) slab   V[(k,a), (j,b)] = sum_P B[(k,a), P] B[(j,b), P]    (B K-contiguous)
//   Gamma          G[(k,a), P]     = sum_(j,b) T[(k,a), (j,b)] B[(j,b), P] (B N-contiguous)
//   P_ab           sum_(k,j,c) T(a, (k,j,c)) X(b, (k,j,c))                (B K-contiguous)
//   P_ij           sum_(k,a,b) T(i, (k,a,b)) X(j, (k,a,b))                (B K-contiguous)
// The slab operands store the reduction index in two levels (runs of kdiv
// contiguous elements, runs ks1 apart), which the loaders follow directly so
// no operand is ever copied or transposed in HBM.
//
// Tiling: 256 threads = 4 waves in a 2 x 2 grid; each wave owns a
// (BM/2) x (BN/2) block of 16 x 16 accumulators fed by
// v_mfma_f64_16x16x4f64.  Lane layout of that instruction on gfx950
// (measured): lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator
// register r of lane l holds D[4r + l/16][l%16].  Operand tiles are staged
// k-major in LDS (double-buffered, one barrier per BK chunk); the next chunk's
// global loads are issued before the current chunk's MFMAs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rimp2 {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Element (r, k) at base[r * rs + (k / kdiv) * ks1 + (k % kdiv)].
struct KOperand {
  const double* base;
  int64_t rs;
  int64_t kdiv;
  int64_t ks1;
};

// Element (k, n) at base[k * ld + n].
struct NOperand {
  const double* base;
  int64_t ld;
};

struct GemmParams {
  int64_t M, N, K;
  int64_t kchunk;       // reduction length per split (multiple of BK)
  int32_t tiles_m, tiles_n, splits, group_m;
  KOperand A;
  KOperand Bk;          // B when K-contiguous
  NOperand Bn;          // B when N-contiguous
  double* C;            // split z writes C + z * split_stride
  int64_t ldc;
  int64_t split_stride;
  const int32_t* status;  // nonzero: do nothing
};

// Maps the hardware workgroup id to a logical id so that the workgroups one
// XCD runs (dispatch is round-robin over the 8 XCDs) get consecutive logical
// ids, and therefore neighbouring tiles that share operand rows in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int w, int G) {
  const int q = G >> 3, rem = G & 7, x = w & 7;
  return x * q + (x < rem ? x : rem) + (w >> 3);
}

// ROLE only gives each contraction its own kernel symbol (profiler names).
enum GemmRole { ROLE_INTS = 0, ROLE_GAMMA = 1, ROLE_PAB = 2, ROLE_PIJ = 3 };

template <int BM, int BN, int BK, bool B_NCONTIG, int ROLE>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(GemmParams p) {
  static_assert(BM % 32 == 0 && BN % 32 == 0 && BK % 4 == 0, "tile shape");
  static_assert(256 % BK == 0 && BM % (256 / BK) == 0 && BN % (256 / BK) == 0, "loader shape");
  if (p.status != nullptr && *p.status != 0) return;

  constexpr int LDA = BM + 1, LDB = BN + 1;
  constexpr int WTM = BM / 2, WTN = BN / 2, MI = WTM / 16, NI = WTN / 16;
  constexpr int RSTEP = 256 / BK;             // rows covered per pass (K-contiguous loader)
  constexpr int AN = BM / RSTEP, BKN = BN / RSTEP;
  constexpr int NSTEP = 256 / BN;             // k rows per pass (N-contiguous loader)
  constexpr int BNN = B_NCONTIG ? BK / (NSTEP > 0 ? NSTEP : 1) : 0;
  static_assert(!B_NCONTIG || (256 % BN == 0 && BK % (256 / BN) == 0), "N loader shape");
  constexpr int BREG = B_NCONTIG ? BNN : BKN;

  __shared__ double As[2][BK * LDA];
  __shared__ double Bs[2][BK * LDB];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;

  // logical workgroup -> (split, tile); tiles grouped group_m m-tiles wide
  const int wl = xcd_remap(blockIdx.x, gridDim.x);
  const int ntiles = p.tiles_m * p.tiles_n;
  const int z = wl / ntiles;
  const int t = wl - z * ntiles;
  const int gsz = p.group_m * p.tiles_n;
  const int grp = t / gsz;
  const int first_m = grp * p.group_m;
  const int gm = min(p.group_m, p.tiles_m - first_m);
  const int tin = t - grp * gsz;
  const int tm = first_m + tin % gm;
  const int tn = tin / gm;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

  const int64_t kbeg = (int64_t)z * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nchunks = (int)((kend - kbeg + BK - 1) / BK);

  // loader state: this thread's reduction column and its two-level offset
  const int kk = tid % BK, r0 = tid / BK;
  int64_t ka = kbeg + kk;
  int64_t aq = ka / p.A.kdiv, ar = ka - aq * p.A.kdiv;
  int64_t bq = 0, br = 0;
  if (!B_NCONTIG) { bq = ka / p.Bk.kdiv; br = ka - bq * p.Bk.kdiv; }
  const int nn = tid % BN, kn0 = tid / BN;  // N-contiguous loader

  double ra[AN], rb[BREG];

  auto load_chunk = [&](int c) {
    const int64_t kc = kbeg + (int64_t)c * BK;
    {
      const bool kv = (kc + kk) < kend;
      const int64_t coff = aq * p.A.ks1 + ar;
#pragma unroll
      for (int s = 0; s < AN; ++s) {
        const int64_t r = m0 + r0 + s * RSTEP;
        ra[s] = (kv && r < p.M) ? p.A.base[r * p.A.rs + coff] : 0.0;
      }
    }
    if (!B_NCONTIG) {
      const bool kv = (kc + kk) < kend;
      const int64_t coff = bq * p.Bk.ks1 + br;
#pragma unroll
      for (int s = 0; s < BKN; ++s) {
        const int64_t r = n0 + r0 + s * RSTEP;
        rb[s] = (kv && r < p.N) ? p.Bk.base[r * p.Bk.rs + coff] : 0.0;
      }
    } else {
      const int64_t n = n0 + nn;
#pragma unroll
      for (int s = 0; s < BNN; ++s) {
        const int64_t k = kc + kn0 + s * NSTEP;
        rb[s] = (k < kend && n < p.N) ? p.Bn.base[k * p.Bn.ld + n] : 0.0;
      }
    }
  };
  auto advance = [&]() {
    ar += BK;
    while (ar >= p.A.kdiv) { ar -= p.A.kdiv; ++aq; }
    if (!B_NCONTIG) {
      br += BK;
      while (br >= p.Bk.kdiv) { br -= p.Bk.kdiv; ++bq; }
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int s = 0; s < AN; ++s) As[buf][kk * LDA + r0 + s * RSTEP] = ra[s];
    if (!B_NCONTIG) {
#pragma unroll
      for (int s = 0; s < BKN; ++s) Bs[buf][kk * LDB + r0 + s * RSTEP] = rb[s];
    } else {
#pragma unroll
      for (int s = 0; s < BNN; ++s) Bs[buf][(kn0 + s * NSTEP) * LDB + nn] = rb[s];
    }
  };

  dbl4 acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  if (nchunks > 0) {
    load_chunk(0);
    advance();
    store_chunk(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      if (c + 1 < nchunks) { load_chunk(c + 1); advance(); }
      const double* as = As[buf];
      const double* bs = Bs[buf];
#pragma unroll
      for (int k4 = 0; k4 < BK; k4 += 4) {
        const int kr = k4 + (lane >> 4);
        double a[MI], b[NI];
#pragma unroll
        for (int i = 0; i < MI; ++i) a[i] = as[kr * LDA + wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < NI; ++j) b[j] = bs[kr * LDB + wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      if (c + 1 < nchunks) store_chunk(buf ^ 1);
      __syncthreads();
    }
  }

  double* C = p.C + (int64_t)z * p.split_stride;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * WTM + i * 16 + 4 * r + (lane >> 4);
        const int64_t n = n0 + wn * WTN + j * 16 + (lane & 15);
        if (m < p.M && n < p.N) C[m * p.ldc + n] = acc[i][j][r];
      }
}

}  // namespace rimp2
