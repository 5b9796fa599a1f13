// FP64 MFMA GEMM for gfx950 (CDNA4): C[m, n] = sum_k A(m, k) B(k, n).
//
// Every dense contraction of the RI-MP2 fragment kernel is one of these:
//   (ia|jb) slab   V[(k,a), (j,b)] = sum_P B[(k,a), P] B[(j,b), P]    (B K-contiguous)
//   Gamma          G[(k,a), P]     = sum_(j,b) T[(k,a), (j,b)] B[(j,b), P] (B N-contiguous)
//   P_ab           sum_(k,j,c) T(a, (k,j,c)) X(b, (k,j,c))                (B K-contiguous)
//   P_ij           sum_(k,a,b) T(i, (k,a,b)) X(j, (k,a,b))                (B K-contiguous)
//   Gamma, transposed blocks (symmetric pair path)
//                  G[(j,b), P]    += sum_(k,a) T[(k,a), (j,b)] B[(k,a), P]
//                                 (A M-contiguous, B N-contiguous)
// and the adjacent gradient steps: the AO back-transform of Gamma (A
// M-contiguous: transposed MO coefficients) and the L' / L'' terms.
// The slab operands store the reduction index in two levels (runs of kdiv
// contiguous elements, runs ks1 apart), which the loaders follow directly so
// no operand is ever copied or transposed in HBM.
//
// Tiling: 256 threads = 4 waves in a 2 x 2 grid; each wave owns a
// (BM/2) x (BN/2) block of 16 x 16 accumulators fed by
// v_mfma_f64_16x16x4f64.  Lane layout of that instruction on gfx950
// (measured): lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator
// register r of lane l holds D[4r + l/16][l%16].  Operand tiles are staged
// k-major in LDS (double-buffered, one barrier per BK chunk).  Global loads
// are 16 bytes (two consecutive reduction indices, or two consecutive columns
// of an N-contiguous operand) when the operands allow it (VEC).  Two loaders:
// the general one (FAST = 0) issues the next chunk's loads before the current
// chunk's MFMAs and stores them to LDS halfway through them, with masks on
// edge tiles; the fast one (FAST = 1, 2; chosen by the host) keeps loads two
// chunks ahead without any branch around them (see gemm_tile).
//
// Triangular launches (TRI): for a symmetric result only tiles with
// tile_m <= tile_n are computed; every element m < n is written at (m, n) and
// (n, m), and elements m > n of diagonal tiles are not written, so the lower
// triangle is always the mirror of the upper one whatever the tile size.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
  KOperand A;           // A when K-contiguous
  NOperand Am;          // A when M-contiguous: element (m, k) at Am.base[k * Am.ld + m]
  KOperand Bk;          // B when K-contiguous
  NOperand Bn;          // B when N-contiguous
  double* C;            // split z writes C + z * split_stride
  int64_t ldc;
  int64_t split_stride;
  int32_t accumulate;   // nonzero: C += A B instead of C = A B (no split-K)
  const int32_t* status;  // nonzero: do nothing
  // Optional pair screening of an (ia|jb) slab: row m belongs to occupied
  // orbital skip_k0 + m / skip_nvir, column n to skip_j0 + n / skip_nvir; a
  // tile whose pairs are all screened out is not computed.  A pair {k, j} is
  // screened out when skip[k * skip_nocc + j] or skip[j * skip_nocc + k] is
  // nonzero (the mask names unordered pairs).
  const uint8_t* skip;
  int32_t skip_nvir, skip_k0, skip_j0, skip_nocc;
  // pair_upper (same row/column to pair mapping): a tile all of whose pairs
  // have pair_lo <= j < k is not computed (their blocks are the transposes of
  // blocks the same launch computes).
  int32_t pair_upper, pair_lo;
};

// True when the tile need not be computed (uniform): every occupied pair it
// touches is screened out, or (pair_upper) has pair_lo <= j < k.
template <int BM, int BN>
__device__ __forceinline__ bool tile_screened(const GemmParams& p, int tm, int tn) {
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  if (p.pair_upper && p.skip_j0 + (min(p.N, n0 + BN) - 1) / p.skip_nvir < p.skip_k0 + m0 / p.skip_nvir &&
      p.skip_j0 + n0 / p.skip_nvir >= p.pair_lo)
    return true;
  if (p.skip == nullptr) return false;
  const int64_t k_lo = m0 / p.skip_nvir, k_hi = (min(p.M, m0 + BM) - 1) / p.skip_nvir;
  const int64_t j_lo = n0 / p.skip_nvir, j_hi = (min(p.N, n0 + BN) - 1) / p.skip_nvir;
  for (int64_t k = k_lo; k <= k_hi; ++k)
    for (int64_t j = j_lo; j <= j_hi; ++j)
      if (p.skip[(p.skip_k0 + k) * p.skip_nocc + p.skip_j0 + j] == 0 &&
          p.skip[(p.skip_j0 + j) * p.skip_nocc + p.skip_k0 + k] == 0)
        return false;
  return true;
}

// Maps the hardware workgroup id to a logical id so that the workgroups one
// XCD runs (dispatch is round-robin over the 8 XCDs) get consecutive logical
// ids, and therefore neighbouring tiles that share operand rows in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int w, int G) {
  const int q = G >> 3, rem = G & 7, x = w & 7;
  return x * q + (x < rem ? x : rem) + (w >> 3);
}

// ROLE gives each contraction its own kernel symbol (profiler names);
// ROLE_GAMMA_T and ROLE_AO also select the M-contiguous A loader.
enum GemmRole { ROLE_INTS = 0, ROLE_GAMMA = 1, ROLE_PAB = 2, ROLE_PIJ = 3, ROLE_GAMMA_T = 4, ROLE_AO = 5,
                ROLE_LTERM = 6 };
// Roles whose A operand is M-contiguous.
constexpr bool role_a_mcontig(int role) { return role == ROLE_GAMMA_T || role == ROLE_AO; }

// Decodes logical tile index t (< tiles of one split) into (tm, tn):
// triangular order (TRI) or groups of group_m m-tiles.
template <bool TRI>
__device__ __forceinline__ void decode_tile(const GemmParams& p, int t, int& tm, int& tn) {
  if (TRI) {
    tm = 0;
    while (t >= p.tiles_m - tm) { t -= p.tiles_m - tm; ++tm; }
    tn = tm + t;
  } else {
    const int gsz = p.group_m * p.tiles_n;
    const int grp = t / gsz;
    const int first_m = grp * p.group_m;
    const int gm = min(p.group_m, p.tiles_m - first_m);
    const int tin = t - grp * gsz;
    tm = first_m + tin % gm;
    tn = tin / gm;
  }
}

// Workgroup barrier that orders LDS accesses only: global loads issued before
// it stay in flight across it (a full __syncthreads waits for them).
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int BM, int BN, int BK>
struct GemmLds {
  double a[2][BK * (BM + 2)];
  __attribute__((aligned(16))) double b[2][BK * (BN + 2)];
};

// One output tile (tm, tn) of split z.  Ends with a workgroup barrier, so the
// LDS can be reused by the next tile.
// A_MC: A is M-contiguous (p.Am) and is loaded like an N-contiguous B, two
// consecutive rows m per 16-byte load, into the same k-major LDS layout.
template <int BM, int BN, int BK, bool B_NCONTIG, bool VEC, bool TRI, int FAST, bool A_MC = false>
__device__ __forceinline__ void gemm_tile(const GemmParams& p, int tm, int tn, int z, GemmLds<BM, BN, BK>& lds) {
  static_assert(BM % 32 == 0 && BN % 32 == 0 && BK % 8 == 0, "tile shape");
  typedef double d2 __attribute__((ext_vector_type(2)));

  constexpr int LDA = BM + 2, LDB = BN + 2;
  constexpr int WTM = BM / 2, WTN = BN / 2, MI = WTM / 16, NI = WTN / 16;
  constexpr int KP = BK / 2;                   // k pairs per row (K-contiguous loader)
  constexpr int RSTEP = 256 / KP;              // rows per pass
  static_assert(BM % RSTEP == 0 && BN % RSTEP == 0, "K loader shape");
  constexpr int AN = BM / RSTEP, BKN = BN / RSTEP;
  constexpr int NP = BN / 2;                   // column pairs per k row (N-contiguous loader)
  constexpr int NSTEP = 256 / NP;              // k rows per pass
  constexpr int BNN = B_NCONTIG ? BK / NSTEP : 1;
  static_assert(!B_NCONTIG || (256 % NP == 0 && BK % NSTEP == 0), "N loader shape");
  constexpr int BREG = B_NCONTIG ? BNN : BKN;
  constexpr int MP = BM / 2;                   // row pairs per k row (M-contiguous A loader)
  constexpr int MSTEP = 256 / MP;              // k rows per pass
  constexpr int AMN = A_MC ? BK / MSTEP : 1;
  static_assert(!A_MC || (256 % MP == 0 && BK % MSTEP == 0), "M loader shape");
  constexpr int AREG = A_MC ? AMN : AN;

  auto& As = lds.a;
  auto& Bs = lds.b;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

  const int64_t kbeg = (int64_t)z * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nchunks = (int)((kend - kbeg + BK - 1) / BK);

  // K-contiguous loaders: thread -> rows r0 + s*RSTEP, reduction pair (kk, kk+1)
  const int kk = 2 * (tid % KP), r0 = tid / KP;
  int64_t aq = 0, ar = 0, bq = 0, br = 0;
  if (!A_MC) { const int64_t k = kbeg + kk; aq = k / p.A.kdiv; ar = k - aq * p.A.kdiv; }
  if (!B_NCONTIG) { const int64_t k = kbeg + kk; bq = k / p.Bk.kdiv; br = k - bq * p.Bk.kdiv; }
  // N-contiguous loader: thread -> column pair nn, k rows kn0 + s*NSTEP
  const int nn = 2 * (tid % NP), kn0 = tid / NP;
  // M-contiguous A loader: thread -> row pair mm, k rows km0 + s*MSTEP
  const int mm = 2 * (tid % MP), km0 = tid / MP;
  const bool fullA = (m0 + BM <= p.M), fullB = (n0 + BN <= p.N);

  d2 ra[AREG], rb[BREG];

  // One K-contiguous operand tile: element (row, k) = base[row*rs + (k/kdiv)*ks1 + k%kdiv].
  // (q, r) is this thread's position for k = kc + kk.  With VEC the host has
  // checked that every pair (kk, kk+1) lies in one run and is 16-byte aligned.
  // The masked path steps (q, r) to kk+1 without division.
#define RIMP2_KLOAD(OP, ROW0, NROWS, FULLROWS, Q, R, DST, CNT)                                        \
  {                                                                                                 \
    if (VEC && (FULLROWS) && fullk) {                                                               \
      const double* src = OP.base + ((ROW0) + r0) * OP.rs + (Q) * OP.ks1 + (R);                     \
      const int64_t st = (int64_t)RSTEP * OP.rs;                                                    \
      _Pragma("unroll") for (int s = 0; s < CNT; ++s) DST[s] = *(const d2*)(src + s * st);          \
    } else {                                                                                        \
      const int64_t k0 = kc + kk;                                                                   \
      const int64_t off0 = (Q) * OP.ks1 + (R);                                                      \
      const int64_t off1 = ((R) + 1 < OP.kdiv) ? off0 + 1 : ((Q) + 1) * OP.ks1;                     \
      _Pragma("unroll") for (int s = 0; s < CNT; ++s) {                                             \
        const int64_t row = (ROW0) + r0 + s * RSTEP;                                                \
        const int64_t rb0 = min(row, (NROWS) - 1) * OP.rs;                                          \
        const bool rv = row < (NROWS);                                                              \
        const double v0 = (rv && k0 < kend) ? OP.base[rb0 + off0] : 0.0;                            \
        const double v1 = (rv && k0 + 1 < kend) ? OP.base[rb0 + off1] : 0.0;                        \
        DST[s][0] = v0;                                                                             \
        DST[s][1] = v1;                                                                             \
      }                                                                                             \
    }                                                                                               \
  }
  auto load_chunk = [&](int c) {
    const int64_t kc = kbeg + (int64_t)c * BK;
    const bool fullk = (kc + BK <= kend);
    if constexpr (!A_MC) {
      RIMP2_KLOAD(p.A, m0, p.M, fullA, aq, ar, ra, AN)
    } else {
      const int64_t m = m0 + mm;
      if (VEC && fullA && fullk) {
        const double* src = p.Am.base + (kc + km0) * p.Am.ld + m;
        const int64_t st = (int64_t)MSTEP * p.Am.ld;
#pragma unroll
        for (int s = 0; s < AMN; ++s) ra[s] = *(const d2*)(src + s * st);
      } else {
#pragma unroll
        for (int s = 0; s < AMN; ++s) {
          const int64_t k = kc + km0 + s * MSTEP;
          const double* row = p.Am.base + min(k, kend - 1) * p.Am.ld;
          const double x0 = (k < kend && m < p.M) ? row[m] : 0.0;
          const double x1 = (k < kend && m + 1 < p.M) ? row[m + 1] : 0.0;
          ra[s][0] = x0;
          ra[s][1] = x1;
        }
      }
    }
    if (!B_NCONTIG) {
      RIMP2_KLOAD(p.Bk, n0, p.N, fullB, bq, br, rb, BKN)
    } else {
      const int64_t n = n0 + nn;
      if (VEC && fullB && fullk) {
        const double* src = p.Bn.base + (kc + kn0) * p.Bn.ld + n;
        const int64_t st = (int64_t)NSTEP * p.Bn.ld;
#pragma unroll
        for (int s = 0; s < BNN; ++s) rb[s] = *(const d2*)(src + s * st);
      } else {
#pragma unroll
        for (int s = 0; s < BNN; ++s) {
          const int64_t k = kc + kn0 + s * NSTEP;
          const double* row = p.Bn.base + min(k, kend - 1) * p.Bn.ld;
          const double x0 = (k < kend && n < p.N) ? row[n] : 0.0;
          const double x1 = (k < kend && n + 1 < p.N) ? row[n + 1] : 0.0;
          rb[s][0] = x0;
          rb[s][1] = x1;
        }
      }
    }
    if (!A_MC) {
      ar += BK;
      while (ar >= p.A.kdiv) { ar -= p.A.kdiv; ++aq; }
    }
    if (!B_NCONTIG) {
      br += BK;
      while (br >= p.Bk.kdiv) { br -= p.Bk.kdiv; ++bq; }
    }
  };
#undef RIMP2_KLOAD
  auto store_from = [&](int buf, const d2 (&sa)[AREG], const d2 (&sb)[BREG]) {
    if (!A_MC) {
#pragma unroll
      for (int s = 0; s < AREG; ++s) {
        As[buf][kk * LDA + r0 + s * RSTEP] = sa[s][0];
        As[buf][(kk + 1) * LDA + r0 + s * RSTEP] = sa[s][1];
      }
    } else {
#pragma unroll
      for (int s = 0; s < AREG; ++s) *(d2*)&As[buf][(km0 + s * MSTEP) * LDA + mm] = sa[s];
    }
    if (!B_NCONTIG) {
#pragma unroll
      for (int s = 0; s < BKN; ++s) {
        Bs[buf][kk * LDB + r0 + s * RSTEP] = sb[s][0];
        Bs[buf][(kk + 1) * LDB + r0 + s * RSTEP] = sb[s][1];
      }
    } else {
#pragma unroll
      for (int s = 0; s < BNN; ++s) *(d2*)&Bs[buf][(kn0 + s * NSTEP) * LDB + nn] = sb[s];
    }
  };
  auto store_chunk = [&](int buf) { store_from(buf, ra, rb); };
  // MFMA fragments of k-step ks (4 reduction indices) from LDS buffer buf
  auto read_frag = [&](int buf, int ks, double* a, double* b) {
    const int kr = 4 * ks + (lane >> 4);
#pragma unroll
    for (int i = 0; i < MI; ++i) a[i] = As[buf][kr * LDA + wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < NI; ++j) b[j] = Bs[buf][kr * LDB + wn * WTN + j * 16 + (lane & 15)];
  };

  dbl4 acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  // FAST > 0 (chosen by the host: 16-byte loads, an even reduction length,
  // runs of the K operands at least one chunk long): the split's full chunks
  // go through a branch-free loader that issues each chunk's global loads two
  // chunks ahead into two register sets.  Rows (and N-contiguous column
  // pairs) past the edge of the matrix read the last valid ones, which only
  // reach accumulators that are never stored.  The loads are unconditional
  // (after the last full chunk it is loaded again), so the compiler's wait
  // counts stay exact, and the barriers order LDS only, so the loads stay in
  // flight across them.  Chunk starts advance by uniform run steps; with
  // FAST = 2 (runs shorter than the reduction and not a multiple of the chunk)
  // a thread whose pair lies in the next run adds one run step.  A ragged
  // last chunk is then loaded with per-element masks and run on its own.
  // Every path sums each output element in the same order.
  if constexpr (FAST > 0) {
    const int nfull = (int)((kend - kbeg) / BK);
    if (nfull > 0) {
      d2 xa[2][AREG], xb[2][BREG];
      // start of the next chunk to load (uniform): offset of each K operand
      // and its position in the current run
      int64_t oa = 0, pa = 0, ob = 0, pb = 0;
      if (!A_MC) { const int64_t q = kbeg / p.A.kdiv; pa = kbeg - q * p.A.kdiv; oa = q * p.A.ks1 + pa; }
      else { oa = kbeg * p.Am.ld; }
      if (!B_NCONTIG) { const int64_t q = kbeg / p.Bk.kdiv; pb = kbeg - q * p.Bk.kdiv; ob = q * p.Bk.ks1 + pb; }
      else { ob = kbeg * p.Bn.ld; }
      int nload = 0;
      const double* ap[AREG];
      if (!A_MC) {
#pragma unroll
        for (int s = 0; s < AREG; ++s) ap[s] = p.A.base + min(m0 + r0 + s * RSTEP, p.M - 1) * p.A.rs + kk;
      } else {
        const int64_t m = min(m0 + mm, p.M - 2);   // M is even here
#pragma unroll
        for (int s = 0; s < AREG; ++s) ap[s] = p.Am.base + (int64_t)(km0 + s * MSTEP) * p.Am.ld + m;
      }
      const double* bp[BREG];
      if (!B_NCONTIG) {
#pragma unroll
        for (int s = 0; s < BREG; ++s) bp[s] = p.Bk.base + min(n0 + r0 + s * RSTEP, p.N - 1) * p.Bk.rs + kk;
      } else {
        const int64_t n = min(n0 + nn, p.N - 2);   // N is even here
#pragma unroll
        for (int s = 0; s < BREG; ++s) bp[s] = p.Bn.base + (int64_t)(kn0 + s * NSTEP) * p.Bn.ld + n;
      }
      // this thread's extra offset when its pair lies in the run after the chunk start's
      auto wrap = [&](const KOperand& o, int64_t pos) -> int64_t {
        return (FAST == 2 && pos + kk >= o.kdiv) ? o.ks1 - o.kdiv : 0;
      };
      auto fload = [&](d2 (&da)[AREG], d2 (&db)[BREG]) {
        const int64_t xa_ = A_MC ? oa : oa + wrap(p.A, pa);
#pragma unroll
        for (int s = 0; s < AREG; ++s) da[s] = *(const d2*)(ap[s] + xa_);
        const int64_t xb_ = B_NCONTIG ? ob : ob + wrap(p.Bk, pb);
#pragma unroll
        for (int s = 0; s < BREG; ++s) db[s] = *(const d2*)(bp[s] + xb_);
        if (++nload < nfull) {
          if (A_MC) {
            oa += (int64_t)BK * p.Am.ld;
          } else {
            oa += BK; pa += BK;
            if (pa >= p.A.kdiv) { pa -= p.A.kdiv; oa += p.A.ks1 - p.A.kdiv; }
          }
          if (B_NCONTIG) {
            ob += (int64_t)BK * p.Bn.ld;
          } else {
            ob += BK; pb += BK;
            if (pb >= p.Bk.kdiv) { pb -= p.Bk.kdiv; ob += p.Bk.ks1 - p.Bk.kdiv; }
          }
        }
      };
      fload(xa[0], xb[0]);
      fload(xa[1], xb[1]);
      store_from(0, xa[0], xb[0]);
      lds_sync();
      // chunk c (c % 2 == S) from LDS buffer S; chunk c+1 waits in register set S^1
      auto step = [&](int c, auto set) {
        constexpr int S = decltype(set)::value;
        const bool more = c + 1 < nfull;
        fload(xa[S], xb[S]);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
          if (ks == BK / 8 && more) store_from(S ^ 1, xa[S ^ 1], xb[S ^ 1]);
          double a[MI], b[NI];
          read_frag(S, ks, a, b);
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        lds_sync();
      };
      int c = 0;
      for (; c + 1 < nfull; c += 2) {
        step(c, std::integral_constant<int, 0>{});
        step(c + 1, std::integral_constant<int, 1>{});
      }
      if (c < nfull) step(c, std::integral_constant<int, 0>{});
    }
    if (nfull < nchunks) {
      // the ragged last chunk: per-element masks (pairs, as the reduction length is even)
      const int64_t kt = kbeg + (int64_t)nfull * BK;
      const d2 zero = {0.0, 0.0};
      if (!A_MC) {
        const int64_t k = kt + kk;
        const bool in = k < kend;
        const int64_t q = in ? k / p.A.kdiv : 0;
        const int64_t off = in ? q * p.A.ks1 + (k - q * p.A.kdiv) : 0;
#pragma unroll
        for (int s = 0; s < AREG; ++s)
          ra[s] = in ? *(const d2*)(p.A.base + min(m0 + r0 + s * RSTEP, p.M - 1) * p.A.rs + off) : zero;
      } else {
        const int64_t m = min(m0 + mm, p.M - 2);
#pragma unroll
        for (int s = 0; s < AREG; ++s) {
          const int64_t k = kt + km0 + s * MSTEP;
          ra[s] = k < kend ? *(const d2*)(p.Am.base + k * p.Am.ld + m) : zero;
        }
      }
      if (!B_NCONTIG) {
        const int64_t k = kt + kk;
        const bool in = k < kend;
        const int64_t q = in ? k / p.Bk.kdiv : 0;
        const int64_t off = in ? q * p.Bk.ks1 + (k - q * p.Bk.kdiv) : 0;
#pragma unroll
        for (int s = 0; s < BREG; ++s)
          rb[s] = in ? *(const d2*)(p.Bk.base + min(n0 + r0 + s * RSTEP, p.N - 1) * p.Bk.rs + off) : zero;
      } else {
        const int64_t n = min(n0 + nn, p.N - 2);
#pragma unroll
        for (int s = 0; s < BREG; ++s) {
          const int64_t k = kt + kn0 + s * NSTEP;
          rb[s] = k < kend ? *(const d2*)(p.Bn.base + k * p.Bn.ld + n) : zero;
        }
      }
      store_chunk(0);
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        double a[MI], b[NI];
        read_frag(0, ks, a, b);
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
  } else if (nchunks > 0) {
    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      const bool more = c + 1 < nchunks;
      if (more) load_chunk(c + 1);
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        if (ks == BK / 8 && more) store_chunk(buf ^ 1);
        double a[MI], b[NI];
        read_frag(buf, ks, a, b);
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
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
        if (m < p.M && n < p.N) {
          if (!TRI) {
            if (p.accumulate) C[m * p.ldc + n] += acc[i][j][r];
            else C[m * p.ldc + n] = acc[i][j][r];
          } else if (m <= n) {   // every lower element is the mirror of an upper one
            C[m * p.ldc + n] = acc[i][j][r];
            if (m < n) C[n * p.ldc + m] = acc[i][j][r];
          }
        }
      }
}


// One workgroup per (split, tile); the hardware id is remapped XCD-aware.
template <int BM, int BN, int BK, bool B_NCONTIG, int ROLE, bool VEC, bool TRI, int FAST = 0>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(GemmParams p) {
  if (p.status != nullptr && *p.status != 0) return;
  __shared__ GemmLds<BM, BN, BK> lds;
  const int wl = xcd_remap(blockIdx.x, gridDim.x);
  const int ntiles = TRI ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  const int z = wl / ntiles;
  int tm, tn;
  decode_tile<TRI>(p, wl - z * ntiles, tm, tn);
  if (tile_screened<BM, BN>(p, tm, tn)) return;
  gemm_tile<BM, BN, BK, B_NCONTIG, VEC, TRI, FAST, role_a_mcontig(ROLE)>(p, tm, tn, z, lds);
}

// Persistent grouped launch over many independent GEMMs (one per fragment):
// problem f owns work items [prefix[f], prefix[f+1]) = its tiles x splits,
// problems ordered largest first.  Each workgroup takes items from *counter
// (which must be zero at launch) until all are taken; no workgroup waits on
// another, so every one exits.
struct GemmGroup {
  const GemmParams* probs;
  const int64_t* prefix;   // [nprob + 1]
  int32_t nprob;
  unsigned long long* counter;
};

template <int BM, int BN, int BK, bool B_NCONTIG, int ROLE, bool VEC, bool TRI, int FAST = 0>
__global__ __launch_bounds__(256, 2) void gemm_f64_grouped(GemmGroup G) {
  __shared__ GemmLds<BM, BN, BK> lds;
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
    const GemmParams p = G.probs[lo];
    if (p.status != nullptr && *p.status != 0) continue;
    const int u = (int)(t - G.prefix[lo]);
    const int ntiles = TRI ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
    const int z = u / ntiles;
    int tm, tn;
    decode_tile<TRI>(p, u - z * ntiles, tm, tn);
    if (tile_screened<BM, BN>(p, tm, tn)) continue;
    gemm_tile<BM, BN, BK, B_NCONTIG, VEC, TRI, FAST>(p, tm, tn, z, lds);
  }
}

}  // namespace rimp2
