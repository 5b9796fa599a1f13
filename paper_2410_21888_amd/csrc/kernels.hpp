// Memory-bound kernels of the RI-MP2 fragment path (gfx950): orbital-energy
// gap check, the amplitude pass (denominators, amplitudes, T = 2X - X^T and
// pair energies), ordered split-K reduction and the compensated energy sum.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rimp2 {

// Error-free transformations (Knuth's TwoSum, Dekker's FastTwoSum).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  e = b - (s - a);
}
// (ah, al) += (bh, bl), double-double addition with both error terms kept.
__device__ __forceinline__ void dd_add(double& ah, double& al, double bh, double bl) {
  double s, e, t, f;
  two_sum(ah, bh, s, e);
  two_sum(al, bl, t, f);
  e += t;
  fast_two_sum(s, e, s, e);
  e += f;
  fast_two_sum(s, e, ah, al);
}

// Fixed-order double-double reduction over the 256 threads of a workgroup.
__device__ __forceinline__ void block_dd_reduce(double& hi, double& lo) {
  __shared__ double sh[256], sl[256];
  const int t = threadIdx.x;
  sh[t] = hi;
  sl[t] = lo;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      double h = sh[t], l = sl[t];
      dd_add(h, l, sh[t + w], sl[t + w]);
      sh[t] = h;
      sl[t] = l;
    }
    __syncthreads();
  }
  hi = sh[0];
  lo = sl[0];
  __syncthreads();
}

// status = RIMP2_EGAP (-5) unless every denominator
// ((eps_i + eps_j) - eps_a) - eps_b is negative.  FP addition is monotone, so
// it is enough that the largest one, built from max eps_occ and min eps_vir
// in the same order, is negative.  A NaN anywhere also fails.  One workgroup.
__device__ __forceinline__ void gap_check_block(const double* eo, int nocc, const double* ev, int nvir,
                                                int32_t* status) {
  __shared__ double smax[256], smin[256];
  __shared__ int snan[256];
  const int t = threadIdx.x;
  double mx = -__builtin_inf(), mn = __builtin_inf();
  int bad = 0;
  for (int i = t; i < nocc; i += 256) { const double v = eo[i]; bad |= (v != v); mx = fmax(mx, v); }
  for (int a = t; a < nvir; a += 256) { const double v = ev[a]; bad |= (v != v); mn = fmin(mn, v); }
  smax[t] = mx; smin[t] = mn; snan[t] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      smax[t] = fmax(smax[t], smax[t + w]);
      smin[t] = fmin(smin[t], smin[t + w]);
      snan[t] |= snan[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double d = ((smax[0] + smax[0]) - smin[0]) - smin[0];
    status[0] = (snan[0] || !(d < 0.0)) ? -5 : 0;
  }
}

__global__ __launch_bounds__(256) void gap_check_kernel(const double* eo, int nocc, const double* ev, int nvir,
                                                        int32_t* status) {
  gap_check_block(eo, nocc, ev, nvir, status);
}

// LDS-only workgroup barrier: orders LDS accesses across the workgroup but,
// unlike __syncthreads, does not wait for outstanding global loads, so the
// next tile's prefetch stays in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Tile pairs (ta <= tb) of an nt x nt tile grid in row order: q -> (ta, tb).
__device__ __forceinline__ void tile_pair_at(int q, int nt, int& ta, int& tb) {
  ta = 0;
  while (q >= nt - ta) { q -= nt - ta; ++ta; }
  tb = ta + q;
}
__device__ __forceinline__ void tile_pair_next(int nt, int& ta, int& tb) {
  if (++tb == nt) { ++ta; tb = ta; }
}

// Writes a workgroup's pair-energy sum: to its (hi, lo) partial slot when the
// pair is split over several workgroups (epart), else to e_kj (and e_jk).
__device__ __forceinline__ void put_pair_energy(double sh, double sl, double* e_pair, int nocc, int k, int j,
                                                bool mirror, double* epart) {
  double h, l;
  fast_two_sum(sh, sl, h, l);
  block_dd_reduce(h, l);
  if (threadIdx.x == 0) {
    if (epart) {
      epart[0] = h;
      epart[1] = l;
    } else {
      e_pair[(int64_t)k * nocc + j] = h + l;
      if (mirror) e_pair[(int64_t)j * nocc + k] = h + l;
    }
  }
}

constexpr int AT = 32;

// Pair (k, j > k) of a slab group k0.. whose slab holds both rows k and j
// and both columns k and j (columns j0 .. j0+ncols-1, j0 <= k), and whose
// block (j, k) was not computed:
// V_jk is V_kj transposed, and D_jk = D_kj, so this workgroup forms both
// pairs from V_kj alone.  For positions (a, b) and (b, a) of the block:
//   X_kj[a,b] = V_kj[a,b] / D[a,b]    X_kj[b,a] = V_kj[b,a] / D[b,a]
//   X_jk[a,b] = V_kj[b,a] / D[a,b]    X_jk[b,a] = V_kj[a,b] / D[b,a]
// with D[a,b] = ((eps_k + eps_j) - eps_a) - eps_b, T = 2X - X^T for each
// pair, X written over V and T to the T slab in both blocks, and
// e_kj = sum_ab T_kj V_kj (compensated) written to e_kj and e_jk.  The
// workgroup covers tile pairs [q0, q1) of the block.  VP and VQ are two
// AT x (AT+1) LDS tiles of the caller.
__device__ __forceinline__ void amplitude_mirror_block(double* S, double* Tslab, const double* eo, const double* ev,
                                                       int nocc, int nvir, bool skip, double* e_pair, int k0, int j0,
                                                       int ncols, int k, int j, int q0, int q1, double* epart,
                                                       double (*VP)[AT + 1], double (*VQ)[AT + 1]) {
  const int64_t ld = (int64_t)ncols * nvir;
  double* bkj = S + ((int64_t)(k - k0) * nvir * ncols + (j - j0)) * nvir;  // element (a,b) of pair (k,j) at bkj[a*ld + b]
  double* bjk = S + ((int64_t)(j - k0) * nvir * ncols + (k - j0)) * nvir;
  double* tkj = Tslab + ((int64_t)(k - k0) * nvir * ncols + (j - j0)) * nvir;
  double* tjk = Tslab + ((int64_t)(j - k0) * nvir * ncols + (k - j0)) * nvir;
  const double ekj = eo[k] + eo[j];
  const int t = threadIdx.x, tc = t & 31, tr0 = t >> 5;
  const int nt = (nvir + AT - 1) / AT;
  double sh = 0.0, sl = 0.0;
  // one element position (a, b) given v = V_kj[a,b] and w = V_kj[b,a]
  auto put = [&](int a, int b, double v, double w) {
    const double dab = (ekj - ev[a]) - ev[b], dba = (ekj - ev[b]) - ev[a];
    const double xkj = v / dab, xkj_t = w / dba, xjk = w / dab, xjk_t = v / dba;
    const double t1 = 2.0 * xkj - xkj_t, t2 = 2.0 * xjk - xjk_t;
    double p = t1 * v, e;
    two_sum(sh, p, sh, e);
    sl += e;
    const int64_t o = (int64_t)a * ld + b;
    bkj[o] = xkj; tkj[o] = t1;
    bjk[o] = xjk; tjk[o] = t2;
  };
  double nP[4], nQ[4];
  auto fetch = [&](int ta, int tb) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = tr0 + 8 * s;
      const int a = ta * AT + r, b = tb * AT + tc, a2 = tb * AT + r, b2 = ta * AT + tc;
      nP[s] = (!skip && a < nvir && b < nvir) ? bkj[(int64_t)a * ld + b] : 0.0;
      nQ[s] = (!skip && ta != tb && a2 < nvir && b2 < nvir) ? bkj[(int64_t)a2 * ld + b2] : 0.0;
    }
  };
  int ta = 0, tb = 0;
  tile_pair_at(q0, nt, ta, tb);
  if (q0 < q1) fetch(ta, tb);
  for (int q = q0; q < q1; ++q) {
    double vP[4], vQ[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) { vP[s] = nP[s]; vQ[s] = nQ[s]; }
    const int cta = ta, ctb = tb;
    const bool diag = (cta == ctb);
    tile_pair_next(nt, ta, tb);
    if (q + 1 < q1) fetch(ta, tb);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = tr0 + 8 * s;
      VP[r][tc] = vP[s];
      VQ[r][tc] = vQ[s];
    }
    lds_barrier();
#pragma unroll 1
    for (int s = 0; s < 4; ++s) {
      const int r = tr0 + 8 * s;
      const int a = cta * AT + r, b = ctb * AT + tc;
      if (a < nvir && b < nvir) put(a, b, vP[s], diag ? VP[tc][r] : VQ[tc][r]);
      const int a2 = ctb * AT + r, b2 = cta * AT + tc;
      if (!diag && a2 < nvir && b2 < nvir) put(a2, b2, vQ[s], VP[tc][r]);
    }
    lds_barrier();
  }
  put_pair_energy(sh, sl, e_pair, nocc, k, j, true, epart);
}

// Amplitude pass over one slab group.
// V/X slab: element (kk, a, jj, b) at S[((kk*nvir + a)*ncols + jj)*nvir + b],
// kk < g, jj < ncols, occupied pair (k, j) = (k0 + kk, j0 + jj).
// Each pair's nvir x nvir block is covered by W workgroups (w < W), each
// taking a contiguous range of its 32 x 32 tile pairs (ta <= tb); with W > 1
// the workgroups write (hi, lo) partial sums to epart[2 (p W + w)] for
// pair_energy_reduce_kernel (p = kk * ncols + jj), else e_pair directly.
// For each tile pair a workgroup reads V at (a,b) and (b,a), forms
// X = V / D with D[a,b] = ((eps_k + eps_j) - eps_a) - eps_b in that order (so
// X^T uses D[b,a] rounded its own way), then T = 2X - X^T, writes X over V
// and T to the T slab (unless energy_only), and accumulates
// e_kj = sum_ab T[a,b] V[a,b] with compensated per-thread sums and a fixed
// reduction order.  The next tile pair's V is fetched before the current one
// is processed.
// sym = 1 (energy only, slab holding j >= k0 only): pairs with j < k are left
// to their mirror and e_kj is written to both e_kj and e_jk (e_ij = e_ji).
// sym = 2 (slab group k0..k0+g-1 over every column, j0 = 0): a pair whose
// second orbital is also in the group is paired with its mirror; the
// (ia|jb) GEMM has not computed the blocks j < k of those pairs, which are
// left to their mirror, and pairs j > k form both blocks
// (amplitude_mirror_block; with energy_only as sym = 1).  Other pairs are
// formed on their own.
// sym = 3 (Gamma without P, slab holding j >= k0 only): pairs inside the
// group as with sym = 2 (both blocks from the block j > k); a pair with j
// past the group forms its own block only (its transpose block T_jk = T_kj^T
// is never formed: the transposed Gamma GEMM reads T_kj instead), and e_kj is
// written to both e_kj and e_jk.
// A screened pair (pair_skip, may be null) writes e = 0 (and, unless
// energy_only, zero X and T) without reading V.
__device__ __forceinline__ bool pair_mirrored(int sym, int k0, int g, int j) {
  return sym == 1 || sym == 3 || (sym == 2 && j >= k0 && j < k0 + g);
}

__device__ __forceinline__ void amplitude_block(double* S, double* Tslab, const double* eo, const double* ev, int nocc,
                                                int nvir, int k0, int j0, int ncols, int sym, int g, int energy_only,
                                                const uint8_t* pair_skip, double* e_pair, int kk, int jj, int w,
                                                int W, double* epart_all) {
  __shared__ double XP[AT][AT + 1], XQ[AT][AT + 1];   // also the mirror path's V tiles
  const int k = k0 + kk, j = j0 + jj;
  const bool paired = pair_mirrored(sym, k0, g, j);
  if (paired && j < k) return;
  double* epart = (W > 1) ? epart_all + 2 * (((int64_t)kk * ncols + jj) * W + w) : nullptr;
  const int64_t ld = (int64_t)ncols * nvir;
  double* blk = S + ((int64_t)kk * nvir * ncols + jj) * nvir;  // element (a,b) at blk[a*ld + b]
  double* tblk = Tslab + ((int64_t)kk * nvir * ncols + jj) * nvir;
  // the mask names unordered pairs: either entry screens the pair out
  const bool skip = pair_skip != nullptr &&
                    (pair_skip[(int64_t)k * nocc + j] != 0 || pair_skip[(int64_t)j * nocc + k] != 0);
  const int nt = (nvir + AT - 1) / AT, npt = nt * (nt + 1) / 2;
  const int q0 = (int)((int64_t)npt * w / W), q1 = (int)((int64_t)npt * (w + 1) / W);
  if ((sym == 2 || sym == 3) && j >= k0 && j < k0 + g && !energy_only && j > k) {
    amplitude_mirror_block(S, Tslab, eo, ev, nocc, nvir, skip, e_pair, k0, j0, ncols, k, j, q0, q1, epart, XP, XQ);
    return;
  }
  if (skip && energy_only) {
    put_pair_energy(0.0, 0.0, e_pair, nocc, k, j, paired, epart);
    return;
  }
  const double ekj = eo[k] + eo[j];
  const int t = threadIdx.x, tc = t & 31, tr0 = t >> 5;  // 8 rows x 32 cols per pass
  double sh = 0.0, sl = 0.0;
  double nP[4], nQ[4];
  auto fetch = [&](int ta, int tb) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = tr0 + 8 * s;
      const int a = ta * AT + r, b = tb * AT + tc;   // tile P element (a, b)
      const int a2 = tb * AT + r, b2 = ta * AT + tc; // tile Q element (a2, b2)
      nP[s] = (!skip && a < nvir && b < nvir) ? blk[(int64_t)a * ld + b] : 0.0;
      nQ[s] = (!skip && ta != tb && a2 < nvir && b2 < nvir) ? blk[(int64_t)a2 * ld + b2] : 0.0;
    }
  };
  int ta = 0, tb = 0;
  tile_pair_at(q0, nt, ta, tb);
  if (q0 < q1) fetch(ta, tb);
  for (int q = q0; q < q1; ++q) {
    const int cta = ta, ctb = tb;
    const bool diag = (cta == ctb);
    double vP[4], vQ[4], xP[4], xQ[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) { vP[s] = nP[s]; vQ[s] = nQ[s]; }
    tile_pair_next(nt, ta, tb);
    if (q + 1 < q1) fetch(ta, tb);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = tr0 + 8 * s;
      const int a = cta * AT + r, b = ctb * AT + tc;
      const int a2 = ctb * AT + r, b2 = cta * AT + tc;
      double x = 0.0;
      if (a < nvir && b < nvir) x = vP[s] / ((ekj - ev[a]) - ev[b]);
      xP[s] = x; XP[r][tc] = x;
      x = 0.0;
      if (!diag && a2 < nvir && b2 < nvir) x = vQ[s] / ((ekj - ev[a2]) - ev[b2]);
      xQ[s] = x; XQ[r][tc] = x;
    }
    lds_barrier();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = tr0 + 8 * s;
      const int a = cta * AT + r, b = ctb * AT + tc;
      const double xt = diag ? XP[tc][r] : XQ[tc][r];   // X[b, a]
      const double tv = 2.0 * xP[s] - xt;
      if (a < nvir && b < nvir) {
        double p = tv * vP[s], e;
        two_sum(sh, p, sh, e);
        sl += e;
        if (!energy_only) { blk[(int64_t)a * ld + b] = xP[s]; tblk[(int64_t)a * ld + b] = tv; }
      }
      if (!diag) {
        const int a2 = ctb * AT + r, b2 = cta * AT + tc;
        const double xt2 = XP[tc][r];
        const double tv2 = 2.0 * xQ[s] - xt2;
        if (a2 < nvir && b2 < nvir) {
          double p = tv2 * vQ[s], e;
          two_sum(sh, p, sh, e);
          sl += e;
          if (!energy_only) { blk[(int64_t)a2 * ld + b2] = xQ[s]; tblk[(int64_t)a2 * ld + b2] = tv2; }
        }
      }
    }
    lds_barrier();
  }
  put_pair_energy(sh, sl, e_pair, nocc, k, j, paired, epart);
}

// One workgroup per (pair, w): blockIdx.x = (kk * ncols + jj) * W + w.
__global__ __launch_bounds__(256) void amplitude_kernel(double* S, double* Tslab, const double* eo, const double* ev,
                                                        int nocc, int nvir, int k0, int j0, int ncols, int sym, int g,
                                                        int energy_only, const uint8_t* pair_skip, double* e_pair,
                                                        int W, double* epart, const int32_t* status) {
  if (*status != 0) return;
  const int p = blockIdx.x / W, w = blockIdx.x - p * W;
  const int kk = p / ncols, jj = p - kk * ncols;
  amplitude_block(S, Tslab, eo, ev, nocc, nvir, k0, j0, ncols, sym, g, energy_only, pair_skip, e_pair, kk, jj, w, W,
                  epart);
}

// e_kj from the W partial sums of each pair of a slab group (double-double,
// added in order w = 0, 1, ...); for a pair paired with its mirror (see
// amplitude_block) also e_jk.  One thread per pair.
__global__ __launch_bounds__(256) void pair_energy_reduce_kernel(const double* epart, int W, int nocc, int k0, int j0,
                                                                 int g, int ncols, int sym, double* e_pair,
                                                                 const int32_t* status) {
  if (*status != 0) return;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= (int64_t)g * ncols) return;
  const int kk = (int)(p / ncols), jj = (int)(p - (int64_t)kk * ncols);
  const int k = k0 + kk, j = j0 + jj;
  const bool paired = pair_mirrored(sym, k0, g, j);
  if (paired && j < k) return;
  double h = 0.0, l = 0.0;
  for (int w = 0; w < W; ++w) dd_add(h, l, epart[2 * (p * W + w)], epart[2 * (p * W + w) + 1]);
  e_pair[(int64_t)k * nocc + j] = h + l;
  if (paired) e_pair[(int64_t)j * nocc + k] = h + l;
}

// out[m*ldo + n] = (accumulate ? out : 0) + alpha * sum_{z < splits} W[z*zs + m*ldw + n],
// summed in increasing z.
__device__ __forceinline__ void splitk_reduce_at(double* out, int64_t ldo, const double* W, int64_t ldw, int64_t zs,
                                                 int splits, int64_t M, int64_t N, double alpha, int accumulate,
                                                 int64_t idx) {
  if (idx >= M * N) return;
  const int64_t m = idx / N, n = idx - m * N;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += W[z * zs + m * ldw + n];
  double* o = out + m * ldo + n;
  *o = (accumulate ? *o : 0.0) + alpha * s;
}

__global__ __launch_bounds__(256) void splitk_reduce_kernel(double* out, int64_t ldo, const double* W, int64_t ldw,
                                                            int64_t zs, int splits, int64_t M, int64_t N, double alpha,
                                                            int accumulate, const int32_t* status) {
  if (*status != 0) return;
  splitk_reduce_at(out, ldo, W, ldw, zs, splits, M, N, alpha, accumulate, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// E = sum of count values, compensated, fixed order; writes (hi, lo).
__device__ __forceinline__ void energy_sum_block(const double* e, int64_t count, double* E) {
  double sh = 0.0, sl = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) {
    double s, err;
    two_sum(sh, e[i], s, err);
    sh = s;
    sl += err;
  }
  double h, l;
  fast_two_sum(sh, sl, h, l);
  block_dd_reduce(h, l);
  if (threadIdx.x == 0) {
    double hi, lo;
    fast_two_sum(h, l, hi, lo);
    E[0] = hi;
    E[1] = lo;
  }
}

__global__ __launch_bounds__(256) void energy_sum_kernel(const double* e, int64_t count, double* E,
                                                         const int32_t* status) {
  if (*status != 0) return;
  energy_sum_block(e, count, E);
}

// status_out[idx] = *status (per-fragment status of a batch).
__global__ void copy_status_kernel(const int32_t* status, int32_t* status_out, int idx) {
  if (threadIdx.x == 0) status_out[idx] = *status;
}

}  // namespace rimp2
