// Host side of the C ABI declared in include/rimp2.h: argument checks,
// workspace planning and the launch sequence of the RI-MP2 fragment kernel.
//
// Path for one fragment (all on the caller's stream, no host synchronisation):
//   gap check -> for each slab group of g occupied orbitals k0..k0+g-1:
//     (ia|jb) slab GEMM  V[(k,a),(j,b)] = sum_P B[k,a,P] B[j,b,P]       (Eq. MP2_ints)
//     amplitude pass     X = V/D, T = 2X - X^T, e_kj = sum T V           (Appendix, X)
//     Gamma GEMM         Gamma[k,a,P] = sum_(j,b) T[k,a,j,b] B[j,b,P]    (Appendix, Gamma)
//     P_ab GEMM          P_ab += sum_(k,j,c) T[k,a,j,c] X[k,b,j,c]       (Appendix, D_ab)
//     P_ij GEMM          P_ij -= sum_(k,a,b) T[k,a,i,b] X[k,a,j,b]       (Appendix, D_ij)
//   -> compensated E = sum e_ij.
// Slab layout [kk][a][j][b]: the (ia|jb) and Gamma GEMMs see plain row-major
// matrices; P_ab and P_ij read the same slabs with a two-level reduction index.
// P_ab and P_ij are symmetric, so their GEMMs compute upper-triangular tiles
// and write each also transposed.  For P_ij every slab's contribution is
// symmetric.  For P_ab only the sum over both orders of each pair is
// (T_kj X_kj^T + T_jk X_jk^T = 2(X X^T + X^T X) - (X X + (X X)^T) with
// X = X_kj), so the mirrored partials of a slab group are not its own lower
// triangle; but the mirror of a sum is the sum of the mirrors, and the total
// over all groups is symmetric, so the accumulated lower triangle is exact.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/rimp2.h"
#include "../../include/rimp2_gradient.h"
#include "common.hpp"
#include "gemm_f64.hpp"
#include "kernels.hpp"
#include "split_int8.hpp"
#include "batch.hpp"

using namespace rimp2;

// Scratch space of rimp2_fragment_noalloc: one array per GPU, part of the
// library's code object, so each device that runs the library holds its own
// copy until the process ends.  Host code never uses the name `scratch` as an
// address: rimp2_fragment_noalloc takes the device address from
// hipGetSymbolAddress once per device (with that device current) and passes
// it to the kernels as the workspace.
constexpr size_t kScratchBytes = (size_t)RIMP2_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {


// ---- kernel timing -------------------------------------------------------
enum Role { R_GAP, R_INTS, R_AMP, R_GAMMA, R_PAB, R_PIJ, R_REDUCE, R_ESUM, R_STATUS, R_SPLIT, R_INTS8, R_GAMMA8,
            R_GAMMA_T, R_GAMMA_AO, R_LTERM, R_RESPONSE, R_GAMMA_T8, R_NROLES };
const char* const kRoleName[R_NROLES] = {"gap_check",  "ints_gemm",     "amplitude",  "gamma_gemm",
                                         "pab_gemm",   "pij_gemm",      "splitk_reduce", "energy_sum",
                                         "status_copy", "digit_split", "ints_oz8",   "gamma_oz8",
                                         "gamma_t_gemm", "gamma_ao_gemm", "l_terms_gemm", "response",
                                         "gamma_t_oz8"};
struct TraceRec {
  int role;
  hipEvent_t e0, e1;
  double af, ef, ab;
};
struct Tracer {
  std::mutex mu;
  bool on = false;
  std::vector<TraceRec> recs;
  std::vector<hipEvent_t> pool;
};
Tracer& tracer() {
  static Tracer t;
  return t;
}

// Set while this thread runs rimp2_fragment_noalloc: no events are created
// or recorded (that entry point allocates nothing).
thread_local bool t_noalloc = false;

// Launches `launch` on stream st; while timing is on, brackets it with events.
template <class F>
int traced(int role, double af, double ef, double ab, hipStream_t st, F&& launch) {
  Tracer& T = tracer();
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool on;
  {
    std::lock_guard<std::mutex> lk(T.mu);
    on = T.on && !t_noalloc;
    for (int i = 0; on && i < 2; ++i) {
      if (!T.pool.empty()) {
        ev[i] = T.pool.back();
        T.pool.pop_back();
      } else {
        HIP_TRY(hipEventCreate(&ev[i]));
      }
    }
  }
  if (on) HIP_TRY(hipEventRecord(ev[0], st));
  launch();
  HIP_TRY(hipGetLastError());
  if (on) {
    HIP_TRY(hipEventRecord(ev[1], st));
    std::lock_guard<std::mutex> lk(T.mu);
    T.recs.push_back(TraceRec{role, ev[0], ev[1], af, ef, ab});
  }
  return RIMP2_OK;
}

constexpr size_t kAlign = 256;
constexpr int64_t kTile = 128;        // M/N tile of the large GEMMs
constexpr int64_t kSmallTile = 64;    // tile of the P_ij GEMM
constexpr int kBK = 16;
constexpr int64_t kSlots = 512;       // resident GEMM workgroups: 2 per CU on 256 CUs

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// A dispatch's grid size is a 32-bit count of work-items (workgroups x 256 here).
constexpr int64_t kMaxWorkgroups = 0xffffffffLL / 256;
int check_grid(int64_t wgs, const char* what) {
  if (wgs <= 0 || wgs > kMaxWorkgroups)
    return fail(RIMP2_EINVAL, "%s grid of %lld workgroups is out of range (1..%lld)", what, (long long)wgs,
                (long long)kMaxWorkgroups);
  return RIMP2_OK;
}
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Split-K factor for a launch of `tiles` output tiles over reduction length K:
// the factor (at most 64, each split at least 2048 long) whose workgroup count
// best fills whole waves of kSlots workgroups.  Launches of eight or more
// full waves split at most 4 ways, only to fill a ragged last wave (4653
// tiles run 9.09 waves unsplit, 9.83 of every 10 slots used with 4 splits).
int64_t choose_splits(int64_t tiles, int64_t K) {
  const bool big = tiles >= 8 * kSlots;
  int64_t smax = std::max<int64_t>(1, std::min<int64_t>(64, K / 2048));
  if (big) smax = std::min<int64_t>(smax, 4);
  int64_t best = 1;
  double best_eff = -1.0;
  for (int64_t s = 1; s <= smax; ++s) {
    const int64_t total = tiles * s;
    const double waves = (double)cdiv(total, kSlots);
    // fill of the last wave, plus a small preference for more waves (tail effects)
    const double eff = (double)total / (waves * kSlots) + 0.002 * std::min(waves, 8.0);
    if (eff > best_eff + (big && s > 1 ? 0.01 : 1e-9)) { best_eff = eff; best = s; }
  }
  return best;
}

// P_ab tile: 96 when it pads nvir by at least 8% less area than 128.
bool pab_tile96(int64_t nvir) {
  const double a128 = (double)cdiv(nvir, 128) * 128.0, a96 = (double)cdiv(nvir, 96) * 96.0;
  return a96 * a96 < 0.92 * a128 * a128;
}

struct Plan {
  int64_t nocc, nvir, naux;
  bool gamma, density;
  bool sym;                  // Gamma without P (FP64): (ia|jb) over pairs j >= k only
  bool g_fixed;              // slab_group given by the caller
  double budget;             // slab budget in bytes (slab_group == 0)
  bool split;                // RIMP2_SPLIT_INT8
  bool autotune;             // in-situ tile choice of the FP64 GEMMs
  bool general;              // FP64 GEMMs take the general loader only
  int sv, sg;                // digits per operand of (ia|jb) and of Gamma
  int64_t kpv, kpg;          // padded reduction lengths of the split products
  size_t off_dbv, off_ev, off_dbg, off_eg, off_cmax, off_dt, off_et;
  // symmetric path with split products: digits of the transposed T blocks and
  // of the group's B rows (the transposed-block product), per group
  size_t off_dtt, off_ett, off_cmt, off_dbk, off_ebk;
  int64_t g;                 // occupied orbitals per slab group
  int64_t s_ab, s_ij, s_gam; // split-K factors
  size_t off_status, off_V, off_T, off_e, off_pab, off_pij, off_gam, off_epart, total;
};

// Workgroups per pair block of an amplitude launch over `pairs` pair blocks
// of nvir x nvir: enough for about 8 waves of the resident workgroups, at
// most kAmpSplitMax and at most one per tile pair.
constexpr int64_t kAmpSplitMax = 64;
int64_t amp_splits(int64_t pairs, int64_t nvir) {
  const int64_t nt = (nvir + 31) / 32, npt = nt * (nt + 1) / 2;
  const int64_t w = (6144 + pairs - 1) / pairs;
  return std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(w, kAmpSplitMax), npt));
}

// Occupied orbitals in the slab group that starts at k0.  The ordered path
// uses one size g for every group.  The symmetric path's slabs hold the
// columns j >= k0 only, so without a caller-given size each group takes the
// most orbitals whose two slabs fit the budget, and later groups grow.
int64_t group_at(const Plan& P, int64_t k0) {
  if (!P.sym || P.g_fixed) return std::min<int64_t>(P.g, P.nocc - k0);
  const double per_k = 2.0 * 8.0 * (double)(P.nocc - k0) * P.nvir * P.nvir;
  // at most as many rows as one reduction launch covers (its grid counts
  // work-items in 32 bits)
  const int64_t red = std::max<int64_t>(1, kMaxWorkgroups * 256 / (P.nvir * P.naux));
  return std::max<int64_t>(1, std::min<int64_t>({(int64_t)(P.budget / per_k), P.nocc - k0, red}));
}

// Split-K factor of the symmetric path's Gamma GEMM over the row blocks of a
// group of gc orbitals starting at k0 (reduction over the pairs j >= k0).
int64_t sym_gamma_splits(const Plan& P, int64_t k0, int64_t gc) {
  return choose_splits(cdiv(gc * P.nvir, kTile) * cdiv(P.naux, kTile), (P.nocc - k0) * P.nvir);
}

// grouped: the fragment runs in a batch wave (whole slab, no split amplitude
// partials).
int make_plan(int64_t nocc, int64_t nvir, int64_t naux, bool gamma, bool density, const rimp2_opts* o, Plan* p,
              bool grouped = false) {
  if (nocc < 1 || nvir < 1 || naux < 1 || nocc > (1 << 20) || nvir > (1 << 24) || naux > (1 << 24))
    return fail(RIMP2_EINVAL, "sizes must be >= 1 (nocc=%lld nvir=%lld naux=%lld)", (long long)nocc,
                (long long)nvir, (long long)naux);
  if ((double)nocc * nvir * naux >= 4.6e18)
    return fail(RIMP2_EINVAL, "nocc*nvir*naux too large");
  if (o && o->precision != RIMP2_FP64 && o->precision != RIMP2_SPLIT_INT8)
    return fail(RIMP2_ENOTSUP, "precision %d is not supported", o->precision);
  p->nocc = nocc; p->nvir = nvir; p->naux = naux; p->gamma = gamma; p->density = density;
  p->split = o && o->precision == RIMP2_SPLIT_INT8;
  p->autotune = o && o->autotune != 0;
  if (o && (o->gemm_loader < 0 || o->gemm_loader > 1))
    return fail(RIMP2_EINVAL, "gemm_loader must be 0 or 1 (got %d)", o->gemm_loader);
  p->general = o && o->gemm_loader == 1;
  p->sv = (o && o->split_slices) ? o->split_slices : 7;
  p->sg = (o && o->split_slices_gamma) ? o->split_slices_gamma : 5;
  if (p->split && (p->sv < 3 || p->sv > 7 || p->sg < 3 || p->sg > 7))
    return fail(RIMP2_EINVAL, "split digit counts must be 3..7 (got %d and %d)", p->sv, p->sg);
  p->kpv = cdiv(naux, 64) * 64;
  p->kpg = cdiv(nocc * nvir, 64) * 64;
  const bool need_T = gamma || density;
  const double slab_per_k = (need_T ? 2.0 : 1.0) * 8.0 * (double)nocc * nvir * nvir;
  p->sym = gamma && !density && !grouped;
  p->g_fixed = o && o->slab_group > 0;
  p->budget = (o && o->slab_budget_bytes) ? (double)o->slab_budget_bytes : 64.0 * (1ull << 30);
  int64_t g;
  if (p->g_fixed) {
    g = std::min<int64_t>(o->slab_group, nocc);
  } else {
    g = (int64_t)(p->budget / slab_per_k);
    g = std::max<int64_t>(1, std::min<int64_t>(g, nocc));
  }
  p->g = g;
  // split-K factors (see choose_splits); P_ab and P_ij use upper-triangular tiles
  const int64_t tab = cdiv(nvir, pab_tile96(nvir) ? 96 : kTile), tij = cdiv(nocc, kSmallTile);
  p->s_ab = density ? choose_splits(tab * (tab + 1) / 2, g * nocc * nvir) : 0;
  p->s_ij = density ? choose_splits(tij * (tij + 1) / 2, g * nvir * nvir) : 0;
  p->s_gam = gamma ? choose_splits(cdiv(g * nvir, kTile) * cdiv(naux, kTile), nocc * nvir) : 0;
  // slab elements (g x ncols pair blocks) and Gamma split partials of the
  // largest group
  double slab_elems = (double)g * nocc * nvir * nvir, gam_part = (double)p->s_gam * g * nvir * naux;
  if (p->sym) {
    slab_elems = gam_part = 0.0;
    for (int64_t k0 = 0; k0 < nocc;) {
      const int64_t gc = group_at(*p, k0), s = sym_gamma_splits(*p, k0, gc);
      slab_elems = std::max(slab_elems, (double)gc * (nocc - k0) * nvir * nvir);
      if (s > 1) gam_part = std::max(gam_part, (double)s * gc * nvir * naux);
      k0 += gc;
    }
  }
  size_t off = 0;
  p->off_status = off; off = align_up(off + 64);
  p->off_V = off; off = align_up(off + (size_t)(8.0 * slab_elems));
  p->off_T = off; if (need_T) off = align_up(off + (size_t)(8.0 * slab_elems));
  p->off_e = off; off = align_up(off + 8 * (size_t)nocc * nocc);
  p->off_pab = off; if (density) off = align_up(off + 8 * (size_t)p->s_ab * nvir * nvir);
  p->off_pij = off; if (density) off = align_up(off + 8 * (size_t)p->s_ij * nocc * nocc);
  p->off_gam = off;
  // (grouped fragments run their Gamma GEMM without split-K: no partials)
  if (gamma && !p->split && !grouped && (p->sym || p->s_gam > 1)) off = align_up(off + (size_t)(8.0 * gam_part));
  p->off_epart = off;
  if (!grouped) {  // largest partial array of the amplitude launches (see run_fragment)
    const bool eonly = !(gamma || density);
    int64_t most = 0;
    for (int64_t k0 = 0; k0 < nocc;) {
      const int64_t gc = group_at(*p, k0);
      const int64_t pairs = gc * ((eonly || p->sym) ? nocc - k0 : nocc);
      const int64_t W = amp_splits(pairs, nvir);
      if (W > 1) most = std::max(most, pairs * W);
      k0 += gc;
    }
    off = align_up(off + 16 * (size_t)most);
  }
  p->off_dbv = p->off_ev = p->off_dbg = p->off_eg = p->off_cmax = p->off_dt = p->off_et = off;
  p->off_dtt = p->off_ett = p->off_cmt = p->off_dbk = p->off_ebk = off;
  if (p->split) {
    const int64_t L = nocc * nvir;
    p->off_dbv = off; off = align_up(off + (size_t)p->sv * L * p->kpv);
    p->off_ev = off; off = align_up(off + 4 * (size_t)L);
    if (gamma && !p->sym) {
      p->off_dbg = off; off = align_up(off + (size_t)p->sg * naux * p->kpg);
      p->off_eg = off; off = align_up(off + 4 * (size_t)naux);
      p->off_cmax = off; off = align_up(off + 8 * (size_t)naux);
      p->off_dt = off; off = align_up(off + (size_t)p->sg * g * nvir * p->kpg);
      p->off_et = off; off = align_up(off + 4 * (size_t)g * nvir);
    } else if (gamma) {
      // per group at k0 (gc orbitals, Lc = (nocc - k0) nvir columns): T row
      // digits [S][gc nvir][pad(Lc)], B column digits of rows >= k0 nvir
      // [S][naux][pad(Lc)], T column digits of the later columns
      // [S][(nocc - k0 - gc) nvir][pad(gc nvir)], B column digits of the
      // group's rows [S][naux][pad(gc nvir)]; sized for the largest group
      double dt = 0, dbg = 0, dtt = 0, dbk = 0, rows = 0, cols = 0;
      int64_t grid = 0;   // largest digit-split grid (split_cols: 32 x 32 tiles)
      for (int64_t k0 = 0; k0 < nocc;) {
        const int64_t gc = group_at(*p, k0), kc = cdiv((nocc - k0) * nvir, 64) * 64, kg = cdiv(gc * nvir, 64) * 64;
        grid = std::max({grid, cdiv(kc, 32) * cdiv(naux, 32), cdiv(kg, 32) * cdiv((nocc - k0 - gc) * nvir, 32)});
        dt = std::max(dt, (double)gc * nvir * kc);
        dbg = std::max(dbg, (double)naux * kc);
        dtt = std::max(dtt, (double)(nocc - k0 - gc) * nvir * kg);
        dbk = std::max(dbk, (double)naux * kg);
        rows = std::max(rows, (double)gc * nvir);
        cols = std::max(cols, (double)(nocc - k0 - gc) * nvir);
        k0 += gc;
      }
      p->off_dbg = off; off = align_up(off + (size_t)(p->sg * dbg));
      p->off_eg = off; off = align_up(off + 4 * (size_t)naux);
      p->off_cmax = off; off = align_up(off + 8 * (size_t)naux);
      p->off_dt = off; off = align_up(off + (size_t)(p->sg * dt));
      p->off_et = off; off = align_up(off + (size_t)(4.0 * rows));
      p->off_dtt = off; off = align_up(off + (size_t)(p->sg * dtt));
      p->off_ett = off; off = align_up(off + (size_t)(4.0 * cols));
      p->off_cmt = off; off = align_up(off + (size_t)(8.0 * cols));
      p->off_dbk = off; off = align_up(off + (size_t)(p->sg * dbk));
      p->off_ebk = off; off = align_up(off + 4 * (size_t)naux);
      if (int rc = check_grid(grid, "digit split")) return rc;
    }
  }
  p->total = off;
  int rc;
  if (gamma && p->s_gam > 1 && !p->sym && (rc = check_grid(cdiv(g * nvir * naux, 256), "reduction"))) return rc;
  if (p->sym && p->g_fixed && (rc = check_grid(cdiv(g * nvir * naux, 256), "reduction"))) return rc;
  if (p->split && ((rc = check_grid(nocc * nvir, "digit split")) || (rc = check_grid(cdiv(p->kpg, 32), "digit split"))))
    return rc;
  return RIMP2_OK;
}

// 16-byte loads need 16-byte aligned bases and even strides (so every pair of
// reduction indices, and every pair of N-contiguous columns, is aligned).
bool kop_vec(const KOperand& o, int64_t K) {
  const bool plain = o.kdiv >= K;
  return (uintptr_t)o.base % 16 == 0 && o.rs % 2 == 0 && (plain || (o.kdiv % 2 == 0 && o.ks1 % 2 == 0));
}

// 16-byte loads for a whole GEMM (the split length is a multiple of kBK, so
// even).  amc: A is M-contiguous (pairs of rows, like an N-contiguous B).
bool gemm_vec(const GemmParams& gp, bool nc, bool amc = false) {
  const bool a = amc ? ((uintptr_t)gp.Am.base % 16 == 0 && gp.Am.ld % 2 == 0) : kop_vec(gp.A, gp.K);
  return a && (nc ? ((uintptr_t)gp.Bn.base % 16 == 0 && gp.Bn.ld % 2 == 0) : kop_vec(gp.Bk, gp.K));
}

// The kernels' FAST path (returns 0 when it does not apply): 16-byte loads,
// an even reduction length (no reduction pair straddles the end), runs of the
// K operands at least one chunk long (a chunk crosses at most one run
// boundary) and an even N for an N-contiguous B (its column pairs past the
// edge are read at N - 2; likewise an even M for an M-contiguous A).  2 when
// a K operand's runs can end inside a chunk.
int fast_level(const GemmParams& gp, bool nc, bool amc = false) {
  auto runs = [&](const KOperand& o) { return o.kdiv >= gp.K || o.kdiv >= kBK; };
  auto wraps = [&](const KOperand& o) { return o.kdiv < gp.K && o.kdiv % kBK != 0; };
  if (!(gp.K % 2 == 0 && gp.kchunk % kBK == 0 && (amc ? gp.M % 2 == 0 : runs(gp.A)) &&
        (nc ? gp.N % 2 == 0 : runs(gp.Bk))))
    return 0;
  return ((!amc && wraps(gp.A)) || (!nc && wraps(gp.Bk))) ? 2 : 1;
}
int gemm_fast(const GemmParams& gp, bool nc, bool amc = false) {
  return gemm_vec(gp, nc, amc) ? fast_level(gp, nc, amc) : 0;
}

template <int BM, int BN, bool NC, int ROLE, bool TRI>
int launch_gemm(GemmParams gp, hipStream_t st, int role, double af, double ab, bool general) {
  gp.tiles_m = (int32_t)cdiv(gp.M, BM);
  gp.tiles_n = (int32_t)cdiv(gp.N, BN);
  gp.group_m = 8;
  if (gp.kchunk <= 0) gp.kchunk = gp.K;
  gp.kchunk = cdiv(gp.kchunk, kBK) * kBK;
  gp.splits = (int32_t)cdiv(gp.K, gp.kchunk);
  if (TRI && (gp.M != gp.N || BM != BN)) return fail(RIMP2_EINVAL, "triangular GEMM needs a square tile grid");
  const int64_t tiles = TRI ? (int64_t)gp.tiles_m * (gp.tiles_m + 1) / 2 : (int64_t)gp.tiles_m * gp.tiles_n;
  const int64_t nwg = tiles * gp.splits;
  if (int rc = check_grid(nwg, "GEMM")) return rc;
  constexpr bool AMC = role_a_mcontig(ROLE);
  if (AMC && gp.splits != 1) return fail(RIMP2_EINVAL, "M-contiguous GEMM without split-K only");
  if (gp.accumulate && (TRI || gp.splits != 1)) return fail(RIMP2_EINVAL, "accumulating GEMM without split-K only");
  const bool vec = gemm_vec(gp, NC, AMC);
  double ef = (TRI ? 0.5 * (1.0 + 1.0 / gp.tiles_m) : 1.0) * 2.0 * (double)gp.M * gp.N * gp.K;
  if (gp.pair_upper) {  // tiles not skipped: those with a pair j >= k or j < pair_lo (see tile_screened)
    int64_t kept = 0;
    for (int64_t tm = 0; tm < gp.tiles_m; ++tm) {
      const int64_t k_lo = gp.skip_k0 + tm * BM / gp.skip_nvir;
      const int64_t below = std::max<int64_t>(0, cdiv((k_lo - gp.skip_j0) * gp.skip_nvir - BN + 1, BN));
      const int64_t from = std::max<int64_t>(0, cdiv((gp.pair_lo - gp.skip_j0) * gp.skip_nvir, BN));
      kept += gp.tiles_n - std::max<int64_t>(0, std::min<int64_t>(below, gp.tiles_n) - from);
    }
    ef *= (double)kept / ((double)gp.tiles_m * gp.tiles_n);
  }
  const int fast = general ? 0 : gemm_fast(gp, NC, AMC);
  return traced(role, af, ef, ab, st, [&] {
    if (fast == 1)
      hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, kBK, NC, ROLE, true, TRI, 1>), dim3((unsigned)nwg), dim3(256), 0,
                         st, gp);
    else if (fast == 2)
      hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, kBK, NC, ROLE, true, TRI, 2>), dim3((unsigned)nwg), dim3(256), 0,
                         st, gp);
    else if (vec)
      hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, kBK, NC, ROLE, true, TRI>), dim3((unsigned)nwg), dim3(256), 0, st, gp);
    else
      hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, kBK, NC, ROLE, false, TRI>), dim3((unsigned)nwg), dim3(256), 0, st, gp);
  });
}


// ---- in-situ tile autotuner (Sec. "GEMM runtime auto-tuning") -------------
// Candidates are output tile shapes; the split length (and with it every
// element's summation order) comes from the plan and is the same for all.
struct TileShape {
  int bm, bn;
};
constexpr int kTuneVars = 4, kTuneTrials = 2;

// Candidate tile shapes of a role's GEMM, the fixed default first.
int tile_candidates(int role, const GemmParams& gp, TileShape* c) {
  switch (role) {
    case R_INTS:
    case R_GAMMA:
    case R_GAMMA_T:
      c[0] = {128, 128}; c[1] = {64, 64};
      return 2;
    case R_PAB: {
      const bool t96 = pab_tile96(gp.M);
      c[0] = t96 ? TileShape{96, 96} : TileShape{128, 128};
      c[1] = t96 ? TileShape{128, 128} : TileShape{96, 96};
      c[2] = {64, 64};
      return 3;
    }
    case R_PIJ:
      c[0] = {64, 64}; c[1] = {128, 128}; c[2] = {32, 32};
      return 3;
    default:
      return 0;
  }
}

// The GEMM of `role` with square tiles of side bm (one of its candidates).
int launch_role(int role, int bm, const GemmParams& gp, hipStream_t st, double af, double ab, bool general) {
  switch (role) {
    case R_INTS:
      return bm == 64 ? launch_gemm<64, 64, false, ROLE_INTS, false>(gp, st, role, af, ab, general)
                      : launch_gemm<128, 128, false, ROLE_INTS, false>(gp, st, role, af, ab, general);
    case R_GAMMA:
      return bm == 64 ? launch_gemm<64, 64, true, ROLE_GAMMA, false>(gp, st, role, af, ab, general)
                      : launch_gemm<128, 128, true, ROLE_GAMMA, false>(gp, st, role, af, ab, general);
    case R_GAMMA_T:
      return bm == 64 ? launch_gemm<64, 64, true, ROLE_GAMMA_T, false>(gp, st, role, af, ab, general)
                      : launch_gemm<128, 128, true, ROLE_GAMMA_T, false>(gp, st, role, af, ab, general);
    case R_PAB:
      return bm == 64   ? launch_gemm<64, 64, false, ROLE_PAB, true>(gp, st, role, af, ab, general)
             : bm == 96 ? launch_gemm<96, 96, false, ROLE_PAB, true>(gp, st, role, af, ab, general)
                        : launch_gemm<128, 128, false, ROLE_PAB, true>(gp, st, role, af, ab, general);
    case R_PIJ:
      return bm == 32    ? launch_gemm<32, 32, false, ROLE_PIJ, true>(gp, st, role, af, ab, general)
             : bm == 128 ? launch_gemm<128, 128, false, ROLE_PIJ, true>(gp, st, role, af, ab, general)
                         : launch_gemm<64, 64, false, ROLE_PIJ, true>(gp, st, role, af, ab, general);
    default:
      return fail(RIMP2_EINVAL, "no GEMM for role %d", role);
  }
}

struct TuneKey {
  int dev, role, vec;
  int64_t M, N, K, kchunk;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, role, vec, M, N, K, kchunk) < std::tie(o.dev, o.role, o.vec, o.M, o.N, o.K, o.kchunk);
  }
};
struct TunePending {
  int var;
  hipEvent_t e0, e1;
};
struct TuneEntry {
  int nvar = 0, best = -1;
  TileShape cand[kTuneVars] = {};
  int launched[kTuneVars] = {}, timed[kTuneVars] = {};
  double min_ms[kTuneVars] = {};
  int64_t uses = 0;
  std::vector<TunePending> pend;
};
struct Tuner {
  std::mutex mu;
  std::map<TuneKey, TuneEntry> tab;
  std::vector<hipEvent_t> pool;
};
Tuner& tuner() {
  static Tuner t;
  return t;
}

// Folds the completed trials of e into its timings without blocking, and
// decides once every candidate has kTuneTrials of them: the fastest (by its
// fastest trial), unless it beats the default by less than 2%.  Caller holds
// the tuner lock.
void tune_poll(Tuner& U, TuneEntry& e) {
  for (size_t i = 0; i < e.pend.size();) {
    const TunePending q = e.pend[i];
    const hipError_t r = hipEventQuery(q.e1);
    if (r == hipErrorNotReady) {
      (void)hipGetLastError();
      ++i;
      continue;
    }
    float ms = 0.f;
    if (r == hipSuccess && hipEventElapsedTime(&ms, q.e0, q.e1) == hipSuccess) {
      e.min_ms[q.var] = e.timed[q.var] ? std::min(e.min_ms[q.var], (double)ms) : (double)ms;
      e.timed[q.var] += 1;
    } else {
      (void)hipGetLastError();
      e.launched[q.var] -= 1;  // trial lost: it is run again
    }
    U.pool.push_back(q.e0);
    U.pool.push_back(q.e1);
    e.pend[i] = e.pend.back();
    e.pend.pop_back();
  }
  if (e.best >= 0) return;
  int best = 0;
  for (int v = 0; v < e.nvar; ++v) {
    if (e.timed[v] < kTuneTrials) return;
    if (e.min_ms[v] < e.min_ms[best] && e.min_ms[v] < 0.98 * e.min_ms[0]) best = v;
  }
  e.best = best;
}

// Runs launch(v) for the candidate v of `key` that the tuner picks (see
// tune_poll): the decided one, else a candidate still owed a trial (bracketed
// by events on st, unless st is capturing), else candidate 0.
template <class F>
int tuned(const TuneKey& key, int nvar, const TileShape* cand, hipStream_t st, F&& launch) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
    (void)hipGetLastError();
    cs = hipStreamCaptureStatusActive;
  }
  const bool capturing = cs != hipStreamCaptureStatusNone;
  Tuner& U = tuner();
  int v = 0;
  bool trial = false;
  hipEvent_t ev[2] = {nullptr, nullptr};
  {
    std::lock_guard<std::mutex> lk(U.mu);
    TuneEntry& e = U.tab[key];
    if (e.nvar == 0) {
      e.nvar = nvar;
      for (int i = 0; i < nvar; ++i) e.cand[i] = cand[i];
    }
    e.uses += 1;
    if (!capturing) tune_poll(U, e);
    if (e.best >= 0) {
      v = e.best;
    } else if (!capturing) {
      for (int i = 0; i < nvar && !trial; ++i)
        if (e.launched[i] < kTuneTrials) { v = i; trial = true; }
    }
    for (int i = 0; trial && i < 2; ++i) {
      if (!U.pool.empty()) {
        ev[i] = U.pool.back();
        U.pool.pop_back();
      } else if (hipEventCreate(&ev[i]) != hipSuccess) {
        (void)hipGetLastError();
        if (i == 1) U.pool.push_back(ev[0]);
        trial = false;
        v = 0;
      }
    }
    if (trial) e.launched[v] += 1;
  }
  const bool rec0 = trial && hipEventRecord(ev[0], st) == hipSuccess;
  const int rc = launch(v);
  if (trial) {
    const bool ok = rec0 && rc == RIMP2_OK && hipEventRecord(ev[1], st) == hipSuccess;
    if (!ok) (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(U.mu);
    TuneEntry& e = U.tab[key];
    if (ok) {
      e.pend.push_back(TunePending{v, ev[0], ev[1]});
    } else {
      e.launched[v] -= 1;
      U.pool.push_back(ev[0]);
      U.pool.push_back(ev[1]);
    }
  }
  return rc;
}

// Launches the GEMM of `role`: the default tile shape, or with autotuning the
// shape's tuned candidate.
int launch_tuned(int role, const GemmParams& gp, bool autotune, bool general, hipStream_t st, double af, double ab) {
  TileShape c[kTuneVars];
  const int nvar = tile_candidates(role, gp, c);
  if (!autotune || nvar < 2) return launch_role(role, c[0].bm, gp, st, af, ab, general);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  // the key's loader field: 16-byte loads, and whether the fast loaders are allowed
  const int loader = (gemm_vec(gp, role == R_GAMMA || role == R_GAMMA_T, role == R_GAMMA_T) ? 1 : 0) + (general ? 2 : 0);
  const TuneKey key{dev, role, loader, gp.M, gp.N, gp.K, gp.kchunk};
  return tuned(key, nvar, c, st, [&](int v) { return launch_role(role, c[v].bm, gp, st, af, ab, general); });
}


template <int S>
void launch_split_rows(const double* X, int64_t rows, int64_t K, int64_t ld, int8_t* D, int64_t kp, int32_t* e,
                       const int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(split_rows_kernel<S>, dim3((unsigned)rows), dim3(256), 0, st, X, rows, K, ld, D, kp, e, status);
}
template <int S>
void launch_split_cols(const double* X, int64_t K, int64_t N, int64_t ld, const unsigned long long* cmax, int8_t* D,
                       int64_t kp, int32_t* e, const int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(split_cols_kernel<S>, dim3((unsigned)cdiv(kp, 32), (unsigned)cdiv(N, 32)), dim3(256), 0, st, X, K,
                     N, ld, cmax, D, kp, e, status);
}
template <int S>
void launch_oz8(OzParams op, bool windowed, hipStream_t st) {
  const int64_t nwg = (int64_t)op.tiles_m * op.tiles_n;
  // one LDS stage (two workgroups per CU) unless a windowed product with at
  // most 5 digits, where the double-buffered stage (still two per CU) was faster
  if (windowed && S <= 5)
    hipLaunchKernelGGL((gemm_oz8_kernel<S, 2>), dim3((unsigned)nwg), dim3(256), 0, st, op);
  else
    hipLaunchKernelGGL((gemm_oz8_kernel<S, 1>), dim3((unsigned)nwg), dim3(256), 0, st, op);
}
#define RIMP2_SWITCH_S(S, CALL)                                   \
  switch (S) {                                                    \
    case 3: { constexpr int SS = 3; CALL; } break;                \
    case 4: { constexpr int SS = 4; CALL; } break;                \
    case 5: { constexpr int SS = 5; CALL; } break;                \
    case 6: { constexpr int SS = 6; CALL; } break;                \
    default: { constexpr int SS = 7; CALL; } break;               \
  }

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// A reduction longer than kOzWindowMax runs in windows of kOzWindow, one
// launch each in stream order, every later window adding into C, with a
// narrower raster (4 row tiles per group).  The tiles of one launch then
// stream digit panels short enough for the caches they share: over the whole
// 360000-long reduction of the Gamma product the launch fetched more than its
// staging bytes from beyond the L2, and the windows made the product about
// 1.7x faster (windows of 5632: 1.6x).
constexpr int64_t kOzWindow = 2816, kOzWindowMax = 8192;

// C[m, n] (m < M, n < N) from split digits; A rows start at a_row0.
// acc0: the first window adds into C too (C already holds a partial sum).
int run_oz8(int S, const int8_t* A, int64_t a_slice, int64_t a_row0, const int32_t* ea, const int8_t* B,
            int64_t b_slice, const int32_t* eb, int64_t M, int64_t N, int64_t kp, double* C, int64_t ldc,
            const int32_t* status, int role, double af, double ab, hipStream_t st, int acc0 = 0) {
  OzParams op{};
  op.M = M; op.N = N; op.kp = kp;
  op.A = A; op.a_slice = a_slice; op.a_row0 = a_row0;
  op.B = B; op.b_slice = b_slice; op.ea = ea; op.eb = eb;
  op.C = C; op.ldc = ldc;
  const bool windowed = kp > kOzWindowMax;
  op.tiles_m = (int32_t)cdiv(M, 64); op.tiles_n = (int32_t)cdiv(N, 64); op.group_m = windowed ? 4 : 8;
  op.status = status;
  const int64_t nwg = (int64_t)op.tiles_m * op.tiles_n;
  if (int rc = check_grid(nwg, "split GEMM")) return rc;
  const double ef = 2.0 * (double)M * N * kp;
  const int64_t kc = windowed ? kOzWindow : kp;
  for (int64_t k0 = 0;; k0 += kc) {
    op.k0 = k0;
    op.kc = std::min(kc, kp - k0);
    op.accumulate = (k0 > 0 || acc0) ? 1 : 0;
    const double fr = kp > 0 ? (double)op.kc / (double)kp : 1.0;
    if (int rc = traced(role, af * fr, ef * fr, ab * fr, st,
                        [&] { RIMP2_SWITCH_S(S, launch_oz8<SS>(op, windowed, st)); }))
      return rc;
    if (k0 + kc >= kp) return RIMP2_OK;
  }
}

KOperand kop(const double* base, int64_t rs, int64_t kdiv, int64_t ks1) { return KOperand{base, rs, kdiv, ks1}; }

// Enqueue the whole path for one fragment.  Pointers already validated.
int run_fragment(const Plan& P, const double* B, const double* eo, const double* ev, double* E, double* Gam,
                 double* Pij, double* Pab, double* e_user, char* ws, const uint8_t* skip, hipStream_t st) {
  const int64_t nocc = P.nocc, nvir = P.nvir, naux = P.naux, L = nocc * nvir;
  const double o = (double)nocc, v = (double)nvir, x = (double)naux;
  int32_t* status = (int32_t*)(ws + P.off_status);
  double* V = (double*)(ws + P.off_V);
  double* T = (double*)(ws + P.off_T);
  double* ep = e_user ? e_user : (double*)(ws + P.off_e);
  int rc;
  if ((rc = traced(R_GAP, 0, 0, 8.0 * (o + v), st, [&] {
         hipLaunchKernelGGL(gap_check_kernel, dim3(1), dim3(256), 0, st, eo, (int)nocc, ev, (int)nvir, status);
       })))
    return rc;
  const bool energy_only = !(P.gamma || P.density);
  // pairs with both orbitals in the slab group: blocks (k, j < k) are not
  // computed and the amplitude pass forms them from their transposes
  const bool mirror = !P.split && !energy_only;
  int8_t* dbv = (int8_t*)(ws + P.off_dbv);
  int32_t* exv = (int32_t*)(ws + P.off_ev);
  int8_t* dbg = (int8_t*)(ws + P.off_dbg);
  int32_t* exg = (int32_t*)(ws + P.off_eg);
  int8_t* dt = (int8_t*)(ws + P.off_dt);
  int32_t* ext = (int32_t*)(ws + P.off_et);
  if (P.split) {
    // digits of every B row (both operands of the (ia|jb) products)
    if ((rc = traced(R_SPLIT, 0, 0, 8.0 * L * naux + (double)P.sv * L * P.kpv, st, [&] {
           RIMP2_SWITCH_S(P.sv, launch_split_rows<SS>(B, L, naux, naux, dbv, P.kpv, exv, status, st));
         })))
      return rc;
    if (P.gamma && !P.sym) {
      // column-scaled, transposed digits of B as the [(j,b)][P] operand of Gamma
      // (the symmetric path splits the rows each group needs, per group)
      unsigned long long* cmax = (unsigned long long*)(ws + P.off_cmax);
      if ((rc = traced(R_SPLIT, 0, 0, 8.0 * naux, st, [&] {
             hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)cdiv(naux, 256)), dim3(256), 0, st, cmax, naux);
           })))
        return rc;
      if ((rc = traced(R_SPLIT, 0, 0, 8.0 * L * naux, st, [&] {
             hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)cdiv(naux, 256), (unsigned)cdiv(L, 1024)), dim3(256), 0,
                                st, B, L, naux, naux, cmax, status);
           })))
        return rc;
      if ((rc = traced(R_SPLIT, 0, 0, 8.0 * L * naux + (double)P.sg * naux * P.kpg, st, [&] {
             RIMP2_SWITCH_S(P.sg, launch_split_cols<SS>(B, L, naux, naux, cmax, dbg, P.kpg, exg, status, st));
           })))
        return rc;
    }
  }
  for (int64_t k0 = 0, gc = 0; k0 < nocc; k0 += gc) {
    gc = group_at(P, k0);
    // (ia|jb) slab: rows (kk, a) of B starting at k0, columns (j, b) over all of B;
    // energy only and the symmetric Gamma path: columns j >= k0 only (pairs
    // j < k come from their mirror)
    const int64_t j0 = (energy_only || P.sym) ? k0 : 0, ncols = nocc - j0, Lc = ncols * nvir;
    const double g = (double)gc, slab = 8.0 * g * (double)ncols * v * v;
    {
      GemmParams gp{};
      gp.M = gc * nvir; gp.N = Lc; gp.K = naux; gp.kchunk = naux;
      gp.A = kop(B + k0 * nvir * naux, naux, INT64_MAX, 0);
      gp.Bk = kop(B + j0 * nvir * naux, naux, INT64_MAX, 0);
      gp.C = V; gp.ldc = Lc; gp.split_stride = 0; gp.status = status;
      gp.skip = skip; gp.skip_nvir = (int32_t)nvir; gp.skip_k0 = (int32_t)k0; gp.skip_j0 = (int32_t)j0;
      gp.skip_nocc = (int32_t)nocc;
      gp.pair_upper = (energy_only || mirror) ? 1 : 0;
      gp.pair_lo = (int32_t)k0;
      // algorithmic FLOPs: unordered pairs whose first orbital is in the group
      // (energy only: exactly the pairs (k, j >= k) computed; otherwise the
      // unordered-pair share of the ordered pairs computed)
      const double npairs = (energy_only || P.sym) ? g * o - (g * (double)k0 + g * (g - 1.0) / 2.0)
                                                   : g * o * (o + 1.0) / (2.0 * o);
      const double af = 2.0 * v * v * x * npairs;
      if (P.split) {
        if ((rc = run_oz8(P.sv, dbv, L * P.kpv, k0 * nvir, exv, dbv + j0 * nvir * P.kpv, L * P.kpv, exv + j0 * nvir,
                          gc * nvir, Lc, P.kpv, V, Lc, status, R_INTS8, af,
                          (double)P.sv * (g * v + o * v) * P.kpv + slab, st)))
          return rc;
      } else if ((rc = launch_tuned(R_INTS, gp, P.autotune, P.general, st, af, 8.0 * (g + o) * v * x + slab))) {
        return rc;
      }
    }
    {
      const int64_t W = amp_splits(gc * ncols, nvir);
      double* epart = (double*)(ws + P.off_epart);
      const int sym = energy_only ? 1 : (P.sym ? 3 : (mirror ? 2 : 0));
      if ((rc = check_grid(gc * ncols * W, "amplitude"))) return rc;
      if ((rc = traced(R_AMP, 0, 0, energy_only ? slab : 3.0 * slab, st, [&] {
             hipLaunchKernelGGL(amplitude_kernel, dim3((unsigned)(gc * ncols * W)), dim3(256), 0, st, V, T, eo, ev,
                                (int)nocc, (int)nvir, (int)k0, (int)j0, (int)ncols, sym, (int)gc,
                                energy_only ? 1 : 0, skip, ep, (int)W, epart, status);
             if (W > 1)
               hipLaunchKernelGGL(pair_energy_reduce_kernel, dim3((unsigned)cdiv(gc * ncols, 256)), dim3(256), 0, st,
                                  (const double*)epart, (int)W, (int)nocc, (int)k0, (int)j0, (int)gc, (int)ncols, sym,
                                  ep, status);
           })))
        return rc;
    }
    if (P.gamma && P.sym) {
      // Gamma rows of the group: Gamma[k] (+)= sum over pairs (k, j >= k0) of T_kj B_j
      const int64_t s_g = sym_gamma_splits(P, k0, gc);
      const int acc = k0 > 0 ? 1 : 0;   // earlier groups' transposed blocks are already in these rows
      GemmParams gp{};
      gp.M = gc * nvir; gp.N = naux; gp.K = Lc;
      gp.kchunk = cdiv(Lc, s_g);
      gp.A = kop(T, Lc, INT64_MAX, 0);
      gp.Bn = NOperand{B + j0 * nvir * naux, naux};
      gp.status = status;
      double* out = Gam + k0 * nvir * naux;
      const double c = (double)ncols;
      const double af = 2.0 * g * v * x * c * v, ab = slab + 8.0 * c * v * x + 8.0 * (1 + acc) * g * v * x;
      const int64_t splits = cdiv(Lc, cdiv(cdiv(Lc, s_g), kBK) * kBK);
      if (P.split) {
        // row product: T rows of the group (reduction over (j >= k0, b)) times
        // the column digits of B's rows j >= k0
        const int64_t kc = cdiv(Lc, 64) * 64;
        unsigned long long* cmax = (unsigned long long*)(ws + P.off_cmax);
        const double* Bj = B + j0 * nvir * naux;
        if ((rc = traced(R_SPLIT, 0, 0, slab + 16.0 * c * v * x + (double)P.sg * (g * v + x) * kc, st, [&] {
               RIMP2_SWITCH_S(P.sg, launch_split_rows<SS>(T, gc * nvir, Lc, Lc, dt, kc, ext, status, st));
               hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)cdiv(naux, 256)), dim3(256), 0, st, cmax, naux);
               hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)cdiv(naux, 256), (unsigned)cdiv(Lc, 1024)), dim3(256),
                                  0, st, Bj, Lc, naux, naux, cmax, status);
               RIMP2_SWITCH_S(P.sg, launch_split_cols<SS>(Bj, Lc, naux, naux, cmax, dbg, kc, exg, status, st));
             })))
          return rc;
        if ((rc = run_oz8(P.sg, dt, gc * nvir * kc, 0, ext, dbg, naux * kc, exg, gc * nvir, naux, kc, out, naux,
                          status, R_GAMMA8, af, (double)P.sg * (g * v + x) * kc + 8.0 * (1 + acc) * g * v * x, st,
                          acc)))
          return rc;
      } else if (splits > 1) {
        double* W = (double*)(ws + P.off_gam);
        gp.C = W; gp.ldc = naux; gp.split_stride = gc * nvir * naux;
        if ((rc = launch_tuned(R_GAMMA, gp, P.autotune, P.general, st, af, ab))) return rc;
        const int64_t n = gc * nvir * naux;
        if ((rc = traced(R_REDUCE, 0, 0, 8.0 * (splits + 1 + acc) * n, st, [&] {
               hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, out, naux, W,
                                  naux, gc * nvir * naux, (int)splits, gc * nvir, naux, 1.0, acc, status);
             })))
          return rc;
      } else {
        gp.C = out; gp.ldc = naux; gp.split_stride = 0; gp.accumulate = acc;
        if ((rc = launch_tuned(R_GAMMA, gp, P.autotune, P.general, st, af, ab))) return rc;
      }
      // Gamma rows of the later orbitals j >= k0 + gc, from the transposed
      // blocks: Gamma[j, b, P] += sum over (kk, a) of T_kj[a, b] B[k0 + kk, a, P]
      // (T_jk = T_kj^T), with the T slab read as an M-contiguous operand
      if (ncols > gc) {
        const int64_t rows = (ncols - gc) * nvir;
        GemmParams gt{};
        gt.M = rows; gt.N = naux; gt.K = gc * nvir; gt.kchunk = gt.K;
        gt.Am = NOperand{T + gc * nvir, Lc};
        gt.Bn = NOperand{B + k0 * nvir * naux, naux};
        gt.C = Gam + (k0 + gc) * nvir * naux; gt.ldc = naux; gt.split_stride = 0; gt.accumulate = acc;
        gt.status = status;
        const double r = (double)(ncols - gc);
        const double aft = 2.0 * r * v * x * g * v, abt = 8.0 * g * v * r * v + 8.0 * g * v * x + 8.0 * (1 + acc) * r * v * x;
        if (P.split) {
          // transposed-block product: the T columns (j >= k0 + gc, b) over the
          // group's rows (kk, a) as column digits [S][rows][pad(gc nvir)], and
          // the group's B rows as column digits [S][naux][pad(gc nvir)]
          const int64_t kg = cdiv(gc * nvir, 64) * 64;
          int8_t* dtt = (int8_t*)(ws + P.off_dtt);
          int32_t* ett = (int32_t*)(ws + P.off_ett);
          unsigned long long* cmt = (unsigned long long*)(ws + P.off_cmt);
          int8_t* dbk = (int8_t*)(ws + P.off_dbk);
          int32_t* ebk = (int32_t*)(ws + P.off_ebk);
          unsigned long long* cmax = (unsigned long long*)(ws + P.off_cmax);
          const double* Tt = T + gc * nvir;
          const double* Bk = B + k0 * nvir * naux;
          if ((rc = traced(R_SPLIT, 0, 0, 16.0 * g * v * r * v + 16.0 * g * v * x + (double)P.sg * (r * v + x) * kg, st,
                           [&] {
                             hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)cdiv(rows, 256)), dim3(256), 0, st,
                                                cmt, rows);
                             hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)cdiv(rows, 256),
                                                                    (unsigned)cdiv(gc * nvir, 1024)),
                                                dim3(256), 0, st, Tt, gc * nvir, rows, Lc, cmt, status);
                             RIMP2_SWITCH_S(P.sg, launch_split_cols<SS>(Tt, gc * nvir, rows, Lc, cmt, dtt, kg, ett,
                                                                        status, st));
                             hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)cdiv(naux, 256)), dim3(256), 0, st,
                                                cmax, naux);
                             hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)cdiv(naux, 256),
                                                                    (unsigned)cdiv(gc * nvir, 1024)),
                                                dim3(256), 0, st, Bk, gc * nvir, naux, naux, cmax, status);
                             RIMP2_SWITCH_S(P.sg, launch_split_cols<SS>(Bk, gc * nvir, naux, naux, cmax, dbk, kg, ebk,
                                                                        status, st));
                           })))
            return rc;
          if ((rc = run_oz8(P.sg, dtt, rows * kg, 0, ett, dbk, naux * kg, ebk, rows, naux, kg,
                            Gam + (k0 + gc) * nvir * naux, naux, status, R_GAMMA_T8, aft,
                            (double)P.sg * (r * v + x) * kg + 8.0 * (1 + acc) * r * v * x, st, acc)))
            return rc;
        } else if ((rc = launch_tuned(R_GAMMA_T, gt, P.autotune, P.general, st, aft, abt))) {
          return rc;
        }
      }
    } else if (P.gamma) {
      GemmParams gp{};
      gp.M = gc * nvir; gp.N = naux; gp.K = L;
      gp.kchunk = cdiv(L, P.s_gam);
      gp.A = kop(T, L, INT64_MAX, 0);
      gp.Bn = NOperand{B, naux};
      double* out = Gam + k0 * nvir * naux;
      const double af = 2.0 * g * v * x * o * v, ab = slab + 8.0 * o * v * x + 8.0 * g * v * x;
      if (P.split) {
        if ((rc = traced(R_SPLIT, 0, 0, slab + (double)P.sg * g * v * P.kpg, st, [&] {
               RIMP2_SWITCH_S(P.sg, launch_split_rows<SS>(T, gc * nvir, L, L, dt, P.kpg, ext, status, st));
             })))
          return rc;
        if ((rc = run_oz8(P.sg, dt, gc * nvir * P.kpg, 0, ext, dbg, naux * P.kpg, exg, gc * nvir, naux, P.kpg, out,
                          naux, status, R_GAMMA8, af, (double)P.sg * (g * v + x) * P.kpg + 8.0 * g * v * x, st)))
          return rc;
      } else if (P.s_gam > 1) {
        double* W = (double*)(ws + P.off_gam);
        gp.C = W; gp.ldc = naux; gp.split_stride = gc * nvir * naux; gp.status = status;
        if ((rc = launch_tuned(R_GAMMA, gp, P.autotune, P.general, st, af, ab))) return rc;
        const int64_t splits = cdiv(L, cdiv(cdiv(L, P.s_gam), kBK) * kBK);
        const int64_t n = gc * nvir * naux;
        if ((rc = traced(R_REDUCE, 0, 0, 8.0 * (splits + 1) * n, st, [&] {
               hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, out, naux, W,
                                  naux, gc * nvir * naux, (int)splits, gc * nvir, naux, 1.0, 0, status);
             })))
          return rc;
      } else {
        gp.C = out; gp.ldc = naux; gp.split_stride = 0; gp.status = status;
        if ((rc = launch_tuned(R_GAMMA, gp, P.autotune, P.general, st, af, ab))) return rc;
      }
    }
    if (P.density) {
      const int accumulate = k0 > 0 ? 1 : 0;
      {  // P_ab[a,b] += sum over (kk, j, c) of T[kk,a,j,c] X[kk,b,j,c]
        GemmParams gp{};
        const int64_t K = gc * L;
        gp.M = nvir; gp.N = nvir; gp.K = K;
        gp.kchunk = cdiv(K, P.s_ab);
        gp.A = kop(T, L, L, nvir * L);
        gp.Bk = kop(V, L, L, nvir * L);
        double* W = (double*)(ws + P.off_pab);
        gp.C = W; gp.ldc = nvir; gp.split_stride = nvir * nvir; gp.status = status;
        const int64_t splits = cdiv(K, cdiv(cdiv(K, P.s_ab), kBK) * kBK);
        if ((rc = launch_tuned(R_PAB, gp, P.autotune, P.general, st, 2.0 * v * v * g * o * v,
                               2.0 * slab + 8.0 * splits * v * v)))
          return rc;
        if ((rc = traced(R_REDUCE, 0, 0, 8.0 * (splits + 2) * v * v, st, [&] {
               hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)cdiv(nvir * nvir, 256)), dim3(256), 0, st, Pab,
                                  nvir, W, nvir, nvir * nvir, (int)splits, nvir, nvir, 1.0, accumulate, status);
             })))
          return rc;
      }
      {  // P_ij[i,j] -= sum over (kk, a, b) of T[kk,a,i,b] X[kk,a,j,b]
        GemmParams gp{};
        const int64_t K = gc * nvir * nvir;
        gp.M = nocc; gp.N = nocc; gp.K = K;
        gp.kchunk = cdiv(K, P.s_ij);
        gp.A = kop(T, nvir, nvir, L);
        gp.Bk = kop(V, nvir, nvir, L);
        double* W = (double*)(ws + P.off_pij);
        gp.C = W; gp.ldc = nocc; gp.split_stride = nocc * nocc; gp.status = status;
        const int64_t splits = cdiv(K, cdiv(cdiv(K, P.s_ij), kBK) * kBK);
        // each slab's contribution to P_ij is symmetric: upper-triangular tiles, mirrored
        if ((rc = launch_tuned(R_PIJ, gp, P.autotune, P.general, st, 2.0 * o * o * g * v * v,
                               2.0 * slab + 8.0 * splits * o * o)))
          return rc;
        if ((rc = traced(R_REDUCE, 0, 0, 8.0 * (splits + 2) * o * o, st, [&] {
               hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)cdiv(nocc * nocc, 256)), dim3(256), 0, st, Pij,
                                  nocc, W, nocc, nocc * nocc, (int)splits, nocc, nocc, -1.0, accumulate, status);
             })))
          return rc;
      }
    }
  }
  return traced(R_ESUM, 0, 0, 8.0 * o * o, st, [&] {
    hipLaunchKernelGGL(energy_sum_kernel, dim3(1), dim3(256), 0, st, ep, nocc * nocc, E, status);
  });
}

int want_of(const double* Gam, const double* Pij, const double* Pab, int* want) {
  if ((Pij == nullptr) != (Pab == nullptr))
    return fail(RIMP2_EINVAL, "P_ij and P_ab must both be given or both be NULL");
  *want = (Gam ? RIMP2_WANT_GAMMA : 0) | (Pij ? RIMP2_WANT_DENSITY : 0);
  return RIMP2_OK;
}


// ---- scratch space of the entry point that allocates nothing ----------------
// The array `scratch` is declared at file scope at the top of this file.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RIMP2_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(RIMP2_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_scratch_ptr[dev];
  return RIMP2_OK;
}

// The plan of rimp2_fragment_noalloc: the caller's options with, unless the
// caller fixed the slab group, the largest slab budget whose workspace fits
// the scratch array.
int noalloc_plan(int64_t nocc, int64_t nvir, int64_t naux, int want, const rimp2_opts* opts, Plan* P) {
  rimp2_opts o{};
  if (opts) o = *opts;
  if (o.autotune) return fail(RIMP2_ENOTSUP, "autotuning records events: not available without allocation");
  int rc;
  if (o.slab_group == 0) {
    o.slab_budget_bytes = kScratchBytes;
    for (int it = 0; it < 64; ++it) {
      if ((rc = make_plan(nocc, nvir, naux, want & RIMP2_WANT_GAMMA, want & RIMP2_WANT_DENSITY, &o, P))) return rc;
      if (P->total <= kScratchBytes) return RIMP2_OK;
      const size_t over = P->total - kScratchBytes;
      if (o.slab_budget_bytes <= over + 1) break;
      o.slab_budget_bytes -= over + 1;   // the slabs shrink by at least the overshoot (or g reaches 1)
    }
  }
  if ((rc = make_plan(nocc, nvir, naux, want & RIMP2_WANT_GAMMA, want & RIMP2_WANT_DENSITY, &o, P))) return rc;
  if (P->total > kScratchBytes)
    return fail(RIMP2_ENOMEM, "fragment nocc=%lld nvir=%lld naux=%lld needs %zu bytes of scratch, more than the "
                "%zu of rimp2_fragment_noalloc", (long long)nocc, (long long)nvir, (long long)naux, P->total,
                kScratchBytes);
  return RIMP2_OK;
}


// One digit split of one fragment in a batch wave (split precision): rows of
// X [N][K] (row stride ld) into D [S][N][kp] with exps e[N] (split_row), or
// columns of X [K][N] into D [S][N][kp] with column maxima cmax[N]
// (colmax_block, split_cols_tile).  gx: the op's blocks along its first grid
// dimension (columns: cdiv(N, 256) for the maxima, cdiv(kp, 32) for the
// digits, which use one op entry each).
struct DigitOp {
  const double* X;
  int64_t K, N, ld, kp, gx;
  int8_t* D;
  int32_t* e;
  unsigned long long* cmax;
  const int32_t* status;
};

// ---- batches -----------------------------------------------------------------
// Grouped GEMM lists of a wave: 4 roles x 2 candidate tiles x 4 loaders
// (0: two chunks ahead, 1: the same with runs ending inside chunks, 2: the
// general loader with 16-byte loads, 3: the general loader, 8-byte loads).
constexpr int kGLists = 32;
struct GemmList {            // grouped GEMM problems of one role in one wave
  std::vector<GemmParams> p;
  std::vector<int64_t> prefix;  // work items (tiles x splits)
};
struct Wave {
  std::vector<int32_t> frags;   // original fragment indices, largest first
  size_t tab_bytes = 0;         // bytes of device tables at the start of the wave region
  size_t host_off = 0;          // offset of this wave's tables in the pinned blob
  size_t bytes = 0;             // tables + fragment partitions
  // offsets within the tables
  size_t o_fs, o_idx, o_amp, o_amp_pre, o_red, o_red_pre, o_cnt;
  // GEMM lists, index glist(role, candidate tile, loader): every GEMM is
  // listed once per candidate tile shape (kBatchTile)
  size_t o_g[kGLists], o_pre[kGLists];
  int n_g[kGLists];
  int64_t items_g[kGLists];
  uint64_t sig = 0;             // hash of the wave's fragment sizes (autotuner key)
  int namp, nred_ab, nred_ij;
  int64_t amp_blocks, red_blocks_ab, red_blocks_ij;
  // split products (precision RIMP2_SPLIT_INT8): grouped (ia|jb) and Gamma
  // product lists, run in reduction windows (win_* launches each), with one
  // work counter per launch
  size_t o_oz[2] = {0, 0}, o_oz_pre[2] = {0, 0}, o_cnt_oz = 0;
  int n_oz[2] = {0, 0};
  int64_t items_oz[2] = {0, 0};
  int win_oz[2] = {0, 0};
  // grouped digit splits: lists 0 (B rows), 1 (B columns: zero, maxima), 2 (B
  // column digits), 3 (T rows); each with its op table and four prefix arrays
  // (one per mode; only the one its launch uses is read)
  static constexpr int kDigitLists = 4;
  size_t o_dop[kDigitLists] = {0, 0, 0, 0}, o_dpre[kDigitLists][4] = {};
  int n_dop[kDigitLists] = {0, 0, 0, 0};
  int64_t blocks_dop[kDigitLists][4] = {};
};
}  // namespace

struct rimp2_batch_s {
  bool autotune = false;
  bool split = false;              // grouped split-precision products
  std::vector<rimp2_frag_desc> d;
  std::vector<int32_t> solo;       // fragments run alone
  std::vector<Plan> plan;          // per fragment (solo: own plan; grouped: full-slab plan)
  std::vector<Wave> waves;
  std::vector<char> blob;          // tables of every wave, as laid out at the start of the workspace
  char* host = nullptr;            // pinned copy of blob (handle path)
  size_t tables_total = 0, ws_bytes = 0;
};

namespace {

uint64_t rel(size_t off) { return kRelTag | (uint64_t)off; }
template <class T>
T* relp(size_t off) { return (T*)(uintptr_t)rel(off); }
bool aligned16(const void* p) { return ((uintptr_t)p & ~kRelTag) % 16 == 0; }
bool kop_vec_rel(const KOperand& o, int64_t K) {
  const bool plain = o.kdiv >= K;
  return aligned16(o.base) && o.rs % 2 == 0 && (plain || (o.kdiv % 2 == 0 && o.ks1 % 2 == 0));
}

// Grouped GEMM roles of a wave, their two candidate square tiles (default
// first) and list index.
const int kBatchRole[4] = {R_INTS, R_GAMMA, R_PAB, R_PIJ};
const int kBatchTile[4][2] = {{128, 64}, {128, 64}, {128, 64}, {64, 32}};
int glist(int rho, int cand, int loader) { return (rho * 2 + cand) * 4 + loader; }
// loader of a grouped GEMM (see kGLists); vec: 16-byte loads apply; general:
// the general loader only
int loader_of(const GemmParams& g, bool nc, bool vec, bool general) {
  if (!vec) return 3;
  if (general) return 2;
  const int f = fast_level(g, nc);
  return f ? f - 1 : 2;
}

// tiles, splits and group size of a GEMM, as launch_gemm sets them
int64_t finalize_gemm(GemmParams& gp, int BM, int BN, bool tri) {
  gp.tiles_m = (int32_t)cdiv(gp.M, BM);
  gp.tiles_n = (int32_t)cdiv(gp.N, BN);
  gp.group_m = 8;
  if (gp.kchunk <= 0) gp.kchunk = gp.K;
  gp.kchunk = cdiv(gp.kchunk, kBK) * kBK;
  gp.splits = (int32_t)cdiv(gp.K, gp.kchunk);
  const int64_t tiles = tri ? (int64_t)gp.tiles_m * (gp.tiles_m + 1) / 2 : (int64_t)gp.tiles_m * gp.tiles_n;
  return tiles * gp.splits;
}

size_t place(size_t& off, size_t bytes) {
  const size_t o = off;
  off = align_up(off + bytes);
  return o;
}

int batch_plan(int32_t nfrag, const rimp2_frag_desc* d, const rimp2_opts* opts, rimp2_batch_s* B) {
  if (nfrag < 0 || (nfrag > 0 && !d)) return fail(RIMP2_EINVAL, "bad batch arguments");
  if (opts && opts->precision != RIMP2_FP64 && opts->precision != RIMP2_SPLIT_INT8)
    return fail(RIMP2_ENOTSUP, "precision %d is not supported", opts->precision);
  if (opts && opts->pair_skip) return fail(RIMP2_ENOTSUP, "pair_skip is not supported for batches");
  const bool split = opts && opts->precision == RIMP2_SPLIT_INT8;
  B->split = split;
  B->d.assign(d, d + nfrag);
  B->autotune = opts && opts->autotune;
  if (opts && (opts->gemm_loader < 0 || opts->gemm_loader > 1))
    return fail(RIMP2_EINVAL, "gemm_loader must be 0 or 1 (got %d)", opts->gemm_loader);
  const bool general = opts && opts->gemm_loader == 1;
  B->plan.resize(nfrag);
  const size_t budget = (opts && opts->slab_budget_bytes) ? opts->slab_budget_bytes : (size_t)64 << 30;
  std::vector<int32_t> order(nfrag), grouped;
  std::vector<char> solo(nfrag, 0);
  for (int32_t f = 0; f < nfrag; ++f) {
    if (!d[f].B || !d[f].eps_occ || !d[f].eps_vir || !d[f].E)
      return fail(RIMP2_EINVAL, "fragment %d: B, eps_occ, eps_vir and E must not be NULL", f);
    int want, rc;
    if ((rc = want_of(d[f].Gamma, d[f].P_ij, d[f].P_ab, &want))) return fail(rc, "fragment %d: %s", f, g_err);
    rimp2_opts o{};
    o.slab_group = d[f].nocc;     // whole slab
    if (split) {
      o.precision = RIMP2_SPLIT_INT8;
      o.split_slices = opts->split_slices;
      o.split_slices_gamma = opts->split_slices_gamma;
    }
    Plan P;
    if ((rc = make_plan(d[f].nocc, d[f].nvir, d[f].naux, want & 1, want & 2, &o, &P, true)))
      return fail(rc, "fragment %d: %s", f, g_err);
    P.s_gam = 1;
    if (P.total > budget) {
      solo[f] = 1;
      if ((rc = make_plan(d[f].nocc, d[f].nvir, d[f].naux, want & 1, want & 2, opts, &P)))
        return fail(rc, "fragment %d: %s", f, g_err);
    }
    B->plan[f] = P;
    order[f] = f;
  }
  auto cost = [&](int32_t f) { return (double)d[f].nocc * d[f].nocc * d[f].nvir * d[f].nvir * d[f].naux; };
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
  size_t ws = kAlign, max_solo = 0;
  for (int32_t f : order) {
    if (solo[f]) { B->solo.push_back(f); max_solo = std::max(max_solo, B->plan[f].total); }
    else grouped.push_back(f);
  }
  // pack waves greedily (largest first) by the sum of full-slab plans
  for (size_t i = 0; i < grouped.size();) {
    Wave W;
    size_t sum = 0;
    while (i < grouped.size() && (W.frags.empty() || sum + B->plan[grouped[i]].total <= budget)) {
      sum += B->plan[grouped[i]].total;
      W.frags.push_back(grouped[i++]);
    }
    B->waves.push_back(W);
  }
  // table layout of every wave (sizes depend only on the wave's fragment count)
  size_t tab = 0;
  for (Wave& W : B->waves) {
    const int n = (int)W.frags.size();
    size_t t = 0;
    W.o_fs = place(t, sizeof(FragSmall) * n);
    W.o_idx = place(t, sizeof(int32_t) * n);
    W.o_amp = place(t, sizeof(AmpDesc) * n);
    W.o_amp_pre = place(t, sizeof(int64_t) * (n + 1));
    W.o_red = place(t, sizeof(ReduceDesc) * 2 * n);
    W.o_red_pre = place(t, sizeof(int64_t) * (2 * n + 1));
    for (int r = 0; r < kGLists; ++r) {
      W.o_g[r] = place(t, sizeof(GemmParams) * n);
      W.o_pre[r] = place(t, sizeof(int64_t) * (n + 1));
    }
    W.o_cnt = place(t, kGLists * sizeof(unsigned long long));
    if (split) {
      for (int r = 0; r < 2; ++r) {
        W.o_oz[r] = place(t, sizeof(OzParams) * n);
        W.o_oz_pre[r] = place(t, sizeof(int64_t) * (n + 1));
      }
      // windows of every fragment in the wave (at most this many launches per product)
      for (int32_t f : W.frags) {
        const Plan& P = B->plan[f];
        W.win_oz[0] = std::max<int>(W.win_oz[0], (int)cdiv(P.kpv, kOzWindow));
        if (P.gamma) W.win_oz[1] = std::max<int>(W.win_oz[1], (int)cdiv(P.kpg, kOzWindow));
      }
      W.o_cnt_oz = place(t, sizeof(unsigned long long) * (W.win_oz[0] + W.win_oz[1]));
      for (int r = 0; r < Wave::kDigitLists; ++r) {
        W.o_dop[r] = place(t, sizeof(DigitOp) * n);
        for (int m = 0; m < 4; ++m) W.o_dpre[r][m] = place(t, sizeof(int64_t) * (n + 1));
      }
    }
    W.tab_bytes = t;
    W.host_off = tab;
    tab = align_up(tab + t);
  }
  B->tables_total = tab;
  B->blob.assign(tab, 0);
  for (Wave& W : B->waves) {
    const int n = (int)W.frags.size();
    std::vector<FragSmall> fs(n);
    std::vector<int32_t> idx(n);
    std::vector<AmpDesc> amp(n);
    std::vector<int64_t> amp_pre(n + 1, 0);
    std::vector<ReduceDesc> red;
    std::vector<int64_t> red_pre(1, 0);
    GemmList gl[kGLists];
    for (auto& l : gl) l.prefix.assign(1, 0);
    std::vector<OzParams> oz[2];
    std::vector<int64_t> oz_pre[2] = {{0}, {0}};
    std::vector<DigitOp> dop[Wave::kDigitLists];
    std::vector<int64_t> dpre[Wave::kDigitLists][4];
    for (auto& l : dpre)
      for (auto& v : l) v.assign(1, 0);
    // op f of list r: workgroups per mode
    auto add_dop = [&](int r, const DigitOp& o, int64_t rows_wgs, int64_t zero_wgs, int64_t max_wgs, int64_t dig_wgs) {
      dop[r].push_back(o);
      const int64_t w[4] = {rows_wgs, zero_wgs, max_wgs, dig_wgs};
      for (int m = 0; m < 4; ++m) dpre[r][m].push_back(dpre[r][m].back() + w[m]);
    };
    // every GEMM goes to the lists of both candidate tiles of its role
    auto add = [&](int rho, const GemmParams& g0, bool vec) {
      for (int c = 0; c < 2; ++c) {
        GemmParams g = g0;
        const int64_t items = finalize_gemm(g, kBatchTile[rho][c], kBatchTile[rho][c], rho >= 2);
        GemmList& l = gl[glist(rho, c, loader_of(g, rho == 1, vec, general))];
        l.p.push_back(g);
        l.prefix.push_back(l.prefix.back() + items);
      }
    };
    uint64_t sig = 1469598103934665603ull;  // FNV-1a over the fragment sizes and outputs
    size_t poff = tab;   // fragment partitions follow all tables (shared by the waves)
    for (int i = 0; i < n; ++i) {
      const int32_t f = W.frags[i];
      const rimp2_frag_desc& q = d[f];
      const Plan& P = B->plan[f];
      const size_t base = poff;
      poff = align_up(poff + P.total);
      const int64_t nocc = q.nocc, nvir = q.nvir, naux = q.naux, L = nocc * nvir;
      for (int64_t w : {nocc, nvir, naux, (int64_t)P.gamma, (int64_t)P.density}) sig = (sig ^ (uint64_t)w) * 1099511628211ull;
      int32_t* status = relp<int32_t>(base + P.off_status);
      double* V = relp<double>(base + P.off_V);
      double* T = relp<double>(base + P.off_T);
      double* ep = q.e_pair ? q.e_pair : relp<double>(base + P.off_e);
      fs[i] = FragSmall{q.eps_occ, q.eps_vir, ep, q.E, status, q.nocc, q.nvir};
      idx[i] = f;
      amp[i] = AmpDesc{V, T, q.eps_occ, q.eps_vir, ep, status, q.nocc, q.nvir, (P.gamma || P.density) ? 0 : 1};
      amp_pre[i + 1] = amp_pre[i] + nocc * nocc;
      if (split) {  // (ia|jb) and Gamma as INT8 digit products of the whole slab
        OzParams z{};
        z.M = L; z.N = L; z.kp = P.kpv; z.k0 = 0; z.kc = P.kpv;
        z.A = relp<int8_t>(base + P.off_dbv); z.a_slice = L * P.kpv; z.a_row0 = 0;
        z.B = z.A; z.b_slice = z.a_slice;
        z.ea = relp<int32_t>(base + P.off_ev); z.eb = z.ea;
        z.C = V; z.ldc = L;
        z.tiles_m = (int32_t)cdiv(L, 64); z.tiles_n = z.tiles_m; z.group_m = 8;
        z.pair_nvir = (int32_t)nvir;   // blocks j < k: the amplitude pass mirrors them
        z.status = status;
        oz[0].push_back(z);
        oz_pre[0].push_back(oz_pre[0].back() + (int64_t)z.tiles_m * z.tiles_n);
        // digits of every B row (both operands of the (ia|jb) products)
        add_dop(0, DigitOp{q.B, naux, L, naux, P.kpv, 0, relp<int8_t>(base + P.off_dbv),
                           relp<int32_t>(base + P.off_ev), nullptr, status}, L, 0, 0, 0);
        if (P.gamma) {
          OzParams y{};
          y.M = L; y.N = naux; y.kp = P.kpg; y.k0 = 0; y.kc = P.kpg;
          y.A = relp<int8_t>(base + P.off_dt); y.a_slice = L * P.kpg; y.a_row0 = 0;
          y.B = relp<int8_t>(base + P.off_dbg); y.b_slice = naux * P.kpg;
          y.ea = relp<int32_t>(base + P.off_et); y.eb = relp<int32_t>(base + P.off_eg);
          y.C = q.Gamma; y.ldc = naux;
          y.tiles_m = (int32_t)cdiv(L, 64); y.tiles_n = (int32_t)cdiv(naux, 64); y.group_m = 8;
          y.status = status;
          oz[1].push_back(y);
          oz_pre[1].push_back(oz_pre[1].back() + (int64_t)y.tiles_m * y.tiles_n);
          // column digits of B (maxima first) and row digits of the T slab
          unsigned long long* cm = relp<unsigned long long>(base + P.off_cmax);
          const int64_t gxm = cdiv(naux, 256), gxd = cdiv(P.kpg, 32);
          add_dop(1, DigitOp{q.B, L, naux, naux, P.kpg, gxm, nullptr, nullptr, cm, status}, 0, gxm,
                  gxm * cdiv(L, 1024), 0);
          add_dop(2, DigitOp{q.B, L, naux, naux, P.kpg, gxd, relp<int8_t>(base + P.off_dbg),
                             relp<int32_t>(base + P.off_eg), cm, status}, 0, 0, 0, gxd * cdiv(naux, 32));
          add_dop(3, DigitOp{relp<double>(base + P.off_T), L, L, L, P.kpg, 0, relp<int8_t>(base + P.off_dt),
                             relp<int32_t>(base + P.off_et), nullptr, status}, L, 0, 0, 0);
        }
      }
      if (!split) {  // (ia|jb)
        GemmParams gp{};
        gp.M = nocc * nvir; gp.N = L; gp.K = naux; gp.kchunk = naux;
        gp.A = KOperand{q.B, naux, INT64_MAX, 0};
        gp.Bk = KOperand{q.B, naux, INT64_MAX, 0};
        gp.C = V; gp.ldc = L; gp.status = status;
        gp.skip_nvir = (int32_t)nvir; gp.skip_nocc = (int32_t)nocc; gp.pair_upper = 1;
        add(0, gp, kop_vec_rel(gp.A, gp.K) && kop_vec_rel(gp.Bk, gp.K));
      }
      if (P.gamma && !split) {
        GemmParams gp{};
        gp.M = nocc * nvir; gp.N = naux; gp.K = L; gp.kchunk = L;
        gp.A = KOperand{T, L, INT64_MAX, 0};
        gp.Bn = NOperand{q.B, naux};
        gp.C = q.Gamma; gp.ldc = naux; gp.status = status;
        add(1, gp, kop_vec_rel(gp.A, gp.K) && aligned16(q.B) && naux % 2 == 0);
      }
      if (P.density) {
        double* Wab = relp<double>(base + P.off_pab);
        double* Wij = relp<double>(base + P.off_pij);
        GemmParams ga{};
        ga.M = nvir; ga.N = nvir; ga.K = nocc * L; ga.kchunk = cdiv(ga.K, P.s_ab);
        ga.A = KOperand{T, L, L, nvir * L};
        ga.Bk = KOperand{V, L, L, nvir * L};
        ga.C = Wab; ga.ldc = nvir; ga.split_stride = nvir * nvir; ga.status = status;
        add(2, ga, kop_vec_rel(ga.A, ga.K) && kop_vec_rel(ga.Bk, ga.K));
        (void)finalize_gemm(ga, kTile, kTile, false);   // splits for the reduction
        GemmParams gi{};
        gi.M = nocc; gi.N = nocc; gi.K = nocc * nvir * nvir; gi.kchunk = cdiv(gi.K, P.s_ij);
        gi.A = KOperand{T, nvir, nvir, L};
        gi.Bk = KOperand{V, nvir, nvir, L};
        gi.C = Wij; gi.ldc = nocc; gi.split_stride = nocc * nocc; gi.status = status;
        add(3, gi, kop_vec_rel(gi.A, gi.K) && kop_vec_rel(gi.Bk, gi.K));
        (void)finalize_gemm(gi, kSmallTile, kSmallTile, true);
        ReduceDesc ra{q.P_ab, Wab, status, nvir, nvir, nvir * nvir, nvir, nvir, 1.0, ga.splits, 0};
        ReduceDesc ri{q.P_ij, Wij, status, nocc, nocc, nocc * nocc, nocc, nocc, -1.0, gi.splits, 0};
        red.push_back(ra); red_pre.push_back(red_pre.back() + cdiv(nvir * nvir, 256));
        red.push_back(ri); red_pre.push_back(red_pre.back() + cdiv(nocc * nocc, 256));
      }
    }
    W.bytes = poff;
    ws = std::max(ws, poff);
    W.namp = n;
    W.amp_blocks = amp_pre[n];
    W.nred_ab = (int)red.size();
    W.red_blocks_ab = red_pre.back();
    for (int r = 0; r < kGLists; ++r) { W.n_g[r] = (int)gl[r].p.size(); W.items_g[r] = gl[r].prefix.back(); }
    W.sig = sig;
    char* blob = B->blob.data() + W.host_off;
    auto put = [&](size_t off, const void* src, size_t bytes) { if (bytes) memcpy(blob + off, src, bytes); };
    put(W.o_fs, fs.data(), sizeof(FragSmall) * n);
    put(W.o_idx, idx.data(), sizeof(int32_t) * n);
    put(W.o_amp, amp.data(), sizeof(AmpDesc) * n);
    put(W.o_amp_pre, amp_pre.data(), sizeof(int64_t) * (n + 1));
    put(W.o_red, red.data(), sizeof(ReduceDesc) * red.size());
    put(W.o_red_pre, red_pre.data(), sizeof(int64_t) * red_pre.size());
    for (int r = 0; r < kGLists; ++r) {
      put(W.o_g[r], gl[r].p.data(), sizeof(GemmParams) * gl[r].p.size());
      put(W.o_pre[r], gl[r].prefix.data(), sizeof(int64_t) * gl[r].prefix.size());
    }
    if (split) {
      for (int r = 0; r < 2; ++r) {
        W.n_oz[r] = (int)oz[r].size();
        W.items_oz[r] = oz_pre[r].back();
        put(W.o_oz[r], oz[r].data(), sizeof(OzParams) * oz[r].size());
        put(W.o_oz_pre[r], oz_pre[r].data(), sizeof(int64_t) * oz_pre[r].size());
      }
      for (int r = 0; r < Wave::kDigitLists; ++r) {
        W.n_dop[r] = (int)dop[r].size();
        put(W.o_dop[r], dop[r].data(), sizeof(DigitOp) * dop[r].size());
        for (int m = 0; m < 4; ++m) {
          W.blocks_dop[r][m] = dpre[r][m].back();
          put(W.o_dpre[r][m], dpre[r][m].data(), sizeof(int64_t) * dpre[r][m].size());
        }
      }
    }
  }
  // solo fragments use the workspace after all tables
  B->ws_bytes = std::max(ws, align_up(tab + max_solo));
  return RIMP2_OK;
}

template <int BM, int BN, bool NC, int ROLE, bool VEC, bool TRI, int FAST>
int launch_grouped(const GemmGroup& G, int64_t items, int role, hipStream_t st) {
  if (G.nprob == 0 || items == 0) return RIMP2_OK;
  const int64_t grid = std::min<int64_t>(items, kSlots);
  return traced(role, 0, 0, 0, st, [&] {
    hipLaunchKernelGGL((gemm_f64_grouped<BM, BN, kBK, NC, ROLE, VEC, TRI, FAST>), dim3((unsigned)grid), dim3(256), 0,
                       st, G);
  });
}

// One grouped launch of batch role rho with candidate tile c (kBatchTile) over
// its list of one loader (see kGLists).
int launch_group_list(int rho, int c, int loader, const GemmGroup& G, int64_t items, hipStream_t st) {
  const int role = kBatchRole[rho];
// (the 128 x 128 Gamma tile with the fast loader runs out of registers in the
// persistent loop: its fast lists take the general 16-byte loader)
#define RIMP2_G(BM, NC, ROLE, TRI, F1, F2)                                                            \
  switch (loader) {                                                                                   \
    case 0: return launch_grouped<BM, BM, NC, ROLE, true, TRI, F1>(G, items, role, st);               \
    case 1: return launch_grouped<BM, BM, NC, ROLE, true, TRI, F2>(G, items, role, st);               \
    case 2: return launch_grouped<BM, BM, NC, ROLE, true, TRI, 0>(G, items, role, st);                \
    default: return launch_grouped<BM, BM, NC, ROLE, false, TRI, 0>(G, items, role, st);              \
  }
  switch (rho * 2 + c) {
    case 0: RIMP2_G(128, false, ROLE_INTS, false, 1, 2);
    case 1: RIMP2_G(64, false, ROLE_INTS, false, 1, 2);
    case 2: RIMP2_G(128, true, ROLE_GAMMA, false, 0, 0);
    case 3: RIMP2_G(64, true, ROLE_GAMMA, false, 1, 2);
    case 4: RIMP2_G(128, false, ROLE_PAB, true, 1, 2);
    case 5: RIMP2_G(64, false, ROLE_PAB, true, 1, 2);
    case 6: RIMP2_G(64, false, ROLE_PIJ, true, 1, 2);
    default: RIMP2_G(32, false, ROLE_PIJ, true, 1, 2);
  }
#undef RIMP2_G
}

__device__ __forceinline__ int digit_op_at(const int64_t* prefix, int n, int64_t t) {
  int lo = 0, hi = n - 1;   // last f with prefix[f] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Grouped digit splits: one launch over every op of a list (prefix counts
// each op's workgroups).  mode 0: rows; 1: zero cmax; 2: column maxima;
// 3: column digits.
template <int S, int MODE>
__global__ __launch_bounds__(256) void digit_split_grouped(const DigitOp* ops, const int64_t* prefix, int n) {
  const int f = digit_op_at(prefix, n, blockIdx.x);
  const DigitOp o = ops[f];
  if (o.status != nullptr && *o.status != 0) return;
  const int64_t u = (int64_t)blockIdx.x - prefix[f];
  if constexpr (MODE == 0) {
    split_row<S>(o.X, o.N, o.K, o.ld, o.D, o.kp, o.e, u);
  } else if constexpr (MODE == 1) {
    const int64_t i = u * 256 + threadIdx.x;
    if (i < o.N) o.cmax[i] = 0ull;
  } else if constexpr (MODE == 2) {
    colmax_block(o.X, o.K, o.N, o.ld, o.cmax, u % o.gx, u / o.gx);
  } else {
    split_cols_tile<S>(o.X, o.K, o.N, o.ld, o.cmax, o.D, o.kp, o.e, u % o.gx, u / o.gx);
  }
}

__global__ void relocate_digit_kernel(char* base, DigitOp* ops, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    DigitOp& o = ops[i];
    reloc_t(o.X, base); reloc_t(o.D, base); reloc_t(o.e, base); reloc_t(o.cmax, base); reloc_t(o.status, base);
  }
}

__global__ void relocate_oz_kernel(char* base, OzParams* z, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    OzParams& p = z[i];
    reloc_t(p.A, base); reloc_t(p.B, base); reloc_t(p.ea, base); reloc_t(p.eb, base);
    reloc_t(p.C, base); reloc_t(p.status, base);
  }
}

// One grouped split-product launch over reduction window `window` of every
// problem in G (same NBUF choice as launch_oz8 for a windowed product).
template <int S>
int launch_oz8_grouped(const OzGroup& G, int64_t items, int64_t window, int role, hipStream_t st) {
  if (G.nprob == 0 || items == 0) return RIMP2_OK;
  const int64_t grid = std::min<int64_t>(items, kSlots);
  return traced(role, 0, 0, 0, st, [&] {
    if (S <= 5)
      hipLaunchKernelGGL((gemm_oz8_grouped<S, 2>), dim3((unsigned)grid), dim3(256), 0, st, G, window, kOzWindow);
    else
      hipLaunchKernelGGL((gemm_oz8_grouped<S, 1>), dim3((unsigned)grid), dim3(256), 0, st, G, window, kOzWindow);
  });
}

// upload: 0 = tables already in the workspace, 1 = copy them from B->host (pinned) on the stream
int batch_run(rimp2_batch_s* B, int32_t* status_dev, void* workspace, size_t bytes, hipStream_t st, int upload) {
  if (!workspace) return fail(RIMP2_EINVAL, "workspace must not be NULL");
  if ((uintptr_t)workspace % kAlign) return fail(RIMP2_EWORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < B->ws_bytes) return fail(RIMP2_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, B->ws_bytes);
  char* ws = (char*)workspace;
  int rc;
  if (upload && B->tables_total) {
    if (!B->host) return fail(RIMP2_EINVAL, "batch tables are not resident");
    HIP_TRY(hipMemcpyAsync(ws, B->host, B->tables_total, hipMemcpyHostToDevice, st));
  }
  // solo fragments run with their own workspace layout after the tables
  char* solo_ws = ws + B->tables_total;
  for (int32_t f : B->solo) {
    const rimp2_frag_desc& q = B->d[f];
    if ((rc = run_fragment(B->plan[f], q.B, q.eps_occ, q.eps_vir, q.E, q.Gamma, q.P_ij, q.P_ab, q.e_pair, solo_ws,
                           nullptr, st)))
      return fail(rc, "fragment %d: %s", f, g_err);
    if (status_dev && (rc = traced(R_STATUS, 0, 0, 8.0, st, [&] {
                         hipLaunchKernelGGL(copy_status_kernel, dim3(1), dim3(64), 0, st,
                                            (const int32_t*)(solo_ws + B->plan[f].off_status), status_dev, (int)f);
                       })))
      return rc;
  }
  for (const Wave& W : B->waves) {
    const int n = (int)W.frags.size();
    GemmParams* gp0 = (GemmParams*)(ws + W.host_off + W.o_g[0]);
    auto at = [&](size_t o) { return ws + W.host_off + o; };
    if ((rc = traced(R_STATUS, 0, 0, 0, st, [&] {
           // relocate every table (GEMM lists are contiguous per role; relocate each list)
           for (int r = 0; r < kGLists; ++r)
             if (W.n_g[r])
               hipLaunchKernelGGL(relocate_tables_kernel, dim3((unsigned)cdiv(W.n_g[r], 256)), dim3(256), 0, st, ws,
                                  (GemmParams*)at(W.o_g[r]), W.n_g[r], (AmpDesc*)nullptr, 0, (ReduceDesc*)nullptr, 0,
                                  (FragSmall*)nullptr, 0);
           const int m = std::max(n, W.nred_ab);
           hipLaunchKernelGGL(relocate_tables_kernel, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, st, ws, gp0, 0,
                              (AmpDesc*)at(W.o_amp), n, (ReduceDesc*)at(W.o_red), W.nred_ab, (FragSmall*)at(W.o_fs),
                              n);
           hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, st, (unsigned long long*)at(W.o_cnt),
                              kGLists);
           hipLaunchKernelGGL(gap_check_grouped, dim3((unsigned)n), dim3(256), 0, st, (const FragSmall*)at(W.o_fs));
           if (B->split) {
             for (int r = 0; r < 2; ++r)
               if (W.n_oz[r])
                 hipLaunchKernelGGL(relocate_oz_kernel, dim3((unsigned)cdiv(W.n_oz[r], 256)), dim3(256), 0, st, ws,
                                    (OzParams*)at(W.o_oz[r]), W.n_oz[r]);
             for (int r = 0; r < Wave::kDigitLists; ++r)
               if (W.n_dop[r])
                 hipLaunchKernelGGL(relocate_digit_kernel, dim3((unsigned)cdiv(W.n_dop[r], 256)), dim3(256), 0, st,
                                    ws, (DigitOp*)at(W.o_dop[r]), W.n_dop[r]);
             const int nc = W.win_oz[0] + W.win_oz[1];
             if (nc)
               hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)cdiv(nc, 256)), dim3(256), 0, st,
                                  (unsigned long long*)at(W.o_cnt_oz), (int64_t)nc);
           }
         })))
      return rc;
    auto grp = [&](int r) {
      return GemmGroup{(const GemmParams*)at(W.o_g[r]), (const int64_t*)at(W.o_pre[r]), W.n_g[r],
                       (unsigned long long*)at(W.o_cnt) + r};
    };
    // each GEMM role: the lists of one candidate tile (with autotuning the
    // tuned one for this wave's fragment sizes)
    auto run_role = [&](int rho) -> int {
      auto items_of = [&](int c) {
        int64_t n = 0;
        for (int k = 0; k < 4; ++k) n += W.items_g[glist(rho, c, k)];
        return n;
      };
      const int64_t i0 = items_of(0);
      if (i0 == 0) return RIMP2_OK;
      auto launch = [&](int c) -> int {
        for (int k = 0; k < 4; ++k) {
          const int li = glist(rho, c, k);
          const int r = launch_group_list(rho, c, k, grp(li), W.items_g[li], st);
          if (r) return r;
        }
        return RIMP2_OK;
      };
      if (!B->autotune) return launch(0);
      int dev = 0;
      HIP_TRY(hipGetDevice(&dev));
      const int64_t i1 = items_of(1);
      const TuneKey key{dev, kBatchRole[rho], 2, n, i0, i1, (int64_t)(W.sig >> 1)};
      const TileShape cand[2] = {{kBatchTile[rho][0], kBatchTile[rho][0]}, {kBatchTile[rho][1], kBatchTile[rho][1]}};
      return tuned(key, 2, cand, st, launch);
    };
    // split products: the per-fragment digit splits, then one grouped launch
    // per reduction window (r = 0: (ia|jb), r = 1: Gamma)
    auto run_split = [&](int r) -> int {
      int rc2;
      // the digit splits of every fragment of the wave: one launch per list and mode
      auto dlaunch = [&](int list, int mode, int S) -> int {
        const int64_t blocks = W.blocks_dop[list][mode];
        if (W.n_dop[list] == 0 || blocks == 0) return RIMP2_OK;
        if (int rc3 = check_grid(blocks, "digit split")) return rc3;
        const DigitOp* ops = (const DigitOp*)at(W.o_dop[list]);
        const int64_t* pre = (const int64_t*)at(W.o_dpre[list][mode]);
        return traced(R_SPLIT, 0, 0, 0, st, [&] {
          switch (mode) {
            case 0: RIMP2_SWITCH_S(S, hipLaunchKernelGGL((digit_split_grouped<SS, 0>), dim3((unsigned)blocks),
                                                        dim3(256), 0, st, ops, pre, W.n_dop[list])); break;
            case 1: hipLaunchKernelGGL((digit_split_grouped<1, 1>), dim3((unsigned)blocks), dim3(256), 0, st, ops,
                                       pre, W.n_dop[list]); break;
            case 2: hipLaunchKernelGGL((digit_split_grouped<1, 2>), dim3((unsigned)blocks), dim3(256), 0, st, ops,
                                       pre, W.n_dop[list]); break;
            default: RIMP2_SWITCH_S(S, hipLaunchKernelGGL((digit_split_grouped<SS, 3>), dim3((unsigned)blocks),
                                                         dim3(256), 0, st, ops, pre, W.n_dop[list])); break;
          }
        });
      };
      const int sv = B->plan[W.frags[0]].sv, sg = B->plan[W.frags[0]].sg;
      if (r == 0) {
        if ((rc2 = dlaunch(0, 0, sv))) return rc2;
      } else if ((rc2 = dlaunch(1, 1, sg)) || (rc2 = dlaunch(1, 2, sg)) || (rc2 = dlaunch(2, 3, sg)) ||
                 (rc2 = dlaunch(3, 0, sg))) {
        return rc2;
      }
      if (W.n_oz[r] == 0) return RIMP2_OK;
      const int S = r == 0 ? B->plan[W.frags[0]].sv : B->plan[W.frags[0]].sg;
      unsigned long long* cnt = (unsigned long long*)at(W.o_cnt_oz) + (r == 0 ? 0 : W.win_oz[0]);
      for (int w = 0; w < W.win_oz[r]; ++w) {
        const OzGroup G{(const OzParams*)at(W.o_oz[r]), (const int64_t*)at(W.o_oz_pre[r]), W.n_oz[r], cnt + w};
        const int role = r == 0 ? R_INTS8 : R_GAMMA8;
        RIMP2_SWITCH_S(S, rc2 = launch_oz8_grouped<SS>(G, W.items_oz[r], w, role, st));
        if (rc2) return rc2;
      }
      return RIMP2_OK;
    };
    if ((rc = B->split ? run_split(0) : run_role(0))) return rc;
    if ((rc = traced(R_AMP, 0, 0, 0, st, [&] {
           hipLaunchKernelGGL(amplitude_grouped, dim3((unsigned)W.amp_blocks), dim3(256), 0, st,
                              (const AmpDesc*)at(W.o_amp), (const int64_t*)at(W.o_amp_pre), n);
         })))
      return rc;
    if ((rc = B->split ? run_split(1) : run_role(1)) || (rc = run_role(2)) || (rc = run_role(3))) return rc;
    if (W.nred_ab && (rc = traced(R_REDUCE, 0, 0, 0, st, [&] {
                        hipLaunchKernelGGL(reduce_grouped, dim3((unsigned)W.red_blocks_ab), dim3(256), 0, st,
                                           (const ReduceDesc*)at(W.o_red), (const int64_t*)at(W.o_red_pre), W.nred_ab);
                      })))
      return rc;
    if ((rc = traced(R_ESUM, 0, 0, 0, st, [&] {
           hipLaunchKernelGGL(energy_sum_grouped, dim3((unsigned)n), dim3(256), 0, st, (const FragSmall*)at(W.o_fs));
           if (status_dev)
             hipLaunchKernelGGL(status_copy_grouped, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st,
                                (const FragSmall*)at(W.o_fs), (const int32_t*)at(W.o_idx), n, status_dev);
         })))
      return rc;
  }
  return RIMP2_OK;
}

}  // namespace

extern "C" {

int rimp2_version(void) { return 10000; }

const char* rimp2_last_error(void) { return g_err; }

const char* rimp2_status_string(int s) {
  switch (s) {
    case RIMP2_OK: return "RIMP2_OK";
    case RIMP2_EINVAL: return "RIMP2_EINVAL";
    case RIMP2_ENOMEM: return "RIMP2_ENOMEM";
    case RIMP2_EWORKSPACE: return "RIMP2_EWORKSPACE";
    case RIMP2_EDEVICE: return "RIMP2_EDEVICE";
    case RIMP2_EGAP: return "RIMP2_EGAP";
    case RIMP2_ENOTSUP: return "RIMP2_ENOTSUP";
    case RIMP2_ENOCONV: return "RIMP2_ENOCONV";
    default: return "unknown rimp2 status";
  }
}

int rimp2_workspace_size(int32_t nocc, int32_t nvir, int32_t naux, int32_t want, const rimp2_opts* opts,
                         size_t* bytes) {
  if (!bytes) return fail(RIMP2_EINVAL, "bytes is NULL");
  if (want & ~(RIMP2_WANT_GAMMA | RIMP2_WANT_DENSITY)) return fail(RIMP2_EINVAL, "bad want mask %d", want);
  Plan P;
  int rc = make_plan(nocc, nvir, naux, want & RIMP2_WANT_GAMMA, want & RIMP2_WANT_DENSITY, opts, &P);
  if (rc) return rc;
  *bytes = P.total;
  return RIMP2_OK;
}

int rimp2_fragment(int32_t nocc, int32_t nvir, int32_t naux, const double* B, const double* eps_occ,
                   const double* eps_vir, double* E, double* Gamma, double* P_ij, double* P_ab, double* e_pair,
                   void* workspace, size_t workspace_bytes, const rimp2_opts* opts, void* stream) {
  if (!B || !eps_occ || !eps_vir || !E || !workspace)
    return fail(RIMP2_EINVAL, "B, eps_occ, eps_vir, E and workspace must not be NULL");
  if ((uintptr_t)workspace % kAlign) return fail(RIMP2_EWORKSPACE, "workspace must be 256-byte aligned");
  int want, rc;
  if ((rc = want_of(Gamma, P_ij, P_ab, &want))) return rc;
  Plan P;
  if ((rc = make_plan(nocc, nvir, naux, want & RIMP2_WANT_GAMMA, want & RIMP2_WANT_DENSITY, opts, &P))) return rc;
  if (workspace_bytes < P.total)
    return fail(RIMP2_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, P.total);
  return run_fragment(P, B, eps_occ, eps_vir, E, Gamma, P_ij, P_ab, e_pair, (char*)workspace,
                      opts ? opts->pair_skip : nullptr, (hipStream_t)stream);
}

int rimp2_fragment_noalloc(int32_t nocc, int32_t nvir, int32_t naux, const double* B, const double* eps_occ,
                           const double* eps_vir, double* E, double* Gamma, double* P_ij, double* P_ab,
                           double* e_pair, int32_t* status_dev, const rimp2_opts* opts, void* stream) {
  if (!B || !eps_occ || !eps_vir || !E) return fail(RIMP2_EINVAL, "B, eps_occ, eps_vir and E must not be NULL");
  int want, rc;
  if ((rc = want_of(Gamma, P_ij, P_ab, &want))) return rc;
  Plan P;
  if ((rc = noalloc_plan(nocc, nvir, naux, want, opts, &P))) return rc;
  char* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  hipStream_t st = (hipStream_t)stream;
  t_noalloc = true;
  rc = run_fragment(P, B, eps_occ, eps_vir, E, Gamma, P_ij, P_ab, e_pair, ws, opts ? opts->pair_skip : nullptr, st);
  if (rc == RIMP2_OK && status_dev) {
    rc = traced(R_STATUS, 0, 0, 8.0, st, [&] {
      hipLaunchKernelGGL(copy_status_kernel, dim3(1), dim3(64), 0, st, (const int32_t*)(ws + P.off_status),
                         status_dev, 0);
    });
  }
  t_noalloc = false;
  return rc;
}

int rimp2_read_status(const void* workspace, void* stream, int32_t* status) {
  if (!workspace || !status) return fail(RIMP2_EINVAL, "workspace and status must not be NULL");
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(hipMemcpy(status, workspace, sizeof(int32_t), hipMemcpyDeviceToHost));
  return RIMP2_OK;
}

int rimp2_batch_create(int32_t nfrag, const rimp2_frag_desc* descs, const rimp2_opts* opts, rimp2_batch* batch,
                       size_t* workspace_bytes) {
  if (!batch || !workspace_bytes) return fail(RIMP2_EINVAL, "batch and workspace_bytes must not be NULL");
  rimp2_batch_s* B = new rimp2_batch_s();
  int rc = batch_plan(nfrag, descs, opts, B);
  if (!rc && B->tables_total) {
    if (hipHostMalloc((void**)&B->host, B->tables_total, hipHostMallocDefault) != hipSuccess) {
      B->host = nullptr;
      rc = fail(RIMP2_EDEVICE, "hipHostMalloc of %zu bytes failed", B->tables_total);
    } else {
      memcpy(B->host, B->blob.data(), B->tables_total);
    }
  }
  if (rc) {
    if (B->host) (void)hipHostFree(B->host);
    delete B;
    return rc;
  }
  *batch = B;
  *workspace_bytes = B->ws_bytes;
  return RIMP2_OK;
}

int rimp2_batch_run(rimp2_batch batch, int32_t* status_dev, void* workspace, size_t workspace_bytes, void* stream) {
  if (!batch) return fail(RIMP2_EINVAL, "batch is NULL");
  return batch_run(batch, status_dev, workspace, workspace_bytes, (hipStream_t)stream, 1);
}

int rimp2_batch_destroy(rimp2_batch batch) {
  if (!batch) return RIMP2_OK;
  if (batch->host) HIP_TRY(hipHostFree(batch->host));
  delete batch;
  return RIMP2_OK;
}

int rimp2_batch_workspace_size(int32_t nfrag, const rimp2_frag_desc* descs, const rimp2_opts* opts, size_t* bytes) {
  if (!bytes) return fail(RIMP2_EINVAL, "bytes is NULL");
  rimp2_batch_s B;
  const int rc = batch_plan(nfrag, descs, opts, &B);
  if (rc) return rc;
  *bytes = B.ws_bytes;
  return RIMP2_OK;
}

int rimp2_fragment_batch(int32_t nfrag, const rimp2_frag_desc* descs, int32_t* status_dev, void* workspace,
                         size_t workspace_bytes, const rimp2_opts* opts, void* stream) {
  if (!workspace) return fail(RIMP2_EINVAL, "workspace must not be NULL");
  if ((uintptr_t)workspace % kAlign) return fail(RIMP2_EWORKSPACE, "workspace must be 256-byte aligned");
  rimp2_batch_s B;
  int rc = batch_plan(nfrag, descs, opts, &B);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (workspace_bytes < B.ws_bytes)
    return fail(RIMP2_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, B.ws_bytes);
  // earlier work on the stream may still use the workspace: wait, then upload the tables synchronously
  HIP_TRY(hipStreamSynchronize(st));
  if (B.tables_total) HIP_TRY(hipMemcpy(workspace, B.blob.data(), B.tables_total, hipMemcpyHostToDevice));
  return batch_run(&B, status_dev, workspace, workspace_bytes, st, 0);
}

int rimp2_timing_enable(int enable) {
  Tracer& T = tracer();
  std::lock_guard<std::mutex> lk(T.mu);
  for (auto& r : T.recs) {
    T.pool.push_back(r.e0);
    T.pool.push_back(r.e1);
  }
  T.recs.clear();
  T.on = enable != 0;
  return RIMP2_OK;
}

int rimp2_timing_collect(rimp2_kernel_stat* stats, int32_t capacity, int32_t* count) {
  if (!count || (capacity > 0 && !stats)) return fail(RIMP2_EINVAL, "bad timing_collect arguments");
  Tracer& T = tracer();
  std::lock_guard<std::mutex> lk(T.mu);
  rimp2_kernel_stat acc[R_NROLES];
  memset(acc, 0, sizeof acc);
  for (int r = 0; r < R_NROLES; ++r) snprintf(acc[r].name, sizeof acc[r].name, "%s", kRoleName[r]);
  for (auto& r : T.recs) {
    HIP_TRY(hipEventSynchronize(r.e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.e0, r.e1));
    rimp2_kernel_stat& a = acc[r.role];
    a.launches += 1;
    a.total_ms += ms;
    a.alg_flops += r.af;
    a.exec_flops += r.ef;
    a.alg_bytes += r.ab;
    T.pool.push_back(r.e0);
    T.pool.push_back(r.e1);
  }
  T.recs.clear();
  int32_t n = 0;
  for (int r = 0; r < R_NROLES; ++r)
    if (acc[r].launches > 0) {
      if (n < capacity) stats[n] = acc[r];
      ++n;
    }
  *count = std::min(n, capacity);
  return RIMP2_OK;
}

int rimp2_autotune_report(rimp2_tune_stat* stats, int32_t capacity, int32_t* count) {
  if (!count || (capacity > 0 && !stats)) return fail(RIMP2_EINVAL, "bad autotune_report arguments");
  Tuner& U = tuner();
  std::lock_guard<std::mutex> lk(U.mu);
  int32_t n = 0;
  for (auto& kv : U.tab) {
    TuneEntry& e = kv.second;
    tune_poll(U, e);
    if (n >= capacity) break;
    rimp2_tune_stat& t = stats[n++];
    memset(&t, 0, sizeof t);
    snprintf(t.role, sizeof t.role, "%s", kRoleName[kv.first.role]);
    t.device = kv.first.dev;
    t.nvar = e.nvar;
    t.best = e.best;
    t.vec = kv.first.vec;
    t.M = kv.first.M; t.N = kv.first.N; t.K = kv.first.K; t.kchunk = kv.first.kchunk;
    for (int v = 0; v < e.nvar && v < 4; ++v) {
      t.tile_m[v] = e.cand[v].bm;
      t.tile_n[v] = e.cand[v].bn;
      t.timed[v] = e.timed[v];
      t.min_ms[v] = e.min_ms[v];
    }
    t.uses = e.uses;
  }
  *count = n;
  return RIMP2_OK;
}

int rimp2_autotune_reset(void) {
  Tuner& U = tuner();
  std::lock_guard<std::mutex> lk(U.mu);
  for (auto& kv : U.tab)
    for (auto& q : kv.second.pend) {
      U.pool.push_back(q.e0);
      U.pool.push_back(q.e1);
    }
  U.tab.clear();
  return RIMP2_OK;
}

// ---- adjacent gradient steps (include/rimp2_gradient.h) --------------------

int rimp2_gamma_ao_workspace_size(int32_t nocc, int32_t nao, int32_t pcount, size_t* bytes) {
  if (!bytes) return fail(RIMP2_EINVAL, "bytes is NULL");
  if (nocc < 1 || nao < 1 || pcount < 1) return fail(RIMP2_EINVAL, "sizes must be >= 1");
  *bytes = align_up(64) + align_up((size_t)8 * nocc * nao * pcount);
  return RIMP2_OK;
}

int rimp2_gamma_ao(int32_t nocc, int32_t nvir, int32_t nao, int32_t naux, int32_t p0, int32_t pcount,
                   const double* Gamma, const double* C_occ, const double* C_vir, double* out, void* workspace,
                   size_t workspace_bytes, void* stream) {
  if (nocc < 1 || nvir < 1 || nao < 1 || naux < 1 || pcount < 1 || p0 < 0 || (int64_t)p0 + pcount > naux)
    return fail(RIMP2_EINVAL, "sizes must be >= 1 and 0 <= p0, p0 + pcount <= naux (nocc=%d nvir=%d nao=%d naux=%d "
                "p0=%d pcount=%d)", nocc, nvir, nao, naux, p0, pcount);
  if (!Gamma || !C_occ || !C_vir || !out || !workspace)
    return fail(RIMP2_EINVAL, "Gamma, C_occ, C_vir, out and workspace must not be NULL");
  if ((uintptr_t)workspace % kAlign) return fail(RIMP2_EWORKSPACE, "workspace must be 256-byte aligned");
  size_t need = 0;
  int rc;
  if ((rc = rimp2_gamma_ao_workspace_size(nocc, nao, pcount, &need))) return rc;
  if (workspace_bytes < need) return fail(RIMP2_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  unsigned long long* status = (unsigned long long*)ws;
  double* H = (double*)(ws + align_up(64));
  const int64_t pc = pcount, na = nao;
  if ((rc = traced(R_STATUS, 0, 0, 8.0, st, [&] {
         hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, st, status, 1);
       })))
    return rc;
  // H[i][n][P] = sum_a C_vir[a][n] Gamma[i][a][p0 + P], one GEMM per occupied orbital
  for (int64_t i = 0; i < nocc; ++i) {
    GemmParams gp{};
    gp.M = na; gp.N = pc; gp.K = nvir; gp.kchunk = nvir;
    gp.Am = NOperand{C_vir, na};
    gp.Bn = NOperand{Gamma + i * nvir * (int64_t)naux + p0, naux};
    gp.C = H + i * na * pc; gp.ldc = pc; gp.status = (const int32_t*)status;
    if ((rc = launch_gemm<128, 128, true, ROLE_AO, false>(gp, st, R_GAMMA_AO, 2.0 * na * pc * nvir,
                                                           8.0 * (nvir * (na + pc) + na * pc), false)))
      return rc;
  }
  // out[m][(n, P)] = sum_i C_occ[i][m] H[i][(n, P)]
  GemmParams gp{};
  gp.M = na; gp.N = na * pc; gp.K = nocc; gp.kchunk = nocc;
  gp.Am = NOperand{C_occ, na};
  gp.Bn = NOperand{H, na * pc};
  gp.C = out; gp.ldc = na * pc; gp.status = (const int32_t*)status;
  return launch_gemm<128, 128, true, ROLE_AO, false>(gp, st, R_GAMMA_AO, 2.0 * na * na * pc * nocc,
                                                     8.0 * (nocc * na + nocc * na * pc + na * na * pc), false);
}

namespace {
// Split-K plan of the two L-term GEMMs: M x N outputs over reduction K.
struct LPlan {
  int64_t s1, s2;
  size_t part_bytes;
};
LPlan l_plan(int64_t nocc, int64_t nvir, int64_t nmo, int64_t naux) {
  LPlan L;
  L.s1 = choose_splits(cdiv(nocc, kTile) * cdiv(nmo, kTile), nvir * naux);
  L.s2 = choose_splits(cdiv(nvir, kTile) * cdiv(nmo, kTile), nocc * naux);
  L.part_bytes = std::max((size_t)8 * L.s1 * nocc * nmo, (size_t)8 * L.s2 * nvir * nmo);
  return L;
}
}  // namespace

int rimp2_l_terms_workspace_size(int32_t nocc, int32_t nvir, int32_t nmo, int32_t naux, size_t* bytes) {
  if (!bytes) return fail(RIMP2_EINVAL, "bytes is NULL");
  if (nocc < 1 || nvir < 1 || nmo < 1 || naux < 1) return fail(RIMP2_EINVAL, "sizes must be >= 1");
  *bytes = align_up(64) + align_up(l_plan(nocc, nvir, nmo, naux).part_bytes);
  return RIMP2_OK;
}

int rimp2_l_terms(int32_t nocc, int32_t nvir, int32_t nmo, int32_t naux, const double* Gamma, const double* I_qa,
                  const double* I_iq, double* L1, double* L2, void* workspace, size_t workspace_bytes, void* stream) {
  if (nocc < 1 || nvir < 1 || nmo < 1 || naux < 1) return fail(RIMP2_EINVAL, "sizes must be >= 1");
  if (!Gamma || !workspace) return fail(RIMP2_EINVAL, "Gamma and workspace must not be NULL");
  if ((L1 == nullptr) != (I_qa == nullptr) || (L2 == nullptr) != (I_iq == nullptr))
    return fail(RIMP2_EINVAL, "L1 needs I_qa and L2 needs I_iq (both or neither)");
  if ((uintptr_t)workspace % kAlign) return fail(RIMP2_EWORKSPACE, "workspace must be 256-byte aligned");
  size_t need = 0;
  int rc;
  if ((rc = rimp2_l_terms_workspace_size(nocc, nvir, nmo, naux, &need))) return rc;
  if (workspace_bytes < need) return fail(RIMP2_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  int32_t* status = (int32_t*)ws;
  double* W = (double*)(ws + align_up(64));
  const LPlan lp = l_plan(nocc, nvir, nmo, naux);
  const double o = nocc, v = nvir, q = nmo, x = naux;
  if ((rc = traced(R_STATUS, 0, 0, 8.0, st, [&] {
         hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, st, (unsigned long long*)status, 1);
       })))
    return rc;
  auto run = [&](GemmParams gp, int64_t s, double* out, double af, double ab) -> int {
    gp.kchunk = cdiv(gp.K, s);
    gp.C = W; gp.ldc = gp.N; gp.split_stride = gp.M * gp.N; gp.status = status;
    const int64_t splits = cdiv(gp.K, cdiv(gp.kchunk, kBK) * kBK);
    int r;
    if ((r = launch_gemm<128, 128, false, ROLE_LTERM, false>(gp, st, R_LTERM, af, ab, false))) return r;
    const int64_t n = gp.M * gp.N;
    return traced(R_REDUCE, 0, 0, 8.0 * (splits + 1) * n, st, [&] {
      hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, out, gp.N,
                         (const double*)W, gp.N, gp.M * gp.N, (int)splits, gp.M, gp.N, 1.0, 0, status);
    });
  };
  if (L1) {   // L'[i][q] = sum over (a, P) of Gamma[i][a][P] I_qa[q][a][P]
    GemmParams gp{};
    gp.M = nocc; gp.N = nmo; gp.K = (int64_t)nvir * naux;
    gp.A = kop(Gamma, gp.K, INT64_MAX, 0);
    gp.Bk = kop(I_qa, gp.K, INT64_MAX, 0);
    if ((rc = run(gp, lp.s1, L1, 2.0 * o * q * v * x, 8.0 * (o + q) * v * x + 8.0 * o * q))) return rc;
  }
  if (L2) {   // L''[a][q] = sum over (i, P) of Gamma[i][a][P] I_iq[i][q][P]
    GemmParams gp{};
    gp.M = nvir; gp.N = nmo; gp.K = (int64_t)nocc * naux;
    gp.A = kop(Gamma, naux, naux, (int64_t)nvir * naux);
    gp.Bk = kop(I_iq, naux, naux, (int64_t)nmo * naux);
    if ((rc = run(gp, lp.s2, L2, 2.0 * v * q * o * x, 8.0 * (v + q) * o * x + 8.0 * v * q))) return rc;
  }
  return RIMP2_OK;
}

// ---- orbital response: antisymmetrised-integral term, Z-vector, W ---------------
namespace {

// c_part[z][P] = sum over (r, s) pairs of chunk z of Bf[r][s][P] D[r][s]
// (fixed chunking: deterministic after the ordered reduction).
__global__ __launch_bounds__(256) void coulomb_vector_kernel(const double* Bf, const double* D, int64_t npairs,
                                                             int64_t naux, int64_t chunk, double* part,
                                                             const int32_t* status) {
  if (*status != 0) return;
  const int64_t P = (int64_t)blockIdx.x * 256 + threadIdx.x, z = blockIdx.y;
  if (P >= naux) return;
  const int64_t rs0 = z * chunk, rs1 = min(npairs, rs0 + chunk);
  double s = 0.0;
  for (int64_t rs = rs0; rs < rs1; ++rs) s += Bf[rs * naux + P] * D[rs];
  part[z * naux + P] = s;
}

// out[p][q] = 2 sum_P Bf[p][q][P] c[P] - K[p][q] for p < nrows (rows r0..),
// q < ncols (columns c0..); one wave per (p, q), lanes over P, fixed-order
// wave reduction.
__global__ __launch_bounds__(256) void antisym_combine_kernel(const double* Bf, int64_t nmo, int64_t naux,
                                                              int64_t r0, int64_t nrows, int64_t c0, int64_t ncols,
                                                              const double* c, const double* K, double* F,
                                                              int64_t ldf, const int32_t* status) {
  if (*status != 0) return;
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= nrows * ncols) return;
  const int64_t p = e / ncols, q = e - p * ncols;
  const double* row = Bf + ((r0 + p) * nmo + c0 + q) * naux;
  double s = 0.0;
  for (int64_t P = lane; P < naux; P += 64) s += row[P] * c[P];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) F[p * ldf + q] = 2.0 * s - K[p * ncols + q];
}

struct AntisymPlan {
  int64_t nmo, naux, nrows, ncols, chunks, chunk, s_k;
  size_t off_status, off_cpart, off_c, off_Y, off_Kp, off_K, total;
};

AntisymPlan antisym_plan(int64_t nmo, int64_t naux, int64_t nrows, int64_t ncols) {
  AntisymPlan A{};
  A.nmo = nmo; A.naux = naux; A.nrows = nrows; A.ncols = ncols;
  const int64_t npairs = nmo * nmo;
  A.chunks = std::max<int64_t>(1, std::min<int64_t>(256, npairs / 64));
  A.chunk = cdiv(npairs, A.chunks);
  A.chunks = cdiv(npairs, A.chunk);
  A.s_k = choose_splits(cdiv(nrows, kTile) * cdiv(ncols, kTile), nmo * naux);
  size_t off = 0;
  A.off_status = off; off = align_up(off + 64);
  A.off_cpart = off; off = align_up(off + 8 * (size_t)A.chunks * naux);
  A.off_c = off; off = align_up(off + 8 * (size_t)naux);
  A.off_Y = off; off = align_up(off + 8 * (size_t)nmo * ncols * naux);
  A.off_Kp = off; off = align_up(off + 8 * (size_t)A.s_k * nrows * ncols);
  A.off_K = off; off = align_up(off + 8 * (size_t)nrows * ncols);
  A.total = off;
  return A;
}

// F[p - r0][q - c0] (row stride ldf) = sum_rs G_pq^rs D_rs for the rows
// [r0, r0 + nrows) and columns [c0, c0 + ncols), with G_pq^rs = 2 (pq|rs) -
// (ps|rq) and (pq|rs) = sum_P Bf[p][q][P] Bf[r][s][P]:
//   Coulomb  2 sum_P Bf[p][q][P] c_P,   c_P = sum_rs Bf[r][s][P] D_rs
//   exchange sum_(s,P) Bf[p][s][P] Y[s][q][P],   Y[s][q][P] = sum_r D_rs Bf[r][q][P]
// The workspace's status word must be zero (the callers clear it).
int antisym_run(const AntisymPlan& A, const double* Bf, const double* D, int64_t r0, int64_t c0, double* F,
                int64_t ldf, char* ws, hipStream_t st) {
  const int64_t nmo = A.nmo, naux = A.naux, nrows = A.nrows, ncols = A.ncols;
  const int32_t* status = (const int32_t*)(ws + A.off_status);
  double* cpart = (double*)(ws + A.off_cpart);
  double* c = (double*)(ws + A.off_c);
  double* Y = (double*)(ws + A.off_Y);
  double* Kp = (double*)(ws + A.off_Kp);
  double* K = (double*)(ws + A.off_K);
  int rc;
  if ((rc = traced(R_RESPONSE, 0, 0, 8.0 * nmo * nmo * (naux + 1), st, [&] {
         hipLaunchKernelGGL(coulomb_vector_kernel, dim3((unsigned)cdiv(naux, 256), (unsigned)A.chunks), dim3(256), 0,
                            st, Bf, D, nmo * nmo, naux, A.chunk, cpart, status);
         hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)cdiv(naux, 256)), dim3(256), 0, st, c, naux,
                            (const double*)cpart, naux, naux, (int)A.chunks, (int64_t)1, naux, 1.0, 0, status);
       })))
    return rc;
  {  // Y[s][(q, P)] = sum_r D[r][s] Bf[r][c0 + q][P]
    GemmParams gp{};
    gp.M = nmo; gp.N = ncols * naux; gp.K = nmo; gp.kchunk = nmo;
    gp.Am = NOperand{D, nmo};
    gp.Bn = NOperand{Bf + c0 * naux, nmo * naux};
    gp.C = Y; gp.ldc = ncols * naux; gp.status = status;
    if ((rc = launch_gemm<128, 128, true, ROLE_AO, false>(gp, st, R_RESPONSE, 2.0 * nmo * nmo * ncols * naux,
                                                           8.0 * (nmo * nmo + 2.0 * nmo * ncols * naux), false)))
      return rc;
  }
  {  // K[p][q] = sum over (s, P) of Bf[r0 + p][s][P] Y[s][q][P]
    GemmParams gp{};
    gp.M = nrows; gp.N = ncols; gp.K = nmo * naux;
    gp.kchunk = cdiv(gp.K, A.s_k);
    gp.A = kop(Bf + r0 * nmo * naux, nmo * naux, INT64_MAX, 0);
    gp.Bk = kop(Y, naux, naux, ncols * naux);
    gp.C = Kp; gp.ldc = ncols; gp.split_stride = nrows * ncols; gp.status = status;
    const int64_t splits = cdiv(gp.K, cdiv(gp.kchunk, kBK) * kBK);
    if ((rc = launch_gemm<128, 128, false, ROLE_LTERM, false>(gp, st, R_RESPONSE, 2.0 * nrows * ncols * nmo * naux,
                                                               8.0 * (nrows + ncols) * nmo * naux, false)))
      return rc;
    const int64_t n = nrows * ncols;
    if ((rc = traced(R_REDUCE, 0, 0, 8.0 * (splits + 1) * n, st, [&] {
           hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, K, ncols,
                              (const double*)Kp, ncols, n, (int)splits, nrows, ncols, 1.0, 0, status);
         })))
      return rc;
  }
  return traced(R_RESPONSE, 0, 0, 8.0 * nrows * ncols * (naux + 2), st, [&] {
    hipLaunchKernelGGL(antisym_combine_kernel, dim3((unsigned)cdiv(nrows * ncols, 4)), dim3(256), 0, st, Bf, nmo, naux,
                       r0, nrows, c0, ncols, (const double*)c, (const double*)K, F, ldf, status);
  });
}

// D[nmo][nmo]: the blocks given (any may be null: zero); the occupied-virtual
// block is the transpose of D_vo when ov != 0, else zero; hf adds the
// identity on the occupied block.
__global__ __launch_bounds__(256) void assemble_density_kernel(int64_t nocc, int64_t nvir, const double* Doo,
                                                               const double* Dvv, const double* Dvo, int ov, int hf,
                                                               double* D) {
  const int64_t nmo = nocc + nvir, e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nmo * nmo) return;
  const int64_t p = e / nmo, q = e - p * nmo;
  double v = 0.0;
  if (p < nocc && q < nocc) v = Doo ? Doo[p * nocc + q] : 0.0;
  else if (p >= nocc && q >= nocc) v = Dvv ? Dvv[(p - nocc) * nvir + (q - nocc)] : 0.0;
  else if (p >= nocc) v = Dvo ? Dvo[(p - nocc) * nocc + q] : 0.0;
  else v = (Dvo && ov) ? Dvo[(q - nocc) * nocc + p] : 0.0;
  if (hf && p == q && p < nocc) v += 1.0;
  D[e] = v;
}

// Z-vector pieces, element (a, i) of [nvir][nocc].
//   mode 0: out = L2[a][i] - L1[i][nocc + a] - F[a][i]                (right-hand side)
//   mode 1: out = (eps_a - eps_i)/2 x[a][i] + F[a][i]                 (operator)
//   mode 2: out = (eps_a - eps_i)/2 + sum_P Bf[nocc+a][i][P]^2        (diagonal)
__global__ __launch_bounds__(256) void zvector_elem_kernel(int mode, int64_t nocc, int64_t nvir, int64_t naux,
                                                           const double* eo, const double* ev, const double* Bf,
                                                           const double* L1, const double* L2, const double* x,
                                                           const double* F, double* out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nocc * nvir) return;
  const int64_t a = e / nocc, i = e - a * nocc, nmo = nocc + nvir;
  const double gap = (ev[a] - eo[i]) / 2.0;
  if (mode == 0) {
    out[e] = (L2[a * nmo + i] - L1[i * nmo + nocc + a]) - F[e];
  } else if (mode == 1) {
    out[e] = gap * x[e] + F[e];
  } else {
    const double* row = Bf + ((nocc + a) * nmo + i) * naux;
    double s = 0.0;
    for (int64_t P = 0; P < naux; ++P) s += row[P] * row[P];
    out[e] = gap + s;
  }
}

// Sum over n of u[n] v[n] (w == null) or of u[n] v[n] / w[n], one workgroup,
// fixed order; written to out[0].
__global__ __launch_bounds__(256) void dot_kernel(const double* u, const double* v, const double* w, int64_t n,
                                                  double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) s += w ? u[k] * v[k] / w[k] : u[k] * v[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int wdt = 128; wdt > 0; wdt >>= 1) {
    if (threadIdx.x < wdt) sh[threadIdx.x] += sh[threadIdx.x + wdt];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// CG vector updates.
//   mode 0: y = u / w                       (preconditioned residual; initial guess)
//   mode 1: x += alpha p; r -= alpha q      (u = p, v = q, y = x, z = r)
//   mode 2: p = r / w + beta p              (u = r, y = p)
//   mode 3: y = u - v                       (initial residual)
__global__ __launch_bounds__(256) void cg_update_kernel(int mode, int64_t n, double alpha, const double* u,
                                                        const double* v, const double* w, double* y, double* z) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  if (mode == 0) y[k] = u[k] / w[k];
  else if (mode == 1) { y[k] += alpha * u[k]; z[k] -= alpha * v[k]; }
  else if (mode == 2) y[k] = u[k] / w[k] + alpha * y[k];
  else y[k] = u[k] - v[k];
}

// W[p][q] = (eps_p + eps_q)/2 D[p][q] + (p < nocc ? F[p][q] + L1[p][q] : L2[p - nocc][q]),
// D including the HF identity on the occupied block.
__global__ __launch_bounds__(256) void w_assemble_kernel(int64_t nocc, int64_t nvir, const double* eo,
                                                         const double* ev, const double* D, const double* F,
                                                         const double* L1, const double* L2, double* W) {
  const int64_t nmo = nocc + nvir, e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nmo * nmo) return;
  const int64_t p = e / nmo, q = e - p * nmo;
  const double ep = p < nocc ? eo[p] : ev[p - nocc], eq = q < nocc ? eo[q] : ev[q - nocc];
  double w = (ep + eq) / 2.0 * D[e];
  w += p < nocc ? F[e] + L1[e] : L2[(p - nocc) * nmo + q];
  W[e] = w;
}

struct ZPlan {
  AntisymPlan A;
  size_t off_D, off_F, off_rhs, off_diag, off_x, off_r, off_p, off_q, off_dot, total;
};

ZPlan zvector_plan(int64_t nocc, int64_t nvir, int64_t naux) {
  ZPlan Z{};
  const int64_t nmo = nocc + nvir, nov = nocc * nvir;
  Z.A = antisym_plan(nmo, naux, nvir, nocc);
  size_t off = Z.A.total;
  Z.off_D = off; off = align_up(off + 8 * (size_t)nmo * nmo);
  Z.off_F = off; off = align_up(off + 8 * (size_t)nov);
  Z.off_rhs = off; off = align_up(off + 8 * (size_t)nov);
  Z.off_diag = off; off = align_up(off + 8 * (size_t)nov);
  Z.off_x = off; off = align_up(off + 8 * (size_t)nov);
  Z.off_r = off; off = align_up(off + 8 * (size_t)nov);
  Z.off_p = off; off = align_up(off + 8 * (size_t)nov);
  Z.off_q = off; off = align_up(off + 8 * (size_t)nov);
  Z.off_dot = off; off = align_up(off + 64);
  Z.total = off;
  return Z;
}

int response_sizes(int32_t nocc, int32_t nvir, int32_t naux) {
  if (nocc < 1 || nvir < 1 || naux < 1) return fail(RIMP2_EINVAL, "sizes must be >= 1");
  const double nmo = (double)nocc + nvir;
  if (nmo * nmo * naux >= 4.6e18 || nmo > (1 << 20)) return fail(RIMP2_EINVAL, "sizes too large");
  return RIMP2_OK;
}

int clear_status(char* ws, hipStream_t st) {
  return traced(R_STATUS, 0, 0, 8.0, st, [&] {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, st, (unsigned long long*)ws, 1);
  });
}

int read_dot(const double* d, double* h, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return RIMP2_OK;
}

}  // namespace

int rimp2_antisym_workspace_size(int32_t nmo, int32_t naux, int32_t nrows, int32_t ncols, size_t* bytes) {
  if (!bytes) return fail(RIMP2_EINVAL, "bytes is NULL");
  if (nmo < 1 || naux < 1 || nrows < 1 || ncols < 1) return fail(RIMP2_EINVAL, "sizes must be >= 1");
  *bytes = antisym_plan(nmo, naux, nrows, ncols).total;
  return RIMP2_OK;
}

int rimp2_antisym_term(int32_t nmo, int32_t naux, int32_t r0, int32_t nrows, int32_t c0, int32_t ncols,
                       const double* Bf, const double* D, double* F, int64_t ldf, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (nmo < 1 || naux < 1 || nrows < 1 || ncols < 1 || r0 < 0 || c0 < 0 || (int64_t)r0 + nrows > nmo ||
      (int64_t)c0 + ncols > nmo || ldf < ncols)
    return fail(RIMP2_EINVAL, "rows [r0, r0 + nrows) and columns [c0, c0 + ncols) must lie in [0, nmo), ldf >= ncols");
  if (!Bf || !D || !F || !workspace) return fail(RIMP2_EINVAL, "Bf, D, F and workspace must not be NULL");
  if ((uintptr_t)workspace % kAlign) return fail(RIMP2_EWORKSPACE, "workspace must be 256-byte aligned");
  const AntisymPlan A = antisym_plan(nmo, naux, nrows, ncols);
  if (workspace_bytes < A.total) return fail(RIMP2_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, A.total);
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = clear_status((char*)workspace, st))) return rc;
  return antisym_run(A, Bf, D, r0, c0, F, ldf, (char*)workspace, st);
}

int rimp2_zvector_workspace_size(int32_t nocc, int32_t nvir, int32_t naux, size_t* bytes) {
  if (!bytes) return fail(RIMP2_EINVAL, "bytes is NULL");
  int rc;
  if ((rc = response_sizes(nocc, nvir, naux))) return rc;
  *bytes = zvector_plan(nocc, nvir, naux).total;
  return RIMP2_OK;
}

int rimp2_zvector(int32_t nocc, int32_t nvir, int32_t naux, const double* Bf, const double* eps_occ,
                  const double* eps_vir, const double* P_ij, const double* P_ab, const double* L1, const double* L2,
                  double* D_ai, double tol, int32_t max_iter, int32_t* iterations, double* rel_residual,
                  void* workspace, size_t workspace_bytes, void* stream) {
  int rc;
  if ((rc = response_sizes(nocc, nvir, naux))) return rc;
  if (!Bf || !eps_occ || !eps_vir || !P_ij || !P_ab || !L1 || !L2 || !D_ai || !workspace)
    return fail(RIMP2_EINVAL, "Bf, eps_occ, eps_vir, P_ij, P_ab, L1, L2, D_ai and workspace must not be NULL");
  if (!(tol > 0.0) || max_iter < 1) return fail(RIMP2_EINVAL, "tol must be > 0 and max_iter >= 1");
  if ((uintptr_t)workspace % kAlign) return fail(RIMP2_EWORKSPACE, "workspace must be 256-byte aligned");
  const ZPlan Z = zvector_plan(nocc, nvir, naux);
  if (workspace_bytes < Z.total) return fail(RIMP2_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, Z.total);
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const int64_t no = nocc, nv = nvir, na = naux, nmo = no + nv, nov = no * nv;
  double* D = (double*)(ws + Z.off_D);
  double* F = (double*)(ws + Z.off_F);
  double* rhs = (double*)(ws + Z.off_rhs);
  double* diag = (double*)(ws + Z.off_diag);
  double* r = (double*)(ws + Z.off_r);
  double* pv = (double*)(ws + Z.off_p);
  double* q = (double*)(ws + Z.off_q);
  double* dot = (double*)(ws + Z.off_dot);
  double* x = D_ai;
  const unsigned gn = (unsigned)cdiv(nov, 256), gd = (unsigned)cdiv(nmo * nmo, 256);
  auto elem = [&](int mode, const double* xin, double* out) {
    return traced(R_RESPONSE, 0, 0, 8.0 * 3 * nov, st, [&] {
      hipLaunchKernelGGL(zvector_elem_kernel, dim3(gn), dim3(256), 0, st, mode, no, nv, na, eps_occ, eps_vir, Bf, L1,
                         L2, xin, (const double*)F, out);
    });
  };
  auto density = [&](const double* Doo, const double* Dvv, const double* Dvo) {
    return traced(R_RESPONSE, 0, 0, 8.0 * nmo * nmo, st, [&] {
      hipLaunchKernelGGL(assemble_density_kernel, dim3(gd), dim3(256), 0, st, no, nv, Doo, Dvv, Dvo, 0, 0, D);
    });
  };
  // out = (eps_a - eps_i)/2 v_ai + sum_bj G_ai^bj v_bj (only the (b, j) block of D holds v)
  auto apply = [&](const double* v, double* out) -> int {
    int r2;
    if ((r2 = density(nullptr, nullptr, v))) return r2;
    if ((r2 = antisym_run(Z.A, Bf, D, no, 0, F, no, ws, st))) return r2;
    return elem(1, v, out);
  };
  auto dotp = [&](const double* u, const double* v, const double* w, double* h) -> int {
    int r2;
    if ((r2 = traced(R_RESPONSE, 0, 0, 16.0 * nov, st, [&] {
           hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(256), 0, st, u, v, w, nov, dot);
         })))
      return r2;
    return read_dot(dot, h, st);
  };
  auto update = [&](int mode, double alpha, const double* u, const double* v, const double* w, double* y,
                    double* z) {
    return traced(R_RESPONSE, 0, 0, 8.0 * 4 * nov, st, [&] {
      hipLaunchKernelGGL(cg_update_kernel, dim3(gn), dim3(256), 0, st, mode, nov, alpha, u, v, w, y, z);
    });
  };
  if ((rc = clear_status(ws, st))) return rc;
  // right-hand side: L''_ai - L'_ia - sum_pq G_ai^pq Dbar_pq, Dbar = D_ij (+) D_ab
  if ((rc = density(P_ij, P_ab, nullptr))) return rc;
  if ((rc = antisym_run(Z.A, Bf, D, no, 0, F, no, ws, st))) return rc;
  if ((rc = elem(0, nullptr, rhs))) return rc;
  if ((rc = elem(2, nullptr, diag))) return rc;   // Jacobi preconditioner: the operator's diagonal
  // preconditioned conjugate gradients from x = rhs / diag
  double bb = 0.0, rz = 0.0, rr = 0.0;
  if ((rc = dotp(rhs, rhs, nullptr, &bb))) return rc;
  if ((rc = update(0, 0.0, rhs, nullptr, diag, x, nullptr))) return rc;
  if ((rc = apply(x, q))) return rc;
  if ((rc = update(3, 0.0, rhs, q, nullptr, r, nullptr))) return rc;
  if ((rc = update(0, 0.0, r, nullptr, diag, pv, nullptr))) return rc;
  if ((rc = dotp(r, r, diag, &rz))) return rc;
  if ((rc = dotp(r, r, nullptr, &rr))) return rc;
  const double target = tol * tol * bb;
  int it = 0;
  while (rr > target && it < max_iter) {
    if ((rc = apply(pv, q))) return rc;
    double pq = 0.0;
    if ((rc = dotp(pv, q, nullptr, &pq))) return rc;
    if (!(pq > 0.0)) break;   // the operator is not positive definite along p
    const double alpha = rz / pq;
    if ((rc = update(1, alpha, pv, q, nullptr, x, r))) return rc;
    double rz_new = 0.0;
    if ((rc = dotp(r, r, diag, &rz_new))) return rc;
    if ((rc = dotp(r, r, nullptr, &rr))) return rc;
    if ((rc = update(2, rz_new / rz, r, nullptr, diag, pv, nullptr))) return rc;
    rz = rz_new;
    ++it;
  }
  if (iterations) *iterations = it;
  const double rel_res = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
  if (rel_residual) *rel_residual = rel_res;
  if (!(rr <= target))
    return fail(RIMP2_ENOCONV, "Z-vector CG stopped after %d iterations at relative residual %.3e (tol %.3e)", it,
                rel_res, tol);
  return RIMP2_OK;
}

int rimp2_energy_weighted_density_workspace_size(int32_t nocc, int32_t nvir, int32_t naux, size_t* bytes) {
  if (!bytes) return fail(RIMP2_EINVAL, "bytes is NULL");
  int rc;
  if ((rc = response_sizes(nocc, nvir, naux))) return rc;
  const int64_t nmo = (int64_t)nocc + nvir;
  const AntisymPlan A = antisym_plan(nmo, naux, nocc, nmo);
  *bytes = A.total + align_up(8 * (size_t)nmo * nmo) * 2;
  return RIMP2_OK;
}

int rimp2_energy_weighted_density(int32_t nocc, int32_t nvir, int32_t naux, const double* Bf, const double* eps_occ,
                                  const double* eps_vir, const double* P_ij, const double* P_ab, const double* D_ai,
                                  const double* L1, const double* L2, double* W, void* workspace,
                                  size_t workspace_bytes, void* stream) {
  int rc;
  if ((rc = response_sizes(nocc, nvir, naux))) return rc;
  if (!Bf || !eps_occ || !eps_vir || !P_ij || !P_ab || !D_ai || !L1 || !L2 || !W || !workspace)
    return fail(RIMP2_EINVAL, "Bf, eps_occ, eps_vir, P_ij, P_ab, D_ai, L1, L2, W and workspace must not be NULL");
  if ((uintptr_t)workspace % kAlign) return fail(RIMP2_EWORKSPACE, "workspace must be 256-byte aligned");
  size_t need = 0;
  if ((rc = rimp2_energy_weighted_density_workspace_size(nocc, nvir, naux, &need))) return rc;
  if (workspace_bytes < need) return fail(RIMP2_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const int64_t no = nocc, nv = nvir, nmo = no + nv;
  const AntisymPlan A = antisym_plan(nmo, naux, nocc, nmo);
  double* Dm = (double*)(ws + A.total);
  double* F = (double*)(ws + A.total + align_up(8 * (size_t)nmo * nmo));
  const unsigned gd = (unsigned)cdiv(nmo * nmo, 256);
  if ((rc = clear_status(ws, st))) return rc;
  // D^MP2 (every block) for the antisymmetrised term of the occupied rows
  if ((rc = traced(R_RESPONSE, 0, 0, 8.0 * nmo * nmo, st, [&] {
         hipLaunchKernelGGL(assemble_density_kernel, dim3(gd), dim3(256), 0, st, no, nv, P_ij, P_ab, D_ai, 1, 0, Dm);
       })))
    return rc;
  if ((rc = antisym_run(A, Bf, Dm, 0, 0, F, nmo, ws, st))) return rc;
  // D = D^HF + D^MP2 for the energy-weighted piece
  if ((rc = traced(R_RESPONSE, 0, 0, 8.0 * nmo * nmo, st, [&] {
         hipLaunchKernelGGL(assemble_density_kernel, dim3(gd), dim3(256), 0, st, no, nv, P_ij, P_ab, D_ai, 1, 1, Dm);
       })))
    return rc;
  return traced(R_RESPONSE, 0, 0, 8.0 * 4 * nmo * nmo, st, [&] {
    hipLaunchKernelGGL(w_assemble_kernel, dim3(gd), dim3(256), 0, st, no, nv, eps_occ, eps_vir, (const double*)Dm,
                       (const double*)F, L1, L2, W);
  });
}

}  // extern "C"
