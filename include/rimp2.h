/*
 * rimp2.h -- C ABI of the MI355X (gfx950) closed-shell RI-MP2 fragment kernel.
 *
 * What is computed (arXiv 2410.21888; restricted closed shell, no frozen core,
 * Sec. "Background"):
 *
 *   (ia|jb) = sum_P B^P_ia B^P_jb                       (Eq. MP2_ints)
 *   X_ij^ab = (ia|jb) / (eps_i + eps_j - eps_a - eps_b)  (Appendix, amplitudes)
 *   T_ij^ab = 2 X_ij^ab - X_ij^ba
 *   e_ij    = sum_ab T_ij^ab (ia|jb),  E = sum_ij e_ij   (RI-MP2 fragment energy
 *                                                         of Eq. efrag)
 *   Gamma^P_ia = sum_jb T_ij^ab B^P_jb                  (Appendix, Gamma, before
 *                                                         its J^{-1/2} contraction)
 *   P_ij = -sum_kab T_ik^ab X_jk^ab                      (Appendix, D^MP2_ij)
 *   P_ab =  sum_ijc T_ij^ac X_ij^bc                      (Appendix, D^MP2_ab)
 *
 * All arithmetic is IEEE FP64 unless opts->precision selects split products
 * (rimp2_precision).  P_ij and P_ab are formed from their upper triangles and
 * are exactly symmetric.  Results are deterministic: the same inputs and
 * options on the same GPU give bitwise identical outputs (no floating-point
 * atomics; the in-situ autotuner changes tile shapes only, and the GEMM
 * operand loader (opts->gemm_loader) only how operands reach LDS, never a
 * summation order, so neither changes a result bit).
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" are HIP device pointers; the caller owns every
 *    buffer.  The library allocates no device memory: scratch space comes in
 *    through the caller's workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it and the call returns without synchronising.
 *  - Return value: RIMP2_OK, or a negative rimp2_status for an argument error
 *    detected on the host (nothing is enqueued then).  rimp2_last_error()
 *    returns a message for the calling thread's last non-OK return.
 *  - Conditions only the device can see (an orbital-energy gap that would make
 *    a denominator >= 0, or a NaN orbital energy) are written as RIMP2_EGAP to
 *    the device status word in the workspace; every kernel of the call then
 *    does nothing and the outputs are left unwritten.  Read it with
 *    rimp2_read_status() after the stream has run the call.
 *  - Layouts are row-major with the last index fastest:
 *      B, Gamma  [nocc][nvir][naux]     eps_occ [nocc]    eps_vir [nvir]
 *      P_ij, e_pair [nocc][nocc]        P_ab [nvir][nvir] E [2] = (hi, lo)
 *  - Sizes: 1 <= nocc, nvir, naux and nocc*nvir*naux < 2^62.
 */
#ifndef RIMP2_H
#define RIMP2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RIMP2_OK = 0,
  RIMP2_EINVAL = -1,     /* bad size, null required pointer, bad option */
  RIMP2_ENOMEM = -2,     /* workspace smaller than rimp2_workspace_size() */
  RIMP2_EWORKSPACE = -3, /* workspace pointer misaligned (needs 256 B) */
  RIMP2_EDEVICE = -4,    /* a HIP runtime call failed (message says which) */
  RIMP2_EGAP = -5,       /* device: max eps_occ >= min eps_vir, or NaN eps */
  RIMP2_ENOTSUP = -6,    /* option combination not supported */
  RIMP2_ENOCONV = -7     /* an iterative solve stopped before its tolerance */
} rimp2_status;

/* Arithmetic of the two large contractions, (ia|jb) and Gamma. */
typedef enum {
  RIMP2_FP64 = 0,       /* FP64 MFMA throughout */
  RIMP2_SPLIT_INT8 = 1  /* (ia|jb) and Gamma as split products (Ozaki scheme):
                           each FP64 row is scaled by a power of two and cut
                           into S signed 7-bit digits; the S(S+1)/2 digit
                           products that matter are summed exactly in INT32 on
                           INT8 MFMA and combined in FP64.  Denominators,
                           amplitudes, E, P_ij and P_ab stay FP64.  The error
                           of a product is about 2^-7S relative to its
                           operands' row maxima. */
} rimp2_precision;

typedef struct {
  int32_t precision;        /* rimp2_precision */
  int32_t split_slices;     /* RIMP2_SPLIT_INT8: digits per operand of (ia|jb),
                               3..7 (0 = 7) */
  int32_t slab_group;       /* occupied orbitals per slab group, 0 = largest that
                               fits slab_budget_bytes (see rimp2_workspace_size) */
  int32_t split_slices_gamma; /* RIMP2_SPLIT_INT8: digits per operand of Gamma,
                               3..7 (0 = 5) */
  size_t  slab_budget_bytes;/* cap on the slab part of the workspace when
                               slab_group == 0; 0 = 64 GiB */
  const uint8_t* pair_skip; /* device [nocc][nocc] or NULL: a nonzero (i,j) or
                               (j,i) marks the unordered occupied pair {i,j}
                               as screened out: its (ia|jb) blocks are not
                               formed, e_ij = e_ji = 0, and X_ij = T_ij = 0 in
                               Gamma and P (screening) */
  int32_t autotune;         /* nonzero: choose each FP64 GEMM's tile shape in situ
                               (rimp2_autotune_report); 0 = fixed shapes */
  int32_t gemm_loader;      /* 0: each FP64 GEMM takes the fastest operand
                               loader its shape allows; 1: the general loader
                               only.  Both sum every element in the same order,
                               so results are bitwise identical; 1 is for
                               comparison.  Other values: RIMP2_EINVAL. */
} rimp2_opts;

/* Library version, major*10000 + minor*100 + patch. */
int rimp2_version(void);

/* Message for the calling thread's last non-OK return (never NULL). */
const char* rimp2_last_error(void);

/* Name of a rimp2_status value. */
const char* rimp2_status_string(int status);

/*
 * Bytes of device workspace rimp2_fragment needs for these sizes, outputs and
 * options.  `want` is a bit set of RIMP2_WANT_* naming the outputs the call
 * will request; the workspace for a call must be at least this large for the
 * same `want` and options.  `opts` may be NULL (defaults).
 */
enum { RIMP2_WANT_GAMMA = 1, RIMP2_WANT_DENSITY = 2 };
int rimp2_workspace_size(int32_t nocc, int32_t nvir, int32_t naux, int32_t want,
                         const rimp2_opts* opts, size_t* bytes);

/*
 * One fragment.
 *   B        device, read  [nocc][nvir][naux]   three-index factor B^P_ia
 *   eps_occ  device, read  [nocc]               occupied orbital energies
 *   eps_vir  device, read  [nvir]               virtual orbital energies
 *   E        device, write [2]                  E_MP2 as hi + lo, where hi is
 *            the sum rounded to FP64 and lo the rounded remainder (compensated,
 *            fixed-order summation of the e_ij)
 *   Gamma    device, write [nocc][nvir][naux] or NULL (not computed)
 *   P_ij     device, write [nocc][nocc] or NULL (P_ij and P_ab are computed
 *   P_ab     device, write [nvir][nvir] or NULL  together: both or neither)
 *   e_pair   device, write [nocc][nocc] or NULL: e_ij for every ordered pair
 *   workspace, workspace_bytes: device scratch, 256-byte aligned, at least
 *            rimp2_workspace_size() bytes; its content on entry is ignored
 * With opts->pair_skip set, e_ij of a skipped pair is 0 and the pair adds
 * nothing to E, Gamma or P.
 * With Gamma and without P, every unordered pair's (ia|jb) block is formed
 * once (pairs j >= k in each slab group) and Gamma takes each pair's block
 * for both of its orbitals (T_ji = T_ij^T), in FP64 and in split precision;
 * with P, the slab groups hold every ordered pair.
 */
int rimp2_fragment(int32_t nocc, int32_t nvir, int32_t naux,
                   const double* B, const double* eps_occ, const double* eps_vir,
                   double* E, double* Gamma, double* P_ij, double* P_ab, double* e_pair,
                   void* workspace, size_t workspace_bytes,
                   const rimp2_opts* opts, void* stream);

/*
 * rimp2_fragment without a workspace argument and without any allocation,
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * The scratch space is a fixed array of RIMP2_NOALLOC_SCRATCH_BYTES (256 MiB)
 * inside the library's device code: each GPU that runs the library holds its
 * own copy from the first call on that device until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree, events or host tables): its
 * plan takes the largest slab group whose workspace fits the array (or
 * opts->slab_group when given), and a fragment whose workspace does not fit
 * even with one occupied orbital per group returns RIMP2_ENOMEM.
 * opts->autotune is not available here (RIMP2_ENOTSUP), and the timing of
 * rimp2_timing_enable records nothing for this call.
 *
 * Every call on one GPU shares that GPU's array and finds the previous
 * call's contents in it; no kernel relies on its initial contents (every
 * word is written before it is read within a call).  Calls that overlap on
 * one GPU -- on different streams, or from different host threads -- race
 * on the array and give undefined results: serialise them.
 *
 *   status_dev  device, write [1] or NULL: receives the call's device status
 *               (RIMP2_OK or RIMP2_EGAP) when the stream reaches the end of
 *               the call; the other arguments are those of rimp2_fragment.
 */
#define RIMP2_NOALLOC_SCRATCH_BYTES (256ull << 20)
int rimp2_fragment_noalloc(int32_t nocc, int32_t nvir, int32_t naux,
                           const double* B, const double* eps_occ, const double* eps_vir,
                           double* E, double* Gamma, double* P_ij, double* P_ab, double* e_pair,
                           int32_t* status_dev, const rimp2_opts* opts, void* stream);

/*
 * Read the device status word of the last call that used this workspace
 * (synchronises `stream` first).  Writes RIMP2_OK or RIMP2_EGAP to *status.
 */
int rimp2_read_status(const void* workspace, void* stream, int32_t* status);

/* One fragment of a batch.  Pointers are device pointers as in rimp2_fragment;
   Gamma, P_ij, P_ab and e_pair may be NULL. */
typedef struct {
  int32_t nocc, nvir, naux, reserved;
  const double* B;
  const double* eps_occ;
  const double* eps_vir;
  double* E;
  double* Gamma;
  double* P_ij;
  double* P_ab;
  double* e_pair;
} rimp2_frag_desc;

/*
 * Many independent fragments (the monomers, dimers and trimers of an MBE3
 * step; Sec. "Molecular Fragmentation", Eq. mbe3, and the largest-first
 * ordering of Sec. "Asynchronous time steps").
 *
 * Planning (rimp2_batch_create) sorts the fragments largest first (by FLOPs).
 * A fragment whose whole slab (all its occupied pairs) fits the wave budget
 * (opts->slab_budget_bytes, default 64 GiB) is packed into a wave; each step
 * of a wave -- gap check, (ia|jb), amplitudes, Gamma, P_ab, P_ij, reductions,
 * E -- is ONE grouped launch over all of its fragments (the GEMMs are
 * persistent launches whose workgroups take (fragment, tile) items from a
 * counter, largest fragment first).  Larger fragments run alone, as
 * rimp2_fragment does.  With opts->precision = RIMP2_SPLIT_INT8 the (ia|jb)
 * and Gamma products of a wave are grouped split products (one persistent
 * launch per reduction window of 2816 over all fragments of the wave), after
 * grouped digit splits (one launch per split step over the wave); P_ab and
 * P_ij stay FP64.  pair_skip must be NULL.  With opts->autotune the grouped FP64 GEMM
 * launches and the fragments that run alone are tuned in situ (see
 * rimp2_autotune_report).
 *
 *   descs    HOST array of nfrag descriptors; the handle keeps a copy, and the
 *            device buffers they name must stay valid while the handle is used
 *   *batch   receives the handle
 *   *workspace_bytes  receives the workspace size rimp2_batch_run needs
 *
 * rimp2_batch_run enqueues the whole batch on `stream` without host
 * synchronisation: it copies the handle's tables (pinned host memory written
 * once by rimp2_batch_create) into the workspace with hipMemcpyAsync and then
 * launches only kernels, so the call can be captured into a hipGraph and the
 * graph replayed while the handle lives.  status_dev (device, [nfrag] int32,
 * may be NULL) receives each fragment's status (RIMP2_OK or RIMP2_EGAP).
 */
typedef struct rimp2_batch_s* rimp2_batch;
int rimp2_batch_create(int32_t nfrag, const rimp2_frag_desc* descs, const rimp2_opts* opts,
                       rimp2_batch* batch, size_t* workspace_bytes);
int rimp2_batch_run(rimp2_batch batch, int32_t* status_dev, void* workspace,
                    size_t workspace_bytes, void* stream);
int rimp2_batch_destroy(rimp2_batch batch);

/*
 * One-shot convenience over the calls above: plans, synchronises `stream`
 * once, uploads the tables synchronously and enqueues the batch (the host
 * tables are freed before returning).  rimp2_batch_workspace_size returns the
 * workspace it needs for the same descriptors and options.
 */
int rimp2_batch_workspace_size(int32_t nfrag, const rimp2_frag_desc* descs,
                               const rimp2_opts* opts, size_t* bytes);
int rimp2_fragment_batch(int32_t nfrag, const rimp2_frag_desc* descs, int32_t* status_dev,
                         void* workspace, size_t workspace_bytes,
                         const rimp2_opts* opts, void* stream);

/*
 * Kernel timing (tracing).  While enabled, every kernel launch of the library
 * is bracketed by a pair of HIP events recorded on the launch's own stream,
 * and tagged with its role and its algorithmic FLOP and byte counts (FLOPs:
 * 2 per multiply-add, (ia|jb) counted over unordered occupied pairs; bytes:
 * compulsory HBM reads and writes of its operands).  rimp2_timing_collect
 * waits for the recorded events, returns one entry per role with the summed
 * event durations, and clears the records.  Timing adds a few microseconds
 * per launch.
 */
typedef struct {
  char    name[32];     /* kernel role, e.g. "ints_gemm", "gamma_gemm" */
  int64_t launches;
  double  total_ms;     /* sum of event durations over those launches */
  double  alg_flops;    /* algorithmic FLOPs of those launches */
  double  exec_flops;   /* multiply-add FLOPs the kernels execute */
  double  alg_bytes;    /* algorithmic HBM bytes of those launches */
} rimp2_kernel_stat;

/* enable != 0 starts recording (and discards earlier records); 0 stops. */
int rimp2_timing_enable(int enable);
/* Writes up to `capacity` entries to `stats` and their number to *count. */
int rimp2_timing_collect(rimp2_kernel_stat* stats, int32_t capacity, int32_t* count);

/*
 * In-situ GEMM autotuning (Sec. "GEMM runtime auto-tuning": each variant of a
 * GEMM shape is timed with HIP events on real calls, then the fastest is used
 * for every later call of that shape).  Here the variants are the output tile
 * shapes of the FP64 MFMA GEMMs of rimp2_fragment (and of the fragments a
 * batch runs alone), not transposed operand layouts: the slab layout already
 * fixes the operands.  A shape is (role, M, N, K, split length, 16-byte-load
 * eligibility) on one device.  With opts->autotune set, the first launches of
 * a shape run each candidate twice, bracketed by events on the launch's
 * stream; the host never waits for them, and once every candidate's events
 * have completed (checked without blocking at the next launch of the shape),
 * the candidate with the smallest time is used from then on.  Until then
 * launches use the fixed default.  Nothing is trialled while the stream is
 * being captured into a graph.  The tile shape does not change the order in
 * which any output element is summed, so results are bitwise identical
 * whichever candidate runs.  The table is process-wide and thread-safe.
 *
 * Batches (rimp2_batch_run with opts->autotune set at rimp2_batch_create):
 * each grouped GEMM launch of a wave has two candidate tiles, listed in the
 * handle's tables for both, and is tuned the same way; its entry has vec = 2,
 * M = fragments in the wave, N and K = work items of the two candidates and
 * kchunk = a hash of the wave's fragment sizes, so handles built again for
 * the same fragments (a later time step) reuse the decision.
 */
typedef struct {
  char    role[32];      /* "ints_gemm", "gamma_gemm", "pab_gemm", "pij_gemm" */
  int32_t device;
  int32_t nvar;          /* candidates */
  int32_t best;          /* chosen candidate, -1 while trials are pending */
  int32_t vec;           /* 16-byte loads eligible (2: grouped batch launch) */
  int64_t M, N, K, kchunk;
  int32_t tile_m[4], tile_n[4];   /* candidate tile shapes, [0] = default */
  int32_t timed[4];      /* completed trials per candidate */
  double  min_ms[4];     /* fastest completed trial per candidate */
  int64_t uses;          /* launches of this shape so far */
} rimp2_tune_stat;

/* Writes up to `capacity` entries to `stats` and the number written to *count
   (polls pending trials first, without blocking). */
int rimp2_autotune_report(rimp2_tune_stat* stats, int32_t capacity, int32_t* count);
/* Forgets every shape and decision. */
int rimp2_autotune_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* RIMP2_H */
