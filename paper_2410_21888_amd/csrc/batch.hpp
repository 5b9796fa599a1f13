// Grouped kernels for batches of fragments: one launch per step covers every
// fragment of a wave.  Per-fragment descriptors live in device tables built
// once on the host; pointers into the caller's workspace are stored as
// offsets tagged with bit 62 and relocated against the workspace base by
// relocate_tables_kernel at the start of each run, so the host tables never
// change after planning (and a captured graph replays them unchanged).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f64.hpp"
#include "kernels.hpp"

namespace rimp2 {

constexpr uint64_t kRelTag = 1ull << 62;

__device__ __forceinline__ void reloc(const void*& p, char* base) {
  const uint64_t v = (uint64_t)p;
  if (v & kRelTag) p = base + (v & (kRelTag - 1));
}
template <class T>
__device__ __forceinline__ void reloc_t(T*& p, char* base) {
  const void* q = p;
  reloc(q, base);
  p = (T*)q;
}

struct AmpDesc {
  double* V;
  double* T;
  const double* eo;
  const double* ev;
  double* e_pair;
  const int32_t* status;
  int32_t nocc, nvir, energy_only;
};
struct ReduceDesc {
  double* out;
  const double* W;
  const int32_t* status;
  int64_t ldo, ldw, zs, M, N;
  double alpha;
  int32_t splits, accumulate;
};
struct FragSmall {       // gap check, energy sum and status copy
  const double* eo;
  const double* ev;
  const double* e_pair;
  double* E;
  int32_t* status;
  int32_t nocc, nvir;
};

// Relocates every tagged pointer of the tables (one thread per entry).
__global__ void relocate_tables_kernel(char* base, GemmParams* gp, int ngp, AmpDesc* amp, int namp, ReduceDesc* red,
                                       int nred, FragSmall* fs, int nfs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ngp) {
    GemmParams& p = gp[i];
    reloc_t(p.A.base, base); reloc_t(p.Am.base, base); reloc_t(p.Bk.base, base); reloc_t(p.Bn.base, base);
    reloc_t(p.C, base); reloc_t(p.status, base);
  }
  if (i < namp) {
    AmpDesc& d = amp[i];
    reloc_t(d.V, base); reloc_t(d.T, base); reloc_t(d.e_pair, base); reloc_t(d.status, base);
  }
  if (i < nred) {
    ReduceDesc& r = red[i];
    reloc_t(r.out, base); reloc_t(r.W, base); reloc_t(r.status, base);
  }
  if (i < nfs) {
    FragSmall& f = fs[i];
    reloc_t(f.e_pair, base); reloc_t(f.status, base);
  }
}

__global__ void zero_counters_kernel(unsigned long long* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0ull;
}

// last f with prefix[f] <= t
__device__ __forceinline__ int find_problem(const int64_t* prefix, int n, int64_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void gap_check_grouped(const FragSmall* fs) {
  const FragSmall f = fs[blockIdx.x];
  gap_check_block(f.eo, f.nocc, f.ev, f.nvir, f.status);
}

// one workgroup per occupied pair of every fragment (whole slab, k0 = 0,
// blocks j < k not computed by the (ia|jb) GEMM: mirrored)
__global__ __launch_bounds__(256) void amplitude_grouped(const AmpDesc* descs, const int64_t* prefix, int n) {
  const int f = find_problem(prefix, n, blockIdx.x);
  const AmpDesc d = descs[f];
  if (*d.status != 0) return;
  const int64_t u = blockIdx.x - prefix[f];
  const int kk = (int)(u / d.nocc), j = (int)(u - (int64_t)kk * d.nocc);
  amplitude_block(d.V, d.T, d.eo, d.ev, d.nocc, d.nvir, 0, 0, d.nocc, 2, d.nocc, d.energy_only, nullptr, d.e_pair, kk,
                  j, 0, 1, nullptr);
}

// prefix counts 256-element blocks per problem
__global__ __launch_bounds__(256) void reduce_grouped(const ReduceDesc* descs, const int64_t* prefix, int n) {
  const int f = find_problem(prefix, n, blockIdx.x);
  const ReduceDesc r = descs[f];
  if (*r.status != 0) return;
  const int64_t idx = (blockIdx.x - prefix[f]) * 256 + threadIdx.x;
  splitk_reduce_at(r.out, r.ldo, r.W, r.ldw, r.zs, r.splits, r.M, r.N, r.alpha, r.accumulate, idx);
}

__global__ __launch_bounds__(256) void energy_sum_grouped(const FragSmall* fs) {
  const FragSmall f = fs[blockIdx.x];
  if (*f.status != 0) return;
  energy_sum_block(f.e_pair, (int64_t)f.nocc * f.nocc, f.E);
}

__global__ void status_copy_grouped(const FragSmall* fs, const int32_t* index, int n, int32_t* status_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) status_out[index[i]] = *fs[i].status;
}

}  // namespace rimp2
