// Steps adjacent to the fragment kernel on the way to the gradient
// (include/rimp2_gradient.h): the metric contraction of Gamma.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rimp2.h"
#include "../../include/rimp2_gradient.h"
#include "common.hpp"
#include "gemm_f64.hpp"

using namespace rimp2;

namespace {
int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }
}  // namespace

extern "C" int rimp2_gamma_metric(int32_t nocc, int32_t nvir, int32_t naux, const double* Gamma, const double* Jm,
                                  double* out, void* stream) {
  if (nocc < 1 || nvir < 1 || naux < 1) return fail(RIMP2_EINVAL, "sizes must be >= 1");
  if (!Gamma || !Jm || !out) return fail(RIMP2_EINVAL, "Gamma, Jm and out must not be NULL");
  const int64_t M = (int64_t)nocc * nvir, n = naux;
  const char *g0 = (const char*)Gamma, *g1 = (const char*)(Gamma + M * n), *o0 = (const char*)out,
             *o1 = (const char*)(out + M * n);
  if (o0 < g1 && g0 < o1) return fail(RIMP2_EINVAL, "out must not overlap Gamma");
  GemmParams gp{};
  gp.M = M; gp.N = n; gp.K = n; gp.kchunk = n;
  gp.A = KOperand{Gamma, n, INT64_MAX, 0};   // row (i,a), reduction Q
  gp.Bk = KOperand{Jm, n, INT64_MAX, 0};     // row P, reduction Q
  gp.C = out; gp.ldc = n; gp.split_stride = 0; gp.status = nullptr;
  gp.tiles_m = (int32_t)cdiv64(M, 128); gp.tiles_n = (int32_t)cdiv64(n, 128); gp.group_m = 8; gp.splits = 1;
  gp.kchunk = cdiv64(n, 16) * 16;
  const int64_t nwg = (int64_t)gp.tiles_m * gp.tiles_n;
  if (nwg > 0xffffffffLL / 256) return fail(RIMP2_EINVAL, "grid too large");
  const bool vec = (uintptr_t)Gamma % 16 == 0 && (uintptr_t)Jm % 16 == 0 && n % 2 == 0;
  hipStream_t st = (hipStream_t)stream;
  if (vec)   // the loader running two chunks ahead (n is even, both operands plain)
    hipLaunchKernelGGL((gemm_f64_kernel<128, 128, 16, false, ROLE_GAMMA, true, false, 1>), dim3((unsigned)nwg),
                       dim3(256), 0, st, gp);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<128, 128, 16, false, ROLE_GAMMA, false, false>), dim3((unsigned)nwg),
                       dim3(256), 0, st, gp);
  HIP_TRY(hipGetLastError());
  return RIMP2_OK;
}
