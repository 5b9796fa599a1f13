/*
 * rimp2_gradient.h -- steps adjacent to the RI-MP2 fragment kernel on the
 * way to the gradient (gfx950).  Same conventions as rimp2.h: device
 * pointers, caller-owned buffers, `stream` is a hipStream_t as void*,
 * asynchronous, negative rimp2_status on host-detected argument errors.
 */
#ifndef RIMP2_GRADIENT_H
#define RIMP2_GRADIENT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * The Appendix's Gamma^P_ia = sum_{bjQ} (2 X_ij^ab - X_ij^ba) B^Q_jb J^{-1/2}_PQ,
 * formed from the fragment kernel's Gamma (taken before this contraction):
 *
 *   out[i][a][P] = sum_Q Gamma[i][a][Q] Jm[P][Q]
 *
 *   Gamma  device, read  [nocc][nvir][naux]  (rimp2_fragment's Gamma)
 *   Jm     device, read  [naux][naux]        the metric factor J^{-1/2}
 *                                            (symmetric in the paper; used as given)
 *   out    device, write [nocc][nvir][naux]  must not overlap Gamma
 * FP64 MFMA GEMM (M = nocc*nvir, N = K = naux).  With B = B3 J^{-1/2}, out is a
 * quarter of the derivative of E_MP2 with respect to the three-centre
 * integrals B3.
 */
int rimp2_gamma_metric(int32_t nocc, int32_t nvir, int32_t naux, const double* Gamma, const double* Jm,
                       double* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RIMP2_GRADIENT_H */
