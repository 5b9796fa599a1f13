/*
 * rimp2_gradient.h -- steps adjacent to the RI-MP2 fragment kernel on the
 * way to the gradient (gfx950): the metric contraction of Gamma, its AO
 * back-transform, and the L' / L'' terms of the energy-weighted density.  Same conventions as rimp2.h: device
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

/*
 * The Appendix's back-transform of Gamma^P_ia to the AO basis, for the
 * auxiliary indices P in [p0, p0 + pcount) (the AO tensor holds nao^2 naux
 * values, so a caller may form it in auxiliary chunks):
 *
 *   out[m][n][P - p0] = sum_i sum_a C_occ[i][m] Gamma[i][a][P] C_vir[a][n]
 *
 *   Gamma  device, read  [nocc][nvir][naux]  Gamma^P_ia (with or without its
 *                                            metric contraction)
 *   C_occ  device, read  [nocc][nao]         MO coefficients C_{i mu}
 *   C_vir  device, read  [nvir][nao]         MO coefficients C_{a mu}
 *   out    device, write [nao][nao][pcount]
 *   workspace  device, 256-byte aligned, rimp2_gamma_ao_workspace_size bytes
 *              (holds the half-transformed [nocc][nao][pcount] tensor)
 * Two FP64 MFMA stages: per occupied orbital, sum over a (M = nao, N =
 * pcount, K = nvir), then one GEMM over i (M = nao, N = nao pcount, K = nocc).
 * Sizes >= 1 and 0 <= p0 <= naux - pcount, else RIMP2_EINVAL.
 */
int rimp2_gamma_ao_workspace_size(int32_t nocc, int32_t nao, int32_t pcount, size_t* bytes);
int rimp2_gamma_ao(int32_t nocc, int32_t nvir, int32_t nao, int32_t naux, int32_t p0, int32_t pcount,
                   const double* Gamma, const double* C_occ, const double* C_vir, double* out,
                   void* workspace, size_t workspace_bytes, void* stream);

/*
 * The L' and L'' terms of the Appendix's energy-weighted density matrix W:
 *
 *   L1[i][q] = L'_iq  = sum_aP Gamma^P_ia (P|qa)    I_qa [nmo][nvir][naux] = (P|qa)
 *   L2[a][q] = L''_aq = sum_iP Gamma^P_ia (P|iq)    I_iq [nocc][nmo][naux] = (P|iq)
 *
 * for every molecular orbital q < nmo.  Gamma is the Appendix's Gamma (with
 * its metric contraction, rimp2_gamma_metric).  L1 and I_qa are given
 * together or both NULL, likewise L2 and I_iq.  Each is one FP64 MFMA GEMM
 * with split-K partials in the workspace (rimp2_l_terms_workspace_size bytes,
 * 256-byte aligned) and an ordered reduction, so results are deterministic.
 */
int rimp2_l_terms_workspace_size(int32_t nocc, int32_t nvir, int32_t nmo, int32_t naux, size_t* bytes);
int rimp2_l_terms(int32_t nocc, int32_t nvir, int32_t nmo, int32_t naux, const double* Gamma,
                  const double* I_qa, const double* I_iq, double* L1, double* L2,
                  void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RIMP2_GRADIENT_H */
