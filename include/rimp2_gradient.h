/*
 * rimp2_gradient.h -- steps adjacent to the RI-MP2 fragment kernel on the
 * way to the gradient (gfx950): the metric contraction of Gamma, its AO
 * back-transform, the L' / L'' terms, the antisymmetrised-integral term, the
 * Z-vector solve and the energy-weighted density matrix.  Same conventions as rimp2.h: device
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

/*
 * Orbital response (Appendix).  Bf is the three-index factor over every pair
 * of molecular orbitals, [nmo][nmo][naux] with nmo = nocc + nvir (occupied
 * first, symmetric in the two MO indices, P fastest); its occupied-virtual
 * block Bf[i][nocc + a] is rimp2_fragment's B[i][a].
 *
 * The antisymmetrised-integral term, for rows [r0, r0 + nrows) and columns
 * [c0, c0 + ncols) of its result:
 *
 *   F[p - r0][q - c0] = sum_rs G_pq^rs D[r][s],   G_pq^rs = 2 (pq|rs) - (ps|rq),
 *   (pq|rs) = sum_P Bf[p][q][P] Bf[r][s][P]
 *
 *   D  device, read [nmo][nmo];  F device, write, row stride ldf >= ncols
 * The Coulomb part is two fixed-order reductions over the auxiliary index;
 * the exchange part two FP64 MFMA GEMMs (Y[s][q][P] = sum_r D[r][s]
 * Bf[r][q][P], then a contraction over (s, P) with split-K partials and an
 * ordered reduction), so results are deterministic.
 */
int rimp2_antisym_workspace_size(int32_t nmo, int32_t naux, int32_t nrows, int32_t ncols, size_t* bytes);
int rimp2_antisym_term(int32_t nmo, int32_t naux, int32_t r0, int32_t nrows, int32_t c0, int32_t ncols,
                       const double* Bf, const double* D, double* F, int64_t ldf,
                       void* workspace, size_t workspace_bytes, void* stream);

/*
 * The Appendix's Z-vector equation for the occupied-virtual block of the MP2
 * density:
 *
 *   L''_ai - L'_ia - sum_pq G_ai^pq Dbar_pq = (eps_a - eps_i)/2 D_ai + sum_bj G_ai^bj D_bj
 *
 * with Dbar = D_ij (+) D_ab (P_ij and P_ab of rimp2_fragment), L1 = L'
 * [nocc][nmo] and L2 = L'' [nvir][nmo] (rimp2_l_terms).  Solved by conjugate
 * gradients with the operator's diagonal as preconditioner, starting from
 * rhs / diagonal; every operator application is one rimp2_antisym_term
 * evaluation.  The operator is the orbital Hessian, positive definite for a
 * stable closed-shell reference; CG stops when ||rhs - A D_ai|| <= tol ||rhs||
 * or after max_iter iterations.
 *
 *   D_ai          device, write [nvir][nocc]
 *   iterations    host, write (may be NULL): iterations run
 *   rel_residual  host, write (may be NULL): ||rhs - A D_ai|| / ||rhs||
 * The call synchronises `stream` once per iteration (the host reads the CG
 * scalars).  Returns RIMP2_ENOCONV, with D_ai holding the last iterate, when
 * the tolerance is not reached or the operator is not positive definite
 * along a search direction.
 */
int rimp2_zvector_workspace_size(int32_t nocc, int32_t nvir, int32_t naux, size_t* bytes);
int rimp2_zvector(int32_t nocc, int32_t nvir, int32_t naux, const double* Bf, const double* eps_occ,
                  const double* eps_vir, const double* P_ij, const double* P_ab, const double* L1,
                  const double* L2, double* D_ai, double tol, int32_t max_iter, int32_t* iterations,
                  double* rel_residual, void* workspace, size_t workspace_bytes, void* stream);

/*
 * The Appendix's energy-weighted density matrix W [nmo][nmo], read as the sum
 * of its four printed pieces over the parts of the (p, q) domain they fill:
 *
 *   W_pq = (eps_p + eps_q)/2 D_pq                      every p, q
 *        + sum_rs G_pq^rs D^MP2_rs + L'_pq             occupied rows p < nocc
 *        + L''_(p - nocc) q                            virtual rows
 *
 * with D = D^HF + D^MP2, D^HF the identity on the occupied block and D^MP2
 * = P_ij (+) P_ab (+) D_ai (+) D_ai^T.
 */
int rimp2_energy_weighted_density_workspace_size(int32_t nocc, int32_t nvir, int32_t naux, size_t* bytes);
int rimp2_energy_weighted_density(int32_t nocc, int32_t nvir, int32_t naux, const double* Bf,
                                  const double* eps_occ, const double* eps_vir, const double* P_ij,
                                  const double* P_ab, const double* D_ai, const double* L1, const double* L2,
                                  double* W, void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RIMP2_GRADIENT_H */
