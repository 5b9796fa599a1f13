/*
 * rimp2_screen.h -- learned screening of occupied pairs for the RI-MP2
 * fragment kernel (gfx950).  Same conventions as rimp2.h: device pointers,
 * caller-owned buffers, `stream` is a hipStream_t as void*, asynchronous,
 * negative rimp2_status on host-detected argument errors.
 *
 * The paper keeps only polymers whose energy contribution exceeds a cutoff
 * (Sec. "Molecular Fragmentation" and the cutoff study of the results); this
 * screen applies the same idea one level down, to the occupied pairs (i, j)
 * of a fragment: a small network predicts log10|e_ij| from cheap pair
 * features, and pairs predicted below a threshold are skipped by
 * rimp2_fragment (opts->pair_skip).  The full computation stays available as
 * the fallback and as the reference that measures the screening error.
 */
#ifndef RIMP2_SCREEN_H
#define RIMP2_SCREEN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Network: x (4 features) -> 64 -> 64 -> 1, SiLU hidden activations, FP64.
   Parameter vector layout: W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3. */
#define RIMP2_MLP_IN 4
#define RIMP2_MLP_HIDDEN 64
#define RIMP2_MLP_PARAMS (64 * 4 + 64 + 64 * 64 + 64 + 64 + 1)

/*
 * Pair features and the rigorous pair-energy bound.
 *   centroids device [nocc][3]   orbital centroids (angstrom)
 *   features  device [nocc*nocc][4], row i*nocc+j:
 *             ( |r_i - r_j| / 10,  log ||B_i||_F,  log ||B_j||_F,  (eps_i + eps_j) / 10 )
 *   bound     device [nocc][nocc] or NULL:
 *             |e_ij| <= 3 (N N^T)_ij^2 / (2 min eps_vir - eps_i - eps_j),
 *             N[i][P] = ||B^P_i.||_2  (||B_i B_j^T||_F <= (N N^T)_ij by the triangle
 *             inequality; |sum V(2V - V^T)/D| <= 3 ||V||_F^2 / min|D|)
 *   workspace device, rimp2_features_workspace_size() bytes, 256-byte aligned
 */
size_t rimp2_features_workspace_size(int32_t nocc, int32_t naux);
int rimp2_pair_features(int32_t nocc, int32_t nvir, int32_t naux, const double* B, const double* eps_occ,
                        const double* eps_vir, const double* centroids, double* features, double* bound,
                        void* workspace, size_t workspace_bytes, void* stream);

/* y[s] = net(x[s]) for s < n;  x device [n][4], params device [RIMP2_MLP_PARAMS]. */
int rimp2_mlp_forward(int64_t n, const double* x, const double* params, double* y, void* stream);

/*
 * loss = mean_s (net(x[s]) - target[s])^2 and grad = d loss / d params,
 * summed in a fixed order (deterministic).  loss device [1], grad device
 * [RIMP2_MLP_PARAMS], workspace rimp2_mlp_workspace_size(n) bytes.
 */
size_t rimp2_mlp_workspace_size(int64_t n);
int rimp2_mlp_loss_grad(int64_t n, const double* x, const double* target, const double* params, double* loss,
                        double* grad, void* workspace, size_t workspace_bytes, void* stream);

/* One Adam step (Kingma and Ba) on the parameters; m, v device [RIMP2_MLP_PARAMS]
   moment buffers (zero before step 1); step counts from 1. */
int rimp2_mlp_adam(const double* grad, double* params, double* m, double* v, int64_t step, double lr, double beta1,
                   double beta2, double eps, void* stream);

/* out[s] = log10(max(-e[s], 1e-300)) for s < n (training targets from pair energies). */
int rimp2_log_energy(int64_t n, const double* e, double* out, void* stream);

/*
 * Symmetric skip mask from predictions pred[i*nocc+j] (log10|e_ij|) of the
 * pairs i < j: skip[i][j] = skip[j][i] = (pred < threshold_log10); diagonal
 * pairs are never skipped.  skipped_energy device [1] receives the predicted
 * energy of the skipped pairs, sum over skipped ordered pairs of 10^pred.
 * One workgroup; fixed summation order.
 */
int rimp2_screen_mask(int32_t nocc, const double* pred, double threshold_log10, uint8_t* skip,
                      double* skipped_energy, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RIMP2_SCREEN_H */
