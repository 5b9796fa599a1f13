// Learned pair screening for the RI-MP2 fragment kernel (gfx950): pair
// features, the rigorous pair bound, and the forward/backward/Adam kernels of
// the small FP64 network declared in include/rimp2_screen.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/rimp2.h"
#include "../../include/rimp2_screen.h"
#include "common.hpp"

using namespace rimp2;

namespace {

// a dispatch's grid size is a 32-bit count of work-items
constexpr int64_t kMaxItems = 0xffffffffLL;
constexpr int H = RIMP2_MLP_HIDDEN, NIN = RIMP2_MLP_IN, NP = RIMP2_MLP_PARAMS;
constexpr int OW1 = 0, OB1 = OW1 + H * NIN, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;

__device__ __forceinline__ double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }
__device__ __forceinline__ double silu(double z) { return z * sigm(z); }
__device__ __forceinline__ double dsilu(double z) {
  const double s = sigm(z);
  return s * (1.0 + z * (1.0 - s));
}

// ---- features ---------------------------------------------------------------
// N[i][P] = ||B_i[:, P]||_2 (one workgroup per i, threads over P)
__global__ __launch_bounds__(256) void colnorm_kernel(const double* B, int nvir, int naux, double* N) {
  const int i = blockIdx.x;
  const double* Bi = B + (int64_t)i * nvir * naux;
  for (int P = threadIdx.x; P < naux; P += 256) {
    double s = 0.0;
    for (int a = 0; a < nvir; ++a) {
      const double v = Bi[(int64_t)a * naux + P];
      s += v * v;
    }
    N[(int64_t)i * naux + P] = sqrt(s);
  }
}
// nb[i] = ||B_i||_F from N, and evmin = min eps_vir (block 0 also)
__global__ __launch_bounds__(256) void rownorm_kernel(const double* N, int naux, double* nb, const double* ev,
                                                      int nvir, double* evmin) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int P = threadIdx.x; P < naux; P += 256) {
    const double v = N[(int64_t)i * naux + P];
    s += v * v;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) nb[i] = sqrt(sh[0]);
  if (i == 0) {
    __syncthreads();
    double mn = INFINITY;
    for (int a = threadIdx.x; a < nvir; a += 256) mn = fmin(mn, ev[a]);
    sh[threadIdx.x] = mn;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) *evmin = sh[0];
  }
}
// one thread per pair (i, j)
__global__ __launch_bounds__(256) void pair_kernel(int nocc, int naux, const double* N, const double* nb,
                                                   const double* eo, const double* r, const double* evmin,
                                                   double* feat, double* bound) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= (int64_t)nocc * nocc) return;
  const int i = (int)(p / nocc), j = (int)(p - (int64_t)i * nocc);
  const double dx = r[3 * i] - r[3 * j], dy = r[3 * i + 1] - r[3 * j + 1], dz = r[3 * i + 2] - r[3 * j + 2];
  double* f = feat + 4 * p;
  f[0] = sqrt(dx * dx + dy * dy + dz * dz) / 10.0;
  f[1] = log(nb[i]);
  f[2] = log(nb[j]);
  f[3] = (eo[i] + eo[j]) / 10.0;
  if (bound) {
    double s = 0.0;
    for (int P = 0; P < naux; ++P) s += N[(int64_t)i * naux + P] * N[(int64_t)j * naux + P];
    bound[p] = 3.0 * s * s / (2.0 * *evmin - eo[i] - eo[j]);
  }
}

// ---- network ------------------------------------------------------------------
constexpr int FS = 64;   // samples per forward workgroup (64 threads = hidden units)
__global__ __launch_bounds__(64) void mlp_forward_kernel(int64_t n, const double* x, const double* P, double* y) {
  __shared__ double W2[H * H], X[FS][NIN], H1[FS][H + 1], H2[FS][H + 1];
  const int t = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * FS;
  for (int q = t; q < H * H; q += 64) W2[q] = P[OW2 + q];
  for (int q = t; q < FS * NIN; q += 64) {
    const int64_t s = s0 + q / NIN;
    X[q / NIN][q % NIN] = s < n ? x[s * NIN + q % NIN] : 0.0;
  }
  __syncthreads();
  double w1[NIN];
  for (int k = 0; k < NIN; ++k) w1[k] = P[OW1 + t * NIN + k];
  const double b1 = P[OB1 + t], b2 = P[OB2 + t];
  for (int s = 0; s < FS; ++s) {
    double z = b1;
    for (int k = 0; k < NIN; ++k) z += w1[k] * X[s][k];
    H1[s][t] = silu(z);
  }
  __syncthreads();
  for (int s = 0; s < FS; ++s) {
    double z = b2;
    for (int u = 0; u < H; ++u) z += W2[t * H + u] * H1[s][u];
    H2[s][t] = silu(z);
  }
  __syncthreads();
  const int64_t s = s0 + t;
  if (s < n) {
    double o = P[OB3];
    for (int u = 0; u < H; ++u) o += P[OW3 + u] * H2[t][u];
    y[s] = o;
  }
}

constexpr int BS = 32;   // samples per backward workgroup
// per-workgroup gradient of sum_s (y - t)^2 / n (and the loss part) -> part[blockIdx][NP + 1]
__global__ __launch_bounds__(64) void mlp_backward_kernel(int64_t n, const double* x, const double* tgt,
                                                          const double* P, double* part) {
  __shared__ double W2[H * H], X[BS][NIN], Z1[BS][H + 1], A1[BS][H + 1], Z2[BS][H + 1], A2[BS][H + 1];
  __shared__ double dy[BS], red[64];
  const int t = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * BS;
  const int ns = (int)min<int64_t>(BS, n - s0);
  for (int q = t; q < H * H; q += 64) W2[q] = P[OW2 + q];
  for (int q = t; q < BS * NIN; q += 64) {
    const int64_t s = s0 + q / NIN;
    X[q / NIN][q % NIN] = (q / NIN) < ns ? x[s * NIN + q % NIN] : 0.0;
  }
  __syncthreads();
  // forward, keeping pre-activations
  for (int s = 0; s < BS; ++s) {
    double z = P[OB1 + t];
    for (int k = 0; k < NIN; ++k) z += P[OW1 + t * NIN + k] * X[s][k];
    Z1[s][t] = z;
    A1[s][t] = silu(z);
  }
  __syncthreads();
  for (int s = 0; s < BS; ++s) {
    double z = P[OB2 + t];
    for (int u = 0; u < H; ++u) z += W2[t * H + u] * A1[s][u];
    Z2[s][t] = z;
    A2[s][t] = silu(z);
  }
  __syncthreads();
  double lpart = 0.0;
  if (t < BS) {
    double o = P[OB3];
    for (int u = 0; u < H; ++u) o += P[OW3 + u] * A2[t][u];
    const double r = (t < ns) ? o - tgt[s0 + t] : 0.0;
    dy[t] = 2.0 * r / (double)n;
    lpart = r * r / (double)n;
  }
  red[t] = lpart;
  __syncthreads();
  double* g = part + (int64_t)blockIdx.x * (NP + 1);
  // W3, b3
  {
    double gw = 0.0;
    for (int s = 0; s < BS; ++s) gw += dy[s] * A2[s][t];
    g[OW3 + t] = gw;
    if (t == 0) {
      double gb = 0.0, l = 0.0;
      for (int s = 0; s < BS; ++s) gb += dy[s];
      for (int q = 0; q < 64; ++q) l += red[q];
      g[OB3] = gb;
      g[NP] = l;
    }
  }
  // dZ2[s][t] = dy[s] W3[t] silu'(Z2[s][t])  (into Z2)
  const double w3 = P[OW3 + t];
  for (int s = 0; s < BS; ++s) Z2[s][t] = dy[s] * w3 * dsilu(Z2[s][t]);
  __syncthreads();
  // W2[t][u] gradient, b2
  {
    double gb = 0.0;
    for (int s = 0; s < BS; ++s) gb += Z2[s][t];
    g[OB2 + t] = gb;
    for (int u = 0; u < H; ++u) {
      double gw = 0.0;
      for (int s = 0; s < BS; ++s) gw += Z2[s][t] * A1[s][u];
      g[OW2 + t * H + u] = gw;
    }
  }
  // dA1[s][u] = sum_t dZ2[s][t] W2[t][u], thread = u; dZ1 into A2 (free now)
  for (int s = 0; s < BS; ++s) {
    double d = 0.0;
    for (int q = 0; q < H; ++q) d += Z2[s][q] * W2[q * H + t];
    A2[s][t] = d * dsilu(Z1[s][t]);
  }
  __syncthreads();
  {
    double gb = 0.0;
    for (int s = 0; s < BS; ++s) gb += A2[s][t];
    g[OB1 + t] = gb;
    for (int k = 0; k < NIN; ++k) {
      double gw = 0.0;
      for (int s = 0; s < BS; ++s) gw += A2[s][t] * X[s][k];
      g[OW1 + t * NIN + k] = gw;
    }
  }
}
// grad[q] = sum over workgroups (fixed order) of part[w][q]; loss = part[.][NP]
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const double* part, int64_t nw, double* grad, double* loss) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q > NP) return;
  double s = 0.0;
  for (int64_t w = 0; w < nw; ++w) s += part[w * (NP + 1) + q];
  if (q < NP) grad[q] = s; else *loss = s;
}
__global__ __launch_bounds__(256) void adam_kernel(const double* g, double* p, double* m, double* v, double c1,
                                                   double c2, double lr, double b1, double b2, double eps) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= NP) return;
  const double gq = g[q];
  const double mq = b1 * m[q] + (1.0 - b1) * gq, vq = b2 * v[q] + (1.0 - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrt(vq / c2) + eps);
}
__global__ __launch_bounds__(256) void log_energy_kernel(int64_t n, const double* e, double* out) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s < n) out[s] = log10(fmax(-e[s], 1e-300));
}
__global__ __launch_bounds__(256) void screen_mask_kernel(int nocc, const double* pred, double thr, uint8_t* skip,
                                                          double* skipped) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < (int64_t)nocc * nocc; p += 256) {
    const int i = (int)(p / nocc), j = (int)(p - (int64_t)i * nocc);
    const int a = min(i, j), b = max(i, j);
    const double pr = pred[(int64_t)a * nocc + b];
    const bool sk = (a != b) && pr < thr;
    skip[p] = sk ? 1 : 0;
    if (sk) acc += pow(10.0, pr);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *skipped = sh[0];
}

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

extern "C" {

size_t rimp2_features_workspace_size(int32_t nocc, int32_t naux) {
  return align_up(8 * (size_t)nocc * naux) + align_up(8 * (size_t)nocc) + 256;
}

int rimp2_pair_features(int32_t nocc, int32_t nvir, int32_t naux, const double* B, const double* eps_occ,
                        const double* eps_vir, const double* centroids, double* features, double* bound,
                        void* workspace, size_t workspace_bytes, void* stream) {
  if (nocc < 1 || nvir < 1 || naux < 1) return fail(RIMP2_EINVAL, "sizes must be >= 1");
  if (!B || !eps_occ || !eps_vir || !centroids || !features || !workspace)
    return fail(RIMP2_EINVAL, "null pointer argument");
  if (workspace_bytes < rimp2_features_workspace_size(nocc, naux)) return fail(RIMP2_ENOMEM, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  double* N = (double*)ws;
  double* nb = (double*)(ws + align_up(8 * (size_t)nocc * naux));
  double* evmin = (double*)(ws + align_up(8 * (size_t)nocc * naux) + align_up(8 * (size_t)nocc));
  hipLaunchKernelGGL(colnorm_kernel, dim3(nocc), dim3(256), 0, st, B, nvir, naux, N);
  hipLaunchKernelGGL(rownorm_kernel, dim3(nocc), dim3(256), 0, st, N, naux, nb, eps_vir, nvir, evmin);
  hipLaunchKernelGGL(pair_kernel, dim3((unsigned)cdiv((int64_t)nocc * nocc, 256)), dim3(256), 0, st, nocc, naux, N,
                     nb, eps_occ, centroids, evmin, features, bound);
  HIP_TRY(hipGetLastError());
  return RIMP2_OK;
}

int rimp2_mlp_forward(int64_t n, const double* x, const double* params, double* y, void* stream) {
  if (n < 0 || (n > 0 && (!x || !params || !y))) return fail(RIMP2_EINVAL, "bad forward arguments");
  if (n == 0) return RIMP2_OK;
  if (cdiv(n, FS) * 64 > kMaxItems) return fail(RIMP2_EINVAL, "n = %lld is too large for one launch", (long long)n);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)cdiv(n, FS)), dim3(64), 0, (hipStream_t)stream, n, x, params,
                     y);
  HIP_TRY(hipGetLastError());
  return RIMP2_OK;
}

size_t rimp2_mlp_workspace_size(int64_t n) { return align_up(8 * (size_t)cdiv(n, BS) * (NP + 1)); }

int rimp2_mlp_loss_grad(int64_t n, const double* x, const double* target, const double* params, double* loss,
                        double* grad, void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 1 || !x || !target || !params || !loss || !grad || !workspace) return fail(RIMP2_EINVAL, "bad arguments");
  if (workspace_bytes < rimp2_mlp_workspace_size(n)) return fail(RIMP2_ENOMEM, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  const int64_t nw = cdiv(n, BS);
  if (nw * 64 > kMaxItems) return fail(RIMP2_EINVAL, "n = %lld is too large for one launch", (long long)n);
  hipLaunchKernelGGL(mlp_backward_kernel, dim3((unsigned)nw), dim3(64), 0, st, n, x, target, params,
                     (double*)workspace);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)cdiv(NP + 1, 256)), dim3(256), 0, st, (const double*)workspace,
                     nw, grad, loss);
  HIP_TRY(hipGetLastError());
  return RIMP2_OK;
}

int rimp2_mlp_adam(const double* grad, double* params, double* m, double* v, int64_t step, double lr, double beta1,
                   double beta2, double eps, void* stream) {
  if (!grad || !params || !m || !v || step < 1) return fail(RIMP2_EINVAL, "bad Adam arguments");
  const double c1 = 1.0 - pow(beta1, (double)step), c2 = 1.0 - pow(beta2, (double)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)cdiv(NP, 256)), dim3(256), 0, (hipStream_t)stream, grad, params, m,
                     v, c1, c2, lr, beta1, beta2, eps);
  HIP_TRY(hipGetLastError());
  return RIMP2_OK;
}

int rimp2_log_energy(int64_t n, const double* e, double* out, void* stream) {
  if (n < 0 || (n > 0 && (!e || !out))) return fail(RIMP2_EINVAL, "bad arguments");
  if (n == 0) return RIMP2_OK;
  if (cdiv(n, 256) * 256 > kMaxItems) return fail(RIMP2_EINVAL, "n = %lld is too large for one launch", (long long)n);
  hipLaunchKernelGGL(log_energy_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, (hipStream_t)stream, n, e, out);
  HIP_TRY(hipGetLastError());
  return RIMP2_OK;
}

int rimp2_screen_mask(int32_t nocc, const double* pred, double threshold_log10, uint8_t* skip, double* skipped_energy,
                      void* stream) {
  if (nocc < 1 || !pred || !skip || !skipped_energy) return fail(RIMP2_EINVAL, "bad arguments");
  hipLaunchKernelGGL(screen_mask_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, nocc, pred, threshold_log10,
                     skip, skipped_energy);
  HIP_TRY(hipGetLastError());
  return RIMP2_OK;
}

}  // extern "C"
