// Training and inference kernels of the learned selector's MLP (FP32, row-major batches).
//
// One training step on a batch of B samples X [B][8], labels y [B]:
//   forward   H1 = relu(X W1^T + b1), H2 = relu(H1 W2^T + b2), Z = H2 W3^T + b3
//   loss      mean over the batch of -log softmax(Z)[y]
//   backward  dZ = (softmax(Z) - onehot(y)) / B; dW3 = dZ^T H2, db3 = sum dZ;
//             dH2 = (dZ W3) * [H2 > 0]; dW2 = dH2^T H1, db2 = sum dH2;
//             dH1 = (dH2 W2) * [H1 > 0]; dW1 = dH1^T X, db1 = sum dH1
//   update    Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.
// Every output element is computed by one thread with a fixed-order loop: the step is
// deterministic.
#include <hip/hip_runtime.h>
#include <math.h>

#include "mlp.h"

namespace expm {

namespace {

// out[s][j] = act(sum_k W[j][k] in[s][k] + b[j]);  grid covers B * J threads.
__global__ void mlp_dense(const float *in, int K, const float *W, const float *b, int J, int B, int relu, float *out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * J) return;
  const int s = t / J, j = t - s * J;
  float acc = b[j];
  for (int k = 0; k < K; ++k) acc += W[j * K + k] * in[s * K + k];
  out[t] = relu ? fmaxf(acc, 0.0f) : acc;
}

// Softmax cross-entropy per sample: loss[s], dZ[s][:] = (p - onehot) / B.
__global__ void mlp_softmax_ce(const float *Z, const int *y, int B, float *loss, float *dZ) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const float *z = Z + s * kMlpOut;
  float mx = z[0];
  for (int c = 1; c < kMlpOut; ++c) mx = fmaxf(mx, z[c]);
  float sum = 0.0f;
  for (int c = 0; c < kMlpOut; ++c) sum += expf(z[c] - mx);
  const int yc = y[s];
  loss[s] = -(z[yc] - mx - logf(sum));
  for (int c = 0; c < kMlpOut; ++c) dZ[s * kMlpOut + c] = (expf(z[c] - mx) / sum - (c == yc ? 1.0f : 0.0f)) / (float)B;
}

// dW[j][k] = sum_s d[s][j] a[s][k]; db[j] = sum_s d[s][j].  Grid covers J * (K + 1) threads.
__global__ void mlp_wgrad(const float *d, int J, const float *a, int K, int B, float *dW, float *db) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= J * (K + 1)) return;
  const int j = t / (K + 1), k = t - j * (K + 1);
  float acc = 0.0f;
  if (k < K) {
    for (int s = 0; s < B; ++s) acc += d[s * J + j] * a[s * K + k];
    dW[j * K + k] = acc;
  } else {
    for (int s = 0; s < B; ++s) acc += d[s * J + j];
    db[j] = acc;
  }
}

// dIn[s][k] = (sum_j d[s][j] W[j][k]) * [act[s][k] > 0].  Grid covers B * K threads.
__global__ void mlp_bgrad(const float *d, int J, const float *W, int K, const float *act, int B, float *dIn) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * K) return;
  const int s = t / K, k = t - s * K;
  float acc = 0.0f;
  for (int j = 0; j < J; ++j) acc += d[s * J + j] * W[j * K + k];
  dIn[t] = act[t] > 0.0f ? acc : 0.0f;
}

__global__ void mlp_adam(float *p, const float *g, float *mo, float *ve, int n, float lr, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  mo[i] = 0.9f * mo[i] + 0.1f * gi;
  ve[i] = 0.999f * ve[i] + 0.001f * gi * gi;
  p[i] -= lr * (mo[i] / bc1) / (sqrtf(ve[i] / bc2) + 1e-8f);
}

inline unsigned blocks(int n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// Scratch layout (floats): H1 [B][64], H2 [B][64], Z [B][16], dZ [B][16], dH2 [B][64], dH1 [B][64].
size_t mlp_scratch_floats(int B) { return (size_t)B * (kMlpH * 4 + kMlpOut * 2); }

hipError_t mlp_forward(const float *params, const float *X, int B, float *scratch, float *logits, hipStream_t st) {
  float *H1 = scratch, *H2 = H1 + (size_t)B * kMlpH;
  hipLaunchKernelGGL(mlp_dense, dim3(blocks(B * kMlpH)), dim3(256), 0, st, X, kMlpIn, params + kMlpW1, params + kMlpB1,
                     kMlpH, B, 1, H1);
  hipLaunchKernelGGL(mlp_dense, dim3(blocks(B * kMlpH)), dim3(256), 0, st, H1, kMlpH, params + kMlpW2, params + kMlpB2,
                     kMlpH, B, 1, H2);
  hipLaunchKernelGGL(mlp_dense, dim3(blocks(B * kMlpOut)), dim3(256), 0, st, H2, kMlpH, params + kMlpW3,
                     params + kMlpB3, kMlpOut, B, 0, logits);
  return hipGetLastError();
}

hipError_t mlp_grad(const float *params, const float *X, const int *y, int B, float *scratch, float *grads,
                    float *loss, hipStream_t st) {
  float *H1 = scratch, *H2 = H1 + (size_t)B * kMlpH, *Z = H2 + (size_t)B * kMlpH, *dZ = Z + (size_t)B * kMlpOut;
  float *dH2 = dZ + (size_t)B * kMlpOut, *dH1 = dH2 + (size_t)B * kMlpH;
  hipError_t e = mlp_forward(params, X, B, scratch, Z, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_softmax_ce, dim3(blocks(B)), dim3(256), 0, st, Z, y, B, loss, dZ);
  hipLaunchKernelGGL(mlp_wgrad, dim3(blocks(kMlpOut * (kMlpH + 1))), dim3(256), 0, st, dZ, kMlpOut, H2, kMlpH, B,
                     grads + kMlpW3, grads + kMlpB3);
  hipLaunchKernelGGL(mlp_bgrad, dim3(blocks(B * kMlpH)), dim3(256), 0, st, dZ, kMlpOut, params + kMlpW3, kMlpH, H2, B,
                     dH2);
  hipLaunchKernelGGL(mlp_wgrad, dim3(blocks(kMlpH * (kMlpH + 1))), dim3(256), 0, st, dH2, kMlpH, H1, kMlpH, B,
                     grads + kMlpW2, grads + kMlpB2);
  hipLaunchKernelGGL(mlp_bgrad, dim3(blocks(B * kMlpH)), dim3(256), 0, st, dH2, kMlpH, params + kMlpW2, kMlpH, H1, B,
                     dH1);
  hipLaunchKernelGGL(mlp_wgrad, dim3(blocks(kMlpH * (kMlpIn + 1))), dim3(256), 0, st, dH1, kMlpH, X, kMlpIn, B,
                     grads + kMlpW1, grads + kMlpB1);
  return hipGetLastError();
}

hipError_t mlp_adam_step(float *params, const float *grads, float *m, float *v, int step, float lr, hipStream_t st) {
  const float bc1 = 1.0f - powf(0.9f, (float)step), bc2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(mlp_adam, dim3(blocks(kMlpParams)), dim3(256), 0, st, params, grads, m, v, kMlpParams, lr, bc1, bc2);
  return hipGetLastError();
}

}  // namespace expm
