// Cost model of the work-item scheduler: a two-hidden-layer perceptron
//   z1 = W1 x + b1, h1 = tanh(z1);  z2 = W2 h1 + b2, h2 = tanh(z2);  y = w3 . h2 + b3
// with its forward pass, the gradient of the mean squared error, and Adam, all on the GPU.
// It predicts log(cycles) of an <A,B> work item from features the main kernel produces;
// the plan orders items longest-predicted-first (the greedy machine scheduling of
// Sec. III D 1, on predicted rather than static costs).
//
// Parameter layout (FP32): W1[H][F], b1[H], W2[H][H], b2[H], w3[H], b3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hfx_internal.h"

namespace hfx {

constexpr int kMlpMaxH = 64, kMlpMaxF = 16;

__host__ __device__ inline int64_t mlp_n_params(int F, int H) { return (int64_t)H * F + H + (int64_t)H * H + H + H + 1; }

// forward of one sample with parameters in LDS
__device__ inline float mlp_fwd1(const float *P, int F, int H, const float *x, float *h1, float *h2) {
  const float *W1 = P, *b1 = W1 + H * F, *W2 = b1 + H, *b2 = W2 + H * H, *w3 = b2 + H, *b3 = w3 + H;
  for (int j = 0; j < H; ++j) {
    float z = b1[j];
    for (int f = 0; f < F; ++f) z += W1[j * F + f] * x[f];
    h1[j] = tanhf(z);
  }
  float y = b3[0];
  for (int j = 0; j < H; ++j) {
    float z = b2[j];
    for (int k = 0; k < H; ++k) z += W2[j * H + k] * h1[k];
    h2[j] = tanhf(z);
    y += w3[j] * h2[j];
  }
  return y;
}

__global__ __launch_bounds__(256) void k_mlp_predict(const float *__restrict__ Pg, int F, int H,
                                                     const float *__restrict__ X, long long n, float *__restrict__ out) {
  __shared__ float P[kMlpMaxH * kMlpMaxF + 3 * kMlpMaxH + kMlpMaxH * kMlpMaxH + 1];
  const int np = (int)mlp_n_params(F, H);
  for (int q = threadIdx.x; q < np; q += 256) P[q] = Pg[q];
  __syncthreads();
  float x[kMlpMaxF], h1[kMlpMaxH], h2[kMlpMaxH];
  for (long long s = blockIdx.x * 256LL + threadIdx.x; s < n; s += (long long)gridDim.x * 256) {
    for (int f = 0; f < F; ++f) x[f] = X[s * F + f];
    out[s] = mlp_fwd1(P, F, H, x, h1, h2);
  }
}

// loss = mean (y - t)^2 ; grad accumulated (atomics) into G (zeroed by the caller)
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ Pg, int F, int H,
                                                  const float *__restrict__ X, const float *__restrict__ T,
                                                  long long n, float *__restrict__ G, float *__restrict__ loss) {
  __shared__ float P[kMlpMaxH * kMlpMaxF + 3 * kMlpMaxH + kMlpMaxH * kMlpMaxH + 1];
  __shared__ float Gs[kMlpMaxH * kMlpMaxF + 3 * kMlpMaxH + kMlpMaxH * kMlpMaxH + 1];
  __shared__ float ls;
  const int np = (int)mlp_n_params(F, H);
  for (int q = threadIdx.x; q < np; q += 256) {
    P[q] = Pg[q];
    Gs[q] = 0.0f;
  }
  if (threadIdx.x == 0) ls = 0.0f;
  __syncthreads();
  const float *W2 = P + H * F + H, *w3 = W2 + H * H + H;
  float *gW1 = Gs, *gb1 = gW1 + H * F, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gw3 = gb2 + H, *gb3 = gw3 + H;
  float x[kMlpMaxF], h1[kMlpMaxH], h2[kMlpMaxH], d2[kMlpMaxH];
  const float inv_n = 1.0f / (float)n;
  float lacc = 0.0f;
  for (long long s = blockIdx.x * 256LL + threadIdx.x; s < n; s += (long long)gridDim.x * 256) {
    for (int f = 0; f < F; ++f) x[f] = X[s * F + f];
    const float y = mlp_fwd1(P, F, H, x, h1, h2);
    const float r = y - T[s];
    lacc += r * r;
    const float dy = 2.0f * r * inv_n;
    atomicAdd(gb3, dy);
    for (int j = 0; j < H; ++j) {
      atomicAdd(&gw3[j], dy * h2[j]);
      d2[j] = dy * w3[j] * (1.0f - h2[j] * h2[j]);
      atomicAdd(&gb2[j], d2[j]);
    }
    for (int k = 0; k < H; ++k) {
      float dh = 0.0f;
      for (int j = 0; j < H; ++j) {
        atomicAdd(&gW2[j * H + k], d2[j] * h1[k]);
        dh += d2[j] * W2[j * H + k];
      }
      const float d1 = dh * (1.0f - h1[k] * h1[k]);
      atomicAdd(&gb1[k], d1);
      for (int f = 0; f < F; ++f) atomicAdd(&gW1[k * F + f], d1 * x[f]);
    }
  }
  atomicAdd(&ls, lacc * inv_n);
  __syncthreads();
  for (int q = threadIdx.x; q < np; q += 256) atomicAdd(&G[q], Gs[q]);
  if (threadIdx.x == 0) atomicAdd(loss, ls);
}

__global__ void k_mlp_zero(float *__restrict__ g, int np, float *__restrict__ loss) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < np; q += gridDim.x * blockDim.x) g[q] = 0.0f;
  if (blockIdx.x == 0 && threadIdx.x == 0) *loss = 0.0f;
}

// Adam (Kingma & Ba) with bias correction
__global__ void k_mlp_adam(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ m,
                           float *__restrict__ v, int np, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < np; q += gridDim.x * blockDim.x) {
    const float g = G[q];
    const float mq = b1 * m[q] + (1.0f - b1) * g;
    const float vq = b2 * v[q] + (1.0f - b2) * g * g;
    m[q] = mq;
    v[q] = vq;
    P[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
  }
}

// features of every work item from the previous build's per-item counters
//   x = [log1p(units t1..t4), log1p(alive G), log(nF*nG), n_ao(A)/16, n_abf(A)/64], normalised
__global__ void k_item_features(const Item *__restrict__ items, const int *__restrict__ units,
                                 const int *__restrict__ c_start, const int *__restrict__ nao,
                                 const int *__restrict__ nabf, long long n, const float *__restrict__ mu,
                                 const float *__restrict__ sd, float *__restrict__ X) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n; s += (long long)gridDim.x * blockDim.x) {
    const Item it = items[s];
    const int *u = units + s * kItemUnits;
    float f[8];
    for (int t = 0; t < 4; ++t) f[t] = log1pf((float)u[t]);
    f[4] = log1pf((float)u[4]);
    const float nf = (float)(c_start[it.A + 1] - c_start[it.A]), ng = (float)(c_start[it.B + 1] - c_start[it.B]);
    f[5] = logf(fmaxf(nf * ng, 1.0f));
    f[6] = (float)nao[it.A] / 16.0f;
    f[7] = (float)nabf[it.A] / 64.0f;
    for (int q = 0; q < 8; ++q) X[s * 8 + q] = (f[q] - mu[q]) / sd[q];
  }
}

hipError_t mlp_launch_predict(const float *P, int F, int H, const float *X, long long n, float *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nb = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_mlp_predict, dim3(nb), dim3(256), 0, s, P, F, H, X, n, out);
  return hipGetLastError();
}
hipError_t mlp_launch_grad(const float *P, int F, int H, const float *X, const float *T, long long n, float *G,
                           float *loss, hipStream_t s) {
  const int np = (int)mlp_n_params(F, H);
  hipLaunchKernelGGL(k_mlp_zero, dim3(8), dim3(256), 0, s, G, np, loss);
  if (n > 0) {
    const int nb = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, P, F, H, X, T, n, G, loss);
  }
  return hipGetLastError();
}
hipError_t mlp_launch_adam(float *P, const float *G, float *m, float *v, int np, float lr, int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3(8), dim3(256), 0, s, P, G, m, v, np, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}
hipError_t mlp_launch_features(const Item *items, const int *units, const int *c_start, const int *nao,
                               const int *nabf, long long n, const float *mu, const float *sd, float *X,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_features, dim3(1024), dim3(256), 0, s, items, units, c_start, nao, nabf, n, mu, sd, X);
  return hipGetLastError();
}
int64_t mlp_params(int F, int H) { return mlp_n_params(F, H); }
int mlp_max_h() { return kMlpMaxH; }
int mlp_max_f() { return kMlpMaxF; }

}  // namespace hfx
