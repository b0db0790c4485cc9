// Cost model of the work-item scheduler: a two-hidden-layer perceptron with O linear outputs
//   z1 = W1 x + b1, h1 = tanh(z1);  z2 = W2 h1 + b2, h2 = tanh(z2);  y = W3 h2 + b3
// with its forward pass, the gradient of the mean squared error, and Adam, all on the GPU.
// The scheduler's model predicts, for an <A,B> work item, log(cycles) (output 0) and the
// log of its contribution bound (output 1) from features the main kernel produces; the plan
// orders items longest-predicted-first (the greedy machine scheduling of Sec. III D 1, on
// predicted rather than static costs).
//
// Parameter layout (FP32): W1[H][F], b1[H], W2[H][H], b2[H], W3[O][H], b3[O].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "hfx_internal.h"

namespace hfx {

constexpr int kMlpMaxH = 64, kMlpMaxF = 16, kMlpMaxO = 4;
constexpr int kMlpMaxParams = kMlpMaxH * kMlpMaxF + 2 * kMlpMaxH + kMlpMaxH * kMlpMaxH + kMlpMaxO * kMlpMaxH + kMlpMaxO;

__host__ __device__ inline int64_t mlp_n_params(int F, int H, int O) {
  return (int64_t)H * F + H + (int64_t)H * H + H + (int64_t)O * H + O;
}

// forward of one sample with parameters in LDS: y[0..O)
__device__ inline void mlp_fwd1(const float *P, int F, int H, int O, const float *x, float *h1, float *h2, float *y) {
  const float *W1 = P, *b1 = W1 + H * F, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + O * H;
  for (int j = 0; j < H; ++j) {
    float z = b1[j];
    for (int f = 0; f < F; ++f) z += W1[j * F + f] * x[f];
    h1[j] = tanhf(z);
  }
  for (int j = 0; j < H; ++j) {
    float z = b2[j];
    for (int k = 0; k < H; ++k) z += W2[j * H + k] * h1[k];
    h2[j] = tanhf(z);
  }
  for (int o = 0; o < O; ++o) {
    float v = b3[o];
    for (int j = 0; j < H; ++j) v += W3[o * H + j] * h2[j];
    y[o] = v;
  }
}

__global__ __launch_bounds__(256) void k_mlp_predict(const float *__restrict__ Pg, int F, int H, int O,
                                                     const float *__restrict__ X, long long n, float *__restrict__ out) {
  __shared__ float P[kMlpMaxParams];
  const int np = (int)mlp_n_params(F, H, O);
  for (int q = threadIdx.x; q < np; q += 256) P[q] = Pg[q];
  __syncthreads();
  float x[kMlpMaxF], h1[kMlpMaxH], h2[kMlpMaxH], y[kMlpMaxO];
  for (long long s = blockIdx.x * 256LL + threadIdx.x; s < n; s += (long long)gridDim.x * 256) {
    for (int f = 0; f < F; ++f) x[f] = X[s * F + f];
    mlp_fwd1(P, F, H, O, x, h1, h2, y);
    for (int o = 0; o < O; ++o) out[s * O + o] = y[o];
  }
}

// loss = mean over samples of sum_o (y_o - t_o)^2 ; grad accumulated (atomics) into G (zeroed
// by the caller).  T: n x O.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ Pg, int F, int H, int O,
                                                  const float *__restrict__ X, const float *__restrict__ T,
                                                  long long n, float *__restrict__ G, float *__restrict__ loss) {
  __shared__ float P[kMlpMaxParams];
  __shared__ float Gs[kMlpMaxParams];
  __shared__ float ls;
  const int np = (int)mlp_n_params(F, H, O);
  for (int q = threadIdx.x; q < np; q += 256) {
    P[q] = Pg[q];
    Gs[q] = 0.0f;
  }
  if (threadIdx.x == 0) ls = 0.0f;
  __syncthreads();
  const float *W2 = P + H * F + H, *W3 = W2 + H * H + H;
  float *gW1 = Gs, *gb1 = gW1 + H * F, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gW3 = gb2 + H, *gb3 = gW3 + O * H;
  float x[kMlpMaxF], h1[kMlpMaxH], h2[kMlpMaxH], d2[kMlpMaxH], y[kMlpMaxO], dy[kMlpMaxO];
  const float inv_n = 1.0f / (float)n;
  float lacc = 0.0f;
  for (long long s = blockIdx.x * 256LL + threadIdx.x; s < n; s += (long long)gridDim.x * 256) {
    for (int f = 0; f < F; ++f) x[f] = X[s * F + f];
    mlp_fwd1(P, F, H, O, x, h1, h2, y);
    for (int o = 0; o < O; ++o) {
      const float r = y[o] - T[s * O + o];
      lacc += r * r;
      dy[o] = 2.0f * r * inv_n;
      atomicAdd(&gb3[o], dy[o]);
    }
    for (int j = 0; j < H; ++j) {
      float dh = 0.0f;
      for (int o = 0; o < O; ++o) {
        atomicAdd(&gW3[o * H + j], dy[o] * h2[j]);
        dh += dy[o] * W3[o * H + j];
      }
      d2[j] = dh * (1.0f - h2[j] * h2[j]);
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

// features of every work item from the previous build's per-item counters and the geometry
//   x = [log1p(units t1..t4), log1p(alive G), log(nF*nG), n_ao(A)/16, n_abf(A)/64,
//        |r_B + R - r_A| / 10 bohr, log(atoms of the cell)], normalised
__global__ void k_item_features(const Item *__restrict__ items, const int *__restrict__ units,
                                 const int *__restrict__ c_start, const int *__restrict__ nao,
                                 const int *__restrict__ nabf, const float *__restrict__ dist,
                                 const int *__restrict__ cell_of, const int *__restrict__ cell_natoms, long long n,
                                 const float *__restrict__ mu, const float *__restrict__ sd, float *__restrict__ X) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n; s += (long long)gridDim.x * blockDim.x) {
    const Item it = items[s];
    const int *u = units + s * kItemUnits;
    float f[kItemFeatures];
    for (int t = 0; t < 4; ++t) f[t] = log1pf((float)u[t]);
    f[4] = log1pf((float)u[4]);
    const float nf = (float)(c_start[it.A + 1] - c_start[it.A]), ng = (float)(c_start[it.B + 1] - c_start[it.B]);
    f[5] = logf(fmaxf(nf * ng, 1.0f));
    f[6] = (float)nao[it.A] / 16.0f;
    f[7] = (float)nabf[it.A] / 64.0f;
    f[8] = dist[s] / 10.0f;
    f[9] = logf((float)cell_natoms[cell_of[it.A]]);
    for (int q = 0; q < kItemFeatures; ++q) X[s * kItemFeatures + q] = (f[q] - mu[q]) / sd[q];
  }
}

hipError_t mlp_launch_predict(const float *P, int F, int H, int O, const float *X, long long n, float *out,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nb = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_mlp_predict, dim3(nb), dim3(256), 0, s, P, F, H, O, X, n, out);
  return hipGetLastError();
}
hipError_t mlp_launch_grad(const float *P, int F, int H, int O, const float *X, const float *T, long long n, float *G,
                           float *loss, hipStream_t s) {
  const int np = (int)mlp_n_params(F, H, O);
  hipLaunchKernelGGL(k_mlp_zero, dim3(8), dim3(256), 0, s, G, np, loss);
  if (n > 0) {
    const int nb = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, P, F, H, O, X, T, n, G, loss);
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
                               const int *nabf, const float *dist, const int *cell_of, const int *cell_natoms,
                               long long n, const float *mu, const float *sd, float *X, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_features, dim3(1024), dim3(256), 0, s, items, units, c_start, nao, nabf, dist, cell_of,
                     cell_natoms, n, mu, sd, X);
  return hipGetLastError();
}
// ---------------------------------------------------------------------------------------------
// Training without allocation (hfx_mlp_train_static): the gradient, the two Adam moments and the
// per-epoch loss live in one file-scope device array sized for the largest model the library
// takes.  Each GPU holds its own copy until the process ends; every call on a GPU shares it.
constexpr int kMlpScratchFloats = 3 * kMlpMaxParams + 64;
static __device__ __align__(256) float scratch[kMlpScratchFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};  // device address of `scratch` on each GPU (0: not yet looked up)
}  // namespace

// device address of this GPU's copy of `scratch`, looked up once per device with it current
static hipError_t scratch_address(float **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = static_cast<float *>(p);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

__global__ void k_fill_zero(float *__restrict__ p, int n) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) p[q] = 0.0f;
}

int mlp_scratch_max_params() { return kMlpMaxParams; }

// full-batch Adam as hfx_mlp_train, with the optimizer state in `scratch`; stream-ordered, no
// allocation, no synchronisation; loss_dev (optional, device) receives the loss before each step
hipError_t mlp_train_static(int F, int H, int O, float *P, const float *X, const float *T, long long n, int epochs,
                            float lr, float *loss_dev, hipStream_t s) {
  const int np = (int)mlp_n_params(F, H, O);
  if (np > kMlpMaxParams) return hipErrorInvalidValue;
  float *scr = nullptr;
  hipError_t e = scratch_address(&scr);
  if (e != hipSuccess) return e;
  float *G = scr, *m = scr + kMlpMaxParams, *v = m + np, *loss = scr + 3 * kMlpMaxParams;
  hipLaunchKernelGGL(k_fill_zero, dim3(8), dim3(256), 0, s, m, 2 * np);  // moments of the previous call
  e = hipGetLastError();
  for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
    e = mlp_launch_grad(P, F, H, O, X, T, n, G, loss_dev ? loss_dev + ep : loss, s);
    if (e == hipSuccess) e = mlp_launch_adam(P, G, m, v, np, lr, ep + 1, s);
  }
  return e;
}

int64_t mlp_params(int F, int H, int O) { return mlp_n_params(F, H, O); }
int mlp_max_h() { return kMlpMaxH; }
int mlp_max_f() { return kMlpMaxF; }
int mlp_max_o() { return kMlpMaxO; }

}  // namespace hfx
