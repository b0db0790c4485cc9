// Matrix-core throughput probe: the dense peak the roofline of the build is quoted against,
// measured on the GPU the library runs on rather than taken from the data sheet.
//
// Every wave issues kPeakUnroll * rounds rounds of kPeakChains independent MFMAs of one kind on register
// operands (no memory traffic inside the loop), eight waves per SIMD, one grid that fills every
// compute unit.  FLOPs count 2 per multiply-add of the instruction's full shape.  Lane 0 of the
// first wave also reads the shader-clock cycle counter and the constant-rate wall clock around
// its loop, which gives the clock the matrix cores ran at.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hfx {

typedef double pk_d4 __attribute__((ext_vector_type(4)));
typedef float pk_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 pk_bf8 __attribute__((ext_vector_type(8)));

constexpr int kPeakChains = 8;
constexpr int kPeakUnroll = 16;  // rounds of chains per loop trip: loop overhead and accumulator moves amortised
constexpr int kPeakThreads = 256;
constexpr int kPeakBlocksPerCU = 8;  // 32 waves per CU, 8 per SIMD

// FLOPs of one wave-level instruction of each kind
__host__ __device__ constexpr double peak_flops_per_instr(int kind) {
  return kind == 0 ? 2.0 * 16 * 16 * 4 : kind == 1 ? 2.0 * 16 * 16 * 4 : 2.0 * 16 * 16 * 32;
}

template <int KIND>
__global__ __launch_bounds__(kPeakThreads) void k_mfma_peak(int rounds, float seed, double *__restrict__ out,
                                                           long long *__restrict__ clk) {
  const float s = seed * (1.0f + 1e-3f * (float)(threadIdx.x & 63));
  long long c0 = 0, t0 = 0;
  const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
  double sum = 0.0;
  if constexpr (KIND == 0) {
    pk_d4 acc[kPeakChains];
    for (int c = 0; c < kPeakChains; ++c) acc[c] = pk_d4{0.0, 0.0, 0.0, 0.0};
    const double a = (double)s, b = 1.0 - (double)s;
    if (timer) { c0 = clock64(); t0 = wall_clock64(); }
    for (int i = 0; i < rounds; ++i) {
#pragma unroll
      for (int u = 0; u < kPeakUnroll; ++u)
#pragma unroll
        for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    for (int c = 0; c < kPeakChains; ++c) sum += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  } else if constexpr (KIND == 1) {
    pk_f4 acc[kPeakChains];
    for (int c = 0; c < kPeakChains; ++c) acc[c] = pk_f4{0.f, 0.f, 0.f, 0.f};
    const float a = s, b = 1.0f - s;
    if (timer) { c0 = clock64(); t0 = wall_clock64(); }
    for (int i = 0; i < rounds; ++i) {
#pragma unroll
      for (int u = 0; u < kPeakUnroll; ++u)
#pragma unroll
        for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    }
    for (int c = 0; c < kPeakChains; ++c) sum += (double)(acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3]);
  } else {
    pk_f4 acc[kPeakChains];
    for (int c = 0; c < kPeakChains; ++c) acc[c] = pk_f4{0.f, 0.f, 0.f, 0.f};
    pk_bf8 a, b;
    for (int j = 0; j < 8; ++j) {
      a[j] = (__bf16)(s * (float)(j + 1) * 0.125f);
      b[j] = (__bf16)(1.0f - s * (float)j * 0.125f);
    }
    if (timer) { c0 = clock64(); t0 = wall_clock64(); }
    for (int i = 0; i < rounds; ++i) {
#pragma unroll
      for (int u = 0; u < kPeakUnroll; ++u)
#pragma unroll
        for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
    for (int c = 0; c < kPeakChains; ++c) sum += (double)(acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3]);
  }
  if (timer) {
    clk[0] = clock64() - c0;
    clk[1] = wall_clock64() - t0;
  }
  out[(long long)blockIdx.x * kPeakThreads + threadIdx.x] = sum;  // keeps the MFMAs live
}

// Runs the probe of one kind (0 FP64, 1 FP32, 2 BF16) once to warm up (an eighth of the rounds)
// and once timed, with iters (rounded up to whole unrolled trips) rounds of chains per wave.
// out: n_blocks * kPeakThreads doubles, clk: 2 int64 (device).  Returns the kernel time of the
// timed run (ms) and the FLOPs it issued; clk holds its cycle and wall-clock ticks.
hipError_t mfma_peak_run(int kind, int n_cu, int iters, double *out, long long *clk, hipStream_t st, float *ms,
                         double *flops) {
  const int blocks = n_cu * kPeakBlocksPerCU;
  iters = (iters + 8 * kPeakUnroll - 1) / (8 * kPeakUnroll) * (8 * kPeakUnroll);  // whole unrolled trips
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
    const int it = (rep == 0 ? iters / 8 : iters) / kPeakUnroll;
    if (rep == 1) e = hipEventRecord(e0, st);
    if (e != hipSuccess) break;
    if (kind == 0)
      hipLaunchKernelGGL(k_mfma_peak<0>, dim3(blocks), dim3(kPeakThreads), 0, st, it, 0.37f, out, clk);
    else if (kind == 1)
      hipLaunchKernelGGL(k_mfma_peak<1>, dim3(blocks), dim3(kPeakThreads), 0, st, it, 0.37f, out, clk);
    else
      hipLaunchKernelGGL(k_mfma_peak<2>, dim3(blocks), dim3(kPeakThreads), 0, st, it, 0.37f, out, clk);
    e = hipGetLastError();
    if (e == hipSuccess && rep == 1) e = hipEventRecord(e1, st);
  }
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *flops = (double)blocks * (kPeakThreads / 64) * (double)iters * kPeakChains * peak_flops_per_instr(kind);
  return e;
}

int mfma_peak_blocks_per_cu() { return kPeakBlocksPerCU; }
int mfma_peak_threads() { return kPeakThreads; }

}  // namespace hfx
