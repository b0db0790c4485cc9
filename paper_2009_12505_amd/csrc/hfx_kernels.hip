// Device kernels of the periodic exchange-matrix build (gfx950).
//
// The main kernel is persistent: each workgroup takes <A,B> work items
// (Algorithm 2) from a global ticket in schedule order and evaluates all
// four Htilde pieces of eq. HFX_split for every (F,G) neighbour pair of the
// item, with the screening of Algorithm 5.  Per item, in order:
//
//   screen   CS-ERI and CS-matrix stage 1 for each (F,G,term) (Alg. 4 first test)
//   G side   Y_G = V_AB C_BG (Alg. 3), its slice norms (stage 2), T3_G = Y D_AG and
//            T4_G = Y D_AB (both independent of F), their norms (stage 3 of terms
//            3, 4), and the Gram matrices of Y that give the stage-3 norms of terms
//            1 and 2 without forming T1, T2
//   masks    stages 2 and 3 for each surviving unit
//   GEMM-R   terms 3 and 4:  C_A^T [T4_G | T3_G]  over the concatenated (F,f) x (G,.)
//            grid, masked per (F,G) block; term 4 goes straight to Sigma(F,G),
//            term 3 is summed over G before it goes to Sigma(F,B)
//   GEMM-L   terms 1 and 2:  C_A [w D_FG | w D_FB] (the C D products of all kept
//            units), contracted with Y_G in the epilogue: term 1 summed over F and
//            G into Sigma(A,B), term 2 summed over F into Sigma(A,G)
//
// Contractions are block products on the matrix cores: a 128-row output block
// (tile_r = 32, 64 or 128 columns for terms 3/4, 64 for terms 1/2) per step of the
// workgroup, its 16x16 tiles shared by the eight waves, K staged through LDS in
// chunks with a two-chunk register prefetch.  FP64 (v_mfma_f64_16x16x4f64) by
// default; in the tiered forms a block whose kept units all have small stage-2
// bounds runs on FP32 (v_mfma_f32_16x16x4f32) or as split-BF16x3 (three
// v_mfma_f32_16x16x32_bf16 per product).  A tile whose (F,G) blocks are all
// screened out is skipped.  Sigma accumulation is FP64 (global atomics).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hfx_internal.h"

namespace hfx {

typedef double d4 __attribute__((ext_vector_type(4)));

// Global-memory (address space 1) views of device buffers.  Through a generic pointer the
// compiler emits flat loads and stores, which count against the LDS wait counter as well as the
// vector-memory one: every wait for an LDS read then also waits for all global loads in flight, so
// the prefetch of a block product's next chunk would not overlap the current chunk's MFMAs.
template <class T>
using gmem = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ gmem<T> *gptr(T *p) {
  return (gmem<T> *)p;
}
template <class T>
using smem = __attribute__((address_space(3))) T;  // LDS

// x where ok, else +0 (bitwise: no branch, and no NaN or Inf of x survives)
__device__ __forceinline__ double keep_if(double x, bool ok) {
  return __longlong_as_double(__double_as_longlong(x) & -(long long)ok);
}
__device__ __forceinline__ float keep_if(float x, bool ok) { return __int_as_float(__float_as_int(x) & -(int)ok); }
__device__ __forceinline__ void gatomic_add(gmem<double> *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int NT = 512;
constexpr int NW = NT / 64;
constexpr int MAXNB = 160;
constexpr int MAXN = 32;

// v_mfma_f64_16x16x4f64 lane layout (gfx950): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; element e of the result holds D[l/16 + 4e][l%16].
__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

typedef float f4 __attribute__((ext_vector_type(4)));

// v_mfma_f32_16x16x4f32 lane layout (gfx950): operands as for the FP64 form (lane l supplies
// A[l%16][l/16] and B[l/16][l%16]), but element e of the result holds D[4(l/16) + e][l%16].
__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// D block id of (row, col, R) for two atoms of one cell, given the cell's table base and size
__device__ __forceinline__ int lookup_local(const DevPlan &P, int tbase, int n, int lrow, int lcol, int32_t R) {
  const int t = tbase + lrow * n + lcol;
  const int s = P.pstart[t], e = s + P.pcount[t];
  for (int q = s; q < e; ++q)
    if (P.dsort_R[q] == R) return P.dsort_id[q];
  return -1;
}

__device__ __forceinline__ int lookup_d(const DevPlan &P, int row, int col, int32_t R) {
  const int c = P.cell_of[row];
  const int n = P.cell_natoms[c];
  const int t = P.ptab_off[c] + P.local_of[row] * n + P.local_of[col];
  const int s = P.pstart[t], e = s + P.pcount[t];
  for (int q = s; q < e; ++q)
    if (P.dsort_R[q] == R) return P.dsort_id[q];
  return -1;
}

// term bits of the per-(F,G) masks
constexpr uint8_t kT1 = 1, kT2 = 2, kT3 = 4, kT4 = 8, kCsOk = 16, kPend1 = 32, kPend2 = 64;

struct ItemLds {
  int A, B, rb, PA, PB, na, nb, nF, nG, nGa, MR, NR, J;
  int dAB;
  int okAB;  // D_AB usable as operand (exists and kept)
  double gV;
  long long voff;
  int cA, cB;  // first kept C block of A, of B
  // F side (i < nF)
  int f_atom[MAXNB], f_R[MAXNB], f_n[MAXNB], f_row0[MAXNB + 1], f_dFB[MAXNB];
  short f_loc[MAXNB];
  long long f_dFBoff[MAXNB];
  long long f_coff[MAXNB];
  double f_gA[MAXNB], f_gF[MAXNB], f_nA[MAXNB], f_nF[MAXNB], f_Q[MAXNB];
  uint8_t f_on[MAXNB];
  // G side (j < nG)
  int g_atom[MAXNB], g_R[MAXNB], g_n[MAXNB], g_dAG[MAXNB];
  short g_loc[MAXNB];
  int tbase, tn;  // D lookup table of the item's cell
  double gDmax;   // largest sqrt||D D^T|| of the item's cell (stage-1 prefilter of term 1)
  long long g_dAGoff[MAXNB];
  long long g_coff[MAXNB];
  double g_gA[MAXNB], g_gF[MAXNB], g_Q[MAXNB];
  uint8_t g_on[MAXNB];
  int g_alive[MAXNB];
  // alive G (jj < nGa)
  short a_j[MAXNB];
  int a_col0[MAXNB + 1];
  int a_y[MAXNB], a_t3[MAXNB], a_t4[MAXNB], a_n1[MAXNB], a_m2[MAXNB];
  double a_Yb[MAXNB], a_Yg[MAXNB], a_T3n[MAXNB], a_T4n[MAXNB];
  double H1[MAXN * MAXN];
  double DAB[MAXN * MAXN];
  // GEMM block bookkeeping
  unsigned long long blk_act;  // active 16x16 tiles of the current output block (bit: wave * tiles + tile)
  unsigned blk_ub;  // largest stage-2 bound (float bits) of the kept units of the current block
  int t1any, kc, nsel;
  unsigned long long t2any;
  int fpos[MAXNB];
  short fsel[MAXNB];
  int fsrow[MAXNB + 1];
  unsigned long long cnt[kCntN];
  double flops[2];
  double contrib;  // summed screening bounds of the item's kept units
  int scratch_top;
};

struct KParams {
  int rows_cap, cols_cap;  // sizes of the row/col decode tables (bytes) in dynamic LDS
  int ld3;                 // row stride of the per-wave term-3 accumulators in dynamic LDS
  long long wave_off;      // offset (doubles) of the per-wave scratch regions in a slot
  long long wave_doubles;  // size of one per-wave region
  long long wg_off;        // offset (doubles) of the workgroup region (GEMM-L panel, P block)
  long long ub_off;        // offset (doubles) of the per-(F,G) unit bounds used by the precision tiers
  int tier;                // 0: FP64 block products; 1: FP32 for blocks whose bound <= tau; 2: all FP32;
                           // 3: as 1, and split-BF16x3 for term-3/4 blocks whose bound <= tau_bf
  float tau, tau_bf;
};

// ---------------------------------------------------------------------------------------------
// screen: CS-ERI + stage 1 on the F x G grid
__device__ void phase_screen(const DevPlan &P, ItemLds &L, gmem<int> *dfg, gmem<long long> *doff,
                             gmem<uint8_t> *mask) {
  const int tid = threadIdx.x;
  const gmem<const long long> *d_off = gptr(P.d_off);
  const gmem<const double> *gD = gptr(P.gD);
  const gmem<const uint8_t> *keepD = gptr(P.keepD);
  const int nF = L.nF, nG = L.nG;
  const double eps = P.eps_mat, eps_eri = P.eps_eri;
  const bool use_eri = P.stages & kCsEri, use1 = P.stages & kCs1;
  unsigned long long c_eri = 0, c1[4] = {0, 0, 0, 0};
  for (int p = tid; p < nF * nG; p += NT) {
    const int i = p / nG, j = p - i * nG;
    uint8_t bits = 0;
    int dFG = -1;
    if (!use_eri || L.f_Q[i] * L.g_Q[j] > eps_eri) {
      // D_FG is needed by term 1 (operand) and term 4 (target); skip the lookup when
      // neither can pass stage 1
      const bool may1 = !use1 || L.f_gA[i] * L.gV * L.g_gA[j] * L.gDmax > eps;
      const bool may4 = L.okAB && (!use1 || L.f_gF[i] * L.gV * L.g_gF[j] * gD[L.dAB] > eps);
      if (may1 || may4) dFG = lookup_local(P, L.tbase, L.tn, L.f_loc[i], L.g_loc[j], r_sub(L.g_R[j], L.f_R[i]));
      bits = kCsOk;
      ++c_eri;
      // term 1: D_FG operand, target (A,B)
      if (dFG >= 0 && keepD[dFG] && L.dAB >= 0) {
        if (!use1 || L.f_gA[i] * L.gV * L.g_gA[j] * gD[dFG] > eps) bits |= kT1;
      }
      // term 2: D_FB operand, target (A,G)
      const int dFB = L.f_dFB[i];
      if (dFB >= 0 && keepD[dFB] && L.g_dAG[j] >= 0) {
        if (!use1 || L.f_gA[i] * L.gV * L.g_gF[j] * gD[dFB] > eps) bits |= kT2;
      }
      // term 3: D_AG operand, target (F,B)
      const int dAG = L.g_dAG[j];
      if (dAG >= 0 && keepD[dAG] && dFB >= 0) {
        if (!use1 || L.f_gF[i] * L.gV * L.g_gA[j] * gD[dAG] > eps) bits |= kT3;
      }
      // term 4: D_AB operand, target (F,G)
      if (L.okAB && dFG >= 0) {
        if (!use1 || L.f_gF[i] * L.gV * L.g_gF[j] * gD[L.dAB] > eps) bits |= kT4;
      }
      for (int t = 0; t < 4; ++t) c1[t] += (bits >> t) & 1;
      if (bits & 15) L.g_alive[j] = 1;
    }
    dfg[p] = dFG;
    doff[p] = dFG >= 0 ? d_off[dFG] : 0;
    mask[p] = bits;
  }
  atomicAdd(&L.cnt[kCntCsEri], c_eri);
  for (int t = 0; t < 4; ++t)
    if (c1[t]) atomicAdd(&L.cnt[kCntKept + t], c1[t]);
}

// ---------------------------------------------------------------------------------------------
// one 16x16 FP64 MFMA tile product over K with a one-step load prefetch;
// fa(row, k) and fb(k, col) return 0 outside the operands
template <class FA, class FB>
__device__ __forceinline__ d4 tile_mm(int K, FA fa, FB fb) {
  const int lane = threadIdx.x & 63, kk = lane >> 4, l16 = lane & 15;
  d4 acc = {0, 0, 0, 0};
  double a_c = fa(l16, kk), b_c = fb(kk, l16);
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + 4 + kk;
    double a_n = 0.0, b_n = 0.0;
    if (k0 + 4 < K) {
      a_n = fa(l16, k);
      b_n = fb(k, l16);
    }
    acc = mfma64(a_c, b_c, acc);
    a_c = a_n;
    b_c = b_n;
  }
  return acc;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// a 16x16 tile product over K <= 32 with every operand load issued before the first MFMA (the
// G-side products are short, so one wait per tile instead of one per K step); fa(row, k) and
// fb(k, col) return 0 outside the operands
template <class FA, class FB>
__device__ __forceinline__ d4 tile_mm_burst(int K, FA fa, FB fb, d4 acc) {
  const int lane = threadIdx.x & 63, kk = lane >> 4, l16 = lane & 15;
  double a[8], b[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int k = 4 * s + kk;
    a[s] = k < K ? fa(l16, k) : 0.0;
    b[s] = k < K ? fb(k, l16) : 0.0;
  }
#pragma unroll
  for (int s = 0; s < 8; ++s)
    if (4 * s < K) acc = mfma64(a[s], b[s], acc);
  return acc;
}

// step(t, buffer) for t in [0, n), the loads of step t+1 (load(t+1, buffer)) issued before the
// MFMAs of step t, in two register buffers; load takes in-bounds addresses for every t < n
template <class Buf, class Load, class Step>
__device__ __forceinline__ void pipelined(int n, Load load, Step step) {
  if (n <= 0) return;
  Buf b0, b1;
  load(0, b0);
  int t = 0;
  for (; t + 1 < n; t += 2) {
    load(t + 1, b1);
    step(t, b0);
    load(min(t + 2, n - 1), b0);
    step(t + 1, b1);
  }
  if (t < n) step(t, b0);
}

// a 16x16 FP64 tile product over a long K, eight K steps per step of the pipeline above (the next
// eight steps' loads in flight during the current's MFMAs); fa(row, k) and fb(k, col) load from
// in-bounds addresses for every row, col < 16 and k < K (rows and columns past the operands give
// output rows and columns the caller ignores); K steps past K count as zero
template <class FA, class FB>
__device__ __forceinline__ d4 tile_mm_long(int K, FA fa, FB fb) {
  const int lane = threadIdx.x & 63, kk = lane >> 4, l16 = lane & 15;
  struct KB {
    double a[8], b[8];
  };
  d4 acc = {0, 0, 0, 0};
  pipelined<KB>(
      (K + 31) >> 5,
      [&](int t, KB &bb) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = min(32 * t + 4 * s + kk, K - 1);
          bb.a[s] = fa(l16, k);
          bb.b[s] = fb(k, l16);
        }
      },
      [&](int t, const KB &bb) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          if (32 * t + 4 * s >= K) break;
          const bool ok = 32 * t + 4 * s + kk < K;
          acc = mfma64(keep_if(bb.a[s], ok), keep_if(bb.b[s], ok), acc);
        }
      });
  return acc;
}

// ---------------------------------------------------------------------------------------------
// G side for one alive G, by one wave: Y = V_AB C_BG, T4 = D_AB Y, T3 = Y D_AG^T (per alpha),
// the Gram matrices N1[b] = Y_b^T Y_b and M2[g] = Y_g^T Y_g, and the slice norms of stages 2, 3.
// Kept out of line: its load bursts need many registers, and inlined they would push the
// register allocation of the block products past the budget of two waves per SIMD.
template <bool VL>
__device__ __noinline__ void gside_wave(const DevPlan &P, ItemLds &L, gmem<double> *slot, int jj,
                                        const smem<const double> *Vl, const gmem<const double> *Vg) {
  const int lane = threadIdx.x & 63, kk = lane >> 4, l16 = lane & 15;
  const int j = L.a_j[jj];
  const int PA = L.PA, PB = L.PB, na = L.na, nb = L.nb, ng = L.g_n[j];
  const int N = nb * ng;
  const gmem<const double> *C = gptr(P.Cbuf) + L.g_coff[j];
  gmem<double> *Y = slot + L.a_y[jj];
  auto vat = [&](int q) -> double {
    if constexpr (VL)
      return Vl[q];
    else
      return Vg[q];
  };
  unsigned long long nm = 0;
  // Y[al][b*ng+g] = sum_be V[al][be] C[be][b*ng+g]; four alpha tiles share each C fragment, which
  // is fetched 32 K at a time, the next fragment's loads in flight during the current's MFMAs
  const int mt = (PA + 15) >> 4, nt = (N + 15) >> 4, nkc = (PB + 31) >> 5;
  struct YB {
    double v[8];
  };
  for (int rg = 0; rg < mt; rg += 4) {
    d4 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = d4{0, 0, 0, 0};
    pipelined<YB>(
        nt * nkc,
        [&](int t, YB &bb) {
          const int ct = t / nkc, k0 = (t - ct * nkc) << 5, col = min((ct << 4) + l16, N - 1);
#pragma unroll
          for (int s = 0; s < 8; ++s) bb.v[s] = C[(long long)min(k0 + 4 * s + kk, PB - 1) * N + col];
        },
        [&](int t, const YB &bb) {
          const int ct = t / nkc, k0 = (t - ct * nkc) << 5, col = (ct << 4) + l16;
          const bool cok = col < N;
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            if (k0 + 4 * s >= PB) break;
            const int k = k0 + 4 * s + kk;
            const double b = keep_if(bb.v[s], cok & (k < PB));
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (rg + u >= mt) break;
              const int row = ((rg + u) << 4) + l16;
              const double a = (row < PA && k < PB) ? vat(row * PB + k) : 0.0;
              acc[u] = mfma64(a, b, acc[u]);
            }
          }
          if (k0 + 32 >= PB) {  // the column tile is complete
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int r = ((rg + u) << 4) + kk + 4 * e;
                if (rg + u < mt && r < PA && cok) Y[(long long)r * N + col] = acc[u][e];
              }
              acc[u] = d4{0, 0, 0, 0};
            }
          }
        });
    nm += (unsigned long long)nt * min(4, mt - rg) * ((PB + 3) >> 2);
  }
  __threadfence_block();
  // T4[(al,a)][g] = sum_b D_AB[a][b] Y[al][b][g]: D_AB fragments once, two alphas' Y at a time
  double t4max = 0.0;
  if (L.okAB) {
    gmem<double> *T4 = slot + L.a_t4[jj];
    for (int g0 = 0; g0 < ng; g0 += 16) {
      double sq = 0.0;  // sum over (al, a) of T4^2 for column g = g0 + l16 (this lane's rows)
      const int g = g0 + l16;
      for (int a0 = 0; a0 < na; a0 += 16) {
        double av[MAXN / 4];
#pragma unroll
        for (int s = 0; s < MAXN / 4; ++s) {
          const int k = 4 * s + kk;
          av[s] = (a0 + l16 < na && k < nb) ? L.DAB[(a0 + l16) * nb + k] : 0.0;
        }
        if (nb <= 16) {
          // four alphas per step (K = nb <= 16: four K steps), the next four's loads in flight
          struct TB {
            double v[4][4];
          };
          const int gc = min(g, ng - 1);
          pipelined<TB>(
              (PA + 3) >> 2,
              [&](int t, TB &bb) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                  for (int s = 0; s < 4; ++s)
                    bb.v[q][s] = Y[(long long)min(4 * t + q, PA - 1) * N + min(4 * s + kk, nb - 1) * ng + gc];
              },
              [&](int t, const TB &bb) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int al = 4 * t + q;
                  if (al >= PA) break;
                  d4 h = {0, 0, 0, 0};
#pragma unroll
                  for (int s = 0; s < 4; ++s)
                    if (4 * s < nb) h = mfma64(av[s], keep_if(bb.v[q][s], (4 * s + kk < nb) & (g < ng)), h);
                  for (int e = 0; e < 4; ++e) {
                    const int a = a0 + kk + 4 * e;
                    if (a < na && g < ng) {
                      T4[((long long)al * na + a) * ng + g] = h[e];
                      sq += h[e] * h[e];
                    }
                  }
                }
              });
        } else
        for (int al0 = 0; al0 < PA; al0 += 2) {
          double bv[2][MAXN / 4];
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int s = 0; s < MAXN / 4; ++s) {
              const int k = 4 * s + kk, al = al0 + q;
              bv[q][s] = (al < PA && k < nb && g < ng) ? Y[(long long)al * N + k * ng + g] : 0.0;
            }
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int al = al0 + q;
            if (al >= PA) break;
            d4 h = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < MAXN / 4; ++s)
              if (4 * s < nb) h = mfma64(av[s], bv[q][s], h);
            for (int e = 0; e < 4; ++e) {
              const int a = a0 + kk + 4 * e;
              if (a < na && g < ng) {
                T4[((long long)al * na + a) * ng + g] = h[e];
                sq += h[e] * h[e];
              }
            }
          }
        }
        nm += (unsigned long long)PA * ((nb + 3) >> 2);
      }
      sq += __shfl_xor(sq, 16);
      sq += __shfl_xor(sq, 32);
      t4max = fmax(t4max, wave_max(sq));
    }
  }
  // T3[(al,a)][b] = sum_g D_AG[a][g] Y[al][b][g]: D_AG fragments once, two alphas' Y at a time
  double t3max = 0.0;
  const int dAG = L.g_dAG[j];
  if (dAG >= 0 && gptr(P.keepD)[dAG]) {
    const gmem<const double> *DAG = gptr(P.Dbuf) + L.g_dAGoff[j];
    gmem<double> *T3 = slot + L.a_t3[jj];
    for (int b0 = 0; b0 < nb; b0 += 16) {
      double sq = 0.0;  // sum over (al, a) of T3^2 for column b = b0 + l16 (this lane's rows)
      const int b = b0 + l16;
      for (int a0 = 0; a0 < na; a0 += 16) {
        double av[MAXN / 4];
#pragma unroll
        for (int s = 0; s < MAXN / 4; ++s) {
          const int k = 4 * s + kk;
          av[s] = (a0 + l16 < na && k < ng) ? DAG[(a0 + l16) * ng + k] : 0.0;
        }
        if (ng <= 16) {
          // four alphas per step (K = ng <= 16), as for T4
          struct TB {
            double v[4][4];
          };
          const int bc = min(b, nb - 1);
          pipelined<TB>(
              (PA + 3) >> 2,
              [&](int t, TB &bb) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                  for (int s = 0; s < 4; ++s)
                    bb.v[q][s] = Y[(long long)min(4 * t + q, PA - 1) * N + bc * ng + min(4 * s + kk, ng - 1)];
              },
              [&](int t, const TB &bb) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int al = 4 * t + q;
                  if (al >= PA) break;
                  d4 h = {0, 0, 0, 0};
#pragma unroll
                  for (int s = 0; s < 4; ++s)
                    if (4 * s < ng) h = mfma64(av[s], keep_if(bb.v[q][s], (4 * s + kk < ng) & (b < nb)), h);
                  for (int e = 0; e < 4; ++e) {
                    const int a = a0 + kk + 4 * e;
                    if (a < na && b < nb) {
                      T3[((long long)al * na + a) * nb + b] = h[e];
                      sq += h[e] * h[e];
                    }
                  }
                }
              });
        } else
        for (int al0 = 0; al0 < PA; al0 += 2) {
          double bv[2][MAXN / 4];
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int s = 0; s < MAXN / 4; ++s) {
              const int k = 4 * s + kk, al = al0 + q;
              bv[q][s] = (al < PA && k < ng && b < nb) ? Y[(long long)al * N + b * ng + k] : 0.0;
            }
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int al = al0 + q;
            if (al >= PA) break;
            d4 h = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < MAXN / 4; ++s)
              if (4 * s < ng) h = mfma64(av[s], bv[q][s], h);
            for (int e = 0; e < 4; ++e) {
              const int a = a0 + kk + 4 * e;
              if (a < na && b < nb) {
                T3[((long long)al * na + a) * nb + b] = h[e];
                sq += h[e] * h[e];
              }
            }
          }
        }
        nm += (unsigned long long)PA * ((ng + 3) >> 2);
      }
      sq += __shfl_xor(sq, 16);
      sq += __shfl_xor(sq, 32);
      t3max = fmax(t3max, wave_max(sq));
    }
  }
  // N1[b][g][g'] = sum_al Y[al][b][g] Y[al][b][g'];  Yb^2 = max_b trace N1[b]
  gmem<double> *N1 = slot + L.a_n1[jj];
  double ybmax = 0.0;
  struct GB {
    double v[16];
  };
  if (ng <= 16 && PA <= 64) {
    // one 16x16 tile per b over K = PA <= 64; both operands are the same fragment Y[k][b][l16], one
    // load per K step; the next b's loads in flight during the current's MFMAs
    const int gl = min(l16, ng - 1);
    pipelined<GB>(
        nb,
        [&](int b, GB &bb) {
#pragma unroll
          for (int s = 0; s < 16; ++s) bb.v[s] = Y[(long long)min(4 * s + kk, PA - 1) * N + b * ng + gl];
        },
        [&](int b, const GB &bb) {
          d4 h = {0, 0, 0, 0};
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            if (4 * s >= PA) break;
            const double y = keep_if(bb.v[s], (4 * s + kk < PA) & (l16 < ng));
            h = mfma64(y, y, h);
          }
          double tr = 0.0;
          for (int e = 0; e < 4; ++e) {
            const int g = kk + 4 * e, g2 = l16;
            if (g < ng && g2 < ng) {
              N1[((long long)b * ng + g) * ng + g2] = h[e];
              if (g == g2) tr += h[e];
            }
          }
          ybmax = fmax(ybmax, wave_sum(tr));
        });
  } else
  for (int b = 0; b < nb; ++b) {
    double tr = 0.0;
    for (int g0 = 0; g0 < ng; g0 += 16)
      for (int h0 = 0; h0 < ng; h0 += 16) {
        d4 h = {0, 0, 0, 0};
        for (int k0 = 0; k0 < PA; k0 += 32) {
          const gmem<const double> *Yk = Y + (long long)k0 * N + b * ng;
          const int K = min(32, PA - k0);
          h = tile_mm_burst(
              K, [&](int r, int k) { return g0 + r < ng ? Yk[(long long)k * N + g0 + r] : 0.0; },
              [&](int k, int c) { return h0 + c < ng ? Yk[(long long)k * N + h0 + c] : 0.0; }, h);
        }
        for (int e = 0; e < 4; ++e) {
          const int g = g0 + kk + 4 * e, g2 = h0 + l16;
          if (g < ng && g2 < ng) {
            N1[((long long)b * ng + g) * ng + g2] = h[e];
            if (g == g2) tr += h[e];
          }
        }
      }
    ybmax = fmax(ybmax, wave_sum(tr));
  }
  // M2[g][b][b'] = sum_al Y[al][b][g] Y[al][b'][g];  Yg^2 = max_g trace M2[g]
  gmem<double> *M2 = slot + L.a_m2[jj];
  double ygmax = 0.0;
  if (nb <= 16 && PA <= 64) {
    // as N1: one tile per g, both operands the fragment Y[k][l16][g]
    const int bl = min(l16, nb - 1);
    pipelined<GB>(
        ng,
        [&](int g, GB &bb) {
#pragma unroll
          for (int s = 0; s < 16; ++s) bb.v[s] = Y[(long long)min(4 * s + kk, PA - 1) * N + bl * ng + g];
        },
        [&](int g, const GB &bb) {
          d4 h = {0, 0, 0, 0};
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            if (4 * s >= PA) break;
            const double y = keep_if(bb.v[s], (4 * s + kk < PA) & (l16 < nb));
            h = mfma64(y, y, h);
          }
          double tr = 0.0;
          for (int e = 0; e < 4; ++e) {
            const int b = kk + 4 * e, b2 = l16;
            if (b < nb && b2 < nb) {
              M2[((long long)g * nb + b) * nb + b2] = h[e];
              if (b == b2) tr += h[e];
            }
          }
          ygmax = fmax(ygmax, wave_sum(tr));
        });
  } else
  for (int g = 0; g < ng; ++g) {
    double tr = 0.0;
    for (int b0 = 0; b0 < nb; b0 += 16)
      for (int c0 = 0; c0 < nb; c0 += 16) {
        d4 h = {0, 0, 0, 0};
        for (int k0 = 0; k0 < PA; k0 += 32) {
          const gmem<const double> *Yk = Y + (long long)k0 * N + g;
          const int K = min(32, PA - k0);
          h = tile_mm_burst(
              K, [&](int r, int k) { return b0 + r < nb ? Yk[(long long)k * N + (b0 + r) * ng] : 0.0; },
              [&](int k, int c) { return c0 + c < nb ? Yk[(long long)k * N + (c0 + c) * ng] : 0.0; }, h);
        }
        for (int e = 0; e < 4; ++e) {
          const int b = b0 + kk + 4 * e, b2 = c0 + l16;
          if (b < nb && b2 < nb) {
            M2[((long long)g * nb + b) * nb + b2] = h[e];
            if (b == b2) tr += h[e];
          }
        }
      }
    ygmax = fmax(ygmax, wave_sum(tr));
  }
  const int tn = ((ng + 15) >> 4) * ((ng + 15) >> 4) * nb + ((nb + 15) >> 4) * ((nb + 15) >> 4) * ng;
  nm += (unsigned long long)tn * ((PA + 3) >> 2);
  if (lane == 0) {
    L.a_Yb[jj] = sqrt(ybmax);
    L.a_Yg[jj] = sqrt(ygmax);
    L.a_T3n[jj] = sqrt(t3max);
    L.a_T4n[jj] = sqrt(t4max);
    atomicAdd(&L.cnt[kCntMfmaY], nm);
  }
}

// ---------------------------------------------------------------------------------------------
// masks: stages 2 and 3 for the stage-1 survivors of alive G's
__device__ void phase_masks(const DevPlan &P, ItemLds &L, gmem<double> *slot, const gmem<int> *dfg,
                            const gmem<long long> *doff, gmem<uint8_t> *mask, gmem<double> *E2, gmem<double> *wreg,
                            gmem<float> *ub) {
  const gmem<const double> *gD = gptr(P.gD), *Dbuf = gptr(P.Dbuf);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kk = lane >> 4, l16 = lane & 15;
  const int nb = L.nb, nF = L.nF, nGa = L.nGa, nG = L.nG;
  const double eps = P.eps_mat;
  const bool use2 = P.stages & kCs2, use3 = P.stages & kCs3;
  unsigned long long c2[4] = {0, 0, 0, 0}, c3[4] = {0, 0, 0, 0}, nm = 0;
  // the tightest bound of every kept unit (stage 3 where it runs, else stage 2), summed: an
  // upper bound of the Frobenius norm of the item's contribution to Sigma (weights <= 1)
  double cb = 0.0;
  // E2_i = D_FB^T D_FB  [b][b']  (one wave per F)
  for (int i = wave; i < nF; i += NW) {
    gmem<double> *E = E2 + (long long)i * nb * nb;
    const int dFB = L.f_dFB[i];
    const int nf = L.f_n[i];
    if (dFB < 0) continue;
    const gmem<const double> *D = Dbuf + L.f_dFBoff[i];
    for (int b0 = 0; b0 < nb; b0 += 16)
      for (int c0 = 0; c0 < nb; c0 += 16) {
        const d4 h = tile_mm(
            nf, [&](int r, int k) { return (b0 + r < nb && k < nf) ? D[k * nb + b0 + r] : 0.0; },
            [&](int k, int c) { return (k < nf && c0 + c < nb) ? D[k * nb + c0 + c] : 0.0; });
        for (int e = 0; e < 4; ++e) {
          const int b = b0 + kk + 4 * e, b2 = c0 + l16;
          if (b < nb && b2 < nb) E[b * nb + b2] = h[e];
        }
        nm += (nf + 3) >> 2;
      }
  }
  // stage 2 for every term, stage 3 for terms 3 and 4; terms 1 and 2 marked pending
  for (int p = tid; p < nF * nGa; p += NT) {
    const int i = p / nGa, jj = p - i * nGa;
    const int j = L.a_j[jj];
    const int q = i * nG + j;
    uint8_t bits = mask[q];
    if (!(bits & 15)) {
      if (ub) ub[2 * p] = ub[2 * p + 1] = 0.0f;
      continue;
    }
    if (bits & kT1) {
      const double b = L.f_gA[i] * L.a_Yb[jj] * gD[dfg[q]];
      if (!use2 || b > eps) {
        ++c2[0];
        if (use3) {
          bits |= kPend1;
        } else {
          ++c3[0];
          cb += b;
        }
      } else {
        bits &= ~kT1;
      }
    }
    if (bits & kT2) {
      const double b = L.f_gA[i] * L.a_Yg[jj] * gD[L.f_dFB[i]];
      if (!use2 || b > eps) {
        ++c2[1];
        if (use3) {
          bits |= kPend2;
        } else {
          ++c3[1];
          cb += b;
        }
      } else {
        bits &= ~kT2;
      }
    }
    if (bits & kT3) {
      double b = L.f_gF[i] * L.a_Yb[jj] * gD[L.g_dAG[j]];
      bool keep = !use2 || b > eps;
      if (keep) {
        ++c2[2];
        if (use3) {
          b = L.f_nF[i] * L.a_T3n[jj];
          keep = b > eps;
        }
        if (keep) {
          ++c3[2];
          cb += b;
        }
      }
      if (!keep) bits &= ~kT3;
    }
    if (bits & kT4) {
      double b = L.f_gF[i] * L.a_Yg[jj] * gD[L.dAB];
      bool keep = !use2 || b > eps;
      if (keep) {
        ++c2[3];
        if (use3) {
          b = L.f_nF[i] * L.a_T4n[jj];
          keep = b > eps;
        }
        if (keep) {
          ++c3[3];
          cb += b;
        }
      }
      if (!keep) bits &= ~kT4;
    }
    mask[q] = bits;
    if (ub) {
      // stage-2 bounds of the surviving units, per GEMM: [0] terms 1, 2; [1] terms 3, 4
      float bl = 0.0f, br = 0.0f;
      if (bits & kT1) bl = fmaxf(bl, (float)(L.f_gA[i] * L.a_Yb[jj] * gD[dfg[q]]));
      if (bits & kT2) bl = fmaxf(bl, (float)(L.f_gA[i] * L.a_Yg[jj] * gD[L.f_dFB[i]]));
      if (bits & kT3) br = fmaxf(br, (float)(L.f_gF[i] * L.a_Yb[jj] * gD[L.g_dAG[j]]));
      if (bits & kT4) br = fmaxf(br, (float)(L.f_gF[i] * L.a_Yg[jj] * gD[L.dAB]));
      ub[2 * p] = bl;
      ub[2 * p + 1] = br;
    }
  }
  __syncthreads();
  if (use3) {
    // term 2, stage 3: ||T2[:,:,g]||^2 = <E2_F, M2_G[g]> for every (F, G): one 16-F x 16-g tile
    // per (F tile, G) over K = nb*nb
    const int nft = (nF + 15) >> 4;
    for (int t = wave; t < nft * nGa; t += NW) {
      const int it = t / nGa, jj = t - it * nGa;
      const int j = L.a_j[jj], ng = L.g_n[j];
      const int i = (it << 4) + l16;
      const bool pend = i < nF && (mask[i * nG + j] & kPend2);
      if (!__any(pend)) continue;
      const gmem<const double> *M2 = slot + L.a_m2[jj];
      const int K = nb * nb;
      double smax[4] = {0.0, 0.0, 0.0, 0.0};
      for (int g0 = 0; g0 < ng; g0 += 16) {
        const d4 h = tile_mm_long(
            K, [&](int r, int k) { return E2[(long long)min((it << 4) + r, nF - 1) * K + k]; },
            [&](int k, int c) { return M2[(long long)min(g0 + c, ng - 1) * K + k]; });
        nm += (K + 3) >> 2;
        for (int e = 0; e < 4; ++e) smax[e] = fmax(smax[e], (g0 + l16 < ng) ? h[e] : 0.0);
      }
      for (int e = 0; e < 4; ++e) {
        double v = smax[e];
        for (int o = 1; o < 16; o <<= 1) v = fmax(v, __shfl_xor(v, o));
        const int ii = (it << 4) + kk + 4 * e;
        if (l16 == 0 && ii < nF) {
          const int q = ii * nG + j;
          const uint8_t bits = mask[q];
          if (bits & kPend2) {
            const double b = L.f_nA[ii] * sqrt(fmax(v, 0.0));
            const bool keep = b > eps;
            mask[q] = keep ? (uint8_t)(bits & ~kPend2) : (uint8_t)(bits & ~(kPend2 | kT2));
            if (keep) {
              ++c3[1];
              cb += b;
            }
          }
        }
      }
    }
    __syncthreads();
    // term 1, stage 3: ||T1[:,:,b]||^2 = <D_FG^T D_FG, N1_G[b]>; per G, 16 pending F's at a time:
    // E1_F = D_FG^T D_FG into the wave's scratch, then one 16-F x 16-b tile over K = ng*ng
    gmem<double> *E1 = wreg;  // [16][MAXN*MAXN]
    for (int jj = wave; jj < nGa; jj += NW) {
      const int j = L.a_j[jj], ng = L.g_n[j];
      const int K = ng * ng;
      const gmem<const double> *N1 = slot + L.a_n1[jj];
      int ib = 0;
      for (;;) {
        // next batch of up to 16 pending F's
        int fl[16];
        int nbat = 0;
        while (nbat < 16 && ib < nF) {
          const int i = ib + lane;
          const bool pend = i < nF && (mask[i * nG + j] & kPend1);
          unsigned long long bm = __ballot(pend);
          while (bm && nbat < 16) {
            const int o = __builtin_ctzll(bm);
            bm &= bm - 1;
            fl[nbat++] = ib + o;
          }
          ib = bm ? ib + __builtin_ctzll(bm) : ib + 64;
        }
        if (nbat == 0) break;
        for (int r = 0; r < nbat; ++r) {
          const int i = fl[r], nf = L.f_n[i];
          const gmem<const double> *D = Dbuf + doff[i * nG + j];
          for (int g0 = 0; g0 < ng; g0 += 16)
            for (int h0 = 0; h0 < ng; h0 += 16) {
              const d4 h = tile_mm(
                  nf, [&](int rr, int k) { return (g0 + rr < ng && k < nf) ? D[k * ng + g0 + rr] : 0.0; },
                  [&](int k, int c) { return (k < nf && h0 + c < ng) ? D[k * ng + h0 + c] : 0.0; });
              nm += (nf + 3) >> 2;
              for (int e = 0; e < 4; ++e) {
                const int g = g0 + kk + 4 * e, g2 = h0 + l16;
                if (g < ng && g2 < ng) E1[r * MAXN * MAXN + g * ng + g2] = h[e];
              }
            }
        }
        __threadfence_block();
        double smax[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b0 = 0; b0 < nb; b0 += 16) {
          const d4 h = tile_mm_long(
              K, [&](int r, int k) { return E1[min(r, nbat - 1) * MAXN * MAXN + k]; },
              [&](int k, int c) { return N1[(long long)min(b0 + c, nb - 1) * K + k]; });
          nm += (K + 3) >> 2;
          for (int e = 0; e < 4; ++e) smax[e] = fmax(smax[e], (b0 + l16 < nb) ? h[e] : 0.0);
        }
        for (int e = 0; e < 4; ++e) {
          double v = smax[e];
          for (int o = 1; o < 16; o <<= 1) v = fmax(v, __shfl_xor(v, o));
          const int r = kk + 4 * e;
          if (l16 == 0 && r < nbat) {
            const int i = fl[r];
            const int q = i * nG + j;
            const uint8_t bits = mask[q];
            const double b = L.f_nA[i] * sqrt(fmax(v, 0.0));
            const bool keep = b > eps;
            mask[q] = keep ? (uint8_t)(bits & ~kPend1) : (uint8_t)(bits & ~(kPend1 | kT1));
            if (keep) {
              ++c3[0];
              cb += b;
            }
          }
        }
        __threadfence_block();
      }
    }
  }
  for (int t = 0; t < 4; ++t) {
    if (c2[t]) atomicAdd(&L.cnt[kCntKept + 4 + t], c2[t]);
    if (c3[t]) atomicAdd(&L.cnt[kCntKept + 8 + t], c3[t]);
  }
  if (cb != 0.0) atomicAdd(&L.contrib, cb);
  if (lane == 0 && nm) atomicAdd(&L.cnt[kCntMfmaY], nm);
}

// the masks phase out of line, with a register allocation of its own: in the kernels that carry
// the FP32 tier (and not split-BF16x3) this measured faster; in the others inline is faster
__device__ __noinline__ void phase_masks_ool(const DevPlan &P, ItemLds &L, gmem<double> *slot, const gmem<int> *dfg,
                                            const gmem<long long> *doff, gmem<uint8_t> *mask, gmem<double> *E2,
                                            gmem<double> *wreg, gmem<float> *ub) {
  phase_masks(P, L, slot, dfg, doff, mask, E2, wreg, ub);
}

__device__ __forceinline__ double unit_weight(const ItemLds &L, int i, int j) {
  return (L.f_on[i] ? 0.5 : 1.0) * (L.g_on[j] ? 0.5 : 1.0);
}

// ---------------------------------------------------------------------------------------------
// Workgroup block products: a 128-row x W-column output block (W = 128, 64 or 32), K streamed through
// two LDS stages in chunks.  Every thread fetches its share of a chunk's A and B elements into
// registers two chunks ahead: the loads of chunk c+2 are issued before the MFMAs of chunk c, and
// chunk c+1 (fetched one chunk earlier) is stored into the other stage after them, so a load has
// two chunks of matrix-core work to land.  Wave w owns row tile w and the W/16 column tiles (act:
// which of them to compute).
//
// a_at(k) / b_at(k) load this thread's A / B element at k from an in-bounds address for every
// k < K; the element counts only if aok and k < Ka (A) or bok and k < K (B), else a zero is stored
// in its place.  The test is applied when the element is stored into LDS, so that nothing waits
// for a load before then, and fetches and stores run also past the end of K (clamped loads,
// zeros stored): with no branch around them the compiler knows how many loads are in flight at
// each store and waits only for the older chunk's.
constexpr int BM = 128, BN = 64, BK = 16;  // BN: the column width of the terms-1/2 blocks
constexpr int BNR = 128;                    // the widest terms-3/4 block (B stage size)

// The chunk pipeline shared by the block products.  R: one chunk's registers; fetch(k0, R&)
// loads chunk k0, stash(st, k0, const R&) stores it into stage st, compute(st) runs the MFMAs of
// stage st (only in a wave with work, active: the same in all its lanes).  Fetch, MFMAs and store
// of a chunk are independent of each other and branch-free, one basic block, so that the
// compiler can interleave the memory instructions with the MFMAs.  Chunk pairs, then an odd last
// chunk: no exit from the middle of the loop body, whose edge back to the loop head would make
// the compiler wait there for the first chunk's loads.
template <int CK, class R, class Fetch, class Stash, class Compute>
__device__ __forceinline__ void chunk_pipeline(int K, bool active, Fetch fetch, Stash stash, Compute compute) {
  R r0, r1;
  auto step = [&](int k0, int st, R &rf, const R &rs) {
    if (active) {
      fetch(k0 + 2 * CK, rf);
      compute(st);
      stash(st ^ 1, k0 + CK, rs);
    } else {
      fetch(k0 + 2 * CK, rf);
      stash(st ^ 1, k0 + CK, rs);
    }
    __syncthreads();
  };
  __syncthreads();  // the previous user of the stages is done
  fetch(0, r0);
  stash(0, 0, r0);
  fetch(CK, r1);
  __syncthreads();
  const int nch = (K + CK - 1) / CK;
  int c = 0;
  for (; c + 1 < nch; c += 2) {
    step(c * CK, 0, r0, r1);
    step((c + 1) * CK, 1, r1, r0);
  }
  if (c < nch) step(c * CK, 0, r0, r1);
}

// FP64 (v_mfma_f64_16x16x4f64), BK = 16 K per chunk: four A elements (row tid&127) and W/32 B
// elements (column tid%W) per thread.
template <int W, bool SPLIT, class AAt, class BAt>
__device__ __forceinline__ void wg_block_mm(int K, AAt a_at, BAt b_at, bool aok, int Ka, bool bok, unsigned act,
                                            double *As, double *Bs, d4 (&acc)[W / 16]) {
  // As, Bs: two stages each ([2][BK][BM], [2][BK][W])
  constexpr int NV = W / 16, RS = NT / W, NBF = BK / RS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kk = lane >> 4, l16 = lane & 15;
  const int ar = tid & (BM - 1), akq = (tid >> 7) << 2;
  const int bc = tid & (W - 1), bk = tid / W;
  const unsigned actw = __builtin_amdgcn_readfirstlane(act);  // the same in every lane of the wave
  struct Regs {
    double a[4], b[NBF];
  };
  auto fetch = [&](int k0, Regs &r) {
#pragma unroll
    for (int s = 0; s < 4; ++s) r.a[s] = a_at(min(k0 + akq + s, K - 1));
#pragma unroll
    for (int q = 0; q < NBF; ++q) r.b[q] = b_at(min(k0 + bk + q * RS, K - 1));
  };
  auto stash = [&](int st, int k0, const Regs &r) {
    double *a = As + st * BK * BM, *b = Bs + st * BK * W;
#pragma unroll
    for (int s = 0; s < 4; ++s) a[(akq + s) * BM + ar] = keep_if(r.a[s], aok & (k0 + akq + s < Ka));
#pragma unroll
    for (int q = 0; q < NBF; ++q) b[(bk + q * RS) * W + bc] = keep_if(r.b[q], bok & (k0 + bk + q * RS < K));
  };
  // MFMAs of stage st for the tiles in m (all of them: branch-free, so that the step stays one
  // basic block; some: a wave-uniform branch per tile)
  auto compute = [&](int st, unsigned m, bool all) {
    const double *a = As + st * BK * BM + wave * 16 + l16, *b = Bs + st * BK * W + l16;
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const int kr = 4 * s + kk;
      const double av = a[kr * BM];
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (all || (m & (1u << v))) acc[v] = mfma64(av, b[kr * W + v * 16], acc[v]);
    }
  };
  // SPLIT: a wave with every tile active runs the branch-free step, one with some the per-tile
  // one; else every tile of an active wave (where a second copy of the pipeline would spill
  // registers: W = 128, and the kernels that also hold the split-BF16x3 form)
  constexpr unsigned FULL = (1u << NV) - 1u;
  if (!SPLIT || actw == FULL)
    chunk_pipeline<BK, Regs>(K, actw != 0, fetch, stash, [&](int st) { compute(st, FULL, true); });
  else
    chunk_pipeline<BK, Regs>(K, actw != 0, fetch, stash, [&](int st) { compute(st, actw, false); });
}

// FP32 (v_mfma_f32_16x16x4f32), BKF K per chunk: BKF/4 A elements (row tid&127, k rows
// (BKF/4)*(tid>>7)..) and BKF/8 B elements (column tid&63, k rows tid>>6 + 8q) per thread.  B
// arrives in FP64 (T3/T4, the D panel) and is rounded when it is stored into the stage.  (32-K
// FP32 chunks fit the same LDS; measured no faster and they spill more registers.)
constexpr int BKF = 16;
static_assert(BKF * (BM + BN) * 4 <= BK * (BM + BN) * 8, "FP32 stages reuse the FP64 stage buffers");

template <int W, class AAt, class BAt>
__device__ __forceinline__ void wg_block_mm32(int K, AAt a_at, BAt b_at, bool aok, int Ka, bool bok, unsigned act,
                                              float *As, float *Bs, f4 (&acc)[W / 16]) {
  constexpr int NV = W / 16, RS = NT / W, NA = BKF / 4, NB = BKF / RS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kk = lane >> 4, l16 = lane & 15;
  const int ar = tid & (BM - 1), akq = (tid >> 7) * NA;
  const int bc = tid & (W - 1), bk = tid / W;
  const unsigned actw = __builtin_amdgcn_readfirstlane(act);
  struct Regs {
    float a[NA];
    double b[NB];
  };
  auto fetch = [&](int k0, Regs &r) {
#pragma unroll
    for (int s = 0; s < NA; ++s) r.a[s] = a_at(min(k0 + akq + s, K - 1));
#pragma unroll
    for (int q = 0; q < NB; ++q) r.b[q] = b_at(min(k0 + bk + RS * q, K - 1));
  };
  auto stash = [&](int st, int k0, const Regs &r) {
    float *a = As + st * BKF * BM, *b = Bs + st * BKF * W;
#pragma unroll
    for (int s = 0; s < NA; ++s) a[(akq + s) * BM + ar] = keep_if(r.a[s], aok & (k0 + akq + s < Ka));
#pragma unroll
    for (int q = 0; q < NB; ++q)
      b[(bk + RS * q) * W + bc] = keep_if((float)r.b[q], bok & (k0 + bk + RS * q < K));
  };
  // every tile of an active wave, branch-free (a second, per-tile copy of the pipeline as in the
  // FP64 form spills registers in the kernels that hold both forms)
  chunk_pipeline<BKF, Regs>(K, actw != 0, fetch, stash, [&](int st) {
    const float *a = As + st * BKF * BM + wave * 16 + l16, *b = Bs + st * BKF * W + l16;
#pragma unroll
    for (int s = 0; s < BKF / 4; ++s) {
      const int kr = 4 * s + kk;
      const float av = a[kr * BM];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = mfma32(av, b[kr * W + v * 16], acc[v]);
    }
  });
}

// ---------------------------------------------------------------------------------------------
// Split-BF16x3 block product (the lowest precision tier of terms 3 and 4): every FP32 operand is
// split as x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to nearest even), and the
// product is accumulated in FP32 as hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 (lane l
// supplies row l%16 of A and column l%16 of B at k = 8(l/16)..8(l/16)+7; the result layout is the
// FP32 form's).  The dropped lo*lo term and the rounding of lo leave about 2^-16 relative error
// per product.  K is streamed in chunks of 32 through two LDS stages holding hi and lo rows with
// k contiguous.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int BKB = 32;

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <int W, class AAt, class BAt>
__device__ __forceinline__ void wg_block_mm_bf3(int K, AAt a_at, BAt b_at, bool aok, int Ka, bool bok, unsigned act,
                                                uint16_t *As, uint16_t *Bs, f4 (&acc)[W / 16]) {
  constexpr int NV = W / 16, KB = BKB * W / NT;  // B elements per thread and chunk (4 or 2)
  constexpr int ASZ = 2 * BM * BKB, BSZ = 2 * W * BKB;  // one stage: hi block then lo block
  static_assert(2 * ASZ * 2 <= 2 * BK * BM * 8 && 2 * BSZ * 2 <= 2 * BK * BNR * 8, "BF16 stages fit the FP64 ones");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kg = lane >> 4, l16 = lane & 15;
  const int ar = tid & (BM - 1), ako = (tid >> 7) * 8;
  const int bc = tid & (W - 1), bko = (tid / W) * KB;
  const unsigned actw = __builtin_amdgcn_readfirstlane(act);
  struct Regs {
    float a[8];
    double b[KB];
  };
  chunk_pipeline<BKB, Regs>(
      K, actw != 0,
      [&](int k0, Regs &r) {
#pragma unroll
        for (int s = 0; s < 8; ++s) r.a[s] = a_at(min(k0 + ako + s, K - 1));
#pragma unroll
        for (int q = 0; q < KB; ++q) r.b[q] = b_at(min(k0 + bko + q, K - 1));
      },
      [&](int st, int k0, const Regs &r) {
        uint16_t *a = As + st * ASZ, *b = Bs + st * BSZ;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const float x = keep_if(r.a[s], aok & (k0 + ako + s < Ka));
          const uint16_t h = bf16_rne(x);
          a[ar * BKB + ako + s] = h;
          a[BM * BKB + ar * BKB + ako + s] = bf16_rne(x - bf16_val(h));
        }
#pragma unroll
        for (int q = 0; q < KB; ++q) {
          const float x = keep_if((float)r.b[q], bok & (k0 + bko + q < K));
          const uint16_t h = bf16_rne(x);
          b[bc * BKB + bko + q] = h;
          b[W * BKB + bc * BKB + bko + q] = bf16_rne(x - bf16_val(h));
        }
      },
      [&](int st) {
        const uint16_t *a = As + st * ASZ, *b = Bs + st * BSZ;
        const bf8 ahi = *reinterpret_cast<const bf8 *>(a + (wave * 16 + l16) * BKB + kg * 8);
        const bf8 alo = *reinterpret_cast<const bf8 *>(a + BM * BKB + (wave * 16 + l16) * BKB + kg * 8);
#pragma unroll
        for (int v = 0; v < NV; ++v) {  // every tile of an active wave: per-tile tests cost registers
          const bf8 bhi = *reinterpret_cast<const bf8 *>(b + (v * 16 + l16) * BKB + kg * 8);
          const bf8 blo = *reinterpret_cast<const bf8 *>(b + W * BKB + (v * 16 + l16) * BKB + kg * 8);
          acc[v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[v], 0, 0, 0);
          acc[v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[v], 0, 0, 0);
          acc[v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[v], 0, 0, 0);
        }
      });
}

// largest recorded bound over the alive G's whose columns meet [c_lo, c_hi), for row F_i
__device__ __forceinline__ float cols_ub(const ItemLds &L, const gmem<const float> *ub, const short *col2jj, int i,
                                         int c_lo, int c_hi, int which) {
  float m = 0.0f;
  if (c_lo >= c_hi) return m;
  const int jj0 = col2jj[c_lo], jj1 = col2jj[c_hi - 1];
  for (int jj = jj0; jj <= jj1; ++jj) m = fmaxf(m, ub[2 * (i * L.nGa + jj) + which]);
  return m;
}

// which of the four 16-column tiles of [c_lo, c_lo+64) hold a half (g or b) of some alive G
// whose bit for F_i is set: bits_g for the g-half, bits_b for the b-half
__device__ __forceinline__ bool tile_has(const ItemLds &L, const gmem<const uint8_t> *mask, const short *col2jj, int i,
                                         int c_lo, int c_hi, uint8_t bits_g, uint8_t bits_b) {
  if (c_lo >= c_hi) return false;
  const int jj0 = col2jj[c_lo], jj1 = col2jj[c_hi - 1];
  for (int jj = jj0; jj <= jj1; ++jj) {
    const int j = L.a_j[jj];
    const int g0 = L.a_col0[jj], gb = g0 + L.g_n[j], g1 = L.a_col0[jj + 1];
    const uint8_t bits = mask[i * L.nG + j];
    if ((bits & bits_g) && max(c_lo, g0) < min(c_hi, gb)) return true;
    if ((bits & bits_b) && max(c_lo, gb) < min(c_hi, g1)) return true;
  }
  return false;
}

// ---------------------------------------------------------------------------------------------
// GEMM-R: terms 3 and 4.  Rows (F,f), K = (alpha,a), columns (G, [g | b]):
//   out[(F,f)][(G,g)] = sum_{al,a} C_AF[al][a][f] T4_G[al][a][g]  -> Sigma(F,G)  (term 4)
//   out[(F,f)][(G,b)] = sum_{al,a} C_AF[al][a][f] T3_G[al][a][b]  -> summed over G into Sigma(F,B)
// 128 x W blocks (W = 128, 64 or 32, the plan's tile_r) in row-block-major order; a block whose
// tiles hold no kept unit is skipped.
// PR: the precision forms compiled in (0: FP64 only; 1: FP64 and FP32; 2: FP64, FP32 and
// split-BF16x3), so that a plan's kernel carries no code, and no registers, for forms it never runs.
template <int W, int PR>
__device__ void phase_gemm_r(const DevPlan &P, ItemLds &L, const gmem<double> *slot, const gmem<long long> *doff,
                             const gmem<uint8_t> *mask, const uint8_t *row2i, const short *col2jj, double *As,
                             double *Bs, double *acc3, int ld3, const gmem<float> *ub, int tier, float tau,
                             float tau_bf) {
  gmem<double> *Sbuf = gptr(P.Sbuf);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kk = lane >> 4, l16 = lane & 15;
  const int K = L.PA * L.na, nb = L.nb;
  const bool tiered = tier == 1 || tier == 3;
  constexpr int NCT = W / 16;  // column tiles per block
  const int nrb = (L.MR + BM - 1) / BM, ncb = (L.NR + W - 1) / W;
  unsigned long long nmfma = 0, nmfma32 = 0, nmfmabf = 0;
  for (int rb = 0; rb < nrb; ++rb) {
    for (int q = lane; q < 16 * ld3; q += 64) acc3[q] = 0.0;
    bool any3 = false;
    // this thread's A row
    const int r = rb * BM + (tid & (BM - 1));
    const bool rok = r < L.MR;
    const int ia = rok ? row2i[r] : 0;
    const long long a_off = L.f_coff[ia] + (rok ? r - L.f_row0[ia] : 0);
    const gmem<const double> *Ab = gptr(P.Cbuf) + a_off;
    const gmem<const float> *Ab32 = tier ? gptr(P.C32) + a_off : nullptr;
    const int As_ = L.f_n[ia];
    for (int cb = 0; cb < ncb; ++cb) {
      if (tid == 0) {
        L.blk_act = 0;
        L.blk_ub = 0u;
      }
      __syncthreads();
      for (int t = tid; t < 8 * NCT * 16; t += NT) {
        const int sidx = t >> 4, wr = sidx / NCT, ct = sidx % NCT;
        const int rr = rb * BM + wr * 16 + (t & 15);
        if (rr < L.MR) {
          const int c_lo = cb * W + ct * 16, c_hi = min(c_lo + 16, L.NR);
          if (tile_has(L, mask, col2jj, row2i[rr], c_lo, c_hi, kT4, kT3)) {
            atomicOr(&L.blk_act, 1ull << sidx);
            if (tiered) atomicMax(&L.blk_ub, __float_as_uint(cols_ub(L, ub, col2jj, row2i[rr], c_lo, c_hi, 1)));
          }
        }
      }
      __syncthreads();
      const unsigned long long act_all = L.blk_act;
      if (!act_all) continue;
      const float bub = __uint_as_float(L.blk_ub);
      const bool bf = PR == 2 && tier == 3 && bub <= tau_bf;
      const bool fp32 = PR >= 1 && (bf || tier == 2 || (tiered && bub <= tau));
      const unsigned act = (unsigned)((act_all >> (NCT * wave)) & ((1ull << NCT) - 1ull));
      const int c = cb * W + (tid & (W - 1));
      const bool cok = c < L.NR;
      const gmem<const double> *Bb = slot;
      int Bstr = 0;
      if (cok) {
        const int jj = col2jj[c], j = L.a_j[jj];
        const int cc = c - L.a_col0[jj], ng = L.g_n[j];
        if (cc < ng) {
          Bb = slot + L.a_t4[jj] + cc;
          Bstr = ng;
        } else {
          Bb = slot + L.a_t3[jj] + (cc - ng);
          Bstr = nb;
        }
      }
      d4 acc[NCT];
      if constexpr (PR == 2) {
        if (bf) {
          f4 a32[NCT];
#pragma unroll
          for (int v = 0; v < NCT; ++v) a32[v] = f4{0, 0, 0, 0};
          wg_block_mm_bf3<W>(
              K, [&](int k) { return Ab32[(long long)k * As_]; }, [&](int k) { return Bb[(long long)k * Bstr]; },
              rok, K, cok, act, reinterpret_cast<uint16_t *>(As),
              reinterpret_cast<uint16_t *>(Bs), a32);
          nmfmabf += (unsigned long long)(act ? 3 * NCT : 0) * ((K + BKB - 1) / BKB);
#pragma unroll
          for (int v = 0; v < NCT; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[v][e] = (double)a32[v][e];
        }
      }
      if (bf) {
      } else if (fp32) {
        f4 a32[NCT];
#pragma unroll
        for (int v = 0; v < NCT; ++v) a32[v] = f4{0, 0, 0, 0};
        wg_block_mm32<W>(
            K, [&](int k) { return Ab32[(long long)k * As_]; }, [&](int k) { return Bb[(long long)k * Bstr]; }, rok, K,
            cok, act, reinterpret_cast<float *>(As),
            reinterpret_cast<float *>(Bs), a32);
        nmfma32 += (unsigned long long)(act ? NCT : 0) * ((K + 3) >> 2);
#pragma unroll
        for (int v = 0; v < NCT; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[v][e] = (double)a32[v][e];
      } else {
#pragma unroll
        for (int v = 0; v < NCT; ++v) acc[v] = d4{0, 0, 0, 0};
        wg_block_mm<W, (W <= 64 && PR < 2)>(
            K, [&](int k) { return Ab[(long long)k * As_]; }, [&](int k) { return Bb[(long long)k * Bstr]; }, rok, K,
            cok, act, As, Bs, acc);
        nmfma += (unsigned long long)((W <= 64 && PR < 2) ? __builtin_popcount(act) : (act ? NCT : 0)) * ((K + 3) >> 2);
      }
      // epilogue of this wave's tiles, four at a time: the (F,G) records of their elements are
      // loaded before the first atomic, so that the loads overlap one another
      int ei[4], ef[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = rb * BM + wave * 16 + (fp32 ? 4 * kk + e : kk + 4 * e);  // result row (MFMA form)
        ei[e] = rr < L.MR ? row2i[rr] : -1;
        ef[e] = ei[e] >= 0 ? rr - L.f_row0[ei[e]] : 0;
      }
#pragma unroll
      for (int h = 0; h < NCT; h += 4) {
        constexpr int NH = NCT < 4 ? NCT : 4;
        int vj[NH], vc[NH], vn[NH];
#pragma unroll
        for (int u = 0; u < NH; ++u) {
          const int cc0 = cb * W + (h + u) * 16 + l16;
          const bool ok = (act & (1u << (h + u))) && cc0 < L.NR;
          const int jj = ok ? col2jj[cc0] : 0, j = L.a_j[jj];
          vj[u] = ok ? j : -1;
          vc[u] = cc0 - L.a_col0[jj];
          vn[u] = L.g_n[j];
        }
        uint8_t ubits[NH][4];
        long long uoff[NH][4];
#pragma unroll
        for (int u = 0; u < NH; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool ok = vj[u] >= 0 && ei[e] >= 0;
            const int q = ok ? ei[e] * L.nG + vj[u] : 0;
            ubits[u][e] = ok ? mask[q] : 0;
            uoff[u][e] = doff[q];
          }
#pragma unroll
        for (int u = 0; u < NH; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint8_t bits = ubits[u][e];
            if (!(bits & (kT3 | kT4))) continue;
            const int i = ei[e], j = vj[u], cc = vc[u], ng = vn[u];
            const double w = unit_weight(L, i, j);
            const double x = acc[h + u][e];
            if (cc < ng) {
              if (bits & kT4) gatomic_add(Sbuf + uoff[u][e] + ef[e] * ng + cc, -w * x);
            } else if (bits & kT3) {
              atomicAdd(&acc3[(fp32 ? 4 * kk + e : kk + 4 * e) * ld3 + (cc - ng)], -w * x);
              any3 = true;
            }
          }
      }
    }
    // flush term 3 of this wave's 16 rows: Sigma(F,B)[f][b]
    if (__any(any3)) {
      for (int q = lane; q < 16 * nb; q += 64) {
        const int rl = q / nb, b = q - rl * nb;
        const int rr = rb * BM + wave * 16 + rl;
        if (rr >= L.MR) continue;
        const double v = acc3[rl * ld3 + b];
        if (v != 0.0) {
          const int i = row2i[rr], f = rr - L.f_row0[i];
          gatomic_add(Sbuf + L.f_dFBoff[i] + f * nb + b, v);
        }
      }
    }
  }
  if (lane == 0 && nmfma) atomicAdd(&L.cnt[kCntMfmaR], nmfma);
  if (lane == 0 && nmfma32) atomicAdd(&L.cnt[kCntMfmaR32], nmfma32);
  if (lane == 0 && nmfmabf) atomicAdd(&L.cnt[kCntMfmaRbf], nmfmabf);
}

// ---------------------------------------------------------------------------------------------
// One work item of the Y contraction of a GEMM-L column block [c0, c1), by one wave:
//   wi < NW (term 1, alpha part wi):  H1[a][b] += sum_{al in part, c} P[(al,a)][c] Y_G(c)[al][b][g(c)]
//   wi >= NW (term 2, G = jj0 + (wi - NW) / kY2Parts, alpha part (wi - NW) % kY2Parts):
//            Sigma(A,G)[a][g] -= sum_{al in part, c} P[(al,a)][c] Y_G[al][b(c)][g]
// (term 2 is split over alpha like term 1, so that the eight waves share the work evenly)
// The operands of up to eight K steps are loaded before their MFMAs; kept out of line so that
// its registers do not count against the block products.  Returns the MFMAs issued.
constexpr int kY2Parts = 4;
__device__ __noinline__ unsigned long long ycontract_wave(ItemLds &L, const smem<const short> *col2jj,
                                                          const gmem<const double> *Pb,
                                                          const gmem<const double> *slot, gmem<double> *Sbuf, int wi,
                                                          int c0, int c1, int jj0, unsigned long long t2m,
                                                          bool t1any) {
  const int lane = threadIdx.x & 63, kk = lane >> 4, l16 = lane & 15;
  const int PA = L.PA, na = L.na, nb = L.nb;
  unsigned long long nm = 0;
  if (t1any && wi < NW) {
    const int al0 = wi * PA / NW, al1 = (wi + 1) * PA / NW, nc = c1 - c0;
    for (int a0 = 0; a0 < na; a0 += 16)
      for (int b0 = 0; b0 < nb; b0 += 16) {
        d4 h = {0, 0, 0, 0};
        for (int al = al0; al < al1; ++al)
          for (int cg = 0; cg < nc; cg += 32) {
            double av[8], bv[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
              const int cl = cg + 4 * s + kk;
              double x = 0.0, y = 0.0;
              if (cl < nc) {
                const int c = c0 + cl, jj = col2jj[c], j = L.a_j[jj];
                const int cc = c - L.a_col0[jj], ng = L.g_n[j];
                if (cc < ng) {
                  if (a0 + l16 < na) x = Pb[(long long)(al * na + a0 + l16) * BN + cl];
                  if (b0 + l16 < nb) y = slot[L.a_y[jj] + ((long long)al * nb + b0 + l16) * ng + cc];
                }
              }
              av[s] = x;
              bv[s] = y;
            }
#pragma unroll
            for (int s = 0; s < 8; ++s)
              if (cg + 4 * s < nc) {
                h = mfma64(av[s], bv[s], h);
                ++nm;
              }
          }
        for (int e = 0; e < 4; ++e) {
          const int a = a0 + kk + 4 * e, b = b0 + l16;
          if (a < na && b < nb && h[e] != 0.0) atomicAdd(&L.H1[a * MAXN + b], h[e]);
        }
      }
    return nm;
  }
  const int q = (wi - (t1any ? NW : 0)) / kY2Parts, part = (wi - (t1any ? NW : 0)) % kY2Parts;
  if (!((t2m >> q) & 1ull)) return 0;
  const int al0 = part * PA / kY2Parts, al1 = (part + 1) * PA / kY2Parts;
  const int jj = jj0 + q, j = L.a_j[jj], ng = L.g_n[j];
  const int gb = L.a_col0[jj] + ng, g1 = L.a_col0[jj + 1];
  const int bc0 = max(c0, gb), bc1 = min(c1, g1);
  const gmem<const double> *Yj = slot + L.a_y[jj];
  gmem<double> *S = Sbuf + L.g_dAGoff[j];
  for (int a0 = 0; a0 < na; a0 += 16)
    for (int g0 = 0; g0 < ng; g0 += 16) {
      d4 h = {0, 0, 0, 0};
      for (int al = al0; al < al1; ++al) {
        double av[8], bv[8];  // the b columns of this G in the block: at most 32
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int c = bc0 + 4 * s + kk;
          const bool ok = c < bc1;
          av[s] = (ok && a0 + l16 < na) ? Pb[(long long)(al * na + a0 + l16) * BN + (c - c0)] : 0.0;
          bv[s] = (ok && g0 + l16 < ng) ? Yj[((long long)al * nb + (c - gb)) * ng + g0 + l16] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 8; ++s)
          if (bc0 + 4 * s < bc1) {
            h = mfma64(av[s], bv[s], h);
            ++nm;
          }
      }
      for (int e = 0; e < 4; ++e) {
        const int a = a0 + kk + 4 * e, g = g0 + l16;
        if (a < na && g < ng && h[e] != 0.0) gatomic_add(S + a * ng + g, -h[e]);
      }
    }
  return nm;
}

// ---------------------------------------------------------------------------------------------
// GEMM-L's last row block when it holds a single row tile (rows r0..M-1, at most 16): instead of a
// 128-row block product in which one wave of eight works, the eight waves split K, each forms the
// 16x64 product of its K range straight from global memory (four K steps per pipeline step), and
// the partials are summed through LDS (red: [NW][16][64] doubles, the free stage buffers) into P.
// FP64 in every precision form.  Kept out of line (its registers would otherwise count against the
// block products).  Returns the MFMAs issued.
__device__ __noinline__ unsigned long long ksplit_last_block(const gmem<const double> *CT,
                                                             const smem<const long long> *kaddr,
                                                             const gmem<double> *panel, gmem<double> *Pb,
                                                             smem<double> *red, int M, int Kc, int kc, int r0,
                                                             unsigned colact) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kk = lane >> 4, l16 = lane & 15;
  const int nks = Kc >> 2;
  const int s0 = wave * nks / NW, s1 = (wave + 1) * nks / NW;
  const int row = min(r0 + l16, M - 1);  // rows past M: loaded in bounds, their results dropped
  d4 acc[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = d4{0, 0, 0, 0};
  struct KB {
    double a[4], b[4][4];
  };
  pipelined<KB>(
      (s1 - s0 + 3) >> 2,
      [&](int t, KB &bb) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = 4 * min(s0 + 4 * t + u, s1 - 1) + kk;
          bb.a[u] = CT[max(kaddr[k], 0ll) + row];
#pragma unroll
          for (int v = 0; v < 4; ++v) bb.b[u][v] = panel[(long long)k * BN + v * 16 + l16];
        }
      },
      [&](int t, const KB &bb) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int st = s0 + 4 * t + u;
          if (st >= s1) break;
          const double a = keep_if(bb.a[u], 4 * st + kk < kc);
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (colact & (1u << v)) acc[v] = mfma64(a, bb.b[u][v], acc[v]);
        }
      });
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) red[(wave * 16 + kk + 4 * e) * BN + v * 16 + l16] = acc[v][e];
  __syncthreads();
  for (int q = tid; q < 16 * BN; q += NT) {
    const int rl = q / BN, c = q - rl * BN;
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += red[(w * 16 + rl) * BN + c];
    if (r0 + rl < M) Pb[(long long)(r0 + rl) * BN + c] = ((colact >> (c >> 4)) & 1u) ? sum : 0.0;
  }
  return (unsigned long long)__builtin_popcount(colact) * (s1 - s0);
}
static_assert(NW * 16 * BN <= 2 * BK * BM + 2 * BK * BNR, "K-split partials fit the stage buffers");

// ---------------------------------------------------------------------------------------------
// GEMM-L: terms 1 and 2.  Rows (alpha,a), K = (F,f), columns (G, [g | b]).
//   P[(al,a)][(G,g)] = sum_{F,f} C_AF[al][a][f] w D_FG[f][g]   (term 1, kept units only)
//   P[(al,a)][(G,b)] = sum_{F,f} C_AF[al][a][f] w D_FB[f][b]   (term 2, kept units only)
//   H1[a][b]  += sum_{al,G,g} P[(al,a)][(G,g)] Y_G[al][b][g]      -> Sigma(A,B)
//   H2_G[a][g] = sum_{al,b}  P[(al,a)][(G,b)] Y_G[al][b][g]      -> Sigma(A,G)
// Per 64-column block: the masked D panel over the F's with a kept unit in the block is staged
// once in the workgroup's scratch, P (all rows x 64) is formed by 128 x 64 block products with
// C read from the per-block transposed copy, then contracted with Y on the matrix cores.
template <int PR>
__device__ void phase_gemm_l(const DevPlan &P, ItemLds &L, const gmem<double> *slot, const gmem<long long> *doff,
                             const gmem<uint8_t> *mask, uint8_t *row2i, const short *col2jj, double *As, double *Bs,
                             gmem<double> *wg, int rows_cap, long long *kaddr /* LDS [rows_cap] */,
                             const gmem<float> *ub, int tier, float tau) {
  const gmem<const double> *Dbuf = gptr(P.Dbuf);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kk = lane >> 4, l16 = lane & 15;
  const int M = L.PA * L.na, nb = L.nb, nF = L.nF;
  const int ncb = (L.NR + BN - 1) / BN, nrb = (M + BM - 1) / BM;
  gmem<double> *panel = wg;                             // [rows_cap][64]
  gmem<double> *Pb = panel + (long long)rows_cap * BN;  // [M][64]
  const gmem<const double> *CT = gptr(P.CTbuf);
  const gmem<const float> *CT32 = gptr(P.CT32);
  unsigned long long nmfma = 0, nmfma32 = 0;
  for (int cb = 0; cb < ncb; ++cb) {
    const int c0 = cb * BN, c1 = min(c0 + BN, L.NR);
    const int jj0 = col2jj[c0], jj1 = col2jj[c1 - 1];
    // F set of the block, targets with work, active column tiles
    if (tid == 0) {
      L.blk_act = 0;
      L.blk_ub = 0u;
      L.t1any = 0;
      L.t2any = 0ull;
    }
    __syncthreads();
    if (tid < nF) {
      const int i = tid;
      bool hit = false;
      unsigned long long t2 = 0;
      bool t1 = false;
      for (int jj = jj0; jj <= jj1; ++jj) {
        const int j = L.a_j[jj];
        const int g0 = L.a_col0[jj], gb = g0 + L.g_n[j], g1 = L.a_col0[jj + 1];
        const uint8_t bits = mask[i * L.nG + j];
        if ((bits & kT1) && max(c0, g0) < min(c1, gb)) t1 = true;
        if ((bits & kT2) && max(c0, gb) < min(c1, g1)) t2 |= 1ull << (jj - jj0);
      }
      hit = t1 || t2;
      L.fpos[i] = hit ? 1 : 0;
      if (t1) L.t1any = 1;
      if (t2) atomicOr(&L.t2any, t2);
      if (hit) {
        for (int ct = 0; ct < 4; ++ct) {
          const int cl = c0 + ct * 16;
          if (tile_has(L, mask, col2jj, i, cl, min(cl + 16, c1), kT1, kT2)) atomicOr(&L.blk_act, 1ull << ct);
        }
        if (tier == 1 || tier == 3) atomicMax(&L.blk_ub, __float_as_uint(cols_ub(L, ub, col2jj, i, c0, c1, 0)));
      }
    }
    __syncthreads();
    if (!L.blk_act) continue;
    const bool fp32 = PR >= 1 && (tier == 2 || ((tier == 1 || tier == 3) && __uint_as_float(L.blk_ub) <= tau));
    if (tid == 0) {
      int kc = 0, m = 0;
      for (int i = 0; i < nF; ++i)
        if (L.fpos[i]) {
          L.fsel[m] = (short)i;
          L.fsrow[m] = kc;
          ++m;
          kc += L.f_n[i];
        }
      L.fsrow[m] = kc;
      L.nsel = m;
      L.kc = kc;
    }
    __syncthreads();
    const int kc = L.kc, Kc = (kc + BK - 1) / BK * BK, nsel = L.nsel, nj = jj1 - jj0 + 1;
    // panel row -> member table (row2i is free once GEMM-R is done), and per (member, G of the
    // block) the offsets of the two operand blocks, D_FG (term 1) and D_FB (term 2), -1 where the
    // unit is not kept: in the A stage, free here, when they fit
    long long *uoff = reinterpret_cast<long long *>(As);
    const bool tab = nsel * nj * 2 <= 2 * BK * BM;
    for (int m = tid >> 6; m < nsel; m += NW)
      for (int f = lane; f < L.f_n[L.fsel[m]]; f += 64) row2i[L.fsrow[m] + f] = (uint8_t)m;
    if (tab)
      for (int q = tid; q < nsel * nj; q += NT) {
        const int m = q / nj, i = L.fsel[m], j = L.a_j[jj0 + q - m * nj];
        const uint8_t bits = mask[i * L.nG + j];
        uoff[2 * q] = (bits & kT1) ? doff[i * L.nG + j] : -1;
        uoff[2 * q + 1] = (bits & kT2) ? L.f_dFBoff[i] : -1;
      }
    __syncthreads();
    // stage the masked D panel and the C^T row addresses
    for (int e = tid; e < Kc * BN; e += NT) {
      const int k = e >> 6, cl = e & (BN - 1), c = c0 + cl;
      double val = 0.0;
      long long ka = -1;
      if (k < kc) {
        const int m = row2i[k], i = L.fsel[m], f = k - L.fsrow[m];
        ka = L.f_coff[i] + (long long)f * M;
        if (c < c1) {
          const int jj = col2jj[c], j = L.a_j[jj];
          const int cc = c - L.a_col0[jj], ng = L.g_n[j];
          long long o;
          if (tab) {
            o = uoff[2 * (m * nj + jj - jj0) + (cc < ng ? 0 : 1)];
          } else {
            const uint8_t bits = mask[i * L.nG + j];
            o = cc < ng ? ((bits & kT1) ? doff[i * L.nG + j] : -1) : ((bits & kT2) ? L.f_dFBoff[i] : -1);
          }
          if (o >= 0) val = unit_weight(L, i, j) * Dbuf[o + (cc < ng ? f * ng + cc : f * nb + (cc - ng))];
        }
      }
      panel[(long long)k * BN + cl] = val;
      if (cl == 0) kaddr[k] = ka;
    }
    __threadfence_block();
    __syncthreads();
    const unsigned colact = (unsigned)(L.blk_act & 15ull);
    for (int rb = 0; rb < nrb; ++rb) {
      if (M - rb * BM <= 16) {
        // a last row block of one row tile: the eight waves split K instead (see ksplit_last_block)
        nmfma += ksplit_last_block(CT, (const smem<const long long> *)kaddr, panel, Pb, (smem<double> *)As, M, Kc, kc,
                                   rb * BM, colact);
        continue;
      }
      const int r = rb * BM + (tid & (BM - 1));
      const bool rok = r < M;
      const int rc = rok ? r : 0;  // an in-bounds row for the loads of rows past M
      const int bcl = tid & (BN - 1);
      d4 acc[4];
      const unsigned act = (rb * BM + wave * 16 < M) ? colact : 0u;
      if (fp32) {
        f4 a32[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) a32[v] = f4{0, 0, 0, 0};
        wg_block_mm32<BN>(
            Kc, [&](int k) { return CT32[max(kaddr[k], 0ll) + rc]; }, [&](int k) { return panel[(long long)k * BN + bcl]; },
            rok, kc, true, act, reinterpret_cast<float *>(As),
            reinterpret_cast<float *>(Bs), a32);
        nmfma32 += (unsigned long long)(act ? 4 : 0) * (Kc >> 2);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[v][e] = (double)a32[v][e];
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = d4{0, 0, 0, 0};
        wg_block_mm<BN, (PR < 2)>(
            Kc, [&](int k) { return CT[max(kaddr[k], 0ll) + rc]; }, [&](int k) { return panel[(long long)k * BN + bcl]; },
            rok, kc, true, act, As, Bs, acc);
        nmfma += (unsigned long long)(PR < 2 ? __builtin_popcount(act) : (act ? 4 : 0)) * (Kc >> 2);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = rb * BM + wave * 16 + (fp32 ? 4 * kk + e : kk + 4 * e);  // MFMA result row
          if (row < M) Pb[(long long)row * BN + v * 16 + l16] = (act & (1u << v)) ? acc[v][e] : 0.0;
        }
    }
    __threadfence_block();
    __syncthreads();
    // contractions with Y: work items (target, alpha part); target 0 = term 1, 1+q = term 2 of jj0+q
    {
      const int nwork = (L.t1any ? NW : 0) + (jj1 - jj0 + 1) * kY2Parts;
      for (int wi = wave; wi < nwork; wi += NW)
        nmfma += ycontract_wave(L, (const smem<const short> *)col2jj, Pb, slot, gptr(P.Sbuf), wi, c0, c1, jj0, L.t2any,
                                L.t1any != 0);
    }
    __syncthreads();
  }
  if (lane == 0 && nmfma) atomicAdd(&L.cnt[kCntMfmaL], nmfma);
  if (lane == 0 && nmfma32) atomicAdd(&L.cnt[kCntMfmaL32], nmfma32);
}

// ---------------------------------------------------------------------------------------------
template <int W, int PR>
__global__ __launch_bounds__(NT) void k_main(DevPlan P, KParams kp) {
  __shared__ ItemLds L;
  extern __shared__ double dyn[];
  uint8_t *row2i = reinterpret_cast<uint8_t *>(dyn);
  short *col2jj = reinterpret_cast<short *>(reinterpret_cast<uint8_t *>(dyn) + kp.rows_cap);
  double *As = reinterpret_cast<double *>(reinterpret_cast<uint8_t *>(dyn) + kp.rows_cap + 2 * kp.cols_cap);
  double *Bs = As + 2 * BK * BM;
  double *acc3 = Bs + 2 * BK * BNR;  // [NW][16][ld3]
  long long *kaddr = reinterpret_cast<long long *>(acc3 + NW * 16 * kp.ld3);  // [rows_cap]
  const int dyn_doubles = 2 * BK * BM + 2 * BK * BNR + NW * 16 * kp.ld3;
  __shared__ int s_item;
  const int tid = threadIdx.x;
  gmem<double> *slot = gptr(P.scratch) + (long long)blockIdx.x * P.slot_doubles;
  for (;;) {
    if (tid == 0) {
      // the next item of this workgroup's group (workgroup b runs on XCD b mod 8), else of the
      // next group that still has items: each group's segment of the schedule is drained through
      // its own ticket; with one group this is the single global ticket
      int found = P.n_items;
      const int g0 = (int)(blockIdx.x % (unsigned)P.n_groups);
      for (int q = 0; q < P.n_groups; ++q) {
        const int g = g0 + q < P.n_groups ? g0 + q : g0 + q - P.n_groups;
        const int n = P.grp_start[g + 1] - P.grp_start[g];
        if (n <= 0 || __atomic_load_n(&P.ticket[g], __ATOMIC_RELAXED) >= (unsigned)n) continue;
        const unsigned t = atomicAdd(&P.ticket[g], 1u);
        if (t < (unsigned)n) {
          found = P.grp_start[g] + (int)t;
          break;
        }
      }
      s_item = found;
    }
    __syncthreads();
    const int sidx = s_item;
    if (sidx >= P.n_items) break;
    const int item = P.order[sidx];
    const long long t_start = wall_clock64();
    const Item it = P.items[item];
    if (tid < kCntN) L.cnt[tid] = 0;
    if (tid < 2) L.flops[tid] = 0.0;
    if (tid == 0) {
      L.contrib = 0.0;
      L.A = it.A;
      L.B = it.B;
      L.rb = it.rb;
      L.PA = P.nabf[it.A];
      L.PB = P.nabf[it.B];
      L.na = P.nao[it.A];
      L.nb = P.nao[it.B];
      L.cA = P.c_start[it.A];
      L.cB = P.c_start[it.B];
      L.nF = P.c_start[it.A + 1] - L.cA;
      L.nG = P.c_start[it.B + 1] - L.cB;
      L.gV = P.gV[it.vid];
      L.voff = P.v_off[it.vid];
      const int cell = P.cell_of[it.A];
      L.tbase = P.ptab_off[cell];
      L.tn = P.cell_natoms[cell];
      L.gDmax = P.gDmax[cell];
      L.dAB = lookup_d(P, it.A, it.B, it.rb);
      L.okAB = L.dAB >= 0 && P.keepD[L.dAB];
    }
    __syncthreads();
    // F and G lists
    for (int i = tid; i < L.nF; i += NT) {
      const int cf = L.cA + i;
      const int F = P.c_col[cf];
      const int RF = P.c_R[cf];
      L.f_atom[i] = F;
      L.f_R[i] = RF;
      L.f_n[i] = P.nao[F];
      L.f_coff[i] = P.c_off[cf];
      const CNorm cn = P.c_norm[cf];
      L.f_gA[i] = cn.gA;
      L.f_gF[i] = cn.gF;
      L.f_nA[i] = cn.nA;
      L.f_nF[i] = cn.nF;
      L.f_Q[i] = cn.Q;
      L.f_on[i] = (F == L.A && r_zero(RF));
      L.f_loc[i] = (short)P.local_of[F];
      const int d = lookup_d(P, F, L.B, r_sub(L.rb, RF));
      L.f_dFB[i] = d;
      L.f_dFBoff[i] = d >= 0 ? P.d_off[d] : 0;
    }
    for (int j = tid; j < L.nG; j += NT) {
      const int cg = L.cB + j;
      const int G = P.c_col[cg];
      const int RG = r_add(L.rb, P.c_R[cg]);
      L.g_atom[j] = G;
      L.g_R[j] = RG;
      L.g_n[j] = P.nao[G];
      L.g_coff[j] = P.c_off[cg];
      const CNorm cn = P.c_norm[cg];
      L.g_gA[j] = cn.gA;
      L.g_gF[j] = cn.gF;
      L.g_Q[j] = cn.Q;
      L.g_on[j] = (G == L.B && r_zero(P.c_R[cg]));
      L.g_loc[j] = (short)P.local_of[G];
      const int d = lookup_d(P, L.A, G, RG);
      L.g_dAG[j] = d;
      L.g_dAGoff[j] = d >= 0 ? P.d_off[d] : 0;
      L.g_alive[j] = 0;
    }
    for (int q = tid; q < MAXN * MAXN; q += NT) L.H1[q] = 0.0;
    if (L.okAB)
      for (int q = tid; q < L.na * L.nb; q += NT) L.DAB[q] = P.Dbuf[P.d_off[L.dAB] + q];
    __syncthreads();
    if (tid == 0) {
      int r0 = 0;
      for (int i = 0; i < L.nF; ++i) {
        L.f_row0[i] = r0;
        r0 += L.f_n[i];
      }
      L.f_row0[L.nF] = r0;
      L.MR = r0;
    }
    // slot scratch: dfg (int), mask (bytes) and doff (D / Sigma offset of D_FG) over nF*nG, then E2,
    // then per-G buffers
    gmem<int> *dfg = reinterpret_cast<gmem<int> *>(slot);
    const int nFG = L.nF * L.nG;
    gmem<uint8_t> *mask = reinterpret_cast<gmem<uint8_t> *>(slot + ((nFG + 1) >> 1));
    gmem<long long> *doff = reinterpret_cast<gmem<long long> *>(slot + ((nFG + 1) >> 1) + ((nFG + 7) >> 3));
    gmem<double> *E2 = slot + ((nFG + 1) >> 1) + ((nFG + 7) >> 3) + nFG;
    gmem<double> *gbase_d = E2 + L.nF * L.nb * L.nb;
    __syncthreads();
    long long tp = wall_clock64();
    auto tick = [&](int ph) {
      if (tid == 0) {
        const long long t = wall_clock64();
        L.cnt[kCntPhase + ph] += (unsigned long long)(t - tp);
        tp = t;
      }
    };
    tick(5);
    phase_screen(P, L, dfg, doff, mask);
    __syncthreads();
    tick(0);
    // compact alive G and lay out their buffers
    if (tid == 0) {
      int n = 0, col = 0;
      long long off = gbase_d - slot;
      for (int j = 0; j < L.nG; ++j) {
        if (!L.g_alive[j]) continue;
        const int ng = L.g_n[j];
        L.a_j[n] = (short)j;
        L.a_col0[n] = col;
        col += ng + L.nb;
        const int ysz = L.PA * L.nb * ng;
        L.a_y[n] = (int)off;
        off += ysz;
        L.a_t4[n] = (int)off;
        off += L.PA * L.na * ng;
        L.a_t3[n] = (int)off;
        off += L.PA * L.na * L.nb;
        L.a_n1[n] = (int)off;
        off += L.nb * ng * ng;
        L.a_m2[n] = (int)off;
        off += ng * L.nb * L.nb;
        ++n;
      }
      L.nGa = n;
      L.a_col0[n] = col;
      L.NR = col;
      L.cnt[kCntCandidates] = (unsigned long long)L.nF * L.nG;
      L.cnt[kCntG] = n;
      L.scratch_top = (int)off;
    }
    __syncthreads();
    {
      // V_AB in LDS when it fits in the accumulator region (not in use in this phase)
      const bool vlds = L.PA * L.PB <= dyn_doubles;
      const gmem<const double> *Vg = gptr(P.Vbuf) + L.voff;
      if (vlds)
        for (int q = tid; q < L.PA * L.PB; q += NT) As[q] = Vg[q];
      __syncthreads();
      for (int jj = tid >> 6; jj < L.nGa; jj += NW) {
        if (vlds)
          gside_wave<true>(P, L, slot, jj, (const smem<const double> *)As, Vg);
        else
          gside_wave<false>(P, L, slot, jj, (const smem<const double> *)As, Vg);
      }
      __syncthreads();
    }
    tick(1);
    gmem<float> *ub = (kp.tier == 1 || kp.tier == 3) ? reinterpret_cast<gmem<float> *>(slot + kp.ub_off) : nullptr;
    if constexpr (PR == 1)
      phase_masks_ool(P, L, slot, dfg, doff, mask, E2, slot + kp.wave_off + (tid >> 6) * kp.wave_doubles, ub);
    else
      phase_masks(P, L, slot, dfg, doff, mask, E2, slot + kp.wave_off + (tid >> 6) * kp.wave_doubles, ub);
    // decode tables
    for (int r = tid; r < L.MR; r += NT) {
      int lo = 0, hi = L.nF - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.f_row0[mid] <= r)
          lo = mid;
        else
          hi = mid - 1;
      }
      row2i[r] = (uint8_t)lo;
    }
    for (int c = tid; c < L.NR; c += NT) {
      int lo = 0, hi = L.nGa - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.a_col0[mid] <= c)
          lo = mid;
        else
          hi = mid - 1;
      }
      col2jj[c] = (short)lo;
    }
    // FLOP accounting of the item (both counts exclude padding and screened-out work):
    //   paper: Algorithm 3 per kept unit -- T_t and Htilde_t for terms 1, 2; Htilde_t for terms
    //          3, 4 (T3, T4 once per G) -- plus Y, T3, T4 once per alive G
    //   alg:   this kernel -- one C.D or C^T.T product per kept unit, plus Y, T3, T4, the two
    //          Gram matrices and the two Y contractions once per alive G
    {
      double fp = 0.0, fa = 0.0;
      const double PA = L.PA, na = L.na, nb = L.nb;
      for (int p = tid; p < L.nF * L.nGa; p += NT) {
        const int i = p / L.nGa, jj = p - i * L.nGa;
        const int j = L.a_j[jj];
        const uint8_t bits = mask[i * L.nG + j];
        const double nf = L.f_n[i], ng = L.g_n[j];
        if (bits & kT1) { fp += 2 * PA * nf * nb * ng + 2 * na * PA * nf * nb; fa += 2 * PA * na * nf * ng; }
        if (bits & kT2) { fp += 2 * PA * nf * ng * nb + 2 * na * PA * nf * ng; fa += 2 * PA * na * nf * nb; }
        if (bits & kT3) { fp += 2 * nf * PA * na * nb; fa += 2 * nf * PA * na * nb; }
        if (bits & kT4) { fp += 2 * nf * PA * na * ng; fa += 2 * nf * PA * na * ng; }
      }
      for (int jj = tid; jj < L.nGa; jj += NT) {
        const double ng = L.g_n[L.a_j[jj]];
        const double g = 2 * PA * L.PB * nb * ng + 2 * 2 * PA * na * nb * ng;
        fp += g;
        fa += g + 2 * PA * (nb * ng * ng + ng * nb * nb) + 2 * 2 * PA * na * nb * ng;
      }
      if (fp != 0.0) atomicAdd(&L.flops[0], fp);
      if (fa != 0.0) atomicAdd(&L.flops[1], fa);
    }
    __syncthreads();
    tick(2);
    if (L.nGa > 0) {
      phase_gemm_r<W, PR>(P, L, slot, doff, mask, row2i, col2jj, As, Bs, acc3 + (tid >> 6) * 16 * kp.ld3, kp.ld3, ub,
                   kp.tier, kp.tau, kp.tau_bf);
      __syncthreads();
      tick(3);
      phase_gemm_l<PR>(P, L, slot, doff, mask, row2i, col2jj, As, Bs, slot + kp.wg_off, kp.rows_cap, kaddr, ub, kp.tier,
                   kp.tau);
    }
    __syncthreads();
    tick(4);
    // flush term 1: Sigma(A,B)
    if (L.dAB >= 0)
      for (int q = tid; q < L.na * L.nb; q += NT) {
        const int a = q / L.nb, b = q - a * L.nb;
        const double v = L.H1[a * MAXN + b];
        if (v != 0.0) gatomic_add(gptr(P.Sbuf) + P.d_off[L.dAB] + q, -v);
      }
    if (tid < kCntN && L.cnt[tid]) atomicAdd(&P.counters[tid], L.cnt[tid]);
    if (tid < 2 && L.flops[tid] != 0.0) atomicAdd(&P.flops[tid], L.flops[tid]);
    if (tid < 4) P.item_units[item * kItemUnits + tid] = (int)L.cnt[kCntKept + 8 + tid];
    if (tid == 4) P.item_units[item * kItemUnits + 4] = L.nGa;
    if (tid == 0) {
      P.item_cycles[item] = wall_clock64() - t_start;
      P.item_contrib[item] = L.contrib;
      P.item_flops[item] = L.flops[1];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// plan-time: C block norms (Sec. III C 1) -- one workgroup per kept C block
__global__ __launch_bounds__(256) void k_cnorm(const double *__restrict__ Cbuf, const long long *__restrict__ c_off,
                                               const int *__restrict__ c_row, const int *__restrict__ c_col,
                                               const int *__restrict__ nao, const int *__restrict__ nabf, int nC,
                                               CNorm *__restrict__ out) {
  const int cb = blockIdx.x;
  if (cb >= nC) return;
  const int A = c_row[cb], F = c_col[cb];
  const int P = nabf[A], na = nao[A], nf = nao[F];
  const double *C = Cbuf + c_off[cb];
  __shared__ double s_n[2][MAXN], s_g[2][MAXN];
  const int tid = threadIdx.x;
  if (tid < MAXN) {
    s_n[0][tid] = s_n[1][tid] = 0;
    s_g[0][tid] = s_g[1][tid] = 0;
  }
  __syncthreads();
  // ||C[:,a,:]||^2 and ||C[:,:,f]||^2
  for (int q = tid; q < na * nf; q += 256) {
    const int a = q / nf, f = q % nf;
    double s = 0;
    for (int al = 0; al < P; ++al) {
      const double v = C[(al * na + a) * nf + f];
      s += v * v;
    }
    atomicAdd(&s_n[0][a], s);
    atomicAdd(&s_n[1][f], s);
  }
  // Gram (fixed a): G[f][f'] = sum_al C[al][a][f] C[al][a][f'];  sum of squares over (f,f')
  for (int q = tid; q < na * nf * nf; q += 256) {
    const int a = q / (nf * nf), f = (q / nf) % nf, f2 = q % nf;
    double s = 0;
    for (int al = 0; al < P; ++al) s += C[(al * na + a) * nf + f] * C[(al * na + a) * nf + f2];
    atomicAdd(&s_g[0][a], s * s);
  }
  // Gram (fixed f): G[a][a'] = sum_al C[al][a][f] C[al][a'][f]
  for (int q = tid; q < nf * na * na; q += 256) {
    const int f = q / (na * na), a = (q / na) % na, a2 = q % na;
    double s = 0;
    for (int al = 0; al < P; ++al) s += C[(al * na + a) * nf + f] * C[(al * na + a2) * nf + f];
    atomicAdd(&s_g[1][f], s * s);
  }
  __syncthreads();
  if (tid == 0) {
    double nA = 0, gA = 0, nF = 0, gF = 0;
    for (int a = 0; a < na; ++a) {
      nA = fmax(nA, s_n[0][a]);
      gA = fmax(gA, s_g[0][a]);
    }
    for (int f = 0; f < nf; ++f) {
      nF = fmax(nF, s_n[1][f]);
      gF = fmax(gF, s_g[1][f]);
    }
    out[cb].nA = sqrt(nA);
    out[cb].gA = sqrt(sqrt(gA));
    out[cb].nF = sqrt(nF);
    out[cb].gF = sqrt(sqrt(gF));
  }
}

// plan-time: CS-ERI factor Q_AF = sqrt(max_{a,f} (Aa Ff|Aa Ff)) under set semantics
// (eq. CS-ERI); qsrc[5*cb..]: kept indices of C(F,A,-R), V(A,A), V(A,F), V(F,A), V(F,F) or -1
__global__ __launch_bounds__(256) void k_cq(const double *__restrict__ Cbuf, const long long *__restrict__ c_off,
                                            const int *__restrict__ c_row, const int *__restrict__ c_col,
                                            const double *__restrict__ Vbuf, const long long *__restrict__ v_off,
                                            const int *__restrict__ qsrc, const int *__restrict__ nao,
                                            const int *__restrict__ nabf, int nC, CNorm *__restrict__ out) {
  const int cb = blockIdx.x;
  if (cb >= nC) return;
  const int A = c_row[cb], F = c_col[cb];
  const int PA = nabf[A], PF = nabf[F], na = nao[A], nf = nao[F];
  const int *src = qsrc + 5 * cb;
  const double *cAF = Cbuf + c_off[cb];
  const double *cFA = src[0] >= 0 ? Cbuf + c_off[src[0]] : nullptr;
  const double *vAA = src[1] >= 0 ? Vbuf + v_off[src[1]] : nullptr;
  const double *vAF = src[2] >= 0 ? Vbuf + v_off[src[2]] : nullptr;
  const double *vFA = src[3] >= 0 ? Vbuf + v_off[src[3]] : nullptr;
  const double *vFF = src[4] >= 0 ? Vbuf + v_off[src[4]] : nullptr;
  const bool onsite = src[0] == -2;  // marks F == A in the home cell
  __shared__ double s_best[256];
  double best = 0.0;
  for (int q = threadIdx.x; q < na * nf; q += 256) {
    const int a = q / nf, f = q % nf;
    double val = 0.0;
    if (vAA)
      for (int al = 0; al < PA; ++al) {
        const double ua = cAF[(al * na + a) * nf + f];
        double s = 0;
        for (int be = 0; be < PA; ++be) s += vAA[al * PA + be] * cAF[(be * na + a) * nf + f];
        val += ua * s;
      }
    if (!onsite && cFA) {
      if (vAF)
        for (int al = 0; al < PA; ++al) {
          const double ua = cAF[(al * na + a) * nf + f];
          double s = 0;
          for (int be = 0; be < PF; ++be) s += vAF[al * PF + be] * cFA[(be * nf + f) * na + a];
          val += ua * s;
        }
      if (vFA)
        for (int al = 0; al < PF; ++al) {
          const double uf = cFA[(al * nf + f) * na + a];
          double s = 0;
          for (int be = 0; be < PA; ++be) s += vFA[al * PA + be] * cAF[(be * na + a) * nf + f];
          val += uf * s;
        }
      if (vFF)
        for (int al = 0; al < PF; ++al) {
          const double uf = cFA[(al * nf + f) * na + a];
          double s = 0;
          for (int be = 0; be < PF; ++be) s += vFF[al * PF + be] * cFA[(be * nf + f) * na + a];
          val += uf * s;
        }
    }
    best = fmax(best, val);
  }
  s_best[threadIdx.x] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0;
    for (int t = 0; t < 256; ++t) b = fmax(b, s_best[t]);
    out[cb].Q = sqrt(b);
  }
}

// plan-time: gV = sqrt(||V V^T||_F) per kept V block
__global__ __launch_bounds__(256) void k_vnorm(const double *__restrict__ Vbuf, const long long *__restrict__ v_off,
                                               const int *__restrict__ v_row, const int *__restrict__ v_col,
                                               const int *__restrict__ nabf, int nV, double *__restrict__ gV) {
  const int vb = blockIdx.x;
  if (vb >= nV) return;
  const int PA = nabf[v_row[vb]], PB = nabf[v_col[vb]];
  const double *V = Vbuf + v_off[vb];
  __shared__ double s_acc[256];
  double acc = 0;
  for (int q = threadIdx.x; q < PA * PA; q += 256) {
    const int x = q / PA, y = q % PA;
    double s = 0;
    for (int k = 0; k < PB; ++k) s += V[x * PB + k] * V[y * PB + k];
    acc += s * s;
  }
  s_acc[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s_acc[threadIdx.x] += s_acc[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) gV[vb] = sqrt(sqrt(s_acc[0]));
}

// plan-time: per-block transposed copy of C, CT[f][(alpha,a)] = C[(alpha,a)][f]
__global__ __launch_bounds__(256) void k_ctrans(const double *__restrict__ Cbuf, const long long *__restrict__ c_off,
                                                const int *__restrict__ c_row, const int *__restrict__ c_col,
                                                const int *__restrict__ nao, const int *__restrict__ nabf, int nC,
                                                double *__restrict__ CT) {
  const int cb = blockIdx.x;
  if (cb >= nC) return;
  const int A = c_row[cb], F = c_col[cb];
  const int M = nabf[A] * nao[A], nf = nao[F];
  const double *C = Cbuf + c_off[cb];
  double *T = CT + c_off[cb];
  for (int q = threadIdx.x; q < M * nf; q += 256) {
    const int f = q / M, r = q - f * M;
    T[q] = C[r * nf + f];
  }
}

// plan-time: FP32 copy of an FP64 buffer (operands of the FP32 block products)
__global__ void k_to_f32(const double *__restrict__ src, float *__restrict__ dst, long long n) {
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
    dst[q] = (float)src[q];
}

// per build: gather D blocks from the caller layout into the compact layout
__global__ void k_dgather(const double *__restrict__ src, const long long *__restrict__ src_off,
                          const long long *__restrict__ dst_off, int nD, long long base, double *__restrict__ dst) {
  const int b = blockIdx.x;
  if (b >= nD) return;
  const long long n = dst_off[base + b + 1] - dst_off[base + b];
  const double *s = src + src_off[b];
  double *d = dst + dst_off[base + b];
  for (long long q = threadIdx.x; q < n; q += blockDim.x) d[q] = s[q];
}

// per build: D pre-screen (max-abs > eps_D) and gD = sqrt(||D D^T||_F)
__global__ __launch_bounds__(64) void k_dprep(const double *__restrict__ Dbuf, const long long *__restrict__ d_off,
                                              const int *__restrict__ d_row, const int *__restrict__ d_col,
                                              const int *__restrict__ nao, int nD, double eps_D, int pre,
                                              double *__restrict__ gD, uint8_t *__restrict__ keepD) {
  const int b = blockIdx.x * 4 + (threadIdx.x >> 4);
  const int l = threadIdx.x & 15;
  if (b >= nD) return;
  const int nr = nao[d_row[b]], nc = nao[d_col[b]];
  const double *D = Dbuf + d_off[b];
  double mx = 0, acc = 0;
  for (int q = l; q < nr * nr; q += 16) {
    const int x = q / nr, y = q % nr;
    double s = 0;
    for (int k = 0; k < nc; ++k) s += D[x * nc + k] * D[y * nc + k];
    acc += s * s;
  }
  for (int q = l; q < nr * nc; q += 16) mx = fmax(mx, fabs(D[q]));
  for (int o = 8; o > 0; o >>= 1) {
    acc += __shfl_xor(acc, o, 16);
    mx = fmax(mx, __shfl_xor(mx, o, 16));
  }
  if (l == 0) {
    gD[b] = sqrt(sqrt(acc));
    keepD[b] = pre ? (mx > eps_D) : 1;
  }
}

// per build: max over the kept D blocks of each cell of sqrt||D D^T|| (a conservative
// stand-in for gD in a stage-1 prefilter)
__global__ __launch_bounds__(256) void k_dmax(const double *__restrict__ gD, const uint8_t *__restrict__ keepD,
                                              const long long *__restrict__ dbase, double *__restrict__ gDmax) {
  const int c = blockIdx.x;
  __shared__ double sm[256];
  double m = 0;
  for (long long b = dbase[c] + threadIdx.x; b < dbase[c + 1]; b += 256)
    if (keepD[b]) m = fmax(m, gD[b]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) gDmax[c] = sm[0];
}

__global__ void k_zero(double *__restrict__ p, long long n) {
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
    p[q] = 0.0;
}

__global__ void k_reset(unsigned int *ticket, unsigned long long *counters, double *flops) {
  if (threadIdx.x < kMaxGroups) ticket[threadIdx.x] = 0;
  if (threadIdx.x < kCntN) counters[threadIdx.x] = 0;
  if (threadIdx.x < 2) flops[threadIdx.x] = 0.0;
}

// energy: per-workgroup double-double partial sums of <D, Sigma>
__global__ __launch_bounds__(256) void k_energy(const double *__restrict__ D, const double *__restrict__ S,
                                                long long n, double *__restrict__ part) {
  __shared__ double sh[256], sl[256];
  double hi = 0, lo = 0;
  for (long long q = blockIdx.x * 256LL + threadIdx.x; q < n; q += (long long)gridDim.x * 256) {
    const double p = D[q] * S[q];
    const double pe = fma(D[q], S[q], -p);
    const double t = hi + p;
    const double bp = t - hi;
    const double e = (hi - (t - bp)) + (p - bp);
    hi = t;
    lo += e + pe;
  }
  sh[threadIdx.x] = hi;
  sl[threadIdx.x] = lo;
  __syncthreads();
  if (threadIdx.x == 0) {
    double h = 0, c = 0;
    for (int t = 0; t < 256; ++t) {
      const double p = sh[t];
      const double s = h + p;
      const double bp = s - h;
      c += (h - (s - bp)) + (p - bp) + sl[t];
      h = s;
    }
    part[2 * blockIdx.x] = h;
    part[2 * blockIdx.x + 1] = c;
  }
}

// ---------------------------------------------------------------------------------------------
// launch wrappers (host side)
size_t main_dyn_lds(int rows_cap, int cols_cap, int ld3) {
  return (size_t)rows_cap + 2 * (size_t)cols_cap + (size_t)(2 * BK * BM + 2 * BK * BNR + NW * 16 * ld3) * sizeof(double) +
         (size_t)rows_cap * sizeof(long long);
}

hipError_t launch_to_f32(const double *src, float *dst, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t main_set_lds(int rows_cap, int cols_cap, int ld3) {
  const size_t dyn = main_dyn_lds(rows_cap, cols_cap, ld3);
  const void *fns[] = {(const void *)k_main<64, 0>,  (const void *)k_main<32, 0>, (const void *)k_main<128, 0>,
                       (const void *)k_main<64, 1>,  (const void *)k_main<32, 1>, (const void *)k_main<128, 1>,
                       (const void *)k_main<64, 2>,  (const void *)k_main<32, 2>, (const void *)k_main<128, 2>};
  for (const void *f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_main(const DevPlan &P, int n_slots, int rows_cap, int cols_cap, int ld3, long long wave_off,
                       long long wave_doubles, long long wg_off, long long ub_off, int tier, float tau, float tau_bf,
                       int tile_r, hipStream_t s, bool set_lds) {
  KParams kp{rows_cap, cols_cap, ld3, wave_off, wave_doubles, wg_off, ub_off, tier, tau, tau_bf};
  const size_t dyn = main_dyn_lds(rows_cap, cols_cap, ld3);
  if (set_lds) {
    hipError_t e = main_set_lds(rows_cap, cols_cap, ld3);
    if (e != hipSuccess) return e;
  }
  const int pr = tier == 0 ? 0 : tier == 3 ? 2 : 1;
  const dim3 g(n_slots), b(NT);
  if (tile_r == 32) {
    if (pr == 0) hipLaunchKernelGGL((k_main<32, 0>), g, b, dyn, s, P, kp);
    if (pr == 1) hipLaunchKernelGGL((k_main<32, 1>), g, b, dyn, s, P, kp);
    if (pr == 2) hipLaunchKernelGGL((k_main<32, 2>), g, b, dyn, s, P, kp);
  } else if (tile_r == 128) {
    if (pr == 0) hipLaunchKernelGGL((k_main<128, 0>), g, b, dyn, s, P, kp);
    if (pr == 1) hipLaunchKernelGGL((k_main<128, 1>), g, b, dyn, s, P, kp);
    if (pr == 2) hipLaunchKernelGGL((k_main<128, 2>), g, b, dyn, s, P, kp);
  } else {
    if (pr == 0) hipLaunchKernelGGL((k_main<64, 0>), g, b, dyn, s, P, kp);
    if (pr == 1) hipLaunchKernelGGL((k_main<64, 1>), g, b, dyn, s, P, kp);
    if (pr == 2) hipLaunchKernelGGL((k_main<64, 2>), g, b, dyn, s, P, kp);
  }
  return hipGetLastError();
}

size_t main_static_lds() { return sizeof(ItemLds) + sizeof(int); }
int main_threads() { return NT; }
int main_maxnb() { return MAXNB; }
int main_maxn() { return MAXN; }
int main_nwaves() { return NW; }

hipError_t launch_cnorm(const double *Cbuf, const long long *c_off, const int *c_row, const int *c_col,
                        const int *nao, const int *nabf, int nC, CNorm *out, hipStream_t s) {
  if (nC > 0) hipLaunchKernelGGL(k_cnorm, dim3(nC), dim3(256), 0, s, Cbuf, c_off, c_row, c_col, nao, nabf, nC, out);
  return hipGetLastError();
}
hipError_t launch_ctrans(const double *Cbuf, const long long *c_off, const int *c_row, const int *c_col,
                         const int *nao, const int *nabf, int nC, double *CT, hipStream_t s) {
  if (nC > 0) hipLaunchKernelGGL(k_ctrans, dim3(nC), dim3(256), 0, s, Cbuf, c_off, c_row, c_col, nao, nabf, nC, CT);
  return hipGetLastError();
}
hipError_t launch_cq(const double *Cbuf, const long long *c_off, const int *c_row, const int *c_col,
                     const double *Vbuf, const long long *v_off, const int *qsrc, const int *nao, const int *nabf,
                     int nC, CNorm *out, hipStream_t s) {
  if (nC > 0)
    hipLaunchKernelGGL(k_cq, dim3(nC), dim3(256), 0, s, Cbuf, c_off, c_row, c_col, Vbuf, v_off, qsrc, nao, nabf, nC,
                       out);
  return hipGetLastError();
}
hipError_t launch_vnorm(const double *Vbuf, const long long *v_off, const int *v_row, const int *v_col,
                        const int *nabf, int nV, double *gV, hipStream_t s) {
  if (nV > 0) hipLaunchKernelGGL(k_vnorm, dim3(nV), dim3(256), 0, s, Vbuf, v_off, v_row, v_col, nabf, nV, gV);
  return hipGetLastError();
}
hipError_t launch_dgather(const double *src, const long long *src_off, const long long *dst_off, int nD,
                          long long base, double *dst, hipStream_t s) {
  if (nD > 0) hipLaunchKernelGGL(k_dgather, dim3(nD), dim3(64), 0, s, src, src_off, dst_off, nD, base, dst);
  return hipGetLastError();
}
hipError_t launch_dprep(const double *Dbuf, const long long *d_off, const int *d_row, const int *d_col,
                        const int *nao, int nD, double eps_D, int pre, double *gD, uint8_t *keepD, hipStream_t s) {
  if (nD > 0)
    hipLaunchKernelGGL(k_dprep, dim3((nD + 3) / 4), dim3(64), 0, s, Dbuf, d_off, d_row, d_col, nao, nD, eps_D, pre, gD,
                       keepD);
  return hipGetLastError();
}
hipError_t launch_dmax(const double *gD, const uint8_t *keepD, const long long *dbase, double *gDmax, int n_cells,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_dmax, dim3(n_cells), dim3(256), 0, s, gD, keepD, dbase, gDmax);
  return hipGetLastError();
}
hipError_t launch_zero(double *p, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_zero, dim3(2048), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_reset(unsigned int *ticket, unsigned long long *counters, double *flops, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, ticket, counters, flops);
  return hipGetLastError();
}
hipError_t launch_energy(const double *D, const double *S, long long n, double *part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_energy, dim3(nblk), dim3(256), 0, s, D, S, n, part);
  return hipGetLastError();
}

}  // namespace hfx
