// Real-space to k-space sum of the exchange matrix, the step after the build in a band-structure
// calculation (Sec. IV, band-structure calculations, eq. Ham_rs2kspace):
//   H_{Ii,Jj}(k) = sum_R exp(i 2 pi k.R) Sigma_{Ii,Jj}(R),
// k in fractional coordinates of the reciprocal lattice, R the integer lattice vector of the
// column atom, the sum over the blocks of the cell's D pattern (where Sigma lives).
//
// HBM-bound: every Sigma element is read once per batch of kKB k-points and every H element
// is written once.  One workgroup per (kPP consecutive atom pairs I,J, batch of k-points),
// pair after pair (one pair measured fastest: many short workgroups): the phases of a chunk of the pair's R entries go to LDS once, each thread
// then accumulates one block element for all k-points of the batch in registers and writes it
// as one complex number per k.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hfx_fourier.h"
#include "hfx_internal.h"

namespace hfx {

constexpr int kFT = 256;  // threads per workgroup
constexpr int kKB = 8;    // k-points per workgroup
constexpr int kRC = 32;   // R entries per phase chunk
constexpr int kPP = 1;    // atom pairs per workgroup, taken one after the other (8: 10 % slower)

// one atom pair (I, J) for the k-points kb0 .. kb0 + kKB of the chunk
__device__ __forceinline__ void pair_to_k(const double *__restrict__ sigma, const long long *__restrict__ d_off,
                                          long long sbase, const int32_t *__restrict__ pstart,
                                          const int32_t *__restrict__ pcount, const int32_t *__restrict__ dsort_R,
                                          const int32_t *__restrict__ dsort_id, const int32_t *__restrict__ nao,
                                          const int32_t *__restrict__ bofs, int n, long long nbasis,
                                          const KChunk &kc, double2 *__restrict__ H, long long pair, int kb0) {
  const int I = (int)(pair / n), J = (int)(pair - (long long)I * n);
  const int nI = nao[I], nJ = nao[J], ne = nI * nJ;
  const int q0 = pstart[pair], nq = pcount[pair];  // the cell's n x n table
  const int nkb = min(kKB, kc.n - kb0);
  __shared__ double cs[kRC][kKB], sn[kRC][kKB];
  for (int e0 = 0; e0 < ne; e0 += kFT) {
    const int e = e0 + (int)threadIdx.x;
    double re[kKB], im[kKB];
#pragma unroll
    for (int kb = 0; kb < kKB; ++kb) re[kb] = im[kb] = 0.0;
    for (int r0 = 0; r0 < nq; r0 += kRC) {
      const int nr = min(kRC, nq - r0);
      __syncthreads();  // the previous chunk's phases are no longer read
      for (int t = threadIdx.x; t < nr * kKB; t += kFT) {
        const int r = t / kKB, kb = t - r * kKB;
        double c = 0.0, s = 0.0;
        if (kb < nkb) {
          const int32_t R = dsort_R[q0 + r0 + r];
          const double *k = kc.k[kb0 + kb];
          sincospi(2.0 * (k[0] * r_of(R, 0) + k[1] * r_of(R, 1) + k[2] * r_of(R, 2)), &s, &c);
        }
        cs[r][kb] = c;
        sn[r][kb] = s;
      }
      __syncthreads();
      if (e < ne) {
        for (int r = 0; r < nr; ++r) {
          const double v = sigma[d_off[dsort_id[q0 + r0 + r]] - sbase + e];
#pragma unroll
          for (int kb = 0; kb < kKB; ++kb) {
            re[kb] = fma(v, cs[r][kb], re[kb]);
            im[kb] = fma(v, sn[r][kb], im[kb]);
          }
        }
      }
    }
    if (e < ne) {
      const int i = e / nJ, j = e - i * nJ;
      const long long row = bofs[I] + i, col = bofs[J] + j;
#pragma unroll
      for (int kb = 0; kb < kKB; ++kb)
        if (kb < nkb) H[((long long)(kb0 + kb) * nbasis + row) * nbasis + col] = make_double2(re[kb], im[kb]);
    }
  }
}

__global__ __launch_bounds__(kFT) void k_sigma_to_k(const double *__restrict__ sigma, const long long *__restrict__ d_off,
                                                    long long sbase, const int32_t *__restrict__ pstart,
                                                    const int32_t *__restrict__ pcount,
                                                    const int32_t *__restrict__ dsort_R,
                                                    const int32_t *__restrict__ dsort_id, const int32_t *__restrict__ nao,
                                                    const int32_t *__restrict__ bofs, int n, long long nbasis,
                                                    KChunk kc, double2 *__restrict__ H) {
  // XCD-aware order: consecutive workgroups are dealt round-robin to the eight XCDs; each XCD
  // takes a contiguous range of pair groups, so that neighbouring blocks of a row, whose rows
  // share cache lines of H, are written through the same L2
  const unsigned nblk = gridDim.x, b = blockIdx.x, per = nblk / 8, rem = nblk % 8, x = b % 8;
  const int grp = (int)((x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + b / 8);
  const int kb0 = blockIdx.y * kKB;
  for (int pp = 0; pp < kPP; ++pp) {
    const long long pair = (long long)grp * kPP + pp;
    if (pair >= (long long)n * n) break;  // uniform over the workgroup
    pair_to_k(sigma, d_off, sbase, pstart, pcount, dsort_R, dsort_id, nao, bofs, n, nbasis, kc, H, pair, kb0);
  }
}

// ---------------------------------------------------------------------------------------------
// The step before the build: the real-space density matrix from Kohn-Sham eigenvectors (Sec. II,
// eq. DM_realspace), with the phase of the Bloch convention of eq. Ham_rs2kspace (the two are
// each other's inverse):
//   D_{Ii,Jj}(R) = Re (1/N_k) sum_k exp(-i 2 pi k.R) P_k[Ii,Jj],
//   P_k[Ii,Jj]   = sum_n f_nk c_{Ii,n}(k) conj(c_{Jj,n}(k)),
// on the blocks of the cell's D pattern.  One workgroup per (atom pair I,J, chunk of kRD of the
// pair's R entries): the rows of I and J of the eigenvector matrices are staged in LDS, up to
// kKS k-points at a time when there are few bands (32 band-slots per stage row), else one
// k-point and 32 bands at a time; each thread forms one element of the pair's P_k block for the
// staged k-points and adds it, with the phase of each R entry of the chunk, into kRD
// accumulators.  P_k is never stored.
constexpr int kRD = 8;   // R entries per workgroup (16: 7 % slower; 4 with one k-point per stage: 3x slower)
constexpr int kNC = 32;  // band slots per staged row
constexpr int kKS = 8;   // most k-points per stage

__global__ __launch_bounds__(kFT) void k_density_from_k(const double2 *__restrict__ ck,
                                                        const double *__restrict__ occ, int n_occ,
                                                        long long nbasis, const long long *__restrict__ d_off,
                                                        long long sbase, const int32_t *__restrict__ pstart,
                                                        const int32_t *__restrict__ pcount,
                                                        const int32_t *__restrict__ dsort_R,
                                                        const int32_t *__restrict__ dsort_id,
                                                        const int32_t *__restrict__ nao,
                                                        const int32_t *__restrict__ bofs, int n, KChunk kc,
                                                        double scale, int add, double *__restrict__ D) {
  const unsigned nblk = gridDim.x, b = blockIdx.x, per = nblk / 8, rem = nblk % 8, x = b % 8;
  const long long pair = (long long)(x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + b / 8;
  const int r0 = blockIdx.y * kRD;
  const int npc = pcount[pair];
  if (r0 >= npc) return;  // uniform: this pair has fewer R entries
  const int nr = min(kRD, npc - r0), q0 = pstart[pair] + r0;
  const int I = (int)(pair / n), J = (int)(pair - (long long)I * n);
  const int nI = nao[I], nJ = nao[J], ne = nI * nJ;
  const long long rowI = bofs[I], rowJ = bofs[J];
  // bands per stage row and k-points per stage (nc * ksm = kNC)
  const int nc = n_occ <= 4 ? 4 : n_occ <= 8 ? 8 : n_occ <= 16 ? 16 : kNC;
  const int ksm = kNC / nc;
  __shared__ double2 sa[32 * kNC], sb[32 * kNC];  // [k-point][row][band slot]
  __shared__ double sf[kNC], pc[kKS][kRD], ps[kKS][kRD];
  for (int e0 = 0; e0 < ne; e0 += kFT) {
    const int e = e0 + (int)threadIdx.x;
    const bool on = e < ne;
    const int i = on ? e / nJ : 0, j = on ? e - (e / nJ) * nJ : 0;
    double acc[kRD];
#pragma unroll
    for (int r = 0; r < kRD; ++r) acc[r] = 0.0;
    for (int kq0 = 0; kq0 < kc.n; kq0 += ksm) {
      const int nks = min(ksm, kc.n - kq0);
      __syncthreads();  // everyone is done with the previous stage's phases and rows
      for (int t = threadIdx.x; t < nks * nr; t += kFT) {
        const int ks = t / nr, r = t - ks * nr;
        const int32_t R = dsort_R[q0 + r];
        const double *k = kc.k[kq0 + ks];
        double sv, cv;
        sincospi(2.0 * (k[0] * r_of(R, 0) + k[1] * r_of(R, 1) + k[2] * r_of(R, 2)), &sv, &cv);
        pc[ks][r] = cv;
        ps[ks][r] = sv;
      }
      double pre[kKS], pim[kKS];
#pragma unroll
      for (int ks = 0; ks < kKS; ++ks) pre[ks] = pim[ks] = 0.0;
      for (int n0 = 0; n0 < n_occ; n0 += nc) {  // a single pass whenever ksm > 1
        const int nn = min(nc, n_occ - n0);
        for (int t = threadIdx.x; t < nks * nI * nn; t += kFT) {
          const int ks = t / (nI * nn), u = t - ks * nI * nn, rr = u / nn, c = u - rr * nn;
          sa[(ks * 32 + rr) * nc + c] = ck[((long long)(kq0 + ks) * nbasis + rowI + rr) * n_occ + n0 + c];
        }
        for (int t = threadIdx.x; t < nks * nJ * nn; t += kFT) {
          const int ks = t / (nJ * nn), u = t - ks * nJ * nn, rr = u / nn, c = u - rr * nn;
          sb[(ks * 32 + rr) * nc + c] = ck[((long long)(kq0 + ks) * nbasis + rowJ + rr) * n_occ + n0 + c];
        }
        for (int t = threadIdx.x; t < nks * nn; t += kFT) {
          const int ks = t / nn, c = t - ks * nn;
          sf[ks * nc + c] = occ[(long long)(kq0 + ks) * n_occ + n0 + c];
        }
        __syncthreads();
        if (on)
#pragma unroll
          for (int ks = 0; ks < kKS; ++ks)
            if (ks < nks)
              for (int c = 0; c < nn; ++c) {
                const double2 a = sa[(ks * 32 + i) * nc + c], bj = sb[(ks * 32 + j) * nc + c];
                const double w = sf[ks * nc + c];
                pre[ks] = fma(w, fma(a.x, bj.x, a.y * bj.y), pre[ks]);   // Re(a conj(b))
                pim[ks] = fma(w, fma(a.y, bj.x, -a.x * bj.y), pim[ks]);  // Im(a conj(b))
              }
        __syncthreads();  // the rows are rewritten by the next band chunk
      }
      if (n_occ <= 0) __syncthreads();  // the phases are visible before they are read
      if (on)
#pragma unroll
        for (int ks = 0; ks < kKS; ++ks)
          if (ks < nks)
#pragma unroll
            for (int r = 0; r < kRD; ++r)
              if (r < nr) acc[r] = fma(pc[ks][r], pre[ks], fma(ps[ks][r], pim[ks], acc[r]));  // Re(exp(-i t) P)
    }
    if (on)
      for (int r = 0; r < nr; ++r) {
        double *dst = D + (d_off[dsort_id[q0 + r]] - sbase) + e;
        *dst = (add ? *dst : 0.0) + scale * acc[r];
      }
  }
}

hipError_t launch_density_from_k(const double *ck, const double *occ, int n_occ, long long nbasis,
                                 const long long *d_off, long long sbase, const int32_t *pstart,
                                 const int32_t *pcount, const int32_t *dsort_R, const int32_t *dsort_id,
                                 const int32_t *nao, const int32_t *bofs, int n, int max_pcount, const KChunk &kc,
                                 double scale, int add, double *D, hipStream_t s) {
  if (n <= 0 || kc.n <= 0 || max_pcount <= 0) return hipSuccess;
  const dim3 grid((unsigned)((long long)n * n), (unsigned)((max_pcount + kRD - 1) / kRD));
  hipLaunchKernelGGL(k_density_from_k, grid, dim3(kFT), 0, s, reinterpret_cast<const double2 *>(ck), occ, n_occ,
                     nbasis, d_off, sbase, pstart, pcount, dsort_R, dsort_id, nao, bofs, n, kc, scale, add, D);
  return hipGetLastError();
}

hipError_t launch_sigma_to_k(const double *sigma, const long long *d_off, long long sbase, const int32_t *pstart,
                             const int32_t *pcount, const int32_t *dsort_R, const int32_t *dsort_id,
                             const int32_t *nao, const int32_t *bofs, int n, long long nbasis, const KChunk &kc,
                             double *H, hipStream_t s) {
  if (n <= 0 || kc.n <= 0) return hipSuccess;
  const dim3 grid((unsigned)(((long long)n * n + kPP - 1) / kPP), (unsigned)((kc.n + kKB - 1) / kKB));
  hipLaunchKernelGGL(k_sigma_to_k, grid, dim3(kFT), 0, s, sigma, d_off, sbase, pstart, pcount, dsort_R, dsort_id,
                     nao, bofs, n, nbasis, kc, reinterpret_cast<double2 *>(H));
  return hipGetLastError();
}

}  // namespace hfx
