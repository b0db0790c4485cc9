// Library-internal interface of the real-space to k-space sum (hfx_fourier.hip), shared with the
// host plan (hfx_plan.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hfx {

// k-points of one launch (fractional coordinates of the reciprocal lattice)
constexpr int kKChunk = 64;
struct KChunk {
  double k[kKChunk][3];
  int n;
};

// H[k][row][col] (complex, interleaved) of one cell for the k-points of kc; every element of the
// n_basis x n_basis blocks of the kc.n k-points is written.  Tables as in DevPlan: the cell's
// n x n (pstart, pcount) table into the R-sorted pattern (dsort_R, dsort_id), compact offsets
// d_off of the concatenated layout whose cell part starts at sbase; nao and bofs (basis offset
// within the cell) per cell-local atom.
hipError_t launch_sigma_to_k(const double *sigma, const long long *d_off, long long sbase, const int32_t *pstart,
                             const int32_t *pcount, const int32_t *dsort_R, const int32_t *dsort_id,
                             const int32_t *nao, const int32_t *bofs, int n, long long nbasis, const KChunk &kc,
                             double *H, hipStream_t s);

// D of one cell on its pattern from eigenvectors ck [k][n_basis][n_occ] (complex, interleaved)
// and occupations occ [k][n_occ] of the kc.n k-points: D = (add ? D : 0) + scale * sum_k ...;
// max_pcount: the largest number of pattern entries of any atom pair of the cell.
hipError_t launch_density_from_k(const double *ck, const double *occ, int n_occ, long long nbasis,
                                 const long long *d_off, long long sbase, const int32_t *pstart,
                                 const int32_t *pcount, const int32_t *dsort_R, const int32_t *dsort_id,
                                 const int32_t *nao, const int32_t *bofs, int n, int max_pcount, const KChunk &kc,
                                 double scale, int add, double *D, hipStream_t s);

}  // namespace hfx
