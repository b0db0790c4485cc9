// Library-internal layouts shared by the host plan (hfx_plan.hip) and the
// device kernels (hfx_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hfx {

// Lattice vectors are packed as three signed 10-bit fields.
constexpr int kRBias = 512;
__host__ __device__ inline int32_t pack_r(int r0, int r1, int r2) {
  return ((r0 + kRBias) << 20) | ((r1 + kRBias) << 10) | (r2 + kRBias);
}
__host__ __device__ inline int r_of(int32_t p, int k) { return ((p >> (20 - 10 * k)) & 1023) - kRBias; }
__host__ __device__ inline int32_t r_add(int32_t a, int32_t b) {
  return pack_r(r_of(a, 0) + r_of(b, 0), r_of(a, 1) + r_of(b, 1), r_of(a, 2) + r_of(b, 2));
}
__host__ __device__ inline int32_t r_sub(int32_t a, int32_t b) {
  return pack_r(r_of(a, 0) - r_of(b, 0), r_of(a, 1) - r_of(b, 1), r_of(a, 2) - r_of(b, 2));
}
__host__ __device__ inline bool r_zero(int32_t p) { return p == pack_r(0, 0, 0); }

// per kept C block (row atom A, column atom F at lattice vector R): the
// Cauchy-Schwarz factors of the three screening stages and the CS-ERI factor
struct CNorm {
  double nA;  // max_a ||C[:,a,:]||
  double gA;  // max_a sqrt||C_a C_a^T||
  double nF;  // max_f ||C[:,:,f]||
  double gF;  // max_f sqrt||C_f C_f^T||
  double Q;   // sqrt(max_{a,f} (Aa Ff|Aa Ff))
};

// one <A,B> work item: A a home atom, B = (atom b, lattice vector rb)
struct Item {
  int32_t A, B, rb, vid;  // vid: kept V block index
};

// Everything the main kernel reads, as device pointers.
struct DevPlan {
  // atoms (global numbering over cells)
  int32_t n_atoms;
  const int32_t *nao, *nabf, *cell_of, *local_of;
  // kept C blocks, grouped by row atom (c_start), sorted by distance within a row
  const double *Cbuf;
  const double *CTbuf;  // same blocks, each transposed to [n_ao(col)][n_abf(row) * n_ao(row)]
  const float *C32, *CT32;  // FP32 copies of Cbuf and CTbuf (same offsets) for FP32 block products
  const long long *c_off;
  const int32_t *c_col, *c_R;
  const CNorm *c_norm;
  const int32_t *c_start;
  // kept V blocks
  const double *Vbuf;
  const long long *v_off;
  const double *gV;
  // D pattern lookup: for (cell-local row, cell-local col) a range of R-sorted entries
  const int32_t *ptab_off;  // per cell: start of its n_c*n_c table in pstart/pcount
  const int32_t *pstart, *pcount;
  const int32_t *dsort_R, *dsort_id;
  const int32_t *cell_natoms;
  // D / Sigma (compact, D pattern order, all cells concatenated)
  const long long *d_off;
  const double *Dbuf;
  const double *gD;
  const uint8_t *keepD;
  const double *gDmax;  // per cell: max over kept D blocks of sqrt||D D^T||
  double *Sbuf;
  // work
  const Item *items;
  const int32_t *order;  // schedule: item indices in processing order
  int32_t n_items;
  // thresholds and switches
  double eps_eri, eps_mat;
  uint32_t stages;
  // scratch (per persistent slot)
  double *scratch;
  int64_t slot_doubles;
  int32_t max_nbr;  // max kept C blocks of any atom
  int32_t max_p, max_n;
  // counters
  unsigned int *ticket;           // per group: next position within the group's schedule segment
  const int32_t *grp_start;      // n_groups + 1: schedule segments (group g: positions [start[g], start[g+1]))
  int32_t n_groups;              // 1: one global ticket; k-means grouping: one group per XCD
  unsigned long long *counters;  // see kCnt* below
  double *flops;                 // [0] Algorithm-3 count, [1] this kernel's useful count
  long long *item_cycles;        // per item (plan order)
  int *item_units;               // per item x kItemUnits
  double *item_contrib;          // per item: summed screening bounds of its kept units
  double *item_flops;            // per item: its contraction FLOPs (kept units and alive G)
};

enum {
  kCntCandidates = 0,
  kCntCsEri = 1,
  kCntKept = 2,  // 12 entries: stage*4 + term
  kCntG = 14,
  kCntMfmaR = 15,  // MFMA instructions issued, GEMM-R
  kCntMfmaL = 16,  // MFMA instructions issued, GEMM-L
  kCntMfmaY = 17,
  kCntPhase = 18,  // 6 entries: wall-clock ticks per phase, summed over items
  kCntMfmaR32 = 24,  // FP32 MFMA instructions issued, GEMM-R
  kCntMfmaL32 = 25,  // FP32 MFMA instructions issued, GEMM-L
  kCntMfmaRbf = 26,  // BF16 MFMA instructions (16x16x32) issued, GEMM-R
  kCntN = 27
};

constexpr int kItemUnits = 5;  // per item: kept units of terms 1..4, alive G
constexpr int kMaxGroups = 16;  // schedule groups (tickets)
constexpr int kItemFeatures = 10;  // scheduler model inputs per item
constexpr int kItemTargets = 2;   // scheduler model outputs: log cycles, log contribution bound

constexpr uint32_t kPre = 1u, kCsEri = 2u, kCs1 = 4u, kCs2 = 8u, kCs3 = 16u;

}  // namespace hfx
