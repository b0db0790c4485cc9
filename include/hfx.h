/*
 * hfx.h - C ABI of the MI355X (gfx950) library that builds the screened,
 * linear-scaling periodic Hartree-Fock exchange matrix under the localized
 * resolution of identity (Lin, Ren & He, "Efficient Hybrid Density Functional
 * Calculations for Large Periodic Systems Using Numerical Atomic Orbitals").
 *
 * What is computed (Sec. II, eqs. HFX_ERIs, LRI, HFX_LRI, HFX_split,
 * partial_integrals; Sec. III A, Algorithms 2 and 3; Sec. III B-C,
 * Algorithms 4 and 5):
 *
 *   Sigma^X_{Ii,Jj}(R) = - sum_{K,L} sum_{k,l} (Ii Kk | Jj Ll) D_{Kk,Ll}
 *   (Ii Kk | Jj Ll)    = sum_{A in {I,K}} sum_{B in {J,L}} C^{A} V_{AB} C^{B}
 *
 * evaluated as the <A,B> loop of Algorithm 2 in the order C((VC)D) of
 * Algorithm 3, with the block pre-screening of C, V, D by max-abs (Sec. III B),
 * the CS-ERI quartet test (Sec. III C 2, eq. CS-ERI) and the three-stage
 * Cauchy-Schwarz matrix screening (eq. CS_upper_bounds, Algorithm 4), and
 *   E_x = 1/2 <D, Sigma^X>       (Algorithm 5, "Calculate E^X").
 *
 * Conventions (readings of points the paper leaves open):
 *  - All indices are 0-based, lengths in elements, lengths in bohr, energies in Hartree.
 *  - An atom reference is (home-cell atom index, integer lattice vector R) (eq. AO).
 *  - Block-sparse periodic tensors hold one dense row-major FP64 block per
 *    (row atom, column atom, R); the row atom is in the home cell, the column
 *    atom in cell R.  Shapes:  C: [n_abf(row)][n_ao(row)][n_ao(col)]  (the ABF
 *    sits on the row atom, which also carries the first AO index, eq. LRI);
 *    V: [n_abf(row)][n_abf(col)];  D and Sigma: [n_ao(row)][n_ao(col)].
 *    Blocks are translation invariant: the block between X in cell R1 and Y in
 *    cell R2 is the stored (X, Y, R2 - R1).
 *  - On-site pairs follow set semantics: a unit whose F is A itself (same atom,
 *    same cell) is weighted 1/2, likewise G = B; on-site C blocks must be
 *    symmetric in their two AO indices.
 *  - "Kept" means bound > threshold; a threshold of 0 keeps every non-zero bound.
 *  - Sigma is produced on the block pattern of D; contributions to blocks
 *    outside that pattern are not formed.
 *
 * Ownership: inputs are borrowed for the duration of a call.  hfx_plan_create
 * copies what it needs (C, V, the D pattern) into device memory it owns;
 * hfx_build reads D and writes Sigma, stream-ordered on the plan's stream.
 *
 * Errors: every function returns an hfx_status and never aborts; the message
 * of the last failure on the calling thread is in hfx_last_error().  After an
 * error the outputs are unspecified; the plan stays usable except after
 * HFX_ERR_HIP, which poisons it (every later call returns HFX_ERR_STATE).
 *
 * Thread safety: a plan is not thread-safe; distinct plans are independent.
 */
#ifndef HFX_H
#define HFX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HFX_ABI_VERSION 3

typedef enum {
  HFX_OK = 0,
  HFX_ERR_ARG = 1,         /* NULL pointer, bad count, non-finite or negative threshold      */
  HFX_ERR_SHAPE = 2,       /* block index out of range, inconsistent sizes, duplicate blocks  */
  HFX_ERR_SYMMETRY = 3,    /* V(A,B,R) != V(B,A,-R)^T, or a non-symmetric on-site C block     */
  HFX_ERR_OOM = 4,         /* device allocation failed or exceeds max_device_bytes            */
  HFX_ERR_HIP = 5,         /* a HIP runtime call failed (plan is poisoned)                    */
  HFX_ERR_STATE = 6,       /* D does not match the plan's pattern, or poisoned plan           */
  HFX_ERR_UNSUPPORTED = 7  /* option value not implemented, or a size beyond the limits below */
} hfx_status;

typedef struct {
  int32_t n_ao;  /* atomic orbitals per atom of this species  (n_phi)                         */
  int32_t n_abf; /* auxiliary basis functions per atom         (n_P)                          */
} hfx_species;

typedef struct {             /* one periodic home cell                                      */
  int32_t n_atoms;
  double lattice[9];         /* rows a1, a2, a3 (bohr)                                       */
  const double *pos;         /* n_atoms*3 cartesian positions (bohr), host                   */
  const int32_t *species;    /* n_atoms species indices, host                                */
  int32_t n_species;
  const hfx_species *sp;     /* n_species entries, host                                      */
} hfx_cell;

typedef struct {             /* block-sparse periodic tensor                                 */
  int64_t n_blocks;
  const int32_t *row;        /* n_blocks home-cell row atoms, host                           */
  const int32_t *col;        /* n_blocks home-cell index of the column atom, host            */
  const int32_t *R;          /* n_blocks*3 lattice vector of the column atom, host           */
  const int64_t *off;        /* n_blocks start of each block in data (elements), host; blocks
                                may alias each other (read-only)                             */
  const double *data;        /* FP64 block data, host (on_device=0) or device (on_device=1)  */
  int32_t on_device;
} hfx_blocks;

typedef struct {             /* Sec. III B and III C; 0 keeps every non-zero bound           */
  double eps_C;              /* drop C blocks with max-abs <= eps_C                          */
  double eps_V;              /* drop V blocks with max-abs <= eps_V                          */
  double eps_D;              /* drop D blocks with max-abs <= eps_D (per build)              */
  double eps_cs_eri;         /* keep a quartet iff Q_AF * Q_BG > eps_cs_eri                  */
  double eps_cs_mat;         /* keep a unit iff each of the three bounds > eps_cs_mat        */
} hfx_thresholds;

/* precision of the block products that contract C with the (VC)D intermediates
 * (terms 1-4); the screening bounds, Y = V C, T3, T4, the Gram matrices, the
 * accumulation into Sigma and the energy are FP64 in every mode */
#define HFX_PREC_FP64 0     /* every block product in FP64                                 */
#define HFX_PREC_FP32 1     /* every block product on FP32 MFMA (FP32 operands and sums)   */
#define HFX_PREC_TIERED 2   /* a block product runs on FP32 MFMA when the stage-2 bound of
                               every kept unit in it is <= tier_tau, else in FP64           */
#define HFX_PREC_BF16X3 3   /* three tiers: as HFX_PREC_TIERED, and a terms-3/4 block product
                               whose kept units all have a stage-2 bound <= tier_tau_bf runs
                               as split-BF16x3 (each FP32 operand split as hi + lo in BF16,
                               hi*hi + hi*lo + lo*hi on the BF16 matrix cores with FP32 sums,
                               about 2^-16 relative error); the terms-1/2 product's lowest
                               tier stays FP32                                              */

#define HFX_SCREEN_PRE 1u    /* block max-abs pre-screening of C, V, D                     */
#define HFX_SCREEN_CS_ERI 2u /* CS-ERI quartet test                                        */
#define HFX_SCREEN_CS1 4u    /* CS-matrix stage 1: sqrt||CC+|| sqrt||VV+|| sqrt||CC+|| sqrt||DD+|| */
#define HFX_SCREEN_CS2 8u    /* CS-matrix stage 2: sqrt||CC+|| ||VC|| sqrt||DD+||          */
#define HFX_SCREEN_CS3 16u   /* CS-matrix stage 3: ||C|| ||(VC)D||                         */
#define HFX_SCREEN_ALL 31u

/* Order in which the persistent kernel takes the <A,B> work items (the greedy longest-first
 * machine scheduling of Sec. III D 1, Algorithm 6, with different cost estimates).  No order
 * changes which units are computed, only the order of the FP64 accumulations into Sigma. */
#define HFX_SCHED_PLAN 0    /* work items in plan order                                    */
#define HFX_SCHED_LPT 1     /* longest first on |N_C(A)| |N_C(B)| (the pre-screen proxy)    */
#define HFX_SCHED_MLP 2     /* longest predicted first by the learned cost model (mlp_weights);
                               the first build uses HFX_SCHED_LPT                           */
#define HFX_SCHED_EXACT 3   /* longest first on each item's exact contraction FLOPs of the
                               previous build (its kept units and alive G, the count of
                               hfx_build_stats.flops_contract); the first build uses LPT    */
#define HFX_SCHED_NORM 4    /* norm-sorted packing: largest first on the product of the block
                               norms that enter every stage-1 bound of the item,
                               gV_AB * max_F g(C_AF) * max_G g(C_BG), g the sqrt||X X^T||
                               factors of Sec. III C 1 (static, known at plan time)          */
#define HFX_SCHED_KMEANS 5  /* locality groups (the k-means distribution of Sec. III D 2,
                               Algorithm 7, on one GPU): items clustered by k-means on the
                               midpoints of their atom pairs into one group per XCD (8), LPT
                               order inside a group; the workgroups of an XCD drain their own
                               group first, then take items from the others                 */

typedef struct {
  int32_t precision;          /* HFX_PREC_*                                                 */
  uint32_t stages;            /* HFX_SCREEN_* bitmask; 0 means HFX_SCREEN_ALL               */
  double tier_tau;            /* TIERED: a block product whose kept units all have a stage-2
                                 bound <= tier_tau runs on FP32 MFMA (finite, >= 0; < 0: the
                                 value the tuning file holds for this plan)                 */
  double tier_tau_bf;         /* BF16X3: bound of the split-BF16x3 tier (<= tier_tau; < 0: the
                                 tuning file's value)                                      */
  int32_t scheduler;          /* HFX_SCHED_*                                                */
  const char *mlp_weights;    /* file written by the scheduler trainer, or NULL             */
  void *stream;               /* hipStream_t for plan-time and build work; NULL = default   */
  const int32_t *home_subset; /* global atom ids (atom i of cell c is atom_offset(c)+i)
                                 whose <A,B> work items are built; NULL = all              */
  int32_t n_home_subset;
  uint64_t max_device_bytes;  /* 0 = unlimited; else plan creation fails with HFX_ERR_OOM
                                 when its device footprint would exceed this               */
  int32_t n_slots;            /* persistent workgroups (0 = automatic)                      */
  int32_t use_graph;          /* 1: hfx_build replays one captured HIP graph of the whole
                                 device-side build (D gather, D screening, Sigma clear,
                                 persistent kernel, Sigma copy-out); needs D on the device;
                                 the graph is re-captured when the D or Sigma pointers change */
  const char *tuning_db;      /* text file written by the autotuner, or NULL: one choice per line,
                                   hfxtune1 <key> tile_r=<32|64|128> tier_tau=<x> tier_tau_bf=<x>
                                 where <key> is hfx_tune_key's string of the plan; the last
                                 line with the plan's key is used                            */
  int32_t tile_r;             /* column width of the output blocks of the terms-3/4 product:
                                 32, 64 or 128; 0: the tuning file's choice, else 64        */
} hfx_options;

typedef struct {               /* filled by hfx_build when non-NULL (synchronises)          */
  int64_t candidates;          /* (A,B,F,G) grid points visited                             */
  int64_t kept_cs_eri;         /* quartets passing CS-ERI                                   */
  int64_t kept[3][4];          /* [stage 1..3][term 1..4] units surviving each stage        */
  int64_t items;               /* <A,B> work items                                          */
  int64_t g_alive;             /* (A,B,G) triples whose Y = V C was formed                  */
  double flops_contract;       /* useful FLOPs of the contractions this library performs for
                                  the kept units (padding and screened-out work excluded)   */
  double flops_paper;          /* FLOPs of the same kept units counted as in Algorithm 3:
                                  T and Htilde per unit, Y, T3, T4 once per (A,B,G)          */
  double flops_tier[3];        /* flops_contract split by precision: FP64 / FP32 / BF16x3, by the
                                  precision shares of the block products issued (a split-BF16x3
                                  16x16x32 product counts as 16 FP32 16x16x4 ones)          */
  double mfma_flops[3];        /* matrix-core FLOPs issued (with padding): G side and masks,
                                  terms 3+4, terms 1+2                                       */
  double ms_total;             /* device time of the build (events on the plan stream)      */
  double ms_main;              /* device time of the main persistent kernel (graph mode: the
                                  whole graph, as ms_total)                                  */
  double phase_share[6];       /* share of the summed per-item time spent in: screening,
                                  Y = VC and the G-side products, stage-2/3 masks, terms 3+4,
                                  terms 1+2, item set-up                                     */
  double mfma_flops_fp32;      /* part of mfma_flops issued on the FP32 matrix cores         */
  int32_t tile_r;              /* column width of the terms-3/4 output blocks the build used */
  int32_t pad;
  double tier_tau, tier_tau_bf; /* precision-tier bounds the build used                     */
  double mfma_flops_bf16;      /* part of mfma_flops issued on the BF16 matrix cores (split-BF16x3) */
} hfx_build_stats;

typedef struct hfx_plan hfx_plan;

/* Per-geometry set-up (Algorithm 5, "Calculate C and V"): validates the
 * inputs, pre-screens C and V, computes the block norms of the Cauchy-Schwarz
 * bounds and the CS-ERI factors Q_AF = sqrt(max_{a,f} (Aa Ff|Aa Ff)), builds
 * the neighbour lists N[A] (Sec. III B 1) and the <A,B> work items, and
 * copies everything to device memory owned by the plan.
 *   n_cells     >= 1 independent cells, built together in one launch
 *   cells       n_cells cell descriptions
 *   C, V        n_cells block sets each (data host or device)
 *   D_pattern   n_cells D block structures (row/col/R/off; data may be NULL)
 *   th          thresholds; opt: options (NULL = defaults)
 *   out         receives the plan
 * Limits of this implementation (HFX_ERR_UNSUPPORTED, with the reason in hfx_last_error):
 * n_ao of a species 1..32 and n_abf 1..512; at most 160 kept C blocks (neighbours F of
 * Sec. III B 1) per atom; lattice vector indices within +-200; per-item tables that fit the
 * decode tables and 160 KB of LDS per workgroup.  HFX_ERR_OOM when the device footprint
 * exceeds max_device_bytes or an allocation fails.
 * Synchronises before returning. */
hfx_status hfx_plan_create(int32_t n_cells, const hfx_cell *cells, const hfx_blocks *C, const hfx_blocks *V,
                           const hfx_blocks *D_pattern, const hfx_thresholds *th, const hfx_options *opt,
                           hfx_plan **out);

/* Layout of Sigma for one cell.  Sigma^X_{Ii,Jj}(R) of eq. HFX_ERIs is formed on the
 * real-space block pattern of D (Sec. III B 3, the sparsity of D): the D pattern's
 * row/col/R with compact offsets (running sum of n_ao(row)*n_ao(col) in block order).  The arrays
 * are owned by the plan (host memory, valid until hfx_plan_destroy);
 * layout->data is NULL.  *n_elements receives the FP64 count of the cell's
 * Sigma buffer. */
hfx_status hfx_sigma_layout(const hfx_plan *plan, int32_t cell, hfx_blocks *layout, int64_t *n_elements);

/* Per-SCF-step build (Algorithm 5, "Calculate exact-exchange"):
 *   D      n_cells density matrices with the plan's pattern: n_blocks and the
 *          block shapes must match; off (if non-NULL) must equal the
 *          pattern's off, else HFX_ERR_STATE.  data host or device.
 *   sigma  n_cells device buffers of hfx_sigma_layout's size, fully overwritten
 *   stats  optional; when non-NULL the call synchronises and fills it
 * Stream-ordered on opt.stream; returns before completion unless stats is
 * requested.  D is read during the call's stream work; keep it alive until
 * the stream has passed this call's work. */
hfx_status hfx_build(hfx_plan *plan, const hfx_blocks *D, double *const *sigma, hfx_build_stats *stats);

/* E_x = 1/2 <D, Sigma^X> per cell (the exchange energy of the matrix of eq. HFX_ERIs
 * with the density matrix of eq. DM_realspace; Sigma^X = -K, no spin factor) with
 * compensated FP64 summation over the D pattern; D as in hfx_build, sigma device buffers from hfx_build.
 * e_x: n_cells host doubles.  Synchronises. */
hfx_status hfx_energy(hfx_plan *plan, const hfx_blocks *D, double *const *sigma, double *e_x);

/* The step after the build in a band-structure calculation (Sec. IV,
 * band-structure calculations, eq. Ham_rs2kspace): the matrix at k-points
 *   H_{Ii,Jj}(k) = sum_R exp(i 2 pi k.R) Sigma_{Ii,Jj}(R)
 * of one cell, summed over the blocks of the cell's D pattern, R the integer
 * lattice vector of the column atom J.
 *   cell   index of the cell in the plan
 *   sigma  device, the cell's Sigma in hfx_sigma_layout order (e.g. from hfx_build)
 *   n_k    number of k-points (0: nothing is done)
 *   kfrac  host, n_k*3 doubles: k in fractional coordinates of the reciprocal
 *          lattice (k.R = 2 pi kfrac.n_R); read during the call only
 *   hk     device, n_k * n_basis * n_basis complex doubles (re, im interleaved),
 *          row-major [k][row][col] with the basis ordered by atom, then AO;
 *          every element is written.  n_basis = sum of n_ao over the cell's atoms.
 * Stream-ordered on opt.stream; returns before completion.  Errors:
 * HFX_ERR_ARG for a bad cell, n_k < 0, NULL arrays or non-finite k. */
hfx_status hfx_sigma_to_k(hfx_plan *plan, int32_t cell, const double *sigma, int32_t n_k, const double *kfrac,
                          double *hk);

/* The step before the build: the real-space density matrix from Kohn-Sham
 * eigenvectors (Sec. II, eq. DM_realspace) on the cell's D pattern,
 *   D_{Ii,Jj}(R) = Re (1/n_k) sum_k exp(-i 2 pi k.R) sum_n f_nk c_{Ii,n}(k) conj(c_{Jj,n}(k)),
 * R the integer lattice vector of the column atom J.  The phase is the one of
 * the Bloch convention of hfx_sigma_to_k (eigenvectors of that H(k)), for which
 * the two calls are each other's inverse; the real part is the whole value
 * when the k-set is closed under k -> -k with c(-k) = conj(c(k)).
 *   cell   index of the cell in the plan
 *   n_k    number of k-points (>= 1); kfrac: host, n_k*3 fractional coordinates
 *   n_occ  bands per k-point (0: D = 0)
 *   ck     device, n_k * n_basis * n_occ complex doubles (re, im interleaved),
 *          [k][basis][band], basis ordered by atom then AO
 *   occ    device, n_k * n_occ doubles: the occupations f_nk
 *   d      device, the cell's D in hfx_sigma_layout order; fully overwritten
 * Stream-ordered on opt.stream; returns before completion.  Errors:
 * HFX_ERR_ARG for a bad cell, n_k < 1, n_occ < 0, NULL arrays or non-finite k. */
hfx_status hfx_density_from_k(hfx_plan *plan, int32_t cell, int32_t n_k, const double *kfrac, int32_t n_occ,
                              const double *ck, const double *occ, double *d);

/* Per-item labels of the last build, for scheduler training: for each work
 * item in plan order, its main-kernel wall-clock ticks (100 MHz), five
 * counters the kernel produced (kept units of terms 1..4 after stage 3 and
 * the number of G whose Y = V C was formed) and its contribution bound: the
 * sum over its kept units of the tightest screening bound the kernel computed
 * for the unit (the stage-3 bound of Sec. III C 2 where stage 3 runs, else
 * the stage-2 bound), an upper bound of the Frobenius norm of the item's
 * contribution to Sigma.  cycles: n_items int64, units: n_items*5 int64,
 * contrib: n_items doubles (host); any may be NULL.  Synchronises. */
hfx_status hfx_item_profile(hfx_plan *plan, int64_t *n_items, int64_t *cycles, int64_t *units, double *contrib);

/* Learned model of the scheduler (the greedy longest-first machine
 * scheduling of Sec. III D 1, Algorithm 6, applied to predicted instead of
 * static costs): a perceptron x -> tanh(W1 x + b1) -> tanh(W2 h + b2) -> W3 h + b3
 * with n_in inputs, n_hidden units per hidden layer and n_out linear outputs;
 * FP32 parameters laid out as W1[n_hidden][n_in], b1, W2[n_hidden][n_hidden],
 * b2, W3[n_out][n_hidden], b3[n_out].  The scheduler's model has two outputs:
 * log(cycles) and log of the contribution bound (hfx_item_profile), each
 * standardised by the trainer.  All arrays are device memory; stream as in
 * hfx_options.  The model never changes which units are computed, only the
 * order in which items run.
 * Errors: HFX_ERR_ARG for n_in outside 1..16, n_hidden outside 1..64, n_out
 * outside 1..4, NULL arrays, n < 0, epochs < 0 or lr <= 0; HFX_ERR_OOM if the
 * optimizer state cannot be allocated; HFX_ERR_HIP if a launch fails. */
int64_t hfx_mlp_n_params(int32_t n_in, int32_t n_hidden, int32_t n_out);

/* y[i*n_out + o] = output o of the model at X[i*n_in ..], for n samples. */
hfx_status hfx_mlp_predict(int32_t n_in, int32_t n_hidden, int32_t n_out, const float *params, const float *X,
                           int64_t n, float *y, void *stream);

/* loss = mean over samples of sum_o (y_io - t_io)^2 (t: n x n_out) and
 * grad = d loss / d params (overwritten). */
hfx_status hfx_mlp_loss_grad(int32_t n_in, int32_t n_hidden, int32_t n_out, const float *params, const float *X,
                             const float *t, int64_t n, float *grad, float *loss, void *stream);

/* Full-batch Adam on that loss for `epochs` steps (params updated in place);
 * loss_host (host, epochs floats, optional) receives the loss before each
 * step.  Allocates its optimizer state.  Synchronises. */
hfx_status hfx_mlp_train(int32_t n_in, int32_t n_hidden, int32_t n_out, float *params, const float *X, const float *t,
                         int64_t n, int32_t epochs, float lr, float *loss_host, void *stream);

/* hfx_mlp_train without allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same full-batch
 * Adam on the same loss, with the gradient, the Adam moments and the loss of the current epoch in
 * a static device array the library holds on each GPU for the life of the process (sized for the
 * largest model it takes: n_in <= 16, n_hidden <= 64, n_out <= 4, i.e. at most 5508 parameters,
 * 66 KB).  The moments are cleared at the start of each call.  Stream-ordered: returns after
 * enqueueing, without synchronising and without host copies.
 *   params, X, t  device, as in hfx_mlp_train
 *   loss_dev      device, epochs floats (optional): the loss before each step
 * Every call on one GPU shares that array: calls that overlap on one GPU (two streams, two host
 * threads) race and give undefined results; serialise them.  Errors: HFX_ERR_ARG as for
 * hfx_mlp_train, or an argument that is not GPU-accessible memory; HFX_ERR_HIP if a launch fails. */
hfx_status hfx_mlp_train_static(int32_t n_in, int32_t n_hidden, int32_t n_out, float *params, const float *X,
                                const float *t, int64_t n, int32_t epochs, float lr, float *loss_dev, void *stream);

/* The scheduler's 10 input features of every work item: from the last
 * build's counters log1p(kept units of terms 1..4), log1p(G formed); from the
 * plan log(|N(A)| |N(B)|), n_ao(A)/16, n_abf(A)/64, the pair distance
 * |r_B + R - r_A| / 10 bohr and log(atoms of the item's cell); each
 * normalised as (x - mu[k]) / sd[k] (mu, sd: 10 host floats).  X: device,
 * n_items*10 floats.  A plan created with HFX_SCHED_MLP and a model file
 * (mlp_weights: "HFXMLP02", int32 n_in = 10, int32 n_hidden, int32 n_out,
 * float mu[10], float sd[10], float params[...], then any trailing data,
 * which the library does not read) orders each build's items by
 * output 0 of the model applied to these features of the previous build (its
 * first build uses HFX_SCHED_LPT order).  Synchronises. */
hfx_status hfx_item_features(hfx_plan *plan, const float *mu, const float *sd, float *X);

/* The key under which the autotuner files its choices for this plan: the species present (n_ao x
 * n_abf, sorted, '+'-joined), the CS-matrix threshold and the precision form, e.g.
 *   "species=13x60 eps=1e-06 prec=tiered"
 * written into buf (len bytes, NUL-terminated).  HFX_ERR_ARG if buf is too small. */
hfx_status hfx_tune_key(const hfx_plan *plan, char *buf, int32_t len);

/* Dense matrix-core throughput of the current GPU, measured: the peak the roofline fraction of
 * the build (an MFMA-bound dense block contraction, Algorithm 3 and Table multiply) is judged
 * against, taken on this part rather than from its data sheet.  Every wave of a grid that fills all
 * compute units issues independent chains of one MFMA instruction on register operands:
 *   kind 0  FP64  16x16x4  (2048 FLOP per instruction)
 *   kind 1  FP32  16x16x4  (2048)
 *   kind 2  BF16  16x16x32 with FP32 sums (16384)
 * tflops (host) receives FLOPs / kernel time / 1e12, 2 FLOPs per multiply-add; sclk_mhz (host,
 * optional) the shader clock during the run, from the cycle counter against the constant-rate wall
 * clock.  About 60 ms of GPU time on stream (NULL = default).  Allocates and frees a small device
 * buffer; synchronises.  Errors: HFX_ERR_ARG for another kind or NULL tflops, HFX_ERR_OOM,
 * HFX_ERR_HIP. */
hfx_status hfx_mfma_peak(int32_t kind, void *stream, double *tflops, double *sclk_mhz);

void hfx_plan_destroy(hfx_plan *plan);
const char *hfx_last_error(void);
int32_t hfx_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HFX_H */
