// Host side of the C ABI (include/hfx.h): validation, indexing, device
// layouts, and the stream-ordered build.  The paper's per-geometry work
// (Algorithm 5, "Calculate C and V": pre-screening, norms, CS-ERI factors)
// happens in hfx_plan_create; the per-SCF-step work ("Calculate
// exact-exchange") in hfx_build.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hfx.h"
#include "hfx_fourier.h"
#include "hfx_internal.h"

namespace hfx {
hipError_t launch_main(const DevPlan &P, int n_slots, int rows_cap, int cols_cap, int ld3, long long wave_off,
                       long long wave_doubles, long long wg_off, long long ub_off, int tier, float tau, float tau_bf,
                       int tile_r, hipStream_t s, bool set_lds);
hipError_t main_set_lds(int rows_cap, int cols_cap, int ld3);
hipError_t launch_to_f32(const double *src, float *dst, long long n, hipStream_t s);
size_t main_dyn_lds(int rows_cap, int cols_cap, int ld3);
hipError_t launch_ctrans(const double *Cbuf, const long long *c_off, const int *c_row, const int *c_col,
                         const int *nao, const int *nabf, int nC, double *CT, hipStream_t s);
size_t main_static_lds();
int main_threads();
int main_maxnb();
int main_maxn();
int main_nwaves();
hipError_t launch_cnorm(const double *Cbuf, const long long *c_off, const int *c_row, const int *c_col,
                        const int *nao, const int *nabf, int nC, CNorm *out, hipStream_t s);
hipError_t launch_cq(const double *Cbuf, const long long *c_off, const int *c_row, const int *c_col,
                     const double *Vbuf, const long long *v_off, const int *qsrc, const int *nao, const int *nabf,
                     int nC, CNorm *out, hipStream_t s);
hipError_t launch_vnorm(const double *Vbuf, const long long *v_off, const int *v_row, const int *v_col,
                        const int *nabf, int nV, double *gV, hipStream_t s);
hipError_t launch_dgather(const double *src, const long long *src_off, const long long *dst_off, int nD,
                          long long base, double *dst, hipStream_t s);
hipError_t launch_dprep(const double *Dbuf, const long long *d_off, const int *d_row, const int *d_col,
                        const int *nao, int nD, double eps_D, int pre, double *gD, uint8_t *keepD, hipStream_t s);
hipError_t launch_zero(double *p, long long n, hipStream_t s);
hipError_t launch_dmax(const double *gD, const uint8_t *keepD, const long long *dbase, double *gDmax, int n_cells,
                       hipStream_t s);
hipError_t launch_reset(unsigned int *ticket, unsigned long long *counters, double *flops, hipStream_t s);
hipError_t launch_energy(const double *D, const double *S, long long n, double *part, int nblk, hipStream_t s);
hipError_t mlp_launch_predict(const float *P, int F, int H, int O, const float *X, long long n, float *out,
                              hipStream_t s);
hipError_t mlp_launch_grad(const float *P, int F, int H, int O, const float *X, const float *T, long long n, float *G,
                           float *loss, hipStream_t s);
hipError_t mlp_launch_adam(float *P, const float *G, float *m, float *v, int np, float lr, int step, hipStream_t s);
hipError_t mlp_launch_features(const Item *items, const int *units, const int *c_start, const int *nao,
                               const int *nabf, const float *dist, const int *cell_of, const int *cell_natoms,
                               long long n, const float *mu, const float *sd, float *X, hipStream_t s);
int64_t mlp_params(int F, int H, int O);
hipError_t mlp_train_static(int F, int H, int O, float *P, const float *X, const float *T, long long n, int epochs,
                            float lr, float *loss_dev, hipStream_t s);
int mlp_scratch_max_params();
int mlp_max_h();
int mlp_max_f();
int mlp_max_o();
hipError_t mfma_peak_run(int kind, int n_cu, int iters, double *out, long long *clk, hipStream_t st, float *ms,
                         double *flops);
int mfma_peak_blocks_per_cu();
int mfma_peak_threads();
}  // namespace hfx

using namespace hfx;

namespace {

thread_local std::string g_err;

hfx_status fail(hfx_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

struct Key {
  int32_t row, col, r;
  bool operator==(const Key &o) const { return row == o.row && col == o.col && r == o.r; }
};
struct KeyHash {
  size_t operator()(const Key &k) const {
    uint64_t h = (uint64_t)(uint32_t)k.row * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)(uint32_t)k.col + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)k.r * 0xBF58476D1CE4E5B9ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

constexpr int kRMax = 200;

bool r_ok(const int32_t *R) {
  for (int k = 0; k < 3; ++k)
    if (R[k] < -kRMax || R[k] > kRMax) return false;
  return true;
}

// Lloyd's k-means on points x (n x 3) into k groups: seeds by farthest-point selection from the
// first point (deterministic), then `iters` rounds of assignment to the nearest centre and
// re-centring.  Returns the group of every point.
std::vector<int> kmeans_groups(const std::vector<double> &x, int k, int iters) {
  const size_t n = x.size() / 3;
  std::vector<int> g(n, 0);
  if (n == 0 || k <= 1) return g;
  k = (int)std::min<size_t>((size_t)k, n);
  std::vector<double> c(3 * (size_t)k), dmin(n, 1e300);
  auto d2 = [&](size_t i, const double *y) {
    const double a = x[3 * i] - y[0], b = x[3 * i + 1] - y[1], e = x[3 * i + 2] - y[2];
    return a * a + b * b + e * e;
  };
  size_t pick = 0;
  for (int q = 0; q < k; ++q) {
    for (int t = 0; t < 3; ++t) c[3 * q + t] = x[3 * pick + t];
    size_t far = 0;
    for (size_t i = 0; i < n; ++i) {
      dmin[i] = std::min(dmin[i], d2(i, &c[3 * q]));
      if (dmin[i] > dmin[far]) far = i;
    }
    pick = far;
  }
  std::vector<double> sum(3 * (size_t)k);
  std::vector<size_t> cnt(k);
  for (int it = 0; it < iters; ++it) {
    bool moved = false;
    for (size_t i = 0; i < n; ++i) {
      int best = 0;
      double bd = d2(i, &c[0]);
      for (int q = 1; q < k; ++q) {
        const double d = d2(i, &c[3 * q]);
        if (d < bd) {
          bd = d;
          best = q;
        }
      }
      moved |= best != g[i];
      g[i] = best;
    }
    std::fill(sum.begin(), sum.end(), 0.0);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (size_t i = 0; i < n; ++i) {
      for (int t = 0; t < 3; ++t) sum[3 * g[i] + t] += x[3 * i + t];
      ++cnt[g[i]];
    }
    for (int q = 0; q < k; ++q)
      if (cnt[q])
        for (int t = 0; t < 3; ++t) c[3 * q + t] = sum[3 * q + t] / (double)cnt[q];
    if (!moved && it > 0) break;
  }
  return g;
}

}  // namespace

struct hfx_plan {
  int n_cells = 0;
  std::vector<int> atom_off;  // n_cells + 1
  std::vector<int> nao, nabf, cell_of, local_of;
  std::vector<int> cell_natoms;
  hfx_thresholds th{};
  uint32_t stages = HFX_SCREEN_ALL;
  int precision = HFX_PREC_FP64;
  int scheduler = HFX_SCHED_LPT;
  hipStream_t stream = nullptr;
  bool poisoned = false;
  uint64_t max_bytes = 0, used_bytes = 0;
  std::vector<void *> allocs;

  // D pattern per cell
  std::vector<std::vector<int32_t>> d_row, d_col, d_R;
  std::vector<std::vector<int64_t>> d_inoff;  // caller offsets
  std::vector<std::vector<int64_t>> sig_off;  // compact offsets per cell (n+1)
  std::vector<int64_t> dbase;                 // first global D id per cell (n_cells+1)
  std::vector<int64_t> sbase;                 // first element in Sbuf per cell (n_cells+1)
  std::vector<long long *> d_inoff_dev;       // per cell, device copy of caller offsets
  std::vector<int32_t> d_row_g, d_col_g;      // global atom ids per global D id
  int32_t *d_row_dev = nullptr, *d_col_dev = nullptr;
  long long *dbase_dev = nullptr;
  double *gDmax_dev = nullptr;
  int64_t nD = 0;

  // items
  std::vector<Item> items;
  std::vector<int32_t> order;
  int64_t n_items = 0;

  DevPlan dp{};
  int n_slots = 0, rows_cap = 0, cols_cap = 0, ld3 = 0;
  long long wave_off = 0, wave_doubles = 0, wg_off = 0, ub_off = 0;
  int tier = 0;       // 0: FP64 block products; 1: bound-tiered FP32; 2: all FP32
  float tau = 0.0f;
  double tau64 = 0.0, tau_bf = 0.0;  // tier bounds as given or tuned (reported in the stats)
  int tile_r = 64;                   // column width of the terms-3/4 output blocks
  std::string tune_key;
  double *part = nullptr;  // energy partial sums
  // learned scheduler
  bool have_profile = false;
  int mlp_f = 0, mlp_h = 0, mlp_o = 0;
  std::vector<float> item_dist;    // |r_B + R - r_A| of every item (bohr)
  // real-space to k-space sum
  std::vector<int32_t> ptab_off_h;        // per cell: start of its n x n pattern table
  std::vector<int32_t> maxpc_h;           // per cell: most pattern entries of one atom pair
  std::vector<long long> nbasis_cell;     // per cell: basis size
  int32_t *bofs_dev = nullptr;            // per atom: first basis index within its cell
  float *item_dist_dev = nullptr;
  float *feat_musd = nullptr;  // normalisation for hfx_item_features
  float *mlp_params_dev = nullptr, *mlp_mu = nullptr, *mlp_sd = nullptr, *mlp_X = nullptr, *mlp_y = nullptr;
  std::vector<int32_t> lpt_order;
  int n_groups = 1;
  int part_blocks = 1024;
  double *staging = nullptr;  // pinned host staging for D
  size_t staging_n = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  // graph mode: one captured graph of the device-side build, valid for the pointers in gkey
  bool use_graph = false;
  hipStream_t gstream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t gev_in = nullptr, gev_out = nullptr;
  std::vector<const void *> gkey;

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    gkey.clear();
  }

  ~hfx_plan() {
    drop_graph();
    if (gstream) (void)hipStreamDestroy(gstream);
    if (gev_in) (void)hipEventDestroy(gev_in);
    if (gev_out) (void)hipEventDestroy(gev_out);
    for (void *p : allocs) (void)hipFree(p);
    if (staging) (void)hipHostFree(staging);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (ev2) (void)hipEventDestroy(ev2);
  }

  template <class T>
  hfx_status dalloc(T **p, size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (max_bytes && used_bytes + bytes > max_bytes)
      return fail(HFX_ERR_OOM, "device footprint would exceed max_device_bytes (%llu + %zu > %llu)",
                  (unsigned long long)used_bytes, bytes, (unsigned long long)max_bytes);
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(HFX_ERR_OOM, "hipMalloc of %zu bytes failed", bytes);
    }
    allocs.push_back(q);
    used_bytes += bytes;
    *p = (T *)q;
    return HFX_OK;
  }
  template <class T>
  hfx_status upload(T **p, const std::vector<T> &v) {
    hfx_status st = dalloc(p, v.size());
    if (st) return st;
    if (!v.empty() && hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
      return hip_fail("hipMemcpy");
    return HFX_OK;
  }
  hfx_status hip_fail(const char *what) {
    hipError_t e = hipGetLastError();
    poisoned = true;
    return fail(HFX_ERR_HIP, "%s failed: %s", what, hipGetErrorString(e));
  }
};

#define HIPCHK(plan, x)                                  \
  do {                                                   \
    if ((x) != hipSuccess) return (plan)->hip_fail(#x);  \
  } while (0)

namespace {

double max_abs(const double *x, int64_t n) {
  double m = 0;
  for (int64_t i = 0; i < n; ++i) m = std::max(m, std::fabs(x[i]));
  return m;
}

// host view of one cell's block set (data fetched to the host if it lives on the device)
struct HostBlocks {
  const hfx_blocks *b = nullptr;
  const double *data = nullptr;
  std::vector<double> copy;
};

hfx_status fetch(const hfx_blocks &b, const std::vector<int64_t> &sizes, HostBlocks &hb, const char *what) {
  hb.b = &b;
  if (b.n_blocks == 0) return HFX_OK;
  if (!b.data) return fail(HFX_ERR_ARG, "%s: data is NULL", what);
  if (!b.on_device) {
    hb.data = b.data;
    return HFX_OK;
  }
  int64_t end = 0;
  for (int64_t k = 0; k < b.n_blocks; ++k) end = std::max(end, b.off[k] + sizes[k]);
  hb.copy.resize((size_t)end);
  if (hipMemcpy(hb.copy.data(), b.data, (size_t)end * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HFX_ERR_HIP, "%s: copy of device data failed", what);
  }
  hb.data = hb.copy.data();
  return HFX_OK;
}

// a pointer the kernels dereference must be memory the GPU can reach (device, managed, or
// pinned host memory); plain pageable host memory is rejected before any launch
hfx_status check_gpu_ptr(const void *ptr, const char *what) {
  hipPointerAttribute_t at;
  const hipError_t e = hipPointerGetAttributes(&at, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HFX_ERR_ARG, "%s is not GPU-accessible memory (pass a device buffer)", what);
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged && at.type != hipMemoryTypeUnified &&
      !(at.type == hipMemoryTypeHost && at.devicePointer))
    return fail(HFX_ERR_ARG, "%s is not GPU-accessible memory (pass a device buffer)", what);
  return HFX_OK;
}

hfx_status check_blocks(const hfx_blocks &b, int n_atoms, const char *what, bool need_data) {
  if (b.n_blocks < 0) return fail(HFX_ERR_ARG, "%s: negative n_blocks", what);
  if (b.n_blocks > 0 && (!b.row || !b.col || !b.R || !b.off))
    return fail(HFX_ERR_ARG, "%s: NULL index array", what);
  if (need_data && b.n_blocks > 0 && !b.data) return fail(HFX_ERR_ARG, "%s: NULL data", what);
  for (int64_t k = 0; k < b.n_blocks; ++k) {
    if (b.row[k] < 0 || b.row[k] >= n_atoms || b.col[k] < 0 || b.col[k] >= n_atoms)
      return fail(HFX_ERR_SHAPE, "%s: block %lld has atom index out of range", what, (long long)k);
    if (b.off[k] < 0) return fail(HFX_ERR_SHAPE, "%s: block %lld has a negative offset", what, (long long)k);
    if (!r_ok(b.R + 3 * k)) return fail(HFX_ERR_UNSUPPORTED, "%s: lattice vector beyond +-%d", what, kRMax);
  }
  return HFX_OK;
}

}  // namespace

// Copy blocks (source, length) into dst at the packed offsets off[k] (increasing; the gaps are
// zero padding) through a pinned staging buffer of at most 256 MiB.
static hfx_status upload_packed(hfx_plan *p, double *dst, const std::vector<std::pair<const double *, int64_t>> &jobs,
                                const std::vector<long long> &off) {
  if (jobs.empty()) return HFX_OK;
  const int64_t total = off.back() + (jobs.back().second + 31) / 32 * 32;
  const int64_t cap = std::min<int64_t>(total, (int64_t)1 << 25);  // doubles
  double *pin = nullptr;
  if (hipHostMalloc((void **)&pin, (size_t)cap * sizeof(double)) != hipSuccess) return p->hip_fail("hipHostMalloc");
  hfx_status st = HFX_OK;
  int64_t d0 = 0, fill = 0;  // chunk start in dst, doubles staged
  auto flush = [&]() {
    if (fill > 0 && hipMemcpy(dst + d0, pin, (size_t)fill * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return false;
    return true;
  };
  for (size_t k = 0; k < jobs.size() && st == HFX_OK; ++k) {
    const int64_t n = jobs[k].second, padded = (n + 31) / 32 * 32;
    if (padded > cap) {
      st = fail(HFX_ERR_UNSUPPORTED, "a block of %lld elements exceeds the upload stage", (long long)n);
      break;
    }
    if (off[k] + padded - d0 > cap) {
      if (!flush()) {
        st = p->hip_fail("hipMemcpy");
        break;
      }
      d0 = off[k];
      fill = 0;
    }
    double *q = pin + (off[k] - d0);
    if (off[k] - d0 > fill) std::memset(pin + fill, 0, (size_t)(off[k] - d0 - fill) * sizeof(double));
    std::memcpy(q, jobs[k].first, (size_t)n * sizeof(double));
    std::memset(q + n, 0, (size_t)(padded - n) * sizeof(double));
    fill = off[k] - d0 + padded;
  }
  if (st == HFX_OK && !flush()) st = p->hip_fail("hipMemcpy");
  (void)hipHostFree(pin);
  return st;
}

extern "C" {

int32_t hfx_abi_version(void) { return HFX_ABI_VERSION; }

hfx_status hfx_tune_key(const hfx_plan *p, char *buf, int32_t len) {
  if (!p || !buf || len < 1) return fail(HFX_ERR_ARG, "NULL argument or empty buffer");
  if ((int64_t)p->tune_key.size() + 1 > len) return fail(HFX_ERR_ARG, "buffer of %d bytes too small", len);
  std::memcpy(buf, p->tune_key.c_str(), p->tune_key.size() + 1);
  return HFX_OK;
}
const char *hfx_last_error(void) { return g_err.c_str(); }

void hfx_plan_destroy(hfx_plan *plan) { delete plan; }

hfx_status hfx_plan_create(int32_t n_cells, const hfx_cell *cells, const hfx_blocks *C, const hfx_blocks *V,
                           const hfx_blocks *D_pattern, const hfx_thresholds *th, const hfx_options *opt,
                           hfx_plan **out) {
  if (!out) return fail(HFX_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n_cells < 1 || !cells || !C || !V || !D_pattern || !th)
    return fail(HFX_ERR_ARG, "n_cells < 1 or a NULL argument");
  const double eps[5] = {th->eps_C, th->eps_V, th->eps_D, th->eps_cs_eri, th->eps_cs_mat};
  for (double e : eps)
    if (!std::isfinite(e) || e < 0) return fail(HFX_ERR_ARG, "thresholds must be finite and >= 0");
  hfx_options o{};
  if (opt) o = *opt;
  if (o.precision < HFX_PREC_FP64 || o.precision > HFX_PREC_BF16X3)
    return fail(HFX_ERR_ARG, "unknown precision %d", o.precision);
  if (!std::isfinite(o.tier_tau) || !std::isfinite(o.tier_tau_bf))
    return fail(HFX_ERR_ARG, "tier_tau must be finite and >= 0 (or < 0 to take it from the tuning file)");
  if (o.tile_r != 0 && o.tile_r != 32 && o.tile_r != 64 && o.tile_r != 128)
    return fail(HFX_ERR_ARG, "tile_r must be 0, 32, 64 or 128");
  if (o.scheduler < HFX_SCHED_PLAN || o.scheduler > HFX_SCHED_KMEANS)
    return fail(HFX_ERR_ARG, "unknown scheduler %d", o.scheduler);
  if (o.scheduler == HFX_SCHED_MLP && !o.mlp_weights)
    return fail(HFX_ERR_ARG, "HFX_SCHED_MLP needs mlp_weights");

  auto plan = std::make_unique<hfx_plan>();
  hfx_plan *p = plan.get();
  p->n_cells = n_cells;
  p->th = *th;
  p->stages = o.stages ? o.stages : HFX_SCREEN_ALL;
  p->precision = o.precision;
  p->tier = o.precision == HFX_PREC_TIERED ? 1 : o.precision == HFX_PREC_FP32 ? 2 : o.precision == HFX_PREC_BF16X3 ? 3 : 0;
  p->scheduler = o.scheduler;
  p->stream = (hipStream_t)o.stream;
  p->max_bytes = o.max_device_bytes;
  const bool pre = p->stages & HFX_SCREEN_PRE;

  // ---- atoms
  p->atom_off.assign(n_cells + 1, 0);
  for (int c = 0; c < n_cells; ++c) {
    const hfx_cell &cl = cells[c];
    if (cl.n_atoms < 1 || !cl.pos || !cl.species || cl.n_species < 1 || !cl.sp)
      return fail(HFX_ERR_ARG, "cell %d: empty or NULL fields", c);
    const double *L = cl.lattice;
    const double det = L[0] * (L[4] * L[8] - L[5] * L[7]) - L[1] * (L[3] * L[8] - L[5] * L[6]) +
                       L[2] * (L[3] * L[7] - L[4] * L[6]);
    if (!std::isfinite(det) || std::fabs(det) < 1e-8) return fail(HFX_ERR_ARG, "cell %d: singular lattice", c);
    for (int s = 0; s < cl.n_species; ++s)
      if (cl.sp[s].n_ao < 1 || cl.sp[s].n_ao > main_maxn() || cl.sp[s].n_abf < 1 || cl.sp[s].n_abf > 512)
        return fail(HFX_ERR_UNSUPPORTED, "cell %d species %d: n_ao must be 1..%d and n_abf 1..512", c, s,
                    main_maxn());
    p->atom_off[c + 1] = p->atom_off[c] + cl.n_atoms;
    p->cell_natoms.push_back(cl.n_atoms);
    for (int i = 0; i < cl.n_atoms; ++i) {
      const int s = cl.species[i];
      if (s < 0 || s >= cl.n_species) return fail(HFX_ERR_SHAPE, "cell %d atom %d: species out of range", c, i);
      p->nao.push_back(cl.sp[s].n_ao);
      p->nabf.push_back(cl.sp[s].n_abf);
      p->cell_of.push_back(c);
      p->local_of.push_back(i);
    }
  }
  const int NA = p->atom_off[n_cells];

  // ---- autotuner's choices: the plan's key and, if a tuning file is given, its last entry for it
  {
    std::vector<std::pair<int, int>> spc;
    for (int a = 0; a < NA; ++a) spc.emplace_back(p->nao[a], p->nabf[a]);
    std::sort(spc.begin(), spc.end());
    spc.erase(std::unique(spc.begin(), spc.end()), spc.end());
    std::string k = "species=";
    for (size_t q = 0; q < spc.size(); ++q)
      k += (q ? "+" : "") + std::to_string(spc[q].first) + "x" + std::to_string(spc[q].second);
    char eb[64];
    std::snprintf(eb, sizeof(eb), " eps=%.3g prec=%s", th->eps_cs_mat,
                  o.precision == HFX_PREC_TIERED   ? "tiered"
                  : o.precision == HFX_PREC_FP32   ? "fp32"
                  : o.precision == HFX_PREC_BF16X3 ? "bf16x3"
                                                   : "fp64");
    p->tune_key = k + eb;
    int t_tile = 0;
    double t_tau = -1.0, t_tau_bf = -1.0;
    if (o.tuning_db) {
      FILE *fp = std::fopen(o.tuning_db, "r");
      if (!fp) return fail(HFX_ERR_ARG, "cannot open tuning_db '%s'", o.tuning_db);
      char line[1024];
      while (std::fgets(line, sizeof(line), fp)) {
        std::string ln(line);
        if (ln.rfind("hfxtune1 ", 0) != 0) continue;
        const size_t at = ln.find(" tile_r=");
        if (at == std::string::npos || ln.substr(9, at - 9) != p->tune_key) continue;
        int tr = 0;
        double ta = -1.0, tb = -1.0;
        if (std::sscanf(ln.c_str() + at, " tile_r=%d tier_tau=%lf tier_tau_bf=%lf", &tr, &ta, &tb) == 3) {
          t_tile = tr;
          t_tau = ta;
          t_tau_bf = tb;
        }
      }
      std::fclose(fp);
      if (t_tile != 0 && t_tile != 32 && t_tile != 64 && t_tile != 128)
        return fail(HFX_ERR_ARG, "tuning_db '%s': tile_r %d for '%s' is not 32, 64 or 128", o.tuning_db, t_tile,
                    p->tune_key.c_str());
    }
    p->tile_r = o.tile_r ? o.tile_r : (t_tile ? t_tile : 64);
    p->tau64 = o.tier_tau >= 0 ? o.tier_tau : t_tau;
    p->tau_bf = o.tier_tau_bf >= 0 ? o.tier_tau_bf : t_tau_bf;
    if ((o.precision == HFX_PREC_TIERED || o.precision == HFX_PREC_BF16X3) && p->tau64 < 0)
      return fail(HFX_ERR_ARG, "tier_tau < 0 needs a tuning_db entry for '%s'", p->tune_key.c_str());
    if (o.precision == HFX_PREC_BF16X3 && p->tau_bf < 0)
      return fail(HFX_ERR_ARG, "tier_tau_bf < 0 needs a tuning_db entry for '%s'", p->tune_key.c_str());
    p->tau64 = std::max(p->tau64, 0.0);
    p->tau_bf = std::max(p->tau_bf, 0.0);
    p->tau = (float)p->tau64;
  }

  // home set
  std::vector<uint8_t> is_home(NA, o.home_subset ? 0 : 1);
  if (o.home_subset) {
    if (o.n_home_subset < 0) return fail(HFX_ERR_ARG, "negative n_home_subset");
    for (int k = 0; k < o.n_home_subset; ++k) {
      const int a = o.home_subset[k];
      if (a < 0 || a >= NA) return fail(HFX_ERR_ARG, "home_subset entry %d out of range", a);
      is_home[a] = 1;
    }
  }

  // ---- C, V: validation, pre-screening, symmetry checks
  struct KC {
    int cell, k;
    double dist;
  };
  std::vector<std::vector<KC>> crow(NA);     // kept C blocks per global row atom
  std::vector<std::vector<int>> vkept(n_cells);
  std::vector<HostBlocks> hC(n_cells), hV(n_cells);
  std::vector<std::vector<int64_t>> csz(n_cells), vsz(n_cells);
  std::vector<std::unordered_map<Key, int, KeyHash>> vmap(n_cells), cmap(n_cells);
  std::vector<std::vector<uint8_t>> ckeep(n_cells), vkeep(n_cells);
  for (int c = 0; c < n_cells; ++c) {
    const hfx_cell &cl = cells[c];
    const int n = cl.n_atoms, a0 = p->atom_off[c];
    hfx_status st;
    if ((st = check_blocks(C[c], n, "C", true)) || (st = check_blocks(V[c], n, "V", true)) ||
        (st = check_blocks(D_pattern[c], n, "D_pattern", false)))
      return st;
    csz[c].resize(C[c].n_blocks);
    for (int64_t k = 0; k < C[c].n_blocks; ++k)
      csz[c][k] = (int64_t)p->nabf[a0 + C[c].row[k]] * p->nao[a0 + C[c].row[k]] * p->nao[a0 + C[c].col[k]];
    vsz[c].resize(V[c].n_blocks);
    for (int64_t k = 0; k < V[c].n_blocks; ++k)
      vsz[c][k] = (int64_t)p->nabf[a0 + V[c].row[k]] * p->nabf[a0 + V[c].col[k]];
    if ((st = fetch(C[c], csz[c], hC[c], "C")) || (st = fetch(V[c], vsz[c], hV[c], "V"))) return st;
    const double *cd = hC[c].data, *vd = hV[c].data;
    ckeep[c].assign(C[c].n_blocks, 0);
    for (int64_t k = 0; k < C[c].n_blocks; ++k) {
      const int32_t *R = C[c].R + 3 * k;
      Key key{C[c].row[k], C[c].col[k], pack_r(R[0], R[1], R[2])};
      if (!cmap[c].emplace(key, (int)k).second) return fail(HFX_ERR_SHAPE, "C: duplicate block %lld", (long long)k);
      const double *blk = cd + C[c].off[k];
      const double m = max_abs(blk, csz[c][k]);
      ckeep[c][k] = pre ? (m > th->eps_C) : 1;
      if (C[c].row[k] == C[c].col[k] && R[0] == 0 && R[1] == 0 && R[2] == 0) {
        const int P = p->nabf[a0 + C[c].row[k]], na = p->nao[a0 + C[c].row[k]];
        for (int al = 0; al < P; ++al)
          for (int a = 0; a < na; ++a)
            for (int f = a + 1; f < na; ++f)
              if (std::fabs(blk[(al * na + a) * na + f] - blk[(al * na + f) * na + a]) > 1e-12 * m)
                return fail(HFX_ERR_SYMMETRY, "C: on-site block of atom %d is not symmetric in its AO indices",
                            C[c].row[k]);
      }
    }
    vkeep[c].assign(V[c].n_blocks, 0);
    for (int64_t k = 0; k < V[c].n_blocks; ++k) {
      const int32_t *R = V[c].R + 3 * k;
      Key key{V[c].row[k], V[c].col[k], pack_r(R[0], R[1], R[2])};
      if (!vmap[c].emplace(key, (int)k).second) return fail(HFX_ERR_SHAPE, "V: duplicate block %lld", (long long)k);
      vkeep[c][k] = pre ? (max_abs(vd + V[c].off[k], vsz[c][k]) > th->eps_V) : 1;
    }
    for (int64_t k = 0; k < V[c].n_blocks; ++k) {
      const int32_t *R = V[c].R + 3 * k;
      auto it = vmap[c].find(Key{V[c].col[k], V[c].row[k], pack_r(-R[0], -R[1], -R[2])});
      if (it == vmap[c].end())
        return fail(HFX_ERR_SYMMETRY, "V: block (%d,%d,R) has no partner (col,row,-R)", V[c].row[k], V[c].col[k]);
      if (it->second < k) continue;
      const int PA = p->nabf[a0 + V[c].row[k]], PB = p->nabf[a0 + V[c].col[k]];
      const double *x = vd + V[c].off[k], *y = vd + V[c].off[it->second];
      const double m = std::max(max_abs(x, vsz[c][k]), 1e-300);
      for (int a = 0; a < PA; ++a)
        for (int b = 0; b < PB; ++b)
          if (std::fabs(x[a * PB + b] - y[b * PA + a]) > 1e-10 * m)
            return fail(HFX_ERR_SYMMETRY, "V(%d,%d,R) != V(%d,%d,-R)^T", V[c].row[k], V[c].col[k], V[c].col[k],
                        V[c].row[k]);
    }
    // kept C per row atom with the pair distance
    const double *L = cl.lattice;
    for (int64_t k = 0; k < C[c].n_blocks; ++k) {
      if (!ckeep[c][k]) continue;
      const int r = C[c].row[k], q = C[c].col[k];
      const int32_t *R = C[c].R + 3 * k;
      double d[3];
      for (int x = 0; x < 3; ++x)
        d[x] = cl.pos[3 * q + x] - cl.pos[3 * r + x] + R[0] * L[x] + R[1] * L[3 + x] + R[2] * L[6 + x];
      crow[a0 + r].push_back(KC{c, (int)k, std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])});
    }
    for (int64_t k = 0; k < V[c].n_blocks; ++k)
      if (vkeep[c][k]) vkept[c].push_back((int)k);
  }

  // ---- kept C in (row atom, distance) order
  std::vector<int32_t> c_start(NA + 1, 0), c_row, c_col, c_Rp;
  std::vector<long long> c_off;
  int64_t cdoubles = 0;
  int max_nbr = 0;
  std::vector<std::unordered_map<int, int>> cnew(n_cells);  // (cell, caller index) -> kept index
  for (int a = 0; a < NA; ++a) {
    auto &lst = crow[a];
    std::stable_sort(lst.begin(), lst.end(), [](const KC &x, const KC &y) { return x.dist < y.dist; });
    max_nbr = std::max(max_nbr, (int)lst.size());
    for (const KC &kc : lst) {
      const int c = kc.cell, k = kc.k, a0 = p->atom_off[c];
      cnew[c][k] = (int)c_row.size();
      c_row.push_back(a0 + C[c].row[k]);
      c_col.push_back(a0 + C[c].col[k]);
      const int32_t *R = C[c].R + 3 * k;
      c_Rp.push_back(pack_r(R[0], R[1], R[2]));
      c_off.push_back(cdoubles);
      cdoubles += (csz[c][k] + 31) / 32 * 32;
    }
    c_start[a + 1] = (int)c_row.size();
  }
  if (max_nbr > main_maxnb())
    return fail(HFX_ERR_UNSUPPORTED, "an atom has %d kept C blocks (limit %d)", max_nbr, main_maxnb());
  const int nC = (int)c_row.size();
  // kept C blocks in device order: (source, length); the device copy is packed by c_off
  std::vector<std::pair<const double *, int64_t>> cjobs;
  cjobs.reserve(nC);
  for (int a = 0; a < NA; ++a)
    for (const KC &kc : crow[a]) cjobs.emplace_back(hC[kc.cell].data + C[kc.cell].off[kc.k], csz[kc.cell][kc.k]);

  // ---- kept V
  std::vector<int32_t> v_row, v_col, v_Rp;
  std::vector<long long> v_off;
  std::vector<std::unordered_map<int, int>> vnew(n_cells);
  int64_t vdoubles = 0;
  for (int c = 0; c < n_cells; ++c) {
    const int a0 = p->atom_off[c];
    for (int k : vkept[c]) {
      vnew[c][k] = (int)v_row.size();
      v_row.push_back(a0 + V[c].row[k]);
      v_col.push_back(a0 + V[c].col[k]);
      const int32_t *R = V[c].R + 3 * k;
      v_Rp.push_back(pack_r(R[0], R[1], R[2]));
      v_off.push_back(vdoubles);
      vdoubles += (vsz[c][k] + 31) / 32 * 32;
    }
  }
  const int nV = (int)v_row.size();
  std::vector<std::pair<const double *, int64_t>> vjobs;
  vjobs.reserve(nV);
  for (int c = 0; c < n_cells; ++c)
    for (int k : vkept[c]) vjobs.emplace_back(hV[c].data + V[c].off[k], vsz[c][k]);

  // ---- CS-ERI sources per kept C block: C(F,A,-R), V(A,A,0), V(A,F,R), V(F,A,-R), V(F,F,0)
  std::vector<int32_t> qsrc((size_t)nC * 5, -1);
  {
    int kk = 0;
    for (int a = 0; a < NA; ++a)
      for (const KC &kc : crow[a]) {
        const int c = kc.cell, k = kc.k;
        const int A = C[c].row[k], F = C[c].col[k];
        const int32_t *R = C[c].R + 3 * k;
        const int32_t Rp = pack_r(R[0], R[1], R[2]), Rm = pack_r(-R[0], -R[1], -R[2]), R0 = pack_r(0, 0, 0);
        auto vfind = [&](int x, int y, int32_t rr) {
          auto it = vmap[c].find(Key{x, y, rr});
          if (it == vmap[c].end() || !vkeep[c][it->second]) return -1;
          return vnew[c][it->second];
        };
        int32_t *q = &qsrc[(size_t)kk * 5];
        if (A == F && Rp == R0) {
          q[0] = -2;
        } else {
          auto it = cmap[c].find(Key{F, A, Rm});
          q[0] = (it != cmap[c].end() && ckeep[c][it->second]) ? cnew[c][it->second] : -1;
          q[2] = vfind(A, F, Rp);
          q[3] = vfind(F, A, Rm);
          q[4] = vfind(F, F, R0);
        }
        q[1] = vfind(A, A, R0);
        ++kk;
      }
  }

  // ---- items: kept V blocks (A,B,R) with A a home atom; LPT cost = |N(A)| |N(B)|
  std::vector<double> cost, mid;
  for (int vb = 0; vb < nV; ++vb) {
    const int A = v_row[vb], B = v_col[vb];
    if (!is_home[A]) continue;
    const int nF = c_start[A + 1] - c_start[A], nG = c_start[B + 1] - c_start[B];
    if (nF == 0 || nG == 0) continue;
    p->items.push_back(Item{A, B, v_Rp[vb], vb});
    cost.push_back((double)nF * nG);
    {
      const hfx_cell &cl = cells[p->cell_of[A]];
      const int la = p->local_of[A], lb = p->local_of[B];
      const int32_t rp = v_Rp[vb];
      double d2 = 0.0;
      for (int x = 0; x < 3; ++x) {
        const double dx = cl.pos[3 * lb + x] - cl.pos[3 * la + x] + r_of(rp, 0) * cl.lattice[x] +
                          r_of(rp, 1) * cl.lattice[3 + x] + r_of(rp, 2) * cl.lattice[6 + x];
        d2 += dx * dx;
      }
      p->item_dist.push_back((float)std::sqrt(d2));
      // midpoint of the pair (cells kept apart by a large offset so that no group spans two)
      for (int x = 0; x < 3; ++x) {
        const double rb = cl.pos[3 * lb + x] + r_of(rp, 0) * cl.lattice[x] + r_of(rp, 1) * cl.lattice[3 + x] +
                          r_of(rp, 2) * cl.lattice[6 + x];
        mid.push_back(0.5 * (cl.pos[3 * la + x] + rb) + (x == 0 ? 1e5 * p->cell_of[A] : 0.0));
      }
    }
  }
  p->n_items = (int64_t)p->items.size();
  p->order.resize(p->n_items);
  std::iota(p->order.begin(), p->order.end(), 0);
  if (p->scheduler != HFX_SCHED_PLAN)  // learned and exact orders start from LPT until a build has run
    std::stable_sort(p->order.begin(), p->order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<int32_t> grp_start{0, (int32_t)p->n_items};
  if (p->scheduler == HFX_SCHED_KMEANS && p->n_items > 0) {
    // one group per XCD; inside a group the LPT order above
    const int k = 8;
    const std::vector<int> g = kmeans_groups(mid, k, 30);
    std::stable_sort(p->order.begin(), p->order.end(), [&](int x, int y) { return g[x] < g[y]; });
    grp_start.assign(k + 1, 0);
    for (int64_t i = 0; i < p->n_items; ++i) ++grp_start[g[i] + 1];
    for (int q = 0; q < k; ++q) grp_start[q + 1] += grp_start[q];
  }
  p->n_groups = (int)grp_start.size() - 1;

  // ---- D pattern: compact offsets, sorted lookup, pair tables
  p->d_row.resize(n_cells);
  p->d_col.resize(n_cells);
  p->d_R.resize(n_cells);
  p->d_inoff.resize(n_cells);
  p->sig_off.resize(n_cells);
  p->dbase.assign(n_cells + 1, 0);
  p->sbase.assign(n_cells + 1, 0);
  std::vector<long long> d_off_g;
  std::vector<int32_t> ptab_off(n_cells + 1, 0), pstart, pcount, dsort_R, dsort_id;
  for (int c = 0; c < n_cells; ++c) {
    const hfx_blocks &Dp = D_pattern[c];
    const int n = cells[c].n_atoms, a0 = p->atom_off[c];
    const int64_t nb = Dp.n_blocks;
    p->d_row[c].assign(Dp.row, Dp.row + nb);
    p->d_col[c].assign(Dp.col, Dp.col + nb);
    p->d_R[c].assign(Dp.R, Dp.R + 3 * nb);
    p->d_inoff[c].assign(Dp.off, Dp.off + nb);
    p->sig_off[c].assign(nb + 1, 0);
    for (int64_t k = 0; k < nb; ++k)
      p->sig_off[c][k + 1] = p->sig_off[c][k] + (int64_t)p->nao[a0 + Dp.row[k]] * p->nao[a0 + Dp.col[k]];
    p->dbase[c + 1] = p->dbase[c] + nb;
    p->sbase[c + 1] = p->sbase[c] + p->sig_off[c][nb];
    for (int64_t k = 0; k < nb; ++k) {
      d_off_g.push_back(p->sbase[c] + p->sig_off[c][k]);
      p->d_row_g.push_back(a0 + Dp.row[k]);
      p->d_col_g.push_back(a0 + Dp.col[k]);
    }
    std::vector<int64_t> idx(nb);
    std::iota(idx.begin(), idx.end(), 0);
    auto rp = [&](int64_t k) { return pack_r(Dp.R[3 * k], Dp.R[3 * k + 1], Dp.R[3 * k + 2]); };
    std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
      if (Dp.row[x] != Dp.row[y]) return Dp.row[x] < Dp.row[y];
      if (Dp.col[x] != Dp.col[y]) return Dp.col[x] < Dp.col[y];
      return rp(x) < rp(y);
    });
    ptab_off[c] = (int32_t)pstart.size();
    const size_t t0 = pstart.size();
    pstart.resize(t0 + (size_t)n * n, 0);
    pcount.resize(t0 + (size_t)n * n, 0);
    const int32_t sbase0 = (int32_t)dsort_R.size();
    for (int64_t q = 0; q < nb; ++q) {
      const int64_t k = idx[q];
      if (q > 0 && Dp.row[idx[q - 1]] == Dp.row[k] && Dp.col[idx[q - 1]] == Dp.col[k] && rp(idx[q - 1]) == rp(k))
        return fail(HFX_ERR_SHAPE, "D_pattern: duplicate block (%d,%d,R)", Dp.row[k], Dp.col[k]);
      const size_t t = t0 + (size_t)Dp.row[k] * n + Dp.col[k];
      if (pcount[t] == 0) pstart[t] = sbase0 + (int32_t)q;
      pcount[t]++;
      dsort_R.push_back(rp(k));
      dsort_id.push_back((int32_t)(p->dbase[c] + k));
    }
    p->maxpc_h.push_back(n ? *std::max_element(pcount.begin() + t0, pcount.end()) : 0);
  }
  p->nD = p->dbase[n_cells];
  d_off_g.push_back(p->sbase[n_cells]);
  p->ptab_off_h = ptab_off;
  if (p->nD > (1ll << 30)) return fail(HFX_ERR_UNSUPPORTED, "too many D blocks");

  // ---- per-slot scratch and LDS sizing
  int max_n = 0, max_p = 0, min_n = 1 << 30;
  for (int a = 0; a < NA; ++a) {
    max_n = std::max(max_n, p->nao[a]);
    max_p = std::max(max_p, p->nabf[a]);
    min_n = std::min(min_n, p->nao[a]);
  }
  int64_t gside_max = 0;
  for (int b = 0; b < NA; ++b) {
    int64_t s = 0, rows = 0, cols = 0;
    const int nb = p->nao[b];
    for (int q = c_start[b]; q < c_start[b + 1]; ++q) {
      const int64_t ng = p->nao[c_col[q]];
      s += (int64_t)max_p * nb * ng + (int64_t)max_p * max_n * ng + (int64_t)max_p * max_n * nb + nb * ng * ng +
           ng * nb * nb;
      rows += ng;
      cols += ng + nb;
    }
    gside_max = std::max(gside_max, s);
    p->rows_cap = std::max<int>(p->rows_cap, (int)rows);
    p->cols_cap = std::max<int>(p->cols_cap, (int)cols);
  }
  p->rows_cap = (p->rows_cap + 15) / 16 * 16 + 16;
  p->cols_cap = (p->cols_cap + 15) / 16 * 16 + 16;
  if (p->rows_cap > 255 * 64 || p->cols_cap > 16 * 64 * 8)
    return fail(HFX_ERR_UNSUPPORTED, "neighbour lists too long for the decode tables");
  const int64_t nfg = (int64_t)max_nbr * max_nbr;
  p->wave_off = (nfg + 1) / 2 + (nfg + 7) / 8 + nfg + (int64_t)max_nbr * max_n * max_n + gside_max + 64;
  p->wave_doubles = (16 * (int64_t)main_maxn() * main_maxn() + 64 + 31) / 32 * 32;
  p->wg_off = p->wave_off + (int64_t)main_nwaves() * p->wave_doubles;
  const int64_t wg_doubles = (int64_t)p->rows_cap * 64 + (int64_t)max_p * max_n * 64 + 64;
  p->ub_off = p->wg_off + wg_doubles;
  const int64_t slot = p->ub_off + ((p->tier == 1 || p->tier == 3) ? nfg : 0);  // two float bounds per (F,G)
  (void)min_n;
  p->ld3 = max_n;
  const size_t lds = main_static_lds() + main_dyn_lds(p->rows_cap, p->cols_cap, p->ld3);
  if (lds > 160 * 1024)
    return fail(HFX_ERR_UNSUPPORTED, "workgroup would need %zu bytes of LDS (limit 163840)", lds);

  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n_cu = prop.multiProcessorCount;
  }
  (void)hipGetLastError();
  p->n_slots = o.n_slots > 0 ? o.n_slots : n_cu;
  if (p->n_items > 0) p->n_slots = (int)std::min<int64_t>(p->n_slots, p->n_items);
  p->n_slots = std::max(p->n_slots, 1);

  // ---- device memory
  DevPlan &P = p->dp;
  hfx_status st;
  int32_t *d_nao = nullptr, *d_nabf = nullptr, *d_cellof = nullptr, *d_localof = nullptr, *d_cstart = nullptr,
          *d_ccol = nullptr, *d_cR = nullptr, *d_crow = nullptr, *d_vrow = nullptr, *d_vcol = nullptr,
          *d_qsrc = nullptr;
  long long *d_coff = nullptr, *d_voff = nullptr, *d_doff = nullptr;
  float *d_C32 = nullptr, *d_CT32 = nullptr;
  double *d_C = nullptr, *d_CT = nullptr, *d_V = nullptr, *d_gV = nullptr, *d_gD = nullptr, *d_D = nullptr,
         *d_S = nullptr, *d_scr = nullptr;
  CNorm *d_cn = nullptr;
  int32_t *d_ptoff = nullptr, *d_pstart = nullptr, *d_pcount = nullptr, *d_dsR = nullptr, *d_dsid = nullptr,
          *d_cellnat = nullptr, *d_order = nullptr, *d_drow = nullptr, *d_dcol = nullptr;
  uint8_t *d_keepD = nullptr;
  Item *d_items = nullptr;
  unsigned int *d_ticket = nullptr;
  int32_t *d_grp = nullptr;
  unsigned long long *d_cnt = nullptr;
  double *d_flops = nullptr;
  long long *d_icyc = nullptr;
  int *d_iunits = nullptr;
  double *d_icontrib = nullptr, *d_iflops = nullptr;
  std::vector<int32_t> ord32(p->order.begin(), p->order.end());
  if ((st = p->upload(&d_nao, p->nao)) || (st = p->upload(&d_nabf, p->nabf)) ||
      (st = p->upload(&d_cellof, p->cell_of)) || (st = p->upload(&d_localof, p->local_of)) ||
      (st = p->upload(&d_cstart, c_start)) || (st = p->upload(&d_ccol, c_col)) || (st = p->upload(&d_crow, c_row)) ||
      (st = p->upload(&d_cR, c_Rp)) || (st = p->upload(&d_coff, c_off)) || (st = p->dalloc(&d_C, (size_t)cdoubles)) ||
      (st = p->dalloc(&d_CT, (size_t)cdoubles)) ||
      (p->tier && ((st = p->dalloc(&d_C32, (size_t)cdoubles)) || (st = p->dalloc(&d_CT32, (size_t)cdoubles)))) ||
      (st = p->upload(&d_vrow, v_row)) || (st = p->upload(&d_vcol, v_col)) || (st = p->upload(&d_voff, v_off)) ||
      (st = p->dalloc(&d_V, (size_t)vdoubles)) || (st = p->upload(&d_qsrc, qsrc)) || (st = p->dalloc(&d_cn, nC)) ||
      (st = p->dalloc(&d_gV, nV)) || (st = p->upload(&d_ptoff, ptab_off)) || (st = p->upload(&d_pstart, pstart)) ||
      (st = p->upload(&d_pcount, pcount)) || (st = p->upload(&d_dsR, dsort_R)) ||
      (st = p->upload(&d_dsid, dsort_id)) || (st = p->upload(&d_cellnat, p->cell_natoms)) ||
      (st = p->upload(&d_doff, d_off_g)) || (st = p->upload(&d_drow, p->d_row_g)) ||
      (st = p->upload(&d_dcol, p->d_col_g)) || (st = p->dalloc(&d_D, (size_t)p->sbase[n_cells])) ||
      (st = p->dalloc(&d_S, (size_t)p->sbase[n_cells])) || (st = p->dalloc(&d_gD, (size_t)p->nD)) ||
      (st = p->dalloc(&d_keepD, (size_t)p->nD)) || (st = p->upload(&d_items, p->items)) ||
      (st = p->upload(&d_order, ord32)) || (st = p->dalloc(&d_ticket, kMaxGroups)) || (st = p->upload(&d_grp, grp_start)) || (st = p->dalloc(&d_cnt, kCntN)) ||
      (st = p->dalloc(&d_flops, 2)) || (st = p->dalloc(&d_icyc, (size_t)p->n_items)) || (st = p->dalloc(&d_iunits, (size_t)p->n_items * kItemUnits)) ||
      (st = p->dalloc(&d_icontrib, (size_t)p->n_items)) || (st = p->dalloc(&d_iflops, (size_t)p->n_items)) || (st = p->upload(&p->item_dist_dev, p->item_dist)) ||
      (st = p->dalloc(&d_scr, (size_t)p->n_slots * slot)) || (st = p->dalloc(&p->part, 2 * p->part_blocks)))
    return st;
  // block data through a pinned staging buffer, chunk by chunk: the host never holds a packed
  // copy of C or V (blocks that alias in the caller's arrays are read in place)
  if ((st = upload_packed(p, d_C, cjobs, c_off)) || (st = upload_packed(p, d_V, vjobs, v_off))) return st;
  {
    std::vector<long long> db(p->dbase.begin(), p->dbase.end());
    if ((st = p->upload(&p->dbase_dev, db)) || (st = p->dalloc(&p->gDmax_dev, n_cells))) return st;
  }
  p->d_row_dev = d_drow;
  p->d_col_dev = d_dcol;
  p->d_inoff_dev.resize(n_cells);
  for (int c = 0; c < n_cells; ++c) {
    std::vector<long long> tmp(p->d_inoff[c].begin(), p->d_inoff[c].end());
    if ((st = p->upload(&p->d_inoff_dev[c], tmp))) return st;
  }
  // zero-initialise D so that pattern blocks never hold garbage
  HIPCHK(p, launch_zero(d_D, p->sbase[n_cells], p->stream));

  P.n_atoms = NA;
  P.nao = d_nao;
  P.nabf = d_nabf;
  P.cell_of = d_cellof;
  P.local_of = d_localof;
  P.Cbuf = d_C;
  P.CTbuf = d_CT;
  P.C32 = d_C32;
  P.CT32 = d_CT32;
  P.c_off = d_coff;
  P.c_col = d_ccol;
  P.c_R = d_cR;
  P.c_norm = d_cn;
  P.c_start = d_cstart;
  P.Vbuf = d_V;
  P.v_off = d_voff;
  P.gV = d_gV;
  P.ptab_off = d_ptoff;
  P.pstart = d_pstart;
  P.pcount = d_pcount;
  P.dsort_R = d_dsR;
  P.dsort_id = d_dsid;
  P.cell_natoms = d_cellnat;
  P.d_off = d_doff;
  P.Dbuf = d_D;
  P.gD = d_gD;
  P.keepD = d_keepD;
  P.gDmax = p->gDmax_dev;
  P.Sbuf = d_S;
  P.items = d_items;
  P.order = d_order;
  P.n_items = (int32_t)p->n_items;
  P.eps_eri = th->eps_cs_eri;
  P.eps_mat = th->eps_cs_mat;
  P.stages = p->stages;
  P.scratch = d_scr;
  P.slot_doubles = slot;
  P.max_nbr = max_nbr;
  P.max_p = max_p;
  P.max_n = max_n;
  P.ticket = d_ticket;
  P.grp_start = d_grp;
  P.n_groups = p->n_groups;
  P.counters = d_cnt;
  P.flops = d_flops;
  P.item_cycles = d_icyc;
  P.item_units = d_iunits;
  P.item_contrib = d_icontrib;
  P.item_flops = d_iflops;

  {
    const void *must[] = {P.nao, P.nabf, P.cell_of, P.local_of, P.Cbuf, P.CTbuf, P.c_off, P.c_col, P.c_R, P.c_norm,
                          P.c_start, P.Vbuf, P.v_off, P.gV, P.ptab_off, P.pstart, P.pcount, P.dsort_R, P.dsort_id,
                          P.cell_natoms, P.d_off, P.Dbuf, P.gD, P.keepD, P.gDmax, P.Sbuf, P.items, P.order,
                          P.scratch, P.ticket, P.counters, P.flops, P.item_cycles, P.item_units, P.item_contrib,
                          P.item_flops,
                          p->item_dist_dev, p->part,
                          p->d_row_dev, p->d_col_dev, p->dbase_dev};
    for (const void *q : must)
      if (!q) return fail(HFX_ERR_OOM, "internal: a device buffer of the plan was not allocated");
    if (p->tier && (!P.C32 || !P.CT32))
      return fail(HFX_ERR_OOM, "internal: the FP32 operand copies were not allocated");
  }
  p->lpt_order = p->order;
  if (p->scheduler == HFX_SCHED_MLP) {
    FILE *fp = std::fopen(o.mlp_weights, "rb");
    if (!fp) return fail(HFX_ERR_ARG, "cannot open mlp_weights '%s'", o.mlp_weights);
    char magic[8];
    int32_t fh[3];
    bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "HFXMLP02", 8) == 0 &&
              std::fread(fh, sizeof(int32_t), 3, fp) == 3 && fh[0] == kItemFeatures && fh[1] >= 1 &&
              fh[1] <= mlp_max_h() && fh[2] >= 1 && fh[2] <= mlp_max_o();
    std::vector<float> mu, sd, prm;
    if (ok) {
      mu.resize(fh[0]);
      sd.resize(fh[0]);
      prm.resize((size_t)mlp_params(fh[0], fh[1], fh[2]));
      ok = std::fread(mu.data(), sizeof(float), mu.size(), fp) == mu.size() &&
           std::fread(sd.data(), sizeof(float), sd.size(), fp) == sd.size() &&
           std::fread(prm.data(), sizeof(float), prm.size(), fp) == prm.size();
    }
    std::fclose(fp);
    if (!ok) return fail(HFX_ERR_ARG, "mlp_weights '%s' is not a scheduler model file", o.mlp_weights);
    p->mlp_f = fh[0];
    p->mlp_h = fh[1];
    p->mlp_o = fh[2];
    if ((st = p->upload(&p->mlp_params_dev, prm)) || (st = p->upload(&p->mlp_mu, mu)) ||
        (st = p->upload(&p->mlp_sd, sd)) || (st = p->dalloc(&p->mlp_X, (size_t)p->n_items * fh[0])) ||
        (st = p->dalloc(&p->mlp_y, (size_t)p->n_items * fh[2])))
      return st;
  }
  // ---- plan-time kernels: C norms, CS-ERI factors, V norms
  HIPCHK(p, launch_cnorm(d_C, d_coff, d_crow, d_ccol, d_nao, d_nabf, nC, d_cn, p->stream));
  HIPCHK(p, launch_ctrans(d_C, d_coff, d_crow, d_ccol, d_nao, d_nabf, nC, d_CT, p->stream));
  if (p->tier) {
    HIPCHK(p, launch_to_f32(d_C, d_C32, (long long)cdoubles, p->stream));
    HIPCHK(p, launch_to_f32(d_CT, d_CT32, (long long)cdoubles, p->stream));
  }
  HIPCHK(p, launch_cq(d_C, d_coff, d_crow, d_ccol, d_V, d_voff, d_qsrc, d_nao, d_nabf, nC, d_cn, p->stream));
  HIPCHK(p, launch_vnorm(d_V, d_voff, d_vrow, d_vcol, d_nabf, nV, d_gV, p->stream));
  if (p->scheduler == HFX_SCHED_NORM && p->n_items > 0) {
    // norm-sorted packing: gV_AB * max_F g(C_AF) * max_G g(C_BG), largest first
    std::vector<double> gv(nV);
    std::vector<CNorm> cn(nC);
    HIPCHK(p, hipStreamSynchronize(p->stream));
    if (nV) HIPCHK(p, hipMemcpy(gv.data(), d_gV, gv.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (nC) HIPCHK(p, hipMemcpy(cn.data(), d_cn, cn.size() * sizeof(CNorm), hipMemcpyDeviceToHost));
    std::vector<double> gmax(NA, 0.0), key(p->n_items);
    for (int a = 0; a < NA; ++a)
      for (int q = c_start[a]; q < c_start[a + 1]; ++q) gmax[a] = std::max({gmax[a], cn[q].gA, cn[q].gF});
    for (int64_t i = 0; i < p->n_items; ++i) {
      const Item &it = p->items[i];
      key[i] = gv[it.vid] * gmax[it.A] * gmax[it.B];
    }
    std::vector<int32_t> ord(p->n_items);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return key[x] > key[y]; });
    p->order = ord;
    HIPCHK(p, hipMemcpy(d_order, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  HIPCHK(p, hipEventCreate(&p->ev0));
  HIPCHK(p, hipEventCreate(&p->ev1));
  HIPCHK(p, hipEventCreate(&p->ev2));
  p->use_graph = o.use_graph != 0;
  if (p->use_graph) {
    HIPCHK(p, hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking));
    HIPCHK(p, hipEventCreateWithFlags(&p->gev_in, hipEventDisableTiming));
    HIPCHK(p, hipEventCreateWithFlags(&p->gev_out, hipEventDisableTiming));
  }
  HIPCHK(p, hipStreamSynchronize(p->stream));
  *out = plan.release();
  return HFX_OK;
}

hfx_status hfx_sigma_layout(const hfx_plan *p, int32_t cell, hfx_blocks *layout, int64_t *n_elements) {
  if (!p || !layout) return fail(HFX_ERR_ARG, "NULL argument");
  if (cell < 0 || cell >= p->n_cells) return fail(HFX_ERR_ARG, "cell %d out of range", cell);
  layout->n_blocks = (int64_t)p->d_row[cell].size();
  layout->row = p->d_row[cell].data();
  layout->col = p->d_col[cell].data();
  layout->R = p->d_R[cell].data();
  layout->off = p->sig_off[cell].data();
  layout->data = nullptr;
  layout->on_device = 1;
  if (n_elements) *n_elements = p->sig_off[cell].back();
  return HFX_OK;
}

static hfx_status check_d(hfx_plan *p, const hfx_blocks *D) {
  if (!D) return fail(HFX_ERR_ARG, "D is NULL");
  for (int c = 0; c < p->n_cells; ++c) {
    const hfx_blocks &d = D[c];
    const int64_t nb = (int64_t)p->d_row[c].size();
    if (d.n_blocks != nb) return fail(HFX_ERR_STATE, "cell %d: D has %lld blocks, the plan's pattern %lld", c,
                                      (long long)d.n_blocks, (long long)nb);
    if (nb > 0 && !d.data) return fail(HFX_ERR_ARG, "cell %d: D data is NULL", c);
    if (d.off && std::memcmp(d.off, p->d_inoff[c].data(), nb * sizeof(int64_t)) != 0)
      return fail(HFX_ERR_STATE, "cell %d: D offsets differ from the plan's pattern", c);
    if (d.row && (std::memcmp(d.row, p->d_row[c].data(), nb * sizeof(int32_t)) != 0 ||
                  std::memcmp(d.col, p->d_col[c].data(), nb * sizeof(int32_t)) != 0 ||
                  std::memcmp(d.R, p->d_R[c].data(), 3 * nb * sizeof(int32_t)) != 0))
      return fail(HFX_ERR_STATE, "cell %d: D block structure differs from the plan's pattern", c);
  }
  return HFX_OK;
}

// copy D into the plan's compact layout on the plan stream (device D: one gather kernel per cell)
static hfx_status enqueue_d(hfx_plan *p, const hfx_blocks *D) {
  for (int c = 0; c < p->n_cells; ++c) {
    const hfx_blocks &d = D[c];
    const int64_t nb = (int64_t)p->d_row[c].size();
    if (nb == 0) continue;
    if (d.on_device) {
      HIPCHK(p, launch_dgather(d.data, p->d_inoff_dev[c], p->dp.d_off, (int)nb, p->dbase[c],
                               const_cast<double *>(p->dp.Dbuf), p->stream));
    } else {
      const size_t n = (size_t)(p->sbase[c + 1] - p->sbase[c]);
      if (p->staging_n < n) {
        if (p->staging) HIPCHK(p, hipHostFree(p->staging));
        p->staging = nullptr;
        HIPCHK(p, hipHostMalloc((void **)&p->staging, n * sizeof(double)));
        p->staging_n = n;
      }
      HIPCHK(p, hipStreamSynchronize(p->stream));
      for (int64_t k = 0; k < nb; ++k)
        std::memcpy(p->staging + p->sig_off[c][k], d.data + p->d_inoff[c][k],
                    (p->sig_off[c][k + 1] - p->sig_off[c][k]) * sizeof(double));
      HIPCHK(p, hipMemcpyAsync(const_cast<double *>(p->dp.Dbuf) + p->sbase[c], p->staging, n * sizeof(double),
                               hipMemcpyHostToDevice, p->stream));
      HIPCHK(p, hipStreamSynchronize(p->stream));
    }
  }
  return HFX_OK;
}

// the device-side build after D is staged: D screening, Sigma clear, the persistent kernel,
// Sigma copy-out; `eager` adds the timing events and sets the kernel's LDS attribute
static hfx_status enqueue_core(hfx_plan *p, double *const *sigma, bool eager) {
  DevPlan &P = p->dp;
  const long long ntot = p->sbase[p->n_cells];
  HIPCHK(p, launch_dprep(P.Dbuf, P.d_off, p->d_row_dev, p->d_col_dev, P.nao, (int)p->nD, p->th.eps_D,
                         (p->stages & HFX_SCREEN_PRE) ? 1 : 0, const_cast<double *>(P.gD),
                         const_cast<uint8_t *>(P.keepD), p->stream));
  HIPCHK(p, launch_dmax(P.gD, P.keepD, p->dbase_dev, p->gDmax_dev, p->n_cells, p->stream));
  HIPCHK(p, launch_zero(P.Sbuf, ntot, p->stream));
  HIPCHK(p, launch_reset(P.ticket, P.counters, P.flops, p->stream));
  if (eager) HIPCHK(p, hipEventRecord(p->ev1, p->stream));
  if (p->n_items > 0)
    HIPCHK(p, launch_main(P, p->n_slots, p->rows_cap, p->cols_cap, p->ld3, p->wave_off, p->wave_doubles, p->wg_off,
                          p->ub_off, p->tier, p->tau, (float)p->tau_bf, p->tile_r, p->stream, eager));
  if (eager) HIPCHK(p, hipEventRecord(p->ev2, p->stream));
  for (int c = 0; c < p->n_cells; ++c) {
    const size_t n = (size_t)(p->sbase[c + 1] - p->sbase[c]);
    if (n) HIPCHK(p, hipMemcpyAsync(sigma[c], P.Sbuf + p->sbase[c], n * sizeof(double), hipMemcpyDeviceToDevice,
                                    p->stream));
  }
  return HFX_OK;
}

// graph mode: capture D staging + enqueue_core once on the plan's own stream, replay it
static hfx_status graph_build(hfx_plan *p, const hfx_blocks *D, double *const *sigma) {
  std::vector<const void *> key;
  for (int c = 0; c < p->n_cells; ++c) {
    if (!p->d_row[c].empty() && !D[c].on_device)
      return fail(HFX_ERR_ARG, "graph mode needs D in device memory (cell %d is on the host)", c);
    key.push_back(D[c].data);
    key.push_back(sigma[c]);
  }
  if (!p->gexec || key != p->gkey) {
    p->drop_graph();
    HIPCHK(p, main_set_lds(p->rows_cap, p->cols_cap, p->ld3));
    hipStream_t user = p->stream;
    p->stream = p->gstream;
    HIPCHK(p, hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal));
    hfx_status st = enqueue_d(p, D);
    if (!st) st = enqueue_core(p, sigma, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->gstream, &g);
    p->stream = user;
    if (st || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return st ? st : p->hip_fail("hipStreamEndCapture");
    }
    p->graph = g;
    HIPCHK(p, hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
    p->gkey = key;
  }
  // no separate kernel timing inside the graph: ev1 = ev0
  HIPCHK(p, hipEventRecord(p->ev0, p->stream));
  HIPCHK(p, hipEventRecord(p->ev1, p->stream));
  HIPCHK(p, hipEventRecord(p->gev_in, p->stream));
  HIPCHK(p, hipStreamWaitEvent(p->gstream, p->gev_in, 0));
  HIPCHK(p, hipGraphLaunch(p->gexec, p->gstream));
  HIPCHK(p, hipEventRecord(p->gev_out, p->gstream));
  HIPCHK(p, hipStreamWaitEvent(p->stream, p->gev_out, 0));
  HIPCHK(p, hipEventRecord(p->ev2, p->stream));
  return HFX_OK;
}

hfx_status hfx_build(hfx_plan *p, const hfx_blocks *D, double *const *sigma, hfx_build_stats *stats) {
  if (!p) return fail(HFX_ERR_ARG, "plan is NULL");
  if (p->poisoned) return fail(HFX_ERR_STATE, "plan is poisoned by an earlier HIP error");
  if (!sigma) return fail(HFX_ERR_ARG, "sigma is NULL");
  for (int c = 0; c < p->n_cells; ++c)
    if (!sigma[c] && p->sbase[c + 1] > p->sbase[c]) return fail(HFX_ERR_ARG, "sigma[%d] is NULL", c);
  hfx_status st = check_d(p, D);
  if (st) return st;
  for (int c = 0; c < p->n_cells; ++c) {
    if (p->sbase[c + 1] == p->sbase[c]) continue;
    if ((st = check_gpu_ptr(sigma[c], "sigma[c]"))) return st;
    if (D[c].on_device && (st = check_gpu_ptr(D[c].data, "D data (on_device = 1)"))) return st;
  }
  DevPlan &P = p->dp;
  if (p->scheduler == HFX_SCHED_MLP && p->have_profile && p->n_items > 0) {
    // learned costs from the previous build's per-item counters; longest predicted first
    HIPCHK(p, mlp_launch_features(P.items, P.item_units, P.c_start, P.nao, P.nabf, p->item_dist_dev, P.cell_of,
                                  P.cell_natoms, p->n_items, p->mlp_mu, p->mlp_sd, p->mlp_X, p->stream));
    HIPCHK(p, mlp_launch_predict(p->mlp_params_dev, p->mlp_f, p->mlp_h, p->mlp_o, p->mlp_X, p->n_items, p->mlp_y,
                                 p->stream));
    std::vector<float> y((size_t)p->n_items * p->mlp_o), pred(p->n_items);
    HIPCHK(p, hipMemcpyAsync(y.data(), p->mlp_y, y.size() * sizeof(float), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
    for (int64_t i = 0; i < p->n_items; ++i) pred[i] = y[(size_t)i * p->mlp_o];  // output 0: log cost
    // longest predicted first, on a grid of 0.1 (predictions are standardised log times) so that
    // items of similar cost keep the plan order, which groups the items of one atom A and lets
    // concurrent workgroups share its C blocks in cache
    std::vector<int32_t> ord(p->n_items), bucket(p->n_items);
    for (int64_t i = 0; i < p->n_items; ++i) bucket[i] = (int32_t)std::floor(pred[i] * 10.0f);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return bucket[x] > bucket[y]; });
    HIPCHK(p, hipMemcpyAsync(const_cast<int32_t *>(P.order), ord.data(), ord.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
  }
  if (p->scheduler == HFX_SCHED_EXACT && p->have_profile && p->n_items > 0) {
    // exact costs: the contraction FLOPs each item did in the previous build, longest first
    std::vector<double> fl(p->n_items);
    HIPCHK(p, hipStreamSynchronize(p->stream));
    HIPCHK(p, hipMemcpy(fl.data(), P.item_flops, fl.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<int32_t> ord(p->n_items);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return fl[x] > fl[y]; });
    HIPCHK(p, hipMemcpyAsync(const_cast<int32_t *>(P.order), ord.data(), ord.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
  }
  if (p->use_graph) {
    if ((st = graph_build(p, D, sigma))) return st;
  } else {
    HIPCHK(p, hipEventRecord(p->ev0, p->stream));
    if ((st = enqueue_d(p, D)) || (st = enqueue_core(p, sigma, true))) return st;
  }
  p->have_profile = true;
  if (stats) {
    HIPCHK(p, hipStreamSynchronize(p->stream));
    unsigned long long cnt[kCntN];
    HIPCHK(p, hipMemcpy(cnt, P.counters, sizeof(cnt), hipMemcpyDeviceToHost));
    std::memset(stats, 0, sizeof(*stats));
    stats->candidates = (int64_t)cnt[kCntCandidates];
    stats->kept_cs_eri = (int64_t)cnt[kCntCsEri];
    for (int s = 0; s < 3; ++s)
      for (int t = 0; t < 4; ++t) stats->kept[s][t] = (int64_t)cnt[kCntKept + 4 * s + t];
    stats->items = p->n_items;
    stats->g_alive = (int64_t)cnt[kCntG];
    double fl[2];
    HIPCHK(p, hipMemcpy(fl, P.flops, sizeof(fl), hipMemcpyDeviceToHost));
    stats->flops_paper = fl[0];
    stats->flops_contract = fl[1];
    // matrix-core FLOPs issued (16x16x4 in FP64 or FP32: 2048 each; the split-BF16x3 products:
    // three 16x16x32 instructions, 16384 FLOPs each, per 16x16x32 FP32-equivalent product); the
    // precision shares of the contraction FLOPs are estimated by the shares of these products
    const double mR = (double)cnt[kCntMfmaR], mL = (double)cnt[kCntMfmaL];
    const double mR32 = (double)cnt[kCntMfmaR32], mL32 = (double)cnt[kCntMfmaL32];
    const double mRbf = (double)cnt[kCntMfmaRbf];
    const double eq_bf = mRbf * 16384.0 / 3.0;
    const double issued = 2048.0 * ((double)cnt[kCntMfmaY] + mR + mL + mR32 + mL32) + eq_bf;
    const double share32 = issued > 0 ? 2048.0 * (mR32 + mL32) / issued : 0.0;
    const double sharebf = issued > 0 ? eq_bf / issued : 0.0;
    stats->flops_tier[1] = fl[1] * share32;
    stats->flops_tier[2] = fl[1] * sharebf;
    stats->flops_tier[0] = fl[1] - stats->flops_tier[1] - stats->flops_tier[2];
    stats->mfma_flops[0] = 2048.0 * (double)cnt[kCntMfmaY];
    stats->mfma_flops[1] = 2048.0 * (mR + mR32) + 16384.0 * mRbf;
    stats->mfma_flops[2] = 2048.0 * (mL + mL32);
    stats->mfma_flops_fp32 = 2048.0 * (mR32 + mL32);
    stats->mfma_flops_bf16 = 16384.0 * mRbf;
    stats->tile_r = p->tile_r;
    stats->tier_tau = p->tier ? p->tau64 : 0.0;
    stats->tier_tau_bf = p->tier == 3 ? p->tau_bf : 0.0;
    float ms0 = 0, ms1 = 0;
    HIPCHK(p, hipEventElapsedTime(&ms0, p->ev0, p->ev2));
    HIPCHK(p, hipEventElapsedTime(&ms1, p->ev1, p->ev2));
    stats->ms_total = ms0;
    stats->ms_main = ms1;
    double tot = 0;
    for (int k = 0; k < 6; ++k) tot += (double)cnt[kCntPhase + k];
    for (int k = 0; k < 6; ++k) stats->phase_share[k] = tot > 0 ? (double)cnt[kCntPhase + k] / tot : 0.0;
  }
  return HFX_OK;
}

hfx_status hfx_energy(hfx_plan *p, const hfx_blocks *D, double *const *sigma, double *e_x) {
  if (!p || !sigma || !e_x) return fail(HFX_ERR_ARG, "NULL argument");
  if (p->poisoned) return fail(HFX_ERR_STATE, "plan is poisoned by an earlier HIP error");
  hfx_status st = check_d(p, D);
  if (st) return st;
  for (int c = 0; c < p->n_cells; ++c) {
    if (p->sbase[c + 1] == p->sbase[c]) continue;
    if ((st = check_gpu_ptr(sigma[c], "sigma[c]"))) return st;
    if (D[c].on_device && (st = check_gpu_ptr(D[c].data, "D data (on_device = 1)"))) return st;
  }
  if ((st = enqueue_d(p, D))) return st;
  std::vector<double> part(2 * p->part_blocks);
  for (int c = 0; c < p->n_cells; ++c) {
    const long long n = p->sbase[c + 1] - p->sbase[c];
    e_x[c] = 0.0;
    if (!n) continue;
    HIPCHK(p, launch_energy(p->dp.Dbuf + p->sbase[c], sigma[c], n, p->part, p->part_blocks, p->stream));
    HIPCHK(p, hipMemcpyAsync(part.data(), p->part, part.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
    // Neumaier summation of the double-double partials
    double s = 0, comp = 0;
    for (double v : part) {
      const double t = s + v;
      comp += std::fabs(s) >= std::fabs(v) ? (s - t) + v : (v - t) + s;
      s = t;
    }
    e_x[c] = 0.5 * (s + comp);
  }
  return HFX_OK;
}

hfx_status hfx_item_profile(hfx_plan *p, int64_t *n_items, int64_t *cycles, int64_t *units, double *contrib) {
  if (!p || !n_items) return fail(HFX_ERR_ARG, "NULL argument");
  *n_items = p->n_items;
  if (p->poisoned) return fail(HFX_ERR_STATE, "plan is poisoned by an earlier HIP error");
  HIPCHK(p, hipStreamSynchronize(p->stream));
  if (cycles && p->n_items) {
    std::vector<long long> c(p->n_items);
    HIPCHK(p, hipMemcpy(c.data(), p->dp.item_cycles, c.size() * sizeof(long long), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < p->n_items; ++i) cycles[i] = c[i];
  }
  if (units && p->n_items) {
    std::vector<int> u((size_t)kItemUnits * p->n_items);
    HIPCHK(p, hipMemcpy(u.data(), p->dp.item_units, u.size() * sizeof(int), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < u.size(); ++i) units[i] = u[i];
  }
  if (contrib && p->n_items)
    HIPCHK(p, hipMemcpy(contrib, p->dp.item_contrib, (size_t)p->n_items * sizeof(double), hipMemcpyDeviceToHost));
  return HFX_OK;
}

hfx_status hfx_item_features(hfx_plan *p, const float *mu, const float *sd, float *X) {
  if (!p || !mu || !sd || !X) return fail(HFX_ERR_ARG, "NULL argument");
  if (p->poisoned) return fail(HFX_ERR_STATE, "plan is poisoned by an earlier HIP error");
  if (!p->have_profile) return fail(HFX_ERR_STATE, "item features need a completed build");
  hfx_status st;
  if (!p->feat_musd && (st = p->dalloc(&p->feat_musd, 2 * kItemFeatures))) return st;
  float musd[2 * kItemFeatures];
  std::memcpy(musd, mu, kItemFeatures * sizeof(float));
  std::memcpy(musd + kItemFeatures, sd, kItemFeatures * sizeof(float));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  HIPCHK(p, hipMemcpy(p->feat_musd, musd, sizeof(musd), hipMemcpyHostToDevice));
  HIPCHK(p, mlp_launch_features(p->dp.items, p->dp.item_units, p->dp.c_start, p->dp.nao, p->dp.nabf,
                                p->item_dist_dev, p->dp.cell_of, p->dp.cell_natoms, p->n_items, p->feat_musd,
                                p->feat_musd + kItemFeatures, X, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  return HFX_OK;
}

// per atom its first basis index within its cell, per cell the basis size (once per plan)
static hfx_status ensure_basis_offsets(hfx_plan *p) {
  if (p->bofs_dev) return HFX_OK;
  std::vector<int32_t> b(p->nao.size());
  p->nbasis_cell.assign(p->n_cells, 0);
  for (int c = 0; c < p->n_cells; ++c) {
    int32_t o = 0;
    for (int a = p->atom_off[c]; a < p->atom_off[c + 1]; ++a) {
      b[a] = o;
      o += p->nao[a];
    }
    p->nbasis_cell[c] = o;
  }
  return p->upload(&p->bofs_dev, b);
}

hfx_status hfx_density_from_k(hfx_plan *p, int32_t cell, int32_t n_k, const double *kfrac, int32_t n_occ,
                              const double *ck, const double *occ, double *d) {
  if (!p) return fail(HFX_ERR_ARG, "plan is NULL");
  if (p->poisoned) return fail(HFX_ERR_STATE, "plan is poisoned by an earlier HIP error");
  if (cell < 0 || cell >= p->n_cells) return fail(HFX_ERR_ARG, "cell %d out of range (%d cells)", cell, p->n_cells);
  if (n_k < 1 || n_occ < 0) return fail(HFX_ERR_ARG, "need n_k >= 1 and n_occ >= 0");
  if (!kfrac || (n_occ > 0 && (!ck || !occ))) return fail(HFX_ERR_ARG, "NULL k-points, eigenvectors or occupations");
  if (!d && p->sbase[cell + 1] > p->sbase[cell]) return fail(HFX_ERR_ARG, "D is NULL");
  for (int64_t q = 0; q < 3 * (int64_t)n_k; ++q)
    if (!std::isfinite(kfrac[q])) return fail(HFX_ERR_ARG, "k-point %lld is not finite", (long long)(q / 3));
  hfx_status st;
  if (n_occ > 0 && ((st = check_gpu_ptr(ck, "ck")) || (st = check_gpu_ptr(occ, "occ")))) return st;
  if (d && (st = check_gpu_ptr(d, "d"))) return st;
  if ((st = ensure_basis_offsets(p))) return st;
  const int n = p->atom_off[cell + 1] - p->atom_off[cell], a0 = p->atom_off[cell];
  const long long nb = p->nbasis_cell[cell];
  const DevPlan &P = p->dp;
  KChunk kc;
  for (int32_t k0 = 0; k0 < n_k; k0 += kKChunk) {
    kc.n = std::min(kKChunk, n_k - k0);
    for (int q = 0; q < kc.n; ++q)
      for (int x = 0; x < 3; ++x) kc.k[q][x] = kfrac[3 * ((int64_t)k0 + q) + x];
    const size_t kofs = (size_t)k0 * (size_t)n_occ;
    HIPCHK(p, launch_density_from_k(n_occ ? ck + kofs * (size_t)nb * 2 : ck, n_occ ? occ + kofs : occ, n_occ, nb,
                                    P.d_off, p->sbase[cell], P.pstart + p->ptab_off_h[cell],
                                    P.pcount + p->ptab_off_h[cell], P.dsort_R, P.dsort_id, P.nao + a0,
                                    p->bofs_dev + a0, n, p->maxpc_h[cell], kc, 1.0 / n_k, k0 > 0, d, p->stream));
  }
  return HFX_OK;
}

hfx_status hfx_sigma_to_k(hfx_plan *p, int32_t cell, const double *sigma, int32_t n_k, const double *kfrac,
                          double *hk) {
  if (!p) return fail(HFX_ERR_ARG, "plan is NULL");
  if (p->poisoned) return fail(HFX_ERR_STATE, "plan is poisoned by an earlier HIP error");
  if (cell < 0 || cell >= p->n_cells) return fail(HFX_ERR_ARG, "cell %d out of range (%d cells)", cell, p->n_cells);
  if (n_k < 0) return fail(HFX_ERR_ARG, "n_k < 0");
  if (n_k == 0) return HFX_OK;
  if (!kfrac || !hk) return fail(HFX_ERR_ARG, "NULL k-points or output");
  if (!sigma && p->sbase[cell + 1] > p->sbase[cell]) return fail(HFX_ERR_ARG, "sigma is NULL");
  for (int64_t q = 0; q < 3 * (int64_t)n_k; ++q)
    if (!std::isfinite(kfrac[q])) return fail(HFX_ERR_ARG, "k-point %lld is not finite", (long long)(q / 3));
  hfx_status st;
  if ((sigma && (st = check_gpu_ptr(sigma, "sigma"))) || (st = check_gpu_ptr(hk, "hk"))) return st;
  if ((st = ensure_basis_offsets(p))) return st;
  const int n = p->atom_off[cell + 1] - p->atom_off[cell], a0 = p->atom_off[cell];
  const long long nb = p->nbasis_cell[cell];
  const DevPlan &P = p->dp;
  KChunk kc;
  for (int32_t k0 = 0; k0 < n_k; k0 += kKChunk) {
    kc.n = std::min(kKChunk, n_k - k0);
    for (int q = 0; q < kc.n; ++q)
      for (int x = 0; x < 3; ++x) kc.k[q][x] = kfrac[3 * ((int64_t)k0 + q) + x];
    HIPCHK(p, launch_sigma_to_k(sigma, P.d_off, p->sbase[cell], P.pstart + p->ptab_off_h[cell],
                                P.pcount + p->ptab_off_h[cell], P.dsort_R, P.dsort_id, P.nao + a0, p->bofs_dev + a0, n,
                                nb, kc, hk + (size_t)k0 * (size_t)nb * (size_t)nb * 2, p->stream));
  }
  return HFX_OK;
}

int64_t hfx_mlp_n_params(int32_t n_in, int32_t n_hidden, int32_t n_out) { return mlp_params(n_in, n_hidden, n_out); }

static hfx_status mlp_check(int32_t n_in, int32_t n_hidden, int32_t n_out, const void *a, const void *b, int64_t n) {
  if (n_in < 1 || n_in > mlp_max_f() || n_hidden < 1 || n_hidden > mlp_max_h() || n_out < 1 || n_out > mlp_max_o())
    return fail(HFX_ERR_ARG, "n_in must be 1..%d, n_hidden 1..%d and n_out 1..%d", mlp_max_f(), mlp_max_h(),
                mlp_max_o());
  if (!a || !b || n < 0) return fail(HFX_ERR_ARG, "NULL argument or negative n");
  return HFX_OK;
}

hfx_status hfx_mlp_predict(int32_t n_in, int32_t n_hidden, int32_t n_out, const float *params, const float *X,
                           int64_t n, float *y, void *stream) {
  hfx_status st = mlp_check(n_in, n_hidden, n_out, params, X, n);
  if (st) return st;
  if (!y) return fail(HFX_ERR_ARG, "NULL output");
  if (mlp_launch_predict(params, n_in, n_hidden, n_out, X, n, y, (hipStream_t)stream) != hipSuccess)
    return fail(HFX_ERR_HIP, "predict launch failed: %s", hipGetErrorString(hipGetLastError()));
  return HFX_OK;
}

hfx_status hfx_mlp_loss_grad(int32_t n_in, int32_t n_hidden, int32_t n_out, const float *params, const float *X,
                             const float *t, int64_t n, float *grad, float *loss, void *stream) {
  hfx_status st = mlp_check(n_in, n_hidden, n_out, params, X, n);
  if (st) return st;
  if (!t || !grad || !loss) return fail(HFX_ERR_ARG, "NULL argument");
  if (mlp_launch_grad(params, n_in, n_hidden, n_out, X, t, n, grad, loss, (hipStream_t)stream) != hipSuccess)
    return fail(HFX_ERR_HIP, "gradient launch failed: %s", hipGetErrorString(hipGetLastError()));
  return HFX_OK;
}

hfx_status hfx_mlp_train(int32_t n_in, int32_t n_hidden, int32_t n_out, float *params, const float *X, const float *t,
                         int64_t n, int32_t epochs, float lr, float *loss_host, void *stream) {
  hfx_status st = mlp_check(n_in, n_hidden, n_out, params, X, n);
  if (st) return st;
  if (!t || epochs < 0 || !(lr > 0)) return fail(HFX_ERR_ARG, "bad targets, epochs or learning rate");
  const int np = (int)mlp_params(n_in, n_hidden, n_out);
  hipStream_t s = (hipStream_t)stream;
  float *buf = nullptr;
  if (hipMalloc(&buf, sizeof(float) * (3 * (size_t)np + 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(HFX_ERR_OOM, "optimizer state allocation failed");
  }
  float *G = buf, *m = buf + np, *v = buf + 2 * np, *loss = buf + 3 * np;
  hipError_t e = hipMemsetAsync(m, 0, sizeof(float) * 2 * np, s);
  for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
    e = mlp_launch_grad(params, n_in, n_hidden, n_out, X, t, n, G, loss, s);
    if (e == hipSuccess && loss_host) e = hipMemcpyAsync(loss_host + ep, loss, sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = mlp_launch_adam(params, G, m, v, np, lr, ep + 1, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(HFX_ERR_HIP, "training failed: %s", hipGetErrorString(e));
  return HFX_OK;
}

hfx_status hfx_mlp_train_static(int32_t n_in, int32_t n_hidden, int32_t n_out, float *params, const float *X,
                                const float *t, int64_t n, int32_t epochs, float lr, float *loss_dev, void *stream) {
  hfx_status st = mlp_check(n_in, n_hidden, n_out, params, X, n);
  if (st) return st;
  if (!t || epochs < 0 || !(lr > 0)) return fail(HFX_ERR_ARG, "bad targets, epochs or learning rate");
  if (mlp_params(n_in, n_hidden, n_out) > mlp_scratch_max_params())
    return fail(HFX_ERR_ARG, "model has %lld parameters, the static optimizer state holds %d",
                (long long)mlp_params(n_in, n_hidden, n_out), mlp_scratch_max_params());
  if ((st = check_gpu_ptr(params, "params")) || (n > 0 && (st = check_gpu_ptr(X, "X"))) ||
      (n > 0 && (st = check_gpu_ptr(t, "t"))) || (loss_dev && epochs > 0 && (st = check_gpu_ptr(loss_dev, "loss_dev"))))
    return st;
  const hipError_t e = mlp_train_static(n_in, n_hidden, n_out, params, X, t, n, epochs, lr, loss_dev, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HFX_ERR_HIP, "training launch failed: %s", hipGetErrorString(e));
  }
  return HFX_OK;
}

hfx_status hfx_mfma_peak(int32_t kind, void *stream, double *tflops, double *sclk_mhz) {
  if (kind < 0 || kind > 2 || !tflops) return fail(HFX_ERR_ARG, "kind must be 0, 1 or 2 and tflops non-NULL");
  int dev = 0, wall_khz = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return fail(HFX_ERR_HIP, "device query: %s", hipGetErrorString(e));
  const int n_cu = prop.multiProcessorCount;
  const int iters = kind == 0 ? 32768 : kind == 1 ? 65536 : 131072;  // about 50 ms each at 2.4 GHz
  double *out = nullptr;
  long long *clk = nullptr;
  const size_t n_out = (size_t)n_cu * mfma_peak_blocks_per_cu() * mfma_peak_threads();
  if (hipMalloc((void **)&out, n_out * sizeof(double)) != hipSuccess ||
      hipMalloc((void **)&clk, 2 * sizeof(long long)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(out);
    return fail(HFX_ERR_OOM, "probe buffers");
  }
  float ms = 0.f;
  double flops = 0.0;
  long long hclk[2] = {0, 0};
  e = mfma_peak_run(kind, n_cu, iters, out, clk, (hipStream_t)stream, &ms, &flops);
  if (e == hipSuccess) e = hipMemcpy(hclk, clk, sizeof(hclk), hipMemcpyDeviceToHost);
  (void)hipFree(out);
  (void)hipFree(clk);
  if (e != hipSuccess) return fail(HFX_ERR_HIP, "matrix-core probe: %s", hipGetErrorString(e));
  if (!(ms > 0.f)) return fail(HFX_ERR_HIP, "matrix-core probe: no elapsed time");
  *tflops = flops / ((double)ms * 1e-3) / 1e12;
  if (sclk_mhz)
    *sclk_mhz = (wall_khz > 0 && hclk[1] > 0) ? (double)hclk[0] / ((double)hclk[1] / ((double)wall_khz * 1e3)) / 1e6
                                               : 0.0;
  return HFX_OK;
}

}  // extern "C"
