// Host runtime of libisrsgn.so: the C ABI of include/isrsgn.h -- argument validation,
// handle and device-memory ownership, the plan cache, and the order of kernel launches.
#include "isrsgn.h"
#include "isrsgn_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

using namespace isrsgn;

// Device scratch of isrsgn_snr_noalloc: the plan's device copy and the whole workspace of a call
// live here instead of memory the library allocates.  Every GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side stand-in: kernels get the
// per-device address that hipGetSymbolAddress returns (scratch_address below), never the name.
static __device__ __align__(256) unsigned char scratch[ISRSGN_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(ISRSGN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846;

// Device allocation; ISRSGN_FAIL_ALLOC=1 in the environment makes it fail (tests of ENOMEM).
bool dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  const char* inj = std::getenv("ISRSGN_FAIL_ALLOC");
  if (inj && inj[0] == '1') return false;
  if (bytes == 0) bytes = 16;
  return hipMalloc(p, bytes) == hipSuccess;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { if (p) (void)hipFree(p); }
  bool ensure(size_t n) {
    if (n <= bytes && p) return true;
    if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
    if (!dev_alloc(&p, n)) { p = nullptr; return false; }
    bytes = n;
    return true;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

uint64_t fnv1a(const void* data, size_t n, uint64_t h) {
  const unsigned char* c = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  return h;
}

struct GraphEntry {
  int kind;
  double snr_trx;
  hipGraphExec_t exec;
};

// A validated channel plan resident on the device, with its workspace.
struct PlanEntry {
  uint64_t key = 0;
  std::vector<int> off;
  std::vector<double> f, R;
  int n_batch = 0, n_total = 0, nmax = 0, nli = 1;
  int64_t n_tiles = 0;
  DevBuf d_off, d_toff, d_f, d_R, d_alpha, d_aeff, d_gamma, d_cr, d_fpt, d_wpt;
  // workspace
  DevBuf abar, zm, dz, hdz32, step_rec, ell64, lt32, ellL, tiles, pnli, snr, counter;
  DevBuf lr_a, lr_b, lr_rank, lr_res, lr_b64;  // low-rank form of lt32 (FP32 form, ODE profile)
  DevBuf states, state_off, lam, gG, gL, gLL, gP, coef;
  bool grad_ready = false;
  // FP32 gradient: row batches whose per-node S fits the store (see ensure_grad_workspace)
  struct RowBatch { unsigned int t0, t1; int g0, g1; };
  std::vector<RowBatch> batches;
  DevBuf s_store;
  bool store_ok = false;
  // graph mode: owned inputs/outputs and the instantiated graphs
  DevBuf g_P, g_nf, g_a, g_b, g_c, g_thr;
  std::vector<GraphEntry> graphs;
  ~PlanEntry() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
  }
  PlanView view() const {
    PlanView v;
    v.n_batch = n_batch;
    v.n_total = n_total;
    v.nli = nli;
    v.n_tiles = n_tiles;
    v.off = d_off.as<int>();
    v.toff = d_toff.as<int64_t>();
    v.f = d_f.as<double>();
    v.R = d_R.as<double>();
    v.alpha = d_alpha.as<double>();
    v.aeff = d_aeff.as<double>();
    v.gamma = d_gamma.as<double>();
    v.cr = d_cr.as<double>();
    v.fpt = d_fpt.as<double>();
    v.wpt = d_wpt.as<double>();
    return v;
  }
  Work work() const {
    Work w{};
    w.abar = abar.as<double>();
    w.zm = zm.as<double>();
    w.dz = dz.as<double>();
    w.hdz32 = hdz32.as<float>();
    w.step_rec = step_rec.as<double>();
    w.ell64 = ell64.as<double>();
    w.lt32 = lt32.as<float2>();
    w.lr_a = lr_a.as<float>();
    w.lr_b = lr_b.as<float2>();
    w.lr_rank = lr_rank.as<int>();
    w.lr_res = lr_res.as<double>();
    w.lr_b64 = lr_b64.as<double>();
    w.ellL = ellL.as<double>();
    w.tiles = tiles.as<double>();
    w.pnli = pnli.as<double>();
    w.snr = snr.as<double>();
    w.counter = counter.as<unsigned int>();
    w.nodes = reinterpret_cast<unsigned long long*>(counter.as<char>() + 32);
    w.states = states.as<double>();
    w.state_off = state_off.as<int64_t>();
    w.lam = lam.as<double>();
    w.gG = gG.as<double>();
    w.gL = gL.as<double>();
    w.gLL = gLL.as<double>();
    w.gP = gP.as<double>();
    return w;
  }
};

}  // namespace

struct isrsgn_fibre {
  int last_variant = -1;
  int last_grad_batches = 0;  // row batches of the last gradient (0: S recomputed)
  bool graph = false;
  hipStream_t cap_stream = nullptr;
  isrsgn_fibre_desc desc{};
  std::vector<double> tab_f, tab_alpha, tab_aeff;
  DevBuf d_tab_f, d_tab_alpha, d_tab_aeff;
  FibreParams fp{};
  int device = 0, n_cu = 0;
  size_t lds_max = 65536;  // LDS one workgroup may allocate on this device
  std::vector<std::unique_ptr<PlanEntry>> plans;  // most recent first
  // input checks (isrsgn_set_checks): a validation kernel's verdict copied to pinned host memory
  bool checks = true;
  DevBuf d_check;
  int* h_check = nullptr;
  // an event recorded at the end of every call, one per stream used: isrsgn_destroy waits on these
  std::vector<std::pair<hipStream_t, hipEvent_t>> done;
  // timing (isrsgn_set_timing): events recorded by the last call and the stage spans between them
  bool timing = false;
  std::vector<hipEvent_t> evs;
  int ev_count = 0;
  struct Span { int stage, a, b; };
  std::vector<Span> spans;
};

namespace {

bool is_fin(double x) { return std::isfinite(x); }

int validate_desc(const isrsgn_fibre_desc* d) {
  if (!d) return fail(ISRSGN_EINVAL, "desc is NULL");
  if (!(d->span_m > 0) || !is_fin(d->span_m)) return fail(ISRSGN_EINVAL, "span_m must be > 0");
  if (!(d->f_ref_hz > 0) || !is_fin(d->f_ref_hz)) return fail(ISRSGN_EINVAL, "f_ref_hz must be > 0");
  if (d->n_tab < 1 || !d->tab_f_hz || !d->alpha_per_m || !d->aeff_m2)
    return fail(ISRSGN_EINVAL, "need n_tab >= 1 and the three table arrays");
  for (int q = 0; q < d->n_tab; ++q) {
    if (!is_fin(d->tab_f_hz[q]) || !(d->alpha_per_m[q] >= 0) || !(d->aeff_m2[q] > 0))
      return fail(ISRSGN_EINVAL, "table entry %d: need finite f, alpha >= 0, aeff > 0", q);
    if (q > 0 && !(d->tab_f_hz[q] > d->tab_f_hz[q - 1])) return fail(ISRSGN_EINVAL, "tab_f_hz must ascend");
  }
  if (d->profile != ISRSGN_PROFILE_CLOSED_FORM && d->profile != ISRSGN_PROFILE_ODE)
    return fail(ISRSGN_EUNSUPPORTED, "profile %d is not provided", d->profile);
  if (d->profile == ISRSGN_PROFILE_CLOSED_FORM && d->n_tab != 1)
    return fail(ISRSGN_EINVAL, "the closed-form profile needs uniform loss and area (n_tab == 1)");
  if (d->precision != ISRSGN_FP32 && d->precision != ISRSGN_FP64)
    return fail(ISRSGN_EUNSUPPORTED, "precision %d is not provided", d->precision);
  if (d->n_steps < 1 || d->n_steps > 4096) return fail(ISRSGN_EINVAL, "n_steps must be in 1..4096");
  if (d->grid_s < 2 || d->grid_s > kMaxGridS) return fail(ISRSGN_EINVAL, "grid_s must be in 2..%d", kMaxGridS);
  if (d->grid_v < 2 || d->grid_v > 65536) return fail(ISRSGN_EINVAL, "grid_v must be in 2..65536");
  if (!(d->s_decades > 0) || d->s_decades > 40) return fail(ISRSGN_EINVAL, "s_decades must be in (0, 40]");
  if (d->ode_sub < 1 || d->ode_sub > 64) return fail(ISRSGN_EINVAL, "ode_sub must be in 1..64");
  if (d->n_spans < 1 || d->n_spans > 100000) return fail(ISRSGN_EINVAL, "n_spans must be in 1..100000");
  if (!(d->rolloff >= 0.0 && d->rolloff <= 1.0)) return fail(ISRSGN_EINVAL, "rolloff must be in [0, 1]");
  if (d->nli_points < 1 || d->nli_points > 64) return fail(ISRSGN_EINVAL, "nli_points must be in 1..64");
  if (!(d->cr_per_w_m_hz >= 0) || !(d->aeff_ref_m2 > 0)) return fail(ISRSGN_EINVAL, "need cr >= 0 and aeff_ref > 0");
  if (!(d->n2_m2_per_w >= 0) || !(d->gamma_const_per_w_m >= 0)) return fail(ISRSGN_EINVAL, "need n2, gamma >= 0");
  const double vals[] = {d->beta2, d->beta3, d->beta4, d->d_s_per_m2, d->s_s_per_m3, d->sdot_s_per_m4,
                         d->raman_cutoff_hz};
  for (double v : vals)
    if (!is_fin(v)) return fail(ISRSGN_EINVAL, "dispersion and cut-off must be finite");
  return ISRSGN_OK;
}

// Address of this device's copy of `scratch`, looked up once per device (with that device current)
// and kept; isrsgn_setup_fibre calls it for the handle's device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ISRSGN_EDEVICE, "device %d is beyond the %d the library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return hip_fail(err, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(ISRSGN_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ISRSGN_OK;
}

// Plan rules of include/isrsgn.h; *ntiles_out and *nmax_out get the tile count and the largest plan.
int validate_plan(const isrsgn_fibre* h, const isrsgn_plan* p, int64_t* ntiles_out, int* nmax_out) {
  if (!p) return fail(ISRSGN_EINVAL, "plan is NULL");
  if (p->n_batch < 1 || !p->ch_offsets || !p->f_hz || !p->rs_hz) return fail(ISRSGN_EINVAL, "plan needs n_batch >= 1 and arrays");
  if (p->ch_offsets[0] != 0) return fail(ISRSGN_EINVAL, "ch_offsets[0] must be 0");
  int64_t ntiles = 0;
  int nmax = 0;
  for (int b = 0; b < p->n_batch; ++b) {
    const int lo = p->ch_offsets[b], hi = p->ch_offsets[b + 1], n = hi - lo;
    if (n < 1 || n > kMaxChannels) return fail(ISRSGN_EINVAL, "plan %d has %d channels (need 1..%d)", b, n, kMaxChannels);
    for (int c = lo; c < hi; ++c) {
      if (!is_fin(p->f_hz[c]) || !(p->f_hz[c] > 0) || !is_fin(p->rs_hz[c]) || !(p->rs_hz[c] > 0))
        return fail(ISRSGN_EINVAL, "channel %d: need finite f > 0 and symbol rate > 0", c);
      if (c > lo && p->f_hz[c] - p->f_hz[c - 1] < 0.5 * (1.0 + h->fp.rolloff) * (p->rs_hz[c] + p->rs_hz[c - 1]))
        return fail(ISRSGN_EINVAL, "plan %d: channels %d and %d are unsorted or their spectra overlap", b, c - 1 - lo,
                    c - lo);
    }
    ntiles += (int64_t)n * n * h->fp.nli;
    if (n > nmax) nmax = n;
  }
  if (ntiles >= (int64_t)1 << 31) return fail(ISRSGN_EINVAL, "more than 2^31 tiles in one call");
  if (tile_lds(h->fp, nmax) > h->lds_max)
    return fail(ISRSGN_EINVAL, "a plan of %d channels with grid_s %d and %d steps exceeds the %zu B workgroup LDS",
                nmax, h->desc.grid_s, h->desc.n_steps, h->lds_max);
  *ntiles_out = ntiles;
  *nmax_out = nmax;
  return ISRSGN_OK;
}

// Validates a plan and returns its resident copy (uploading and setting it up on a miss).
int get_plan(isrsgn_fibre* h, const isrsgn_plan* p, hipStream_t s, PlanEntry** out) {
  int64_t ntiles = 0;
  int nmax = 0;
  if (const int rc = validate_plan(h, p, &ntiles, &nmax)) return rc;
  const int total = p->ch_offsets[p->n_batch];
  uint64_t key = 1469598103934665603ull;
  key = fnv1a(p->ch_offsets, sizeof(int) * (p->n_batch + 1), key);
  key = fnv1a(p->f_hz, sizeof(double) * total, key);
  key = fnv1a(p->rs_hz, sizeof(double) * total, key);
  for (size_t q = 0; q < h->plans.size(); ++q) {
    PlanEntry* e = h->plans[q].get();
    if (e->key == key && e->n_batch == p->n_batch && e->n_total == total &&
        std::memcmp(e->off.data(), p->ch_offsets, sizeof(int) * (p->n_batch + 1)) == 0 &&
        std::memcmp(e->f.data(), p->f_hz, sizeof(double) * total) == 0 &&
        std::memcmp(e->R.data(), p->rs_hz, sizeof(double) * total) == 0) {
      if (q) std::swap(h->plans[0], h->plans[q]);
      *out = h->plans[0].get();
      return ISRSGN_OK;
    }
  }
  auto e = std::make_unique<PlanEntry>();
  e->key = key;
  e->off.assign(p->ch_offsets, p->ch_offsets + p->n_batch + 1);
  e->f.assign(p->f_hz, p->f_hz + total);
  e->R.assign(p->rs_hz, p->rs_hz + total);
  e->n_batch = p->n_batch;
  e->n_total = total;
  e->n_tiles = ntiles;
  e->nmax = nmax;
  e->nli = h->fp.nli;
  std::vector<int64_t> toff(p->n_batch + 1, 0);
  for (int b = 0; b < p->n_batch; ++b) {
    const int64_t n = p->ch_offsets[b + 1] - p->ch_offsets[b];
    toff[b + 1] = toff[b] + n * n * e->nli;
  }
  const int M = h->desc.n_steps;
  const size_t nt = (size_t)total, nb = (size_t)p->n_batch;
  bool ok = e->d_off.ensure(sizeof(int) * (nb + 1)) && e->d_toff.ensure(sizeof(int64_t) * (nb + 1)) &&
            e->d_f.ensure(8 * nt) && e->d_R.ensure(8 * nt) && e->d_alpha.ensure(8 * nt) && e->d_aeff.ensure(8 * nt) &&
            e->d_gamma.ensure(8 * nt) && e->d_cr.ensure(8 * nt) && e->d_fpt.ensure(8 * nt * e->nli) &&
            e->d_wpt.ensure(8 * nt * e->nli) && e->abar.ensure(8 * nb) &&
            e->zm.ensure(8 * nb * M) && e->dz.ensure(8 * nb * M) && e->hdz32.ensure(4 * nb * M) && e->step_rec.ensure(32 * nb * M) &&
            e->ell64.ensure(8 * nt * M) && e->ellL.ensure(8 * nt) && e->tiles.ensure(8 * (size_t)ntiles) &&
            e->pnli.ensure(8 * nt) && e->snr.ensure(8 * nt) && e->counter.ensure(64) &&
            (h->desc.precision != ISRSGN_FP32 || e->lt32.ensure(8 * nt * M)) &&
            (h->desc.precision != ISRSGN_FP32 || h->desc.profile != ISRSGN_PROFILE_ODE ||
             (e->lr_a.ensure(4 * nb * M * kRank) && e->lr_b.ensure(8 * nt * kRank) && e->lr_rank.ensure(4 * nb) &&
              e->lr_res.ensure(8 * nt * M) && e->lr_b64.ensure(8 * nt * kRank)));
  if (!ok) return fail(ISRSGN_ENOMEM, "device allocation failed for a plan of %d channels", total);
  hipError_t err;
  if ((err = hipMemcpy(e->d_off.p, p->ch_offsets, sizeof(int) * (nb + 1), hipMemcpyHostToDevice)) != hipSuccess ||
      (err = hipMemcpy(e->d_toff.p, toff.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice)) != hipSuccess ||
      (err = hipMemcpy(e->d_f.p, p->f_hz, 8 * nt, hipMemcpyHostToDevice)) != hipSuccess ||
      (err = hipMemcpy(e->d_R.p, p->rs_hz, 8 * nt, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(err, "plan upload");
  if ((err = launch_channel_setup(e->view(), h->fp, s)) != hipSuccess) return hip_fail(err, "channel setup");
  if (h->plans.size() >= 4) h->plans.pop_back();
  h->plans.insert(h->plans.begin(), std::move(e));
  *out = h->plans[0].get();
  return ISRSGN_OK;
}

// Timing: each call starts a new list of events; stages 0 steps + profile, 1 forward tiles,
// 2 reductions, 3 adjoint tiles, 4 rest of the gradient (summed over row batches).
void begin_timing(isrsgn_fibre* h) {
  h->ev_count = 0;
  h->spans.clear();
}

int mark(isrsgn_fibre* h, hipStream_t s) {
  if (!h->timing) return -1;
  if (h->ev_count == (int)h->evs.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    h->evs.push_back(e);
  }
  if (hipEventRecord(h->evs[h->ev_count], s) != hipSuccess) return -1;
  return h->ev_count++;
}

void add_span(isrsgn_fibre* h, int stage, int a, int b) {
  if (a >= 0 && b >= 0) h->spans.push_back({stage, a, b});
}

int tile_grid(isrsgn_fibre* h, int nmax, int variant, int64_t tiles) {
  const int per_cu = tile_blocks_per_cu(h->fp, nmax, variant);
  int64_t g = (int64_t)per_cu * h->n_cu;
  if (g > tiles) g = tiles;
  return (int)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------- autotuner
// The forward tile kernel comes in variants (step-loop unroll x minimum occupancy).  On the
// first call for a discretisation the library times every variant on a slice of the real
// tile list (the middle tiles, a few per CU) and keeps the fastest; the choice is cached per
// process and, when ISRSGN_TUNE_CACHE names a file, across processes.  ISRSGN_TILE_VARIANT
// forces a variant.
struct TuneKey {
  int prec, profile, gs, gv, M;
  bool operator==(const TuneKey& o) const {
    return prec == o.prec && profile == o.profile && gs == o.gs && gv == o.gv && M == o.M;
  }
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, int>> g_tuned;
bool g_tune_file_read = false;

void read_tune_file() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = std::getenv("ISRSGN_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  TuneKey k;
  int v;
  while (std::fscanf(f, "fwd %d %d %d %d %d %d\n", &k.prec, &k.profile, &k.gs, &k.gv, &k.M, &v) == 6)
    if (v >= 0 && v < kTileVariants) g_tuned.emplace_back(k, v);
  std::fclose(f);
}

int pick_variant(isrsgn_fibre* h, PlanEntry* e, const double* P, const Work& w, const PlanView& pv, hipStream_t s,
                 int* out) {
  const char* force = std::getenv("ISRSGN_TILE_VARIANT");
  if (force && *force) {
    const int v = std::atoi(force);
    *out = v >= 0 && v < kTileVariants ? v : 0;
    return ISRSGN_OK;
  }
  const TuneKey key{h->desc.precision, h->desc.profile, h->desc.grid_s, h->desc.grid_v, h->desc.n_steps};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    read_tune_file();
    for (auto& kv : g_tuned)
      if (kv.first == key) { *out = kv.second; return ISRSGN_OK; }
  }
  // enough tiles that every workgroup of the persistent grid takes a dozen or more: with only a
  // few each, the tail of the launch dominates and the ranking differs from the full pass
  const int64_t trial = std::min<int64_t>(e->n_tiles, std::max<int64_t>(64, 48 * (int64_t)h->n_cu));
  const unsigned int begin = (unsigned int)((e->n_tiles - trial) / 2), end = begin + (unsigned int)trial;
  hipEvent_t a, b;
  hipError_t err;
  if ((err = hipEventCreate(&a)) != hipSuccess) return hip_fail(err, "autotune events");
  if ((err = hipEventCreate(&b)) != hipSuccess) { (void)hipEventDestroy(a); return hip_fail(err, "autotune events"); }
  int best = 0;
  float best_ms = 1e30f;
  for (int v = 0; v < kTileVariants && err == hipSuccess; ++v) {
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
      (void)hipEventRecord(a, s);
      err = launch_tiles(pv, h->fp, P, w, e->nmax, tile_grid(h, e->nmax, v, trial), v, begin, end, true, s);
      (void)hipEventRecord(b, s);
      if (err == hipSuccess) err = hipEventSynchronize(b);
      float ms = 0.f;
      if (err == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess && rep == 1 && ms < best_ms) {
        best_ms = ms;
        best = v;
      }
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (err != hipSuccess) return hip_fail(err, "autotune");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.emplace_back(key, best);
  const char* path = std::getenv("ISRSGN_TUNE_CACHE");
  if (path && *path) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f, "fwd %d %d %d %d %d %d\n", key.prec, key.profile, key.gs, key.gv, key.M, best);
      std::fclose(f);
    }
  }
  *out = best;
  return ISRSGN_OK;
}

// Steps, profile and the tile-kernel variant: the first timing stage.  *mk gets its end mark.
int prologue(isrsgn_fibre* h, PlanEntry* e, const double* P, const Work& w, bool keep_states, hipStream_t s,
             int* variant, int* mk) {
  begin_timing(h);
  const int m0 = mark(h, s);
  const PlanView pv = e->view();
  hipError_t err;
  if ((err = launch_steps(pv, h->fp, P, w, s)) != hipSuccess) return hip_fail(err, "steps");
  if ((err = launch_profile(pv, h->fp, P, w, keep_states, s)) != hipSuccess) return hip_fail(err, "profile");
  const int rc = pick_variant(h, e, P, w, pv, s, variant);
  if (rc) return rc;
  h->last_variant = *variant;
  *mk = mark(h, s);
  add_span(h, 0, m0, *mk);
  return ISRSGN_OK;
}

// Steps, profile, pair integrals and reduction.  Outputs may be NULL.  *mk gets the end mark.
int forward(isrsgn_fibre* h, PlanEntry* e, const double* P, const double* nf, double snr_trx, double* eta,
            double* pnli, double* tiles_out, double* snr, double* thr, bool keep_states, hipStream_t s, int* mk) {
  Work w = e->work();
  if (tiles_out && e->nli == 1) w.tiles = tiles_out;  // else folded over the COI points below
  const PlanView pv = e->view();
  int variant = 0, m1 = -1;
  const int rc = prologue(h, e, P, w, keep_states, s, &variant, &m1);
  if (rc) return rc;
  hipError_t err;
  if ((err = launch_tiles(pv, h->fp, P, w, e->nmax, tile_grid(h, e->nmax, variant, e->n_tiles), variant, 0u,
                          (unsigned int)e->n_tiles, true, s)) != hipSuccess)
    return hip_fail(err, "pair integrals");
  const int m2 = mark(h, s);
  add_span(h, 1, m1, m2);
  if ((err = launch_reduce(pv, h->fp, P, nf, snr_trx, w, eta, pnli, snr, thr, s)) != hipSuccess)
    return hip_fail(err, "reduction");
  if (tiles_out && e->nli > 1 && (err = launch_fold_tiles(pv, w, tiles_out, s)) != hipSuccess)
    return hip_fail(err, "tile output");
  *mk = mark(h, s);
  add_span(h, 2, m2, *mk);
  return ISRSGN_OK;
}

enum { kEta = 0, kSnr = 1, kGrad = 2 };

int ensure_grad_workspace(isrsgn_fibre* h, PlanEntry* e) {
  const int M = h->desc.n_steps;
  if (adjoint_lds(e->nmax, h->desc.grid_s, M, h->desc.precision) > h->lds_max)
    return fail(ISRSGN_EUNSUPPORTED, "the adjoint of a %d-channel plan with grid_s %d and %d steps exceeds %zu B LDS",
                e->nmax, h->desc.grid_s, M, h->lds_max);
  if (e->grad_ready) return ISRSGN_OK;
  const size_t nt = (size_t)e->n_total, nb = (size_t)e->n_batch;
  std::vector<int64_t> soff(nb + 1, 0);
  const bool ode = h->desc.profile == ISRSGN_PROFILE_ODE;
  for (size_t b = 0; b < nb; ++b) {
    const int64_t n = e->off[b + 1] - e->off[b];
    soff[b + 1] = soff[b] + (ode ? ((int64_t)M * 2 * h->desc.ode_sub + 1) * n : 0);
  }
  bool ok = e->lam.ensure(8 * nt) && e->gG.ensure(8 * nt) && e->gL.ensure(8 * nt * M) && e->gLL.ensure(8 * nt) &&
            e->gP.ensure(8 * nt) && e->coef.ensure(8 * 8 * nb * (M + 1)) && e->state_off.ensure(8 * (nb + 1)) &&
            e->states.ensure(8 * (size_t)soff[nb]);
  if (!ok) return fail(ISRSGN_ENOMEM, "device allocation failed for the adjoint workspace");
  hipError_t err = hipMemcpy(e->state_off.p, soff.data(), 8 * (nb + 1), hipMemcpyHostToDevice);
  if (err != hipSuccess) return hip_fail(err, "state offsets");
  // The forward pass keeps S of every node for the adjoint (8 B per node in the FP32 form, 16 B
  // in the FP64 form), one batch of complete COI rows at a time (a row's SNR, and so its
  // upstream weight, needs only that row).  The store is bounded by ISRSGN_STORE_MB (0 disables
  // it), by default half of the device memory free at this point (one batch for a 589-channel
  // plan at G=128 on an idle 288 GB device); when a row does not fit or the allocation fails, the
  // adjoint recomputes S instead.
  e->batches.clear();
  e->store_ok = false;
  const char* env = std::getenv("ISRSGN_STORE_MB");
  double store_mb = 0.0;
  if (env && *env) {
    store_mb = std::atof(env);
  } else {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
      store_mb = 0.5 * (double)free_b / 1048576.0;
    } else {
      (void)hipGetLastError();
      store_mb = 16384.0;
    }
  }
  const int64_t per_tile = (int64_t)3 * h->desc.grid_s * h->desc.grid_v *
                           (int64_t)(h->desc.precision == ISRSGN_FP32 ? sizeof(float2) : sizeof(double2));
  const int64_t max_tiles = store_mb > 0 ? (int64_t)(store_mb * 1048576.0 / (double)per_tile) : 0;
  bool fits = max_tiles > 0;
  for (size_t b = 0; b < nb && fits; ++b) fits = (int64_t)(e->off[b + 1] - e->off[b]) * e->nli <= max_tiles;
  if (fits) {
    int64_t t = 0, t0 = 0, cnt = 0, most = 0;
    int g0 = 0;
    for (size_t b = 0; b < nb; ++b) {
      const int64_t row = (int64_t)(e->off[b + 1] - e->off[b]) * e->nli;  // tiles of one COI row
      for (int i = 0; i < e->off[b + 1] - e->off[b]; ++i) {
        const int g = e->off[b] + i;  // global channel of this COI row
        if (cnt + row > max_tiles && cnt > 0) {
          e->batches.push_back({(unsigned int)t0, (unsigned int)t, g0, g});
          most = std::max(most, cnt);
          t0 = t;
          g0 = g;
          cnt = 0;
        }
        t += row;
        cnt += row;
      }
    }
    e->batches.push_back({(unsigned int)t0, (unsigned int)t, g0, e->n_total});
    most = std::max(most, cnt);
    e->store_ok = e->s_store.ensure((size_t)(most * per_tile));
    if (!e->store_ok) e->batches.clear();
  }
  e->grad_ready = true;
  return ISRSGN_OK;
}

// Gradient with the per-node S store: per row batch, forward tiles (keeping S), the batch's
// P_NLI, SNR and upstream weights, then its adjoint tiles; then throughput and profile adjoint.
int enqueue_grad_stored(isrsgn_fibre* h, PlanEntry* e, const double* P, const double* nf, double snr_trx,
                        double* snr, double* thr, double* dthr, hipStream_t s) {
  Work w = e->work();
  const PlanView pv = e->view();
  int variant = 0, mk = -1;
  const int rc = prologue(h, e, P, w, h->desc.profile == ISRSGN_PROFILE_ODE, s, &variant, &mk);
  if (rc) return rc;
  w.s_store = e->s_store.p;
  hipError_t err = launch_grad_init(pv, h->fp, w, s);
  if (err != hipSuccess) return hip_fail(err, "adjoint");
  const int adj_per_cu = adjoint_blocks_per_cu(h->fp, e->nmax, true, h->lds_max);
  bool first = true;
  for (const auto& bt : e->batches) {
    const int64_t nt = (int64_t)bt.t1 - bt.t0;
    if ((err = launch_tiles(pv, h->fp, P, w, e->nmax, tile_grid(h, e->nmax, variant, nt), variant, bt.t0, bt.t1, first,
                            s)) != hipSuccess)
      return hip_fail(err, "pair integrals");
    first = false;
    const int ma = mark(h, s);
    add_span(h, 1, mk, ma);
    // the SNR goes to the workspace (w.snr) and reaches the caller after the last batch
    err = launch_reduce_rows(pv, h->fp, P, nf, snr_trx, w, nullptr, nullptr, nullptr, bt.g0, bt.g1, s);
    if (err == hipSuccess) err = launch_grad_rows(pv, h->fp, P, nf, snr_trx, w, bt.g0, bt.g1, s);
    if (err != hipSuccess) return hip_fail(err, "reduction");
    const int mb = mark(h, s);
    add_span(h, 2, ma, mb);
    const int64_t grid = std::min<int64_t>((int64_t)adj_per_cu * h->n_cu, nt);
    if ((err = launch_adjoint_tiles(pv, h->fp, P, w, e->nmax, (int)(grid < 1 ? 1 : grid), bt.t0, bt.t1, true,
                                    h->lds_max, s)) != hipSuccess)
      return hip_fail(err, "adjoint");
    mk = mark(h, s);
    add_span(h, 3, mb, mk);
  }
  if ((err = launch_throughput(pv, P, w, thr, s)) != hipSuccess) return hip_fail(err, "throughput");
  if ((err = launch_copy(snr, w.snr, pv.n_total, s)) != hipSuccess) return hip_fail(err, "snr");
  if ((err = launch_grad_finish(pv, h->fp, P, w, e->coef.as<double>(), dthr, s)) != hipSuccess)
    return hip_fail(err, "adjoint");
  add_span(h, 4, mk, mark(h, s));
  return ISRSGN_OK;
}

// The whole sequence of one call, enqueued on s.
int enqueue_call(isrsgn_fibre* h, PlanEntry* e, int kind, const double* P, const double* nf, double snr_trx,
                 double* eta, double* pnli, double* tiles, double* snr, double* thr, double* dthr, hipStream_t s) {
  if (kind == kGrad) h->last_grad_batches = e->store_ok ? (int)e->batches.size() : 0;
  if (kind == kGrad && e->store_ok) return enqueue_grad_stored(h, e, P, nf, snr_trx, snr, thr, dthr, s);
  int m3 = -1;
  int rc = forward(h, e, P, nf, snr_trx, eta, pnli, tiles, snr, thr,
                   kind == kGrad && h->desc.profile == ISRSGN_PROFILE_ODE, s, &m3);
  if (rc || kind != kGrad) return rc;
  const int per_cu = adjoint_blocks_per_cu(h->fp, e->nmax, false, h->lds_max);
  int64_t grid = (int64_t)per_cu * h->n_cu;
  if (grid > e->n_tiles) grid = e->n_tiles;
  const Work w = e->work();
  const PlanView pv = e->view();
  hipError_t err = launch_grad_init(pv, h->fp, w, s);
  if (err == hipSuccess) err = launch_grad_rows(pv, h->fp, P, nf, snr_trx, w, 0, pv.n_total, s);
  if (err == hipSuccess)
    err = launch_adjoint_tiles(pv, h->fp, P, w, e->nmax, (int)(grid < 1 ? 1 : grid), 0u, (unsigned int)e->n_tiles,
                               false, h->lds_max, s);
  if (err != hipSuccess) return hip_fail(err, "adjoint");
  const int m4 = mark(h, s);
  add_span(h, 3, m3, m4);
  if ((err = launch_grad_finish(pv, h->fp, P, w, e->coef.as<double>(), dthr, s)) != hipSuccess)
    return hip_fail(err, "adjoint");
  add_span(h, 4, m4, mark(h, s));
  return ISRSGN_OK;
}

bool variant_known(isrsgn_fibre* h) {
  const char* force = std::getenv("ISRSGN_TILE_VARIANT");
  if (force && *force) return true;
  const TuneKey key{h->desc.precision, h->desc.profile, h->desc.grid_s, h->desc.grid_v, h->desc.n_steps};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  read_tune_file();
  for (auto& kv : g_tuned)
    if (kv.first == key) return true;
  return false;
}

// Graph mode: the call's kernels are captured once per (plan, kind, transceiver SNR) on the
// handle's capture stream, working on buffers the plan owns; each call then copies the inputs
// in, launches the graph on the caller's stream and copies the outputs out (all kernels: no
// memset or memcpy nodes).
int run_graph(isrsgn_fibre* h, PlanEntry* e, int kind, const double* P, const double* nf, double snr_trx,
              double* eta, double* pnli, double* tiles, double* snr, double* thr, double* dthr, hipStream_t s) {
  const size_t nt = (size_t)e->n_total, nb = (size_t)e->n_batch;
  if (!e->g_P.ensure(8 * nt) || !e->g_nf.ensure(8 * nt) || !e->g_a.ensure(8 * nt) || !e->g_b.ensure(8 * nt) ||
      !e->g_c.ensure(8 * std::max(nt, nb)) || !e->g_thr.ensure(8 * nb))
    return fail(ISRSGN_ENOMEM, "device allocation failed for the graph buffers");
  GraphEntry* ge = nullptr;
  for (auto& g : e->graphs)
    if (g.kind == kind && g.snr_trx == snr_trx) ge = &g;
  double* o_a = e->g_a.as<double>();  // eta | snr
  double* o_b = e->g_b.as<double>();  // pnli | dthr
  double* o_t = e->g_thr.as<double>();
  if (!ge) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const bool timing = h->timing;
    h->timing = false;
    hipError_t err = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) { h->timing = timing; return hip_fail(err, "hipStreamBeginCapture"); }
    int rc;
    if (kind == kEta)
      rc = enqueue_call(h, e, kind, e->g_P.as<double>(), nullptr, 0.0, o_a, o_b, nullptr, nullptr, nullptr, nullptr,
                        h->cap_stream);
    else
      rc = enqueue_call(h, e, kind, e->g_P.as<double>(), e->g_nf.as<double>(), snr_trx, nullptr, nullptr, nullptr,
                        o_a, o_t, kind == kGrad ? o_b : nullptr, h->cap_stream);
    err = hipStreamEndCapture(h->cap_stream, &graph);
    h->timing = timing;
    if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
    if (err != hipSuccess) return hip_fail(err, "hipStreamEndCapture");
    err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (err != hipSuccess) return hip_fail(err, "hipGraphInstantiate");
    e->graphs.push_back(GraphEntry{kind, snr_trx, exec});
    ge = &e->graphs.back();
  }
  begin_timing(h);
  mark(h, s);
  hipError_t err = launch_copy(e->g_P.as<double>(), P, (int64_t)nt, s);
  if (err == hipSuccess && nf) err = launch_copy(e->g_nf.as<double>(), nf, (int64_t)nt, s);
  if (err == hipSuccess) err = hipGraphLaunch(ge->exec, s);
  if (err == hipSuccess) {
    if (kind == kEta) {
      err = launch_copy(eta, o_a, (int64_t)nt, s);
      if (err == hipSuccess && pnli) err = launch_copy(pnli, o_b, (int64_t)nt, s);
      if (err == hipSuccess && tiles)
        err = e->nli == 1 ? launch_copy(tiles, e->tiles.as<double>(), e->n_tiles, s)
                          : launch_fold_tiles(e->view(), e->work(), tiles, s);
    } else {
      err = launch_copy(snr, o_a, (int64_t)nt, s);
      if (err == hipSuccess) err = launch_copy(thr, o_t, (int64_t)nb, s);
      if (err == hipSuccess && kind == kGrad) err = launch_copy(dthr, o_b, (int64_t)nt, s);
    }
  }
  if (err != hipSuccess) return hip_fail(err, "graph launch");
  mark(h, s);
  return ISRSGN_OK;
}

// The boundary's input rules: every launch power finite and >= 0 (P = 0 marks an empty channel)
// and every noise figure, when given, finite and >= 0.  A one-block kernel counts the violations
// and the host waits for its verdict (the stream's earlier work included), so a rejected call
// writes no output.  Skipped while the stream is being captured into a graph, where a host wait
// is not allowed, and when the caller has switched the checks off.
int check_inputs(isrsgn_fibre* h, const double* P, const double* nf, int n, hipStream_t s) {
  if (!h->checks) return ISRSGN_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return ISRSGN_OK;
  hipError_t err = launch_check_inputs(P, nf, n, h->d_check.as<int>(), s);
  if (err == hipSuccess) err = hipMemcpyAsync(h->h_check, h->d_check.p, 3 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  if (err != hipSuccess) return hip_fail(err, "input check");
  if (h->h_check[0] == 0) return ISRSGN_OK;
  if (h->h_check[1] < n)
    return fail(ISRSGN_EINVAL, "P_w_dev[%d] is negative or not finite (launch powers must be finite and >= 0)",
                h->h_check[1]);
  return fail(ISRSGN_EINVAL, "nf_lin_dev[%d] is negative or not finite (noise figures must be finite and >= 0)",
              h->h_check[2]);
}

// Marks the end of a call on stream s (isrsgn_destroy waits for these, not for the whole device).
int record_done(isrsgn_fibre* h, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return ISRSGN_OK;
  hipEvent_t ev = nullptr;
  for (auto& d : h->done)
    if (d.first == s) ev = d.second;
  if (!ev) {
    hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (err != hipSuccess) return hip_fail(err, "completion event");
    h->done.emplace_back(s, ev);
  }
  hipError_t err = hipEventRecord(ev, s);
  return err == hipSuccess ? ISRSGN_OK : hip_fail(err, "completion event");
}

int run_call(isrsgn_fibre* h, const isrsgn_plan* plan, int kind, const double* P, const double* nf, double snr_trx,
             double* eta, double* pnli, double* tiles, double* snr, double* thr, double* dthr, hipStream_t s) {
  PlanEntry* e;
  int rc = get_plan(h, plan, s, &e);
  if (rc) return rc;
  if (kind == kGrad && (rc = ensure_grad_workspace(h, e))) return rc;
  if ((rc = check_inputs(h, P, nf, e->n_total, s))) return rc;
  if (h->graph && variant_known(h))
    rc = run_graph(h, e, kind, P, nf, snr_trx, eta, pnli, tiles, snr, thr, dthr, s);
  else
    rc = enqueue_call(h, e, kind, P, nf, snr_trx, eta, pnli, tiles, snr, thr, dthr, s);
  return rc ? rc : record_done(h, s);
}

// ---------------------------------------------------------------------------- no allocation
// The workspace of one isrsgn_snr_noalloc call, carved out of the scratch array from `base`
// (256-byte aligned sections): the plan's device copy and the Work fields the forward kernels
// use.  Returns the bytes it takes (with base = 0 it only sizes).
size_t carve_noalloc(const isrsgn_fibre* h, int nb, int nt, int64_t ntiles, uintptr_t base, PlanView* pv, Work* w) {
  size_t used = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = reinterpret_cast<char*>(base + used);
    used += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const size_t M = (size_t)h->desc.n_steps, n = (size_t)nt, b = (size_t)nb;
  const bool fp32 = h->desc.precision == ISRSGN_FP32, lr = fp32 && h->desc.profile == ISRSGN_PROFILE_ODE;
  *pv = PlanView{};
  pv->n_batch = nb;
  pv->n_total = nt;
  pv->nli = h->fp.nli;
  pv->n_tiles = ntiles;
  pv->off = reinterpret_cast<int*>(take(4 * (b + 1)));
  pv->toff = reinterpret_cast<int64_t*>(take(8 * (b + 1)));
  pv->f = reinterpret_cast<double*>(take(8 * n));
  pv->R = reinterpret_cast<double*>(take(8 * n));
  pv->alpha = reinterpret_cast<double*>(take(8 * n));
  pv->aeff = reinterpret_cast<double*>(take(8 * n));
  pv->gamma = reinterpret_cast<double*>(take(8 * n));
  pv->cr = reinterpret_cast<double*>(take(8 * n));
  pv->fpt = reinterpret_cast<double*>(take(8 * n * h->fp.nli));
  pv->wpt = reinterpret_cast<double*>(take(8 * n * h->fp.nli));
  *w = Work{};
  w->abar = reinterpret_cast<double*>(take(8 * b));
  w->zm = reinterpret_cast<double*>(take(8 * b * M));
  w->dz = reinterpret_cast<double*>(take(8 * b * M));
  w->hdz32 = reinterpret_cast<float*>(take(4 * b * M));
  w->step_rec = reinterpret_cast<double*>(take(32 * b * M));
  w->ell64 = reinterpret_cast<double*>(take(8 * n * M));
  if (fp32) w->lt32 = reinterpret_cast<float2*>(take(8 * n * M));
  if (lr) {
    w->lr_a = reinterpret_cast<float*>(take(4 * b * M * kRank));
    w->lr_b = reinterpret_cast<float2*>(take(8 * n * kRank));
    w->lr_rank = reinterpret_cast<int*>(take(4 * b));
    w->lr_res = reinterpret_cast<double*>(take(8 * n * M));
    w->lr_b64 = reinterpret_cast<double*>(take(8 * n * kRank));
  }
  w->ellL = reinterpret_cast<double*>(take(8 * n));
  w->tiles = reinterpret_cast<double*>(take(8 * (size_t)ntiles));
  w->pnli = reinterpret_cast<double*>(take(8 * n));
  w->snr = reinterpret_cast<double*>(take(8 * n));
  char* counter = take(64);
  w->counter = reinterpret_cast<unsigned int*>(counter);
  w->nodes = reinterpret_cast<unsigned long long*>(counter + 32);
  return used;
}

// Host values to the device through kernel arguments: dst[q] = fill(q) for q < n (8-byte words).
template <class Fill>
hipError_t put_words(void* dst, int64_t n, Fill&& fill, hipStream_t s) {
  WordChunk c;
  for (int64_t q0 = 0; q0 < n; q0 += kChunkWords) {
    c.n = (int)std::min<int64_t>(kChunkWords, n - q0);
    for (int j = 0; j < c.n; ++j) c.w[j] = fill(q0 + j);
    const hipError_t e = launch_put_words(static_cast<unsigned long long*>(dst) + q0, c, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

unsigned long long word_of(double x) {
  unsigned long long u;
  std::memcpy(&u, &x, sizeof(u));
  return u;
}

// Tile-kernel variant without tuning: forced, or the autotuner's earlier choice, or a default.
int noalloc_variant(isrsgn_fibre* h) {
  const char* force = std::getenv("ISRSGN_TILE_VARIANT");
  if (force && *force) {
    const int v = std::atoi(force);
    return v >= 0 && v < kTileVariants ? v : 0;
  }
  const TuneKey key{h->desc.precision, h->desc.profile, h->desc.grid_s, h->desc.grid_v, h->desc.n_steps};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  read_tune_file();
  for (auto& kv : g_tuned)
    if (kv.first == key) return kv.second;
  return h->desc.precision == ISRSGN_FP32 ? 2 : 0;  // unroll 2 at 5 waves/SIMD; FP64: unroll 1
}

}  // namespace

extern "C" {

int isrsgn_setup_fibre(const isrsgn_fibre_desc* d, isrsgn_fibre** out) {
  g_err.clear();
  if (!out) return fail(ISRSGN_EINVAL, "out is NULL");
  int rc = validate_desc(d);
  if (rc) return rc;
  auto h = std::make_unique<isrsgn_fibre>();
  h->desc = *d;
  h->tab_f.assign(d->tab_f_hz, d->tab_f_hz + d->n_tab);
  h->tab_alpha.assign(d->alpha_per_m, d->alpha_per_m + d->n_tab);
  h->tab_aeff.assign(d->aeff_m2, d->aeff_m2 + d->n_tab);
  h->desc.tab_f_hz = h->desc.alpha_per_m = h->desc.aeff_m2 = nullptr;
  FibreParams& fp = h->fp;
  fp.span = d->span_m;
  fp.f_ref = d->f_ref_hz;
  if (d->disp_from_d) {  // eqs. (d), (d_slope), (d_curve) at lambda = c / f_ref
    const double lam = kC / d->f_ref_hz, w = 2.0 * kPi * kC, D = d->d_s_per_m2, S = d->s_s_per_m3,
                 Sd = d->sdot_s_per_m4;
    fp.b2 = -D * lam * lam / w;
    fp.b3 = lam * lam * lam / (w * w) * (2.0 * D + S * lam);
    fp.b4 = -(lam * lam * lam * lam) / (w * w * w) * (6.0 * D + 6.0 * S * lam + Sd * lam * lam);
  } else {
    fp.b2 = d->beta2;
    fp.b3 = d->beta3;
    fp.b4 = d->beta4;
  }
  fp.n2 = d->n2_m2_per_w;
  fp.gamma_const = d->gamma_const_per_w_m;
  fp.cr = d->cr_per_w_m_hz;
  fp.aeff_ref = d->aeff_ref_m2;
  fp.cutoff = d->raman_cutoff_hz;
  fp.profile = d->profile;
  fp.photon_ratio = d->photon_ratio ? 1 : 0;
  fp.n_steps = d->n_steps;
  fp.grid_s = d->grid_s;
  fp.grid_v = d->grid_v;
  fp.ode_sub = d->ode_sub;
  fp.precision = d->precision;
  fp.n_spans = d->n_spans;
  fp.rolloff = d->rolloff;
  fp.nli = d->nli_points;
  {
    const char* lr = std::getenv("ISRSGN_LOWRANK");
    const int cap = lr && *lr ? std::atoi(lr) : kRank;
    fp.lowrank = cap < 0 ? 0 : (cap > kRank ? kRank : cap);
    const char* aw = std::getenv("ISRSGN_ADJOINT_WAVES");
    fp.adj_wide = aw && *aw && std::atoi(aw) == 4 ? 0 : 1;
  }
  fp.s_decades = d->s_decades;
  fp.n_tab = d->n_tab;
  hipError_t err;
  if ((err = hipGetDevice(&h->device)) != hipSuccess) return hip_fail(err, "hipGetDevice");
  {
    void* sp = nullptr;
    if ((rc = scratch_address(h->device, &sp))) return rc;
  }
  int lds_max = 0;
  if ((err = hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device)) != hipSuccess ||
      (err = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device)) != hipSuccess)
    return hip_fail(err, "device attributes");
  if (lds_max > 0) h->lds_max = (size_t)lds_max;
  const size_t tb = 8 * (size_t)d->n_tab;
  if (!h->d_tab_f.ensure(tb) || !h->d_tab_alpha.ensure(tb) || !h->d_tab_aeff.ensure(tb))
    return fail(ISRSGN_ENOMEM, "device allocation failed for the fibre tables");
  if ((err = hipMemcpy(h->d_tab_f.p, h->tab_f.data(), tb, hipMemcpyHostToDevice)) != hipSuccess ||
      (err = hipMemcpy(h->d_tab_alpha.p, h->tab_alpha.data(), tb, hipMemcpyHostToDevice)) != hipSuccess ||
      (err = hipMemcpy(h->d_tab_aeff.p, h->tab_aeff.data(), tb, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(err, "table upload");
  fp.tab_f = h->d_tab_f.as<double>();
  fp.tab_alpha = h->d_tab_alpha.as<double>();
  fp.tab_aeff = h->d_tab_aeff.as<double>();
  if (!h->d_check.ensure(4 * sizeof(int))) return fail(ISRSGN_ENOMEM, "device allocation failed for the input check");
  if ((err = hipHostMalloc(reinterpret_cast<void**>(&h->h_check), 4 * sizeof(int), hipHostMallocDefault)) != hipSuccess)
    return hip_fail(err, "pinned host memory for the input check");
  *out = h.release();
  return ISRSGN_OK;
}

int isrsgn_eta(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P, double* eta, double* pnli, double* tiles,
               void* stream) {
  g_err.clear();
  if (!h || !P || !eta) return fail(ISRSGN_EINVAL, "handle, P_w_dev and eta_dev are required");
  return run_call(h, plan, kEta, P, nullptr, 0.0, eta, pnli, tiles, nullptr, nullptr, nullptr,
                  static_cast<hipStream_t>(stream));
}

int isrsgn_snr(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P, const double* nf, double snr_trx,
               double* snr, double* thr, void* stream) {
  g_err.clear();
  if (!h || !P || !nf || !snr || !thr) return fail(ISRSGN_EINVAL, "handle, P, NF, snr and thr pointers are required");
  if (!(snr_trx >= 0) || !is_fin(snr_trx)) return fail(ISRSGN_EINVAL, "snr_trx_lin must be finite and >= 0");
  return run_call(h, plan, kSnr, P, nf, snr_trx, nullptr, nullptr, nullptr, snr, thr, nullptr,
                  static_cast<hipStream_t>(stream));
}

int isrsgn_snr_grad(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P, const double* nf, double snr_trx,
                    double* snr, double* thr, double* dthr, void* stream) {
  g_err.clear();
  if (!h || !P || !nf || !snr || !thr || !dthr)
    return fail(ISRSGN_EINVAL, "handle, P, NF, snr, thr and dthr pointers are required");
  if (!(snr_trx >= 0) || !is_fin(snr_trx)) return fail(ISRSGN_EINVAL, "snr_trx_lin must be finite and >= 0");
  return run_call(h, plan, kGrad, P, nf, snr_trx, nullptr, nullptr, nullptr, snr, thr, dthr,
                  static_cast<hipStream_t>(stream));
}

int isrsgn_snr_noalloc(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P, const double* nf, double snr_trx,
                       double* snr, double* thr, void* stream) {
  g_err.clear();
  if (!h || !P || !nf || !snr || !thr) return fail(ISRSGN_EINVAL, "handle, P, NF, snr and thr pointers are required");
  if (!(snr_trx >= 0) || !is_fin(snr_trx)) return fail(ISRSGN_EINVAL, "snr_trx_lin must be finite and >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t ntiles = 0;
  int nmax = 0;
  int rc = validate_plan(h, plan, &ntiles, &nmax);
  if (rc) return rc;
  int dev = -1;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return hip_fail(err, "hipGetDevice");
  if (dev != h->device)
    return fail(ISRSGN_EINVAL, "the handle was set up on device %d but device %d is current", h->device, dev);
  void* base = nullptr;
  if ((rc = scratch_address(dev, &base))) return rc;
  const int nb = plan->n_batch, nt = plan->ch_offsets[nb];
  PlanView pv;
  Work w;
  const size_t need = carve_noalloc(h, nb, nt, ntiles, 0, &pv, &w);
  if (need > (size_t)ISRSGN_NOALLOC_SCRATCH_BYTES)
    return fail(ISRSGN_EINVAL, "the plan needs %zu B of workspace; the no-allocation scratch holds %zu B (isrsgn_snr "
                "has no such limit)", need, (size_t)ISRSGN_NOALLOC_SCRATCH_BYTES);
  carve_noalloc(h, nb, nt, ntiles, reinterpret_cast<uintptr_t>(base), &pv, &w);
  if ((rc = check_inputs(h, P, nf, nt, s))) return rc;
  // the plan: offsets as pairs of ints per word, tile offsets, centres and symbol rates
  const int* off = plan->ch_offsets;
  err = put_words(const_cast<int*>(pv.off), (nb + 2) / 2, [&](int64_t q) {
    const unsigned long long lo = (unsigned int)off[2 * q];
    const unsigned long long hi = 2 * q + 1 <= nb ? (unsigned int)off[2 * q + 1] : 0u;
    return lo | (hi << 32);
  }, s);
  int64_t acc = 0;
  if (err == hipSuccess)
    err = put_words(const_cast<int64_t*>(pv.toff), nb + 1, [&](int64_t q) {
      const unsigned long long v = (unsigned long long)acc;
      if (q < nb) {
        const int64_t n = off[q + 1] - off[q];
        acc += n * n * h->fp.nli;
      }
      return v;
    }, s);
  if (err == hipSuccess) err = put_words(const_cast<double*>(pv.f), nt, [&](int64_t q) { return word_of(plan->f_hz[q]); }, s);
  if (err == hipSuccess)
    err = put_words(const_cast<double*>(pv.R), nt, [&](int64_t q) { return word_of(plan->rs_hz[q]); }, s);
  if (err != hipSuccess) return hip_fail(err, "plan upload");
  if ((err = launch_channel_setup(pv, h->fp, s)) != hipSuccess) return hip_fail(err, "channel setup");
  if ((err = launch_steps(pv, h->fp, P, w, s)) != hipSuccess) return hip_fail(err, "steps");
  if ((err = launch_profile(pv, h->fp, P, w, false, s)) != hipSuccess) return hip_fail(err, "profile");
  const int variant = noalloc_variant(h);
  if ((err = launch_tiles(pv, h->fp, P, w, nmax, tile_grid(h, nmax, variant, ntiles), variant, 0u,
                          (unsigned int)ntiles, true, s)) != hipSuccess)
    return hip_fail(err, "pair integrals");
  if ((err = launch_reduce(pv, h->fp, P, nf, snr_trx, w, nullptr, nullptr, snr, thr, s)) != hipSuccess)
    return hip_fail(err, "reduction");
  return ISRSGN_OK;
}

int isrsgn_set_graph(isrsgn_fibre* h, int enabled) {
  g_err.clear();
  if (!h) return fail(ISRSGN_EINVAL, "handle is NULL");
  if (enabled && !h->cap_stream) {
    hipError_t err = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (err != hipSuccess) return hip_fail(err, "capture stream");
  }
  h->graph = enabled != 0;
  return ISRSGN_OK;
}

int isrsgn_profile(isrsgn_fibre* h, const isrsgn_plan* plan, const double* P, double* zm, double* dz, double* ell,
                   double* ellL, void* stream) {
  g_err.clear();
  if (!h || !P) return fail(ISRSGN_EINVAL, "handle and P_w_dev are required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanEntry* e;
  int rc = get_plan(h, plan, s, &e);
  if (rc) return rc;
  if ((rc = check_inputs(h, P, nullptr, e->n_total, s))) return rc;
  Work w = e->work();
  PlanView pv = e->view();
  hipError_t err;
  if ((err = launch_steps(pv, h->fp, P, w, s)) != hipSuccess) return hip_fail(err, "steps");
  if ((err = launch_profile(pv, h->fp, P, w, false, s)) != hipSuccess) return hip_fail(err, "profile");
  if ((err = launch_copy_profile(pv, h->fp, w, zm, dz, ell, ellL, s)) != hipSuccess) return hip_fail(err, "copy");
  return record_done(h, s);
}

int isrsgn_set_checks(isrsgn_fibre* h, int enabled) {
  g_err.clear();
  if (!h) return fail(ISRSGN_EINVAL, "handle is NULL");
  h->checks = enabled != 0;
  return ISRSGN_OK;
}

int isrsgn_set_timing(isrsgn_fibre* h, int enabled) {
  g_err.clear();
  if (!h) return fail(ISRSGN_EINVAL, "handle is NULL");
  h->timing = enabled != 0;
  return ISRSGN_OK;
}

int isrsgn_stage_times(isrsgn_fibre* h, double* ms, int n) {
  g_err.clear();
  if (!h || !ms || n < 1) return fail(ISRSGN_EINVAL, "handle and output are required");
  for (int q = 0; q < n && q < 6; ++q) ms[q] = 0.0;
  if (h->ev_count < 1) return ISRSGN_OK;
  hipError_t err = hipEventSynchronize(h->evs[h->ev_count - 1]);
  if (err != hipSuccess) return hip_fail(err, "hipEventSynchronize");
  auto elapsed = [&](int a, int b) -> double {
    float t = 0.f;
    return hipEventElapsedTime(&t, h->evs[a], h->evs[b]) == hipSuccess ? (double)t : 0.0;
  };
  double st[6] = {0, 0, 0, 0, 0, 0};
  for (const auto& sp : h->spans) st[sp.stage] += elapsed(sp.a, sp.b);
  st[5] = elapsed(0, h->ev_count - 1);
  for (int q = 0; q < n && q < 6; ++q) ms[q] = st[q];
  return ISRSGN_OK;
}

int isrsgn_work_counts(isrsgn_fibre* h, double* out, int n) {
  g_err.clear();
  if (!h || !out || n < 1) return fail(ISRSGN_EINVAL, "handle and output are required");
  for (int q = 0; q < n && q < 7; ++q) out[q] = 0.0;
  if (n > 3) out[3] = h->last_variant;
  if (h->plans.empty()) return ISRSGN_OK;
  const PlanEntry* e = h->plans[0].get();
  if (n > 4) out[4] = h->last_grad_batches;
  unsigned long long nodes = 0;
  hipError_t err = hipMemcpy(&nodes, e->counter.as<char>() + 32, sizeof(nodes), hipMemcpyDeviceToHost);
  if (err != hipSuccess) return hip_fail(err, "work counters");
  if (n > 5 && e->lr_rank.p) {
    std::vector<int> rk((size_t)e->n_batch);
    err = hipMemcpy(rk.data(), e->lr_rank.p, sizeof(int) * rk.size(), hipMemcpyDeviceToHost);
    if (err != hipSuccess) return hip_fail(err, "low-rank counters");
    int used = 0, most = 0;
    for (int r : rk)
      if (r >= 0) {
        ++used;
        most = std::max(most, r);
      }
    out[5] = used;
    if (n > 6) out[6] = most;
  }
  const double v[3] = {(double)nodes, (double)nodes * h->desc.n_steps, (double)e->n_tiles};
  for (int q = 0; q < n && q < 3; ++q) out[q] = v[q];
  return ISRSGN_OK;
}

void isrsgn_destroy(isrsgn_fibre* h) {
  if (!h) return;
  // wait for the handle's own work only: the last call on every stream it was given
  for (auto& d : h->done) {
    (void)hipEventSynchronize(d.second);
    (void)hipEventDestroy(d.second);
  }
  for (hipEvent_t ev : h->evs) (void)hipEventDestroy(ev);
  if (h->h_check) (void)hipHostFree(h->h_check);
  h->plans.clear();
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  delete h;
}

const char* isrsgn_last_error(void) { return g_err.c_str(); }

}  // extern "C"
