// C ABI of libfsest (declared in include/fsest.h): argument validation, the
// workspace layout, the call-order state machine, HIP-graph capture and the
// launch-shape autotuner.  All kernels live in deposit.hip, fft.hip and
// spectral.hip.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "fsest_internal.hpp"

using namespace fsest;

namespace {

thread_local char g_err[512] = "";

est_status fail(est_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

est_status ok() { return EST_OK; }

enum State { kCreated = 0, kDeposited = 1, kXY = 2, kSpectrum = 3 };

// no prime factor above 5
bool smooth235(int v) {
  if (v < 1) return false;
  for (int p : {2, 3, 5})
    while (v % p == 0) v /= p;
  return v == 1;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

enum ProfLabel {
  kPSort = 0, kPDeposit, kPFftX, kPFftY, kPFftZ, kPPower, kPAdjoint, kPIfftY, kPIfftX, kPGather,
  kPModes, kPBispec, kPDirect, kPBsFields, kPBsTriple, kPNumLabels
};
static const char* kProfNames[kPNumLabels] = {
    "bucket_sort", "deposit", "fft_x", "fft_y", "fft_z", "power_fused_z", "adjoint_fused_z",
    "ifft_y", "ifft_x", "gather_grad", "mode_table", "bispectrum", "direct_sum",
    "bispec_fields", "bispec_triple"};

struct ProfRec {
  double total_ms = 0.0;
  int64_t launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

struct est_ctx {
  est_config cfg;
  Geom g;
  Buffers b;
  Tune tu;
  hipStream_t stream;
  int device;
  int state = kCreated;
  int mode_dk = -1, mode_nbins = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* tune_out = nullptr;
  bool prof = false;
  bool capturing = false;
  const float* weights = nullptr;  // masses for the particle calls (EST_FLAG_WEIGHTS)
  // the bispectrum's count sums (sum_x J J J per job entry) of the last
  // (field grid, shell width, shells, jobs), reused while they match
  int bs_M = 0, bs_dk = 0, bs_nbins = 0;
  std::vector<int32_t> bs_jobs;
  std::vector<double> bs_runj;
  ProfRec rec[kPNumLabels];
  std::vector<hipEvent_t> pool;
};

namespace {

hipEvent_t prof_event(est_ctx* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches of one kernel group with events when profiling.
struct ProfScope {
  est_ctx* h;
  int label;
  hipEvent_t a = nullptr;
  ProfScope(est_ctx* hh, int l) : h(hh), label(l) {
    if (h->prof && !h->capturing) {
      a = prof_event(h);
      if (a) (void)hipEventRecord(a, h->stream);
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = prof_event(h);
    if (!b) return;
    (void)hipEventRecord(b, h->stream);
    h->rec[label].pending.emplace_back(a, b);
  }
};

void prof_fold(est_ctx* h) {
  for (auto& r : h->rec) {
    for (auto& pr : r.pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
        r.total_ms += ms;
        r.launches += 1;
      }
      h->pool.push_back(pr.first);
      h->pool.push_back(pr.second);
    }
    r.pending.clear();
  }
}

est_status check_config(const est_config* c) {
  if (!c) return fail(EST_EINVAL, "config is NULL");
  if (c->order < 1 || c->order > 6) return fail(EST_EINVAL, "order must be 1..6 (got %d)", c->order);
  if (c->interlace < 0 || c->interlace > 3)
    return fail(EST_EINVAL, "interlace must be 0, 1, 2 or 3 (got %d)", c->interlace);
  if (c->interlace >= 2 && c->batch > 65535 / (1 << (c->interlace - 1)))
    return fail(EST_EINVAL, "batch times complex grids per set must be <= 65535");
  if (c->batch < 1 || c->batch > 65535) return fail(EST_EINVAL, "batch must be 1..65535 (got %d)", c->batch);
  if (!(c->box > 0.0) || !std::isfinite(c->box)) return fail(EST_EINVAL, "box must be finite and > 0");
  if (c->max_particles < 1 || c->max_particles > 2147483647LL)
    return fail(EST_EINVAL, "max_particles must be 1..2^31-1");
  if ((c->flags & ~(EST_FLAG_ATOMIC_SORT | EST_FLAG_WEIGHTS)) != 0 || c->reserved != 0)
    return fail(EST_EINVAL,
                "flags must combine EST_FLAG_ATOMIC_SORT and EST_FLAG_WEIGHTS only, reserved 0");
  if (c->n_grid < 8 || c->n_grid > 1024 || c->n_grid % kBucket != 0 || !smooth235(c->n_grid))
    return fail(EST_EUNSUPPORTED,
                "n_grid must be a multiple of 4 in [8, 1024] with prime factors 2, 3, 5 only (got %d)",
                c->n_grid);
  if (c->n_grid > kTileMax && c->n_grid < kTileMax + c->order - 1)
    return fail(EST_EUNSUPPORTED, "n_grid = %d is too small for a tiled deposit of order %d",
                c->n_grid, c->order);
  const int64_t nb = c->n_grid / kBucket;
  if ((int64_t)c->batch * nb * nb * nb + 1 >= 4294967295LL)
    return fail(EST_EINVAL, "batch * (N/4)^3 exceeds the 32-bit bucket index");
  return ok();
}

Geom make_geom(const est_config& c) {
  Geom g;
  g.n = c.n_grid;
  g.nz = c.interlace ? c.n_grid : c.n_grid / 2;
  g.code = c.interlace;
  g.ng = 1 << (c.interlace == 0 ? 0 : c.interlace);  // 1, 2, 4, 8
  g.npair = g.ng > 1 ? g.ng / 2 : 1;
  g.order = c.order;
  g.il = c.interlace ? 1 : 0;
  g.batch = c.batch;
  g.nb = c.n_grid / kBucket;
  // Super-bucket edge fb: a divisor of nb up to kFineMax, so super-buckets
  // tile the axis, and at least 5 unless it is nb itself, so that a deposit
  // run of up to 6 buckets in z meets at most one super-bucket edge (nb has
  // no prime factor above 5, so such a divisor exists when nb > kFineMax).
  // Of these, the smallest whose super-bucket count batch (nb/fb)^3 stays at
  // or below max_particles / 16384: about 16K particles per super-bucket,
  // enough per (workgroup chunk, super-bucket) for whole-line writes in the
  // super-bucket pass, and as many super-buckets as that allows for the
  // bucket pass, which runs one workgroup per super-bucket (many uneven sets
  // then spread over the chip).  If none qualifies, the largest.
  {
    const int64_t target = c.max_particles / 16384 > 1 ? c.max_particles / 16384 : 1;
    int small_ok = 0, largest = 0;
    for (int d = 1; d <= kFineMax && d <= g.nb; ++d) {
      if (g.nb % d != 0 || (d < 5 && d != g.nb)) continue;
      largest = d;
      const int64_t sa = g.nb / d;
      if (!small_ok && (int64_t)c.batch * sa * sa * sa <= target) small_ok = d;
    }
    g.fb = small_ok ? small_ok : largest;
  }
  g.sa = g.nb / g.fb;
  g.fb_mul = g.fb >= 2 ? (uint32_t)(4294967296ull / (uint64_t)g.fb + 1) : 0u;
  const int64_t nsup = (int64_t)c.batch * g.sa * g.sa * g.sa;
  // the two-level sort runs when nsup <= kMaxSuper; a larger value selects the atomic sort
  g.nsup = ((c.flags & EST_FLAG_ATOMIC_SORT) || nsup > kMaxSuper) ? kMaxSuper + 1 : (int)nsup;
  g.tile = c.n_grid < kTileMax ? c.n_grid : kTileMax;
  g.box = c.box;
  g.inv = (double)c.n_grid / c.box;
  const int64_t plane = (int64_t)g.n * g.nz;
  g.ps = plane + (plane >= 65536 ? 512 : 0);
  return g;
}

// Workspace layout; with base == nullptr only the size is computed.
size_t layout(const est_config& c, char* base, Buffers* b, void** tune_out) {
  const Geom g = make_geom(c);
  const size_t n = (size_t)g.n, batch = (size_t)g.batch, half = n / 2;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  const size_t nkeys = batch * (size_t)g.nb * g.nb * g.nb + 1;
  Buffers bb;
  bb.grid = (float2*)take(batch * g.npair * n * (size_t)g.ps * sizeof(float2));
  bb.recs = (uint4*)take((size_t)c.max_particles * sizeof(uint4));
  bb.rank = (uint32_t*)take((size_t)c.max_particles * sizeof(uint32_t));
  bb.boff = (uint32_t*)take(nkeys * sizeof(uint32_t));
  bb.bcnt = (uint32_t*)take(nkeys * sizeof(uint32_t));
  const bool two_level = g.nsup <= kMaxSuper;
  bb.trecs = two_level ? (uint4*)take((size_t)c.max_particles * sizeof(uint4)) : nullptr;
  // block-major histograms (kMaxSortBlocks rows of nsup) and the nsup + 1 super-bucket starts
  const size_t nh = two_level ? (size_t)g.nsup * kMaxSortBlocks + g.nsup + 1 : 0;
  bb.hsup = two_level ? (uint32_t*)take(nh * sizeof(uint32_t)) : nullptr;
  const size_t nscan = nkeys > nh ? nkeys : nh;
  bb.scan_tmp = (uint32_t*)take(((nscan + 2047) / 2048 + 1) * sizeof(uint32_t));
  bb.stats = (uint32_t*)take(64 * sizeof(uint32_t));
  bb.tw_n = (float2*)take(n * sizeof(float2));
  bb.tw_nz = (float2*)take((size_t)g.nz * sizeof(float2));
  bb.inv_w2 = (float*)take(n * sizeof(float));
  bb.win1 = (float*)take(n * sizeof(float));
  bb.phase = (float2*)take(2 * n * sizeof(float2));
  bb.partials = (double*)take(batch * kMaxBinBlocks * half * sizeof(double));
  bb.mode_n = (int64_t*)take(half * sizeof(int64_t));
  bb.mode_k = (double*)take(half * sizeof(double));
  bb.np = (int64_t*)take(batch * sizeof(int64_t));
  bb.norm = (double*)take(batch * 2 * sizeof(double));
  const bool weighted = (c.flags & EST_FLAG_WEIGHTS) != 0;
  bb.sw = weighted ? (float*)take((size_t)c.max_particles * sizeof(float)) : nullptr;
  bb.tw = weighted && two_level ? (float*)take((size_t)c.max_particles * sizeof(float)) : nullptr;
  bb.wpart = weighted ? (double*)take(batch * weight_slices(c.batch) * 2 * sizeof(double)) : nullptr;
  bb.cbuf = c.interlace >= 2 ? (float2*)take(batch * n * n * (half + 1) * sizeof(float2)) : nullptr;
  bb.coef = (double*)take(batch * half * sizeof(double));
  bb.mode_partials_n = (uint64_t*)take(512 * half * sizeof(uint64_t));
  bb.mode_partials_k = (double*)take(512 * half * sizeof(double));
  char* to = take(batch * half * 3 * sizeof(double));
  if (b) *b = bb;
  if (tune_out) *tune_out = to;
  return off;
}

est_status dev_err(hipError_t e, const char* what) {
  if (e == hipSuccess) return EST_OK;
  return fail(EST_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// HIP keeps the last error of any API call in the thread (the caller's own
// included) until it is read; launch checks read it, so every entry point
// clears what was left before it starts launching.
void clear_stale_error() { (void)hipGetLastError(); }

est_status check_handle(est_handle h) {
  if (!h) return fail(EST_EINVAL, "handle is NULL");
  clear_stale_error();
  return ok();
}

est_status check_particles(est_handle h, const void* pos, est_dtype dt, const int64_t* offsets,
                           int64_t n_total) {
  if (!pos) return fail(EST_EINVAL, "pos is NULL");
  if (dt != EST_F32 && dt != EST_F64) return fail(EST_EINVAL, "dtype must be EST_F32 or EST_F64");
  if (n_total < 1 || n_total > h->cfg.max_particles)
    return fail(EST_EINVAL, "n_total must be 1..max_particles (%lld), got %lld",
                (long long)h->cfg.max_particles, (long long)n_total);
  if (h->cfg.batch == 1 && offsets) return fail(EST_EINVAL, "offsets must be NULL when batch == 1");
  if (h->cfg.batch > 1 && !offsets) return fail(EST_EINVAL, "offsets required when batch > 1");
  return ok();
}

est_status check_bins(est_handle h, int32_t n_dk, int32_t n_bins) {
  if (n_dk < 1) return fail(EST_EINVAL, "n_dk must be >= 1");
  const int maxb = h->g.n / (2 * n_dk);
  if (n_bins < 1 || n_bins > maxb)
    return fail(EST_EINVAL, "n_bins must be 1..N/(2 n_dk) = %d (got %d)", maxb, n_bins);
  return ok();
}

est_status ensure_modes(est_handle h, int n_dk, int n_bins) {
  if (h->mode_dk == n_dk && h->mode_nbins == n_bins) return ok();
  ProfScope ps(h, kPModes);
  est_status st = dev_err(launch_mode_table(h->g, h->b, n_dk, n_bins, h->stream), "mode table");
  if (st != EST_OK) return st;
  h->mode_dk = n_dk;
  h->mode_nbins = n_bins;
  return ok();
}

est_status run_deposit(est_handle h, const void* pos, est_dtype dt, const int64_t* offsets,
                       int64_t n_total) {
  est_status st;
  {
    ProfScope ps(h, kPSort);
    st = dev_err(launch_set_counts(offsets, n_total, h->g.batch, h->b.np, h->b.norm, h->stream),
                 "counts");
    if (st) return st;
    if (h->weights) {
      st = dev_err(launch_weight_stats(h->weights, offsets, n_total, h->g.batch, h->b.wpart,
                                       h->b.norm, h->b.stats, h->stream),
                   "mass sums");
      if (st) return st;
    }
    st = dev_err(launch_sort(h->g, pos, dt, offsets, n_total, h->weights, h->b, h->stream),
                 "bucket sort");
    if (st) return st;
  }
  ProfScope ps(h, kPDeposit);
  return dev_err(launch_deposit(h->g, h->b, h->tu, h->weights != nullptr, h->stream), "deposit");
}

est_status run_xy(est_handle h, int dir) {
  est_status st;
  if (dir < 0) {
    {
      ProfScope ps(h, kPFftX);
      st = dev_err(launch_fft_axis(h->g, h->b.grid, 0, -1, h->g.batch * h->g.npair, h->g.nz, h->b.tw_n, h->tu, h->stream), "fft x");
      if (st) return st;
    }
    ProfScope ps(h, kPFftY);
    return dev_err(launch_fft_axis(h->g, h->b.grid, 1, -1, h->g.batch * h->g.npair, h->g.nz, h->b.tw_n, h->tu, h->stream), "fft y");
  }
  {
    ProfScope ps(h, kPIfftY);
    st = dev_err(launch_fft_axis(h->g, h->b.grid, 1, +1, h->g.batch * h->g.npair, h->g.nz, h->b.tw_n, h->tu, h->stream), "ifft y");
    if (st) return st;
  }
  ProfScope ps(h, kPIfftX);
  return dev_err(launch_fft_axis(h->g, h->b.grid, 0, +1, h->g.batch * h->g.npair, h->g.nz, h->b.tw_n, h->tu, h->stream), "ifft x");
}

est_status to_spectrum(est_handle h) {
  if (h->state == kSpectrum) return ok();
  if (h->state != kXY) return fail(EST_ESTATE, "needs estimator_transform first");
  ProfScope ps(h, kPFftZ);
  est_status st = dev_err(launch_fft_axis(h->g, h->b.grid, 2, -1, h->g.batch * h->g.npair, h->g.nz, h->b.tw_nz, h->tu, h->stream), "fft z");
  if (st) return st;
  h->state = kSpectrum;
  return ok();
}

// state after a forward pass (the last FFT axis is fused with the shell sums)
int forward_state(est_handle) { return kXY; }

est_status run_forward(est_handle h, const void* pos, est_dtype dt, const int64_t* offsets,
                       int64_t n_total, int n_dk, int n_bins, int sub, double* k, double* p,
                       int64_t* nm) {
  est_status st = run_deposit(h, pos, dt, offsets, n_total);
  if (st) return st;
  st = run_xy(h, -1);
  if (st) return st;
  ProfScope ps(h, kPPower);
  return dev_err(launch_power(h->g, h->b, h->tu, true, n_dk, n_bins, sub, k, p, nm, h->stream), "power");
}

}  // namespace

extern "C" {

const char* estimator_last_error(void) { return g_err; }

est_status estimator_workspace_bytes(const est_config* cfg, size_t* bytes) {
  est_status st = check_config(cfg);
  if (st) return st;
  if (!bytes) return fail(EST_EINVAL, "bytes is NULL");
  *bytes = layout(*cfg, nullptr, nullptr, nullptr);
  return ok();
}

est_status estimator_create(const est_config* cfg, void* workspace, size_t workspace_bytes,
                            void* stream, est_handle* out) {
  est_status st = check_config(cfg);
  if (st) return st;
  if (!out) return fail(EST_EINVAL, "out is NULL");
  *out = nullptr;
  if (!workspace) return fail(EST_EINVAL, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail(EST_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = layout(*cfg, nullptr, nullptr, nullptr);
  if (workspace_bytes < need)
    return fail(EST_ENOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
  est_ctx* h = new (std::nothrow) est_ctx();
  if (!h) return fail(EST_ENOMEM, "host allocation failed");
  h->cfg = *cfg;
  h->g = make_geom(*cfg);
  layout(*cfg, (char*)workspace, &h->b, &h->tune_out);
  h->stream = (hipStream_t)stream;
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
        cus > 0)
      h->tu.cus = cus;
  }
  clear_stale_error();
  // device address of the static workspace of estimator_direct_delta_noalloc
  // (once per device)
  st = dev_err(direct_static_scratch_init(h->device), "static workspace lookup");
  if (!st) st = dev_err(launch_tables(h->g, h->b, h->stream), "tables");
  if (st) {
    delete h;
    return st;
  }
  *out = h;
  return ok();
}

est_status estimator_destroy(est_handle h) {
  if (!h) return ok();
  for (auto& r : h->rec)
    for (auto& pr : r.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  delete h;
  return ok();
}

est_status estimator_deposit(est_handle h, const void* pos, est_dtype dtype, const int64_t* offsets,
                             int64_t n_total) {
  est_status st = check_handle(h);
  if (st) return st;
  if ((st = check_particles(h, pos, dtype, offsets, n_total))) return st;
  h->state = kCreated;
  if ((st = run_deposit(h, pos, dtype, offsets, n_total))) return st;
  h->state = kDeposited;
  return ok();
}

est_status estimator_transform(est_handle h) {
  est_status st = check_handle(h);
  if (st) return st;
  if (h->state != kDeposited) return fail(EST_ESTATE, "estimator_transform needs a fresh deposit");
  if ((st = run_xy(h, -1))) return st;
  h->state = kXY;
  return ok();
}

est_status estimator_power(est_handle h, int32_t n_dk, int32_t n_bins, int32_t subtract_shot,
                           double* k, double* p, int64_t* nmodes) {
  est_status st = check_handle(h);
  if (st) return st;
  if ((st = check_bins(h, n_dk, n_bins))) return st;
  if (!k || !p || !nmodes) return fail(EST_EINVAL, "output pointers must not be NULL");
  if (subtract_shot != 0 && subtract_shot != 1) return fail(EST_EINVAL, "subtract_shot must be 0 or 1");
  if (h->state != kXY && h->state != kSpectrum)
    return fail(EST_ESTATE, "estimator_power needs estimator_transform first");
  if ((st = ensure_modes(h, n_dk, n_bins))) return st;
  ProfScope ps(h, kPPower);
  return dev_err(launch_power(h->g, h->b, h->tu, h->state == kXY, n_dk, n_bins, subtract_shot, k, p,
                              nmodes, h->stream),
                 "power");
}

// Host checks shared by the bispectrum's size query and the call: shells
// below the triangle limit k_max = k_f N / 3 of Sec. 4.1, (n_bins + 1/2)
// n_dk < N/3.
static est_status check_bispec_bins(est_handle h, int32_t n_dk, int32_t n_bins, int64_t n_tri) {
  if (n_dk < 1) return fail(EST_EINVAL, "n_dk must be >= 1");
  if (n_bins < 1 || n_bins > kMaxBins) return fail(EST_EINVAL, "n_bins out of range");
  if (3LL * (2 * n_bins + 1) * n_dk >= 2LL * h->g.n)
    return fail(EST_EINVAL, "(n_bins + 1/2) n_dk must be < N/3 (triangle aliasing limit)");
  if (n_tri < 1) return fail(EST_EINVAL, "n_tri must be >= 1");
  return ok();
}

// the plan the caller's workspace is sized for: as many jobs as triangles,
// at most every job of n_bins shells
static est_status bispec_size_plan(est_handle h, int32_t n_dk, int32_t n_bins, int64_t n_tri,
                                   BsPlan* pl) {
  int64_t nj = bs_max_jobs(n_bins);
  if (nj > n_tri) nj = n_tri;
  if (!bs_plan(h->g.n, n_dk, n_bins, nj, n_tri, pl))
    return fail(EST_EUNSUPPORTED, "no alias-free field grid for these shells");
  return ok();
}

est_status estimator_bispectrum_workspace_bytes(est_handle h, int32_t n_dk, int32_t n_bins,
                                                int64_t n_tri, size_t* bytes) {
  est_status st = check_handle(h);
  if (st) return st;
  if (!bytes) return fail(EST_EINVAL, "bytes is NULL");
  if ((st = check_bispec_bins(h, n_dk, n_bins, n_tri))) return st;
  BsPlan pl;
  if ((st = bispec_size_plan(h, n_dk, n_bins, n_tri, &pl))) return st;
  *bytes = pl.bytes;
  return ok();
}

est_status estimator_bispectrum(est_handle h, int32_t mock, int32_t n_dk, int32_t n_bins,
                                const int32_t* tri_host, int64_t n_tri, void* bws, size_t bws_bytes,
                                double* bk, double* ntri) {
  est_status st = check_handle(h);
  if (st) return st;
  const Geom& g = h->g;
  if (mock < 0 || mock >= g.batch) return fail(EST_EINVAL, "mock out of range");
  if (!tri_host || n_tri < 1) return fail(EST_EINVAL, "triangles missing");
  if ((st = check_bispec_bins(h, n_dk, n_bins, n_tri))) return st;
  if (!bws || !bk || !ntri) return fail(EST_EINVAL, "NULL device pointer");
  if (((uintptr_t)bws & 255) != 0) return fail(EST_EINVAL, "bispectrum workspace must be 256-byte aligned");
  for (int64_t t = 0; t < n_tri; ++t) {
    const int32_t a = tri_host[3 * t], b = tri_host[3 * t + 1], c = tri_host[3 * t + 2];
    if (!(1 <= c && c <= b && b <= a && a <= n_bins))
      return fail(EST_EINVAL, "triangle %lld must satisfy 1 <= b3 <= b2 <= b1 <= n_bins", (long long)t);
  }
  BsPlan sized;
  if ((st = bispec_size_plan(h, n_dk, n_bins, n_tri, &sized))) return st;
  if (bws_bytes < sized.bytes)
    return fail(EST_ENOMEM, "bispectrum workspace too small: %zu < %zu", bws_bytes, sized.bytes);
  // this call's tile jobs and the entry of every triangle; the plan with the
  // actual job count fits in the sized workspace
  std::vector<int32_t> jobs, tmap;
  bs_jobs(tri_host, n_tri, jobs, tmap);
  const int64_t njobs = (int64_t)jobs.size() / 4;
  BsPlan pl;
  if (!bs_plan(g.n, n_dk, n_bins, njobs, n_tri, &pl))
    return fail(EST_EUNSUPPORTED, "no alias-free field grid for these shells");
  if ((st = to_spectrum(h))) return st;
  char* base = (char*)bws;
  double* run_i = (double*)(base + pl.off_run);
  double* run_j = run_i + njobs * 256;
  if ((st = dev_err(hipMemcpyAsync(base + pl.off_jobs, jobs.data(), jobs.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, h->stream), "copy jobs")) ||
      (st = dev_err(hipMemcpyAsync(base + pl.off_tmap, tmap.data(), tmap.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, h->stream), "copy triangle map")))
    return st;
  {
    ProfScope ps(h, kPBispec);
    if ((st = dev_err(launch_bs_setup(g, h->b, mock, n_dk, n_bins, pl, base, h->stream), "delta cube")))
      return st;
  }
  // slab by slab: the fields, then their triple sums
  auto sums = [&](bool counts, double* run) -> est_status {
    for (int sl = 0; sl < pl.nslab; ++sl) {
      est_status e;
      {
        ProfScope ps(h, kPBsFields);
        if ((e = dev_err(launch_bs_fields(n_dk, n_bins, pl, base, counts, sl, h->stream), "shell fields")))
          return e;
      }
      ProfScope ps(h, kPBsTriple);
      if ((e = dev_err(launch_bs_triple(n_bins, pl, base, sl == 0, run, h->stream), "triple sums")))
        return e;
    }
    return EST_OK;
  };
  if ((st = sums(false, run_i))) return st;
  // the counts' sums depend only on the grid M, the shells and the jobs:
  // computed on the first call and kept by the handle
  const bool cached = h->bs_M == pl.M && h->bs_dk == n_dk && h->bs_nbins == n_bins &&
                      h->bs_jobs == jobs && h->bs_runj.size() == (size_t)njobs * 256;
  if (cached) {
    if ((st = dev_err(hipMemcpyAsync(run_j, h->bs_runj.data(), h->bs_runj.size() * sizeof(double),
                                     hipMemcpyHostToDevice, h->stream), "cached counts")))
      return st;
  } else {
    h->bs_M = 0;
    if ((st = sums(true, run_j))) return st;
    std::vector<double> runj((size_t)njobs * 256);
    if ((st = dev_err(hipMemcpyAsync(runj.data(), run_j, runj.size() * sizeof(double),
                                     hipMemcpyDeviceToHost, h->stream), "keep counts")) ||
        (st = dev_err(hipStreamSynchronize(h->stream), "synchronize")))
      return st;
    h->bs_runj.swap(runj);
    h->bs_jobs = jobs;
    h->bs_M = pl.M;
    h->bs_dk = n_dk;
    h->bs_nbins = n_bins;
  }
  {
    ProfScope ps(h, kPBispec);
    if ((st = dev_err(launch_bs_finalize(pl, base, n_tri, g.box * g.box * g.box, bk, ntri, h->stream),
                      "bispectrum")))
      return st;
  }
  // the host job and triangle buffers must outlive their copies
  return dev_err(hipStreamSynchronize(h->stream), "synchronize");
}

est_status estimator_backward(est_handle h, const void* pos, est_dtype dtype, const int64_t* offsets,
                              int64_t n_total, const double* dldp, int32_t n_dk, int32_t n_bins,
                              void* grad) {
  est_status st = check_handle(h);
  if (st) return st;
  if ((st = check_particles(h, pos, dtype, offsets, n_total))) return st;
  if ((st = check_bins(h, n_dk, n_bins))) return st;
  if (!dldp || !grad) return fail(EST_EINVAL, "NULL device pointer");
  if ((st = ensure_modes(h, n_dk, n_bins))) return st;
  h->state = kCreated;
  if ((st = run_deposit(h, pos, dtype, offsets, n_total))) return st;
  if ((st = run_xy(h, -1))) return st;
  if (h->g.npair > 1) {
    // more than two grids: separate z passes around the gradient spectra
    h->state = kXY;
    if ((st = to_spectrum(h))) return st;
    {
      ProfScope ps(h, kPAdjoint);
      if ((st = dev_err(launch_multi_adjoint(h->g, h->b, dldp, n_dk, n_bins, h->stream), "adjoint spectrum")))
        return st;
    }
    ProfScope ps(h, kPFftZ);
    if ((st = dev_err(launch_fft_axis(h->g, h->b.grid, 2, +1, h->g.batch * h->g.npair, h->g.nz,
                                      h->b.tw_nz, h->tu, h->stream), "ifft z")))
      return st;
  } else {
    ProfScope ps(h, kPAdjoint);
    if ((st = dev_err(launch_adjoint_spectrum(h->g, h->b, h->tu, dldp, n_dk, n_bins, h->stream), "adjoint spectrum")))
      return st;
  }
  if ((st = run_xy(h, +1))) return st;
  {
    ProfScope ps(h, kPGather);
    if ((st = dev_err(launch_gather_grad(h->g, pos, dtype, offsets, n_total, h->weights, h->b, grad,
                                                    h->stream), "gather")))
      return st;
  }
  h->state = kCreated;  // the grid now holds dL/drho, not a density
  return ok();
}

est_status estimator_graph_capture(est_handle h, const void* pos, est_dtype dtype, const int64_t* offsets,
                                   int64_t n_total, int32_t n_dk, int32_t n_bins, int32_t subtract_shot,
                                   double* k, double* p, int64_t* nmodes) {
  est_status st = check_handle(h);
  if (st) return st;
  if ((st = check_particles(h, pos, dtype, offsets, n_total))) return st;
  if ((st = check_bins(h, n_dk, n_bins))) return st;
  if (!k || !p || !nmodes) return fail(EST_EINVAL, "output pointers must not be NULL");
  if (subtract_shot != 0 && subtract_shot != 1) return fail(EST_EINVAL, "subtract_shot must be 0 or 1");
  if ((st = ensure_modes(h, n_dk, n_bins))) return st;
  // one eager run (also sets kernel attributes outside the capture)
  if ((st = run_forward(h, pos, dtype, offsets, n_total, n_dk, n_bins, subtract_shot, k, p, nmodes)))
    return st;
  if ((st = dev_err(hipStreamSynchronize(h->stream), "synchronize"))) return st;
  if (h->exec) { (void)hipGraphExecDestroy(h->exec); h->exec = nullptr; }
  if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
  hipStream_t cs;
  if ((st = dev_err(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream"))) return st;
  hipStream_t saved = h->stream;
  h->stream = cs;
  h->capturing = true;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = run_forward(h, pos, dtype, offsets, n_total, n_dk, n_bins, subtract_shot, k, p, nmodes);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (st == EST_OK && e2 != hipSuccess) st = dev_err(e2, "end capture");
    if (st == EST_OK) {
      h->graph = graph;
      st = dev_err(hipGraphInstantiate(&h->exec, graph, nullptr, nullptr, 0), "instantiate graph");
    } else if (graph) {
      (void)hipGraphDestroy(graph);
    }
  } else {
    st = dev_err(e, "begin capture");
  }
  h->stream = saved;
  h->capturing = false;
  (void)hipStreamDestroy(cs);
  h->state = (st == EST_OK) ? forward_state(h) : kCreated;
  return st;
}

est_status estimator_graph_launch(est_handle h) {
  est_status st = check_handle(h);
  if (st) return st;
  if (!h->exec) return fail(EST_ESTATE, "no captured graph");
  if ((st = dev_err(hipGraphLaunch(h->exec, h->stream), "graph launch"))) return st;
  h->state = forward_state(h);
  return ok();
}

static Tune tune_from_index(const int* id, int cus) {
  static const int vals_cols[2] = {8, 16};
  static const int vals_bins[3] = {256, 1024, 2048};
  static const int vals_dep[2] = {512, 1024};
  Tune t;
  t.cus = cus;
  t.cols_c = vals_cols[id[0]];
  t.bin_blocks = vals_bins[id[1]];
  t.dep_threads = vals_dep[id[2]];
  t.dep_narrow = id[3];
  t.dep_xcd = id[4];
  return t;
}

est_status estimator_set_launch(est_handle h, int32_t choice) {
  est_status st = check_handle(h);
  if (st) return st;
  if (choice < 0 || choice >= 48) return fail(EST_EINVAL, "launch choice must be in [0, 48)");
  int id[5];
  id[4] = choice % 2;
  id[3] = (choice / 2) % 2;
  id[2] = (choice / 4) % 2;
  id[1] = (choice / 8) % 3;
  id[0] = choice / 24;
  h->tu = tune_from_index(id, h->tu.cus);
  return ok();
}

est_status estimator_set_weights(est_handle h, const float* weights) {
  est_status st = check_handle(h);
  if (st) return st;
  if (!(h->cfg.flags & EST_FLAG_WEIGHTS))
    return fail(EST_EINVAL, "the handle was created without EST_FLAG_WEIGHTS");
  h->weights = weights;
  return ok();
}

est_status estimator_autotune(est_handle h, const void* pos, est_dtype dtype, const int64_t* offsets,
                              int64_t n_total, int32_t n_dk, int32_t n_bins, int32_t iters, int32_t* choice) {
  est_status st = check_handle(h);
  if (st) return st;
  if ((st = check_particles(h, pos, dtype, offsets, n_total))) return st;
  if ((st = check_bins(h, n_dk, n_bins))) return st;
  if (iters < 1 || iters > 1000) return fail(EST_EINVAL, "iters must be 1..1000");
  if ((st = ensure_modes(h, n_dk, n_bins))) return st;
  // coordinate descent over the launch-shape parameters: each parameter in
  // turn takes the value with the shortest measured pipeline, the others
  // fixed at their current best
  const size_t per = (size_t)h->g.batch * n_bins;
  double* kk = (double*)h->tune_out;
  double* pp = kk + per;
  int64_t* nm = (int64_t*)(pp + per);
  hipEvent_t e0, e1;
  if ((st = dev_err(hipEventCreate(&e0), "event"))) return st;
  if ((st = dev_err(hipEventCreate(&e1), "event"))) { (void)hipEventDestroy(e0); return st; }
  const Tune saved = h->tu;
  auto measure = [&](const Tune& t, float* ms) -> est_status {
    h->tu = t;
    est_status s2 = run_forward(h, pos, dtype, offsets, n_total, n_dk, n_bins, 0, kk, pp, nm);
    if (s2) return s2;
    if ((s2 = dev_err(hipEventRecord(e0, h->stream), "event record"))) return s2;
    for (int it = 0; it < iters && s2 == EST_OK; ++it)
      s2 = run_forward(h, pos, dtype, offsets, n_total, n_dk, n_bins, 0, kk, pp, nm);
    if (s2) return s2;
    if ((s2 = dev_err(hipEventRecord(e1, h->stream), "event record"))) return s2;
    if ((s2 = dev_err(hipEventSynchronize(e1), "synchronize"))) return s2;
    return dev_err(hipEventElapsedTime(ms, e0, e1), "elapsed time");
  };
  int idx[5] = {1, 1, 0, 1, 1};  // start from the defaults
  const int cus = h->tu.cus;
  auto make = [&](const int* id) { return tune_from_index(id, cus); };
  // the 32-bit deposit format (parameter 3) is not a launch shape: it stays
  // on (it is used only when provably safe, and is then always the faster)
  const int nvals[5] = {2, 3, 2, 1, 2};
  float best_ms = 1e30f;
  if (st == EST_OK) st = measure(make(idx), &best_ms);
  for (int p = 0; p < 5 && st == EST_OK; ++p) {
    if (nvals[p] < 2) continue;
    int best_v = idx[p];
    for (int v = 0; v < nvals[p] && st == EST_OK; ++v) {
      if (v == idx[p]) continue;
      int trial[5];
      for (int q = 0; q < 5; ++q) trial[q] = idx[q];
      trial[p] = v;
      float ms = 0.f;
      st = measure(make(trial), &ms);
      if (st == EST_OK && ms < best_ms) { best_ms = ms; best_v = v; }
    }
    idx[p] = best_v;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->tu = (st == EST_OK) ? make(idx) : saved;
  h->state = (st == EST_OK) ? forward_state(h) : kCreated;
  if (st == EST_OK && choice) *choice = (((idx[0] * 3 + idx[1]) * 2 + idx[2]) * 2 + idx[3]) * 2 + idx[4];
  return st;
}

est_status estimator_copy_grid(est_handle h, int32_t which, int32_t mock, float* dst) {
  est_status st = check_handle(h);
  if (st) return st;
  if (which < 1 || which > h->g.ng)
    return fail(EST_EINVAL, "which must be 1..%d (grids of this handle)", h->g.ng);
  if (mock < 0 || mock >= h->g.batch) return fail(EST_EINVAL, "mock out of range");
  if (!dst) return fail(EST_EINVAL, "dst is NULL");
  if (h->state != kDeposited) return fail(EST_ESTATE, "grids are only available right after a deposit");
  return dev_err(launch_copy_grid(h->g, h->b, which, mock, dst, h->stream), "copy grid");
}

est_status estimator_sample_delta(est_handle h, int32_t mock, const int32_t* modes, int64_t n, double* out) {
  est_status st = check_handle(h);
  if (st) return st;
  if (mock < 0 || mock >= h->g.batch) return fail(EST_EINVAL, "mock out of range");
  if (!modes || !out || n < 1) return fail(EST_EINVAL, "modes/out missing");
  if ((st = to_spectrum(h))) return st;
  return dev_err(launch_sample_delta(h->g, h->b, mock, modes, n, out, h->stream), "sample delta");
}

est_status estimator_direct_workspace_bytes(est_handle h, int64_t n, size_t* bytes) {
  est_status st = check_handle(h);
  if (st) return st;
  if (!bytes) return fail(EST_EINVAL, "bytes is NULL");
  if (n < 1 || n > 2147483647LL) return fail(EST_EINVAL, "n must be 1..2^31-1");
  *bytes = direct_workspace(h->g.n, n);
  return ok();
}

est_status estimator_direct_delta(est_handle h, const void* pos, est_dtype dtype, int64_t n,
                                  void* dws, size_t dws_bytes, double* out) {
  est_status st = check_handle(h);
  if (st) return st;
  if (!pos || !out || !dws) return fail(EST_EINVAL, "pos, dws and out are required");
  if (dtype != EST_F32 && dtype != EST_F64) return fail(EST_EINVAL, "dtype must be EST_F32 or EST_F64");
  if (n < 1 || n > 2147483647LL) return fail(EST_EINVAL, "n must be 1..2^31-1");
  if (((uintptr_t)dws & 255) != 0) return fail(EST_EINVAL, "dws must be 256-byte aligned");
  const size_t need = direct_workspace(h->g.n, n);
  if (dws_bytes < need) return fail(EST_ENOMEM, "direct workspace too small: %zu < %zu", dws_bytes, need);
  ProfScope ps(h, kPDirect);
  return dev_err(launch_direct(h->g, pos, dtype, n, h->weights, dws, out, h->stream), "direct sum");
}

est_status estimator_direct_delta_noalloc(est_handle h, const void* pos, est_dtype dtype, int64_t n,
                                          double* out) {
  est_status st = check_handle(h);
  if (st) return st;
  if (!pos || !out) return fail(EST_EINVAL, "pos and out are required");
  if (dtype != EST_F32 && dtype != EST_F64) return fail(EST_EINVAL, "dtype must be EST_F32 or EST_F64");
  if (n < 1 || n > 2147483647LL) return fail(EST_EINVAL, "n must be 1..2^31-1");
  const size_t need = direct_workspace(h->g.n, n);
  if (need > kDirectStaticBytes)
    return fail(EST_ENOMEM,
                "direct sum of %lld particles on N = %d needs %zu bytes of workspace, more than the "
                "%zu-byte static workspace of estimator_direct_delta_noalloc",
                (long long)n, h->g.n, need, kDirectStaticBytes);
  void* ws = direct_static_scratch(h->device);
  if (!ws) return fail(EST_EDEVICE, "static workspace not set up on device %d", h->device);
  clear_stale_error();
  return dev_err(launch_direct(h->g, pos, dtype, n, h->weights, ws, out, h->stream), "direct sum");
}

est_status estimator_export_delta(est_handle h, int32_t mock, double* out) {
  est_status st = check_handle(h);
  if (st) return st;
  if (mock < 0 || mock >= h->g.batch) return fail(EST_EINVAL, "mock out of range");
  if (!out) return fail(EST_EINVAL, "out is NULL");
  if ((st = to_spectrum(h))) return st;
  return dev_err(launch_export_delta(h->g, h->b, mock, out, h->stream), "export delta");
}

est_status estimator_spectrum_power(est_handle h, const double* a, const double* b, int32_t n_dk,
                                    int32_t n_bins, double shot, double* k, double* p,
                                    int64_t* nmodes) {
  est_status st = check_handle(h);
  if (st) return st;
  if (!a || !k || !p || !nmodes) return fail(EST_EINVAL, "a, k, p and nmodes are required");
  if (!std::isfinite(shot)) return fail(EST_EINVAL, "shot must be finite");
  if ((st = check_bins(h, n_dk, n_bins))) return st;
  if ((st = ensure_modes(h, n_dk, n_bins))) return st;
  return dev_err(launch_spectrum_power(h->g, h->b, a, b, n_dk, n_bins, shot, k, p, nmodes, h->stream),
                 "spectrum power");
}

est_status estimator_profile(est_handle h, int32_t enable) {
  est_status st = check_handle(h);
  if (st) return st;
  if (enable != 0 && enable != 1) return fail(EST_EINVAL, "enable must be 0 or 1");
  if (enable) {
    if ((st = dev_err(hipStreamSynchronize(h->stream), "synchronize"))) return st;
    prof_fold(h);
    for (auto& r : h->rec) {
      r.total_ms = 0.0;
      r.launches = 0;
    }
  }
  h->prof = enable != 0;
  return ok();
}

est_status estimator_profile_read(est_handle h, int32_t idx, char* name, size_t name_len,
                                  double* total_ms, int64_t* launches, int32_t* n_labels) {
  est_status st = check_handle(h);
  if (st) return st;
  if (n_labels) *n_labels = kPNumLabels;
  if (idx < 0 || idx >= kPNumLabels) return fail(EST_EINVAL, "label index out of range");
  if ((st = dev_err(hipStreamSynchronize(h->stream), "synchronize"))) return st;
  prof_fold(h);
  if (name && name_len > 0) {
    strncpy(name, kProfNames[idx], name_len - 1);
    name[name_len - 1] = '\0';
  }
  if (total_ms) *total_ms = h->rec[idx].total_ms;
  if (launches) *launches = h->rec[idx].launches;
  return ok();
}

}  // extern "C"
