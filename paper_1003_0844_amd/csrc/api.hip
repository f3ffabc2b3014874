// The C ABI of include/fstat.h: validation, plan state, workspace and the
// launch sequence of a grid call.  Host code only; every arithmetic step of the
// method runs in the kernels of sky.hip, grid.hip, prep.hip and grad.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/fstat.h"
#include "internal.h"
#include "persist_sched.h"

namespace {
// A roctx range over one call of the library (rocprofv3 --marker-trace shows
// it beside the kernels; without a tracer attached it costs a function call).
struct Range {
  explicit Range(const char* what) { roctxRangePushA(what); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};
}  // namespace

namespace {

constexpr double C_LIGHT = 299792458.0;
constexpr double TWO_PI = 6.283185307179586476925286766559;

struct SegPlan {
  SegDev dev{};
  int B2 = 0;
  int node_cap = 16;  // nodes per FFT batch
  int streams = 1;    // 1: both FFT passes on the caller's stream; 2: pass 2 on the side stream
  void* twC = nullptr;
  void* twR = nullptr;
  void* twlo = nullptr;
  void* twhi = nullptr;
  double* x = nullptr;
  float* xf = nullptr;
  double* y = nullptr;
  float* yf = nullptr;
  double* M = nullptr;
  float* Mf = nullptr;
  uint8_t* mask = nullptr;
  double* mom = nullptr;  // SegDev::mom
};

struct ProfPair {
  hipEvent_t a, b;
  int kind;
  double bytes;
};
struct ProfKind {
  int64_t launches = 0;
  double ms = 0.0;
  double bytes = 0.0;
};
struct Prof {
  bool on = false;
  std::vector<ProfPair> pending, pool;
  ProfKind kinds[4];
};

}  // namespace

struct fstat_plan_s {
  Prof prof;
  int device = 0;
  int interp = 1;
  int prec = 0;
  int max_batch = 0;
  std::vector<SegPlan> segs;
  SegDev* d_segs = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  hipStream_t side = nullptr;  // second stream of the grid pipeline (default priority)
  int force_streams = 0;  // FSTAT_STREAMS: 1 or 2 for every segment, 0 = per segment
  hipEvent_t ev_p1[2] = {nullptr, nullptr}, ev_p2[2] = {nullptr, nullptr}, ev_sky[2] = {nullptr, nullptr};
  hipEvent_t ev_join = nullptr;
  bool capturing = false;  // a graph capture is recording the launch sequence
  int launch = 0;                // FSTAT_LAUNCH_PASSES / FSTAT_LAUNCH_PERSISTENT
  uint32_t* d_error = nullptr;   // sticky error flag of persistent launches
  int persist_blocks[3] = {0, 0, 0};  // resident workgroups of the persistent kernel per output mode
  int persist_slots = 128;       // spill slots of a persistent launch (FSTAT_PERSIST_SLOTS)
  int persist_chunk = 32;        // tiles a workgroup of the persistent kernel claims at once (FSTAT_PERSIST_CHUNK)
  uint64_t spin_ticks = 0;       // wall-clock ticks a wait of the persistent kernel may last
};

// A grid call recorded once as a HIP graph, with a workspace of its own.
struct fstat_graph_s {
  fstat_plan_s* plan = nullptr;
  void* ws = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

fstat_status from_hip(hipError_t e) {
  if (e == hipSuccess) return FSTAT_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return FSTAT_ENOMEM;
  return FSTAT_EDEVICE;
}

#define HIP_TRY(expr)                               \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return from_hip(e_);      \
  } while (0)

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}
double frac_turns(double v) {
  double f = v - std::floor(v);
  return f >= 1.0 ? 0.0 : f;
}

// nfft = R * C for the two FFT passes
void choose_split(int prec, int64_t nfft, int& R, int& C) {
  int64_t c = prec == 0 ? 4096 : 2048;
  if (nfft / 16 < c) c = nfft / 16;
  if (nfft / c > 1024) c = nfft / 1024;
  C = (int)c;
  R = (int)(nfft / c);
}

size_t elem_real(int prec) { return prec == 0 ? 4 : 8; }

// FFT split of a segment: first pass over R columns of length C, second pass
// over length R in blocks of B2 columns.
void apply_split(SegPlan& sp, int prec, int C) {
  SegDev& d = sp.dev;
  d.C = C;
  d.R = (int)(d.nfft / C);
  d.Ceff = (int)((d.n + d.R - 1) / d.R);
  sp.B2 = fsk::pass2_b2(prec, d.R);
}

bool split_valid(int prec, int64_t nfft, int C) {
  const int64_t R = nfft / C;
  const int64_t cmax = prec == 0 ? 4096 : 4096;
  return C >= 64 && C <= cmax && R >= 16 && R <= 1024 && (int64_t)C * R == nfft;
}

hipError_t make_split_tables(const SegPlan& sp, int prec, hipStream_t st) {
  hipError_t e = fsk::make_twiddles(prec, sp.dev.C, sp.dev.C, 1, sp.twC, st);
  if (e == hipSuccess) e = fsk::make_twiddles(prec, sp.dev.R, sp.dev.R, 1, sp.twR, st);
  return e;
}

void free_seg(SegPlan& s) {
  void* ptrs[] = {s.twC, s.twR, s.twlo, s.twhi, s.x, s.xf, s.y, s.yf, s.M, s.Mf, s.mask, s.mom};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  s = SegPlan{};
}

void destroy_plan(fstat_plan_s* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  for (auto& s : p->segs) free_seg(s);
  if (p->d_segs) (void)hipFree(p->d_segs);
  if (p->ws) (void)hipFree(p->ws);
  if (p->pinned) (void)hipHostFree(p->pinned);
  if (p->staged) (void)hipEventDestroy(p->staged);
  if (p->d_error) (void)hipFree(p->d_error);
  for (hipEvent_t ev : {p->ev_p1[0], p->ev_p1[1], p->ev_p2[0], p->ev_p2[1], p->ev_sky[0], p->ev_sky[1], p->ev_join})
    if (ev) (void)hipEventDestroy(ev);
  if (p->side) (void)hipStreamDestroy(p->side);
  for (auto* v : {&p->prof.pending, &p->prof.pool})
    for (auto& pr : *v) {
      (void)hipEventDestroy(pr.a);
      (void)hipEventDestroy(pr.b);
    }
  (void)hipSetDevice(cur);
  delete p;
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = 0;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    ok = hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (ok) (void)hipSetDevice(prev);
  }
};

fstat_status validate_segment(const fstat_segment& s, const fstat_ephemeris& eph, int prec) {
  if (!s.x || s.n <= 0 || !(s.dt > 0.0) || !std::isfinite(s.dt) || s.n_sidereal_days <= 0 ||
      !std::isfinite(s.f_ref_hz) || !std::isfinite(s.t0) || !std::isfinite(s.sigma2))
    return FSTAT_EINVAL;
  if (s.n < 16) return FSTAT_EUNSUPPORTED;
  if (std::fabs((double)s.n * s.dt - (double)s.n_sidereal_days * eph.sidereal_day_s) > 0.5 * s.dt)
    return FSTAT_ENOTINTDAYS;
  const int64_t nfft = s.nfft ? s.nfft : next_pow2(2 * s.n);
  if (nfft < 0) return FSTAT_EINVAL;
  if (!is_pow2(nfft) || nfft < s.n || nfft < (1 << 10) || nfft > (1 << 22)) return FSTAT_EUNSUPPORTED;
  for (int64_t i = 0; i < s.n; ++i)
    if (!std::isfinite(s.x[i])) return FSTAT_EINVAL;
  if (s.mask) {  // a segment made only of gaps has no data (A = B = 0)
    int64_t kept = 0;
    for (int64_t i = 0; i < s.n && kept == 0; ++i) kept += s.mask[i] != 0;
    if (kept == 0) return FSTAT_EINVAL;
  }
  (void)prec;
  return FSTAT_OK;
}

fstat_status build_segment(const fstat_segment& s, const fstat_detector& det, const fstat_ephemeris& eph, int prec,
                           int interp, SegPlan& sp) {
  const int64_t n = s.n;
  const int64_t nfft = s.nfft ? s.nfft : next_pow2(2 * n);
  SegDev& d = sp.dev;
  // geometry constants (turns for the angles, light-seconds for distances)
  d.geo.orb_r = eph.orbit_radius_m / C_LIGHT;
  d.geo.orb_rate_c = eph.orbit_omega / TWO_PI;
  d.geo.orb_c0 = frac_turns(eph.orbit_phase0 / TWO_PI + s.t0 * d.geo.orb_rate_c);
  d.geo.site_rc = det.radius_m * std::cos(det.lat_rad) / C_LIGHT;
  d.geo.site_rz = det.radius_m * std::sin(det.lat_rad) / C_LIGHT;
  d.geo.sid_rate_c = 1.0 / eph.sidereal_day_s;
  d.geo.sid_c0 = frac_turns((eph.gmst0_rad + det.lon_rad) / TWO_PI + s.t0 / eph.sidereal_day_s);
  d.geo.cth0 = std::cos(TWO_PI * d.geo.sid_c0);
  d.geo.sth0 = std::sin(TWO_PI * d.geo.sid_c0);
  d.geo.ceps = std::cos(eph.obliquity_rad);
  d.geo.seps = std::sin(eph.obliquity_rad);
  d.geo.sin_zeta = std::sin(det.zeta_rad);
  d.geo.s2g = std::sin(2.0 * det.gamma_rad);
  d.geo.c2g = std::cos(2.0 * det.gamma_rad);
  d.geo.sl = std::sin(det.lat_rad);
  d.geo.cl = std::cos(det.lat_rad);
  d.geo.s2l = std::sin(2.0 * det.lat_rad);
  d.geo.c2l = std::cos(2.0 * det.lat_rad);
  d.n = n;
  d.dt = s.dt;
  d.f_ref = s.f_ref_hz;
  d.nfft = nfft;
  int R, C;
  choose_split(prec, nfft, R, C);
  apply_split(sp, prec, C);
  d.interp = interp;

  const size_t er = elem_real(prec);
  double* xraw = nullptr;
  void* work = nullptr;
  double* dvar = nullptr;
  double* mpart = nullptr;
  fstat_status rc = FSTAT_OK;
  auto fail = [&](hipError_t e) {
    rc = from_hip(e);
    return rc;
  };
  hipError_t e = hipSuccess;
  do {
    if ((e = hipMalloc(&xraw, n * sizeof(double))) != hipSuccess) break;
    if ((e = hipMalloc(&sp.x, n * sizeof(double))) != hipSuccess) break;
    if ((e = hipMalloc(&sp.xf, n * sizeof(float))) != hipSuccess) break;
    if ((e = hipMemcpy(xraw, s.x, n * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) break;
    if (s.mask) {
      if ((e = hipMalloc(&sp.mask, n)) != hipSuccess) break;
      if ((e = hipMemcpy(sp.mask, s.mask, n, hipMemcpyHostToDevice)) != hipSuccess) break;
    }
    if ((e = fsk::prep_mask(xraw, sp.mask, n, sp.x, sp.xf, nullptr)) != hipSuccess) break;
    // the mask moments that give every sky position's A, B, C
    d.mask = sp.mask;
    if ((e = hipMalloc(&sp.mom, 10 * sizeof(double))) != hipSuccess) break;
    if ((e = hipMalloc(&mpart, (size_t)fsk::mask_moment_blocks(d) * 9 * sizeof(double))) != hipSuccess) break;
    if ((e = fsk::mask_moments(d, mpart, sp.mom, nullptr)) != hipSuccess) break;
    double sigma2 = s.sigma2;
    if (!(sigma2 > 0.0)) {
      if ((e = hipMalloc(&dvar, sizeof(double))) != hipSuccess) break;
      if ((e = fsk::prep_variance(xraw, sp.mask, n, dvar, nullptr)) != hipSuccess) break;
      if ((e = hipMemcpy(&sigma2, dvar, sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) break;
      if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) {
        rc = FSTAT_EINVAL;
        break;
      }
    }
    d.sigma2 = sigma2;
    if (interp != FSTAT_NEAREST) {
      if ((e = hipMalloc(&sp.y, 2 * n * sizeof(double))) != hipSuccess) break;
      if ((e = hipMalloc(&sp.yf, 2 * n * sizeof(float))) != hipSuccess) break;
      if (interp == FSTAT_CUBIC_UP2) {
        if ((e = hipMalloc(&sp.M, 2 * n * sizeof(double))) != hipSuccess) break;
        if ((e = hipMalloc(&sp.Mf, 2 * n * sizeof(float))) != hipSuccess) break;
      }
      if ((e = hipMalloc(&work, fsk::prep_work_bytes(n))) != hipSuccess) break;
      if ((e = fsk::prep_upsample(sp.x, n, interp, sp.y, sp.yf, sp.M, sp.Mf, work, nullptr)) != hipSuccess) break;
    }
    // twiddle tables in the working precision
    const int64_t nlo = nfft < 4096 ? nfft : 4096;
    const int64_t nhi = nfft / 4096 > 1 ? nfft / 4096 : 1;
    // (room for every split the tuner may choose: C <= 4096, R <= 1024)
    if ((e = hipMalloc(&sp.twC, 4096 * 2 * er)) != hipSuccess) break;
    if ((e = hipMalloc(&sp.twR, 1024 * 2 * er)) != hipSuccess) break;
    if ((e = hipMalloc(&sp.twlo, 4096 * 2 * er)) != hipSuccess) break;
    if ((e = hipMalloc(&sp.twhi, nhi * 2 * er)) != hipSuccess) break;
    if ((e = make_split_tables(sp, prec, nullptr)) != hipSuccess) break;
    if ((e = fsk::make_twiddles(prec, nfft, nlo, 1, sp.twlo, nullptr)) != hipSuccess) break;
    if ((e = fsk::make_twiddles(prec, nfft, nhi, 4096, sp.twhi, nullptr)) != hipSuccess) break;
    if ((e = hipDeviceSynchronize()) != hipSuccess) break;
  } while (0);
  if (e != hipSuccess) fail(e);
  (void)hipDeviceSynchronize();
  if (xraw) (void)hipFree(xraw);
  if (work) (void)hipFree(work);
  if (dvar) (void)hipFree(dvar);
  if (mpart) (void)hipFree(mpart);
  d.x = sp.x;
  d.xf = sp.xf;
  d.y = sp.y;
  d.yf = sp.yf;
  d.M = sp.M;
  d.Mf = sp.Mf;
  d.mask = sp.mask;
  d.mom = sp.mom;
  return rc;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
fstat_status ensure_ws(fstat_plan_s* p, size_t bytes) {
  if (p->ws_bytes >= bytes) return FSTAT_OK;
  HIP_TRY(hipDeviceSynchronize());
  if (p->ws) (void)hipFree(p->ws);
  p->ws = nullptr;
  p->ws_bytes = 0;
  HIP_TRY(hipMalloc(&p->ws, bytes));
  p->ws_bytes = bytes;
  return FSTAT_OK;
}

fstat_status ensure_pinned(fstat_plan_s* p, size_t bytes) {
  if (p->staged_pending) {
    HIP_TRY(hipEventSynchronize(p->staged));
    p->staged_pending = false;
  }
  if (p->pinned_bytes >= bytes) return FSTAT_OK;
  if (p->pinned) (void)hipHostFree(p->pinned);
  p->pinned = nullptr;
  p->pinned_bytes = 0;
  HIP_TRY(hipHostMalloc(&p->pinned, bytes, hipHostMallocDefault));
  p->pinned_bytes = bytes;
  return FSTAT_OK;
}

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Launch through f(); when profiling is on, bracket it with two events.
template <class F>
hipError_t timed(fstat_plan_s* p, int kind, double bytes, hipStream_t st, F&& f) {
  if (!p->prof.on || p->capturing) return f();
  ProfPair pr{};
  if (!p->prof.pool.empty()) {
    pr = p->prof.pool.back();
    p->prof.pool.pop_back();
  } else {
    hipError_t e = hipEventCreate(&pr.a);
    if (e == hipSuccess) e = hipEventCreate(&pr.b);
    if (e != hipSuccess) return e;
  }
  pr.kind = kind;
  pr.bytes = bytes;
  hipError_t e = hipEventRecord(pr.a, st);
  if (e == hipSuccess) e = f();
  if (e == hipSuccess) e = hipEventRecord(pr.b, st);
  if (e != hipSuccess) {
    p->prof.pool.push_back(pr);
    return e;
  }
  p->prof.pending.push_back(pr);
  return hipSuccess;
}

struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    T* r = (T*)(base + off);
    off = align_up(off + count * sizeof(T));
    return r;
  }
};

// one unit of work: a batch of sky positions of one segment, and its nodes
struct SkyBatch {
  int seg;
  int sky0, nsky;    // into the call's sky list (alpha, delta pairs)
  int node0, nnode;  // into the call's NodeDev list (sky = index within the batch)
};

}  // namespace

// Host-side schedule of a grid call: nodes grouped by segment and sky position
// into batches, and the workspace layout they need.
struct GridSched {
  std::vector<double> sky_ad;   // (alpha, delta) per sky of the call
  std::vector<NodeDev> ndev;    // per node, grouped by batch
  std::vector<SkyBatch> batches;
  size_t max_quads = 0, max_spill = 0, max_part = 0;
  int max_sky = 0;
  size_t desc_bytes = 0;        // sky list + node list, staged at the start of the workspace
  size_t need_ws = 0;
};

void schedule_grid(const fstat_plan_s* p, const fstat_node* nodes, int64_t n_nodes, GridSched& gs) {
  const int prec = p->prec;
  std::vector<int64_t> order(n_nodes);
  for (int64_t i = 0; i < n_nodes; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    const fstat_node &x = nodes[a], &y = nodes[b];
    if (x.seg != y.seg) return x.seg < y.seg;
    if (x.alpha != y.alpha) return x.alpha < y.alpha;
    return x.delta < y.delta;
  });
  std::vector<double>& sky_ad = gs.sky_ad;
  std::vector<NodeDev>& ndev = gs.ndev;
  std::vector<SkyBatch>& batches = gs.batches;
  int64_t i = 0;
  while (i < n_nodes) {
    const int sg = nodes[order[i]].seg;
    const SegDev& d = p->segs[sg].dev;
    const size_t quad_bytes = (size_t)d.R * d.Ceff * 4 * elem_real(prec);
    int sky_cap = (int)std::max<size_t>(1, std::min<size_t>(64, ((size_t)1 << 30) / quad_bytes));
    SkyBatch b{sg, (int)(sky_ad.size() / 2), 0, (int)ndev.size(), 0};
    while (i < n_nodes && nodes[order[i]].seg == sg) {
      const fstat_node& nd = nodes[order[i]];
      const bool new_sky = b.nsky == 0 || sky_ad[sky_ad.size() - 2] != nd.alpha || sky_ad.back() != nd.delta;
      if (new_sky) {
        if (b.nsky == sky_cap) {
          batches.push_back(b);
          b = SkyBatch{sg, (int)(sky_ad.size() / 2), 0, (int)ndev.size(), 0};
        }
        sky_ad.push_back(nd.alpha);
        sky_ad.push_back(nd.delta);
        ++b.nsky;
      }
      ndev.push_back(NodeDev{nd.fdot, (double)nd.bin_offset / (double)d.nfft, b.nsky - 1, (int32_t)order[i]});
      ++b.nnode;
      ++i;
    }
    batches.push_back(b);
  }
  // workspace: descriptors; two sets of sky data (one per sky-batch parity);
  // two spill buffers and two sets of max partials (one per node-chunk parity)
  for (const auto& bt : batches) {
    const SegPlan& sp = p->segs[bt.seg];
    const SegDev& d = sp.dev;
    gs.max_quads = std::max(gs.max_quads, (size_t)bt.nsky * d.R * d.Ceff * 4 * elem_real(prec));
    gs.max_spill = std::max(gs.max_spill, (size_t)sp.node_cap * d.nfft * 4 * elem_real(prec));
    gs.max_part = std::max(gs.max_part, (size_t)sp.node_cap * (d.C / sp.B2) * sizeof(MaxPartial));
    gs.max_sky = std::max(gs.max_sky, bt.nsky);
  }
  gs.desc_bytes = align_up(sky_ad.size() * sizeof(double)) + align_up(ndev.size() * sizeof(NodeDev));
  const size_t set_bytes =
      align_up(gs.max_quads) + align_up(gs.max_sky * sizeof(SkyConst)) + align_up(gs.max_sky * sizeof(SkyCoef));
  gs.need_ws = gs.desc_bytes + 2 * set_bytes + 2 * align_up(gs.max_spill) + 2 * align_up(gs.max_part + 16) + 4096;
}

// Copy the call's descriptors (sky list, node list) into host memory laid out
// as the start of the workspace.
void pack_descriptors(const GridSched& gs, char* hp) {
  std::memcpy(hp, gs.sky_ad.data(), gs.sky_ad.size() * sizeof(double));
  std::memcpy(hp + align_up(gs.sky_ad.size() * sizeof(double)), gs.ndev.data(), gs.ndev.size() * sizeof(NodeDev));
}

// The launch sequence of a grid call on stream st; ws holds gs.need_ws bytes
// whose first gs.desc_bytes are the staged descriptors.
fstat_status launch_grid(fstat_plan_s* p, const GridSched& gs, void* ws, const fstat_out* out, hipStream_t st) {
  const int prec = p->prec;
  const std::vector<SkyBatch>& batches = gs.batches;
  const size_t max_quads = gs.max_quads, max_spill = gs.max_spill, max_part = gs.max_part;
  const int max_sky = gs.max_sky;
  Carve cv{(char*)ws};
  double* d_ad = cv.take<double>(gs.sky_ad.size());
  NodeDev* d_nodes = cv.take<NodeDev>(gs.ndev.size());
  struct SkySet {
    void* quads;
    SkyConst* sky;
    SkyCoef* coef;
  } sets[2];
  for (auto& ss : sets) {
    ss.quads = cv.take<char>(max_quads);
    ss.sky = cv.take<SkyConst>(max_sky);
    ss.coef = cv.take<SkyCoef>(max_sky);
  }
  void* d_spill[2];
  d_spill[0] = cv.take<char>(max_spill);
  d_spill[1] = cv.take<char>(max_spill);
  MaxPartial* d_part[2];
  d_part[0] = cv.take<MaxPartial>(max_part / sizeof(MaxPartial) + 1);
  d_part[1] = cv.take<MaxPartial>(max_part / sizeof(MaxPartial) + 1);
  GridOut go{};
  go.mode = out->mode;
  go.interbin = out->interbin;
  go.k_lo = out->k_lo;
  go.k_hi = out->k_hi;
  go.threshold = out->threshold;
  go.F = out->F;
  go.Fmax = out->Fmax;
  go.kmax = out->kmax;
  go.xing = out->crossings;
  go.n_xing = out->n_crossings;
  go.max_xing = out->max_crossings;
  if (out->mode == 2) HIP_TRY(fsk::zero_u64(out->n_crossings, st));

  // The sky preparation and the first FFT pass run on the caller's stream; the
  // second pass runs there too (one-stream segments) or on the plan's side
  // stream (two-stream segments), where pass 1 of chunk c+1 overlaps pass 2 of
  // chunk c.  Chunk c uses spill buffer and max partials c % 2; sky batch s
  // uses sky set s % 2.  Chunk c's pass 2 may run beside chunk c+1's (when c
  // is on the side stream and c+1 on the caller's), so nothing chunk-level is
  // shared between consecutive chunks; every reuse of a buffer (by chunk c+2,
  // sky batch s+2) waits for an event recorded on the stream that last read
  // it, so segments of either kind may follow each other in any order.
  bool used_side = false;
  const double er = (double)elem_real(prec);
  int64_t chunk = 0;
  int sbi = 0;
  for (const auto& b : batches) {
    const SegPlan& sp = p->segs[b.seg];
    const SegDev& d = sp.dev;
    const SkySet& ss = sets[sbi % 2];
    hipStream_t s2 = sp.streams == 2 ? p->side : st;
    used_side = used_side || sp.streams == 2;
    const int64_t qstride = (int64_t)d.R * d.Ceff;
    const double rec_bytes = 4.0 * er * (double)qstride;  // one sky record
    if (sbi >= 2) HIP_TRY(hipStreamWaitEvent(st, p->ev_sky[sbi % 2], 0));
    HIP_TRY(timed(p, FSTAT_K_OTHER, 0.0, st, [&] { return fsk::sky_setup(d_ad + 2 * b.sky0, b.nsky, d, ss.sky, st); }));
    HIP_TRY(timed(p, FSTAT_K_SKY, rec_bytes * b.nsky, st, [&] {
      return fsk::sky_prep(prec, d, ss.sky, b.nsky, ss.quads, qstride, st);
    }));
    HIP_TRY(timed(p, FSTAT_K_OTHER, 0.0, st, [&] { return fsk::sky_finalize(d, ss.sky, b.nsky, ss.coef, st); }));
    const int node_cap = sp.node_cap;
    for (int n0 = 0; n0 < b.nnode; n0 += node_cap, ++chunk) {
      const int nn = std::min(node_cap, b.nnode - n0);
      const NodeDev* dn = d_nodes + b.node0 + n0;
      void* spill = d_spill[chunk % 2];
      const double sbytes = 4.0 * er * (double)d.nfft * nn;
      const double ibf = out->interbin ? 2.0 : 1.0;  // outputs per bin
      const double outb = out->mode == 0 ? ibf * er * (double)(out->k_hi - out->k_lo) * nn : 0.0;
      const double p2read = out->interbin ? sbytes * (sp.B2 + 1) / sp.B2 : sbytes;
      if (chunk >= 2) HIP_TRY(hipStreamWaitEvent(st, p->ev_p2[chunk % 2], 0));
      HIP_TRY(timed(p, FSTAT_K_PASS1, sbytes + rec_bytes * nn / std::max(1, b.nnode / b.nsky), st, [&] {
        return fsk::grid_pass1(prec, d.C, d, ss.quads, qstride, ss.sky, dn, nn, sp.twC, sp.twlo, sp.twhi, spill, st);
      }));
      HIP_TRY(hipEventRecord(p->ev_p1[chunk % 2], st));
      HIP_TRY(hipStreamWaitEvent(s2, p->ev_p1[chunk % 2], 0));
      HIP_TRY(timed(p, FSTAT_K_PASS2, p2read + outb, s2, [&] {
        return fsk::grid_pass2(prec, d.R, d, spill, dn, nn, ss.coef, sp.twR, go, d_part[chunk % 2], s2);
      }));
      if (out->mode == 1)
        HIP_TRY(timed(p, FSTAT_K_OTHER, 0.0, s2,
                      [&] { return fsk::max_finalize(d_part[chunk % 2], d.C / sp.B2, dn, nn, prec, go, s2); }));
      HIP_TRY(hipEventRecord(p->ev_p2[chunk % 2], s2));
    }
    HIP_TRY(hipEventRecord(p->ev_sky[sbi % 2], s2));  // sky set free once its last pass 2 is done
    ++sbi;
  }
  if (used_side) {
    HIP_TRY(hipEventRecord(p->ev_join, p->side));
    HIP_TRY(hipStreamWaitEvent(st, p->ev_join, 0));
  }
  return FSTAT_OK;
}

// An eager grid call: schedule, stage the descriptors through pinned memory,
// launch.
fstat_status run_grid(fstat_plan_s* p, const fstat_node* nodes, int64_t n_nodes, const fstat_out* out,
                      hipStream_t st) {
  GridSched gs;
  schedule_grid(p, nodes, n_nodes, gs);
  fstat_status rc = ensure_ws(p, gs.need_ws);
  if (rc != FSTAT_OK) return rc;
  rc = ensure_pinned(p, gs.desc_bytes);
  if (rc != FSTAT_OK) return rc;
  pack_descriptors(gs, (char*)p->pinned);
  HIP_TRY(hipMemcpyAsync(p->ws, p->pinned, gs.desc_bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(p->staged, st));
  p->staged_pending = true;
  return launch_grid(p, gs, p->ws, out, st);
}


// ---------------------------------------------------------------------------
// autotuner: FFT split and node-batch size per segment
// ---------------------------------------------------------------------------
// A persistent plan splits FP32 segments of 2^18 <= nfft <= 2^22 with C = 4096
// (R = nfft / 4096 in [64, 1024]): the shapes the persistent kernel holds.
bool persistent_split(const fstat_plan_s* p, int64_t nfft) {
  return p->launch == FSTAT_LAUNCH_PERSISTENT && p->prec == 0 && nfft >= (1 << 18) && nfft <= (1 << 22);
}

// ---------------------------------------------------------------------------
// the persistent launch: host layout of the work queue
// ---------------------------------------------------------------------------
// Calls the persistent kernel runs: FP32, no interbinning, every segment of
// the call split with C = 4096 (64 <= R <= 1024).
// kPersistentEnabled gates the dispatch (false: every call runs as passes).
constexpr bool kPersistentEnabled = true;

bool persistent_call(const fstat_plan_s* p, const fstat_node* nodes, int64_t n_nodes, const fstat_out* out) {
  if (!kPersistentEnabled) return false;
  if (p->launch != FSTAT_LAUNCH_PERSISTENT || p->prec != 0 || out->interbin) return false;
  for (int64_t i = 0; i < n_nodes; ++i) {
    const SegDev& d = p->segs[nodes[i].seg].dev;
    if (d.C != 4096 || d.R < 64 || d.R > 1024) return false;
  }
  return true;
}

// The launches of a persistent call on st (counters cleared, crossing counter
// cleared, the kernel); ws holds ps.need_ws bytes starting with the packed
// descriptors.
fstat_status launch_persistent(fstat_plan_s* p, const PersistSched& ps, void* ws, const fstat_out* out,
                               hipStream_t st) {
  const int mode = out->mode;
  if (p->persist_blocks[mode] <= 0) {
    p->persist_blocks[mode] = fsk::persistent_blocks(mode);
    if (p->persist_blocks[mode] <= 0) return FSTAT_EDEVICE;
  }
  Carve cv{(char*)ws};
  PersistArgs a{};
  a.sky_ad = cv.take<double>(ps.sky_ad.size());
  a.nodes = cv.take<NodeDev>(ps.ndev.size());
  a.node_batch = cv.take<int32_t>(ps.node_batch.size());
  a.batches = cv.take<PBatch>(ps.batches.size());
  a.units = cv.take<PUnit>(ps.units.size());
  a.tw = cv.take<PSegTw>(ps.tw.size());
  for (int k = 0; k < 2; ++k) {
    a.quads[k] = cv.take<char>(ps.max_quads);
    a.sky[k] = cv.take<SkyConst>(ps.max_sky);
    a.coef[k] = cv.take<SkyCoef>(ps.max_sky);
  }
  a.spill = cv.take<Pair<float>>((size_t)ps.nslots * ps.slot_elems);
  a.cnt = cv.take<uint32_t>(ps.nzero);
  a.best = reinterpret_cast<unsigned long long*>(a.cnt + ps.best_off);
  a.head = cv.take<unsigned long long>(1);
  a.chunk = p->persist_chunk;
  a.segs = p->d_segs;
  a.nitems = (int64_t)ps.units.size() * PUNIT;
  a.nbatch = (int32_t)ps.batches.size();
  a.nslots = ps.nslots;
  a.slot_elems = ps.slot_elems;
  a.error = p->d_error;
  a.spin_ticks = p->spin_ticks;
  GridOut& go = a.out;
  go.mode = out->mode;
  go.interbin = 0;
  go.k_lo = out->k_lo;
  go.k_hi = out->k_hi;
  go.threshold = out->threshold;
  go.F = out->F;
  go.Fmax = out->Fmax;
  go.kmax = out->kmax;
  go.xing = out->crossings;
  go.n_xing = out->n_crossings;
  go.max_xing = out->max_crossings;
  HIP_TRY(fsk::persist_zero(a.cnt, ps.nzero, a.head, st));
  if (out->mode == 2) HIP_TRY(fsk::zero_u64(out->n_crossings, st));
  return from_hip(fsk::grid_persistent(a, mode, p->persist_blocks[mode], st));
}

std::vector<SegShape> seg_shapes(const fstat_plan_s* p) {
  std::vector<SegShape> v(p->segs.size());
  for (size_t s = 0; s < p->segs.size(); ++s) {
    const SegPlan& sp = p->segs[s];
    v[s] = SegShape{sp.dev.nfft, sp.dev.R, sp.dev.Ceff, PSegTw{sp.twC, sp.twR, sp.twlo, sp.twhi}};
  }
  return v;
}

fstat_status run_persistent(fstat_plan_s* p, const fstat_node* nodes, int64_t n_nodes, const fstat_out* out,
                            hipStream_t st) {
  PersistSched ps;
  schedule_persistent(seg_shapes(p), p->persist_slots, nodes, n_nodes, ps);
  if (!ps.ordered) return FSTAT_EUNSUPPORTED;
  fstat_status rc = ensure_ws(p, ps.need_ws);
  if (rc != FSTAT_OK) return rc;
  rc = ensure_pinned(p, ps.desc_bytes);
  if (rc != FSTAT_OK) return rc;
  pack_persistent(ps, (char*)p->pinned);
  HIP_TRY(hipMemcpyAsync(p->ws, p->pinned, ps.desc_bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(p->staged, st));
  p->staged_pending = true;
  return launch_persistent(p, ps, p->ws, out, st);
}

struct TuneKey {
  int prec, interp;
  int64_t nfft, n;
};

bool cache_lookup(const TuneKey& k, int& C, int& batch, int& streams) {
  const char* path = std::getenv("FSTAT_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    int pr, ip, c, b, ns;
    long long nf, nn;
    if (std::sscanf(line, "fstat-tune-v3 %d %d %lld %lld %d %d %d", &pr, &ip, &nf, &nn, &c, &b, &ns) == 7 &&
        pr == k.prec && ip == k.interp && nf == k.nfft && nn == k.n) {
      C = c;
      batch = b;
      streams = ns;
      found = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const TuneKey& k, int C, int batch, int streams) {
  const char* path = std::getenv("FSTAT_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "fstat-tune-v3 %d %d %lld %lld %d %d %d\n", k.prec, k.interp, (long long)k.nfft, (long long)k.n,
               C, batch, streams);
  std::fclose(f);
}

// Times every valid (C, batch, streams) on a 64-sky (FP64: 8-sky) x 16-spindown
// sample of the segment (full map into a scratch buffer) and keeps the fastest.  After a
// warm-up, the candidates are timed in two sweeps, in order and then in
// reverse order, three runs per visit after one untimed run; a candidate's
// time is its fastest run, so that neither the clock ramp at the start nor
// drift during the sweep favours a position in the list.  The default
// schedule (timed first) stays unless the fastest is at least 3 % faster, so
// that timing noise does not pick a schedule that is no better.
fstat_status tune_segment(fstat_plan_s* p, int si) {
  SegPlan& sp = p->segs[si];
  const int prec = p->prec;
  const int64_t nfft = sp.dev.nfft;
  const TuneKey key{prec, p->interp, nfft, sp.dev.n};
  int C = sp.dev.C, batch = sp.node_cap, streams = sp.streams;
  if (cache_lookup(key, C, batch, streams) && split_valid(prec, nfft, C) && batch > 0 &&
      (streams == 1 || streams == 2) && (!persistent_split(p, nfft) || C == 4096)) {
    apply_split(sp, prec, C);
    sp.node_cap = batch;
    sp.streams = p->force_streams ? p->force_streams : streams;
    HIP_TRY(make_split_tables(sp, prec, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return FSTAT_OK;
  }
  // the default first: split of choose_split, largest batch; a persistent plan
  // keeps C = 4096 where its kernel applies
  std::vector<int> cands = {sp.dev.C};
  for (int c : {4096, 2048, 1024})
    if (split_valid(prec, nfft, c) && std::find(cands.begin(), cands.end(), c) == cands.end()) cands.push_back(c);
  if (persistent_split(p, nfft)) cands = {4096};
  std::vector<int> batches;
  if (p->max_batch > 0) batches = {p->max_batch};
  else if (prec == 0) batches = {256, 128, 64, 32};
  else batches = {8, 4, 2};
  // one stream first (the two passes in turn), then two (pass 2 of a batch
  // beside pass 1 of the next)
  std::vector<int> stream_modes;
  if (p->force_streams) stream_modes = {p->force_streams};
  else stream_modes = {1, 2};
  // FP64 runs ~30x slower per node: a smaller sample keeps its tuning short
  const int nsky = prec == 0 ? 64 : 8, nfd = 16;
  std::vector<fstat_node> nodes(nsky * nfd);
  for (int s = 0; s < nsky; ++s)
    for (int f = 0; f < nfd; ++f) {
      fstat_node& nd = nodes[s * nfd + f];
      nd.alpha = 0.4 + 0.09 * s;
      nd.delta = -1.2 + 2.4 * s / (nsky - 1);
      nd.fdot = -1e-9 * f / (nfd - 1);
      nd.seg = si;
      nd.bin_offset = 0.0f;
    }
  const int64_t kh = nfft / 2;
  void* scratch = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t ea = nullptr, eb = nullptr;
  fstat_status rc = FSTAT_OK;
  hipError_t e = hipMalloc(&scratch, (size_t)nodes.size() * kh * elem_real(prec));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&ea);
  if (e == hipSuccess) e = hipEventCreate(&eb);
  if (e != hipSuccess) rc = from_hip(e);
  fstat_out out{};
  out.mode = FSTAT_OUT_MAP;
  out.k_lo = 0;
  out.k_hi = kh;
  out.F = scratch;
  struct Cand {
    int C, batch, streams;
    double ms;
  };
  std::vector<Cand> cs;
  for (int c : cands)
    for (int b : batches)
      for (int ns : stream_modes) cs.push_back(Cand{c, b, ns, 1e300});
  int cur_C = -1;
  // one visit: switch to the candidate, one untimed run, then `timed` timed runs
  auto visit = [&](Cand& c, int timed) -> fstat_status {
    if (c.C != cur_C) {
      apply_split(sp, prec, c.C);
      hipError_t e2 = make_split_tables(sp, prec, st);
      if (e2 != hipSuccess) return from_hip(e2);
      cur_C = c.C;
    }
    sp.node_cap = c.batch;
    sp.streams = c.streams;
    for (int rep = 0; rep <= timed; ++rep) {
      hipError_t e2 = hipEventRecord(ea, st);
      if (e2 != hipSuccess) return from_hip(e2);
      fstat_status r2 = run_grid(p, nodes.data(), (int64_t)nodes.size(), &out, st);
      if (r2 != FSTAT_OK) return r2;
      if ((e2 = hipEventRecord(eb, st)) != hipSuccess || (e2 = hipEventSynchronize(eb)) != hipSuccess)
        return from_hip(e2);
      float ms = 0.f;
      if ((e2 = hipEventElapsedTime(&ms, ea, eb)) != hipSuccess) return from_hip(e2);
      if (rep > 0) c.ms = std::min(c.ms, (double)ms);  // rep 0 warms up
    }
    return FSTAT_OK;
  };
  if (rc == FSTAT_OK) {  // warm-up: clocks up, workspace allocated
    Cand w = cs[0];
    rc = visit(w, 3);
  }
  for (size_t k = 0; rc == FSTAT_OK && k < 2 * cs.size(); ++k)
    rc = visit(cs[k < cs.size() ? k : 2 * cs.size() - 1 - k], 3);
  int best = 0;
  for (size_t k = 1; k < cs.size(); ++k)
    if (cs[k].ms < cs[best].ms) best = (int)k;
  if (!(cs[best].ms < 0.97 * cs[0].ms)) best = 0;
  const int best_C = cs[best].C, best_b = cs[best].batch, best_s = cs[best].streams;
  (void)hipDeviceSynchronize();
  if (scratch) (void)hipFree(scratch);
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  if (st) (void)hipStreamDestroy(st);
  apply_split(sp, prec, best_C);
  sp.node_cap = best_b;
  sp.streams = best_s;
  if (rc != FSTAT_OK) return rc;
  HIP_TRY(make_split_tables(sp, prec, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  cache_store(key, best_C, best_b, best_s);
  return FSTAT_OK;
}

// ===========================================================================
extern "C" {

const char* fstat_strerror(fstat_status s) {
  switch (s) {
    case FSTAT_OK: return "ok";
    case FSTAT_EINVAL: return "invalid argument";
    case FSTAT_ENOTINTDAYS: return "observation time is not a whole number of sidereal days";
    case FSTAT_ENOMEM: return "out of memory";
    case FSTAT_EDEVICE: return "HIP device error";
    case FSTAT_EUNSUPPORTED: return "unsupported size";
    default: return "unknown status";
  }
}

fstat_status fstat_plan(const fstat_segment* segs, int32_t nseg, const fstat_detector* det,
                        const fstat_ephemeris* eph, const fstat_options* opt, fstat_plan_t* out) {
  Range rg("fstat_plan");
  if (!segs || nseg <= 0 || !det || !eph || !opt || !out) return FSTAT_EINVAL;
  if (opt->interp < 0 || opt->interp > 2 || opt->prec < 0 || opt->prec > 1 || opt->max_batch < 0 ||
      opt->max_batch > 256 || opt->autotune < 0 || opt->autotune > 1 ||
      (opt->launch != FSTAT_LAUNCH_PASSES && opt->launch != FSTAT_LAUNCH_PERSISTENT))
    return FSTAT_EINVAL;
  if (!(eph->sidereal_day_s > 0.0) || !std::isfinite(eph->orbit_radius_m) || !std::isfinite(eph->orbit_omega) ||
      !std::isfinite(det->radius_m) || !std::isfinite(det->lat_rad))
    return FSTAT_EINVAL;
  for (int i = 0; i < nseg; ++i) {
    fstat_status v = validate_segment(segs[i], *eph, opt->prec);
    if (v != FSTAT_OK) return v;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return FSTAT_EDEVICE;
  if (opt->device < 0 || opt->device >= ndev) return FSTAT_EINVAL;
  DeviceGuard guard(opt->device);
  if (!guard.ok) return FSTAT_EDEVICE;

  fstat_plan_s* p = new (std::nothrow) fstat_plan_s();
  if (!p) return FSTAT_ENOMEM;
  p->device = opt->device;
  p->interp = opt->interp;
  p->prec = opt->prec;
  p->max_batch = opt->max_batch;
  p->launch = opt->launch;
  if (const char* sl = std::getenv("FSTAT_PERSIST_SLOTS")) {
    const int v = std::atoi(sl);
    if (v >= 3 && v <= 128) p->persist_slots = v;
  }
  if (const char* ch = std::getenv("FSTAT_PERSIST_CHUNK")) {
    const int v = std::atoi(ch);
    if (v >= 1 && v <= PUNIT && PUNIT % v == 0) p->persist_chunk = v;
  }
  p->segs.resize(nseg);
  for (int i = 0; i < nseg; ++i) {
    fstat_status rc = build_segment(segs[i], *det, *eph, opt->prec, opt->interp, p->segs[i]);
    if (rc != FSTAT_OK) {
      destroy_plan(p);
      return rc;
    }
  }
  for (auto& sp : p->segs) {
    sp.node_cap = opt->max_batch > 0 ? opt->max_batch : (opt->prec == 0 ? 16 : 4);
    if (persistent_split(p, sp.dev.nfft) && sp.dev.C != 4096) {
      apply_split(sp, opt->prec, 4096);
      if (make_split_tables(sp, opt->prec, nullptr) != hipSuccess) {
        destroy_plan(p);
        return FSTAT_EDEVICE;
      }
    }
  }
  if (const char* s1 = std::getenv("FSTAT_STREAMS")) {
    if (s1[0] == '1') p->force_streams = 1;
    if (s1[0] == '2') p->force_streams = 2;
  }
  if (p->force_streams)
    for (auto& sp : p->segs) sp.streams = p->force_streams;
  hipError_t e = hipEventCreateWithFlags(&p->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&p->d_error, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(p->d_error, 0, sizeof(uint32_t));
  if (e == hipSuccess) {
    int khz = 0;
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, opt->device);
    p->spin_ticks = (uint64_t)(khz > 0 ? khz : 100000) * 2000ull;  // 2 s
    // a shorter bound (0: a wait not satisfied at once expires), for tests of the error path
    if (const char* sp = std::getenv("FSTAT_PERSIST_SPIN_TICKS")) {
      char* end = nullptr;
      const long long v = std::strtoll(sp, &end, 10);
      if (end != sp && v >= 0) p->spin_ticks = std::min<uint64_t>(p->spin_ticks, (uint64_t)v);
    }
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
  for (hipEvent_t* ev : {&p->ev_p1[0], &p->ev_p1[1], &p->ev_p2[0], &p->ev_p2[1], &p->ev_sky[0], &p->ev_sky[1], &p->ev_join})
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    destroy_plan(p);
    return from_hip(e);
  }
  if (opt->autotune) {
    for (int i = 0; i < nseg; ++i) {
      // segments of equal length and FFT size share one tuning run
      int same = -1;
      for (int j = 0; j < i && same < 0; ++j)
        if (p->segs[j].dev.nfft == p->segs[i].dev.nfft && p->segs[j].dev.n == p->segs[i].dev.n) same = j;
      fstat_status rc = FSTAT_OK;
      if (same >= 0) {
        apply_split(p->segs[i], opt->prec, p->segs[same].dev.C);
        p->segs[i].node_cap = p->segs[same].node_cap;
        p->segs[i].streams = p->segs[same].streams;
        rc = from_hip(make_split_tables(p->segs[i], opt->prec, nullptr));
      } else {
        rc = tune_segment(p, i);
      }
      if (rc != FSTAT_OK) {
        destroy_plan(p);
        return rc;
      }
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      destroy_plan(p);
      return from_hip(e);
    }
  }
  std::vector<SegDev> hs(nseg);
  for (int i = 0; i < nseg; ++i) hs[i] = p->segs[i].dev;
  e = hipMalloc(&p->d_segs, nseg * sizeof(SegDev));
  if (e == hipSuccess) e = hipMemcpy(p->d_segs, hs.data(), nseg * sizeof(SegDev), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    destroy_plan(p);
    return from_hip(e);
  }
  *out = p;
  return FSTAT_OK;
}

fstat_status fstat_plan_schedule(fstat_plan_t p, int32_t seg, int32_t* R, int32_t* C, int32_t* B2, int32_t* batch,
                                 int32_t* streams) {
  if (!p || seg < 0 || seg >= (int32_t)p->segs.size()) return FSTAT_EINVAL;
  const SegPlan& sp = p->segs[seg];
  if (R) *R = sp.dev.R;
  if (C) *C = sp.dev.C;
  if (B2) *B2 = sp.B2;
  if (batch) *batch = sp.node_cap;
  if (streams) *streams = sp.streams;
  return FSTAT_OK;
}

void fstat_destroy(fstat_plan_t p) { destroy_plan(p); }

fstat_status fstat_plan_status(fstat_plan_t p) {
  if (!p) return FSTAT_EINVAL;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  HIP_TRY(hipDeviceSynchronize());
  uint32_t flag = 0;
  HIP_TRY(hipMemcpy(&flag, p->d_error, sizeof(flag), hipMemcpyDeviceToHost));
  if (flag == 0) return FSTAT_OK;
  HIP_TRY(hipMemset(p->d_error, 0, sizeof(uint32_t)));
  return FSTAT_EDEVICE;
}

fstat_status fstat_plan_info(fstat_plan_t p, int32_t seg, int64_t* n, int64_t* nfft, double* sigma2, int32_t* R,
                             int32_t* C) {
  if (!p || seg < 0 || seg >= (int32_t)p->segs.size()) return FSTAT_EINVAL;
  const SegDev& d = p->segs[seg].dev;
  if (n) *n = d.n;
  if (nfft) *nfft = d.nfft;
  if (sigma2) *sigma2 = d.sigma2;
  if (R) *R = d.R;
  if (C) *C = d.C;
  return FSTAT_OK;
}

}  // extern "C"

namespace {
fstat_status check_grid_args(const fstat_plan_s* p, const fstat_node* nodes, int64_t n_nodes, const fstat_out* out) {
  if (!p || !nodes || n_nodes <= 0 || !out) return FSTAT_EINVAL;
  if (n_nodes > (int64_t)INT32_MAX) return FSTAT_EUNSUPPORTED;
  if (out->mode < 0 || out->mode > 2) return FSTAT_EINVAL;
  if (out->interbin != 0 && out->interbin != 1) return FSTAT_EINVAL;
  if (out->k_lo < 0 || out->k_hi <= out->k_lo) return FSTAT_EINVAL;
  if (out->mode == 0 && !out->F) return FSTAT_EINVAL;
  if (out->mode == 1 && (!out->Fmax || !out->kmax)) return FSTAT_EINVAL;
  if (out->mode == 2 && (!out->n_crossings || (out->max_crossings > 0 && !out->crossings) || out->max_crossings < 0))
    return FSTAT_EINVAL;
  const int nseg = (int)p->segs.size();
  for (int64_t i = 0; i < n_nodes; ++i) {
    const fstat_node& nd = nodes[i];
    if (nd.seg < 0 || nd.seg >= nseg || !std::isfinite(nd.alpha) || !std::isfinite(nd.delta) ||
        !std::isfinite(nd.fdot) || !(std::fabs(nd.bin_offset) < 1.0f))
      return FSTAT_EINVAL;
    if (out->k_hi > p->segs[nd.seg].dev.nfft / 2) return FSTAT_EINVAL;
  }
  return FSTAT_OK;
}

void destroy_graph(fstat_graph_s* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->ws) (void)hipFree(g->ws);
  delete g;
}
}  // namespace

extern "C" {

fstat_status fstat_grid(fstat_plan_t p, const fstat_node* nodes, int64_t n_nodes, const fstat_out* out,
                        void* hip_stream) {
  Range rg("fstat_grid");
  fstat_status rc = check_grid_args(p, nodes, n_nodes, out);
  if (rc != FSTAT_OK) return rc;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  if (persistent_call(p, nodes, n_nodes, out)) return run_persistent(p, nodes, n_nodes, out, (hipStream_t)hip_stream);
  return run_grid(p, nodes, n_nodes, out, (hipStream_t)hip_stream);
}

fstat_status fstat_graph_create(fstat_plan_t p, const fstat_node* nodes, int64_t n_nodes, const fstat_out* out,
                                fstat_graph_t* g_out) {
  Range rg("fstat_graph_create");
  if (!g_out) return FSTAT_EINVAL;
  fstat_status rc = check_grid_args(p, nodes, n_nodes, out);
  if (rc != FSTAT_OK) return rc;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  const bool persist = persistent_call(p, nodes, n_nodes, out);
  GridSched gs;
  PersistSched ps;
  if (persist) {
    schedule_persistent(seg_shapes(p), p->persist_slots, nodes, n_nodes, ps);
    if (!ps.ordered) return FSTAT_EUNSUPPORTED;
  } else {
    schedule_grid(p, nodes, n_nodes, gs);
  }
  fstat_graph_s* g = new (std::nothrow) fstat_graph_s;
  if (!g) return FSTAT_ENOMEM;
  g->plan = p;
  std::vector<char> desc(persist ? ps.desc_bytes : gs.desc_bytes);
  if (persist) pack_persistent(ps, desc.data());
  else pack_descriptors(gs, desc.data());
  hipStream_t cs = nullptr;
  hipError_t e = hipMalloc(&g->ws, persist ? ps.need_ws : gs.need_ws);
  if (e == hipSuccess) e = hipMemcpy(g->ws, desc.data(), desc.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess && persist && p->persist_blocks[out->mode] <= 0)  // occupancy query outside the capture
    p->persist_blocks[out->mode] = fsk::persistent_blocks(out->mode);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    p->capturing = true;
    rc = persist ? launch_persistent(p, ps, g->ws, out, cs) : launch_grid(p, gs, g->ws, out, cs);
    p->capturing = false;
    e = hipStreamEndCapture(cs, &g->graph);  // ends the capture whatever launch_grid returned
    if (rc == FSTAT_OK && e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  }
  if (cs) (void)hipStreamDestroy(cs);
  if (rc == FSTAT_OK && e != hipSuccess) rc = from_hip(e);
  if (rc != FSTAT_OK) {
    destroy_graph(g);
    return rc;
  }
  *g_out = g;
  return FSTAT_OK;
}

fstat_status fstat_graph_launch(fstat_graph_t g, void* hip_stream) {
  Range rg("fstat_graph_launch");
  if (!g || !g->exec) return FSTAT_EINVAL;
  DeviceGuard guard(g->plan->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)hip_stream));
  return FSTAT_OK;
}

void fstat_graph_destroy(fstat_graph_t g) {
  if (!g) return;
  DeviceGuard guard(g->plan->device);
  (void)hipDeviceSynchronize();
  destroy_graph(g);
}

fstat_status fstat_profile(fstat_plan_t p, int32_t enable) {
  if (!p) return FSTAT_EINVAL;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  HIP_TRY(hipDeviceSynchronize());
  for (auto& pr : p->prof.pending) p->prof.pool.push_back(pr);
  p->prof.pending.clear();
  for (auto& k : p->prof.kinds) k = ProfKind{};
  p->prof.on = enable != 0;
  return FSTAT_OK;
}

fstat_status fstat_profile_read(fstat_plan_t p, int32_t kind, int64_t* launches, double* ms, double* bytes) {
  if (!p || kind < 0 || kind >= 4) return FSTAT_EINVAL;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  HIP_TRY(hipDeviceSynchronize());
  for (auto& pr : p->prof.pending) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, pr.a, pr.b));
    ProfKind& k = p->prof.kinds[pr.kind];
    k.launches += 1;
    k.ms += t;
    k.bytes += pr.bytes;
    p->prof.pool.push_back(pr);
  }
  p->prof.pending.clear();
  const ProfKind& k = p->prof.kinds[kind];
  if (launches) *launches = k.launches;
  if (ms) *ms = k.ms;
  if (bytes) *bytes = k.bytes;
  return FSTAT_OK;
}

fstat_status fstat_eval(fstat_plan_t p, const double* params, const int32_t* seg, int64_t n, double* F,
                        double* state, void* hip_stream) {
  if (!p || !params || n <= 0 || !F) return FSTAT_EINVAL;
  if (n > (int64_t)INT32_MAX) return FSTAT_EUNSUPPORTED;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  return from_hip(fsk::grad_forward(p->d_segs, (int)p->segs.size(), seg, params, n, F, state, (hipStream_t)hip_stream));
}

fstat_status fstat_adjoint(fstat_plan_t p, const double* params, const int32_t* seg, int64_t n, const double* state,
                           const double* gF, double* dparams, void* hip_stream) {
  if (!p || !params || n <= 0 || !state || !dparams) return FSTAT_EINVAL;
  if (n > (int64_t)INT32_MAX) return FSTAT_EUNSUPPORTED;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  return from_hip(fsk::grad_adjoint(p->d_segs, (int)p->segs.size(), seg, params, n, state, gF, dparams, (hipStream_t)hip_stream));
}

fstat_status fstat_eval_exact(fstat_plan_t p, const double* params, const int32_t* seg, int64_t n, double* F,
                              void* hip_stream) {
  if (!p || !params || n <= 0 || !F) return FSTAT_EINVAL;
  if (n > (int64_t)INT32_MAX) return FSTAT_EUNSUPPORTED;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  return from_hip(fsk::eval_exact(p->d_segs, (int)p->segs.size(), seg, params, n, F, (hipStream_t)hip_stream));
}

fstat_status fstat_refine(fstat_plan_t p, const double* params, const int32_t* seg, int64_t n,
                          const fstat_refine_options* opt, double* params_out, double* F_out, int32_t* evals_out,
                          void* hip_stream) {
  if (!p || !params || n <= 0 || !opt || !params_out || !F_out) return FSTAT_EINVAL;
  if (n > (int64_t)INT32_MAX) return FSTAT_EUNSUPPORTED;
  for (int d = 0; d < 4; ++d)
    if (!(opt->scale[d] > 0.0) || !std::isfinite(opt->scale[d])) return FSTAT_EINVAL;
  if (!(opt->tol > 0.0) || opt->max_evals < 5 || opt->max_evals > 100000 || (opt->exact != 0 && opt->exact != 1))
    return FSTAT_EINVAL;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  return from_hip(fsk::nelder_mead(p->d_segs, (int)p->segs.size(), seg, params, n, opt->scale, opt->tol,
                                   opt->max_evals, opt->exact, params_out, F_out, evals_out,
                                   (hipStream_t)hip_stream));
}

fstat_status fstat_threshold(double alpha, double n_cells, double* F0) {
  if (!F0 || !(alpha > 0.0 && alpha < 1.0) || !(n_cells >= 1.0) || !std::isfinite(n_cells)) return FSTAT_EINVAL;
  // per-cell false-alarm probability from Eq. (FP): P_F = 1 - (1 - alpha)^(1/N_c)
  const double pf = -std::expm1(std::log1p(-alpha) / n_cells);
  if (!(pf > 0.0) || !(pf < 1.0)) return FSTAT_EINVAL;
  // invert Eq. (PF), P_F(F0) = (1 + F0) e^{-F0}, decreasing on F0 >= 0:
  // solve h(F) = F - log(1 + F) + log P_F = 0 by bisection
  const double lp = std::log(pf);
  double lo = 0.0, hi = 1.0;
  while (hi - std::log1p(hi) + lp < 0.0) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid - std::log1p(mid) + lp < 0.0) lo = mid;
    else hi = mid;
  }
  *F0 = 0.5 * (lo + hi);
  return FSTAT_OK;
}

fstat_status fstat_amplitudes(fstat_plan_t p, const double* params, const int32_t* seg, int64_t n,
                              const double* state, double* out, void* hip_stream) {
  if (!p || !params || n <= 0 || !state || !out) return FSTAT_EINVAL;
  if (n > (int64_t)INT32_MAX) return FSTAT_EUNSUPPORTED;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  return from_hip(fsk::amplitudes(p->d_segs, (int)p->segs.size(), seg, params, n, state, out, (hipStream_t)hip_stream));
}

fstat_status fstat_grad(fstat_plan_t p, const double* params, const int32_t* seg, int64_t n, double* F, double* dF,
                        void* hip_stream) {
  Range rg("fstat_grad");
  if (!p || !params || n <= 0 || !F) return FSTAT_EINVAL;
  if (n > (int64_t)INT32_MAX) return FSTAT_EUNSUPPORTED;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  hipStream_t st = (hipStream_t)hip_stream;
  if (!dF) return from_hip(fsk::grad_forward(p->d_segs, (int)p->segs.size(), seg, params, n, F, nullptr, st));
  fstat_status rc = ensure_ws(p, align_up((size_t)n * FSTATE * sizeof(double)));
  if (rc != FSTAT_OK) return rc;
  double* state = (double*)p->ws;
  HIP_TRY(fsk::grad_forward(p->d_segs, (int)p->segs.size(), seg, params, n, F, state, st));
  return from_hip(fsk::grad_adjoint(p->d_segs, (int)p->segs.size(), seg, params, n, state, nullptr, dF, st));
}

}  // extern "C"

// The plan's device segment table, its length and device, for entry points
// defined in other sources (null for a null plan).
const SegDev* fstat_plan_device_segments(fstat_plan_t p, int* nseg, int* device) {
  if (!p) return nullptr;
  *nseg = (int)p->segs.size();
  *device = p->device;
  return p->d_segs;
}

extern "C" {

fstat_status fstat_bin_params(fstat_plan_t p, const fstat_node* nodes, const int64_t* k, int64_t n, int32_t interbin,
                              double* params, int32_t* seg) {
  if (!p || n < 0 || (n > 0 && (!nodes || !k || !params)) || (interbin != 0 && interbin != 1)) return FSTAT_EINVAL;
  const int nseg = (int)p->segs.size();
  for (int64_t i = 0; i < n; ++i) {
    const fstat_node& nd = nodes[i];
    if (nd.seg < 0 || nd.seg >= nseg || !(std::fabs(nd.bin_offset) < 1.0f)) return FSTAT_EINVAL;
    const int64_t kmax = p->segs[nd.seg].dev.nfft / 2 * (interbin ? 2 : 1);
    if (k[i] < 0 || k[i] >= kmax) return FSTAT_EINVAL;
  }
  for (int64_t i = 0; i < n; ++i) {
    const fstat_node& nd = nodes[i];
    const SegDev& d = p->segs[nd.seg].dev;
    // output index 2k + h of an interbinned call is the bin k + h/2
    const double bin = interbin ? 0.5 * (double)k[i] : (double)k[i];
    params[4 * i] = (bin + (double)nd.bin_offset) / ((double)d.nfft * d.dt);
    params[4 * i + 1] = nd.fdot;
    params[4 * i + 2] = nd.alpha;
    params[4 * i + 3] = nd.delta;
    if (seg) seg[i] = nd.seg;
  }
  return FSTAT_OK;
}

fstat_status fstat_demod_series(fstat_plan_t p, const fstat_node* node, double* out, void* hip_stream) {
  if (!p || !node || !out) return FSTAT_EINVAL;
  if (node->seg < 0 || node->seg >= (int32_t)p->segs.size()) return FSTAT_EINVAL;
  if (!std::isfinite(node->alpha) || !std::isfinite(node->delta) || !std::isfinite(node->fdot) ||
      !(std::fabs(node->bin_offset) < 1.0f))
    return FSTAT_EINVAL;
  DeviceGuard guard(p->device);
  if (!guard.ok) return FSTAT_EDEVICE;
  hipStream_t st = (hipStream_t)hip_stream;
  const SegDev& d = p->segs[node->seg].dev;
  const size_t qbytes = (size_t)d.R * d.Ceff * 4 * elem_real(p->prec);
  const size_t need = 256 + align_up(qbytes) + align_up(sizeof(SkyConst)) + 1024;
  fstat_status rc = ensure_ws(p, need);
  if (rc != FSTAT_OK) return rc;
  rc = ensure_pinned(p, 256);
  if (rc != FSTAT_OK) return rc;
  Carve cv{(char*)p->ws};
  double* d_ad = cv.take<double>(2);
  void* d_quads = cv.take<char>(qbytes);
  SkyConst* d_sky = cv.take<SkyConst>(1);
  double* hp = (double*)p->pinned;
  hp[0] = node->alpha;
  hp[1] = node->delta;
  HIP_TRY(hipMemcpyAsync(d_ad, hp, 2 * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(p->staged, st));
  p->staged_pending = true;
  const int64_t qstride = (int64_t)d.R * d.Ceff;
  HIP_TRY(fsk::sky_setup(d_ad, 1, d, d_sky, st));
  HIP_TRY(fsk::sky_prep(p->prec, d, d_sky, 1, d_quads, qstride, st));
  return from_hip(fsk::demod_series(p->prec, d, d_sky, d_quads, qstride, node->fdot,
                                    (double)node->bin_offset / (double)d.nfft, out, st));
}

}  // extern "C"
