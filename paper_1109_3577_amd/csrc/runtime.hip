// Host runtime of libhjb: error state, caching device allocator, input
// validation and upload, and the round engine of the tiled sweeps.

#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>

namespace hjb {

// ---------------------------------------------------------------- errors

static thread_local std::string g_last_error;

void set_last_error(const std::string &s) { g_last_error = s; }
const char *last_error_cstr() { return g_last_error.c_str(); }

void throw_error(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw ApiError{code, std::string(buf)};
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- memory pool

namespace {
struct Pool {
  std::mutex m;
  std::map<int, std::multimap<size_t, void *>> free_by_dev;
  std::unordered_map<void *, std::pair<int, size_t>> info;
  size_t cached = 0;
};
Pool &pool() {
  static Pool *p = new Pool();  // never destroyed: device memory outlives static teardown order
  return *p;
}
size_t round_size(size_t b) {
  if (b < 4096) return 4096;
  // round to a multiple of 1/8 of the next power of two, limits waste to 12.5%
  size_t p2 = 1;
  while (p2 < b) p2 <<= 1;
  const size_t q = std::max<size_t>(p2 / 8, 4096);
  return (b + q - 1) / q * q;
}
void *pool_get(size_t bytes, size_t *cap) {
  int dev = 0;
  HJB_HIP(hipGetDevice(&dev));
  const size_t want = round_size(bytes);
  Pool &P = pool();
  {
    std::lock_guard<std::mutex> g(P.m);
    auto &fl = P.free_by_dev[dev];
    auto it = fl.lower_bound(want);
    if (it != fl.end() && it->first <= want + want / 2) {
      void *p = it->second;
      *cap = it->first;
      P.cached -= it->first;
      fl.erase(it);
      return p;
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    pool_trim();
    e = hipMalloc(&p, want);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw_error(HJB_ENOMEM, "device allocation of %zu bytes failed", want);
  }
  std::lock_guard<std::mutex> g(P.m);
  P.info[p] = {dev, want};
  *cap = want;
  return p;
}
void pool_put(void *p) {
  if (!p) return;
  Pool &P = pool();
  std::lock_guard<std::mutex> g(P.m);
  auto it = P.info.find(p);
  if (it == P.info.end()) return;
  P.free_by_dev[it->second.first].insert({it->second.second, p});
  P.cached += it->second.second;
}
}  // namespace

size_t pool_cached_bytes() {
  std::lock_guard<std::mutex> g(pool().m);
  return pool().cached;
}

void pool_trim() {
  Pool &P = pool();
  std::lock_guard<std::mutex> g(P.m);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &kv : P.free_by_dev) {
    if (kv.first != cur) continue;
    for (auto &e : kv.second) {
      (void)hipFree(e.second);
      P.info.erase(e.second);
      P.cached -= e.first;
    }
    kv.second.clear();
  }
}

DBuf::DBuf(size_t bytes) { reset(bytes); }
DBuf::~DBuf() { release(); }
DBuf &DBuf::operator=(DBuf &&o) noexcept {
  if (this != &o) {
    release();
    p_ = o.p_;
    bytes_ = o.bytes_;
    cap_ = o.cap_;
    o.p_ = nullptr;
    o.bytes_ = o.cap_ = 0;
  }
  return *this;
}
void DBuf::reset(size_t bytes) {
  if (p_ && bytes <= cap_) {
    bytes_ = bytes;
    return;
  }
  release();
  if (bytes == 0) return;
  p_ = pool_get(bytes, &cap_);
  bytes_ = bytes;
}
void DBuf::release() {
  if (p_) pool_put(p_);
  p_ = nullptr;
  bytes_ = cap_ = 0;
}

// Pinned host blocks are kept for reuse (allocating and freeing pinned
// memory is slow and can synchronise the device).
namespace {
struct PinnedPool {
  std::mutex m;
  std::multimap<size_t, void *> free_blocks;
  std::unordered_map<void *, size_t> size_of;
};
PinnedPool &pinned_pool() {
  static PinnedPool *P = new PinnedPool();  // lives until the process ends
  return *P;
}
}  // namespace

PinnedBuf::PinnedBuf(size_t bytes) {
  size_t want = 64;
  while (want < bytes) want *= 2;
  PinnedPool &P = pinned_pool();
  {
    std::lock_guard<std::mutex> g(P.m);
    auto it = P.free_blocks.lower_bound(want);
    if (it != P.free_blocks.end() && it->first <= 4 * want) {
      p_ = it->second;
      P.free_blocks.erase(it);
      return;
    }
  }
  HJB_HIP(hipHostMalloc(&p_, want, hipHostMallocDefault));
  std::lock_guard<std::mutex> g(P.m);
  P.size_of[p_] = want;
}
PinnedBuf::~PinnedBuf() {
  if (!p_) return;
  PinnedPool &P = pinned_pool();
  std::lock_guard<std::mutex> g(P.m);
  P.free_blocks.insert({P.size_of[p_], p_});
}

// ---------------------------------------------------------------- validation

static constexpr double kReachLimit = 1.999;  // |displacement| per axis, cells

void validate_header(const hjb_problem *P) {
  HJB_REQUIRE(P != nullptr, "problem is NULL");
  HJB_REQUIRE(P->dim == 2 || P->dim == 3, "dim must be 2 or 3 (got %d)", P->dim);
  for (int d = 0; d < P->dim; ++d)
    HJB_REQUIRE(P->n[d] >= 2, "n[%d] must be >= 2 (got %d)", d, P->n[d]);
  if (P->dim == 2) HJB_REQUIRE(P->n[2] == 1, "2D problems need n[2] == 1 (got %d)", P->n[2]);
  const double Nd = (double)P->n[0] * P->n[1] * P->n[2];
  HJB_REQUIRE(Nd < 2147483647.0, "grid too large (%.0f nodes)", Nd);
  HJB_REQUIRE(P->beta >= 0.5 && P->beta < 1.0, "beta must lie in [0.5, 1) (got %.17g)", P->beta);
  HJB_REQUIRE(P->one_minus_beta == 1.0 - P->beta, "one_minus_beta must equal 1 - beta exactly");
  HJB_REQUIRE(P->n_controls >= 1 && P->n_controls <= 255, "n_controls must be in 1..255 (got %d)",
              P->n_controls);
  HJB_REQUIRE(P->n_parts >= 1 && P->n_parts <= 32767, "n_parts must be in 1..32767 (got %d)",
              P->n_parts);
  HJB_REQUIRE(P->controls && P->speed && P->target_part, "controls, speed and target_part are required");
  HJB_REQUIRE(P->mem == HJB_MEM_HOST || P->mem == HJB_MEM_DEVICE, "mem must be HJB_MEM_HOST or HJB_MEM_DEVICE");
  for (int d = 0; d < P->dim; ++d)
    HJB_REQUIRE(std::isfinite(P->step[d]) && P->step[d] > 0.0, "step[%d] must be finite and > 0", d);
}

void validate_problem(const hjb_problem *P, hipStream_t s, std::vector<double> *ctrl_out,
                      void *scan_dev) {
  validate_header(P);
  const size_t N = (size_t)P->n[0] * P->n[1] * P->n[2];
  const int dim = P->dim, nc = P->n_controls;
  double ctrl[255 * 3];
  const size_t nctrl = (size_t)nc * dim;
  if (P->mem == HJB_MEM_HOST) {
    std::memcpy(ctrl, P->controls, nctrl * sizeof(double));
  } else {
    HJB_HIP(hipMemcpyAsync(ctrl, P->controls, nctrl * sizeof(double), hipMemcpyDeviceToHost, s));
    HJB_HIP(hipStreamSynchronize(s));
  }
  double amax[3] = {0, 0, 0};
  for (int k = 0; k < nc; ++k)
    for (int d = 0; d < dim; ++d) {
      const double a = ctrl[(size_t)k * dim + d];
      HJB_REQUIRE(std::isfinite(a), "control %d is not finite", k);
      amax[d] = std::max(amax[d], std::fabs(a));
    }
  double reach[3] = {0, 0, 0};
  int maxpart = -1;
  if (P->mem == HJB_MEM_HOST) {
    for (size_t g = 0; g < N; ++g) {
      const double c = P->speed[g];
      HJB_REQUIRE(std::isfinite(c) && c >= 0.0, "speed[%zu] must be finite and >= 0", g);
      for (int d = 0; d < dim; ++d) {
        const double w = P->drift ? P->drift[g * dim + d] : 0.0;
        HJB_REQUIRE(std::isfinite(w), "drift[%zu] is not finite", g);
        reach[d] = std::max(reach[d], P->step[d] * (c * amax[d] + std::fabs(w)));
      }
      const int tp = P->target_part[g];
      HJB_REQUIRE(tp >= -2, "target_part[%zu] = %d < -2", g, tp);
      maxpart = std::max(maxpart, tp);
    }
  } else {
    DBuf out;
    if (!scan_dev) out.reset(kScanBytes);
    unsigned long long *o4 =
        static_cast<unsigned long long *>(scan_dev ? scan_dev : out.get());
    HJB_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(o4), 0u, kScanBytes / 4, s));
    int *bad = reinterpret_cast<int *>(o4 + 4);
    HJB_HIP(launch_scan_problem(*P, N, amax, o4, bad, s));
    unsigned long long h[5] = {0, 0, 0, 0, 0};
    HJB_HIP(hipMemcpyAsync(h, o4, sizeof h, hipMemcpyDeviceToHost, s));
    HJB_HIP(hipStreamSynchronize(s));
    int badv = 0;
    std::memcpy(&badv, &h[4], sizeof(int));
    HJB_REQUIRE(!badv, "speed must be finite and >= 0, drift finite, target_part >= -2");
    for (int d = 0; d < 3; ++d) std::memcpy(&reach[d], &h[d], sizeof(double));
    double t;
    std::memcpy(&t, &h[3], sizeof(double));
    maxpart = (int)t - 2;
  }
  HJB_REQUIRE(!P->beta_pk || P->foot, "beta_pk needs foot (tabulated dynamics)");
  if (P->foot) {
    // tabulated dynamics: every displacement within the halo, beta in [0, 1)
    const size_t M = (size_t)nc * N;
    bool ok = true;
    if (P->mem == HJB_MEM_HOST) {
      for (size_t i = 0; i < M * dim && ok; ++i)
        ok = P->foot[i] >= -kReachLimit && P->foot[i] <= kReachLimit;
      for (size_t i = 0; P->beta_pk && i < M && ok; ++i)
        ok = P->beta_pk[i] >= 0.0 && P->beta_pk[i] < 1.0;
    } else {
      DBuf bad(sizeof(int));
      HJB_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), s));
      HJB_HIP(launch_check_range(P->foot, M * dim, -kReachLimit,
                                 std::nextafter(kReachLimit, 3.0), bad.as<int>(), s));
      if (P->beta_pk) HJB_HIP(launch_check_range(P->beta_pk, M, 0.0, 1.0, bad.as<int>(), s));
      int hb = 0;
      HJB_HIP(hipMemcpyAsync(&hb, bad.get(), sizeof hb, hipMemcpyDeviceToHost, s));
      HJB_HIP(hipStreamSynchronize(s));
      ok = hb == 0;
    }
    HJB_REQUIRE(ok, "foot must stay within %.3f cells and beta_pk in [0, 1)", kReachLimit);
    for (int d = 0; d < 3; ++d) reach[d] = 0.0;  // speed and drift are not used
  }
  if (P->beta_node) {
    // per-node beta of the variable step: finite, in [0, 1)
    bool ok = true;
    if (P->mem == HJB_MEM_HOST) {
      for (size_t g = 0; g < N && ok; ++g) ok = P->beta_node[g] >= 0.0 && P->beta_node[g] < 1.0;
    } else {
      DBuf bad(sizeof(int));
      HJB_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), s));
      HJB_HIP(launch_check_range(P->beta_node, N, 0.0, 1.0, bad.as<int>(), s));
      int hb = 0;
      HJB_HIP(hipMemcpyAsync(&hb, bad.get(), sizeof hb, hipMemcpyDeviceToHost, s));
      HJB_HIP(hipStreamSynchronize(s));
      ok = hb == 0;
    }
    HJB_REQUIRE(ok, "beta_node must lie in [0, 1) at every node");
  }
  if (ctrl_out) ctrl_out->assign(ctrl, ctrl + nctrl);
  for (int d = 0; d < dim; ++d)
    HJB_REQUIRE(reach[d] <= kReachLimit,
                "foot points reach %.4f cells on axis %d; the kernels support < 2 (halo)", reach[d], d);
  HJB_REQUIRE(maxpart < P->n_parts, "target_part holds part %d >= n_parts %d", maxpart, P->n_parts);
}

std::unique_ptr<ProblemDev> upload_problem(const hjb_problem &P, bool need32, hipStream_t s,
                                           const std::vector<double> *ctrl) {
  auto D = std::make_unique<ProblemDev>();
  D->dim = P.dim;
  for (int d = 0; d < 3; ++d) {
    D->n[d] = P.n[d];
    D->step[d] = P.step[d];
  }
  D->N = (size_t)P.n[0] * P.n[1] * P.n[2];
  D->nc = P.n_controls;
  D->n_parts = P.n_parts;
  D->drift = P.drift != nullptr;
  D->beta = P.beta;
  D->omb = P.one_minus_beta;
  const size_t N = D->N, cb = (size_t)P.n_controls * P.dim * sizeof(double);
  D->ctrl_host.resize((size_t)P.n_controls * P.dim);
  if (P.mem == HJB_MEM_HOST) {
    std::memcpy(D->ctrl_host.data(), P.controls, cb);
    D->own_speed64.reset(N * sizeof(double));
    D->own_tp.reset(N * sizeof(int16_t));
    HJB_HIP(hipMemcpyAsync(D->own_speed64.get(), P.speed, N * sizeof(double), hipMemcpyHostToDevice, s));
    HJB_HIP(hipMemcpyAsync(D->own_tp.get(), P.target_part, N * sizeof(int16_t), hipMemcpyHostToDevice, s));
    D->speed64 = D->own_speed64.as<double>();
    D->tp = D->own_tp.as<int16_t>();
    if (P.beta_node) {
      D->own_beta64.reset(N * sizeof(double));
      HJB_HIP(hipMemcpyAsync(D->own_beta64.get(), P.beta_node, N * sizeof(double),
                             hipMemcpyHostToDevice, s));
      D->beta64 = D->own_beta64.as<double>();
    }
    const size_t M = (size_t)P.n_controls * N;
    if (P.foot) {
      D->own_foot64.reset(M * P.dim * sizeof(double));
      HJB_HIP(hipMemcpyAsync(D->own_foot64.get(), P.foot, M * P.dim * sizeof(double),
                             hipMemcpyHostToDevice, s));
      D->foot64 = D->own_foot64.as<double>();
    }
    if (P.beta_pk) {
      D->own_bpk64.reset(M * sizeof(double));
      HJB_HIP(hipMemcpyAsync(D->own_bpk64.get(), P.beta_pk, M * sizeof(double),
                             hipMemcpyHostToDevice, s));
      D->bpk64 = D->own_bpk64.as<double>();
    }
    if (P.drift) {
      D->own_drift64.reset(N * P.dim * sizeof(double));
      HJB_HIP(hipMemcpyAsync(D->own_drift64.get(), P.drift, N * P.dim * sizeof(double),
                             hipMemcpyHostToDevice, s));
      D->drift64 = D->own_drift64.as<double>();
    }
  } else {
    if (ctrl && ctrl->size() == D->ctrl_host.size()) {
      D->ctrl_host = *ctrl;  // the validated host copy
    } else {
      HJB_HIP(hipMemcpyAsync(D->ctrl_host.data(), P.controls, cb, hipMemcpyDeviceToHost, s));
      HJB_HIP(hipStreamSynchronize(s));
    }
    D->speed64 = P.speed;
    D->drift64 = P.drift;
    D->tp = P.target_part;
    D->beta64 = P.beta_node;
    D->foot64 = P.foot;
    D->bpk64 = P.beta_pk;
  }
  // Control tables padded to a whole number of groups of 4 plus one more
  // group, the extra rows repeating the last control: the sweep reads the
  // controls four at a time and fetches the next group ahead, and a repeated
  // control leaves the minimum over the set unchanged.  FP32 rows carry
  // s_d * a_kd rounded to FP32.
  // The tables are staged in pinned memory owned by the handle, so the
  // copies stay asynchronous; every entry point synchronises its stream
  // before it returns.
  const int nc = P.n_controls, dim = P.dim;
  const int rows = ((nc + 3) & ~3) + 4;
  const size_t b64 = (size_t)rows * dim * sizeof(double), b32 = (size_t)rows * dim * sizeof(float);
  D->ctrl_stage = std::make_unique<PinnedBuf>(b64 + b32);
  double *pad64 = D->ctrl_stage->as<double>();
  float *pad32 = reinterpret_cast<float *>(D->ctrl_stage->as<char>() + b64);
  for (int k = 0; k < rows; ++k)
    for (int d = 0; d < dim; ++d) {
      const double a = D->ctrl_host[(size_t)(k < nc ? k : nc - 1) * dim + d];
      pad64[(size_t)k * dim + d] = a;
      pad32[(size_t)k * dim + d] = (float)(P.step[d] * a);
    }
  D->own_ctrl64.reset(b64);
  HJB_HIP(hipMemcpyAsync(D->own_ctrl64.get(), pad64, b64, hipMemcpyHostToDevice, s));
  D->ctrl64 = D->own_ctrl64.as<double>();
  if (need32) {
    D->ctrl32.reset(b32);
    HJB_HIP(hipMemcpyAsync(D->ctrl32.get(), pad32, b32, hipMemcpyHostToDevice, s));
    D->speed32.reset(N * sizeof(float));
    HJB_HIP(launch_f64_to_f32(D->speed64, D->speed32.as<float>(), N, s));
    if (D->beta64) {
      D->beta32.reset(N * sizeof(float));
      D->omb32.reset(N * sizeof(float));
      HJB_HIP(launch_beta_f32(D->beta64, D->beta32.as<float>(), D->omb32.as<float>(), N, s));
    }
    const size_t M = (size_t)P.n_controls * N;
    if (D->foot64) {
      D->foot32.reset(M * P.dim * sizeof(float));
      HJB_HIP(launch_f64_to_f32(D->foot64, D->foot32.as<float>(), M * P.dim, s));
    }
    if (D->bpk64) {
      D->bpk32.reset(M * sizeof(float));
      D->opk32.reset(M * sizeof(float));
      HJB_HIP(launch_beta_f32(D->bpk64, D->bpk32.as<float>(), D->opk32.as<float>(), M, s));
    }
    if (P.drift) {
      D->drift32.reset(N * P.dim * sizeof(float));
      HJB_HIP(launch_scaled_f32(D->drift64, D->drift32.as<float>(), N, P.dim, P.step, s));
    }
  }
  return D;
}

// ---------------------------------------------------------------- config

static SweepShape default_shape(int dim, bool fp64) {
  (void)fp64;
  if (dim == 2) return SweepShape{2, 32, 8, 1, 256};
  return SweepShape{3, 8, 8, 8, 256};
}

SolveConfig make_config(int dim, bool fp64, const hjb_solve_opts *opts, double tol,
                        int32_t max_sweeps) {
  SolveConfig c;
  c.fp64 = fp64;
  c.shape = default_shape(dim, fp64);
  c.inner_sweeps = dim == 2 ? 8 : 2;
  c.tol = tol;
  c.max_rounds = max_sweeps > 0 ? max_sweeps : 1000000;
  HJB_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
  if (opts) {
    // A tile shape names its dimension (tile[2] > 1 only in 3D); a batch
    // or server with both kinds applies it to the matching engine only.
    const bool tile3 = opts->tile[2] > 1;
    if (opts->tile[0] > 0 && tile3 == (dim == 3)) {
      c.shape.tx = opts->tile[0];
      c.shape.ty = opts->tile[1];
      c.shape.tz = dim == 3 ? opts->tile[2] : 1;
      if (opts->threads > 0) c.shape.nt = opts->threads;
      HJB_REQUIRE(sweep_shape_supported(c.shape.dim, c.shape.tx, c.shape.ty, c.shape.tz,
                                        c.shape.nt),
                  "unsupported tile shape %dx%dx%d with %d threads for dim %d", c.shape.tx,
                  c.shape.ty, c.shape.tz, c.shape.nt, dim);
    } else if (opts->tile[0] <= 0 && opts->threads > 0 &&
               sweep_shape_supported(c.shape.dim, c.shape.tx, c.shape.ty, c.shape.tz,
                                     opts->threads)) {
      c.shape.nt = opts->threads;
    }
    if (opts->tile[0] > 0 && tile3 == (dim == 3) && opts->inner_sweeps > 0)
      c.inner_sweeps = opts->inner_sweeps;
    else if (opts->tile[0] <= 0 && opts->inner_sweeps > 0)
      c.inner_sweeps = opts->inner_sweeps;
    if (opts->rounds_per_poll > 0) c.rounds_per_poll = opts->rounds_per_poll;
    c.use_graph = opts->use_graph != 0;
    c.time_kernels = opts->time_kernels != 0;
    HJB_REQUIRE(opts->schedule == HJB_SCHED_TILED || opts->schedule == HJB_SCHED_JACOBI ||
                    opts->schedule == HJB_SCHED_ASYNC,
                "unknown schedule %d", opts->schedule);
    c.async = opts->schedule == HJB_SCHED_ASYNC;
    HJB_REQUIRE(std::isfinite(opts->control_cone) && opts->control_cone >= 0.0,
                "control_cone must be finite and >= 0");
    HJB_REQUIRE(opts->patch_bc == HJB_BC_STATE || opts->patch_bc == HJB_BC_DIRICHLET,
                "unknown patch_bc %d", opts->patch_bc);
    c.dbc = opts->patch_bc == HJB_BC_DIRICHLET;
    c.cone_r = opts->control_cone > 1.0 ? opts->control_cone : 0.0;
    HJB_REQUIRE(std::isfinite(opts->order_window) && opts->order_window >= 0.0,
                "order_window must be finite and >= 0");
    c.win_dt = opts->order_window;
    HJB_REQUIRE(c.win_dt == 0.0 || !c.async, "order_window needs the rounds schedule");
    HJB_REQUIRE(opts->start_u0 == 0 || opts->start_u0 == 1, "start_u0 must be 0 or 1");
    c.start_u0 = opts->start_u0 == 1;
    if (c.start_u0) {
      HJB_REQUIRE(!c.async, "start_u0 needs the rounds schedule");
      HJB_REQUIRE(tol >= (fp64 ? 1e-13 : 1e-7),
                  "start_u0 needs tol >= %g (the iteration from U^(0) is not monotone)",
                  fp64 ? 1e-13 : 1e-7);
    }
    if (c.cone_r > 0.0) {
      // fewer controls per update: longer in-tile runs pay off in 2D
      if (dim == 2 && opts->inner_sweeps <= 0) c.inner_sweeps = 16;
      HJB_REQUIRE(opts->schedule == HJB_SCHED_TILED, "control_cone needs HJB_SCHED_TILED");
      HJB_REQUIRE(sweep_cone_shape_supported(c.shape.dim, c.shape.tx, c.shape.ty, c.shape.tz,
                                             c.shape.nt),
                  "control_cone supports the tile shapes 2D 32x8, 32x16 and 3D 8x8x8 with 256 "
                  "threads (got %dx%dx%d with %d)",
                  c.shape.tx, c.shape.ty, c.shape.tz, c.shape.nt);
    }
    HJB_REQUIRE(!c.async || max_sweeps <= 0, "HJB_SCHED_ASYNC takes no sweep cap (max_sweeps 0)");
    HJB_REQUIRE(!c.async || !c.use_graph, "HJB_SCHED_ASYNC has no rounds to replay as a graph");
  }
  if (c.use_graph) c.rounds_per_poll = std::max(6, (c.rounds_per_poll + 5) / 6 * 6);
  return c;
}

// ---------------------------------------------------------------- engine

ProblemItems build_items(const ProblemDev &P, const int16_t *code, int n_patches, SweepShape sh,
                         hipStream_t s) {
  ProblemItems pi;
  pi.n_patches = n_patches;
  const int T[3] = {sh.tx, sh.ty, P.dim == 3 ? sh.tz : 1};
  for (int a = 0; a < 3; ++a) pi.ntile[a] = div_up(P.n[a], T[a]);
  const int ntiles = pi.ntile[0] * pi.ntile[1] * pi.ntile[2];
  // one bit per patch plus the last bit of the row for "holds a target node"
  const int words = (n_patches + 1 + 31) / 32;
  DBuf bits((size_t)ntiles * words * sizeof(uint32_t));
  HJB_HIP(launch_fill_u32(bits.as<uint32_t>(), 0u, (size_t)ntiles * words, s));
  const int32_t tile3[3] = {T[0], T[1], T[2]};
  const int32_t n3[3] = {P.n[0], P.n[1], P.n[2]};
  HJB_HIP(launch_tile_bits(P.dim, code, n3, tile3, pi.ntile, words, bits.as<uint32_t>(), s));
  std::vector<uint32_t> hb((size_t)ntiles * words);
  HJB_HIP(hipMemcpyAsync(hb.data(), bits.get(), hb.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HJB_HIP(hipStreamSynchronize(s));
  const int tbit = words * 32 - 1;
  std::vector<int32_t> imap((size_t)n_patches * ntiles, -1);
  std::vector<uint8_t> seed_tile(ntiles, 0);
  const int nt0 = pi.ntile[0], nt1 = pi.ntile[1], nt2 = pi.ntile[2];
  for (int t = 0; t < ntiles; ++t) {
    const uint32_t *row = &hb[(size_t)t * words];
    if (row[tbit >> 5] & (1u << (tbit & 31))) {
      // a target node reaches (through the 2-node halo) this tile and its neighbours
      const int tx = t % nt0, ty = (t / nt0) % nt1, tz = t / (nt0 * nt1);
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int x = tx + dx, y = ty + dy, z = tz + dz;
            if (x < 0 || y < 0 || z < 0 || x >= nt0 || y >= nt1 || z >= nt2) continue;
            seed_tile[x + nt0 * (y + nt1 * z)] = 1;
          }
    }
    for (int j = 0; j < n_patches; ++j)
      if (row[j >> 5] & (1u << (j & 31))) {
        imap[(size_t)j * ntiles + t] = (int32_t)pi.items.size();
        pi.items.push_back(Item{0, j, t, 0});
      }
  }
  for (size_t i = 0; i < pi.items.size(); ++i)
    if (seed_tile[pi.items[i].tile]) pi.seeds.push_back((int32_t)i);
  pi.item_map.reset(std::max<size_t>(imap.size(), 1) * sizeof(int32_t));
  HJB_HIP(hipMemcpyAsync(pi.item_map.get(), imap.data(), imap.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, s));
  HJB_HIP(hipStreamSynchronize(s));  // imap is a host temporary
  return pi;
}

void build_item_keys(const ProblemDev &P, const int16_t *code, const double *u0, SweepShape sh,
                     ProblemItems &items, hipStream_t s) {
  const int ntiles = items.ntile[0] * items.ntile[1] * items.ntile[2];
  const size_t cnt = (size_t)items.n_patches * ntiles;
  items.item_key.reset(cnt * sizeof(float));
  HJB_HIP(launch_fill_u32(items.item_key.as<uint32_t>(), 0x7f800000u, cnt, s));
  const int32_t n3[3] = {P.n[0], P.n[1], P.n[2]};
  const int32_t t3[3] = {sh.tx, sh.ty, P.dim == 3 ? sh.tz : 1};
  HJB_HIP(launch_item_keys(code, u0, n3, t3, items.ntile, items.item_key.as<uint32_t>(), s));
}

SweepEngine::SweepEngine(const SolveConfig &cfg, hipStream_t s) : cfg_(cfg), s_(s) {
  count_.reset(4 * sizeof(uint32_t));
  host_ = std::make_unique<PinnedBuf>(4096);
}

SweepEngine::~SweepEngine() {
  if (graph_) (void)hipGraphExecDestroy(graph_);
  for (auto e : events_) (void)hipEventDestroy(e);
  for (auto e : poll_ev_)
    if (e) (void)hipEventDestroy(e);
  if (blk_ev_) (void)hipEventDestroy(blk_ev_);
}

int SweepEngine::add_problem(const ProblemDev &P, const int16_t *code, const ProblemItems *items,
                             void *v, const double *dbc) {
  HJB_REQUIRE(cfg_.shape.dim == P.dim, "tile shape dimension mismatch");
  HJB_REQUIRE(cfg_.fp64 || (P.ctrl32.get() && P.speed32.get()), "FP32 inputs missing");
  DevProblem d;
  std::memset(&d, 0, sizeof d);
  d.dim = P.dim;
  for (int a = 0; a < 3; ++a) {
    d.n[a] = P.n[a];
    d.ntile[a] = items->ntile[a];
    d.step[a] = P.step[a];
  }
  d.nc = P.nc;
  d.n_patches = items->n_patches;
  d.has_drift = P.drift ? 1 : 0;
  d.prob_index = (int)dps_.size();
  d.beta = P.beta;
  d.omb = P.omb;
  d.betaf = (float)P.beta;
  d.ombf = (float)P.omb;
  d.ctrl64 = P.ctrl64;
  d.ctrl32 = P.ctrl32.as<float>();
  d.beta64 = P.beta64;
  d.beta32 = P.beta32.as<float>();
  d.omb32 = P.omb32.as<float>();
  d.foot64 = P.foot64;
  d.foot32 = P.foot32.as<float>();
  d.bpk64 = P.bpk64;
  d.bpk32 = P.bpk32.as<float>();
  d.opk32 = P.opk32.as<float>();
  d.speed64 = P.speed64;
  d.speed32 = P.speed32.as<float>();
  d.drift64 = P.drift64;
  d.drift32 = P.drift32.as<float>();
  d.code = code;
  d.v = v;
  d.u0 = dbc;
  d.plain = cfg_.start_u0 ? 1 : 0;
  if (cfg_.win_dt > 0.0 && items->item_key.get()) {
    // the window is given in time steps h = -ln(beta) of the scheme
    d.item_key = items->item_key.as<float>();
    d.win_dt = (float)(cfg_.win_dt * -std::log(P.beta));
  }
  d.item_map = items->item_map.as<int32_t>();
  d.item_base = (int32_t)items_h_.size();
  bases_.push_back(d.item_base);
  for (const Item &it : items->items) {
    Item g = it;
    g.prob = (int32_t)dps_.size();
    items_h_.push_back(g);
  }
  pitems_.push_back(items);
  dps_.push_back(d);
  return (int)dps_.size() - 1;
}

void SweepEngine::begin(const std::vector<int32_t> *seeds, bool unordered) {
  const size_t np = dps_.size();
  counters_.reset(std::max<size_t>(np, 1) * kCounterWords * sizeof(unsigned long long));
  HJB_HIP(hipMemsetAsync(counters_.get(), 0, counters_.bytes(), s_));
  std::vector<uint32_t> winit(6 * np);  // copied from before the final synchronisation
  for (size_t i = 0; i < np; ++i) {
    unsigned long long *c = counters_.as<unsigned long long>() + i * kCounterWords;
    dps_[i].residual = c;                                             // [3][kSlots]
    dps_[i].pactive = reinterpret_cast<uint32_t *>(c + 3 * kSlots);   // 3 x u32
    dps_[i].work = c + 3 * kSlots + 2;                                // [2][kSlots]
    if (dps_[i].item_key) {
      // round 0: base win_dt, smallest queued key 0 (seeds lie at the target)
      dps_[i].win = reinterpret_cast<uint32_t *>(c + 5 * kSlots + 2);  // [6]
      uint32_t *w0 = &winit[6 * i];
      const float b0 = unordered ? INFINITY : dps_[i].win_dt;
      std::memcpy(&w0[0], &b0, sizeof b0);
      w0[1] = w0[2] = 0u;
      w0[3] = 0u;
      w0[4] = w0[5] = 0x7f800000u;
      HJB_HIP(hipMemcpyAsync(dps_[i].win, w0, 6 * sizeof(uint32_t), hipMemcpyHostToDevice, s_));
    }
  }
  probs_d_.reset(std::max<size_t>(np, 1) * sizeof(DevProblem));
  HJB_HIP(hipMemcpyAsync(probs_d_.get(), dps_.data(), np * sizeof(DevProblem),
                         hipMemcpyHostToDevice, s_));
  const size_t ni = std::max<size_t>(items_h_.size(), 1);
  items_d_.reset(ni * sizeof(Item));
  HJB_HIP(hipMemcpyAsync(items_d_.get(), items_h_.data(), items_h_.size() * sizeof(Item),
                         hipMemcpyHostToDevice, s_));
  for (int i = 0; i < 2; ++i) {
    lists_[i].reset(ni * sizeof(int32_t));
    flags_[i].reset(ni * sizeof(uint32_t));
    HJB_HIP(launch_fill_u32(flags_[i].as<uint32_t>(), 0u, ni, s_));
  }
  std::vector<int32_t> sd;
  if (seeds) {
    sd = *seeds;
  } else {
    for (size_t i = 0; i < np; ++i)
      for (int32_t l : pitems_[i]->seeds) sd.push_back(bases_[i] + l);
  }
  seeds_ = sd;
  // per-problem queued counts of the first round
  std::vector<uint32_t> pa(np, 0);
  for (int32_t g : sd) pa[items_h_[g].prob]++;
  for (size_t i = 0; i < np; ++i)
    HJB_HIP(hipMemcpyAsync(dps_[i].pactive, &pa[i], sizeof(uint32_t), hipMemcpyHostToDevice, s_));
  const uint32_t cnt[4] = {(uint32_t)sd.size(), 0u, 0u, 0u};
  if (!sd.empty())
    HJB_HIP(hipMemcpyAsync(lists_[0].get(), sd.data(), sd.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s_));
  HJB_HIP(hipMemcpyAsync(count_.get(), cnt, sizeof cnt, hipMemcpyHostToDevice, s_));
  HJB_HIP(hipStreamSynchronize(s_));  // host vectors above are temporaries
  grid_ = (int)std::min<size_t>(std::max<size_t>(items_h_.size(), 1), 4096);
  r_ = 0;
  rounds_ = 0;
  if (graph_) {
    (void)hipGraphExecDestroy(graph_);
    graph_ = nullptr;
  }
}

void SweepEngine::launch_round(uint32_t r) {
  RoundArgs ra;
  std::memset(&ra, 0, sizeof ra);
  ra.list_in = lists_[r & 1].as<int32_t>();
  ra.list_out = lists_[(r + 1) & 1].as<int32_t>();
  ra.flags_in = flags_[r & 1].as<uint32_t>();
  ra.flags_out = flags_[(r + 1) & 1].as<uint32_t>();
  ra.count = count_.as<uint32_t>();
  ra.work = nullptr;
  ra.round = r;
  ra.inner_sweeps = cfg_.inner_sweeps;
  ra.nprob = (int)dps_.size();
  ra.tol = cfg_.tol;
  if (cfg_.tab)
    HJB_HIP(launch_sweep_tab(cfg_.fp64, cfg_.shape, grid_, probs_d_.as<DevProblem>(),
                             items_d_.as<Item>(), ra, s_));
  else if (cone_)
    HJB_HIP(launch_sweep_cone(cfg_.fp64, cfg_.shape, grid_, probs_d_.as<DevProblem>(),
                              items_d_.as<Item>(), ra, dps_[0].nc, dps_[0].cone_stride, s_));
  else
    HJB_HIP(launch_sweep(cfg_.fp64, cfg_.shape, grid_, probs_d_.as<DevProblem>(),
                         items_d_.as<Item>(), ra, s_));
}

void SweepEngine::launch_block(int rounds) {
  const bool timing = cfg_.time_kernels;
  // (capture is not possible on the legacy null stream: rounds are then
  // launched one by one)
  if (cfg_.use_graph && s_ != nullptr && rounds % 6 == 0 && r_ % 6 == 0) {
    // rounds depend on r only through r mod 2 and r mod 3: one captured
    // block of a multiple of 6 rounds replays for every later block
    if (!graph_) {
      hipGraph_t g = nullptr;
      HJB_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < rounds; ++i) launch_round((uint32_t)i);
      HJB_HIP(hipStreamEndCapture(s_, &g));
      HJB_HIP(hipGraphInstantiate(&graph_, g, nullptr, nullptr, 0));
      (void)hipGraphDestroy(g);
    }
    if (timing) {
      while (events_.size() < (size_t)(2 * (kernel_blocks_ + 1))) {
        hipEvent_t e;
        HJB_HIP(hipEventCreate(&e));
        events_.push_back(e);
      }
      HJB_HIP(hipEventRecord(events_[2 * kernel_blocks_], s_));
    }
    HJB_HIP(hipGraphLaunch(graph_, s_));
    if (timing) {
      HJB_HIP(hipEventRecord(events_[2 * kernel_blocks_ + 1], s_));
      ++kernel_blocks_;
      kernel_launches_ += rounds;
    }
    r_ += rounds;
  } else {
    // Kernel time: one event pair around the block of rounds (the block
    // holds nothing but sweep launches).
    if (timing) {
      while (events_.size() < (size_t)(2 * (kernel_blocks_ + 1))) {
        hipEvent_t e;
        HJB_HIP(hipEventCreate(&e));
        events_.push_back(e);
      }
      HJB_HIP(hipEventRecord(events_[2 * kernel_blocks_], s_));
    }
    for (int i = 0; i < rounds; ++i) {
      launch_round(r_);
      ++r_;
    }
    if (timing) {
      HJB_HIP(hipEventRecord(events_[2 * kernel_blocks_ + 1], s_));
      ++kernel_blocks_;
      kernel_launches_ += rounds;
    }
  }
  rounds_ += rounds;
}

void SweepEngine::launch_rounds_async(int rounds) {
  launch_block(rounds);
  const size_t np = dps_.size();
  const size_t cb = std::max<size_t>(np, 1) * kCounterWords * sizeof(unsigned long long);
  if (!host_cnt_ || host_cnt_bytes_ < cb) {
    host_cnt_ = std::make_unique<PinnedBuf>(cb);
    host_cnt_bytes_ = cb;
  }
  HJB_HIP(hipMemcpyAsync(host_->as<uint32_t>(), count_.as<uint32_t>() + (r_ % 3), sizeof(uint32_t),
                         hipMemcpyDeviceToHost, s_));
  if (np)
    HJB_HIP(hipMemcpyAsync(host_cnt_->as<void>(), counters_.get(),
                           np * kCounterWords * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s_));
  if (!blk_ev_) HJB_HIP(hipEventCreateWithFlags(&blk_ev_, hipEventDisableTiming));
  HJB_HIP(hipEventRecord(blk_ev_, s_));
}

bool SweepEngine::rounds_done() {
  const hipError_t e = hipEventQuery(blk_ev_);
  if (e == hipErrorNotReady) return false;
  HJB_HIP(e);
  return true;
}

int SweepEngine::rounds_result(std::vector<uint32_t> *pactive) {
  HJB_HIP(hipEventSynchronize(blk_ev_));
  if (pactive) {
    const size_t np = dps_.size();
    const unsigned long long *cnt = host_cnt_->as<unsigned long long>();
    pactive->resize(np);
    for (size_t i = 0; i < np; ++i)
      (*pactive)[i] = reinterpret_cast<const uint32_t *>(&cnt[i * kCounterWords + 3 * kSlots])[r_ % 3];
  }
  return (int)host_->as<uint32_t>()[0];
}

int SweepEngine::run_rounds(int rounds) {
  launch_block(rounds);
  uint32_t *h = host_->as<uint32_t>();
  HJB_HIP(hipMemcpyAsync(h, count_.as<uint32_t>() + (r_ % 3), sizeof(uint32_t),
                         hipMemcpyDeviceToHost, s_));
  HJB_HIP(hipStreamSynchronize(s_));
  return (int)h[0];
}

int SweepEngine::run() {
  // Pipelined polling: the next block of rounds is enqueued before the host
  // waits for the queue count that the previous block left, so the device
  // never idles on a poll.  Once the queue is empty the block in flight
  // runs empty rounds only (a few microseconds each).
  for (int i = 0; i < 2; ++i)
    if (!poll_ev_[i]) HJB_HIP(hipEventCreateWithFlags(&poll_ev_[i], hipEventDisableTiming));
  uint32_t *h = host_->as<uint32_t>();
  auto enqueue = [&](int slot) -> bool {
    const long long left = cfg_.max_rounds - rounds_;
    if (left <= 0) return false;
    launch_block((int)std::min<long long>(cfg_.rounds_per_poll, left));
    HJB_HIP(hipMemcpyAsync(h + slot, count_.as<uint32_t>() + (r_ % 3), sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s_));
    HJB_HIP(hipEventRecord(poll_ev_[slot], s_));
    return true;
  };
  int status = HJB_OK;
  int cur = 0;
  if (enqueue(cur)) {
    while (true) {
      const bool next = enqueue(1 - cur);
      HJB_HIP(hipEventSynchronize(poll_ev_[cur]));
      if (h[cur] == 0) break;
      if (!next) {
        status = HJB_ENOCONV;
        break;
      }
      cur = 1 - cur;
    }
  }
  HJB_HIP(hipStreamSynchronize(s_));
  if (cfg_.time_kernels && kernel_blocks_ > 0) {
    kernel_ms_ = 0.0;
    for (int i = 0; i < kernel_blocks_; ++i) {
      float ms = 0.0f;
      HJB_HIP(hipEventElapsedTime(&ms, events_[2 * i], events_[2 * i + 1]));
      kernel_ms_ += ms;
    }
  }
  return status;
}

std::vector<int32_t> SweepEngine::queue_now() {
  uint32_t n = 0;
  HJB_HIP(hipMemcpyAsync(&n, count_.as<uint32_t>() + (r_ % 3), sizeof n, hipMemcpyDeviceToHost, s_));
  HJB_HIP(hipStreamSynchronize(s_));
  std::vector<int32_t> q(n);
  if (n)
    HJB_HIP(hipMemcpyAsync(q.data(), lists_[r_ & 1].get(), n * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s_));
  HJB_HIP(hipStreamSynchronize(s_));
  return q;
}

bool SweepEngine::async_ok() const { return cfg_.async; }

void SweepEngine::set_cone(const ConeArgs &c) {
  HJB_REQUIRE(dps_.size() == 1 && !cfg_.async, "control cones need one problem, rounds schedule");
  HJB_REQUIRE(c.fb && c.idx && c.len > 0 && c.stride >= c.len && c.stride % 4 == 0,
              "bad control cone table");
  HJB_REQUIRE(sweep_cone_lds_bytes(cfg_.fp64, cfg_.shape.dim, dps_[0].nc, c.stride) <= 32 * 1024,
              "control cone tables exceed 32 KiB of LDS (N_c = %d, cone stride %d)", dps_[0].nc,
              c.stride);
  dps_[0].fb = c.fb;
  dps_[0].cone_idx = c.idx;
  dps_[0].cone_len = c.len;
  dps_[0].cone_stride = c.stride;
  cone_ = true;
}

ConeTable make_cone_table(const std::vector<double> &ctrl, int nc, int dim, double r) {
  // the dot products are summed over the axes in order, FP64, with
  // separate multiplies and adds (the library is built without contraction)
  constexpr double kPi = 3.14159265358979323846;
  const double cr = std::cos(kPi / r);
  std::vector<std::vector<uint8_t>> rows((size_t)nc);
  ConeTable t;
  for (int ks = 0; ks < nc; ++ks) {
    for (int k = 0; k < nc; ++k) {
      double dot = 0.0;
      for (int d = 0; d < dim; ++d) {
        const double pr = ctrl[(size_t)k * dim + d] * ctrl[(size_t)ks * dim + d];
        dot = dot + pr;
      }
      if (k == ks || dot >= cr) rows[ks].push_back((uint8_t)k);
    }
    t.len = std::max(t.len, (int)rows[ks].size());
  }
  t.stride = (t.len + 3) / 4 * 4;
  t.idx.assign((size_t)nc * t.stride, 0);
  for (int ks = 0; ks < nc; ++ks)
    for (int i = 0; i < t.stride; ++i)
      t.idx[(size_t)ks * t.stride + i] = i < (int)rows[ks].size() ? rows[ks][i] : (uint8_t)ks;
  return t;
}

int SweepEngine::run_async() {
  const size_t ni = items_h_.size();
  // about four workgroups of 256 threads per CU stay resident
  const int per_cu = std::max(1, 1024 / cfg_.shape.nt);
  const int grid = (int)std::max<size_t>(1, std::min<size_t>(ni, (size_t)256 * per_cu));
  // tickets in use never exceed the queued items plus one per workgroup
  uint32_t cap = 2;
  while (cap < 2 * (ni + (size_t)grid) + 2) cap <<= 1;
  DBuf ring(cap * sizeof(int32_t)), state(ni * sizeof(uint32_t)), sides(ni * sizeof(uint32_t)),
      ctr(4 * sizeof(uint32_t));
  HJB_HIP(launch_fill_u32(sides.as<uint32_t>(), 0u, ni, s_));
  // seeds: queued, in the first ring slots
  const size_t ns = seeds_.size();
  PinnedBuf stage((ni + 4) * sizeof(uint32_t));
  uint32_t *st = stage.as<uint32_t>();
  std::memset(st, 0, ni * sizeof(uint32_t));
  for (int32_t g : seeds_) st[g] = 1u;  // queued
  // seeds hold tickets 0 .. ns-1; the ring is written whole
  PinnedBuf rstage((size_t)cap * sizeof(int32_t));
  int32_t *rg = rstage.as<int32_t>();
  for (uint32_t i = 0; i < cap; ++i) rg[i] = -1;
  for (size_t i = 0; i < ns; ++i) rg[(uint32_t(i) * 0x9E3779B1u) & (cap - 1)] = seeds_[i];
  uint32_t *c4 = st + ni;
  c4[0] = 0u;
  c4[1] = (uint32_t)ns;
  c4[2] = (uint32_t)ns;
  c4[3] = 0u;
  HJB_HIP(hipMemcpyAsync(state.get(), st, ni * sizeof(uint32_t), hipMemcpyHostToDevice, s_));
  HJB_HIP(hipMemcpyAsync(ring.get(), rg, (size_t)cap * sizeof(int32_t), hipMemcpyHostToDevice, s_));
  HJB_HIP(hipMemcpyAsync(ctr.get(), c4, 4 * sizeof(uint32_t), hipMemcpyHostToDevice, s_));
  AsyncQ q;
  q.ring = ring.as<int32_t>();
  q.mask = cap - 1;
  q.state = state.as<uint32_t>();
  q.sides = sides.as<uint32_t>();
  q.ctr = ctr.as<uint32_t>();
  RoundArgs ra;
  std::memset(&ra, 0, sizeof ra);
  ra.round = 0;
  ra.inner_sweeps = cfg_.inner_sweeps;
  ra.nprob = (int)dps_.size();
  ra.tol = cfg_.tol;
  const bool timing = cfg_.time_kernels;
  if (timing) {
    while (events_.size() < (size_t)(2 * (kernel_blocks_ + 1))) {
      hipEvent_t e;
      HJB_HIP(hipEventCreate(&e));
      events_.push_back(e);
    }
    HJB_HIP(hipEventRecord(events_[2 * kernel_blocks_], s_));
  }
  HJB_HIP(launch_sweep_async(cfg_.fp64, cfg_.shape, grid, probs_d_.as<DevProblem>(),
                             items_d_.as<Item>(), ra, q, s_));
  if (timing) {
    HJB_HIP(hipEventRecord(events_[2 * kernel_blocks_ + 1], s_));
    ++kernel_blocks_;
    kernel_launches_ += 1;
  }
  uint32_t *h = host_->as<uint32_t>();
  HJB_HIP(hipMemcpyAsync(h, ctr.get(), 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s_));
  HJB_HIP(hipStreamSynchronize(s_));
  rounds_ += 1;
  async_ran_ = true;
  if (timing) {
    kernel_ms_ = 0.0;
    for (int i = 0; i < kernel_blocks_; ++i) {
      float ms = 0.0f;
      HJB_HIP(hipEventElapsedTime(&ms, events_[2 * i], events_[2 * i + 1]));
      kernel_ms_ += ms;
    }
  }
  HJB_REQUIRE_CODE(h[3] == 0u && h[2] == 0u, HJB_EDEVICE,
                   "asynchronous sweep stopped with work left (code %u, %u pending)", h[3], h[2]);
  return HJB_OK;
}

std::vector<uint32_t> SweepEngine::pactive_now() {
  const size_t np = dps_.size();
  const size_t W = kCounterWords;
  std::vector<unsigned long long> cnt(np * W);
  if (np)
    HJB_HIP(hipMemcpyAsync(cnt.data(), counters_.get(), np * W * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s_));
  HJB_HIP(hipStreamSynchronize(s_));
  std::vector<uint32_t> out(np);
  for (size_t i = 0; i < np; ++i)
    out[i] = reinterpret_cast<const uint32_t *>(&cnt[i * W + 3 * kSlots])[r_ % 3];
  return out;
}

std::vector<EngineResult> SweepEngine::results() {
  const size_t np = dps_.size();
  const size_t W = kCounterWords;
  std::vector<unsigned long long> cnt(np * W);
  if (np)
    HJB_HIP(hipMemcpyAsync(cnt.data(), counters_.get(), np * W * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s_));
  HJB_HIP(hipStreamSynchronize(s_));
  std::vector<EngineResult> out(np);
  for (size_t i = 0; i < np; ++i) {
    const unsigned long long *c = &cnt[i * W];
    // residual of the last executed round lives in row (r - 1) mod 3; the
    // FP64 bits of non-negative values order like the values
    unsigned long long rb = 0;
    for (int k = 0; k < kSlots; ++k) rb = std::max(rb, c[((r_ + 2) % 3) * kSlots + k]);
    double rd;
    std::memcpy(&rd, &rb, sizeof rd);
    // the asynchronous schedule has no rounds: it ends with no item queued
    out[i].residual = async_ran_ ? 0.0 : rd;
    unsigned long long wn = 0, ir = 0;
    for (int k = 0; k < kSlots; ++k) {
      wn += c[3 * kSlots + 2 + k];
      ir += c[3 * kSlots + 2 + kSlots + k];
    }
    out[i].work_nodes = wn;
    out[i].item_runs = ir;
  }
  return out;
}

// ---------------------------------------------------------------- Jacobi

DevProblem jacobi_problem(const ProblemDev &P, const int16_t *code) {
  DevProblem d;
  std::memset(&d, 0, sizeof d);
  d.dim = P.dim;
  for (int a = 0; a < 3; ++a) {
    d.n[a] = P.n[a];
    d.step[a] = P.step[a];
  }
  d.nc = P.nc;
  d.has_drift = P.drift ? 1 : 0;
  d.beta = P.beta;
  d.omb = P.omb;
  d.betaf = (float)P.beta;
  d.ombf = (float)P.omb;
  d.ctrl64 = P.ctrl64;
  d.ctrl32 = P.ctrl32.as<float>();
  d.beta64 = P.beta64;
  d.beta32 = P.beta32.as<float>();
  d.omb32 = P.omb32.as<float>();
  d.foot64 = P.foot64;
  d.foot32 = P.foot32.as<float>();
  d.bpk64 = P.bpk64;
  d.bpk32 = P.bpk32.as<float>();
  d.opk32 = P.opk32.as<float>();
  d.speed64 = P.speed64;
  d.speed32 = P.speed32.as<float>();
  d.drift64 = P.drift64;
  d.drift32 = P.drift32.as<float>();
  d.code = code;
  return d;
}

int run_jacobi(const ProblemDev &P, const int16_t *code, bool fp64, void *v_out, double tol,
               long long max_sweeps, int poll, bool time_kernels, hipStream_t s, hjb_stats *st) {
  const size_t es = fp64 ? sizeof(double) : sizeof(float);
  poll = std::max(1, poll);
  DBuf tmp(P.N * es), dprob(sizeof(DevProblem)), res((size_t)poll * sizeof(unsigned long long));
  PinnedBuf hres((size_t)poll * sizeof(unsigned long long));
  const DevProblem d = jacobi_problem(P, code);
  const JacobiWork w{tmp.get(), dprob.as<DevProblem>(), res.as<unsigned long long>(),
                     hres.as<unsigned long long>()};
  return run_jacobi_in(d, P.N, fp64, v_out, tol, max_sweeps, poll, time_kernels, w, s, st);
}

int run_jacobi_in(const DevProblem &d, size_t N, bool fp64, void *v_out, double tol,
                  long long max_sweeps, int poll, bool time_kernels, const JacobiWork &w,
                  hipStream_t s, hjb_stats *st) {
  const size_t es = fp64 ? sizeof(double) : sizeof(float);
  poll = std::max(1, poll);
  // `d` stays alive until the stream is synchronised below
  HJB_HIP(hipMemcpyAsync(w.dprob, &d, sizeof d, hipMemcpyHostToDevice, s));
  HJB_HIP(launch_init_values(fp64, d.code, N, v_out, s));
  void *a = v_out, *b = w.tmp;
  long long sweeps = 0, executed = 0;
  int status = HJB_ENOCONV;
  double last_res = 0.0;
  std::vector<hipEvent_t> ev;
  int launches = 0;
  while (executed < max_sweeps) {
    // a fill kernel rather than a memset node (see the graph notes of the engine)
    HJB_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(w.res), 0u, 2 * (size_t)poll, s));
    const int m = (int)std::min<long long>(poll, max_sweeps - executed);
    for (int i = 0; i < m; ++i) {
      if (time_kernels) {
        while (ev.size() < (size_t)(2 * (launches + 1))) {
          hipEvent_t e;
          HJB_HIP(hipEventCreate(&e));
          ev.push_back(e);
        }
        HJB_HIP(hipEventRecord(ev[2 * launches], s));
      }
      HJB_HIP(launch_jacobi(fp64, d.dim, w.dprob, N, a, b, w.res + i, s));
      if (time_kernels) {
        HJB_HIP(hipEventRecord(ev[2 * launches + 1], s));
        ++launches;
      }
      std::swap(a, b);
    }
    executed += m;
    HJB_HIP(hipMemcpyAsync(w.hres, w.res, (size_t)m * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    HJB_HIP(hipStreamSynchronize(s));
    bool stop = false;
    for (int i = 0; i < m; ++i) {
      double rd;
      std::memcpy(&rd, &w.hres[i], sizeof rd);
      last_res = rd;
      if (rd <= tol) {
        sweeps = executed - m + i + 1;
        stop = true;
        break;
      }
    }
    if (stop) {
      status = HJB_OK;
      break;
    }
    sweeps = executed;
  }
  if (a != v_out) HJB_HIP(hipMemcpyAsync(v_out, a, N * es, hipMemcpyDeviceToDevice, s));
  HJB_HIP(hipStreamSynchronize(s));
  if (st) {
    // active non-target nodes: count once on the host side of the caller;
    // node_updates is filled there
    st->rounds = (int32_t)executed;
    st->residual = last_res;
    st->items = 0;
    st->item_runs = 0;
    double ms = 0.0;
    for (int i = 0; i < launches; ++i) {
      float t = 0.0f;
      HJB_HIP(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
      ms += t;
    }
    st->ms_kernel = ms;
    st->kernel_launches = launches;
    st->sweeps = (int32_t)sweeps;
  }
  for (auto e : ev) (void)hipEventDestroy(e);
  return status;
}

}  // namespace hjb
