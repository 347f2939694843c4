// Host runtime of libhjb: errors, device memory, problem upload and the
// round engine that drives the tiled sweep kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "hjb_internal.h"

namespace hjb {

// ---------------------------------------------------------------- errors

struct ApiError {
  int code;
  std::string msg;
};

[[noreturn]] void throw_error(int code, const char *fmt, ...);
void set_last_error(const std::string &s);

#define HJB_HIP(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      ::hjb::throw_error(e_ == hipErrorOutOfMemory ? HJB_ENOMEM : HJB_EDEVICE, "%s: %s (%s:%d)", \
                         #expr, hipGetErrorString(e_), __FILE__, __LINE__);               \
  } while (0)

#define HJB_REQUIRE(cond, ...)                            \
  do {                                                    \
    if (!(cond)) ::hjb::throw_error(HJB_EINVAL, __VA_ARGS__); \
  } while (0)

#define HJB_REQUIRE_CODE(cond, code, ...)            \
  do {                                                \
    if (!(cond)) ::hjb::throw_error((code), __VA_ARGS__); \
  } while (0)

// Runs f() and converts exceptions into a status code + last error.
template <typename F>
int guarded(F &&f) {
  try {
    return f();
  } catch (const ApiError &e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_last_error("host allocation failed");
    return HJB_ENOMEM;
  } catch (...) {
    set_last_error("unexpected internal error");
    return HJB_EDEVICE;
  }
}

// ---------------------------------------------------------------- memory

// Device memory from a per-process caching pool (hipMalloc only when no
// cached block of a suitable size exists; blocks return to the pool when the
// owning DBuf dies).  Every API call synchronises its stream before it
// returns, so a block handed back is idle.
class DBuf {
 public:
  DBuf() = default;
  explicit DBuf(size_t bytes);
  ~DBuf();
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept : p_(o.p_), bytes_(o.bytes_), cap_(o.cap_) {
    o.p_ = nullptr;
    o.bytes_ = o.cap_ = 0;
  }
  DBuf &operator=(DBuf &&o) noexcept;
  void reset(size_t bytes);
  void release();
  template <typename T>
  T *as() const { return static_cast<T *>(p_); }
  void *get() const { return p_; }
  size_t bytes() const { return bytes_; }

 private:
  void *p_ = nullptr;
  size_t bytes_ = 0;
  size_t cap_ = 0;
};

size_t pool_cached_bytes();
void pool_trim();

// Pinned host staging (allocated with hipHostMalloc).
class PinnedBuf {
 public:
  explicit PinnedBuf(size_t bytes);
  ~PinnedBuf();
  PinnedBuf(const PinnedBuf &) = delete;
  PinnedBuf &operator=(const PinnedBuf &) = delete;
  template <typename T>
  T *as() const { return static_cast<T *>(p_); }

 private:
  void *p_ = nullptr;
};

// ---------------------------------------------------------------- problems

struct ProblemDev {
  int dim = 2;
  int n[3] = {1, 1, 1};
  size_t N = 0;
  int nc = 0;
  int n_parts = 1;
  bool drift = false;
  double step[3] = {0, 0, 0};
  double beta = 0, omb = 0;
  // FP64 inputs on the device (owned copies when the caller passed host data)
  DBuf own_ctrl64, own_speed64, own_drift64, own_tp, own_beta64, own_foot64, own_bpk64;
  const double *ctrl64 = nullptr;
  const double *speed64 = nullptr;
  const double *drift64 = nullptr;
  const int16_t *tp = nullptr;
  const double *beta64 = nullptr;  // per-node beta (variable step) or null
  const double *foot64 = nullptr;  // [nc][N][dim] tabulated displacement or null
  const double *bpk64 = nullptr;   // [nc][N] tabulated beta or null
  // FP32 copies (s_d folded into controls and drift)
  DBuf ctrl32, speed32, drift32;
  DBuf beta32, omb32;              // per-node beta and 1 - beta (FP64) rounded to FP32
  DBuf foot32, bpk32, opk32;       // the tables rounded to FP32 (1 - beta from FP64)
  std::vector<double> ctrl_host;         // controls on the host
  std::unique_ptr<PinnedBuf> ctrl_stage;  // pinned staging of the padded tables
};

// Checks every documented requirement of an hjb_problem; throws HJB_EINVAL.
// ctrl_out (optional) receives the controls as read for the checks.
// scan_dev (optional, kScanBytes of device memory) holds the results of the
// device-side scan of device inputs; null: a pool block is used.
constexpr size_t kScanBytes = 48;
// The checks of validate_problem that need no pass over the nodes: sizes,
// beta, controls count, pointers, memory kind, steps.
void validate_header(const hjb_problem *P);
void validate_problem(const hjb_problem *P, hipStream_t s, std::vector<double> *ctrl_out = nullptr,
                      void *scan_dev = nullptr);
// Uploads / borrows the inputs; builds FP32 copies when need32.  `ctrl` is
// the host copy of the controls from validate_problem (read again if null).
// Work is enqueued on s; the caller synchronises before the inputs go.
std::unique_ptr<ProblemDev> upload_problem(const hjb_problem &P, bool need32, hipStream_t s,
                                           const std::vector<double> *ctrl = nullptr);

// ---------------------------------------------------------------- engine

struct SolveConfig {
  bool fp64 = false;
  SweepShape shape{2, 64, 16, 1};
  int inner_sweeps = 48;
  int rounds_per_poll = 16;
  bool use_graph = false;
  bool time_kernels = false;
  bool async = false;  // HJB_SCHED_ASYNC: one persistent launch, device work queue
  double cone_r = 0.0; // add-on AO3 reduction factor r (> 1: control cones on)
  bool dbc = false;    // HJB_BC_DIRICHLET: patch boundaries hold U^(0)
  double win_dt = 0.0; // add-on AO2 ordering window per round (> 0: on)
  bool start_u0 = false; // add-on AO1: start at U^(0), plain v <- F(v)
  bool tab = false;      // tabulated dynamics (set from the problem)
  double tol = 0.0;
  long long max_rounds = 1000000;
};

SolveConfig make_config(int dim, bool fp64, const hjb_solve_opts *opts, double tol,
                        int32_t max_sweeps);

// Work items of one problem for one tile shape, built once (tile bitmap on
// the device, item list on the host).  Item ids are local to the problem.
struct ProblemItems {
  std::vector<Item> items;       // prob field is set by the engine
  DBuf item_map;                 // [n_patches][ntiles] local id or -1
  DBuf item_key;                 // [n_patches][ntiles] FP32 keys of the ordered schedule
  std::vector<int32_t> seeds;    // local ids of the items that can change first
  int ntile[3] = {1, 1, 1};
  int n_patches = 1;
};

ProblemItems build_items(const ProblemDev &P, const int16_t *code, int n_patches, SweepShape sh,
                         hipStream_t s);
// Keys of the value-ordered schedule (add-on AO2) from the Step 2 values.
void build_item_keys(const ProblemDev &P, const int16_t *code, const double *u0, SweepShape sh,
                     ProblemItems &items, hipStream_t s);

// Control cones of add-on AO3: for every feedback control ks, the controls
// a_k with a_k . a_ks >= cos(pi / r) (ks itself always), in index order,
// each row padded with ks to `stride` bytes (a multiple of 4).
struct ConeTable {
  std::vector<uint8_t> idx;  // [nc][stride]
  int len = 0;               // largest cone
  int stride = 0;
};
ConeTable make_cone_table(const std::vector<double> &ctrl, int nc, int dim, double r);

// Device side of a cone solve: the feedback of every node and the rows.
struct ConeArgs {
  const uint8_t *fb = nullptr;
  const uint8_t *idx = nullptr;
  int len = 0;
  int stride = 0;
};

// Per-problem result of an engine run.
struct EngineResult {
  unsigned long long work_nodes = 0;
  unsigned long long item_runs = 0;
  double residual = 0.0;
};

// Drives rounds of the tiled sweep kernel over the work items of one or
// more problems (same dimension and precision).  Problems, their values and
// items are borrowed and must outlive the engine.
class SweepEngine {
 public:
  SweepEngine(const SolveConfig &cfg, hipStream_t s);
  ~SweepEngine();
  SweepEngine(const SweepEngine &) = delete;
  SweepEngine &operator=(const SweepEngine &) = delete;
  // Adds a problem; returns its index.  `v`, `code` and the inputs are on
  // the device.
  // `dbc` (optional, FP64 [N]): Dirichlet data of the patch boundaries.
  // With items->item_key set and cfg.win_dt > 0 the problem's items run in
  // the value-ordered schedule.
  int add_problem(const ProblemDev &P, const int16_t *code, const ProblemItems *items, void *v,
                  const double *dbc = nullptr);
  // Uploads the tables and queues `seeds` (global ids) or, when null, the
  // seeds of every problem.  `unordered`: the value-ordered schedule lets
  // every queued item run at once (threshold +inf).
  void begin(const std::vector<int32_t> *seeds = nullptr, bool unordered = false);
  // Runs rounds until no item is queued or the round cap (HJB_OK / HJB_ENOCONV).
  int run();
  // One persistent launch draining a device work queue (no rounds, no cap).
  int run_async();
  // Whether the configuration asks for run_async (HJB_SCHED_ASYNC).
  bool async_ok() const;
  // Switches the engine's only problem to the control cones of add-on AO3
  // (before begin()).
  void set_cone(const ConeArgs &c);
  // Enqueues `rounds` rounds, waits, returns the length of the next queue.
  int run_rounds(int rounds);
  // The same without waiting: the queue length and the per-problem
  // counters are copied to host memory behind an event.  rounds_done()
  // tells whether the block has finished; rounds_result() waits for it and
  // returns the queue length and (optionally) the per-problem queued counts.
  void launch_rounds_async(int rounds);
  bool rounds_done();
  int rounds_result(std::vector<uint32_t> *pactive);
  // The next round's queue (global ids) and per-problem queued counts.
  std::vector<int32_t> queue_now();
  std::vector<uint32_t> pactive_now();
  std::vector<EngineResult> results();

  int item_base(int prob) const { return bases_[prob]; }
  int n_problems() const { return (int)dps_.size(); }
  long long rounds() const { return rounds_; }
  double kernel_ms() const { return kernel_ms_; }
  int kernel_launches() const { return kernel_launches_; }
  int total_items() const { return (int)items_h_.size(); }

 private:
  void launch_round(uint32_t r);
  // Enqueues `rounds` rounds without waiting.
  void launch_block(int rounds);
  SolveConfig cfg_;
  hipStream_t s_;
  std::vector<DevProblem> dps_;
  std::vector<int> bases_;
  std::vector<const ProblemItems *> pitems_;
  std::vector<Item> items_h_;
  DBuf probs_d_, items_d_, lists_[2], flags_[2], count_, counters_;
  std::unique_ptr<PinnedBuf> host_;
  std::unique_ptr<PinnedBuf> host_cnt_;  // counters copied by launch_rounds_async
  size_t host_cnt_bytes_ = 0;
  hipEvent_t blk_ev_ = nullptr;
  hipEvent_t poll_ev_[2] = {nullptr, nullptr};
  std::vector<int32_t> seeds_;
  bool async_ran_ = false;
  bool cone_ = false;
  long long rounds_ = 0;
  uint32_t r_ = 0;
  double kernel_ms_ = 0.0;
  int kernel_launches_ = 0;
  int kernel_blocks_ = 0;
  int grid_ = 1;
  hipGraphExec_t graph_ = nullptr;
  std::vector<hipEvent_t> events_;
};

// Handles of the C ABI.
struct CoarseHandle {
  int dim = 2;
  int n[3] = {1, 1, 1};
  size_t N = 0;
  DBuf v;  // FP64 coarse values
  hjb_stats st{};
};

struct PatchesHandle {
  int dim = 2;
  int n[3] = {1, 1, 1};
  size_t N = 0;
  int n_parts = 1;
  DBuf labels, feedback, u0, code;
  hjb_stats st{};
};

// Engine options of the Step 1 solves (null: the defaults); buf holds them.
const hjb_solve_opts *coarse_opts(int dim, hjb_solve_opts *buf);
// Step 1: coarse solve (FP64 exact fixed point for tol = 0).
std::unique_ptr<CoarseHandle> coarse_solve_impl(const hjb_problem *coarse, double tol,
                                                int32_t max_sweeps, hipStream_t s, int *status);
// Steps 2 and 3.1 in three stages, so that problems of one dimension can
// share the rounds of the colour transport.
struct TraceJob {
  std::unique_ptr<PatchesHandle> h;
  TraceArgs a{};
  DBuf phi, masks, tp_eff, nex;
  double t0 = 0.0, t1 = 0.0, ms_rounds = 0.0;
  long long rounds = 0;
  int64_t trace_node_updates = 0, item_runs = 0;  // of the shared rounds
};
// Prolongation, obstacles and exclusion, feedback, colour fields.
std::unique_ptr<TraceJob> trace_begin(const ProblemDev &F, const CoarseHandle &C, hipStream_t s,
                                      double exclude_at = 0.0);
// Device bytes a job holds until trace_end (colour fields included).
size_t trace_job_bytes(const hjb_problem &F);
// Workgroups that share one tile activation of the colour transport of
// `jobs` problems (each takes the parts of one residue of the part index):
// two for one 2D problem, whose rounds are short and wait for their
// slowest activations; one for 3D and for shared rounds of several
// problems, which are throughput-bound.
int trace_split(int dim, size_t jobs);
// Colour transport of the jobs (one dimension) in shared rounds.
void trace_rounds(const std::vector<TraceJob *> &jobs, hipStream_t s);
// Labels, codes, statistics; releases the colour fields.
std::unique_ptr<PatchesHandle> trace_end(TraceJob &job, hipStream_t s);
// Steps 2 and 3.1 on an uploaded fine problem.
// exclude_at > 0: nodes off the target with U^(0) >= exclude_at are
// excluded (Section 4.6) and treated as obstacle nodes.
std::unique_ptr<PatchesHandle> build_patches_impl(const ProblemDev &F, const CoarseHandle &C,
                                                  hipStream_t s, double exclude_at = 0.0);
// Value iteration of one problem with the tiled engine (v is initialised).
// With `cone`, each node uses the controls of add-on AO3 only.
int engine_solve(const ProblemDev &P, const int16_t *code, int n_patches, void *v, bool fp64,
                 const hjb_solve_opts *opts, double tol, int32_t max_sweeps, hipStream_t s,
                 hjb_stats *st, double t0, const ConeArgs *cone = nullptr,
                 const double *dbc = nullptr, const double *u0 = nullptr);

// Plain Jacobi on the whole grid (one launch per sweep).
int run_jacobi(const ProblemDev &P, const int16_t *code, bool fp64, void *v_out, double tol,
               long long max_sweeps, int poll, bool time_kernels, hipStream_t s, hjb_stats *st);
// The same iteration in caller-provided buffers: `tmp` [N] values of the
// solve's precision, `dprob` one device DevProblem, `res` 2 x poll u32 words
// (poll u64 slots) on the device, `hres` poll u64 slots on the host.
// Allocates nothing unless time_kernels (events).
struct JacobiWork {
  void *tmp;
  DevProblem *dprob;
  unsigned long long *res;
  unsigned long long *hres;
};
DevProblem jacobi_problem(const ProblemDev &P, const int16_t *code);
int run_jacobi_in(const DevProblem &d, size_t N, bool fp64, void *v_out, double tol,
                  long long max_sweeps, int poll, bool time_kernels, const JacobiWork &w,
                  hipStream_t s, hjb_stats *st);

double now_ms();

}  // namespace hjb
