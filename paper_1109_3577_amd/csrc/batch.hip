// Batched solves and the continuous-batching server of libhjb.
//
// Both rest on the independence of the patches (Section 3 of the paper:
// each patch is computed with no information from the others, which is
// what its distributed "Method 2" exploits).  Work items of many problems --
// (problem, patch, tile) triples -- share the rounds of one tiled sweep
// kernel per dimension.  Since every update is monotone and items never
// write outside their own patch of their own problem, the result of each
// problem is bitwise the one it gets when solved alone, whatever else is in
// the mix.

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace hjb;

namespace {

hipStream_t as_stream(hjb_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

// One problem prepared for the shared sweep rounds: Steps 1-3.1 done, value
// grid initialised, work items built.
struct Prepared {
  std::unique_ptr<ProblemDev> P;
  std::unique_ptr<PatchesHandle> patches;
  DBuf v;
  ProblemItems items;
  int dim = 2;
  int engine_index = -1;
  hjb_stats st{};
  double ms_prepare = 0.0;
};

// Host copy of an hjb_problem's arrays (for requests queued by the server).
// The arrays are not zero-filled before the copy: a 193^3 request holds
// about 100 MB, copied on the caller's thread while the rounds wait.
struct ProblemCopy {
  hjb_problem p{};
  std::unique_ptr<double[]> ctrl, speed, drift, bnode;
  std::unique_ptr<int16_t[]> tp;
  template <typename T>
  static std::unique_ptr<T[]> copy(const T *src, size_t n, int32_t mem, hipStream_t s) {
    std::unique_ptr<T[]> dst(new T[n]);
    if (mem == HJB_MEM_HOST) std::memcpy(dst.get(), src, n * sizeof(T));
    else HJB_HIP(hipMemcpyAsync(dst.get(), src, n * sizeof(T), hipMemcpyDeviceToHost, s));
    return dst;
  }
  void take(const hjb_problem &src, hipStream_t s) {
    p = src;
    const size_t N = (size_t)src.n[0] * src.n[1] * src.n[2];
    ctrl = copy(src.controls, (size_t)src.n_controls * src.dim, src.mem, s);
    speed = copy(src.speed, N, src.mem, s);
    tp = copy(src.target_part, N, src.mem, s);
    if (src.drift) drift = copy(src.drift, N * src.dim, src.mem, s);
    if (src.beta_node) bnode = copy(src.beta_node, N, src.mem, s);
    if (src.mem != HJB_MEM_HOST) HJB_HIP(hipStreamSynchronize(s));
    p.controls = ctrl.get();
    p.speed = speed.get();
    p.drift = src.drift ? drift.get() : nullptr;
    p.target_part = tp.get();
    p.beta_node = src.beta_node ? bnode.get() : nullptr;
    p.mem = HJB_MEM_HOST;
  }
};

// `server`: the continuous engine of the server admits requests between
// rounds, so it runs in rounds only; a batch may also drain its items in
// one persistent launch (HJB_SCHED_ASYNC).
SweepShape engine_shape(int dim, bool fp64, const hjb_solve_opts *opts, bool server = false) {
  HJB_REQUIRE(!server || !opts || opts->schedule != HJB_SCHED_ASYNC,
              "the server runs in rounds (HJB_SCHED_ASYNC is for single solves and batches)");
  HJB_REQUIRE(!opts || opts->schedule != HJB_SCHED_ASYNC ||
                  (opts->order_window == 0.0 && opts->start_u0 == 0 && !opts->use_graph),
              "HJB_SCHED_ASYNC runs without order_window, start_u0 and use_graph");
  HJB_REQUIRE(!opts || opts->control_cone == 0.0,
              "control_cone is an option of hjb_solve_patches only");
  HJB_REQUIRE(!opts || opts->start_u0 == 0 || opts->start_u0 == 1, "start_u0 must be 0 or 1");
  if (!opts) return make_config(dim, fp64, nullptr, 0.0, 0).shape;
  hjb_solve_opts o = *opts;
  o.start_u0 = 0;  // the tolerance it needs is checked with the batch's own
  return make_config(dim, fp64, &o, 0.0, 0).shape;
}

// Host threads that prepare the problems of a batch at once.
constexpr int kPrepareThreads = 8;
// Default device bytes of colour fields (and the rest of Steps 2-3.1) that
// one shared colour transport of a batch may hold; larger batches go in
// chunks.  Fewer chunks mean fewer short tail rounds: 512 uneven 2D
// problems (18 GB of colour transport data) prepare in 0.35 s in three
// chunks of at most 8 GiB and in 0.33 s in one.
constexpr size_t kTraceBatchBytes = size_t(32) << 30;

// The rest of the preparation after Step 3.1: value grid (add-on AO1 starts
// it at U^(0)), work items, keys of the value-ordered schedule (add-on AO2),
// and release of what the sweeps do not read.
void finish_prepared(Prepared &pr, bool fp64, const hjb_solve_opts *opts, hipStream_t s) {
  const size_t N = pr.P->N;
  const bool start_u0 = opts && opts->start_u0 == 1;
  pr.v.reset(N * (fp64 ? sizeof(double) : sizeof(float)));
  HJB_HIP(launch_init_values(fp64, pr.patches->code.as<int16_t>(), N, pr.v.get(), s,
                             start_u0 ? pr.patches->u0.as<double>() : nullptr));
  const SweepShape sh = engine_shape(pr.P->dim, fp64, opts);
  pr.items = build_items(*pr.P, pr.patches->code.as<int16_t>(), pr.P->n_parts, sh, s);
  if (opts && opts->order_window > 0.0)
    build_item_keys(*pr.P, pr.patches->code.as<int16_t>(), pr.patches->u0.as<double>(), sh,
                    pr.items, s);
  if (start_u0 || (opts && opts->patch_bc == HJB_BC_DIRICHLET)) {
    // every item starts away from its fixed point (from U^(0), or reading
    // other patches' U^(0) as Dirichlet data); seeds sweep all bricks first
    pr.items.seeds.resize(pr.items.items.size());
    for (size_t i = 0; i < pr.items.seeds.size(); ++i) pr.items.seeds[i] = (int32_t)i;
  }
  // keep only what the sweeps need (U^(0) as Dirichlet data of eq. dbc);
  // the stream is synchronised first since the buffers return to the pool
  HJB_HIP(hipStreamSynchronize(s));
  if (!opts || opts->patch_bc != HJB_BC_DIRICHLET) pr.patches->u0.release();
  pr.patches->feedback.release();
}

void check_batchable(const hjb_problem *fine, const hjb_problem *coarse) {
  HJB_REQUIRE(fine->foot == nullptr && (!coarse || coarse->foot == nullptr),
              "tabulated dynamics (foot) are not supported in batches and the server");
  HJB_REQUIRE(coarse && coarse->dim == fine->dim, "coarse problem missing or of another dimension");
}

// One problem on its own (a server request): Steps 1-3.1 and the rest.
std::unique_ptr<Prepared> prepare(const hjb_problem *fine, const hjb_problem *coarse, bool fp64,
                                  const hjb_solve_opts *opts, hipStream_t s) {
  const double t0 = now_ms();
  std::vector<double> ctrl;
  validate_problem(fine, s, &ctrl);
  check_batchable(fine, coarse);
  int cst = HJB_OK;
  auto C = coarse_solve_impl(coarse, 0.0, 0, s, &cst);
  HJB_REQUIRE(cst == HJB_OK, "coarse solve did not converge");
  auto pr = std::make_unique<Prepared>();
  pr->dim = fine->dim;
  pr->P = upload_problem(*fine, !fp64, s, &ctrl);
  pr->patches = build_patches_impl(*pr->P, *C, s);
  finish_prepared(*pr, fp64, opts, s);
  pr->ms_prepare = now_ms() - t0;
  return pr;
}

// Runs fn(i, stream) for every i < count on up to kPrepareThreads host
// threads, each with a stream of its own that is synchronised before the
// call returns.  The first error is raised again on the calling thread.
template <typename Fn>
void for_each_prepare(int count, Fn &&fn) {
  if (count <= 0) return;
  const int workers = std::min(count, kPrepareThreads);
  int dev = 0;
  HJB_HIP(hipGetDevice(&dev));
  std::atomic<int> next{0};
  std::mutex em;
  int err_code = HJB_OK;
  std::string err_msg;
  auto work = [&]() {
    hipStream_t ws = nullptr;
    try {
      HJB_HIP(hipSetDevice(dev));
      HJB_HIP(hipStreamCreate(&ws));
      for (int i = next++; i < count; i = next++) {
        {
          std::lock_guard<std::mutex> g(em);
          if (err_code != HJB_OK) break;
        }
        fn(i, ws);
      }
      HJB_HIP(hipStreamSynchronize(ws));
    } catch (const ApiError &e) {
      std::lock_guard<std::mutex> g(em);
      if (err_code == HJB_OK) {
        err_code = e.code;
        err_msg = e.msg;
      }
    } catch (const std::exception &e) {
      std::lock_guard<std::mutex> g(em);
      if (err_code == HJB_OK) {
        err_code = HJB_EDEVICE;
        err_msg = e.what();
      }
    }
    if (ws) {
      (void)hipStreamSynchronize(ws);
      (void)hipStreamDestroy(ws);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 0; t < workers; ++t) pool.emplace_back(work);
  for (auto &t : pool) t.join();
  if (err_code != HJB_OK) throw_error(err_code, "%s", err_msg.c_str());
}

// A batch's Step 1 problem on the device, solved with the others.
struct CoarseJob {
  std::unique_ptr<ProblemDev> P;
  DBuf code;
  ProblemItems items;
  std::unique_ptr<CoarseHandle> h;
};

// Prepares every problem of a batch.  The per-problem parts (checks,
// uploads, feedback, labels, items) run on host threads, a stream each; the
// iterative parts share their rounds across problems: the Step 1 solves of
// all problems in one FP64 engine per dimension, and the colour transports
// (Step 3.1) of a chunk of problems in one round list per dimension.  Every
// problem gets the bits it gets alone: both iterations are monotone and
// stop at their exact fixed points.
void prepare_all(const hjb_problem *const *fine, const hjb_problem *const *coarse, int count,
                 bool fp64, const hjb_solve_opts *opts, size_t chunk_bytes, hipStream_t s,
                 std::vector<std::unique_ptr<Prepared>> &out) {
  const double t0 = now_ms();
  HJB_HIP(hipStreamSynchronize(s));  // inputs the caller produced on s are ready
  std::vector<CoarseJob> cj(count);
  for_each_prepare(count, [&](int i, hipStream_t ws) {
    std::vector<double> ctrl, cctrl;
    validate_problem(fine[i], ws, &ctrl);
    check_batchable(fine[i], coarse[i]);
    validate_problem(coarse[i], ws, &cctrl);
    auto pr = std::make_unique<Prepared>();
    pr->dim = fine[i]->dim;
    pr->P = upload_problem(*fine[i], !fp64, ws, &ctrl);
    CoarseJob &J = cj[i];
    J.P = upload_problem(*coarse[i], false, ws, &cctrl);
    const size_t Nc = J.P->N;
    J.code.reset(Nc * sizeof(int16_t));
    HJB_HIP(launch_make_code(J.P->tp, nullptr, nullptr, Nc, J.code.as<int16_t>(), ws));
    J.h = std::make_unique<CoarseHandle>();
    J.h->dim = J.P->dim;
    for (int d = 0; d < 3; ++d) J.h->n[d] = J.P->n[d];
    J.h->N = Nc;
    J.h->v.reset(Nc * sizeof(double));
    HJB_HIP(launch_init_values(true, J.code.as<int16_t>(), Nc, J.h->v.get(), ws, nullptr));
    hjb_solve_opts eo;
    const SweepShape sh = make_config(J.P->dim, true, coarse_opts(J.P->dim, &eo), 0.0, 0).shape;
    J.items = build_items(*J.P, J.code.as<int16_t>(), 1, sh, ws);
    out[i] = std::move(pr);
  });
  // Step 1 of every problem: one FP64 engine per dimension, exact fixed point
  for (int dim = 2; dim <= 3; ++dim) {
    hjb_solve_opts eo;
    const SolveConfig cfg = make_config(dim, true, coarse_opts(dim, &eo), 0.0, 0);
    std::unique_ptr<SweepEngine> e;
    std::vector<int> idx;
    for (int i = 0; i < count; ++i) {
      if (cj[i].P->dim != dim) continue;
      if (!e) e = std::make_unique<SweepEngine>(cfg, s);
      e->add_problem(*cj[i].P, cj[i].code.as<int16_t>(), &cj[i].items, cj[i].h->v.get());
      idx.push_back(i);
    }
    if (!e) continue;
    e->begin();
    HJB_REQUIRE(e->run() == HJB_OK, "coarse solve did not converge");
    const std::vector<EngineResult> res = e->results();
    for (size_t k = 0; k < idx.size(); ++k) {
      hjb_stats &st = cj[idx[k]].h->st;
      st.node_updates = (int64_t)res[k].work_nodes;
      st.updates = (int64_t)res[k].work_nodes * cj[idx[k]].P->nc;
      st.item_runs = (int64_t)res[k].item_runs;
      st.rounds = (int32_t)e->rounds();
      st.residual = res[k].residual;
    }
  }
  // Steps 2 and 3.1 in chunks bounded by the colour-field budget
  for (int i0 = 0; i0 < count;) {
    int i1 = i0;
    size_t bytes = 0;
    while (i1 < count && (i1 == i0 || bytes + trace_job_bytes(*fine[i1]) <= chunk_bytes))
      bytes += trace_job_bytes(*fine[i1++]);
    std::vector<std::unique_ptr<TraceJob>> tj(i1 - i0);
    for_each_prepare(i1 - i0, [&](int k, hipStream_t ws) {
      tj[k] = trace_begin(*out[i0 + k]->P, *cj[i0 + k].h, ws);
    });
    for (int dim = 2; dim <= 3; ++dim) {
      std::vector<TraceJob *> js;
      for (auto &j : tj)
        if (j->h->dim == dim) js.push_back(j.get());
      trace_rounds(js, s);
    }
    for_each_prepare(i1 - i0, [&](int k, hipStream_t ws) {
      Prepared &pr = *out[i0 + k];
      pr.patches = trace_end(*tj[k], ws);
      tj[k].reset();
      cj[i0 + k] = CoarseJob();
      finish_prepared(pr, fp64, opts, ws);
    });
    i0 = i1;
  }
  const double ms = now_ms() - t0;
  for (auto &p : out) p->ms_prepare = ms;
}

size_t footprint_bytes(const hjb_problem &f, const hjb_problem &c, bool fp64) {
  const size_t N = (size_t)f.n[0] * f.n[1] * f.n[2];
  const size_t Nc = (size_t)c.n[0] * c.n[1] * c.n[2];
  const size_t per_node = (fp64 ? 8 : 4) /* v */ + 8 + 4 /* speed */ + 2 /* target part */ +
                          2 + 2 /* labels, code */ + (f.drift ? (8 + 4) * f.dim : 0);
  const size_t transient = N * (8 /* u0 */ + 1 /* feedback */ + 8 /* best */ +
                                8 * (size_t)(f.dim == 2 ? 8 : 4) /* colour chunk */);
  return N * per_node + transient + Nc * 32 + (1u << 20);
}

}  // namespace

// ---------------------------------------------------------------- batch

struct hjb_batch_s {
  hjb_batch_opts opts{};
  bool fp64 = false;
  hipStream_t s = nullptr;
  std::vector<std::unique_ptr<Prepared>> probs;
  std::unique_ptr<SweepEngine> eng[2];
  long long rounds[2] = {0, 0};
  double ms_run = 0.0;
  int status = HJB_OK;
  bool ran = false;
};

extern "C" {

int hjb_batch_create(const hjb_problem *const *fine, const hjb_problem *const *coarse,
                     int32_t count, const hjb_batch_opts *opts, hjb_stream_t stream,
                     hjb_batch_t **out) {
  return guarded([&]() -> int {
    HJB_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    HJB_REQUIRE(count >= 1 && fine && coarse, "need count >= 1 fine and coarse problems");
    auto b = std::make_unique<hjb_batch_s>();
    if (opts) b->opts = *opts;
    else b->opts.precision = HJB_F32;
    HJB_REQUIRE(b->opts.precision == HJB_F32 || b->opts.precision == HJB_F64,
                "precision must be HJB_F32 or HJB_F64");
    b->fp64 = b->opts.precision == HJB_F64;
    b->s = as_stream(stream);
    for (int i = 0; i < count; ++i) HJB_REQUIRE(fine[i] && coarse[i], "problem %d is NULL", i);
    // Preparation (coarse solve, feedback, colours, labels, items) is a
    // chain of short, mostly latency-bound steps per problem: several host
    // threads prepare problems at once, each on a stream of its own.
    b->probs.resize(count);
    const size_t chunk = b->opts.prepare_bytes ? (size_t)b->opts.prepare_bytes : kTraceBatchBytes;
    prepare_all(fine, coarse, count, b->fp64, &b->opts.solve, chunk, b->s, b->probs);
    for (int d = 0; d < 2; ++d) {
      const int dim = d + 2;
      SolveConfig cfg = make_config(dim, b->fp64, &b->opts.solve, b->opts.tol, b->opts.max_sweeps);
      std::unique_ptr<SweepEngine> e;
      for (auto &p : b->probs) {
        if (p->dim != dim) continue;
        if (!e) e = std::make_unique<SweepEngine>(cfg, b->s);
        p->engine_index = e->add_problem(*p->P, p->patches->code.as<int16_t>(), &p->items,
                                         p->v.get(), p->patches->u0.as<double>());
      }
      if (e) e->begin();
      b->eng[d] = std::move(e);
    }
    *out = b.release();
    return HJB_OK;
  });
}

int hjb_batch_run(hjb_batch_t *b, hjb_stream_t stream, hjb_stats *st) {
  return guarded([&]() -> int {
    HJB_REQUIRE(b != nullptr, "batch is NULL");
    HJB_REQUIRE(!b->ran, "batch already ran");
    (void)stream;
    const double t0 = now_ms();
    const long long cap = b->opts.max_sweeps > 0 ? b->opts.max_sweeps : 1000000;
    const int rpp = std::max(1, b->opts.solve.rounds_per_poll > 0 ? b->opts.solve.rounds_per_poll : 6);
    bool live[2] = {b->eng[0] != nullptr, b->eng[1] != nullptr};
    int status = HJB_OK;
    // HJB_SCHED_ASYNC: each dimension's items in one persistent launch
    for (int d = 0; d < 2; ++d) {
      if (!live[d] || !b->eng[d]->async_ok()) continue;
      const int sa = b->eng[d]->run_async();
      if (sa != HJB_OK) status = sa;
      live[d] = false;
    }
    while (live[0] || live[1]) {
      for (int d = 0; d < 2; ++d) {
        if (!live[d]) continue;
        const int q = b->eng[d]->run_rounds(rpp);
        b->rounds[d] += rpp;
        if (q == 0) live[d] = false;
        else if (b->rounds[d] >= cap) {
          live[d] = false;
          status = HJB_ENOCONV;
        }
      }
    }
    b->ms_run = now_ms() - t0;
    b->ran = true;
    b->status = status;
    int64_t upd = 0, nodes = 0, runs = 0, items = 0;
    for (int d = 0; d < 2; ++d) {
      if (!b->eng[d]) continue;
      auto res = b->eng[d]->results();
      items += b->eng[d]->total_items();
      for (auto &p : b->probs) {
        if (p->dim != d + 2) continue;
        const EngineResult &r = res[p->engine_index];
        p->st.node_updates = (int64_t)r.work_nodes;
        p->st.updates = (int64_t)r.work_nodes * p->P->nc;
        p->st.item_runs = (int64_t)r.item_runs;
        p->st.items = (int32_t)p->items.items.size();
        p->st.residual = r.residual;
        p->st.rounds = (int32_t)b->rounds[d];
        p->st.status = status;
        p->st.ms_prolong_feedback = p->patches->st.ms_prolong_feedback;
        p->st.ms_trace = p->patches->st.ms_trace;
        p->st.unreached = p->patches->st.unreached;
        p->st.detached = p->patches->st.detached;
        upd += p->st.updates;
        nodes += p->st.node_updates;
        runs += p->st.item_runs;
      }
    }
    if (st) {
      std::memset(st, 0, sizeof *st);
      st->updates = upd;
      st->node_updates = nodes;
      st->item_runs = runs;
      st->items = (int32_t)items;
      st->rounds = (int32_t)std::max(b->rounds[0], b->rounds[1]);
      st->ms_wall = b->ms_run;
      st->status = status;
    }
    return status;
  });
}

int hjb_batch_result(const hjb_batch_t *b, int32_t i, void *v_out, int32_t mem, hjb_stats *st) {
  return guarded([&]() -> int {
    HJB_REQUIRE(b != nullptr, "batch is NULL");
    HJB_REQUIRE(i >= 0 && i < (int)b->probs.size(), "problem index %d out of range", i);
    HJB_REQUIRE(b->ran, "hjb_batch_run has not been called");
    HJB_REQUIRE(v_out != nullptr, "v_out is NULL");
    HJB_REQUIRE(mem == HJB_MEM_HOST || mem == HJB_MEM_DEVICE, "bad mem");
    const Prepared &p = *b->probs[i];
    HJB_HIP(hipMemcpyAsync(v_out, p.v.get(), p.v.bytes(),
                           mem == HJB_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, b->s));
    HJB_HIP(hipStreamSynchronize(b->s));
    if (st) *st = p.st;
    return b->status;
  });
}

void hjb_batch_free(hjb_batch_t *b) { delete b; }

}  // extern "C"

// ---------------------------------------------------------------- server

namespace {

enum ReqState { QUEUED = 0, PREPARING = 1, LIVE = 2, DONE = 3 };

struct Request {
  uint64_t ticket = 0;
  ProblemCopy fine, coarse;
  size_t footprint = 0;
  ReqState state = QUEUED;
  std::unique_ptr<Prepared> prep;
  long long rounds_live = 0;
  // work of the engines this request left behind (they are rebuilt when
  // requests join or leave)
  unsigned long long work_acc = 0, runs_acc = 0;
  int status = HJB_OK;
  std::string error;     // message of a failed preparation
  double ms_prepare = 0.0;
  hjb_stats st{};
};

}  // namespace

// Admitted requests are prepared (coarse solve, feedback, colours, labels,
// items) by a pool of host threads, each with a stream of its own, while
// the live requests keep sweeping; a prepared request joins the shared
// rounds at the next step.
struct hjb_server_s {
  size_t budget = 0, used = 0;
  hjb_server_opts opts{};
  bool fp64 = false;
  hipStream_t s = nullptr;
  int device = 0;
  uint64_t next_ticket = 1;
  std::deque<Request *> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::unique_ptr<SweepEngine> eng[2];
  std::vector<Request *> members[2];  // engine problem index -> request
  // Each dimension's rounds run on a stream of their own and are polled
  // separately, so that cheap 2D rounds keep going while a block of 3D
  // rounds is in flight.
  hipStream_t es[2] = {nullptr, nullptr};
  bool inflight[2] = {false, false};
  int inflight_rounds[2] = {0, 0};
  std::vector<Request *> joining[2];  // prepared, waiting for their engine to be idle
  std::vector<std::unique_ptr<Request>> retired;  // collected, still listed by an engine
  SolveConfig cfg[2];
  // preparation pool
  std::mutex pm;
  std::condition_variable pcv;   // work for the pool, or stop
  std::condition_variable dcv;   // a preparation finished
  std::deque<Request *> to_prepare;
  std::vector<Request *> prepared;
  int preparing = 0;             // handed to the pool, not yet joined
  bool stopping = false;
  std::vector<std::thread> workers;

  void worker();
  ~hjb_server_s() {
    {
      std::lock_guard<std::mutex> g(pm);
      stopping = true;
    }
    pcv.notify_all();
    for (auto &t : workers) t.join();
    for (int d = 0; d < 2; ++d) {
      if (es[d]) (void)hipStreamSynchronize(es[d]);
      eng[d].reset();
      if (es[d]) (void)hipStreamDestroy(es[d]);
    }
  }
};

void hjb_server_s::worker() {
  hipStream_t ws = nullptr;
  bool ok = hipSetDevice(device) == hipSuccess && hipStreamCreate(&ws) == hipSuccess;
  while (true) {
    Request *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(pm);
      pcv.wait(lk, [&] { return stopping || !to_prepare.empty(); });
      if (stopping) break;
      r = to_prepare.front();
      to_prepare.pop_front();
    }
    std::unique_ptr<Prepared> p;
    int code = HJB_OK;
    std::string msg;
    const double t0 = now_ms();
    if (!ok) {
      code = HJB_EDEVICE;
      msg = "preparation thread has no stream";
    } else {
      try {
        p = prepare(&r->fine.p, &r->coarse.p, fp64, &opts.solve, ws);
        HJB_HIP(hipStreamSynchronize(ws));
      } catch (const ApiError &e) {
        code = e.code;
        msg = e.msg;
        p.reset();
      } catch (const std::exception &e) {
        code = HJB_EDEVICE;
        msg = e.what();
        p.reset();
      }
    }
    {
      std::lock_guard<std::mutex> g(pm);
      r->prep = std::move(p);
      r->status = code;
      r->error = msg;
      r->ms_prepare = now_ms() - t0;
      prepared.push_back(r);
    }
    dcv.notify_all();
  }
  if (ws) {
    (void)hipStreamSynchronize(ws);
    (void)hipStreamDestroy(ws);
  }
}

namespace {

// Rebuilds the engine of one dimension with the live requests plus `added`,
// carrying the queued items of the running ones over (a queued item keeps
// its place; only its global id changes).
void rebuild_engine(hjb_server_s &S, int d, const std::vector<Request *> &added) {
  std::vector<Request *> keep;
  std::vector<std::vector<int32_t>> carry_local;
  if (S.eng[d]) {
    const std::vector<EngineResult> res = S.eng[d]->results();
    for (size_t m = 0; m < S.members[d].size(); ++m) {
      Request *r = S.members[d][m];
      if (r->state != LIVE) continue;
      r->work_acc += res[m].work_nodes;
      r->runs_acc += res[m].item_runs;
    }
    const std::vector<int32_t> q = S.eng[d]->queue_now();
    std::vector<std::vector<int32_t>> per(S.members[d].size());
    // map a global id back to (member, local id) through the bases
    for (int32_t g : q) {
      int m = (int)S.members[d].size() - 1;
      while (m > 0 && S.eng[d]->item_base(m) > g) --m;
      per[m].push_back(g - S.eng[d]->item_base(m));
    }
    for (size_t m = 0; m < S.members[d].size(); ++m) {
      Request *r = S.members[d][m];
      if (r->state == LIVE) {
        keep.push_back(r);
        carry_local.push_back(per[m]);
      }
    }
  }
  for (Request *r : added) {
    keep.push_back(r);
    carry_local.push_back(r->prep->items.seeds);
  }
  S.eng[d].reset();
  S.members[d].clear();
  if (keep.empty()) return;
  auto e = std::make_unique<SweepEngine>(S.cfg[d], S.es[d]);
  std::vector<int32_t> seeds;
  for (size_t i = 0; i < keep.size(); ++i) {
    Prepared &p = *keep[i]->prep;
    p.engine_index = e->add_problem(*p.P, p.patches->code.as<int16_t>(), &p.items, p.v.get(),
                                    p.patches->u0.as<double>());
  }
  for (size_t i = 0; i < keep.size(); ++i)
    for (int32_t l : carry_local[i]) seeds.push_back(e->item_base((int)i) + l);
  e->begin(&seeds);
  S.members[d] = keep;
  S.eng[d] = std::move(e);
}

// Deletes collected requests that no engine lists any more.
void drop_retired(hjb_server_s &S) {
  std::vector<std::unique_ptr<Request>> still;
  for (auto &r : S.retired) {
    bool listed = false;
    for (int d = 0; d < 2; ++d)
      for (Request *m : S.members[d]) listed |= (m == r.get());
    if (listed) still.push_back(std::move(r));
  }
  S.retired = std::move(still);
}

}  // namespace

extern "C" {

int hjb_server_create(size_t hbm_budget, const hjb_server_opts *opts, hjb_stream_t stream,
                      hjb_server_t **out) {
  return guarded([&]() -> int {
    HJB_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    HJB_REQUIRE(hbm_budget > 0, "hbm_budget must be > 0");
    auto S = std::make_unique<hjb_server_s>();
    S->budget = hbm_budget;
    if (opts) S->opts = *opts;
    else S->opts.precision = HJB_F32;
    HJB_REQUIRE(S->opts.precision == HJB_F32 || S->opts.precision == HJB_F64,
                "precision must be HJB_F32 or HJB_F64");
    S->fp64 = S->opts.precision == HJB_F64;
    S->s = as_stream(stream);
    for (int d = 0; d < 2; ++d)
      S->cfg[d] = make_config(d + 2, S->fp64, &S->opts.solve, S->opts.tol, 0);
    (void)engine_shape(2, S->fp64, &S->opts.solve, true);  // rejects HJB_SCHED_ASYNC
    HJB_HIP(hipGetDevice(&S->device));
    for (int d = 0; d < 2; ++d) HJB_HIP(hipStreamCreate(&S->es[d]));
    for (int t = 0; t < kPrepareThreads; ++t) S->workers.emplace_back([p = S.get()] { p->worker(); });
    *out = S.release();
    return HJB_OK;
  });
}

int hjb_server_submit(hjb_server_t *S, const hjb_problem *fine, const hjb_problem *coarse,
                      uint64_t *ticket) {
  return guarded([&]() -> int {
    HJB_REQUIRE(S != nullptr && ticket != nullptr, "server or ticket is NULL");
    // The per-node checks (finite data, reach, target parts) run in the
    // preparation pool, off the serving loop; a request that fails them
    // returns the error from hjb_server_poll.
    validate_header(fine);
    validate_header(coarse);
    HJB_REQUIRE(fine->dim == coarse->dim, "fine and coarse dimensions differ");
    auto r = std::make_unique<Request>();
    r->footprint = footprint_bytes(*fine, *coarse, S->fp64);
    HJB_REQUIRE(r->footprint <= S->budget, "request needs %zu bytes, the budget is %zu",
                r->footprint, S->budget);
    r->fine.take(*fine, S->s);
    r->coarse.take(*coarse, S->s);
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->reqs[r->ticket] = std::move(r);
    return HJB_OK;
  });
}

int hjb_server_step(hjb_server_t *S, int32_t rounds, int32_t *live, int32_t *queued) {
  return guarded([&]() -> int {
    HJB_REQUIRE(S != nullptr, "server is NULL");
    // Admission by HBM footprint, first come first served: the footprint is
    // reserved and the request goes to the preparation pool.
    {
      std::lock_guard<std::mutex> g(S->pm);
      while (!S->queue.empty() && S->used + S->queue.front()->footprint <= S->budget) {
        Request *r = S->queue.front();
        S->queue.pop_front();
        S->used += r->footprint;
        r->state = PREPARING;
        S->to_prepare.push_back(r);
        ++S->preparing;
      }
    }
    S->pcv.notify_all();
    // Prepared requests join the live rounds.  With nothing live, wait a
    // little for one instead of returning at once.
    bool any_live = false;
    for (int d = 0; d < 2; ++d)
      for (Request *r : S->members[d]) any_live |= r->state == LIVE;
    std::vector<Request *> ready;
    {
      std::unique_lock<std::mutex> lk(S->pm);
      if (!any_live && S->prepared.empty() && S->preparing > 0)
        S->dcv.wait_for(lk, std::chrono::milliseconds(2), [&] { return !S->prepared.empty(); });
      ready.swap(S->prepared);
      S->preparing -= (int)ready.size();
    }
    for (Request *r : ready) {
      // the request's host copies are no longer needed
      r->fine = ProblemCopy();
      r->coarse = ProblemCopy();
      if (r->status != HJB_OK || !r->prep) {
        r->state = DONE;
        if (r->status == HJB_OK) r->status = HJB_EDEVICE;
        r->st.status = r->status;
        continue;
      }
      r->st.ms_prolong_feedback = r->prep->patches->st.ms_prolong_feedback;
      r->st.ms_trace = r->prep->patches->st.ms_trace;
      r->st.unreached = r->prep->patches->st.unreached;
      r->st.detached = r->prep->patches->st.detached;
      r->st.ms_wall = r->ms_prepare;
      r->state = LIVE;
      S->joining[r->prep->dim - 2].push_back(r);
    }
    const long long cap = S->opts.max_sweeps > 0 ? S->opts.max_sweeps : 1000000;
    const int n = std::max(1, rounds);
    // A dimension whose engine is idle takes its joiners and enqueues its
    // next block of rounds; the step then returns as soon as one
    // dimension's block has finished (the other keeps running).
    for (int d = 0; d < 2; ++d) {
      if (S->inflight[d]) continue;
      if (!S->joining[d].empty()) {
        rebuild_engine(*S, d, S->joining[d]);
        S->joining[d].clear();
      }
      if (!S->eng[d]) continue;
      bool any = false;
      for (Request *r : S->members[d]) any |= r->state == LIVE;
      if (!any) continue;
      S->eng[d]->launch_rounds_async(n);
      S->inflight[d] = true;
      S->inflight_rounds[d] = n;
    }
    for (bool finished = false; !finished && (S->inflight[0] || S->inflight[1]);) {
      for (int d = 0; d < 2; ++d) {
        if (!S->inflight[d] || !S->eng[d]->rounds_done()) continue;
        finished = true;
        S->inflight[d] = false;
        std::vector<uint32_t> pa;
        (void)S->eng[d]->rounds_result(&pa);
        const int nr = S->inflight_rounds[d];
        std::vector<EngineResult> res;
        bool capped = false;
        for (size_t m = 0; m < S->members[d].size(); ++m) {
          Request *r = S->members[d][m];
          if (r->state != LIVE) continue;
          r->rounds_live += nr;
          const bool conv = pa[m] == 0;
          if (conv || r->rounds_live >= cap) {
            if (res.empty()) res = S->eng[d]->results();
            r->state = DONE;
            r->status = conv ? HJB_OK : HJB_ENOCONV;
            capped |= !conv;
            r->st.node_updates = (int64_t)(r->work_acc + res[m].work_nodes);
            r->st.updates = r->st.node_updates * r->prep->P->nc;
            r->st.item_runs = (int64_t)(r->runs_acc + res[m].item_runs);
            r->st.items = (int32_t)r->prep->items.items.size();
            r->st.residual = res[m].residual;
            r->st.rounds = (int32_t)r->rounds_live;
            r->st.status = r->status;
          }
        }
        // A request stopped by the round cap may still have queued items:
        // rebuild without it so that its buffers are never touched again.
        if (capped) rebuild_engine(*S, d, {});
      }
      if (!finished) std::this_thread::yield();
    }
    drop_retired(*S);
    int nl = 0;
    for (int d = 0; d < 2; ++d) {
      for (Request *r : S->members[d]) nl += r->state == LIVE;
      nl += (int)S->joining[d].size();
    }
    if (live) *live = nl;
    if (queued) {
      std::lock_guard<std::mutex> g(S->pm);
      *queued = (int32_t)S->queue.size() + S->preparing;
    }
    return HJB_OK;
  });
}

int hjb_server_poll(hjb_server_t *S, uint64_t ticket, void *v_out, int32_t mem, hjb_stats *st) {
  return guarded([&]() -> int {
    HJB_REQUIRE(S != nullptr, "server is NULL");
    auto it = S->reqs.find(ticket);
    HJB_REQUIRE(it != S->reqs.end(), "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second.get();
    if (r->state != DONE) return HJB_EAGAIN;
    if (!r->prep) {
      // preparation failed: report its error and forget the request
      const int status = r->status;
      const std::string msg = r->error;
      S->used -= r->footprint;
      if (st) *st = r->st;
      S->retired.push_back(std::move(it->second));
      S->reqs.erase(it);
      drop_retired(*S);
      throw_error(status, "request preparation failed: %s", msg.c_str());
    }
    HJB_REQUIRE(v_out != nullptr, "v_out is NULL");
    HJB_REQUIRE(mem == HJB_MEM_HOST || mem == HJB_MEM_DEVICE, "bad mem");
    HJB_HIP(hipMemcpyAsync(v_out, r->prep->v.get(), r->prep->v.bytes(),
                           mem == HJB_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, S->s));
    HJB_HIP(hipStreamSynchronize(S->s));
    if (st) *st = r->st;
    const int status = r->status;
    // A finished request has no queued item left (converged, or removed
    // from its engine when capped), so its device buffers can go now; the
    // request record lives on while an engine still lists it.
    S->used -= r->footprint;
    r->prep.reset();
    S->retired.push_back(std::move(it->second));
    S->reqs.erase(it);
    drop_retired(*S);
    return status;
  });
}

void hjb_server_free(hjb_server_t *S) { delete S; }

}  // extern "C"
