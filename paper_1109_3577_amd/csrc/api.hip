// Exported C ABI of libhjb (declared in include/hjb.h): the four calls of
// the Patchy Algorithm of the paper (Section 3) plus handle accessors.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "runtime.h"

using namespace hjb;

struct hjb_coarse_s : CoarseHandle {};
struct hjb_patches_s : PatchesHandle {};

namespace hjb {
const char *last_error_cstr();
}

namespace {

hipStream_t as_stream(hjb_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

void copy_out(void *dst, const void *src, size_t bytes, int32_t mem, hipStream_t s) {
  HJB_REQUIRE(dst != nullptr, "output pointer is NULL");
  HJB_REQUIRE(mem == HJB_MEM_HOST || mem == HJB_MEM_DEVICE, "mem must be HJB_MEM_HOST or HJB_MEM_DEVICE");
  HJB_HIP(hipMemcpyAsync(dst, src, bytes, mem == HJB_MEM_HOST ? hipMemcpyDeviceToHost
                                                               : hipMemcpyDeviceToDevice, s));
  HJB_HIP(hipStreamSynchronize(s));
}

}  // namespace

namespace hjb {

// Value iteration on one problem with the tiled engine; fills st.
int engine_solve(const ProblemDev &P, const int16_t *code, int n_patches, void *v, bool fp64,
                 const hjb_solve_opts *opts, double tol, int32_t max_sweeps, hipStream_t s,
                 hjb_stats *st, double t0, const ConeArgs *cone, const double *dbc,
                 const double *u0) {
  SolveConfig cfg = make_config(P.dim, fp64, opts, tol, max_sweeps);
  cfg.tab = P.foot64 != nullptr;
  if (cfg.tab) {
    HJB_REQUIRE(!cfg.async && cfg.cone_r == 0.0,
                "tabulated dynamics run in rounds, without control_cone");
    HJB_REQUIRE(sweep_tab_shape_supported(cfg.shape.dim, cfg.shape.tx, cfg.shape.ty,
                                          cfg.shape.tz, cfg.shape.nt),
                "tabulated dynamics support the tile shapes 2D 16x16 (256 or 512 threads), "
                "32x8 and 3D 8x8x8 (256 threads)");
  }
  HJB_REQUIRE(!cfg.start_u0 || u0 != nullptr, "start_u0 needs the Step 2 values");
  HJB_HIP(launch_init_values(fp64, code, P.N, v, s, cfg.start_u0 ? u0 : nullptr));
  HJB_REQUIRE((cfg.cone_r > 0.0) == (cone != nullptr), "control cone tables missing");
  HJB_REQUIRE(cfg.dbc == (dbc != nullptr), "patch boundary data missing");
  HJB_REQUIRE(cfg.win_dt == 0.0 || u0 != nullptr, "order_window needs the Step 2 values");
  ProblemItems items = build_items(P, code, n_patches, cfg.shape, s);
  if (cfg.win_dt > 0.0) build_item_keys(P, code, u0, cfg.shape, items, s);
  SweepEngine eng(cfg, s);
  eng.add_problem(P, code, &items, v, dbc);
  if (cone) eng.set_cone(*cone);
  std::vector<int32_t> all((size_t)eng.total_items());
  for (size_t i = 0; i < all.size(); ++i) all[i] = (int32_t)i;
  // With the Dirichlet data of eq. dbc a node whose stencil reads another
  // patch's U^(0) < 1 starts above its fixed point anywhere in the patch,
  // not only next to the target.  The rounds follow the changes outward
  // from the target; a pass that then queues every item (the first run of
  // an item sweeps all of its bricks) checks every node, and is repeated
  // only when it changed a value (an item ran twice).  The asynchronous
  // schedule has no end of rounds to check at: it starts from every item.
  const bool verify = cfg.dbc && !cfg.start_u0 && !cfg.async;
  if (cfg.start_u0 || (cfg.dbc && cfg.async)) {
    // every item starts away from its fixed point
    eng.begin(&all);
  } else {
    eng.begin();
  }
  int status = eng.async_ok() ? eng.run_async() : eng.run();
  EngineResult acc = eng.results()[0];
  long long rounds = eng.rounds();  // kernel time and launches accumulate in the engine
  while (verify && status == HJB_OK) {
    eng.begin(&all, true);
    status = eng.run();
    const EngineResult r = eng.results()[0];
    acc.work_nodes += r.work_nodes;
    acc.item_runs += r.item_runs;
    acc.residual = r.residual;
    rounds += eng.rounds();
    if (r.item_runs <= (unsigned long long)all.size()) break;  // nothing was queued again
    if (rounds >= cfg.max_rounds) status = HJB_ENOCONV;
  }
  if (st) {
    const EngineResult &r = acc;
    st->node_updates = (int64_t)r.work_nodes;
    // controls evaluated per node update: N_c, or the (padded) cone length
    st->updates = (int64_t)r.work_nodes * (cone ? cone->len : P.nc);
    st->item_runs = (int64_t)r.item_runs;
    st->items = eng.total_items();
    st->rounds = (int32_t)rounds;
    st->residual = r.residual;
    st->ms_kernel = eng.kernel_ms();
    st->kernel_launches = eng.kernel_launches();
    st->status = status;
    st->ms_wall = now_ms() - t0;
    st->tile[0] = cfg.shape.tx;
    st->tile[1] = cfg.shape.ty;
    st->tile[2] = cfg.shape.tz;
    st->threads = cfg.shape.nt;
    st->inner_sweeps = cfg.inner_sweeps;
  }
  return status;
}

// In-tile sweeps of one colour-transport tile activation before it is
// queued again.

// Steps 2 and 3.1, first stage: prolongation, obstacles and exclusion,
// feedback, colour fields and part masks of one problem.
std::unique_ptr<TraceJob> trace_begin(const ProblemDev &F, const CoarseHandle &C, hipStream_t s,
                                      double exclude_at) {
  auto job = std::make_unique<TraceJob>();
  job->h = std::make_unique<PatchesHandle>();
  PatchesHandle &H = *job->h;
  H.dim = F.dim;
  for (int d = 0; d < 3; ++d) H.n[d] = F.n[d];
  H.N = F.N;
  H.n_parts = F.n_parts;
  const size_t N = F.N;
  const int dim = F.dim;
  job->t0 = now_ms();
  HJB_REQUIRE(H.n_parts <= trace_max_parts(), "at most %d target parts are supported (got %d)",
              trace_max_parts(), H.n_parts);
  H.u0.reset(N * sizeof(double));
  H.feedback.reset(N);
  H.labels.reset(N * sizeof(int16_t));
  H.code.reset(N * sizeof(int16_t));

  // Per-axis prolongation tables: coarse cell Q and local coordinate T of
  // every fine index, X = p (nc - 1) / (nf - 1).
  std::vector<int32_t> Q;
  std::vector<double> T;
  for (int d = 0; d < 3; ++d) {
    const int nf = F.n[d], nc = C.n[d];
    for (int p = 0; p < nf; ++p) {
      if (d >= dim) {
        Q.push_back(0);
        T.push_back(0.0);
        continue;
      }
      const double X = (double)((long long)p * (nc - 1)) / (double)(nf - 1);
      double q = std::floor(X);
      if (q > (double)(nc - 2)) q = (double)(nc - 2);
      Q.push_back((int32_t)q);
      T.push_back(X - q);
    }
  }
  DBuf dQ(Q.size() * sizeof(int32_t)), dT(T.size() * sizeof(double));
  HJB_HIP(hipMemcpyAsync(dQ.get(), Q.data(), Q.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HJB_HIP(hipMemcpyAsync(dT.get(), T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const int32_t nf3[3] = {F.n[0], F.n[1], F.n[2]};
  const int32_t nc3[3] = {C.n[0], C.n[1], C.n[2]};
  HJB_HIP(launch_prolong(dim, nf3, nc3, C.v.as<double>(), dQ.as<int32_t>(), dT.as<double>(),
                         H.u0.as<double>(), s));
  // Obstacle nodes, and the unreachable nodes excluded after Step 1, hold
  // U^(0) = 1 and take no part in Steps 2 and 3.
  job->tp_eff.reset(N * sizeof(int16_t));
  job->nex.reset(sizeof(unsigned long long));
  HJB_HIP(launch_fill_u32(job->nex.as<uint32_t>(), 0u, 2, s));
  HJB_HIP(launch_obstacles(F.tp, H.u0.as<double>(), N, exclude_at, job->tp_eff.as<int16_t>(),
                           job->nex.as<unsigned long long>(), s));

  TraceArgs &a = job->a;
  std::memset(&a, 0, sizeof a);
  const SweepShape tsh = trace_shape(dim);
  const int TT[3] = {tsh.tx, tsh.ty, dim == 3 ? tsh.tz : 1};
  for (int d = 0; d < 3; ++d) {
    a.n[d] = F.n[d];
    a.ntile[d] = div_up(F.n[d], TT[d]);
    a.step[d] = F.step[d];
  }
  a.nc = F.nc;
  a.has_drift = F.drift ? 1 : 0;
  a.beta = F.beta;
  a.ctrl64 = F.ctrl64;
  a.speed64 = F.speed64;
  a.drift64 = F.drift64;
  a.target_part = job->tp_eff.as<int16_t>();
  a.beta_node = F.beta64;
  a.foot = F.foot64;
  a.beta_pk = F.bpk64;
  a.feedback = H.feedback.as<uint8_t>();
  a.N = N;
  HJB_HIP(launch_feedback(dim, a, H.u0.as<double>(), H.feedback.as<uint8_t>(), s));
  HJB_HIP(hipStreamSynchronize(s));
  job->t1 = now_ms();

  // Colour fields (Step 3.1): zero, then 1 on the target nodes of their own
  // part, with the part bits of their tiles.
  const int ntiles = a.ntile[0] * a.ntile[1] * a.ntile[2];
  a.n_parts = H.n_parts;
  a.words = (H.n_parts + 31) / 32;
  job->phi.reset((size_t)H.n_parts * N * sizeof(double));
  job->masks.reset((size_t)ntiles * a.words * sizeof(uint32_t));
  a.phi = job->phi.as<double>();
  a.masks = job->masks.as<uint32_t>();
  HJB_HIP(launch_fill_f64(a.phi, 0.0, (size_t)H.n_parts * N, s));
  HJB_HIP(launch_fill_u32(a.masks, 0u, (size_t)ntiles * a.words, s));
  HJB_HIP(launch_trace_init(dim, a, s));
  return job;
}

size_t trace_job_bytes(const hjb_problem &F) {
  const size_t N = (size_t)F.n[0] * F.n[1] * F.n[2];
  return N * ((size_t)F.n_parts * sizeof(double) + 8 + 1 + 2 + 2 + 2) + (1u << 16);
}

// Second stage: the colour transport of every job (all of one dimension)
// to its exact fixed point, in rounds shared by the jobs.  A tile id is the
// job's tile_base plus its tile index.
void trace_rounds(const std::vector<TraceJob *> &jobs, hipStream_t s) {
  if (jobs.empty()) return;
  const int dim = jobs[0]->h->dim;
  const double t0 = now_ms();
  std::vector<TraceArgs> args;
  std::vector<int32_t> tile_prob;
  int max_words = 1;
  long long total = 0;
  for (size_t j = 0; j < jobs.size(); ++j) {
    TraceArgs &a = jobs[j]->a;
    HJB_REQUIRE(jobs[j]->h->dim == dim, "colour transport jobs of mixed dimensions");
    const long long nt = (long long)a.ntile[0] * a.ntile[1] * a.ntile[2];
    HJB_REQUIRE(total + nt < (1ll << 31), "too many tiles in one colour transport");
    a.tile_base = (int32_t)total;
    total += nt;
    max_words = std::max(max_words, a.words);
    args.push_back(a);
    if (jobs.size() > 1) tile_prob.insert(tile_prob.end(), (size_t)nt, (int32_t)j);
  }
  const int ntiles = (int)total;
  DBuf args_d(args.size() * sizeof(TraceArgs)), prob_d(tile_prob.size() * sizeof(int32_t));
  HJB_HIP(hipMemcpyAsync(args_d.get(), args.data(), args_d.bytes(), hipMemcpyHostToDevice, s));
  if (!tile_prob.empty())
    HJB_HIP(hipMemcpyAsync(prob_d.get(), tile_prob.data(), prob_d.bytes(), hipMemcpyHostToDevice,
                           s));
  DBuf lists[2], flags[2], count(4 * sizeof(uint32_t)),
      work(2 * kSlots * sizeof(unsigned long long));
  for (int i = 0; i < 2; ++i) {
    lists[i].reset((size_t)ntiles * sizeof(int32_t));
    flags[i].reset((size_t)ntiles * sizeof(uint32_t));
    HJB_HIP(launch_fill_u32(flags[i].as<uint32_t>(), 0u, ntiles, s));
  }
  HJB_HIP(launch_fill_u32(count.as<uint32_t>(), 0u, 4, s));
  HJB_HIP(launch_fill_u32(work.as<uint32_t>(), 0u, 4 * kSlots, s));
  PinnedBuf host(64);
  RoundArgs ra;
  std::memset(&ra, 0, sizeof ra);
  ra.count = count.as<uint32_t>();
  ra.work = work.as<unsigned long long>();
  ra.inner_sweeps = trace_inner_sweeps(dim);
  // seeding appends to list[0]/count[0] as if it were round -1 (== 2 mod 3)
  ra.list_out = lists[0].as<int32_t>();
  ra.flags_out = flags[0].as<uint32_t>();
  ra.round = 2;
  for (const TraceJob *j : jobs) HJB_HIP(launch_trace_seed(dim, j->a, ra, s));
  const int split = trace_split(dim, jobs.size());
  const int grid = (int)std::min<long long>((long long)ntiles * split, 4096);
  const TraceArgs *args_dev = args_d.as<TraceArgs>();
  const int32_t *prob_dev = tile_prob.empty() ? nullptr : prob_d.as<int32_t>();
  // Rounds in blocks of 16; the next block is enqueued before the host
  // reads the queue count that the previous one left (pipelined polling).
  const int rpp = 16;
  long long rounds = 0;
  uint32_t r = 0;
  hipEvent_t pev[2];
  for (auto &e : pev) HJB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  } evguard{pev};
  uint32_t *hc = host.as<uint32_t>();
  auto enqueue = [&](int slot) {
    for (int i = 0; i < rpp; ++i, ++r) {
      ra.list_in = lists[r & 1].as<int32_t>();
      ra.list_out = lists[(r + 1) & 1].as<int32_t>();
      ra.flags_in = flags[r & 1].as<uint32_t>();
      ra.flags_out = flags[(r + 1) & 1].as<uint32_t>();
      ra.round = r;
      HJB_HIP(launch_trace(dim, grid, split, args_dev, prob_dev, max_words, ra, s));
    }
    rounds += rpp;
    HJB_HIP(hipMemcpyAsync(hc + slot, count.as<uint32_t>() + (r % 3), sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    HJB_HIP(hipEventRecord(pev[slot], s));
  };
  int cur = 0;
  enqueue(cur);
  while (true) {
    enqueue(1 - cur);
    HJB_HIP(hipEventSynchronize(pev[cur]));
    if (hc[cur] == 0) break;
    if (rounds >= 4000000) {
      (void)hipStreamSynchronize(s);  // nothing in flight uses the buffers below
      HJB_REQUIRE(false, "colour transport did not settle");
    }
    cur = 1 - cur;
  }
  unsigned long long ws[2 * kSlots];
  HJB_HIP(hipMemcpyAsync(ws, work.get(), sizeof ws, hipMemcpyDeviceToHost, s));
  HJB_HIP(hipStreamSynchronize(s));
  unsigned long long w[2] = {0, 0};
  for (int k = 0; k < kSlots; ++k) {
    w[0] += ws[k];
    w[1] += ws[kSlots + k];
  }
  const SweepShape tsh = trace_shape(dim);
  const double ms = now_ms() - t0;
  for (TraceJob *j : jobs) {
    j->rounds = rounds;
    // tile activations x parts loaded x tile nodes (upper bound of the
    // per-node colour updates of one in-tile sweep), over all jobs
    j->trace_node_updates = (int64_t)w[0] * tsh.tx * tsh.ty * (dim == 3 ? tsh.tz : 1);
    j->item_runs = (int64_t)w[1];
    j->ms_rounds = ms;
  }
}

// Third stage: labels (with the fill of Remark 3.1 where no colour
// arrived), codes and statistics; frees the colour fields.
std::unique_ptr<PatchesHandle> trace_end(TraceJob &job, hipStream_t s) {
  PatchesHandle &H = *job.h;
  const TraceArgs &a = job.a;
  const int dim = H.dim;
  const size_t N = H.N;
  const double t1 = now_ms();
  HJB_REQUIRE(N < (size_t)INT32_MAX, "grid of %zu nodes is too large for the labels", N);
  // [0] unreached, [1] fill flag, [2] nodes of cut-off pieces
  DBuf unreached(sizeof(uint32_t) * 4);
  HJB_HIP(launch_fill_u32(unreached.as<uint32_t>(), 0u, 4, s));
  HJB_HIP(launch_labels(dim, a, H.labels.as<int16_t>(), unreached.as<uint32_t>(), s));
  // pieces of a patch cut off from their own target part are uncoloured
  DBuf parent(N * sizeof(int32_t)), attached(N);
  const int32_t nn[3] = {H.n[0], H.n[1], H.n[2]};
  HJB_HIP(launch_detach_pieces(nn, job.tp_eff.as<int16_t>(), H.labels.as<int16_t>(),
                               parent.as<int32_t>(), attached.as<uint8_t>(),
                               unreached.as<uint32_t>() + 2, s));
  uint32_t cnt4[4] = {0, 0, 0, 0};
  PinnedBuf host(64);
  HJB_HIP(hipMemcpyAsync(cnt4, unreached.get(), sizeof cnt4, hipMemcpyDeviceToHost, s));
  HJB_HIP(hipStreamSynchronize(s));
  const uint32_t un = cnt4[0], detached = cnt4[2];
  // the fill's second buffer lives until the stream is synchronised below
  // (a block handed back to the pool may be reused by another thread)
  DBuf tmp;
  if (un + detached > 0) {
    // Remark 3.1 fill of the nodes no colour reached, layer by layer
    tmp.reset(N * sizeof(int16_t));
    int16_t *cur = H.labels.as<int16_t>(), *nxt = tmp.as<int16_t>();
    const int32_t n3[3] = {H.n[0], H.n[1], H.n[2]};
    uint32_t *flag = unreached.as<uint32_t>() + 1;
    uint32_t *hflag = host.as<uint32_t>();
    for (long long layer = 0;; ++layer) {
      HJB_HIP(launch_fill_u32(flag, 0u, 1, s));
      HJB_HIP(launch_label_fill(n3, cur, nxt, flag, s));
      HJB_HIP(hipMemcpyAsync(hflag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      HJB_HIP(hipStreamSynchronize(s));
      std::swap(cur, nxt);
      if (hflag[0] == 0) break;
      HJB_REQUIRE(layer < (long long)N, "label fill did not settle");
    }
    if (cur != H.labels.as<int16_t>())
      HJB_HIP(hipMemcpyAsync(H.labels.get(), cur, N * sizeof(int16_t), hipMemcpyDeviceToDevice, s));
  }
  HJB_HIP(launch_make_code(job.tp_eff.as<int16_t>(), H.labels.as<int16_t>(), nullptr, N,
                           H.code.as<int16_t>(), s));
  unsigned long long excluded = 0;
  HJB_HIP(hipMemcpyAsync(&excluded, job.nex.get(), sizeof excluded, hipMemcpyDeviceToHost, s));
  HJB_HIP(hipStreamSynchronize(s));
  job.phi.release();
  job.masks.release();
  const double t2 = now_ms();
  std::memset(&H.st, 0, sizeof H.st);
  H.st.ms_prolong_feedback = job.t1 - job.t0;
  H.st.ms_trace = job.ms_rounds + (t2 - t1);
  H.st.trace_node_updates = job.trace_node_updates;
  H.st.unreached = (int32_t)un;
  H.st.detached = (int32_t)detached;
  H.st.excluded = (int32_t)excluded;
  H.st.rounds = (int32_t)job.rounds;
  H.st.item_runs = job.item_runs;
  H.st.updates = (int64_t)N * a.nc;  // feedback evaluations
  H.st.ms_wall = H.st.ms_prolong_feedback + H.st.ms_trace;
  return std::move(job.h);
}

// Steps 2 and 3.1 of one problem: prolongation, feedback, colour transport
// of all parts, labels.
std::unique_ptr<PatchesHandle> build_patches_impl(const ProblemDev &F, const CoarseHandle &C,
                                                  hipStream_t s, double exclude_at) {
  auto job = trace_begin(F, C, s, exclude_at);
  trace_rounds({job.get()}, s);
  return trace_end(*job, s);
}

std::unique_ptr<CoarseHandle> coarse_solve_impl(const hjb_problem *coarse, double tol,
                                                int32_t max_sweeps, hipStream_t s, int *status) {
  const double t0 = now_ms();
  std::vector<double> ctrl;
  validate_problem(coarse, s, &ctrl);
  auto P = upload_problem(*coarse, false, s, &ctrl);
  auto h = std::make_unique<CoarseHandle>();
  h->dim = P->dim;
  for (int d = 0; d < 3; ++d) h->n[d] = P->n[d];
  h->N = P->N;
  h->v.reset(P->N * sizeof(double));
  DBuf code(P->N * sizeof(int16_t));
  HJB_HIP(launch_make_code(P->tp, nullptr, nullptr, P->N, code.as<int16_t>(), s));
  hjb_solve_opts eo;
  *status = engine_solve(*P, code.as<int16_t>(), 1, h->v.get(), true, coarse_opts(P->dim, &eo),
                         tol, max_sweeps, s, &h->st, t0);
  return h;
}

const hjb_solve_opts *coarse_opts(int dim, hjb_solve_opts *buf) {
  // The coarse grid is small (tens of nodes a side): small tiles keep the
  // per-round latency down, and two control slices per tile (512 threads
  // for 16 x 16 nodes) shorten each FP64 sweep.
  std::memset(buf, 0, sizeof *buf);
  if (dim != 2) return nullptr;
  buf->tile[0] = 16;
  buf->tile[1] = 16;
  buf->tile[2] = 1;
  buf->threads = 512;
  buf->inner_sweeps = 8;
  buf->rounds_per_poll = 16;
  return buf;
}

}  // namespace hjb

extern "C" {

const char *hjb_last_error(void) { return hjb::last_error_cstr(); }

const char *hjb_version(void) { return "hjb-mi355x 0.1 (gfx950)"; }

int hjb_coarse_solve(const hjb_problem *coarse, double tol, int32_t max_sweeps, hjb_stream_t stream,
                     hjb_coarse_t **out) {
  return guarded([&]() -> int {
    HJB_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    int status = HJB_OK;
    auto h = coarse_solve_impl(coarse, tol, max_sweeps, as_stream(stream), &status);
    auto* ph = new hjb_coarse_s();
    static_cast<CoarseHandle &>(*ph) = std::move(*h);
    *out = ph;
    return status;
  });
}

int hjb_coarse_values(const hjb_coarse_t *c, double *out, int32_t mem) {
  return guarded([&]() -> int {
    HJB_REQUIRE(c != nullptr, "coarse handle is NULL");
    copy_out(out, c->v.get(), c->N * sizeof(double), mem, nullptr);
    return HJB_OK;
  });
}

void hjb_coarse_free(hjb_coarse_t *c) { delete c; }

int hjb_build_patches(const hjb_problem *fine, const hjb_coarse_t *coarse, hjb_stream_t stream,
                      hjb_patches_t **out, hjb_stats *st) {
  return hjb_build_patches_ex(fine, coarse, nullptr, stream, out, st);
}

int hjb_build_patches_ex(const hjb_problem *fine, const hjb_coarse_t *coarse,
                         const hjb_build_opts *opts, hjb_stream_t stream, hjb_patches_t **out,
                         hjb_stats *st) {
  return guarded([&]() -> int {
    HJB_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    HJB_REQUIRE(coarse != nullptr, "coarse handle is NULL");
    const double theta = opts ? opts->exclude_at : 0.0;
    HJB_REQUIRE(theta == 0.0 || (theta > 0.0 && theta <= 1.0),
                "exclude_at must be 0 (off) or in (0, 1]");
    hipStream_t s = as_stream(stream);
    std::vector<double> ctrl;
    validate_problem(fine, s, &ctrl);
    HJB_REQUIRE(fine->dim == coarse->dim, "fine and coarse dimensions differ");
    auto F = upload_problem(*fine, false, s, &ctrl);
    auto h = build_patches_impl(*F, *coarse, s, theta);
    if (st) *st = h->st;
    auto* ph = new hjb_patches_s();
    static_cast<PatchesHandle &>(*ph) = std::move(*h);
    *out = ph;
    return HJB_OK;
  });
}

int hjb_patches_labels(const hjb_patches_t *p, int16_t *out, int32_t mem) {
  return guarded([&]() -> int {
    HJB_REQUIRE(p != nullptr, "patches handle is NULL");
    copy_out(out, p->labels.get(), p->N * sizeof(int16_t), mem, nullptr);
    return HJB_OK;
  });
}

int hjb_patches_feedback(const hjb_patches_t *p, uint8_t *out, int32_t mem) {
  return guarded([&]() -> int {
    HJB_REQUIRE(p != nullptr, "patches handle is NULL");
    copy_out(out, p->feedback.get(), p->N, mem, nullptr);
    return HJB_OK;
  });
}

int hjb_patches_u0(const hjb_patches_t *p, double *out, int32_t mem) {
  return guarded([&]() -> int {
    HJB_REQUIRE(p != nullptr, "patches handle is NULL");
    copy_out(out, p->u0.get(), p->N * sizeof(double), mem, nullptr);
    return HJB_OK;
  });
}

void hjb_patches_free(hjb_patches_t *p) { delete p; }

int hjb_solve_patches(const hjb_problem *fine, const hjb_patches_t *p, int32_t precision,
                      double tol, int32_t max_sweeps, void *v_out, const hjb_solve_opts *opts,
                      hjb_stats *st, hjb_stream_t stream) {
  return guarded([&]() -> int {
    const double t0 = now_ms();
    HJB_REQUIRE(p != nullptr, "patches handle is NULL");
    HJB_REQUIRE(v_out != nullptr, "v_out is NULL");
    HJB_REQUIRE(precision == HJB_F32 || precision == HJB_F64, "precision must be HJB_F32 or HJB_F64");
    hipStream_t s = as_stream(stream);
    std::vector<double> ctrl;
    validate_problem(fine, s, &ctrl);
    HJB_REQUIRE(fine->dim == p->dim && fine->n[0] == p->n[0] && fine->n[1] == p->n[1] &&
                    fine->n[2] == p->n[2],
                "problem grid does not match the patches handle");
    HJB_REQUIRE(fine->n_parts == p->n_parts, "n_parts does not match the patches handle");
    const bool fp64 = precision == HJB_F64;
    auto P = upload_problem(*fine, !fp64, s, &ctrl);
    const int16_t *code = p->code.as<int16_t>();
    const double *dbc =
        opts && opts->patch_bc == HJB_BC_DIRICHLET ? p->u0.as<double>() : nullptr;
    DBuf selcode, sel;
    if (opts && opts->patch_select) {
      sel.reset((size_t)p->n_parts);
      HJB_HIP(hipMemcpyAsync(sel.get(), opts->patch_select, (size_t)p->n_parts,
                             hipMemcpyHostToDevice, s));
      selcode.reset(P->N * sizeof(int16_t));
      HJB_HIP(launch_make_code(P->tp, p->labels.as<int16_t>(), sel.as<uint8_t>(), P->N,
                               selcode.as<int16_t>(), s));
      code = selcode.as<int16_t>();
    }
    if (opts && opts->control_cone > 1.0) {
      HJB_REQUIRE(std::isfinite(opts->control_cone), "control_cone must be finite");
      const ConeTable t = make_cone_table(ctrl, fine->n_controls, fine->dim, opts->control_cone);
      DBuf idx(t.idx.size());
      HJB_HIP(hipMemcpyAsync(idx.get(), t.idx.data(), t.idx.size(), hipMemcpyHostToDevice, s));
      ConeArgs c;
      c.fb = p->feedback.as<uint8_t>();
      c.idx = idx.as<uint8_t>();
      c.len = t.len;
      c.stride = t.stride;
      // engine_solve synchronises the stream before it returns (t stays alive)
      return engine_solve(*P, code, p->n_parts, v_out, fp64, opts, tol, max_sweeps, s, st, t0,
                          &c, dbc, p->u0.as<double>());
    }
    return engine_solve(*P, code, p->n_parts, v_out, fp64, opts, tol, max_sweeps, s, st, t0,
                        nullptr, dbc, p->u0.as<double>());
  });
}

int hjb_solve_global(const hjb_problem *fine, int32_t precision, double tol, int32_t max_sweeps,
                     void *v_out, const hjb_solve_opts *opts, hjb_stats *st,
                     hjb_stream_t stream) {
  return guarded([&]() -> int {
    const double t0 = now_ms();
    HJB_REQUIRE(v_out != nullptr, "v_out is NULL");
    HJB_REQUIRE(precision == HJB_F32 || precision == HJB_F64, "precision must be HJB_F32 or HJB_F64");
    hipStream_t s = as_stream(stream);
    std::vector<double> ctrl;
    validate_problem(fine, s, &ctrl);
    const bool fp64 = precision == HJB_F64;
    auto P = upload_problem(*fine, !fp64, s, &ctrl);
    DBuf code(P->N * sizeof(int16_t));
    HJB_HIP(launch_make_code(P->tp, nullptr, nullptr, P->N, code.as<int16_t>(), s));
    HJB_REQUIRE(!opts || opts->control_cone == 0.0,
                "control_cone needs the Step 2 feedback (hjb_solve_patches only)");
    HJB_REQUIRE(!opts || opts->patch_bc == HJB_BC_STATE,
                "patch_bc applies to patch solves (the global solve has no patches)");
    HJB_REQUIRE(!opts || opts->order_window == 0.0,
                "order_window needs the Step 2 values (hjb_solve_patches only)");
    HJB_REQUIRE(!opts || opts->start_u0 == 0,
                "start_u0 needs the Step 2 values (hjb_solve_patches only)");
    const int sched = opts ? opts->schedule : HJB_SCHED_TILED;
    if (sched == HJB_SCHED_JACOBI) {
      (void)make_config(P->dim, fp64, opts, tol, max_sweeps);  // validates opts and tol
      DBuf cnt(sizeof(unsigned long long));
      HJB_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(unsigned long long), s));
      HJB_HIP(launch_count_active(code.as<int16_t>(), P->N, cnt.as<unsigned long long>(), s));
      unsigned long long active = 0;
      HJB_HIP(hipMemcpyAsync(&active, cnt.get(), sizeof active, hipMemcpyDeviceToHost, s));
      HJB_HIP(hipStreamSynchronize(s));
      hjb_stats local{};
      const int poll = opts && opts->rounds_per_poll > 0 ? opts->rounds_per_poll : 4;
      const int status = run_jacobi(*P, code.as<int16_t>(), fp64, v_out, tol,
                                    max_sweeps > 0 ? max_sweeps : 1000000, poll,
                                    opts && opts->time_kernels, s, &local);
      if (st) {
        *st = local;
        st->node_updates = (int64_t)active * local.rounds;
        st->updates = st->node_updates * P->nc;
        st->status = status;
        st->ms_wall = now_ms() - t0;
      }
      return status;
    }
    return engine_solve(*P, code.as<int16_t>(), 1, v_out, fp64, opts, tol, max_sweeps, s, st, t0);
  });
}

}  // extern "C"
