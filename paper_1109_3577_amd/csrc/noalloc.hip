// Allocation-free variant of the plain global solve (hjb_solve_global with
// HJB_SCHED_JACOBI), for callers that cannot allocate device memory: code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc.  Every buffer beyond the caller's inputs and output lives in one
// file-scope device array, `scratch`, which each GPU holds once for the life
// of the process; calls that overlap on one GPU share it and race.

#include <cmath>
#include <cstring>
#include <mutex>

#include "runtime.h"

using namespace hjb;

namespace {

constexpr size_t kScratchBytes = size_t(48) << 20;
constexpr int kMaxDevices = 64;
constexpr int kPoll = 4;  // sweeps between host polls (the Jacobi default)

// The scratch memory.  In host code this name is only a stand-in for the
// symbol: kernels receive the address hipGetSymbolAddress returned for the
// current device (scratch_base), never the name itself.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current).
unsigned char *scratch_base() {
  int dev = 0;
  HJB_HIP(hipGetDevice(&dev));
  HJB_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d out of range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw_error(HJB_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
    }
    g_scratch_dev[dev] = p;
  }
  return static_cast<unsigned char *>(g_scratch_dev[dev]);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

int hjb_solve_global_noalloc(const hjb_problem *fine, int32_t precision, double tol,
                             int32_t max_sweeps, void *v_out, hjb_stats *st,
                             hjb_stream_t stream) {
  return guarded([&]() -> int {
    HJB_REQUIRE(fine != nullptr, "problem is NULL");
    HJB_REQUIRE(v_out != nullptr, "v_out is NULL");
    HJB_REQUIRE(precision == HJB_F32 || precision == HJB_F64,
                "precision must be HJB_F32 or HJB_F64");
    HJB_REQUIRE(fine->mem == HJB_MEM_DEVICE,
                "hjb_solve_global_noalloc takes device inputs only (mem = HJB_MEM_DEVICE)");
    HJB_REQUIRE(!fine->beta_node && !fine->foot && !fine->beta_pk,
                "hjb_solve_global_noalloc supports f = c(x) a + w(x) with one beta "
                "(no beta_node, foot or beta_pk)");
    HJB_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
    HJB_REQUIRE(fine->dim == 2 || fine->dim == 3, "dim must be 2 or 3 (got %d)", fine->dim);
    const double Nd = (double)fine->n[0] * fine->n[1] * fine->n[2];
    HJB_REQUIRE(Nd >= 1.0 && Nd <= (double)HJB_NOALLOC_MAX_NODES,
                "hjb_solve_global_noalloc takes at most %d nodes (got %.0f)",
                HJB_NOALLOC_MAX_NODES, Nd);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const double t0 = now_ms();
    unsigned char *base = scratch_base();
    const bool fp64 = precision == HJB_F64;
    const int dim = fine->dim, nc = fine->n_controls;
    const size_t N = (size_t)Nd;

    // Scratch layout (256-byte aligned regions).
    const int rows = ((nc + 3) & ~3) + 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      unsigned char *p = base + off;
      off += align256(bytes);
      return p;
    };
    void *scan = take(kScanBytes);
    DevProblem *dprob = reinterpret_cast<DevProblem *>(take(sizeof(DevProblem)));
    unsigned long long *res = reinterpret_cast<unsigned long long *>(
        take(kPoll * sizeof(unsigned long long)));
    unsigned long long *active = reinterpret_cast<unsigned long long *>(take(8));
    double *ctrl64 = reinterpret_cast<double *>(take((size_t)rows * dim * sizeof(double)));
    float *ctrl32 = reinterpret_cast<float *>(take((size_t)rows * dim * sizeof(float)));
    int16_t *code = reinterpret_cast<int16_t *>(take(N * sizeof(int16_t)));
    void *tmp = take(N * (fp64 ? sizeof(double) : sizeof(float)));
    float *speed32 = fp64 ? nullptr : reinterpret_cast<float *>(take(N * sizeof(float)));
    float *drift32 = (fp64 || !fine->drift)
                         ? nullptr
                         : reinterpret_cast<float *>(take(N * dim * sizeof(float)));
    HJB_REQUIRE(off <= kScratchBytes, "problem needs %zu bytes of scratch, %zu available", off,
                kScratchBytes);

    // Checks of hjb_solve_global, with the device scan in scratch.
    validate_problem(fine, s, nullptr, scan);
    // Control tables as the other solves build them: rows padded to whole
    // groups of four plus one more group repeating the last control; FP32
    // rows carry s_d a_kd.
    double ch[255 * 3];
    HJB_HIP(hipMemcpyAsync(ch, fine->controls, (size_t)nc * dim * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HJB_HIP(hipStreamSynchronize(s));
    double pad64[(255 + 8) * 3];
    float pad32[(255 + 8) * 3];
    for (int k = 0; k < rows; ++k)
      for (int d = 0; d < dim; ++d) {
        const double a = ch[(size_t)(k < nc ? k : nc - 1) * dim + d];
        pad64[(size_t)k * dim + d] = a;
        pad32[(size_t)k * dim + d] = (float)(fine->step[d] * a);
      }
    HJB_HIP(hipMemcpyAsync(ctrl64, pad64, (size_t)rows * dim * sizeof(double),
                           hipMemcpyHostToDevice, s));
    HJB_HIP(hipMemcpyAsync(ctrl32, pad32, (size_t)rows * dim * sizeof(float),
                           hipMemcpyHostToDevice, s));
    if (!fp64) {
      HJB_HIP(launch_f64_to_f32(fine->speed, speed32, N, s));
      if (fine->drift) HJB_HIP(launch_scaled_f32(fine->drift, drift32, N, dim, fine->step, s));
    }
    HJB_HIP(launch_make_code(fine->target_part, nullptr, nullptr, N, code, s));

    DevProblem d;
    std::memset(&d, 0, sizeof d);
    d.dim = dim;
    for (int a = 0; a < 3; ++a) {
      d.n[a] = fine->n[a];
      d.step[a] = fine->step[a];
    }
    d.nc = nc;
    d.has_drift = fine->drift ? 1 : 0;
    d.beta = fine->beta;
    d.omb = fine->one_minus_beta;
    d.betaf = (float)fine->beta;
    d.ombf = (float)fine->one_minus_beta;
    d.ctrl64 = ctrl64;
    d.ctrl32 = ctrl32;
    d.speed64 = fine->speed;
    d.speed32 = speed32;
    d.drift64 = fine->drift;
    d.drift32 = drift32;
    d.code = code;

    HJB_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(active), 0u, 2, s));
    HJB_HIP(launch_count_active(code, N, active, s));
    unsigned long long nact = 0;
    HJB_HIP(hipMemcpyAsync(&nact, active, sizeof nact, hipMemcpyDeviceToHost, s));
    unsigned long long hres[kPoll];
    const JacobiWork w{tmp, dprob, res, hres};
    hjb_stats local;
    std::memset(&local, 0, sizeof local);
    const int status = run_jacobi_in(d, N, fp64, v_out, tol, max_sweeps > 0 ? max_sweeps : 1000000,
                                     kPoll, false, w, s, &local);
    if (st) {
      *st = local;
      st->node_updates = (int64_t)nact * local.rounds;
      st->updates = st->node_updates * nc;
      st->status = status;
      st->ms_wall = now_ms() - t0;
    }
    return status;
  });
}

}  // extern "C"
