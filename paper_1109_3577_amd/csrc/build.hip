// Kernels of Steps 2 and 3.1 of the Patchy Algorithm (Section 3 of the
// paper), all in FP64 with separate multiplies and adds so that the labels
// they produce are reproducible bit for bit by a plain CPU evaluation:
//
//   k_prolong        U^(0) = linear interpolation of the coarse values;
//   k_feedback       discrete feedback, eq. feedbackcontrol: the first
//                    control minimising the scheme's right-hand side at the
//                    foot point, beta_k I[U^(0)] + 1 - beta_k (I alone when
//                    beta does not depend on the control);
//   k_trace          colour transport with frozen feedback, eq.
//                    HJBridotta_discreta, for a chunk of parts at once,
//                    iterated from below (phi <- max(phi, I[phi])) on LDS
//                    tiles with active-tile lists until nothing changes;
//   k_labels         projection/assembly (eq. proiezionecolore, Remark 3.1):
//                    argmax over the parts, lowest index on ties;
//   k_piece_*        pieces of a patch cut off from its own target part
//                    (union-find over equal labels) are uncoloured;
//   k_label_fill     uncoloured nodes take their neighbours' colour
//                    (Remark 3.1), one layer per launch.
//
// The transport update is monotone in the colours and starts from below,
// so like the value iteration it reaches the same least fixed point in any
// fair order; the tiled schedule changes the work, not the bits.

#include "device_math.h"
#include "hjb_internal.h"

namespace hjb {

// ---------------------------------------------------------------- prolongation

template <int DIM>
__global__ void k_prolong(int nf0, int nf1, int nf2, int nc0, int nc1, const double *__restrict__ vc,
                          const int32_t *__restrict__ Q, const double *__restrict__ T, double *u0) {
  const size_t N = (size_t)nf0 * nf1 * nf2;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int x = (int)(g % nf0), y = (int)((g / nf0) % nf1), z = (int)(g / ((size_t)nf0 * nf1));
  // per-axis tables: [0, nf0) x, [nf0, nf0+nf1) y, then z
  const int qx = Q[x], qy = Q[nf0 + y];
  const double tx = T[x], ty = T[nf0 + y];
  int qz = 0;
  double tz = 0.0;
  if (DIM == 3) {
    qz = Q[nf0 + nf1 + z];
    tz = T[nf0 + nf1 + z];
  }
  auto cv = [&](int a, int b, int c) {
    return vc[(size_t)(qx + a) + (size_t)nc0 * ((size_t)(qy + b) + (size_t)nc1 * (qz + c))];
  };
  double r0 = Ar<double>::lin(tx, cv(0, 0, 0), cv(1, 0, 0));
  double r1 = Ar<double>::lin(tx, cv(0, 1, 0), cv(1, 1, 0));
  double val = Ar<double>::lin(ty, r0, r1);
  if (DIM == 3) {
    double q0 = Ar<double>::lin(tx, cv(0, 0, 1), cv(1, 0, 1));
    double q1 = Ar<double>::lin(tx, cv(0, 1, 1), cv(1, 1, 1));
    double v1 = Ar<double>::lin(ty, q0, q1);
    val = Ar<double>::lin(tz, val, v1);
  }
  u0[g] = val;
}

hipError_t launch_prolong(int dim, const int32_t nf[3], const int32_t nc[3], const double *vc,
                          const int32_t *Q, const double *T, double *u0, hipStream_t s) {
  const size_t N = (size_t)nf[0] * nf[1] * nf[2];
  const dim3 grid((unsigned)((N + 255) / 256));
  if (dim == 2)
    hipLaunchKernelGGL(k_prolong<2>, grid, dim3(256), 0, s, nf[0], nf[1], nf[2], nc[0], nc[1], vc,
                       Q, T, u0);
  else
    hipLaunchKernelGGL(k_prolong<3>, grid, dim3(256), 0, s, nf[0], nf[1], nf[2], nc[0], nc[1], vc,
                       Q, T, u0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- feedback

// Foot-point displacement d = s (c a_k + w), FP64, separate operations.
template <int DIM>
__device__ __forceinline__ void displacement64(const TraceArgs &a, size_t g, int k, double *d) {
  if (a.foot) {  // tabulated dynamics
#pragma unroll
    for (int q = 0; q < DIM; ++q) d[q] = a.foot[((size_t)k * a.N + g) * DIM + q];
    return;
  }
  const double c = a.speed64[g];
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    double gg = c * a.ctrl64[k * DIM + q];
    if (a.has_drift) gg = gg + a.drift64[g * DIM + q];
    d[q] = a.step[q] * gg;
  }
}

template <int DIM>
__global__ void __launch_bounds__(256)
k_feedback(TraceArgs a, const double *__restrict__ u0, uint8_t *__restrict__ fb) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.N) return;
  if (a.target_part[g] != -1) {  // target or obstacle: no feedback
    fb[g] = 255;
    return;
  }
  const int px = (int)(g % a.n[0]), py = (int)((g / a.n[0]) % a.n[1]);
  const int pz = (int)(g / ((size_t)a.n[0] * a.n[1]));
  double best = 0.0;
  int bk = 0;
  for (int k = 0; k < a.nc; ++k) {
    double d[DIM];
    displacement64<DIM>(a, g, k, d);
    double I = interp_global<double, DIM>(u0, a.n, px, py, pz, d);
    if (a.beta_pk) {
      // the step depends on the control: compare the scheme's right-hand
      // side beta_k I + 1 - beta_k (time at the foot plus the step)
      const double b = a.beta_pk[(size_t)k * a.N + g];
      const double bI = b * I;
      I = bI + (1.0 - b);
    }
    if (k == 0 || I < best) {
      best = I;
      bk = k;
    }
  }
  fb[g] = (uint8_t)bk;
}

hipError_t launch_feedback(int dim, const TraceArgs &a, const double *u0, uint8_t *fb,
                           hipStream_t s) {
  const dim3 grid((unsigned)((a.N + 255) / 256));
  if (dim == 2) hipLaunchKernelGGL(k_feedback<2>, grid, dim3(256), 0, s, a, u0, fb);
  else hipLaunchKernelGGL(k_feedback<3>, grid, dim3(256), 0, s, a, u0, fb);
  return hipGetLastError();
}

// ---------------------------------------------------------------- tracing
//
// All parts are transported in one pass.  phi[j][N] holds every part's
// colour (zero-initialised, so any value read is a valid lower bound), and
// mask[tile][w] has bit j set once part j is nonzero somewhere in the tile.
// An activation loads only the parts whose bit is set in its tile or a
// neighbouring tile (the others are zero in its whole stencil region and
// stay zero); each part's transport is independent of the others, so
// processing a subset changes no bit of any colour.

// Colour update phi <- max(phi, Q(beta I[phi])): beta = exp(-h) is the
// scheme's per-step factor in the Kruzkov variable, so a colour is the
// share of exp(-T) part j carries along the frozen feedback and the map is a
// beta-contraction (undamped, near-closed loops of the frozen feedback make
// the iteration contract arbitrarily slowly).  Q rounds down to a multiple
// of 2^-24: only the projection of the colours is used (the paper lets this
// iteration stop very roughly), so increments below the lattice spacing are
// not pursued, and each part's support stays compact.  Q is monotone, so
// the rounded map is too, and every fair order of updates stops at the same
// colours.  Scaling by a power of two is exact.
constexpr double kColourLattice = 16777216.0;  // 2^24

// Colour-transport tiles: 2D 32 x 16 nodes, 512 threads, 8 FP64 fields per
// LDS group, up to 24 in-tile sweeps per activation; 3D 8 x 8 x 8, 256
// threads, 2 fields, 6 sweeps.  In 2D a tile sees about 2 parts and the
// rounds are latency-bound; in 3D trilinear transport mixes the colours of
// the 64 small target parts (about 15 per tile) and the work is throughput-
// bound, where small LDS groups (more workgroups per CU) and short
// activations pay.
constexpr int TR2_TX = 32, TR2_TY = 16, TR2_NT = 512, TR2_CL = 8, TR2_K = 24, TR2_SPLIT = 2;
constexpr int TR3_TX = 8, TR3_TY = 8, TR3_TZ = 8, TR3_NT = 256, TR3_CL = 2, TR3_K = 6;
constexpr int kMaxTraceWords = 32;  // up to 1024 parts

int trace_chunk_capacity(int dim) { return dim == 2 ? TR2_CL : TR3_CL; }
int trace_max_parts() { return kMaxTraceWords * 32; }
int trace_inner_sweeps(int dim) { return dim == 2 ? TR2_K : TR3_K; }
int trace_split(int dim, size_t jobs) { return dim == 2 && jobs == 1 ? TR2_SPLIT : 1; }
SweepShape trace_shape(int dim) {
  return dim == 2 ? SweepShape{2, TR2_TX, TR2_TY, 1, TR2_NT}
                  : SweepShape{3, TR3_TX, TR3_TY, TR3_TZ, TR3_NT};
}

// phi = 1 on the target nodes of their own part (the rest of phi is zero
// from a fill), and the part bit of the node's tile.
__global__ void k_trace_init(TraceArgs a, int tx, int ty, int tz) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.N) return;
  const int tp = a.target_part[g];
  if (tp < 0) return;
  a.phi[(size_t)tp * a.N + g] = 1.0;
  const int x = (int)(g % a.n[0]), y = (int)((g / a.n[0]) % a.n[1]);
  const int z = (int)(g / ((size_t)a.n[0] * a.n[1]));
  const int t = x / tx + a.ntile[0] * (y / ty + a.ntile[1] * (z / tz));
  atomicOr(&a.masks[(size_t)t * a.words + (tp >> 5)], 1u << (tp & 31));
}

hipError_t launch_trace_init(int dim, const TraceArgs &a, hipStream_t s) {
  const SweepShape sh = trace_shape(dim);
  hipLaunchKernelGGL(k_trace_init, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, s, a, sh.tx,
                     sh.ty, sh.tz);
  return hipGetLastError();
}

// One colour update from the corner values of the foot cell (x fastest):
// beta times the nested linear interpolation, rounded down to the lattice.
template <int DIM>
__device__ __forceinline__ double colour_step(const double *c, double t0, double t1, double t2,
                                              double beta) {
  const double r0 = Ar<double>::lin(t0, c[0], c[1]);
  const double r1 = Ar<double>::lin(t0, c[2], c[3]);
  double I = Ar<double>::lin(t1, r0, r1);
  if (DIM == 3) {
    const double q0 = Ar<double>::lin(t0, c[4], c[5]);
    const double q1 = Ar<double>::lin(t0, c[6], c[7]);
    const double I1 = Ar<double>::lin(t1, q0, q1);
    I = Ar<double>::lin(t2, I, I1);
  }
  I = beta * I;
  return __builtin_floor(I * kColourLattice) * (1.0 / kColourLattice);
}

// A load from a device buffer through the global address space.  The
// problem's pointers are read from a device table, so the compiler takes them
// as generic and would emit flat loads (which count against the LDS counter
// too, so every LDS wait would also wait for them).
template <typename T>
__device__ __forceinline__ T gld(const T *p, size_t i) {
  return ((const __attribute__((address_space(1))) T *)p)[i];
}

// A round of tile activations.  The list holds tile ids of one or several
// problems of the same dimension: tile_prob (null: every tile is of
// problem 0) names the problem of a tile id, whose tiles are numbered from
// its tile_base.
// Each activation is shared by SPLIT workgroups (trace_split): share h
// transports the parts whose index is h mod SPLIT.  The parts' transports are independent
// (one frozen foot point per node, no minimum over parts), and a part
// always has the same owner, so no two workgroups write the same field of
// a tile; each share queues the neighbours its own changes reach.
// In 3D the kernel is throughput-bound: asking for 4 waves per SIMD caps it
// at 128 registers (147 otherwise, 3 waves), 8% faster despite a few spills.
template <int DIM, int TX, int TY, int TZ, int NT, int CL, int SPLIT>
__global__ void __launch_bounds__(NT, DIM == 3 ? 4 : 1)
k_trace(const TraceArgs *__restrict__ args, const int32_t *__restrict__ tile_prob, RoundArgs ra) {
  constexpr int LX = TX + 2 * HALO;
  constexpr int LY = TY + 2 * HALO;
  constexpr int LZ = (DIM == 3) ? TZ + 2 * HALO : 1;
  constexpr int LN = LX * LY * LZ;
  constexpr int TN = TX * TY * (DIM == 3 ? TZ : 1);
  constexpr int NPT = TN / NT;  // bricks per wave
  constexpr int NW = NT / 64;
  constexpr int BX = Brick<DIM>::X, BY = Brick<DIM>::Y, BZ = Brick<DIM>::Z;
  constexpr int NBX = TX / BX, NBY = TY / BY, NBZ = (DIM == 3) ? TZ / BZ : 1;
  static_assert(TN % NT == 0 && NT % 64 == 0, "tile must be a multiple of the block");
  static_assert(TX % BX == 0 && TY % BY == 0 && (DIM == 2 || TZ % BZ == 0), "brick tiling");
  static_assert(NBX * NBY * NBZ <= 32, "brick mask is one word");
  __shared__ double s_phi[CL * LN];
  __shared__ uint32_t s_msk[4];
  __shared__ uint32_t s_act[kMaxTraceWords];
  __shared__ int s_list[kMaxTraceWords * 32];
  __shared__ int s_nact;
  __shared__ int s_int[8];
  __shared__ int s_nz[CL];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const uint32_t r = ra.round;
  if (blockIdx.x == 0 && tid == 0) ra.count[(r + 2) % 3] = 0u;
  const uint32_t nin = ra.count[r % 3];
  const int K = ra.inner_sweeps;

  const unsigned long long nvirt = (unsigned long long)nin * SPLIT;
  for (unsigned long long vi = blockIdx.x; vi < nvirt; vi += gridDim.x) {
    const uint32_t li = (uint32_t)(vi / SPLIT);
    const int share = (int)(vi % SPLIT);
    const int gt = ra.list_in[li];
    const TraceArgs a = args[tile_prob ? tile_prob[gt] : 0];
    const int tt = gt - a.tile_base;
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const int W = a.words;
    if (tid == 0) ra.flags_in[gt] = 0u;
    const int tix = tt % a.ntile[0];
    const int tiy = (tt / a.ntile[0]) % a.ntile[1];
    const int tiz = tt / (a.ntile[0] * a.ntile[1]);
    const int ox = tix * TX, oy = tiy * TY, oz = (DIM == 3) ? tiz * TZ : 0;

    // Parts present in the stencil region: OR of the neighbourhood masks.
    for (int w = tid; w < W; w += NT) s_act[w] = 0u;
    __syncthreads();
    constexpr int NNB = (DIM == 3) ? 27 : 9;
    for (int i = tid; i < NNB * W; i += NT) {
      const int nb = i / W, w = i % W;
      const int dx = nb % 3 - 1, dy = (nb / 3) % 3 - 1, dz = (DIM == 3) ? nb / 9 - 1 : 0;
      const int nx = tix + dx, ny = tiy + dy, nz = tiz + dz;
      if (nx < 0 || ny < 0 || nz < 0 || nx >= a.ntile[0] || ny >= a.ntile[1] || nz >= a.ntile[2])
        continue;
      const uint32_t m = a.masks[(size_t)(nx + a.ntile[0] * (ny + a.ntile[1] * nz)) * W + w];
      if (m) atomicOr(&s_act[w], m);
    }
    __syncthreads();
    if (tid == 0) {
      int c = 0;
      for (int w = 0; w < W; ++w) {
        uint32_t b = s_act[w];
        while (b) {
          const int j = __builtin_ctz(b);
          b &= b - 1u;
          const int part = w * 32 + j;
          if (SPLIT == 1 || part % SPLIT == share) s_list[c++] = part;
        }
      }
      s_nact = c;
    }
    if constexpr (SPLIT > 1) {
      // a share with no part of its own has nothing to transport or queue
      __syncthreads();
      if (s_nact == 0) {
        if (tid == 0 && share == 0) atomicAdd(&ra.work[kSlots + blockIdx.x % kSlots], 1ull);
        __syncthreads();  // s_act and s_list are rewritten by the next entry
        continue;
      }
    }

    // Per owned node: fixed foot point of its feedback control (FP64).
    // This thread's nodes: lane `lane` of brick `wave + j NW`, j < NPT.
    int base[NPT], own[NPT];
    double t0[NPT], t1[NPT], t2[NPT];
    double bt[NPT];  // the node's per-step factor (per-node beta of the variable step)
    bool act[NPT], any[NPT];
    size_t gid[NPT];
    uint32_t nbm[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      const int bb = wave + j * NW;
      const int lx = (bb % NBX) * BX + lane % BX;
      const int ly = ((bb / NBX) % NBY) * BY + (lane / BX) % BY;
      const int lz = (bb / (NBX * NBY)) * BZ + lane / (BX * BY);
      nbm[j] = brick_neighbours<NBX, NBY, NBZ>(bb);
      any[j] = false;
      const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
      bool inb = gx < n0 && gy < n1;
      if (DIM == 3) inb = inb && gz < n2;
      const size_t g = (size_t)gx + (size_t)n0 * ((size_t)gy + (size_t)n1 * (DIM == 3 ? gz : 0));
      gid[j] = g;
      // The node's role, feedback, speed, drift and beta are loaded whatever
      // the role (from node 0 outside the box) so that they are in flight
      // together; only the control row and the tables wait for the feedback.
      const size_t gs = inb ? g : 0;
      const int tp = gld(a.target_part, gs);
      const int fbk = gld(a.feedback, gs);
      const double sp = a.foot ? 0.0 : gld(a.speed64, gs);
      double dr[DIM];
#pragma unroll
      for (int q = 0; q < DIM; ++q) dr[q] = a.has_drift ? gld(a.drift64, gs * DIM + q) : 0.0;
      const double bn = a.beta_node ? gld(a.beta_node, gs) : a.beta;
      act[j] = inb && tp == -1;
      own[j] = (lx + HALO) + LX * ((ly + HALO) + LY * (DIM == 3 ? lz + HALO : 0));
      base[j] = own[j];
      t0[j] = t1[j] = t2[j] = 0.0;
      bt[j] = !act[j]       ? a.beta
              : a.beta_pk   ? a.beta_pk[(size_t)fbk * a.N + g]
              : a.beta_node ? bn
                            : a.beta;
      if (act[j]) {
        // displacement of the feedback control (as in displacement64)
        double d[DIM];
        if (a.foot) {
#pragma unroll
          for (int q = 0; q < DIM; ++q) d[q] = a.foot[((size_t)fbk * a.N + g) * DIM + q];
        } else {
#pragma unroll
          for (int q = 0; q < DIM; ++q) {
            double gg = sp * a.ctrl64[fbk * DIM + q];
            if (a.has_drift) gg = gg + dr[q];
            d[q] = a.step[q] * gg;
          }
        }
        const double f0 = __builtin_floor(d[0]), f1 = __builtin_floor(d[1]);
        t0[j] = d[0] - f0;
        t1[j] = d[1] - f1;
        int o = own[j] + (int)f0 + (int)f1 * LX;
        if (DIM == 3) {
          const double f2 = __builtin_floor(d[2]);
          t2[j] = d[2] - f2;
          o += (int)f2 * (LX * LY);
        }
        base[j] = o;
      }
    }
    if (tid < 8) s_int[tid] = tid < 3 ? (1 << 30) : -1;
    __syncthreads();
    const int nact = s_nact;
    bool converged_all = true;

    for (int g0 = 0; g0 < nact; g0 += CL) {
      const int nf = min(CL, nact - g0);
      // Stage the group's fields (tile + halo, 0 outside the box).
      if constexpr (DIM == 3) {
        // 7 elements per thread and field: all of them are loaded before
        // the first LDS store, so that one wait covers them instead of one
        // round trip per element (a quarter of the 3D build time; four at a
        // time cost 3% more, two 8% more)
        constexpr int SIT = (LN + NT - 1) / NT;  // elements per thread
        constexpr int SQ = SIT;                    // of them in flight at once
        const double *src[CL];
#pragma unroll
        for (int f = 0; f < CL; ++f)
          src[f] = a.phi +
                   (size_t)__builtin_amdgcn_readfirstlane(s_list[g0 + (f < nf ? f : 0)]) * a.N;
#pragma unroll
        for (int q0 = 0; q0 < SIT; q0 += SQ) {
          double sv[SQ][CL];
#pragma unroll
          for (int q = 0; q < SQ; ++q) {
            const int i = tid + (q0 + q) * NT;
            const int lx = i % LX, ly = (i / LX) % LY, lz = i / (LX * LY);
            const int gx = ox + lx - HALO, gy = oy + ly - HALO, gz = oz + lz - HALO;
            const bool inb = q0 + q < SIT && i < LN && (unsigned)gx < (unsigned)n0 &&
                             (unsigned)gy < (unsigned)n1 && (unsigned)gz < (unsigned)n2;
            const size_t g = inb ? (size_t)gx + (size_t)n0 * ((size_t)gy + (size_t)n1 * gz) : 0;
#pragma unroll
            for (int f = 0; f < CL; ++f) sv[q][f] = (f < nf && inb) ? gld(src[f], g) : 0.0;
          }
#pragma unroll
          for (int q = 0; q < SQ; ++q) {
            const int i = tid + (q0 + q) * NT;
            if (q0 + q < SIT && i < LN) {
#pragma unroll
              for (int f = 0; f < CL; ++f)
                if (f < nf) s_phi[f * LN + i] = sv[q][f];
            }
          }
        }
      } else {
        for (int i = tid; i < LN; i += NT) {
          const int lx = i % LX, ly = i / LX;
          const int gx = ox + lx - HALO, gy = oy + ly - HALO;
          const bool inb = (unsigned)gx < (unsigned)n0 && (unsigned)gy < (unsigned)n1;
          const size_t g = inb ? (size_t)gx + (size_t)n0 * (size_t)gy : 0;
#pragma unroll
          for (int f = 0; f < CL; ++f)
            if (f < nf) s_phi[f * LN + i] = inb ? a.phi[(size_t)s_list[g0 + f] * a.N + g] : 0.0;
        }
      }
      if (tid < CL) s_nz[tid] = 0;
      // brick-change masks in rotation (as in the value sweep): sweep s
      // reads the mask of sweep s - 1; every brick is swept first
      if (tid == 0) {
        s_msk[0] = 0u;
        s_msk[1] = 0u;
        s_msk[2] = ~0u;
      }
      __syncthreads();
      double old[NPT][CL];
#pragma unroll
      for (int j = 0; j < NPT; ++j)
#pragma unroll
        for (int f = 0; f < CL; ++f) old[j][f] = f < nf ? s_phi[f * LN + own[j]] : 0.0;

      bool converged = false;
      for (int it = 0; it < K; ++it) {
        const uint32_t prev = s_msk[(it + 2) % 3];
        if (tid == 0) s_msk[(it + 1) % 3] = 0u;
        uint32_t mine = 0u;
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
          // a brick none of whose neighbours changed in the last sweep
          // would read the same colours again
          if ((prev & nbm[j]) == 0u) continue;
          bool ch = false;
          const int o = base[j];
#pragma unroll
          for (int f = 0; f < CL; ++f) {
            if (f >= nf) break;
            const double *sp = s_phi + f * LN;
            double c[8];
            c[0] = sp[o];
            c[1] = sp[o + 1];
            c[2] = sp[o + LX];
            c[3] = sp[o + LX + 1];
            if (DIM == 3) {
              const int oz = o + LX * LY;
              c[4] = sp[oz];
              c[5] = sp[oz + 1];
              c[6] = sp[oz + LX];
              c[7] = sp[oz + LX + 1];
            }
            const double I = colour_step<DIM>(c, t0[j], t1[j], t2[j], bt[j]);
            if (act[j] && I > sp[own[j]]) {
              s_phi[f * LN + own[j]] = I;
              ch = true;
            }
          }
          if (__ballot(ch) != 0ull) mine |= 1u << (wave + j * NW);
        }
        if (lane == 0 && mine) atomicOr(&s_msk[it % 3], mine);
        __syncthreads();
        if (s_msk[it % 3] == 0u) {
          converged = true;
          break;
        }
      }
      if (!converged) converged_all = false;

#pragma unroll
      for (int j = 0; j < NPT; ++j) {
        if (!act[j]) continue;
        bool changed = false;
#pragma unroll
        for (int f = 0; f < CL; ++f) {
          if (f >= nf) break;
          const double nv = s_phi[f * LN + own[j]];
          if (nv != old[j][f]) {
            a.phi[(size_t)s_list[g0 + f] * a.N + gid[j]] = nv;
            changed = true;
            if (old[j][f] == 0.0) s_nz[f] = 1;
          }
        }
        any[j] = any[j] || changed;
      }
      __syncthreads();
      if (tid < nf && s_nz[tid]) {
        const int part = s_list[g0 + tid];
        atomicOr(&a.masks[(size_t)tt * W + (part >> 5)], 1u << (part & 31));
      }
      __syncthreads();  // LDS is refilled by the next group
    }

    // changed-node box: per brick from a wave ballot, merged by one LDS
    // atomic per wave
    int bx0 = 1 << 30, by0 = 1 << 30, bz0 = 1 << 30, bx1 = -1, by1 = -1, bz1 = -1;
#pragma unroll
    for (int j = 0; j < NPT; ++j)
      brick_box<DIM, NBX, NBY>(__ballot(any[j]), wave + j * NW, bx0, bx1, by0, by1, bz0, bz1);
    if (lane == 0 && bx1 >= 0) {
      atomicMin(&s_int[0], bx0); atomicMin(&s_int[1], by0); atomicMin(&s_int[2], bz0);
      atomicMax(&s_int[3], bx1); atomicMax(&s_int[4], by1); atomicMax(&s_int[5], bz1);
    }
    const int conv_all = __syncthreads_and(converged_all ? 1 : 0);
    const int cx0 = s_int[0], cy0 = s_int[1], cz0 = s_int[2];
    const int cx1 = s_int[3], cy1 = s_int[4], cz1 = s_int[5];
    if (cx1 >= 0 && tid < 64) {
      int qt = -1;
      if (tid < NNB) {
        const int dx = tid % 3 - 1, dy = (tid / 3) % 3 - 1, dz = (DIM == 3) ? tid / 9 - 1 : 0;
        bool need;
        if (dx == 0 && dy == 0 && dz == 0) need = !conv_all;
        else
          need = (dx < 0 ? cx0 < HALO : dx > 0 ? cx1 >= TX - HALO : true) &&
                 (dy < 0 ? cy0 < HALO : dy > 0 ? cy1 >= TY - HALO : true) &&
                 (dz < 0 ? cz0 < HALO : dz > 0 ? cz1 >= TZ - HALO : true);
        const int nx = tix + dx, ny = tiy + dy, nz = tiz + dz;
        if (need && nx >= 0 && ny >= 0 && nz >= 0 && nx < a.ntile[0] && ny < a.ntile[1] &&
            nz < a.ntile[2]) {
          const int t2 = a.tile_base + nx + a.ntile[0] * (ny + a.ntile[1] * nz);
          if (atomicCAS(&ra.flags_out[t2], 0u, 1u) == 0u) qt = t2;
        }
      }
      queue_items(ra, qt, nullptr);
    }
    if (tid == 0) {
      const int slot = blockIdx.x % kSlots;
      if (share == 0) atomicAdd(&ra.work[kSlots + slot], 1ull);
      atomicAdd(&ra.work[slot], (unsigned long long)nact);
    }
    __syncthreads();
  }
}

hipError_t launch_trace(int dim, int grid, int split, const TraceArgs *args,
                        const int32_t *tile_prob, int max_words, const RoundArgs &ra,
                        hipStream_t s) {
  if (max_words > kMaxTraceWords) return hipErrorInvalidValue;
  if (dim == 2 && split == TR2_SPLIT)
    hipLaunchKernelGGL((k_trace<2, TR2_TX, TR2_TY, 1, TR2_NT, TR2_CL, TR2_SPLIT>), dim3(grid),
                       dim3(TR2_NT), 0, s, args, tile_prob, ra);
  else if (dim == 2 && split == 1)
    hipLaunchKernelGGL((k_trace<2, TR2_TX, TR2_TY, 1, TR2_NT, TR2_CL, 1>), dim3(grid),
                       dim3(TR2_NT), 0, s, args, tile_prob, ra);
  else if (dim == 3 && split == 1)
    hipLaunchKernelGGL((k_trace<3, TR3_TX, TR3_TY, TR3_TZ, TR3_NT, TR3_CL, 1>), dim3(grid),
                       dim3(TR3_NT), 0, s, args, tile_prob, ra);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Queue, for round 0, every tile next to (or holding) a tile with a target
// node: one thread per tile reads the part masks of its neighbourhood.
__global__ void k_trace_seed(TraceArgs a, RoundArgs ra) {
  const int ntiles = a.ntile[0] * a.ntile[1] * a.ntile[2];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int q = -1;
  if (t < ntiles) {
    const int tx = t % a.ntile[0], ty = (t / a.ntile[0]) % a.ntile[1];
    const int tz = t / (a.ntile[0] * a.ntile[1]);
    const int dz0 = a.ntile[2] > 1 ? -1 : 0, dz1 = a.ntile[2] > 1 ? 1 : 0;
    bool near = false;
    for (int dz = dz0; dz <= dz1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int x = tx + dx, y = ty + dy, z = tz + dz;
          if (x < 0 || y < 0 || z < 0 || x >= a.ntile[0] || y >= a.ntile[1] || z >= a.ntile[2])
            continue;
          const size_t nb = (size_t)(x + a.ntile[0] * (y + a.ntile[1] * z));
          for (int w = 0; w < a.words; ++w) near = near || a.masks[nb * a.words + w] != 0u;
        }
    if (near) {
      ra.flags_out[a.tile_base + t] = 1u;
      q = a.tile_base + t;
    }
  }
  queue_items(ra, q, nullptr);
}

hipError_t launch_trace_seed(int dim, const TraceArgs &a, const RoundArgs &ra, hipStream_t s) {
  (void)dim;
  const int ntiles = a.ntile[0] * a.ntile[1] * a.ntile[2];
  hipLaunchKernelGGL(k_trace_seed, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, a, ra);
  return hipGetLastError();
}

// ---------------------------------------------------------------- labels

// Label of every node (eq. proiezionecolore with Remark 3.1): its part on
// the target; elsewhere the part with the largest colour, lowest index on
// ties (ascending scan, strict >), -1 when every colour is zero.  Only the
// parts set in the node's tile mask can be nonzero there.
__global__ void k_labels(TraceArgs a, int tx, int ty, int tz, int16_t *labels, uint32_t *unreached) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int u = 0;
  if (g < a.N) {
    const int tp = a.target_part[g];
    if (tp >= 0 || tp == TP_OBSTACLE) {
      labels[g] = (int16_t)tp;
    } else {
      const int x = (int)(g % a.n[0]), y = (int)((g / a.n[0]) % a.n[1]);
      const int z = (int)(g / ((size_t)a.n[0] * a.n[1]));
      const size_t t = (size_t)(x / tx + a.ntile[0] * (y / ty + a.ntile[1] * (z / tz)));
      double best = 0.0;
      int L = -1;
      for (int w = 0; w < a.words; ++w) {
        uint32_t b = a.masks[t * a.words + w];
        while (b) {
          const int j = w * 32 + __builtin_ctz(b);
          b &= b - 1u;
          const double p = a.phi[(size_t)j * a.N + g];
          if (p > best) {
            best = p;
            L = j;
          }
        }
      }
      labels[g] = (int16_t)L;
      u = L < 0;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) u += __shfl_xor(u, o, 64);
  if ((threadIdx.x & 63) == 0 && u) atomicAdd(unreached, (uint32_t)u);
}

hipError_t launch_labels(int dim, const TraceArgs &a, int16_t *labels, uint32_t *unreached,
                         hipStream_t s) {
  const SweepShape sh = trace_shape(dim);
  hipLaunchKernelGGL(k_labels, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, s, a, sh.tx,
                     sh.ty, sh.tz, labels, unreached);
  return hipGetLastError();
}

// ---------------------------------------------------------------- cut-off pieces

// The argmax projection can leave a piece of the nodes of label j that holds
// no target node of part j: no characteristic of patch j runs from it to its
// target part, and under the state constraint of Step 3.2 its values would
// stay at or near 1.  Pieces are connected through the 4 (2D) or 6 (3D) axis
// neighbours: a chain of nodes that touch only at corners is too thin for the
// interpolation stencil to carry values along it.  Such a piece is uncoloured
// (label -1) and then takes its neighbours' colour like the nodes no colour
// reached (Remark 3.1).  Target nodes carry their own part as label, so a
// piece is attached iff it contains a target node.
//
// The pieces are found by union-find: first within each tile in LDS, then
// across tile faces in global memory.  Parent pointers only ever decrease
// (atomicMin), so every chain ends at a root and the partition does not
// depend on the order of the unions.  Parent reads in the cross-tile merge go
// to the device-coherent level (the workgroups of one launch run on
// different XCDs).

constexpr int PC2_TX = 16, PC2_TY = 16;            // 2D piece tiles (256 nodes)
constexpr int PC3_TX = 8, PC3_TY = 8, PC3_TZ = 4;  // 3D piece tiles (256 nodes)

__device__ __forceinline__ int uf_root(const int32_t *p, int x) {
  int y = ld_dev(p + x);
  while (y != x) {
    x = y;
    y = ld_dev(p + x);
  }
  return x;
}

__device__ __forceinline__ void uf_unite(int32_t *p, int a, int b) {
  for (;;) {
    a = uf_root(p, a);
    b = uf_root(p, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    // link the larger root under the smaller; if a stopped being a root in
    // the meantime, its new parent is joined with b in the next pass
    const int old = atomicMin(p + a, b);
    if (old == a) return;
    a = old;
  }
}

__device__ __forceinline__ int lds_root(const int *p, int x) {
  int y = __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  while (y != x) {
    x = y;
    y = __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  return x;
}

__device__ __forceinline__ void lds_unite(int *p, int a, int b) {
  for (;;) {
    a = lds_root(p, a);
    b = lds_root(p, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(p + a, b);
    if (old == a) return;
    a = old;
  }
}

// Pieces within one tile: parent[g] = the smallest flat index of g's piece
// inside the tile (local order and flat order agree within a tile).
template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX * TY * TZ)
k_piece_local(int n0, int n1, int n2, int nt0, int nt1, const int16_t *__restrict__ labels,
              int32_t *parent) {
  constexpr int TN = TX * TY * TZ;
  __shared__ int s_par[TN];
  __shared__ int s_lab[TN];
  const int t = threadIdx.x;
  const int tile = blockIdx.x;
  const int ox = (tile % nt0) * TX, oy = ((tile / nt0) % nt1) * TY, oz = (tile / (nt0 * nt1)) * TZ;
  const int lx = t % TX, ly = (t / TX) % TY, lz = t / (TX * TY);
  const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
  const bool inb = gx < n0 && gy < n1 && gz < n2;
  const size_t g = (size_t)gx + (size_t)n0 * ((size_t)gy + (size_t)n1 * gz);
  const int L = inb ? labels[g] : -1;
  s_lab[t] = L;
  s_par[t] = t;
  __syncthreads();
  if (L >= 0) {
    if (lx + 1 < TX && s_lab[t + 1] == L) lds_unite(s_par, t, t + 1);
    if (ly + 1 < TY && s_lab[t + TX] == L) lds_unite(s_par, t, t + TX);
    if (TZ > 1 && lz + 1 < TZ && s_lab[t + TX * TY] == L) lds_unite(s_par, t, t + TX * TY);
  }
  __syncthreads();
  if (L >= 0) {
    const int r = lds_root(s_par, t);
    const int rx = ox + r % TX, ry = oy + (r / TX) % TY, rz = oz + r / (TX * TY);
    parent[g] = (int32_t)((size_t)rx + (size_t)n0 * ((size_t)ry + (size_t)n1 * rz));
  }
}

// Unions across tile faces: a labelled node on the +x, +y or +z face of its
// tile with the axis neighbour beyond it, when that carries the same label.
template <int TX, int TY, int TZ>
__global__ void k_piece_faces(int n0, int n1, int n2, const int16_t *__restrict__ labels,
                              int32_t *parent) {
  const size_t N = (size_t)n0 * n1 * n2;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int L = labels[g];
  if (L < 0) return;
  const int x = (int)(g % n0), y = (int)((g / n0) % n1), z = (int)(g / ((size_t)n0 * n1));
  if (x % TX == TX - 1 && x + 1 < n0 && labels[g + 1] == L) uf_unite(parent, (int)g, (int)g + 1);
  if (y % TY == TY - 1 && y + 1 < n1 && labels[g + n0] == L)
    uf_unite(parent, (int)g, (int)(g + n0));
  if (n2 > 1 && z % TZ == TZ - 1 && z + 1 < n2 && labels[g + (size_t)n0 * n1] == L)
    uf_unite(parent, (int)g, (int)(g + (size_t)n0 * n1));
}

__global__ void k_piece_clear(size_t N, uint8_t *attached) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < N) attached[g] = 0;
}

// Every labelled node points at its root; the root of a piece with a
// target node is marked attached.
__global__ void k_piece_flatten(size_t N, const int16_t *__restrict__ labels,
                                const int16_t *__restrict__ tp, int32_t *parent,
                                uint8_t *attached) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N || labels[g] < 0) return;
  const int r = uf_root(parent, (int)g);
  parent[g] = r;
  if (tp[g] == labels[g]) attached[r] = 1;  // a target node of the piece's part
}

__global__ void k_piece_detach(size_t N, const int16_t *__restrict__ tp,
                               const int32_t *__restrict__ parent,
                               const uint8_t *__restrict__ attached, int16_t *labels,
                               uint32_t *count) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int cut = 0;
  if (g < N && tp[g] < 0 && labels[g] >= 0 && !attached[parent[g]]) {
    labels[g] = -1;
    cut = 1;
  }
  for (int o = 32; o >= 1; o >>= 1) cut += __shfl_xor(cut, o, 64);
  if ((threadIdx.x & 63) == 0 && cut) atomicAdd(count, (uint32_t)cut);
}

hipError_t launch_detach_pieces(const int32_t n[3], const int16_t *tp, int16_t *labels,
                                int32_t *parent, uint8_t *attached, uint32_t *count,
                                hipStream_t s) {
  const size_t N = (size_t)n[0] * n[1] * n[2];
  const dim3 grid((unsigned)((N + 255) / 256)), block(256);
  if (n[2] == 1) {
    const int nt0 = (n[0] + PC2_TX - 1) / PC2_TX, nt1 = (n[1] + PC2_TY - 1) / PC2_TY;
    hipLaunchKernelGGL((k_piece_local<PC2_TX, PC2_TY, 1>), dim3((unsigned)(nt0 * nt1)),
                       dim3(PC2_TX * PC2_TY), 0, s, n[0], n[1], n[2], nt0, nt1, labels, parent);
    hipLaunchKernelGGL((k_piece_faces<PC2_TX, PC2_TY, 1>), grid, block, 0, s, n[0], n[1], n[2],
                       labels, parent);
  } else {
    const int nt0 = (n[0] + PC3_TX - 1) / PC3_TX, nt1 = (n[1] + PC3_TY - 1) / PC3_TY;
    const int nt2 = (n[2] + PC3_TZ - 1) / PC3_TZ;
    hipLaunchKernelGGL((k_piece_local<PC3_TX, PC3_TY, PC3_TZ>), dim3((unsigned)(nt0 * nt1 * nt2)),
                       dim3(PC3_TX * PC3_TY * PC3_TZ), 0, s, n[0], n[1], n[2], nt0, nt1, labels,
                       parent);
    hipLaunchKernelGGL((k_piece_faces<PC3_TX, PC3_TY, PC3_TZ>), grid, block, 0, s, n[0], n[1],
                       n[2], labels, parent);
  }
  hipLaunchKernelGGL(k_piece_clear, grid, block, 0, s, N, attached);
  hipLaunchKernelGGL(k_piece_flatten, grid, block, 0, s, N, labels, tp, parent, attached);
  hipLaunchKernelGGL(k_piece_detach, grid, block, 0, s, N, tp, parent, attached, labels, count);
  return hipGetLastError();
}

// Remark 3.1: a node no colour reached takes the smallest label among its
// labelled axis neighbours (4 in 2D, 6 in 3D), so that it joins a piece of
// that patch through a face.  One Jacobi layer per launch;
// repeated until nothing changes, the result is the lowest label among the
// nearest labelled nodes, independent of the launch schedule.
__global__ void k_label_fill(int n0, int n1, int n2, const int16_t *__restrict__ in, int16_t *out,
                             uint32_t *changed) {
  const size_t N = (size_t)n0 * n1 * n2;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  int L = in[g];
  if (L == -1) {  // not an obstacle (-2), not labelled
    const int x = (int)(g % n0), y = (int)((g / n0) % n1), z = (int)(g / ((size_t)n0 * n1));
    const int dz0 = n2 > 1 ? -1 : 0, dz1 = n2 > 1 ? 1 : 0;
    int best = -1;
    for (int dz = dz0; dz <= dz1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (abs(dx) + abs(dy) + abs(dz) != 1) continue;  // axis neighbours only
          const int X = x + dx, Y = y + dy, Z = z + dz;
          if (X < 0 || Y < 0 || Z < 0 || X >= n0 || Y >= n1 || Z >= n2) continue;
          const int M = in[(size_t)X + (size_t)n0 * ((size_t)Y + (size_t)n1 * Z)];
          if (M >= 0 && (best < 0 || M < best)) best = M;
        }
    if (best >= 0) {
      L = best;
      *changed = 1u;
    }
  }
  out[g] = (int16_t)L;
}

hipError_t launch_label_fill(const int32_t n[3], const int16_t *in, int16_t *out,
                             uint32_t *changed, hipStream_t s) {
  const size_t N = (size_t)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_label_fill, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, n[0], n[1],
                     n[2], in, out, changed);
  return hipGetLastError();
}

}  // namespace hjb
