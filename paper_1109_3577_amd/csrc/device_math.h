// Device arithmetic shared by every kernel of libhjb: the FP32 / FP64
// linear interpolation in weights form, the Kruzkov update and small
// reductions.  FP64 variants keep each multiply and add separate; the
// library is compiled with floating-point contraction off, so these are
// plain IEEE binary64 operations in a fixed order.
#pragma once

#include <hip/hip_runtime.h>

#include "hjb_internal.h"

namespace hjb {

typedef const __attribute__((address_space(4))) float *cf32p;
typedef const __attribute__((address_space(4))) double *cf64p;

// ---------------------------------------------------------------- arithmetic

template <typename T>
struct Ar;

template <>
struct Ar<float> {
  // (1 - t) lo + t hi in weights form: lo (1 - t) is one correctly rounded
  // fma, then t hi is fused on top.  Monotone in lo and hi, and exactly 1
  // when lo = hi = 1.
  static __device__ __forceinline__ float lin(float t, float lo, float hi) {
    return __builtin_fmaf(t, hi, __builtin_fmaf(-t, lo, lo));
  }
  static __device__ __forceinline__ float kruzkov(float b, float I, float omb) {
    return __builtin_fmaf(b, I, omb);
  }
  static __device__ __forceinline__ float flr(float x) { return __builtin_floorf(x); }
};

template <>
struct Ar<double> {
  static __device__ __forceinline__ double lin(double t, double lo, double hi) {
    double omt = 1.0 - t;
    double a = omt * lo;
    double b = t * hi;
    return a + b;
  }
  static __device__ __forceinline__ double kruzkov(double b, double I, double omb) {
    double x = b * I;
    return x + omb;
  }
  static __device__ __forceinline__ double flr(double x) { return __builtin_floor(x); }
};

// a * b + c on 24-bit unsigned operands in one instruction.  Written out so
// that the compiler keeps the multiply-add (two instructions with the final
// shift-add of the byte address) instead of distributing the word-to-byte
// shift over both terms (three instructions).
__device__ __forceinline__ int mad_u24(int a, int b, int c) {
  int r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

// LDS interpolation.  Corners enumerate x fastest; nesting x, then y, then
// z.  LXS is the row stride of the LDS tile (words), LY its rows.
//
// FP32 foot point in offset form: the foot-point fma yields y = d + 2 in
// [0, 4) (|d| < 2 is checked on the host), so the cell is a plain
// float-to-int conversion (truncation is floor on y >= 0) and the local
// coordinate is fract(y), exact on [0, 4).  The offset costs one rounding of
// the displacement at 2^-22 cells; every FP32 kernel uses this evaluation.
// `b2` is the LDS word index of the node minus 2 cells along every axis, so
// the lower corner is b2 + y0 + LXS y1 (+ LXS LY y2).
template <int DIM, int LXS, int LY>
__device__ __forceinline__ float interp_lds_f32(const float *s, int b2, const float *y) {
  const int i0 = (int)y[0];
  const int i1 = (int)y[1];
  const float t0 = __builtin_amdgcn_fractf(y[0]);
  const float t1 = __builtin_amdgcn_fractf(y[1]);
  int o = mad_u24(i1, LXS, i0);
  float t2 = 0.0f;
  if constexpr (DIM == 3) {
    const int i2 = (int)y[2];
    t2 = __builtin_amdgcn_fractf(y[2]);
    o = mad_u24(i2, LXS * LY, o);
  }
  const float *p = s + (b2 + o);
  const float r0 = Ar<float>::lin(t0, p[0], p[1]);
  const float r1 = Ar<float>::lin(t0, p[LXS], p[LXS + 1]);
  const float y0 = Ar<float>::lin(t1, r0, r1);
  if constexpr (DIM == 2) {
    return y0;
  } else {
    const float *q = p + LXS * LY;
    const float q0 = Ar<float>::lin(t0, q[0], q[1]);
    const float q1 = Ar<float>::lin(t0, q[LXS], q[LXS + 1]);
    const float y1 = Ar<float>::lin(t1, q0, q1);
    return Ar<float>::lin(t2, y0, y1);
  }
}

// FP64: displacement d (cells), cell floor(d), local coordinate d - floor(d),
// each multiply and add separate, as in the CPU evaluation.  `base` is the
// LDS word index of the node itself.
template <int DIM, int LXS, int LY>
__device__ __forceinline__ double interp_lds_f64(const double *s, int base, const double *d) {
  double f0 = Ar<double>::flr(d[0]), f1 = Ar<double>::flr(d[1]);
  double t0 = d[0] - f0, t1 = d[1] - f1;
  int o = base + (int)f0 + (int)f1 * LXS;
  double f2 = 0.0, t2 = 0.0;
  if constexpr (DIM == 3) {
    f2 = Ar<double>::flr(d[2]);
    t2 = d[2] - f2;
    o += (int)f2 * (LXS * LY);
  }
  double r0 = Ar<double>::lin(t0, s[o], s[o + 1]);
  double r1 = Ar<double>::lin(t0, s[o + LXS], s[o + LXS + 1]);
  double y0 = Ar<double>::lin(t1, r0, r1);
  if constexpr (DIM == 2) {
    return y0;
  } else {
    const int oz = o + LXS * LY;
    double q0 = Ar<double>::lin(t0, s[oz], s[oz + 1]);
    double q1 = Ar<double>::lin(t0, s[oz + LXS], s[oz + LXS + 1]);
    double y1 = Ar<double>::lin(t1, q0, q1);
    return Ar<double>::lin(t2, y0, y1);
  }
}

__device__ __forceinline__ void wave_min_i(int &x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
}

__device__ __forceinline__ void wave_max_i(int &x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
}

// Work of one wave is a brick of 64 nodes: 8 x 8 in 2D, 4 x 4 x 4 in 3D;
// lane = x + 8 y (2D), x + 4 y + 16 z (3D) within the brick.
template <int DIM>
struct Brick {
  static constexpr int X = DIM == 2 ? 8 : 4;
  static constexpr int Y = DIM == 2 ? 8 : 4;
  static constexpr int Z = DIM == 2 ? 1 : 4;
};

// Grows the box [x0, x1] x [y0, y1] x [z0, z1] (tile-local nodes) by the
// lanes set in `m` (a wave ballot) of brick `b` of a tile of NBX x NBY x .
// bricks.  Uniform across the wave.
template <int DIM, int NBX, int NBY>
__device__ __forceinline__ void brick_box(unsigned long long m, int b, int &x0, int &x1, int &y0,
                                          int &y1, int &z0, int &z1) {
  if (!m) return;
  constexpr int BX = Brick<DIM>::X, BY = Brick<DIM>::Y, BZ = Brick<DIM>::Z;
  const int ox = (b % NBX) * BX, oy = ((b / NBX) % NBY) * BY, oz = (b / (NBX * NBY)) * BZ;
  uint32_t xs, ys = 0u, zs;
  if constexpr (DIM == 2) {
    unsigned long long c = m | (m >> 32);
    c |= c >> 16;
    c |= c >> 8;
    xs = (uint32_t)(c & 0xffu);
#pragma unroll
    for (int y = 0; y < 8; ++y) ys |= ((m >> (8 * y)) & 0xffull) ? (1u << y) : 0u;
    zs = 1u;
  } else {
    const unsigned long long g = (m | (m >> 16) | (m >> 32) | (m >> 48)) & 0xffffull;
    unsigned long long c = g | (g >> 8);
    c |= c >> 4;
    xs = (uint32_t)(c & 0xfu);
    zs = 0u;
#pragma unroll
    for (int y = 0; y < 4; ++y) ys |= ((g >> (4 * y)) & 0xfull) ? (1u << y) : 0u;
#pragma unroll
    for (int z = 0; z < 4; ++z) zs |= ((m >> (16 * z)) & 0xffffull) ? (1u << z) : 0u;
  }
  x0 = min(x0, ox + __builtin_ctz(xs));
  x1 = max(x1, ox + 31 - __builtin_clz(xs));
  y0 = min(y0, oy + __builtin_ctz(ys));
  y1 = max(y1, oy + 31 - __builtin_clz(ys));
  z0 = min(z0, oz + __builtin_ctz(zs));
  z1 = max(z1, oz + 31 - __builtin_clz(zs));
}

// Bricks that a change in brick b can reach in one sweep (b and its
// neighbours; the reach, 2 nodes, is below the brick side).
template <int NBX, int NBY, int NBZ>
__device__ __forceinline__ uint32_t brick_neighbours(int b) {
  const int bx = b % NBX, by = (b / NBX) % NBY, bz = b / (NBX * NBY);
  uint32_t m = 0u;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = bx + dx, y = by + dy, z = bz + dz;
        if (x >= 0 && x < NBX && y >= 0 && y < NBY && z >= 0 && z < NBZ)
          m |= 1u << (x + NBX * (y + NBY * z));
      }
  return m;
}

template <typename T>
__device__ __forceinline__ void wave_max(T &x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    T y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
}

// Appends the items claimed by the lanes of one wave (it >= 0: this lane
// won the item's flag) to the next round's list: one atomic reserves the
// slots of the whole wave, and the problem's queued count grows by as many.
// Every lane of the wave must call it.
__device__ __forceinline__ void queue_items(const RoundArgs &ra, int it, uint32_t *pactive_next) {
  const unsigned long long m = __ballot(it >= 0);
  if (m == 0ull) return;
  const int n = __popcll(m);
  const int lane = threadIdx.x & 63;
  const int first = __ffsll((long long)m) - 1;
  uint32_t base = 0u;
  if (lane == first) {
    base = atomicAdd(&ra.count[(ra.round + 1) % 3], (uint32_t)n);
    if (pactive_next) atomicAdd(pactive_next, (uint32_t)n);
  }
  base = __shfl(base, first, 64);
  if (it >= 0) {
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    ra.list_out[base + rank] = it;
  }
}

// ---------------------------------------------------------------- async queue
//
// Device-scope atomics order the queue; values exchanged between workgroups
// (which may run on different XCDs, each with its own L2) are read and
// written with device-scope coherent loads and stores, and a workgroup
// waits for its stores to complete before it queues anyone.  (Fences at
// device scope would write back and invalidate a whole L2 per item.)

template <typename T>
__device__ __forceinline__ T ld_dev(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until this wave's vector memory operations (stores included) have
// completed: s_waitcnt vmcnt(0), other counters untouched.
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

enum : uint32_t { kQIdle = 0u, kQQueued = 1u, kQRunning = 2u, kQRerun = 3u };
enum : uint32_t { kAbortIdle = 1u, kAbortSlot = 2u, kAbortState = 3u, kAbortPush = 4u };

__device__ __forceinline__ void q_abort(const AsyncQ &q, uint32_t code) {
  atomicCAS(&q.ctr[3], 0u, code);
}

// Ring slot of ticket t: an odd multiplier permutes the ring, so that
// consecutive tickets (and the workgroups waiting on them) fall on
// different cache lines.
__device__ __forceinline__ uint32_t q_slot(const AsyncQ &q, uint32_t t) {
  return (t * 0x9E3779B1u) & q.mask;
}

// Appends an item whose state was just set to queued.  `pending` grows
// first, so it never reads 0 while the item is queued.
__device__ __forceinline__ void q_enqueue(const AsyncQ &q, int it) {
  atomicAdd(&q.ctr[2], 1u);
  const uint32_t t = atomicAdd(&q.ctr[1], 1u);
  int32_t *slot = &q.ring[q_slot(q, t)];
  // the slot's previous ticket (t - ring size) was taken long ago; wait in
  // case its holder has not emptied it yet
  for (unsigned spins = 0; ld_dev(slot) >= 0; ++spins) {
    if (spins > (1u << 20)) {
      q_abort(q, kAbortSlot);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  st_dev(slot, (int32_t)it);
}

// Requests a (re)run of `it`: queued if idle, marked to run again if running.
__device__ __forceinline__ void q_push(const AsyncQ &q, int it) {
  for (int tries = 0; tries < 4096; ++tries) {
    const uint32_t st = ld_dev(&q.state[it]);
    if (st == kQQueued || st == kQRerun) return;
    if (st == kQIdle) {
      if (atomicCAS(&q.state[it], kQIdle, kQQueued) == kQIdle) {
        q_enqueue(q, it);
        return;
      }
    } else if (st == kQRunning) {
      if (atomicCAS(&q.state[it], kQRunning, kQRerun) == kQRunning) return;
    } else {
      q_abort(q, kAbortState);
      return;
    }
  }
  q_abort(q, kAbortPush);
}

// Ends a run of `it` (thread 0, after the item's pushes): idle, or queued
// again when a neighbour asked for it meanwhile or `again` is set.
__device__ __forceinline__ void q_finish(const AsyncQ &q, int it, bool again) {
  for (int tries = 0; tries < 4096; ++tries) {
    const uint32_t st = ld_dev(&q.state[it]);
    if (st != kQRunning && st != kQRerun) {
      q_abort(q, kAbortState);
      break;
    }
    if (st == kQRerun || again) {
      if (atomicCAS(&q.state[it], st, kQQueued) == st) {
        q_enqueue(q, it);
        break;
      }
    } else if (atomicCAS(&q.state[it], kQRunning, kQIdle) == kQRunning) {
      break;
    }
    if (tries == 4095) q_abort(q, kAbortPush);
  }
  atomicSub(&q.ctr[2], 1u);
}

// One attempt to take an item (thread 0).  A workgroup draws a ticket once
// (fetch-and-add on the head) and then waits on that ticket's slot only.
// Returns the item, -1 when the slot is still empty (after a sleep), -2
// when the work is done (no item queued or running) or the launch aborted.
// `idle` counts consecutive empty attempts; past the limit the launch
// aborts instead of waiting for ever.
__device__ __forceinline__ int q_pop(const AsyncQ &q, int64_t &ticket, unsigned &idle) {
  // About 1.8 s at the longest back-off: far above the few milliseconds a
  // workgroup waits while others finish their items, short enough that a
  // lost wake-up ends the launch with an abort code instead of holding the
  // GPU.
  constexpr unsigned kIdleLimit = 1u << 19;
  if (ticket < 0) ticket = (int64_t)atomicAdd(&q.ctr[0], 1u);
  int32_t *slot = &q.ring[q_slot(q, (uint32_t)ticket)];
  const int32_t it = ld_dev(slot);
  if (it >= 0) {
    st_dev(slot, (int32_t)-1);
    ticket = -1;
    if (atomicCAS(&q.state[it], kQQueued, kQRunning) != kQQueued) {
      q_abort(q, kAbortState);
      return -2;
    }
    // no cache invalidation: the values the item reads from other
    // workgroups are loaded at device scope
    idle = 0;
    return it;
  }
  ++idle;
  // the shared counters are read on every 8th empty poll only
  if ((idle & 7u) == 0u) {
    if (ld_dev(&q.ctr[3]) != 0u || ld_dev(&q.ctr[2]) == 0u) return -2;
  }
  if (idle > kIdleLimit) {
    q_abort(q, kAbortIdle);
    return -2;
  }
  // back-off: short at first, then about 3.4 us between polls
  if (idle < 16) __builtin_amdgcn_s_sleep(4);
  else if (idle < 64) __builtin_amdgcn_s_sleep(32);
  else __builtin_amdgcn_s_sleep(127);
  return -1;
}

// Interpolate a global-memory grid at the foot point, ghost 1 outside the
// box (every box node active).  Same nesting and the same per-precision
// foot-point evaluation as the LDS variants: FP32 takes y = d + 2, FP64
// takes d.
template <typename T, int DIM>
__device__ __forceinline__ T interp_global(const T *__restrict__ v, const int n[3], int px, int py,
                                           int pz, const T *d) {
  int x0, y0, z0 = 0;
  T t0, t1, t2 = T(0);
  if constexpr (sizeof(T) == 4) {
    x0 = px + (int)d[0] - 2;
    y0 = py + (int)d[1] - 2;
    t0 = __builtin_amdgcn_fractf(d[0]);
    t1 = __builtin_amdgcn_fractf(d[1]);
    if constexpr (DIM == 3) {
      z0 = pz + (int)d[2] - 2;
      t2 = __builtin_amdgcn_fractf(d[2]);
    }
  } else {
    T f0 = Ar<T>::flr(d[0]), f1 = Ar<T>::flr(d[1]);
    t0 = d[0] - f0;
    t1 = d[1] - f1;
    x0 = px + (int)f0;
    y0 = py + (int)f1;
    if constexpr (DIM == 3) {
      T f2 = Ar<T>::flr(d[2]);
      t2 = d[2] - f2;
      z0 = pz + (int)f2;
    }
  }
  auto at = [&](int x, int y, int z) -> T {
    bool inb = (unsigned)x < (unsigned)n[0] && (unsigned)y < (unsigned)n[1];
    if constexpr (DIM == 3) inb = inb && (unsigned)z < (unsigned)n[2];
    if (!inb) return T(1);
    return v[(size_t)x + (size_t)n[0] * ((size_t)y + (size_t)n[1] * z)];
  };
  T r0 = Ar<T>::lin(t0, at(x0, y0, z0), at(x0 + 1, y0, z0));
  T r1 = Ar<T>::lin(t0, at(x0, y0 + 1, z0), at(x0 + 1, y0 + 1, z0));
  T y0v = Ar<T>::lin(t1, r0, r1);
  if constexpr (DIM == 2) {
    return y0v;
  } else {
    T q0 = Ar<T>::lin(t0, at(x0, y0, z0 + 1), at(x0 + 1, y0, z0 + 1));
    T q1 = Ar<T>::lin(t0, at(x0, y0 + 1, z0 + 1), at(x0 + 1, y0 + 1, z0 + 1));
    T y1v = Ar<T>::lin(t1, q0, q1);
    return Ar<T>::lin(t2, y0v, y1v);
  }
}

}  // namespace hjb
