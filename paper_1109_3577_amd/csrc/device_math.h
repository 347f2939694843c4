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

// Interpolate the LDS tile at base + d (d in cells, |d| < 2).  Corners
// enumerate x fastest; nesting x, then y, then z.
template <typename T, int DIM, int LX, int LY>
__device__ __forceinline__ T interp_lds(const T *s, int base, const T *d);

// FP32: cell index by floor-convert, local coordinate by fract, 24-bit
// index arithmetic.  (fract clamps its result below 1, so a displacement a
// hair below an integer lands on t = 1 - 2^-24 of the lower cell instead
// of t = 1: the same value up to the last bit; every FP32 kernel uses this
// one evaluation.)
template <int DIM, int LX, int LY>
__device__ __forceinline__ float interp_lds_f32(const float *s, int base, const float *d) {
  const int i0 = (int)__builtin_floorf(d[0]);
  const int i1 = (int)__builtin_floorf(d[1]);
  const float t0 = __builtin_amdgcn_fractf(d[0]);
  const float t1 = __builtin_amdgcn_fractf(d[1]);
  // byte offset of the lower corner: one 24-bit multiply-add, one shift-add
  int ob = __mul24(i1, LX * 4) + (base << 2);
  float t2 = 0.0f;
  if constexpr (DIM == 3) {
    const int i2 = (int)__builtin_floorf(d[2]);
    t2 = __builtin_amdgcn_fractf(d[2]);
    ob += __mul24(i2, LX * LY * 4);
  }
  ob += i0 << 2;
  const float *p = reinterpret_cast<const float *>(reinterpret_cast<const char *>(s) + ob);
  const float r0 = Ar<float>::lin(t0, p[0], p[1]);
  const float r1 = Ar<float>::lin(t0, p[LX], p[LX + 1]);
  const float y0 = Ar<float>::lin(t1, r0, r1);
  if constexpr (DIM == 2) {
    return y0;
  } else {
    const float *q = p + LX * LY;
    const float q0 = Ar<float>::lin(t0, q[0], q[1]);
    const float q1 = Ar<float>::lin(t0, q[LX], q[LX + 1]);
    const float y1 = Ar<float>::lin(t1, q0, q1);
    return Ar<float>::lin(t2, y0, y1);
  }
}

template <typename T, int DIM, int LX, int LY>
__device__ __forceinline__ T interp_lds(const T *s, int base, const T *d) {
  if constexpr (sizeof(T) == 4) return interp_lds_f32<DIM, LX, LY>(s, base, d);
  T f0 = Ar<T>::flr(d[0]), f1 = Ar<T>::flr(d[1]);
  T t0 = d[0] - f0, t1 = d[1] - f1;
  int o = base + (int)f0 + (int)f1 * LX;
  T f2 = T(0), t2 = T(0);
  if constexpr (DIM == 3) {
    f2 = Ar<T>::flr(d[2]);
    t2 = d[2] - f2;
    o += (int)f2 * (LX * LY);
  }
  T r0 = Ar<T>::lin(t0, s[o], s[o + 1]);
  T r1 = Ar<T>::lin(t0, s[o + LX], s[o + LX + 1]);
  T y0 = Ar<T>::lin(t1, r0, r1);
  if constexpr (DIM == 2) {
    return y0;
  } else {
    const int oz = o + LX * LY;
    T q0 = Ar<T>::lin(t0, s[oz], s[oz + 1]);
    T q1 = Ar<T>::lin(t0, s[oz + LX], s[oz + LX + 1]);
    T y1 = Ar<T>::lin(t1, q0, q1);
    return Ar<T>::lin(t2, y0, y1);
  }
}

template <typename T>
__device__ __forceinline__ void wave_max(T &x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    T y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
}

__device__ __forceinline__ void queue_item(const RoundArgs &ra, int item, uint32_t *pactive_next) {
  if (atomicCAS(&ra.flags_out[item], 0u, 1u) == 0u) {
    uint32_t idx = atomicAdd(&ra.count[(ra.round + 1) % 3], 1u);
    ra.list_out[idx] = item;
    atomicAdd(pactive_next, 1u);
  }
}

// Interpolate a global-memory grid at p + d, ghost 1 outside the box (every
// box node active).  Same nesting as the LDS variant.
template <typename T, int DIM>
__device__ __forceinline__ T interp_global(const T *__restrict__ v, const int n[3], int px, int py,
                                           int pz, const T *d) {
  T f0 = Ar<T>::flr(d[0]), f1 = Ar<T>::flr(d[1]);
  T t0 = d[0] - f0, t1 = d[1] - f1;
  const int x0 = px + (int)f0, y0 = py + (int)f1;
  T f2 = T(0), t2 = T(0);
  int z0 = 0;
  if constexpr (DIM == 3) {
    f2 = Ar<T>::flr(d[2]);
    t2 = d[2] - f2;
    z0 = pz + (int)f2;
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
