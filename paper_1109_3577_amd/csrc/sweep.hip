// Value-iteration kernels of the Kruzkov-form semi-Lagrangian scheme
// (Section 2.1 of the paper, eqs. SLscheme and iterativeSLscheme):
//
//   v_p <- min(v_p, beta * min_k I[v](p + s (c_p a_k + w_p)) + 1 - beta)
//
// on the non-target nodes of one patch (Step 3.2 of the Patchy Algorithm),
// of the whole grid (global solve) or of the coarse grid (Step 1).
//
// Every update is monotone in the values it reads (linear interpolation in
// weights form, min, multiply-add by beta > 0), and value iteration starts
// from above (v = 1 off the target).  Hence any fair order of updates --
// Jacobi, in-place, tiled, several tiles at once -- decreases towards the
// same greatest fixed point and stops on the same bits when nothing changes.
// The kernels exploit this freedom: a tile plus a 2-node halo is staged in
// LDS, swept in place until it stops changing, written back, and only the
// tiles next to changed nodes are queued for the next round.
//
// FP64 kernels keep every multiply and add separate (the library is built
// with contraction off) so that they reproduce the plain CPU evaluation bit
// for bit.  FP32 kernels use fused multiply-adds.

#include <algorithm>
#include <type_traits>

#include "device_math.h"
#include "hjb_internal.h"

namespace hjb {

// ---------------------------------------------------------------- tiled sweep

// LDS row stride of a tile: FP32 2D rows are padded to 8 words mod 32 so
// that the four rows of a half-wave brick fall on distinct banks.
template <typename T, int DIM, int LX>
constexpr int lds_stride() {
  return (DIM == 2 && sizeof(T) == 4) ? LX + ((8 - LX % 32) + 32) % 32 : LX;
}

// Control slices of a workgroup: a block with more threads than its tile
// has nodes splits each node's controls over NT / TN threads.
template <int DIM, int TX, int TY, int TZ, int NT>
constexpr int ctrl_slices() {
  return NT > TX * TY * (DIM == 3 ? TZ : 1) ? NT / (TX * TY * (DIM == 3 ? TZ : 1)) : 1;
}

// Bricks on side (sx, sy, sz) of a tile of NBX x NBY x NBZ bricks: for each
// axis, the first layer (s = -1), the last (s = +1) or all (s = 0).
template <int NBX, int NBY, int NBZ>
__device__ __forceinline__ uint32_t side_bricks(int sx, int sy, int sz) {
  uint32_t m = 0u;
#pragma unroll
  for (int b = 0; b < NBX * NBY * NBZ; ++b) {
    const int bx = b % NBX, by = (b / NBX) % NBY, bz = b / (NBX * NBY);
    const bool in = (sx < 0 ? bx == 0 : sx > 0 ? bx == NBX - 1 : true) &&
                    (sy < 0 ? by == 0 : sy > 0 ? by == NBY - 1 : true) &&
                    (sz < 0 ? bz == 0 : sz > 0 ? bz == NBZ - 1 : true);
    m |= in ? (1u << b) : 0u;
  }
  return m;
}

// Tables of add-on AO3 in LDS: the controls [nc][cone_cols] (FP32: s_d a_kd,
// FP64: a_kd; rows padded with zeros to an aligned vector), then the cone
// index rows [nc][cone_stride] bytes.
template <int DIM>
constexpr int cone_cols() {
  return DIM == 2 ? 2 : 4;
}

template <typename T, int DIM>
__host__ __device__ constexpr size_t cone_idx_offset(int nc) {
  return ((size_t)nc * cone_cols<DIM>() * sizeof(T) + 15) / 16 * 16;
}

// One activation of a work item.  ASYNC: values are exchanged with other
// workgroups of the same launch (device-scope loads and stores, a release
// fence before the pushes) and neighbours go to the work queue; otherwise
// to the next round's list.  MODE 1 (cones): each node minimises over the
// controls of its feedback's cone only (add-on AO3), read per lane from the
// LDS tables at s_cone.  MODE 2 (tabulated dynamics): displacement and beta
// per control and node come from the tables.  Returns whether the tile
// settled.
template <typename T, int DIM, int TX, int TY, int TZ, int NT, bool DRIFT, bool ASYNC,
          int MODE = 0>
__device__ __forceinline__ bool sweep_item(const DevProblem &P, const Item &item, int item_id,
                                           uint32_t fl, const RoundArgs &ra, const AsyncQ &aq,
                                           T *s_v, int *s_int, double *s_red,
                                           unsigned long long *s_wrk, uint32_t *s_msk,
                                           const unsigned char *s_cone = nullptr) {
  constexpr bool CONE = MODE == 1, TAB = MODE == 2;
  constexpr int LX = TX + 2 * HALO;
  constexpr int LY = TY + 2 * HALO;
  constexpr int LZ = (DIM == 3) ? TZ + 2 * HALO : 1;
  constexpr int LXS = lds_stride<T, DIM, LX>();
  constexpr int LN = LX * LY * LZ;
  constexpr int TN = TX * TY * (DIM == 3 ? TZ : 1);
  // CS > 1 control slices: the workgroup holds CS copies of the tile's
  // bricks, slice c evaluating the c-th share of the controls; slice 0
  // takes the minimum over the slices and owns the update.  The minimum is
  // exact, so the values are the same bits as with CS = 1.
  constexpr int CS = ctrl_slices<DIM, TX, TY, TZ, NT>();
  constexpr int NTS = NT / CS;    // threads per slice
  constexpr int NPT = TN / NTS;   // bricks per wave
  constexpr int NW = NTS / 64;    // waves per slice (brick stride)
  constexpr int NWT = NT / 64;    // waves of the workgroup
  static_assert(CS == 1 || MODE != 1, "control cones run with one control slice");
  __shared__ T s_part[CS > 1 ? (CS - 1) * TN : 1];  // partial minima of slices 1..CS-1
  constexpr int BX = Brick<DIM>::X, BY = Brick<DIM>::Y, BZ = Brick<DIM>::Z;
  constexpr int NBX = TX / BX, NBY = TY / BY, NBZ = (DIM == 3) ? TZ / BZ : 1;
  static_assert(TN % NTS == 0 && NTS % 64 == 0 && NT % CS == 0,
                "tile must be a multiple of the block");
  static_assert(TX % BX == 0 && TY % BY == 0 && (DIM == 2 || TZ % BZ == 0), "brick tiling");
  static_assert(NBX * NBY * NBZ <= 32, "brick mask is one word");

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  // control slice (wave-uniform, so that its control range stays scalar) and
  // wave within the slice
  const int slice = CS == 1 ? 0 : __builtin_amdgcn_readfirstlane(wave / NW);
  const int wv = CS == 1 ? wave : wave % NW;
  const bool owner = CS == 1 || slice == 0;
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const int tt = item.tile;
  const int tix = tt % P.ntile[0];
  const int tiy = (tt / P.ntile[0]) % P.ntile[1];
  const int tiz = tt / (P.ntile[0] * P.ntile[1]);
  const int ox = tix * TX, oy = tiy * TY, oz = (DIM == 3) ? tiz * TZ : 0;
  const int patch = item.patch;
  T *__restrict__ v = (T *)P.v;
  const int16_t *__restrict__ code = P.code;

  // Stage tile + halo: stored value where the node is active in this patch
  // (target nodes are 0, patch nodes carry v); other box nodes hold the
  // Dirichlet data U^(0) when given, else the ghost value 1, as do nodes
  // outside the box.  The code and the value are fetched together.
  for (int i = tid; i < LN; i += NT) {
    const int lx = i % LX;
    const int ly = (i / LX) % LY;
    const int lz = i / (LX * LY);
    const int gx = ox + lx - HALO, gy = oy + ly - HALO, gz = oz + lz - HALO;
    T val = T(1);
    bool inb = (unsigned)gx < (unsigned)n0 && (unsigned)gy < (unsigned)n1;
    if constexpr (DIM == 3) inb = inb && (unsigned)gz < (unsigned)n2;
    if (inb) {
      const size_t g = (size_t)gx + (size_t)n0 * ((size_t)gy + (size_t)n1 * (DIM == 3 ? gz : 0));
      const int cd = code[g];
      const T vg = ASYNC ? ld_dev(&v[g]) : v[g];
      val = cd == CODE_TARGET ? T(0)
            : cd == patch     ? vg
            : (P.u0 && cd != CODE_OBST) ? (T)P.u0[g]
                                          : T(1);
    }
    s_v[lx + LXS * (ly + LY * lz)] = val;
  }

  // This thread's nodes: lane `lane` of brick `wv + j NW`, j < NPT.
  T cc[NPT];
  T ww[NPT][DIM];
  T bb[NPT], oo[NPT];  // beta and 1 - beta of the node (variable step) or the scalars
  int krow[NPT];  // CONE: byte offset of the node's cone index row
  int off[NPT];
  size_t gid[NPT];
  bool act[NPT];
  uint32_t nbm[NPT];  // bricks whose change can reach brick j
  bool bact[NPT];     // brick j holds a node of this patch
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int b = wv + j * NW;
    const int bx = b % NBX, by = (b / NBX) % NBY, bz = b / (NBX * NBY);
    const int lx = bx * BX + lane % BX;
    const int ly = by * BY + (lane / BX) % BY;
    const int lz = bz * BZ + lane / (BX * BY);
    nbm[j] = brick_neighbours<NBX, NBY, NBZ>(b);
    const int gx = ox + lx, gy = oy + ly, gz = oz + lz;
    bool inb = gx < n0 && gy < n1;
    if constexpr (DIM == 3) inb = inb && gz < n2;
    off[j] = (lx + HALO) + LXS * ((ly + HALO) + LY * (DIM == 3 ? lz + HALO : 0));
    const size_t g = (size_t)gx + (size_t)n0 * ((size_t)gy + (size_t)n1 * (DIM == 3 ? gz : 0));
    gid[j] = g;
    act[j] = inb && code[g] == patch;
    bact[j] = __ballot(act[j]) != 0ull;
    if constexpr (CONE) {
      const int ks = act[j] ? (int)P.fb[g] : 0;
      krow[j] = (ks < P.nc ? ks : 0) * P.cone_stride;
    }
    if constexpr (sizeof(T) == 4) {
      bb[j] = (P.beta32 && act[j]) ? P.beta32[g] : P.betaf;
      oo[j] = (P.beta32 && act[j]) ? P.omb32[g] : P.ombf;
    } else {
      bb[j] = (P.beta64 && act[j]) ? P.beta64[g] : P.beta;
      oo[j] = (P.beta64 && act[j]) ? 1.0 - bb[j] : P.omb;
    }
    if constexpr (sizeof(T) == 4) {
      // offset foot point: y = c a + (w + 2)
      cc[j] = act[j] ? P.speed32[g] : 0.0f;
#pragma unroll
      for (int q = 0; q < DIM; ++q)
        ww[j][q] = ((DRIFT && act[j]) ? P.drift32[g * DIM + q] : 0.0f) + 2.0f;
    } else {
      cc[j] = act[j] ? P.speed64[g] : 0.0;
#pragma unroll
      for (int q = 0; q < DIM; ++q) ww[j][q] = (DRIFT && act[j]) ? P.drift64[g * DIM + q] : 0.0;
    }
  }
  // Bricks of the first sweep.  `fl` holds one bit per side of the tile
  // whose halo a neighbour changed since this item last ran (bit of the
  // centre: the item did not settle; no bit: first activation).  An item
  // that settled is at its own fixed point except next to those sides, so
  // only the bricks on them need the first sweep.
  constexpr int CENTER = (DIM == 3) ? 13 : 4;
  uint32_t first = ~0u;
  if (fl != 0u && !(fl & ((1u << CENTER) | kFlagFull))) {
    first = 0u;
    for (uint32_t f = fl; f; f &= f - 1u) {
      const int d = __builtin_ctz(f);
      const int sx = d % 3 - 1, sy = (d / 3) % 3 - 1, sz = d / 9 - 1;
      first |= side_bricks<NBX, NBY, NBZ>(sx, sy, DIM == 3 ? sz : 0);
    }
  }
  // brick-change masks, three in rotation: sweep s reads the mask of sweep
  // s - 1, ORs its own into slot s % 3 and clears the slot of sweep s + 1
  if (tid == 0) {
    s_msk[0] = 0u;
    s_msk[1] = 0u;
    s_msk[2] = 0u;
  }
  __syncthreads();

  T old[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) old[j] = s_v[off[j]];

  const T tolT = (T)ra.tol;
  const bool plain = P.plain != 0;
  const int ng = (P.nc + 3) >> 2;  // groups of 4 controls (table is padded)
  // this slice's share of the control groups (of the controls, tabulated)
  const int g_lo = slice * ng / CS, g_hi = (slice + 1) * ng / CS;
  const int k_lo = slice * P.nc / CS, k_hi = (slice + 1) * P.nc / CS;
  const int K = ra.inner_sweeps;
  unsigned long long upd = 0;
  bool converged = false;
  // the owner's update of node j from the minimum over the controls
  auto update = [&](int j, T mI, uint32_t &mine) {
    bool chg = false;
    if (act[j]) {
      // min_k (beta I_k + omb) == beta (min_k I_k) + omb: the map is
      // monotone, also after rounding.  The iteration only decreases
      // v, except from a start below the fixed point (add-on AO1: plain
      // v <- F(v)).
      const T cand = TAB ? mI : Ar<T>::kruzkov(bb[j], mI, oo[j]);
      const T cur = s_v[off[j]];
      if (plain ? cand != cur : cand < cur) {
        s_v[off[j]] = cand;
        chg = cur - cand > tolT || cand - cur > tolT;
      }
    }
    if (__ballot(chg) != 0ull) mine |= 1u << (wv + j * NW);
  };
  for (int it = 0; it < K; ++it) {
    const uint32_t prev = s_msk[(it + 2) % 3];
    if (tid == 0) s_msk[(it + 1) % 3] = 0u;
    uint32_t mine = 0u;
    bool run[NPT];
    T mIs[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      // Skip the brick when nothing within its reach changed in the last
      // sweep: its update would read the same values and change nothing.
      // A brick with no node of this patch (tiles that straddle patches) has
      // nothing to update either.  Every slice takes the same decision.
      const uint32_t bj = 1u << (wv + j * NW);
      run[j] = bact[j] && (it == 0 ? (first & bj) != 0u : (prev & nbm[j]) != 0u);
      if (!run[j]) continue;
      if (owner) upd += act[j] ? 1u : 0u;
      T mI = T(3);
      if constexpr (CONE) {
        // the node's cone: its index row holds four control indices per
        // LDS word; full words first, then the uniform remainder
        constexpr int CC = cone_cols<DIM>();
        const T *ctl = reinterpret_cast<const T *>(s_cone);
        const unsigned char *row = s_cone + cone_idx_offset<T, DIM>(P.nc) + krow[j];
        const int b2 = off[j] - 2 - 2 * LXS - (DIM == 3 ? 2 * LXS * LY : 0);
        auto group = [&](auto g_tag, uint32_t w4) {
          constexpr int G = decltype(g_tag)::value;
          T a[G][CC];
#pragma unroll
          for (int u = 0; u < G; ++u) {
            const int k = (int)((w4 >> (8 * u)) & 255u);
            if constexpr (sizeof(T) == 4 && DIM == 2) {
              const float2 t2 = *reinterpret_cast<const float2 *>(ctl + k * CC);
              a[u][0] = t2.x;
              a[u][1] = t2.y;
            } else if constexpr (sizeof(T) == 4) {
              const float4 t4 = *reinterpret_cast<const float4 *>(ctl + k * CC);
              a[u][0] = t4.x;
              a[u][1] = t4.y;
              a[u][2] = t4.z;
              a[u][3] = t4.w;
            } else {
#pragma unroll
              for (int q = 0; q < CC; ++q) a[u][q] = ctl[k * CC + q];
            }
          }
#pragma unroll
          for (int u = 0; u < G; ++u) {
            if constexpr (sizeof(T) == 4) {
              float y[DIM];
#pragma unroll
              for (int q = 0; q < DIM; ++q) y[q] = __builtin_fmaf(cc[j], a[u][q], ww[j][q]);
              mI = __builtin_fminf(mI, interp_lds_f32<DIM, LXS, LY>(s_v, b2, y));
            } else {
              T d[DIM];
#pragma unroll
              for (int q = 0; q < DIM; ++q) {
                T gq = cc[j] * a[u][q];
                if (DRIFT) gq = gq + ww[j][q];
                d[q] = P.step[q] * gq;
              }
              const T I = interp_lds_f64<DIM, LXS, LY>(s_v, off[j], d);
              mI = I < mI ? I : mI;
            }
          }
        };
        const int cl = P.cone_len;
        int i = 0;
        for (; i + 4 <= cl; i += 4)
          group(std::integral_constant<int, 4>{}, *reinterpret_cast<const uint32_t *>(row + i));
        const int rem = cl - i;
        if (rem > 0) {
          const uint32_t w4 = *reinterpret_cast<const uint32_t *>(row + i);
          if (rem == 1)
            group(std::integral_constant<int, 1>{}, w4);
          else if (rem == 2)
            group(std::integral_constant<int, 2>{}, w4);
          else
            group(std::integral_constant<int, 3>{}, w4);
        }
      } else if constexpr (TAB) {
        // mI collects the candidates beta I + 1 - beta themselves
        const size_t Nn = (size_t)n0 * n1 * n2;
        const int b2 = off[j] - 2 - 2 * LXS - (DIM == 3 ? 2 * LXS * LY : 0);
        for (int k = k_lo; k < k_hi; ++k) {
          const size_t e = act[j] ? (size_t)k * Nn + gid[j] : 0;
          T b = bb[j], o = oo[j], I;
          if constexpr (sizeof(T) == 4) {
            float y[DIM];
#pragma unroll
            for (int q = 0; q < DIM; ++q) y[q] = P.foot32[e * DIM + q] + 2.0f;
            I = interp_lds_f32<DIM, LXS, LY>(s_v, b2, y);
            if (P.bpk32) {
              b = P.bpk32[e];
              o = P.opk32[e];
            }
          } else {
            T d[DIM];
#pragma unroll
            for (int q = 0; q < DIM; ++q) d[q] = P.foot64[e * DIM + q];
            I = interp_lds_f64<DIM, LXS, LY>(s_v, off[j], d);
            if (P.bpk64) {
              b = P.bpk64[e];
              o = 1.0 - b;
            }
          }
          const T ck = Ar<T>::kruzkov(b, I, o);
          mI = ck < mI ? ck : mI;
        }
      } else if constexpr (sizeof(T) == 4) {
        const int b2 = off[j] - 2 - 2 * LXS - (DIM == 3 ? 2 * LXS * LY : 0);
        for (int g4 = g_lo; g4 < g_hi; ++g4) {
          float a[4 * DIM];
#pragma unroll
          for (int q = 0; q < 4 * DIM; ++q) a[q] = ((cf32p)P.ctrl32)[g4 * 4 * DIM + q];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            float y[DIM];
#pragma unroll
            for (int q = 0; q < DIM; ++q) y[q] = __builtin_fmaf(cc[j], a[u * DIM + q], ww[j][q]);
            mI = __builtin_fminf(mI, interp_lds_f32<DIM, LXS, LY>(s_v, b2, y));
          }
        }
      } else {
        for (int k = 4 * g_lo; k < 4 * g_hi; ++k) {
          T d[DIM];
#pragma unroll
          for (int q = 0; q < DIM; ++q) {
            T g = cc[j] * ((cf64p)P.ctrl64)[k * DIM + q];
            if (DRIFT) g = g + ww[j][q];
            d[q] = P.step[q] * g;
          }
          const T I = interp_lds_f64<DIM, LXS, LY>(s_v, off[j], d);
          mI = I < mI ? I : mI;
        }
      }
      if constexpr (CS == 1) {
        update(j, mI, mine);
      } else if (owner) {
        mIs[j] = mI;
      } else {
        s_part[(slice - 1) * TN + (wv + j * NW) * 64 + lane] = mI;
      }
    }
    if constexpr (CS > 1) {
      // the partial minima of the other slices are in LDS after the barrier
      __syncthreads();
      if (owner) {
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
          if (!run[j]) continue;
          T mI = mIs[j];
#pragma unroll
          for (int c = 1; c < CS; ++c) {
            const T pc = s_part[(c - 1) * TN + (wv + j * NW) * 64 + lane];
            mI = pc < mI ? pc : mI;
          }
          update(j, mI, mine);
        }
      }
    }
    if (lane == 0 && mine) atomicOr(&s_msk[it % 3], mine);
    __syncthreads();
    if (s_msk[it % 3] == 0u) {
      converged = true;
      break;
    }
  }

  // Write back, FP64 residual, bounding box of the changed nodes.  The box
  // is found per brick from a wave ballot of the changed lanes, then merged
  // by one LDS atomic per wave and bound.
  double dmax = 0.0;
  int bx0 = 1 << 30, by0 = 1 << 30, bz0 = 1 << 30, bx1 = -1, by1 = -1, bz1 = -1;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    bool big = false;
    if (owner && act[j]) {
      const T nv = s_v[off[j]];
      if (nv != old[j]) {
        if (ASYNC) st_dev(&v[gid[j]], nv);
        else v[gid[j]] = nv;
        const double dd = fabs((double)old[j] - (double)nv);
        dmax = dd > dmax ? dd : dmax;
        big = old[j] - nv > tolT || nv - old[j] > tolT;
      }
    }
    brick_box<DIM, NBX, NBY>(__ballot(big), wv + j * NW, bx0, bx1, by0, by1, bz0, bz1);
  }
  // The value stores are device-scope (written through to the coherent
  // level); each wave waits for its stores to complete, so after the
  // barrier below every new value is visible device-wide before any
  // neighbour is queued.
  if (ASYNC) wait_stores();
  if (tid == 0) {
    s_int[0] = 1 << 30; s_int[1] = 1 << 30; s_int[2] = 1 << 30;
    s_int[3] = -1; s_int[4] = -1; s_int[5] = -1;
  }
  wave_max(dmax);
  // node updates executed: active nodes of the bricks swept, per sweep
  unsigned long long cw = upd;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) cw += __shfl_xor(cw, o, 64);
  __syncthreads();
  if (lane == 0) {
    s_red[wave] = dmax;
    s_wrk[wave] = cw;
    if (bx1 >= 0) {
      atomicMin(&s_int[0], bx0); atomicMin(&s_int[1], by0); atomicMin(&s_int[2], bz0);
      atomicMax(&s_int[3], bx1); atomicMax(&s_int[4], by1); atomicMax(&s_int[5], bz1);
    }
  }
  __syncthreads();
  const int cx0 = s_int[0], cy0 = s_int[1], cz0 = s_int[2];
  const int cx1 = s_int[3], cy1 = s_int[4], cz1 = s_int[5];
  const int slot = blockIdx.x % kSlots;
  if (tid == 0) {
    double m = 0.0;
    unsigned long long wsum = 0;
    for (int w = 0; w < NWT; ++w) {
      m = s_red[w] > m ? s_red[w] : m;
      wsum += s_wrk[w];
    }
    if (m > 0.0)
      atomicMax(&P.residual[(ra.round % 3) * kSlots + slot],
                (unsigned long long)__double_as_longlong(m));
    if (wsum) atomicAdd(&P.work[slot], wsum);
    atomicAdd(&P.work[kSlots + slot], 1ull);
  }

  // Queue the neighbour items (same patch) whose halo holds a changed node,
  // and this item again if its in-LDS sweeps did not settle.  The lanes of
  // wave 0 claim their items' flags, then reserve list slots with one atomic.
  if (cx1 >= 0 && wave == 0) {
    constexpr int NNB = (DIM == 3) ? 27 : 9;
    int it2 = -1;
    if (lane < NNB) {
      const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = (DIM == 3) ? lane / 9 - 1 : 0;
      bool need;
      if (dx == 0 && dy == 0 && dz == 0) {
        need = !converged;
      } else {
        need = (dx < 0 ? cx0 < HALO : dx > 0 ? cx1 >= TX - HALO : true) &&
               (dy < 0 ? cy0 < HALO : dy > 0 ? cy1 >= TY - HALO : true) &&
               (dz < 0 ? cz0 < HALO : dz > 0 ? cz1 >= TZ - HALO : true);
      }
      const int nx = tix + dx, ny = tiy + dy, nz = tiz + dz;
      if (need && nx >= 0 && ny >= 0 && nz >= 0 && nx < P.ntile[0] && ny < P.ntile[1] &&
          nz < P.ntile[2]) {
        const int t2 = nx + P.ntile[0] * (ny + P.ntile[1] * nz);
        const int ntiles = P.ntile[0] * P.ntile[1] * P.ntile[2];
        const int l = P.item_map[(size_t)patch * ntiles + t2];
        // the receiver sees the change on its side (-dx, -dy, -dz); the
        // first setter of any side queues the item
        const uint32_t side = 1u << ((1 - dx) + 3 * (1 - dy) + 9 * (1 - dz));
        if (ASYNC) {
          // the item itself is queued again by its finish
          if (l >= 0 && !(dx == 0 && dy == 0 && dz == 0)) {
            atomicOr(&aq.sides[P.item_base + l], side);
            q_push(aq, P.item_base + l);
          }
        } else if (l >= 0 && atomicOr(&ra.flags_out[P.item_base + l], side) == 0u) {
          it2 = P.item_base + l;
          if (P.item_key)
            atomicMin(&P.win[3 + (ra.round + 1) % 3],
                      __float_as_uint(P.item_key[(size_t)patch * ntiles + t2]));
        }
      }
    }
    if (!ASYNC) queue_items(ra, it2, &P.pactive[(ra.round + 1) % 3]);
  }
  (void)item_id;
  return converged;
}

// Value-ordered schedule: the threshold of round r is the larger of its
// base and the smallest key queued for it; block 0 sets the base of round
// r + 1 to that threshold plus win_dt and clears the minimum of round r + 2
// (neither slot is read in round r).
__device__ __forceinline__ float window_threshold(const DevProblem &P, uint32_t r) {
  return fmaxf(__uint_as_float(P.win[r % 3]), __uint_as_float(P.win[3 + r % 3]));
}

__device__ __forceinline__ void window_advance(const DevProblem &P, uint32_t r) {
  P.win[(r + 1) % 3] = __float_as_uint(window_threshold(P, r) + P.win_dt);
  P.win[3 + (r + 2) % 3] = 0x7f800000u;
}

// Carries item `it` (not run in round r) to the next round's list with its
// pending sides, and records its key.  One thread.
__device__ __forceinline__ void window_defer(const DevProblem &P, const RoundArgs &ra, int it,
                                             uint32_t fl, float key) {
  if (atomicOr(&ra.flags_out[it], fl ? fl : kFlagFull) == 0u) {
    const uint32_t slot = atomicAdd(&ra.count[(ra.round + 1) % 3], 1u);
    ra.list_out[slot] = it;
    atomicAdd(&P.pactive[(ra.round + 1) % 3], 1u);
  }
  atomicMin(&P.win[3 + (ra.round + 1) % 3], __float_as_uint(key));
}

template <typename T, int DIM, int TX, int TY, int TZ, int NT>
__global__ void __launch_bounds__(NT)
k_sweep(const DevProblem *__restrict__ probs, const Item *__restrict__ items, RoundArgs ra) {
  constexpr int LX = TX + 2 * HALO;
  constexpr int LY = TY + 2 * HALO;
  constexpr int LZ = (DIM == 3) ? TZ + 2 * HALO : 1;
  constexpr int LXS = lds_stride<T, DIM, LX>();
  __shared__ T s_v[LXS * LY * LZ];
  __shared__ int s_int[8];
  __shared__ uint32_t s_msk[4];
  __shared__ double s_red[NT / 64];
  __shared__ unsigned long long s_wrk[NT / 64];
  const uint32_t r = ra.round;
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) ra.count[(r + 2) % 3] = 0u;
    for (int p = threadIdx.x; p < ra.nprob * kSlots; p += NT) {
      const int q = p / kSlots, k = p % kSlots;
      if (k == 0) {
        probs[q].pactive[(r + 2) % 3] = 0u;
        if (probs[q].item_key) window_advance(probs[q], r);
      }
      probs[q].residual[((r + 2) % 3) * kSlots + k] = 0ull;
    }
  }
  const uint32_t nin = ra.count[r % 3];
  for (uint32_t li = blockIdx.x; li < nin; li += gridDim.x) {
    const int it = ra.list_in[li];
    const Item item = items[it];
    const DevProblem &P = probs[item.prob];
    const uint32_t fl = ra.flags_in[it];
    __syncthreads();  // every thread has read the flag before it is cleared
    if (threadIdx.x == 0) ra.flags_in[it] = 0u;
    if (P.item_key) {
      const int ntiles = P.ntile[0] * P.ntile[1] * P.ntile[2];
      const float key = P.item_key[(size_t)item.patch * ntiles + item.tile];
      if (key > window_threshold(P, r)) {
        if (threadIdx.x == 0) window_defer(P, ra, it, fl, key);
        continue;
      }
    }
    if (P.has_drift)
      sweep_item<T, DIM, TX, TY, TZ, NT, true, false>(P, item, it, fl, ra, AsyncQ{}, s_v, s_int,
                                                      s_red, s_wrk, s_msk);
    else
      sweep_item<T, DIM, TX, TY, TZ, NT, false, false>(P, item, it, fl, ra, AsyncQ{}, s_v, s_int,
                                                       s_red, s_wrk, s_msk);
    __syncthreads();
  }}

// Rounds schedule of problems with tabulated dynamics (as k_sweep).
template <typename T, int DIM, int TX, int TY, int TZ, int NT>
__global__ void __launch_bounds__(NT)
k_sweep_tab(const DevProblem *__restrict__ probs, const Item *__restrict__ items, RoundArgs ra) {
  constexpr int LX = TX + 2 * HALO;
  constexpr int LY = TY + 2 * HALO;
  constexpr int LZ = (DIM == 3) ? TZ + 2 * HALO : 1;
  constexpr int LXS = lds_stride<T, DIM, LX>();
  __shared__ T s_v[LXS * LY * LZ];
  __shared__ int s_int[8];
  __shared__ uint32_t s_msk[4];
  __shared__ double s_red[NT / 64];
  __shared__ unsigned long long s_wrk[NT / 64];
  const uint32_t r = ra.round;
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) ra.count[(r + 2) % 3] = 0u;
    for (int p = threadIdx.x; p < ra.nprob * kSlots; p += NT) {
      const int q = p / kSlots, k = p % kSlots;
      if (k == 0) {
        probs[q].pactive[(r + 2) % 3] = 0u;
        if (probs[q].item_key) window_advance(probs[q], r);
      }
      probs[q].residual[((r + 2) % 3) * kSlots + k] = 0ull;
    }
  }
  const uint32_t nin = ra.count[r % 3];
  for (uint32_t li = blockIdx.x; li < nin; li += gridDim.x) {
    const int it = ra.list_in[li];
    const Item item = items[it];
    const DevProblem &P = probs[item.prob];
    const uint32_t fl = ra.flags_in[it];
    __syncthreads();  // every thread has read the flag before it is cleared
    if (threadIdx.x == 0) ra.flags_in[it] = 0u;
    if (P.item_key) {
      const int ntiles = P.ntile[0] * P.ntile[1] * P.ntile[2];
      const float key = P.item_key[(size_t)item.patch * ntiles + item.tile];
      if (key > window_threshold(P, r)) {
        if (threadIdx.x == 0) window_defer(P, ra, it, fl, key);
        continue;
      }
    }
    // tabulated dynamics: speed and drift are not used
    sweep_item<T, DIM, TX, TY, TZ, NT, false, false, 2>(P, item, it, fl, ra, AsyncQ{}, s_v, s_int,
                                                        s_red, s_wrk, s_msk);
    __syncthreads();
  }}

// Rounds schedule with the control cones of add-on AO3 (one problem).  The
// controls and the cone index rows are staged in dynamic LDS once per
// workgroup.
template <typename T, int DIM, int TX, int TY, int TZ, int NT>
__global__ void __launch_bounds__(NT)
k_sweep_cone(const DevProblem *__restrict__ probs, const Item *__restrict__ items, RoundArgs ra) {
  constexpr int LX = TX + 2 * HALO;
  constexpr int LY = TY + 2 * HALO;
  constexpr int LZ = (DIM == 3) ? TZ + 2 * HALO : 1;
  constexpr int LXS = lds_stride<T, DIM, LX>();
  constexpr int CC = cone_cols<DIM>();
  __shared__ T s_v[LXS * LY * LZ];
  __shared__ int s_int[8];
  __shared__ uint32_t s_msk[4];
  __shared__ double s_red[NT / 64];
  __shared__ unsigned long long s_wrk[NT / 64];
  extern __shared__ __attribute__((aligned(16))) unsigned char s_cone[];
  const uint32_t r = ra.round;
  const DevProblem &P = probs[0];
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) ra.count[(r + 2) % 3] = 0u;
    for (int k = threadIdx.x; k < kSlots; k += NT) {
      if (k == 0) {
        P.pactive[(r + 2) % 3] = 0u;
        if (P.item_key) window_advance(P, r);
      }
      P.residual[((r + 2) % 3) * kSlots + k] = 0ull;
    }
  }
  const uint32_t nin = ra.count[r % 3];
  if (blockIdx.x >= nin) return;
  {
    T *ctl = reinterpret_cast<T *>(s_cone);
    for (int i = threadIdx.x; i < P.nc * CC; i += NT) {
      const int k = i / CC, q = i % CC;
      T a = T(0);
      if (q < DIM) a = sizeof(T) == 4 ? (T)P.ctrl32[k * DIM + q] : (T)P.ctrl64[k * DIM + q];
      ctl[i] = a;
    }
    uint32_t *idx = reinterpret_cast<uint32_t *>(s_cone + cone_idx_offset<T, DIM>(P.nc));
    const uint32_t *gidx = reinterpret_cast<const uint32_t *>(P.cone_idx);
    for (int i = threadIdx.x; i < P.nc * (P.cone_stride / 4); i += NT) idx[i] = gidx[i];
  }
  for (uint32_t li = blockIdx.x; li < nin; li += gridDim.x) {
    const int it = ra.list_in[li];
    const Item item = items[it];
    const uint32_t fl = ra.flags_in[it];
    __syncthreads();  // flag read by every thread (and, first, the tables staged)
    if (threadIdx.x == 0) ra.flags_in[it] = 0u;
    if (P.item_key) {
      const int ntiles = P.ntile[0] * P.ntile[1] * P.ntile[2];
      const float key = P.item_key[(size_t)item.patch * ntiles + item.tile];
      if (key > window_threshold(P, r)) {
        if (threadIdx.x == 0) window_defer(P, ra, it, fl, key);
        continue;
      }
    }
    if (P.has_drift)
      sweep_item<T, DIM, TX, TY, TZ, NT, true, false, 1>(P, item, it, fl, ra, AsyncQ{}, s_v,
                                                         s_int, s_red, s_wrk, s_msk, s_cone);
    else
      sweep_item<T, DIM, TX, TY, TZ, NT, false, false, 1>(P, item, it, fl, ra, AsyncQ{}, s_v,
                                                          s_int, s_red, s_wrk, s_msk, s_cone);
    __syncthreads();
  }
}

// Asynchronous schedule: one persistent launch; every workgroup takes items
// from the work queue until no item is queued or running.
template <typename T, int DIM, int TX, int TY, int TZ, int NT>
__global__ void __launch_bounds__(NT)
k_sweep_async(const DevProblem *__restrict__ probs, const Item *__restrict__ items, RoundArgs ra,
              AsyncQ q) {
  constexpr int LX = TX + 2 * HALO;
  constexpr int LY = TY + 2 * HALO;
  constexpr int LZ = (DIM == 3) ? TZ + 2 * HALO : 1;
  constexpr int LXS = lds_stride<T, DIM, LX>();
  constexpr int CENTER = (DIM == 3) ? 13 : 4;
  __shared__ T s_v[LXS * LY * LZ];
  __shared__ int s_int[8];
  __shared__ uint32_t s_msk[4];
  __shared__ double s_red[NT / 64];
  __shared__ unsigned long long s_wrk[NT / 64];
  __shared__ int s_it;
  __shared__ uint32_t s_fl;
  unsigned idle = 0;
  int64_t ticket = -1;
  while (true) {
    if (threadIdx.x == 0) {
      const int it = q_pop(q, ticket, idle);
      s_it = it;
      s_fl = it >= 0 ? atomicExch(&q.sides[it], 0u) : 0u;
    }
    __syncthreads();
    const int it = s_it;
    const uint32_t fl = s_fl;
    __syncthreads();
    if (it == -2) break;
    if (it < 0) continue;
    const Item item = items[it];
    const DevProblem &P = probs[item.prob];
    bool conv;
    if (P.has_drift)
      conv = sweep_item<T, DIM, TX, TY, TZ, NT, true, true>(P, item, it, fl, ra, q, s_v, s_int,
                                                             s_red, s_wrk, s_msk);
    else
      conv = sweep_item<T, DIM, TX, TY, TZ, NT, false, true>(P, item, it, fl, ra, q, s_v, s_int,
                                                              s_red, s_wrk, s_msk);
    __syncthreads();
    if (threadIdx.x == 0) {
      if (!conv) atomicOr(&q.sides[it], 1u << CENTER);
      q_finish(q, it, !conv);
    }
  }
}

#define HJB_SHAPES(X)      \
  X(2, 16, 16, 1, 256)     \
  X(2, 32, 8, 1, 256)      \
  X(2, 64, 16, 1, 256)     \
  X(2, 32, 32, 1, 256)     \
  X(2, 64, 8, 1, 256)      \
  X(2, 32, 16, 1, 256)     \
  X(2, 64, 8, 1, 512)      \
  X(2, 32, 16, 1, 512)     \
  X(2, 64, 16, 1, 512)     \
  X(2, 32, 32, 1, 512)     \
  X(2, 32, 8, 1, 512)      \
  X(2, 32, 8, 1, 1024)     \
  X(2, 16, 16, 1, 512)     \
  X(2, 16, 16, 1, 1024)    \
  X(2, 32, 16, 1, 1024)    \
  X(3, 16, 8, 8, 256)      \
  X(3, 8, 8, 8, 256)       \
  X(3, 32, 8, 4, 256)      \
  X(3, 8, 8, 8, 512)       \
  X(3, 16, 8, 8, 512)

bool sweep_shape_supported(int dim, int tx, int ty, int tz, int nt) {
#define HJB_CHECK_SHAPE(D, A, B, C, NT) \
  if (dim == D && tx == A && ty == B && tz == C && nt == NT) return true;
  HJB_SHAPES(HJB_CHECK_SHAPE)
#undef HJB_CHECK_SHAPE
  return false;
}

hipError_t launch_sweep_async(bool fp64, SweepShape sh, int grid, const DevProblem *probs,
                              const Item *items, const RoundArgs &ra, const AsyncQ &q,
                              hipStream_t s) {
#define HJB_LAUNCH_ASYNC(D, A, B, C, NT)                                                    \
  if (sh.dim == D && sh.tx == A && sh.ty == B && sh.tz == C && sh.nt == NT) {               \
    if (fp64)                                                                               \
      hipLaunchKernelGGL((k_sweep_async<double, D, A, B, C, NT>), dim3(grid), dim3(NT), 0, \
                         s, probs, items, ra, q);                                           \
    else                                                                                    \
      hipLaunchKernelGGL((k_sweep_async<float, D, A, B, C, NT>), dim3(grid), dim3(NT), 0,  \
                         s, probs, items, ra, q);                                           \
    return hipGetLastError();                                                               \
  }
  HJB_SHAPES(HJB_LAUNCH_ASYNC)
#undef HJB_LAUNCH_ASYNC
  return hipErrorInvalidValue;
}

hipError_t launch_sweep(bool fp64, SweepShape sh, int grid, const DevProblem *probs,
                        const Item *items, const RoundArgs &ra, hipStream_t s) {
#define HJB_LAUNCH_SHAPE(D, A, B, C, NT)                                                    \
  if (sh.dim == D && sh.tx == A && sh.ty == B && sh.tz == C && sh.nt == NT) {               \
    if (fp64)                                                                               \
      hipLaunchKernelGGL((k_sweep<double, D, A, B, C, NT>), dim3(grid), dim3(NT), 0, s,    \
                         probs, items, ra);                                                 \
    else                                                                                    \
      hipLaunchKernelGGL((k_sweep<float, D, A, B, C, NT>), dim3(grid), dim3(NT), 0, s,     \
                         probs, items, ra);                                                 \
    return hipGetLastError();                                                               \
  }
  HJB_SHAPES(HJB_LAUNCH_SHAPE)
#undef HJB_LAUNCH_SHAPE
  return hipErrorInvalidValue;
}

#define HJB_CONE_SHAPES(X) \
  X(2, 32, 8, 1, 256)        \
  X(2, 32, 16, 1, 256)       \
  X(3, 8, 8, 8, 256)

bool sweep_cone_shape_supported(int dim, int tx, int ty, int tz, int nt) {
#define HJB_CHECK_SHAPE(D, A, B, C, NT) \
  if (dim == D && tx == A && ty == B && tz == C && nt == NT) return true;
  HJB_CONE_SHAPES(HJB_CHECK_SHAPE)
#undef HJB_CHECK_SHAPE
  return false;
}

size_t sweep_cone_lds_bytes(bool fp64, int dim, int nc, int cone_stride) {
  const size_t off = fp64 ? (dim == 2 ? cone_idx_offset<double, 2>(nc)
                                      : cone_idx_offset<double, 3>(nc))
                          : (dim == 2 ? cone_idx_offset<float, 2>(nc)
                                      : cone_idx_offset<float, 3>(nc));
  return off + (size_t)nc * (size_t)cone_stride;
}

hipError_t launch_sweep_cone(bool fp64, SweepShape sh, int grid, const DevProblem *probs,
                             const Item *items, const RoundArgs &ra, int nc, int cone_stride,
                             hipStream_t s) {
  const size_t lds = sweep_cone_lds_bytes(fp64, sh.dim, nc, cone_stride);
#define HJB_LAUNCH_CONE(D, A, B, C, NT)                                                     \
  if (sh.dim == D && sh.tx == A && sh.ty == B && sh.tz == C && sh.nt == NT) {               \
    if (fp64)                                                                               \
      hipLaunchKernelGGL((k_sweep_cone<double, D, A, B, C, NT>), dim3(grid), dim3(NT), lds, \
                         s, probs, items, ra);                                              \
    else                                                                                    \
      hipLaunchKernelGGL((k_sweep_cone<float, D, A, B, C, NT>), dim3(grid), dim3(NT), lds,  \
                         s, probs, items, ra);                                              \
    return hipGetLastError();                                                               \
  }
  HJB_CONE_SHAPES(HJB_LAUNCH_CONE)
#undef HJB_LAUNCH_CONE
  return hipErrorInvalidValue;
}

#define HJB_TAB_SHAPES(X) \
  X(2, 16, 16, 1, 256)      \
  X(2, 16, 16, 1, 512)      \
  X(2, 32, 8, 1, 256)       \
  X(3, 8, 8, 8, 256)

bool sweep_tab_shape_supported(int dim, int tx, int ty, int tz, int nt) {
#define HJB_CHECK_SHAPE(D, A, B, C, NT) \
  if (dim == D && tx == A && ty == B && tz == C && nt == NT) return true;
  HJB_TAB_SHAPES(HJB_CHECK_SHAPE)
#undef HJB_CHECK_SHAPE
  return false;
}

hipError_t launch_sweep_tab(bool fp64, SweepShape sh, int grid, const DevProblem *probs,
                            const Item *items, const RoundArgs &ra, hipStream_t s) {
#define HJB_LAUNCH_TAB(D, A, B, C, NT)                                                     \
  if (sh.dim == D && sh.tx == A && sh.ty == B && sh.tz == C && sh.nt == NT) {              \
    if (fp64)                                                                              \
      hipLaunchKernelGGL((k_sweep_tab<double, D, A, B, C, NT>), dim3(grid), dim3(NT), 0, s, \
                         probs, items, ra);                                                \
    else                                                                                   \
      hipLaunchKernelGGL((k_sweep_tab<float, D, A, B, C, NT>), dim3(grid), dim3(NT), 0, s,  \
                         probs, items, ra);                                                \
    return hipGetLastError();                                                              \
  }
  HJB_TAB_SHAPES(HJB_LAUNCH_TAB)
#undef HJB_LAUNCH_TAB
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- plain Jacobi

// One full-grid Jacobi sweep: vout = min(vin, F(vin)); the plain global solve.
template <typename T, int DIM>
__global__ void __launch_bounds__(256)
k_jacobi(const DevProblem *__restrict__ Pp, const T *__restrict__ vin, T *__restrict__ vout,
         unsigned long long *res_slot) {
  const DevProblem &P = *Pp;
  const size_t N = (size_t)P.n[0] * P.n[1] * P.n[2];
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dd = 0.0;
  if (g < N) {
    const int cd = P.code[g];
    const T old = vin[g];
    T nv = old;
    if (cd == CODE_TARGET) {
      nv = T(0);
    } else if (cd >= 0) {
      const int px = (int)(g % P.n[0]);
      const int py = (int)((g / P.n[0]) % P.n[1]);
      const int pz = (int)(g / ((size_t)P.n[0] * P.n[1]));
      T c, w[DIM];
      if constexpr (sizeof(T) == 4) {
        // offset foot point, as in the tiled sweep: y = c a + (w + 2)
        c = P.speed32[g];
        for (int a = 0; a < DIM; ++a) w[a] = (P.has_drift ? P.drift32[g * DIM + a] : 0.0f) + 2.0f;
      } else {
        c = P.speed64[g];
        for (int a = 0; a < DIM; ++a) w[a] = P.has_drift ? P.drift64[g * DIM + a] : 0.0;
      }
      T beta, omb;
      if constexpr (sizeof(T) == 4) {
        beta = P.beta32 ? P.beta32[g] : P.betaf;
        omb = P.beta32 ? P.omb32[g] : P.ombf;
      } else {
        beta = P.beta64 ? P.beta64[g] : P.beta;
        omb = P.beta64 ? 1.0 - beta : P.omb;
      }
      T cand;
      if (sizeof(T) == 4 ? P.foot32 != nullptr : P.foot64 != nullptr) {
        // tabulated dynamics: displacement (and beta) per control and node;
        // the minimum is taken over the candidates themselves
        T best = T(3);
        for (int k = 0; k < P.nc; ++k) {
          T d[DIM];
          const size_t e = (size_t)k * N + g;
          T b = beta, o = omb;
          if constexpr (sizeof(T) == 4) {
            for (int q = 0; q < DIM; ++q) d[q] = P.foot32[e * DIM + q] + 2.0f;
            if (P.bpk32) {
              b = P.bpk32[e];
              o = P.opk32[e];
            }
          } else {
            for (int q = 0; q < DIM; ++q) d[q] = P.foot64[e * DIM + q];
            if (P.bpk64) {
              b = P.bpk64[e];
              o = 1.0 - b;
            }
          }
          const T I = interp_global<T, DIM>(vin, P.n, px, py, pz, d);
          const T ck = Ar<T>::kruzkov(b, I, o);
          best = ck < best ? ck : best;
        }
        cand = best;
      } else {
        T mI = T(3);
        for (int k = 0; k < P.nc; ++k) {
          T d[DIM];
          for (int q = 0; q < DIM; ++q) {
            if constexpr (sizeof(T) == 4) {
              const float a = ((cf32p)P.ctrl32)[k * DIM + q];
              d[q] = __builtin_fmaf(c, a, w[q]);
            } else {
              const double a = ((cf64p)P.ctrl64)[k * DIM + q];
              double gg = c * a;
              if (P.has_drift) gg = gg + w[q];
              d[q] = P.step[q] * gg;
            }
          }
          const T I = interp_global<T, DIM>(vin, P.n, px, py, pz, d);
          mI = I < mI ? I : mI;
        }
        cand = Ar<T>::kruzkov(beta, mI, omb);
      }
      nv = cand < old ? cand : old;
      dd = (double)old - (double)nv;
    }
    vout[g] = nv;
  }
  wave_max(dd);
  if ((threadIdx.x & 63) == 0 && dd > 0.0)
    atomicMax(res_slot, (unsigned long long)__double_as_longlong(dd));
}

hipError_t launch_jacobi(bool fp64, int dim, const DevProblem *prob_dev, size_t N, const void *vin,
                         void *vout, unsigned long long *res_slot, hipStream_t s) {
  const int grid = (int)((N + 255) / 256);
  if (fp64) {
    if (dim == 2)
      hipLaunchKernelGGL((k_jacobi<double, 2>), dim3(grid), dim3(256), 0, s, prob_dev,
                         (const double *)vin, (double *)vout, res_slot);
    else
      hipLaunchKernelGGL((k_jacobi<double, 3>), dim3(grid), dim3(256), 0, s, prob_dev,
                         (const double *)vin, (double *)vout, res_slot);
  } else {
    if (dim == 2)
      hipLaunchKernelGGL((k_jacobi<float, 2>), dim3(grid), dim3(256), 0, s, prob_dev,
                         (const float *)vin, (float *)vout, res_slot);
    else
      hipLaunchKernelGGL((k_jacobi<float, 3>), dim3(grid), dim3(256), 0, s, prob_dev,
                         (const float *)vin, (float *)vout, res_slot);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- helpers

// bits[tile][w]: bit j set when the tile holds a non-target node of patch
// j; the last bit of the row (index words*32-1) marks tiles holding a
// target node.  One workgroup per tile ORs into an LDS row, then stores it.
constexpr int kMaxBitWords = 1024;

__global__ void __launch_bounds__(256)
k_tile_bits(const int16_t *__restrict__ code, int n0, int n1, int n2, int tx, int ty, int tz,
            int nt0, int nt1, int words, uint32_t *bits) {
  __shared__ uint32_t row[kMaxBitWords];
  const int t = blockIdx.x;
  const int ox = (t % nt0) * tx, oy = ((t / nt0) % nt1) * ty, oz = (t / (nt0 * nt1)) * tz;
  for (int w = threadIdx.x; w < words; w += blockDim.x) row[w] = 0u;
  __syncthreads();
  const int tbit = words * 32 - 1;
  const int cnt = tx * ty * tz;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int x = ox + i % tx, y = oy + (i / tx) % ty, z = oz + i / (tx * ty);
    if (x >= n0 || y >= n1 || z >= n2) continue;
    const int cd = code[(size_t)x + (size_t)n0 * ((size_t)y + (size_t)n1 * z)];
    const int bit = cd == CODE_TARGET ? tbit : cd;
    if (bit >= 0) atomicOr(&row[bit >> 5], 1u << (bit & 31));
  }
  __syncthreads();
  for (int w = threadIdx.x; w < words; w += blockDim.x) bits[(size_t)t * words + w] = row[w];
}

__global__ void __launch_bounds__(256)
k_item_keys(const int16_t *__restrict__ code, const double *__restrict__ u0, int n0, int n1,
            int n2, int tx, int ty, int tz, int nt0, int nt1, int ntiles, uint32_t *keys) {
  const size_t N = (size_t)n0 * n1 * n2;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < N;
       g += (size_t)gridDim.x * blockDim.x) {
    const int cd = code[g];
    if (cd < 0) continue;
    const int x = (int)(g % n0), y = (int)((g / n0) % n1), z = (int)(g / ((size_t)n0 * n1));
    const int t = x / tx + nt0 * (y / ty + nt1 * (z / tz));
    const double u = u0[g];
    const float key = u < 1.0 ? (float)(-log1p(-u)) : __int_as_float(0x7f800000);
    atomicMin(&keys[(size_t)cd * ntiles + t], __float_as_uint(key > 0.0f ? key : 0.0f));
  }
}

hipError_t launch_item_keys(const int16_t *code, const double *u0, const int32_t n[3],
                            const int32_t tile[3], const int32_t ntile[3], uint32_t *keys,
                            hipStream_t s) {
  const size_t N = (size_t)n[0] * n[1] * n[2];
  const int grid = (int)std::min<size_t>((N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_item_keys, dim3(grid), dim3(256), 0, s, code, u0, n[0], n[1], n[2],
                     tile[0], tile[1], tile[2], ntile[0], ntile[1],
                     ntile[0] * ntile[1] * ntile[2], keys);
  return hipGetLastError();
}

hipError_t launch_tile_bits(int dim, const int16_t *code, const int32_t n[3], const int32_t tile[3],
                            const int32_t ntile[3], int words, uint32_t *bits, hipStream_t s) {
  (void)dim;
  if (words > kMaxBitWords) return hipErrorInvalidValue;
  const int ntiles = ntile[0] * ntile[1] * ntile[2];
  hipLaunchKernelGGL(k_tile_bits, dim3((unsigned)ntiles), dim3(256), 0, s, code, n[0], n[1], n[2],
                     tile[0], tile[1], tile[2], ntile[0], ntile[1], words, bits);
  return hipGetLastError();
}

template <typename T>
__global__ void k_init_values(const int16_t *__restrict__ code, size_t N, T *v,
                              const double *__restrict__ start) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < N) {
    const int cd = code[g];
    v[g] = cd == CODE_TARGET ? T(0) : ((start && cd >= 0) ? (T)start[g] : T(1));
  }
}

hipError_t launch_init_values(bool fp64, const int16_t *code, size_t N, void *v, hipStream_t s,
                              const double *start) {
  const unsigned grid = (unsigned)((N + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(k_init_values<double>, dim3(grid), dim3(256), 0, s, code, N, (double *)v,
                       start);
  else
    hipLaunchKernelGGL(k_init_values<float>, dim3(grid), dim3(256), 0, s, code, N, (float *)v,
                       start);
  return hipGetLastError();
}

__global__ void k_beta_f32(const double *__restrict__ beta, float *beta32, float *omb32,
                           size_t n) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) {
    const double b = beta[g];
    beta32[g] = (float)b;
    omb32[g] = (float)(1.0 - b);
  }
}

hipError_t launch_beta_f32(const double *beta, float *beta32, float *omb32, size_t n,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_beta_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, beta, beta32,
                     omb32, n);
  return hipGetLastError();
}

__global__ void k_check_range(const double *__restrict__ x, size_t n, double lo, double hi,
                              int *bad) {
  int b = 0;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (size_t)gridDim.x * blockDim.x)
    if (!(x[g] >= lo && x[g] < hi)) b = 1;
  if (__ballot(b) != 0ull && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

hipError_t launch_check_range(const double *x, size_t n, double lo, double hi, int *bad,
                              hipStream_t s) {
  const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_check_range, dim3(grid), dim3(256), 0, s, x, n, lo, hi, bad);
  return hipGetLastError();
}

__global__ void k_f64_to_f32(const double *__restrict__ src, float *dst, size_t n) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) dst[g] = (float)src[g];
}

hipError_t launch_f64_to_f32(const double *src, float *dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// dst[r][d] = float(step[d] * src[r][d]) (per-axis scaling of vectors)
__global__ void k_scaled_f32(const double *__restrict__ src, float *dst, size_t rows, int dim,
                             double s0, double s1, double s2) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= rows * dim) return;
  const int d = (int)(g % dim);
  const double sc = d == 0 ? s0 : (d == 1 ? s1 : s2);
  dst[g] = (float)(sc * src[g]);
}

hipError_t launch_scaled_f32(const double *src, float *dst, size_t rows, int dim,
                             const double step[3], hipStream_t s) {
  const size_t n = rows * dim;
  hipLaunchKernelGGL(k_scaled_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst,
                     rows, dim, step[0], step[1], step[2]);
  return hipGetLastError();
}

// code = target ? TARGET : obstacle (in tp or as label) ? OBST :
//        (labels ? (selected(label) ? label : NONE) : 0)
__global__ void k_make_code(const int16_t *__restrict__ tp, const int16_t *__restrict__ lab,
                            const uint8_t *__restrict__ sel, size_t N, int16_t *code) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  int16_t c;
  if (tp[g] >= 0) c = CODE_TARGET;
  else if (tp[g] == TP_OBSTACLE) c = CODE_OBST;
  else if (!lab) c = 0;
  else {
    const int L = lab[g];
    c = L == TP_OBSTACLE ? CODE_OBST : (L >= 0 && (!sel || sel[L])) ? (int16_t)L : CODE_NONE;
  }
  code[g] = c;
}

__global__ void k_obstacles(const int16_t *__restrict__ tp, double *u0, size_t N, double theta,
                            int16_t *tp_out, unsigned long long *count) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ex = false;
  if (g < N) {
    int16_t t = tp[g];
    if (t == -1 && theta > 0.0 && u0[g] >= theta) {
      t = TP_OBSTACLE;
      ex = true;
    }
    if (t == TP_OBSTACLE) u0[g] = 1.0;
    tp_out[g] = t;
  }
  const unsigned long long m = __ballot(ex);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, (unsigned long long)__popcll(m));
}

hipError_t launch_obstacles(const int16_t *tp, double *u0, size_t N, double theta,
                            int16_t *tp_out, unsigned long long *count, hipStream_t s) {
  hipLaunchKernelGGL(k_obstacles, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, tp, u0, N,
                     theta, tp_out, count);
  return hipGetLastError();
}

hipError_t launch_make_code(const int16_t *target_part, const int16_t *labels,
                            const uint8_t *select, size_t N, int16_t *code, hipStream_t s) {
  hipLaunchKernelGGL(k_make_code, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, target_part,
                     labels, select, N, code);
  return hipGetLastError();
}

// Input scan of a device-resident problem: out[0..2] = max displacement
// bound per axis, out[3] = max target part + 2 (FP64 bits, non-negative);
// *bad = 1 on a non-finite or negative speed, non-finite drift or a target
// part below -2 (-2 marks an obstacle node).  Block reduction, one atomic
// per block and quantity.
__global__ void __launch_bounds__(256)
k_scan(const double *__restrict__ speed, const double *__restrict__ drift,
       const int16_t *__restrict__ tp, size_t N, int dim, double ax, double ay, double az,
       double s0, double s1, double s2, unsigned long long *out, int *bad) {
  __shared__ double red[4][4];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  double r[4] = {0.0, 0.0, 0.0, 0.0};
  int b = 0;
  const double am[3] = {ax, ay, az};
  const double st[3] = {s0, s1, s2};
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < N;
       g += (size_t)gridDim.x * blockDim.x) {
    const double c = speed[g];
    if (!(c >= 0.0) || !(c < 1e300)) b = 1;
    for (int d = 0; d < dim; ++d) {
      const double w = drift ? drift[g * dim + d] : 0.0;
      if (!(w < 1e300 && w > -1e300)) b = 1;
      const double x = st[d] * (c * am[d] + (w < 0 ? -w : w));
      r[d] = x > r[d] ? x : r[d];
    }
    const double t = (double)tp[g] + 2.0;
    r[3] = t > r[3] ? t : r[3];
    if (tp[g] < -2) b = 1;
  }
  __syncthreads();
  if (b) sbad = 1;
  for (int q = 0; q < 4; ++q) {
    double x = r[q];
    wave_max(x);
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double m = 0.0;
    for (int w = 0; w < 4; ++w) m = red[threadIdx.x][w] > m ? red[threadIdx.x][w] : m;
    if (m > 0.0) atomicMax(&out[threadIdx.x], (unsigned long long)__double_as_longlong(m));
  }
  if (threadIdx.x == 0 && sbad) atomicOr(bad, 1);
}

hipError_t launch_scan_problem(const hjb_problem &P, size_t N, const double amax[3],
                               unsigned long long *out4, int *bad, hipStream_t s) {
  const unsigned grid = (unsigned)std::min<size_t>((N + 255) / 256, 1024);
  hipLaunchKernelGGL(k_scan, dim3(grid), dim3(256), 0, s, P.speed, P.drift, P.target_part, N,
                     P.dim, amax[0], amax[1], amax[2], P.step[0], P.step[1], P.step[2], out4, bad);
  return hipGetLastError();
}

__global__ void k_count_active(const int16_t *__restrict__ code, size_t N, unsigned long long *out) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = (g < N && code[g] >= 0) ? 1 : 0;
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, (unsigned long long)c);
}

hipError_t launch_count_active(const int16_t *code, size_t N, unsigned long long *out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_count_active, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, code, N, out);
  return hipGetLastError();
}

template <typename T>
__global__ void k_fill(T *p, T v, size_t n) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) p[g] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t *p, int32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_i16(int16_t *p, int16_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<int16_t>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace hjb
