// Internal definitions shared by the kernels and the host runtime of libhjb.
//
// Device data model (one problem = one fine grid of the patchy solve, or a
// coarse grid, or the whole grid of a global solve):
//   - v[N]      value grid (float or double) in x-fastest order;
//   - code[N]   int16 node role: CODE_TARGET (v fixed at 0), CODE_NONE (never
//               updated, ghost in every patch), or the patch label j >= 0;
//   - tiles     the box is cut into TX x TY (x TZ) tiles; a work item is one
//               (problem, patch, tile) triple and only updates that patch's
//               nodes of that tile.  Items are scheduled through per-round
//               active lists (see RoundArgs).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "hjb.h"

namespace hjb {

constexpr int HALO = 2;  // foot points lie within 2 cells (checked on input)
constexpr int16_t CODE_TARGET = -2;
constexpr int16_t CODE_NONE = -1;
constexpr int16_t CODE_OBST = -3;  // obstacle or excluded node: ghost 1, never updated
// target_part / label value of an obstacle node (or an excluded one)
constexpr int16_t TP_OBSTACLE = -2;
// Statistics and residual counters are spread over kSlots addresses (slot =
// workgroup index mod kSlots) so that the workgroups of a round do not all
// update one address; the host reduces the slots.
constexpr int kSlots = 16;
// Per problem: residual [3][kSlots], pactive (3 u32), work [2][kSlots],
// ordering window (6 u32).
constexpr int kCounterWords = 3 * kSlots + 2 + 2 * kSlots + 3;  // u64 words per problem
// Item flag bit: the item must sweep all its bricks first (set when an item
// that had not run yet is carried to a later round).
constexpr uint32_t kFlagFull = 1u << 31;

// Per-problem parameters as the kernels see them.  Lives in device memory
// (an array of these for a batch).  Pointers are device pointers.
struct DevProblem {
  int32_t dim;
  int32_t n[3];
  int32_t ntile[3];     // tiles per axis for the sweep tile shape
  int32_t nc;           // number of controls
  int32_t n_patches;    // patches addressed by item_map
  int32_t has_drift;
  int32_t prob_index;   // index in the batch
  int32_t pad0;
  double beta, omb;     // FP64 Kruzkov constants
  double step[3];       // FP64 h / k_d
  float betaf, ombf;    // FP32 Kruzkov constants
  const double *ctrl64; // [rows][dim] a_k (FP64, as given); rows = round4(nc) + 4,
                        // rows past nc repeat the last control
  const float *ctrl32;  // [rows][dim] s_d * a_kd rounded to FP32
  const double *speed64;
  const float *speed32;
  const double *beta64;   // [N] per-node beta of the variable step, or null
  const float *beta32;    // [N] beta_i and 1 - beta_i rounded to FP32, or null
  const float *omb32;
  const double *foot64;   // [nc][N][dim] tabulated displacement (cells), or null
  const float *foot32;
  const double *bpk64;    // [nc][N] tabulated beta, or null
  const float *bpk32;     // and beta, 1 - beta rounded to FP32
  const float *opk32;
  const double *drift64;  // [N][dim] or null
  const float *drift32;   // [N][dim] s_d * w_d rounded to FP32, or null
  const int16_t *code;    // [N]
  void *v;                // [N] float or double
  const int32_t *item_map;  // [n_patches][ntiles]: local item id or -1
  int32_t item_base;        // global id of local item 0
  int32_t pad1;
  unsigned long long *residual;  // [3][kSlots] per-round max decrease (FP64 bits)
  uint32_t *pactive;             // [3] per-round count of queued items
  unsigned long long *work;      // [2][kSlots] node updates, item runs
  // Control cones of add-on AO3 (null / 0 without them): node p minimises
  // over the controls cone_idx[fb[p]][0..cone_len) only.  Rows are
  // cone_stride bytes (a multiple of 4), padded with the row's feedback
  // control.
  const double *u0;         // [N] Dirichlet data of other patches' nodes, or null
                            // (state constraint: ghost 1)
  const uint8_t *fb;        // [N] Step 2 feedback control of every node
  const uint8_t *cone_idx;  // [nc][cone_stride]
  int32_t cone_len;
  int32_t cone_stride;
  // Value-ordered schedule (add-on AO2, null / 0 without it): a queued item
  // runs in round r only if its key (the smallest minimal time -ln(1 - U^(0))
  // of its nodes) is at most the round's threshold, else it is carried to
  // the next round.  win[r % 3] is the base threshold of round r, win[3 + r %
  // 3] the smallest key queued for it (FP32 bits); the threshold is the
  // larger of the two, and the base of the next round exceeds it by win_dt.
  const float *item_key;  // [n_patches][ntiles] (like item_map)
  uint32_t *win;          // [6]
  float win_dt;
  int32_t plain;          // add-on AO1: v <- F(v) from U^(0) (updates may rise)
};

struct Item {
  int32_t prob;
  int32_t patch;
  int32_t tile;
  int32_t pad;
};

// Active-list rings of one engine.  Round r reads list[r&1] of length
// count[r%3] (built in round r-1 with flags[r&1]), appends the items to
// revisit to list[(r+1)&1] / count[(r+1)%3] using flags[(r+1)&1], and resets
// count[(r+2)%3] (unused in round r).  Every item clears its own flag of
// flags[r&1] when it is processed, so the flag array of the next-but-one
// round starts clear.
struct RoundArgs {
  const int32_t *list_in;
  int32_t *list_out;
  uint32_t *flags_in;
  uint32_t *flags_out;
  uint32_t *count;            // [3]
  unsigned long long *work;   // [2][kSlots]: node updates, item runs (colour transport)
  uint32_t round;
  int32_t inner_sweeps;
  int32_t nprob;
  int32_t pad;
  double tol;                 // a node "changes" when it decreases by more than tol
};

// Work queue of the asynchronous schedule: a ring of item ids filled by
// the workgroups that change a neighbour's halo and drained by every
// workgroup of one persistent launch.  An item is never queued twice nor run
// by two workgroups at once (per-item state), and the launch ends when no
// item is queued or running (`pending`).
struct AsyncQ {
  int32_t *ring;    // [mask + 1] item ids, -1 in an empty slot
  uint32_t mask;    // ring size - 1 (a power of two above the item count)
  uint32_t *state;  // [items] 0 idle, 1 queued, 2 running, 3 running and queued again
  uint32_t *sides;  // [items] tile sides whose halo changed since the item started
  uint32_t *ctr;    // [0] head, [1] tail, [2] pending, [3] abort code (0 = none)
};

// Trace (colour transport) engine arguments.
struct TraceArgs {
  int32_t n[3];
  int32_t ntile[3];
  int32_t nc;
  int32_t has_drift;
  int32_t n_parts;   // R
  int32_t words;     // mask words per tile, ceil(R / 32)
  int32_t tile_base; // id of the problem's first tile in a shared round list
  double step[3];
  double beta;       // per-step factor of the colour transport
  const double *ctrl64;
  const double *speed64;
  const double *drift64;
  const int16_t *target_part;
  const double *beta_node;  // [N] per-node beta (variable step) or null
  const double *foot;       // [nc][N][dim] tabulated displacement or null
  const double *beta_pk;    // [nc][N] tabulated beta or null
  const uint8_t *feedback;
  double *phi;       // [R][N], zero-initialised
  uint32_t *masks;   // [ntiles][words]: parts nonzero somewhere in the tile
  size_t N;
};

inline int div_up(int a, int b) { return (a + b - 1) / b; }

// Launchers (defined in the .hip translation units).
struct SweepShape {
  int dim, tx, ty, tz;
  int nt = 256;  // workgroup size
};
bool sweep_shape_supported(int dim, int tx, int ty, int tz, int nt);
hipError_t launch_sweep_async(bool fp64, SweepShape sh, int grid, const DevProblem *probs,
                              const Item *items, const RoundArgs &ra, const AsyncQ &q,
                              hipStream_t s);
hipError_t launch_sweep(bool fp64, SweepShape sh, int grid, const DevProblem *probs,
                        const Item *items, const RoundArgs &ra, hipStream_t s);
// Sweep of problems with tabulated dynamics (foot / beta tables).
bool sweep_tab_shape_supported(int dim, int tx, int ty, int tz, int nt);
hipError_t launch_sweep_tab(bool fp64, SweepShape sh, int grid, const DevProblem *probs,
                            const Item *items, const RoundArgs &ra, hipStream_t s);
// Sweep with the control cones of add-on AO3 (one problem, probs[0]); nc and
// cone_stride size the LDS tables.
bool sweep_cone_shape_supported(int dim, int tx, int ty, int tz, int nt);
size_t sweep_cone_lds_bytes(bool fp64, int dim, int nc, int cone_stride);
hipError_t launch_sweep_cone(bool fp64, SweepShape sh, int grid, const DevProblem *probs,
                             const Item *items, const RoundArgs &ra, int nc, int cone_stride,
                             hipStream_t s);
hipError_t launch_jacobi(bool fp64, int dim, const DevProblem *prob_dev, size_t N, const void *vin,
                         void *vout, unsigned long long *res_slot, hipStream_t s);
// keys[patch][tile] = min over the tile's nodes of that patch of
// -ln(1 - u0) (FP32 bits, +inf when the tile has none); keys preset to +inf.
hipError_t launch_item_keys(const int16_t *code, const double *u0, const int32_t n[3],
                            const int32_t tile[3], const int32_t ntile[3], uint32_t *keys,
                            hipStream_t s);
hipError_t launch_tile_bits(int dim, const int16_t *code, const int32_t n[3], const int32_t tile[3],
                            const int32_t ntile[3], int words, uint32_t *bits, hipStream_t s);
// v = 0 on the target, `start` (when given) on patch nodes, 1 elsewhere.
hipError_t launch_init_values(bool fp64, const int16_t *code, size_t N, void *v, hipStream_t s,
                              const double *start = nullptr);
hipError_t launch_f64_to_f32(const double *src, float *dst, size_t n, hipStream_t s);
// beta32 = (float)beta, omb32 = (float)(1 - beta) (the difference in FP64).
hipError_t launch_beta_f32(const double *beta, float *beta32, float *omb32, size_t n,
                           hipStream_t s);
// *bad = 1 when some x[i] is not in [lo, hi) (NaN included).
hipError_t launch_check_range(const double *x, size_t n, double lo, double hi, int *bad,
                              hipStream_t s);
hipError_t launch_scaled_f32(const double *src, float *dst, size_t rows, int dim,
                             const double step[3], hipStream_t s);
// Obstacles and exclusion (Sections 4.5, 4.6): tp_out = tp with
// TP_OBSTACLE where tp is -1 and theta > 0 and u0 >= theta; u0 = 1 at every
// obstacle node of tp_out.  *count (zeroed by the caller) receives the
// number of excluded nodes.
hipError_t launch_obstacles(const int16_t *tp, double *u0, size_t N, double theta,
                            int16_t *tp_out, unsigned long long *count, hipStream_t s);
hipError_t launch_make_code(const int16_t *target_part, const int16_t *labels,
                            const uint8_t *select, size_t N, int16_t *code, hipStream_t s);
hipError_t launch_scan_problem(const hjb_problem &P, size_t N, const double amax[3],
                               unsigned long long *out4, int *bad, hipStream_t s);

// Build step launchers.
hipError_t launch_prolong(int dim, const int32_t nf[3], const int32_t nc[3], const double *vc,
                          const int32_t *Q, const double *T, double *u0, hipStream_t s);
hipError_t launch_feedback(int dim, const TraceArgs &a, const double *u0, uint8_t *fb,
                           hipStream_t s);
hipError_t launch_trace_init(int dim, const TraceArgs &a, hipStream_t s);
int trace_chunk_capacity(int dim);
int trace_max_parts();
SweepShape trace_shape(int dim);
int trace_inner_sweeps(int dim);
// One round of colour transport over the tile ids in ra.list_in: `args`
// (device) holds the problems, `tile_prob` (device, null for one problem)
// the problem of every tile id, `max_words` the largest words of them;
// `split` workgroups share each activation (trace_split).
hipError_t launch_trace(int dim, int grid, int split, const TraceArgs *args,
                        const int32_t *tile_prob, int max_words, const RoundArgs &ra,
                        hipStream_t s);
// Queues the problem's tiles next to target nodes (ids from a.tile_base).
hipError_t launch_trace_seed(int dim, const TraceArgs &a, const RoundArgs &ra, hipStream_t s);
hipError_t launch_labels(int dim, const TraceArgs &a, int16_t *labels, uint32_t *unreached,
                         hipStream_t s);
hipError_t launch_label_fill(const int32_t n[3], const int16_t *in, int16_t *out,
                             uint32_t *changed, hipStream_t s);
// Pieces of a patch cut off from their own target part (labels of nodes
// off the target, tp = effective target_part) become -1; count += nodes
// relabelled.  parent [N] and attached [N] are scratch.  N < 2^31.
hipError_t launch_detach_pieces(const int32_t n[3], const int16_t *tp, int16_t *labels,
                                int32_t *parent, uint8_t *attached, uint32_t *count,
                                hipStream_t s);
hipError_t launch_count_active(const int16_t *code, size_t N, unsigned long long *out,
                               hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s);
hipError_t launch_fill_i16(int16_t *p, int16_t v, size_t n, hipStream_t s);

}  // namespace hjb
