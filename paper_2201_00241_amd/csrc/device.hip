// Device path of librh: the batched adjoint-adjoint reduction on gfx950.
//
// One launch processes a block of k directions W (Sec. 4.3, Algorithm 2).
// The directions are independent, so each workgroup owns C of them and runs
// every step of the reduction for its directions ("direction-owned" scheme):
//
//   1. SpMul            B' = -P G_p W                        (row-parallel)
//   2. BatchSparseSolve Z' = Uh^{-1} D^{-1} L^{-1} B'        (level-scheduled;
//      U = D Uh, so every sweep has a unit diagonal)
//   3. BatchTensorProjection (Sec. 4.2, forward-over-reverse of the branch
//      flows): every bus sums the second-order terms of its incident branches
//      (gather form of the "edges, then nodes" accumulation: no atomics), plus
//      the slack-cost rank-one term and the 2 c2 diagonal of the generator
//      costs.  The x part is written negated as the right-hand side of
//      step 4, the p part straight into the output.
//   4. BatchSparseSolve (transposed)  Psi' = L^{-T} D^{-1} Uh^{-T} (-P Y_x)
//   5. SpMulAdd         H W = Y_p + G_p^T Psi
//
// The working vector X (n_x x C, the C directions of a row contiguous) lives in
// LDS when it fits (the 10k-bus case: 149 KB for one FP64 direction of the
// 160 KB per CU), else in a per-workgroup global scratch slice.  Vectors in x
// space use the permuted (factor) numbering, so no permutation pass exists.
// Dependencies between triangular-sweep levels only ever cross threads of the
// same workgroup, so a workgroup barrier is the only synchronisation: no
// inter-workgroup flags or grid barrier.
//
// Rows of a level are spread over groups of 2^lg lanes (lg chosen per level
// on the host from the level's width and row lengths); a group's partial sums
// are combined by a butterfly of wave shuffles.  Every thread carries all C
// directions of its workgroup, so the arithmetic of one direction is the same
// for any k, any C and any workgroup it lands on (bitwise block-size
// invariance).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <exception>
#include <mutex>
#include <thread>

#include "rh_internal.h"

// Launch scratch of the allocation-free entry point (rh_hvp_device_noalloc):
// one fixed array per GPU, held from the code object's load until the process
// ends.  Its name is a host-side stand-in: host code takes the device address
// once per device with hipGetSymbolAddress (device_fixed_scratch_init) and
// passes only that address to kernels.
static __device__ __align__(256) double scratch[RH_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace rh {

namespace {

// One workgroup size for every variant: the sweep schedules (lane groups,
// wave steps) are built for it, so all variants do the same arithmetic.
// Read-only descriptors are read through the constant address space, so the
// compiler keeps their fields in scalar registers across global stores.
#define AS4 __attribute__((address_space(4)))

constexpr int kThreads = 1024;
constexpr int kThreadsLds = kThreads;
constexpr int kWaves = kThreads / 64;
// lanes x rows budget used to pick a level's lane-group size (fixed, so the
// schedule never depends on the launch shape)
constexpr int kLaneBudget = 1024;

constexpr int kBlockRows = 64;  // rows of a merged block of narrow levels (one wave)

// A triangular sweep in device form (see Packed in the host planner): steps,
// units with per-lane entry slots, row info and dense block inverses.
struct DevSweep {
  int32_t n_steps;
  const int4 *steps;  // {unit or wave directory offset, 0, kind, dense offset}
  const int4 *units;  // level and block units, 2 x int4: {slot_base, info_base, rows, groups}, {lg, E, lanes, -1}
  const int32_t *wdir;
  const int32_t *scol, *irow;
  int32_t n_slots, n_irow;  // lengths of the slot and row arrays
  const double *sval, *dense;   // unit diagonal (pivots are applied between sweeps)
  const float *sval32, *dense32;  // FP32 copies (refined mode)
  // wave units (see Packed): the FP64 and FP32 records, wide (any network)
  // and compact (null when the padded vector has more than 65,536 rows;
  // the kernels with X in LDS read these)
  int32_t n_wunits;
  const char *wrec, *wrec32;
  const char *wrecc, *wrecc32;
};

template <class T>
__device__ __forceinline__ const T *sw_val(const DevSweep AS4 &s);
template <>
__device__ __forceinline__ const double *sw_val<double>(const DevSweep AS4 &s) { return s.sval; }
template <>
__device__ __forceinline__ const float *sw_val<float>(const DevSweep AS4 &s) { return s.sval32; }
template <class T>
__device__ __forceinline__ const T *sw_dense(const DevSweep AS4 &s);
template <>
__device__ __forceinline__ const double *sw_dense<double>(const DevSweep AS4 &s) { return s.dense; }
template <>
__device__ __forceinline__ const float *sw_dense<float>(const DevSweep AS4 &s) { return s.dense32; }

// Tensor projection records.  Buses are taken in passes of kThreads (ordered
// by decreasing degree, so a pass's lanes have similar incidence counts); lane
// t of pass p holds bus p * kThreads + t of that order, and its incidence e
// is slot pass.x + e * kThreads + t for e < pass.y (the pass's largest
// degree), padded with slots whose ot is kPadInc.  Every record of a pass is
// addressed without reading another one, so a lane issues all its loads at
// once.  Records are planes of 16-byte words (a wave's load of one plane is
// 1 KB contiguous):
//   bus b:  {bits(tx, vs), ve}, {sth, sv}          planes of passes x kThreads words
//   slot k: {K, Hps}, {H, A2}, {vo, bits(ot, ov)}  planes of proj_slots words
// bits(a, b) holds two int32 (a in the low half) in the bytes of a double.
constexpr int32_t kPadInc = -2;
// record arrays stay below the out-of-range offset (see kOffRange)
constexpr int64_t kProjMaxBytes = 0x3f000000;

// A sparse matrix for row-parallel products with a vector in LDS (the
// residuals of the refined mode).  Rows are taken kThreads per pass in order
// of decreasing length; lane t of pass p owns row rows[p * kThreads + t] (-1:
// none), and its entry e sits in slot pass_first[p] + e * kThreads + t of the
// column and value planes (padding: column 0, value 0).  A pass is read in
// chunks of kEllChunk entries; chunk c is {first slot, pass, flags}, flags
// bit 0 = first chunk of its pass, bit 1 = last.  norm = max row sum of |a|.
constexpr int kEllChunk = 8;
struct EllMat {
  int32_t n_chunks, n_slots;
  const int4 *chunks;
  const int32_t *rows, *col;
  const double *val;
  double norm;
};

struct NetDesc {
  int32_t n_x, n_p, n_bus, n_slack, n_proj_pass, n_gp_rows;
  DevSweep L, U, Ut, Lt;  // U and Ut hold the unit factor D^{-1} U
  const double *pivinv;   // D^{-1}, applied between the two sweeps of a solve
  const float *pivinv32;
  // G_p, rows in permuted x order: one record {row, first entry, end, 0}
  // per row with entries, in row order, and the entries' columns and values
  const int4 *gp_rows;
  const int32_t *gp_col;
  const double *gp_val;
  const int32_t *gpt_ptr, *gpt_col;  // G_p^T, columns in permuted x order
  const double *gpt_val;
  // bus tangent sources: theta from X[tx] (-1: reference, zero tangent);
  // v from X[vs] if vs >= 0, else from W[-vs - 1] (generator magnitude)
  const double2 *proj_bus, *proj_inc;
  const int2 *proj_pass;  // {first slot, slots per lane}
  int32_t proj_slots;
  const int32_t *slack_thx, *slack_vs;
  const double *slack_gth, *slack_gv;
  // 2 c2 of the generator whose output is parameter q; NaN where parameter q
  // is a voltage magnitude (its Y_p comes from the projection)
  const double *p_c2x2;
  // first-order adjoint lambda (permuted x order) and grad_p f at the
  // operating point: the reduced gradient is grad_p f + G_p^T lambda
  const double *lam, *fp;
  // G_x and G_x^T in permuted numbering (residuals of the refined mode)
  EllMat gx, gxt;
};

// One unit of work: a block of k directions of one network (column-major
// W and HW with leading dimensions ldw, ldhw; identity_from >= 0 means W is
// columns identity_from .. of the identity and is not read).
struct WorkItem {
  const NetDesc *nd;  // device copy of the network's descriptor
  const double *W;
  double *HW;
  int64_t ldw, ldhw;
  int32_t k, identity_from;
  int32_t chunk0;  // first chunk of C directions of this item in the launch
  int32_t pad;
  // refined mode: per direction {backward error of Z, corrections of Z,
  // backward error of Psi, corrections of Psi} (4 doubles), or nullptr
  double *rinfo;
};

struct LaunchArgs {
  const WorkItem *items;  // n_items entries in device memory; nullptr: `one`
  WorkItem one;
  int32_t n_items, n_chunks;
  int32_t refine;  // refined mode: at most this many correction steps after the first FP32 solve
  double refine_tol;  // refined mode: stop a direction once ||r|| <= tol ||A|| ||x|| (inf-norms)
  double *scratch;
  int64_t scratch_stride;  // doubles per workgroup
  int32_t pad_rows;        // rows of the padded working vector: the largest n_x + kWavePadRows
  long long *stamps;       // kStamps wall-clock stamps per workgroup, or nullptr
  long long *step_stamps;  // debug: workgroup 0 stamps the steps of its sweeps (4 x kSweepStamps)
};

constexpr int kMaxStepStamps = 128;
constexpr int kSweepStamps = kMaxStepStamps;

constexpr int kStamps = 8;

__device__ __forceinline__ double w_at(const WorkItem &a, int32_t q, int32_t dir) {
  if (dir >= a.k) return 0.0;
  if (a.identity_from >= 0) return (q == a.identity_from + dir) ? 1.0 : 0.0;
  return a.W[(int64_t)dir * a.ldw + q];
}

// The work item that holds global chunk `chunk` (items sorted by chunk0).
__device__ __forceinline__ WorkItem item_of(const LaunchArgs &la, int32_t chunk) {
  if (!la.items) return la.one;
  int32_t lo = 0, hi = la.n_items - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (la.items[mid].chunk0 <= chunk)
      lo = mid;
    else
      hi = mid - 1;
  }
  return la.items[lo];
}

// A unit of a sweep (see DevSweep): its slot layout.
struct Unit {
  int32_t slot_base, info_base, rows, groups, lg, E, lanes;
  bool assign;  // x_i = sum (second half of a wave block) instead of x_i - sum
};

// Descriptors are read through the constant address space: scalar loads,
// which wait on their own counter instead of behind the vector loads in
// flight (the arrays are never written while a kernel runs).
__device__ __forceinline__ Unit unit_at(const DevSweep AS4 &s, int32_t u) {
  const int32_t AS4 *w = (const int32_t AS4 *)(s.units + 2 * u);
  return Unit{w[0], w[1], w[2], w[3], w[4], w[5], w[6], false};
}

__device__ __forceinline__ int4 step_at(const DevSweep AS4 &s, int32_t k) {
  const int32_t AS4 *w = (const int32_t AS4 *)(s.steps + k);
  return make_int4(w[0], w[1], w[2], w[3]);
}

// The first kPre entry slots of one lane in one pass of a unit, with its
// row's matrix row.  None of it depends on the solution
// vector, so it is loaded a unit (or a step) ahead and the only dependent
// accesses left on the critical path are LDS gathers and wave shuffles.
constexpr int kPre = 4;
template <class T>
struct Slots {
  int32_t col[kPre];
  T val[kPre];
  int32_t row;
};

// Buffer resources of a sweep's slot and row arrays: loads take a uniform
// byte offset in a scalar register and the lane's offset in a vector
// register, so a unit's loads need no per-lane address arithmetic (and reads
// past the end return 0).
struct WaveBufs {
  __amdgpu_buffer_rsrc_t col, val, row;
};

constexpr int kBufWord3 = 0x00020000;  // raw (untyped) buffer access on gfx9-family targets

template <class T>
__device__ __forceinline__ WaveBufs wave_bufs(const DevSweep AS4 &s) {
  WaveBufs b;
  b.col = __builtin_amdgcn_make_buffer_rsrc((void *)s.scol, 0, s.n_slots * 4, kBufWord3);
  b.val = __builtin_amdgcn_make_buffer_rsrc((void *)sw_val<T>(s), 0, s.n_slots * (int)sizeof(T), kBufWord3);
  b.row = __builtin_amdgcn_make_buffer_rsrc((void *)s.irow, 0, s.n_irow * 4, kBufWord3);
  return b;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <class T>
__device__ __forceinline__ T buf_load_val(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double buf_load_val<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_load_val<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// Lanes past the unit's rows use a lane offset beyond every buffer's range:
// their loads return 0 (column 0, value 0) without touching memory, so their
// gathers all hit one LDS word.
constexpr int kOffRange = 0x40000000;

// Two values of a lane's slot pair with one access.
template <class T>
__device__ __forceinline__ void buf_load_pair(__amdgpu_buffer_rsrc_t r, int voff, int soff, T &a, T &b);
template <>
__device__ __forceinline__ void buf_load_pair<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff, double &a,
                                                      double &b) {
  const f64x2 v = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  a = v.x;
  b = v.y;
}
template <>
__device__ __forceinline__ void buf_load_pair<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff, float &a,
                                                     float &b) {
  const f32x2 v = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  a = v.x;
  b = v.y;
}

// The first kPre slots of one pass of a unit for one lane, and the lane's
// row (see Packed): base is the pass's first slot, rbase the row-info index
// of its first row; the lane's column quad sits at base + 4 lane, its value
// pairs at base + 2 lane and base + 2 lanes + 2 lane.  A lane without a row
// (act false), or a pass without slots, reads nothing: out-of-range offsets
// return zeros.  Every call issues the same four loads.
template <class T>
__device__ __forceinline__ Slots<T> unit_load(const WaveBufs &B, int32_t base, int32_t rbase, int32_t lanes,
                                              int32_t lg, int lane, bool act, bool slots) {
  static_assert(kPre == 4, "one column quad and two value pairs per lane");
  Slots<T> L;
  const int vc = act && slots ? lane * 16 : kOffRange;
  const int vv = act && slots ? lane * 2 * (int)sizeof(T) : kOffRange;
  const int vr = act ? (lane >> lg) * 4 : kOffRange;
  // uniform offsets: say so, or the compiler may keep them in vector
  // registers and loop over their distinct values
  const int32_t s0 = __builtin_amdgcn_readfirstlane(base), s1 = __builtin_amdgcn_readfirstlane(base + 2 * lanes);
  const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(B.col, vc, s0 * 4, 0);
  buf_load_pair<T>(B.val, vv, s0 * (int)sizeof(T), L.val[0], L.val[1]);
  buf_load_pair<T>(B.val, vv, s1 * (int)sizeof(T), L.val[2], L.val[3]);
  L.col[0] = (int32_t)c.x;
  L.col[1] = (int32_t)c.y;
  L.col[2] = (int32_t)c.z;
  L.col[3] = (int32_t)c.w;
  L.row = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(B.row, vr, __builtin_amdgcn_readfirstlane(rbase) * 4, 0);
  return L;
}

// Pass `pass` of a level or block unit.
template <class T>
__device__ __forceinline__ Slots<T> load_slots(const WaveBufs &B, const Unit &U, int32_t pass, int lane) {
  const bool act = lane < U.lanes && pass * U.groups + (lane >> U.lg) < U.rows;
  return unit_load<T>(B, U.slot_base + pass * U.E * U.lanes, U.info_base + pass * U.groups, U.lanes, U.lg, lane,
                      act, U.E > 0);
}


// Cross-lane moves within a row of 16 lanes (DPP, no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over aligned groups of 2^lg lanes (lg uniform, 0..6); the group's first
// lane receives the total.  Pairs within a quad (lane ^ 1, lane ^ 2), then
// the mirror within 8 and within 16 lanes (every lane of the smaller group
// holds its total by then), then lane ^ 16 and lane ^ 32 by permute.  The
// tests are nested so that the common sizes (4 and 8 lanes) take two or
// three uniform branches.
template <class T>
__device__ __forceinline__ T group_sum(T v, int lg) {
  if (lg >= 2) {
    v += dpp_move<0xB1>(v);  // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);  // quad_perm [2,3,0,1]
    if (lg >= 3) {
      v += dpp_move<0x141>(v);  // row_half_mirror
      if (lg >= 4) {
        v += dpp_move<0x140>(v);  // row_mirror
        if (lg >= 5) {
          v += __shfl_xor(v, 16);
          if (lg >= 6) v += __shfl_xor(v, 32);
        }
      }
    }
  } else if (lg == 1) {
    v += dpp_move<0xB1>(v);
  }
  return v;
}

// The dense inverse of a block (rows <= kBlockRows, row-major) is applied
// by all NT threads: NT / kBlockRows lanes per row, each with E entries
// (columns j, j + lanes, ...) that it loads a step ahead, then a group sum.
template <int NT>
struct DenseShape {
  static constexpr int lanes = NT / kBlockRows;
  static constexpr int E = kBlockRows / lanes;
  static_assert(lanes * E == kBlockRows && (lanes & (lanes - 1)) == 0 && lanes <= 64, "dense block shape");
};

template <class T, int NT>
struct DenseRow {
  T m[DenseShape<NT>::E];
  int32_t row;
};

template <class T, int NT>
__device__ __forceinline__ DenseRow<T, NT> load_dense(const DevSweep AS4 &s, int32_t off, const Unit &U, int tid) {
  using D = DenseShape<NT>;
  DenseRow<T, NT> R;
  const T *Dz = sw_dense<T>(s);  // Dz[0] is a zero
  const int32_t a = tid / D::lanes, j = tid % D::lanes;
#pragma unroll
  for (int e = 0; e < D::E; ++e) {
    const int32_t b = j + e * D::lanes;
    const bool ok = a < U.rows && b <= a;
    R.m[e] = Dz[ok ? off + a * U.rows + b : 0];
  }
  R.row = s.irow[a < U.rows ? U.info_base + a : 0];  // written only by j == 0, a < rows
  return R;
}

// x = M^{-1} r for a block's rows: r in s_r (rows of C), x to X[row].
template <int C, int NT, class T>
__device__ __forceinline__ void dense_apply(const Unit &U, const DenseRow<T, NT> &R, T *__restrict__ X,
                                            const T *__restrict__ s_r, int tid) {
  using D = DenseShape<NT>;
  const int32_t a = tid / D::lanes, j = tid % D::lanes;
  T acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = T(0);
#pragma unroll
  for (int e = 0; e < D::E; ++e) {
    const int32_t b = j + e * D::lanes;
    const bool ok = a < U.rows && b <= a;
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = fma(R.m[e], ok ? s_r[b * C + c] : T(0), acc[c]);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = group_sum(acc[c], __builtin_ctz(D::lanes));  // to lane j == 0
  if (j == 0 && a < U.rows) {
#pragma unroll
    for (int c = 0; c < C; ++c) X[R.row * C + c] = acc[c];
  }
}

// One lane's share of one pass of a unit, in two halves so that a caller can
// reuse the slot registers in between: lane_dot forms the partial dot product
// of the lane's slots with X (the X values of the prefetched slots gathered
// first, then any further slots), lane_finish sums over the lane group and
// the group's first lane writes the row (or, in a block, its residual into
// s_r; in an assigning unit, the sum itself).  Padding slots are (0, 0).  An
// assigning unit has one pass, so all its lanes read X before any lane of the
// wave writes.  Every lane of the wave takes part (the group sum needs them).
template <int C, class T>
struct Part {
  T v[C];
};

template <int C, class T>
__device__ __forceinline__ Part<C, T> lane_dot(const WaveBufs &B, const Unit &U, int32_t pass, int lane,
                                               const Slots<T> &L, const T *__restrict__ X) {
  Part<C, T> P;
  T xv[kPre][C];
#pragma unroll
  for (int e = 0; e < kPre; ++e)
#pragma unroll
    for (int c = 0; c < C; ++c) xv[e][c] = X[L.col[e] * C + c];
#pragma unroll
  for (int c = 0; c < C; ++c) P.v[c] = T(0);
#pragma unroll
  for (int e = 0; e < kPre; ++e)
#pragma unroll
    for (int c = 0; c < C; ++c) P.v[c] = fma(L.val[e], xv[e][c], P.v[c]);
  // remaining slots, a column quad and two value pairs at a time
  if (U.E > kPre) {
    const bool act = lane < U.lanes && pass * U.groups + (lane >> U.lg) < U.rows;
    const int vc = act ? lane * 16 : kOffRange;
    const int vv = act ? lane * 2 * (int)sizeof(T) : kOffRange;
    const int32_t base = U.slot_base + pass * U.E * U.lanes;
    for (int32_t e0 = kPre; e0 < U.E; e0 += 4) {
      const int32_t s0 = __builtin_amdgcn_readfirstlane(base + e0 * U.lanes);
      const int32_t s1 = __builtin_amdgcn_readfirstlane(base + (e0 + 2) * U.lanes);
      const u32x4 cq = __builtin_amdgcn_raw_buffer_load_b128(B.col, vc, s0 * 4, 0);
      T v[4];
      buf_load_pair<T>(B.val, vv, s0 * (int)sizeof(T), v[0], v[1]);
      buf_load_pair<T>(B.val, vv, s1 * (int)sizeof(T), v[2], v[3]);
      const int32_t j[4] = {(int32_t)cq.x, (int32_t)cq.y, (int32_t)cq.z, (int32_t)cq.w};
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < C; ++c) P.v[c] = fma(v[e], X[j[e] * C + c], P.v[c]);
    }
  }
  return P;
}

template <int C, class T>
__device__ __forceinline__ void lane_finish(const Unit &U, int32_t pass, int lane, int32_t row, Part<C, T> P,
                                            T *__restrict__ X, T *__restrict__ s_r,
                                            bool block) {
#pragma unroll
  for (int c = 0; c < C; ++c) P.v[c] = group_sum(P.v[c], U.lg);
  const int32_t r = pass * U.groups + (lane >> U.lg);
  if (lane < U.lanes && r < U.rows && (lane & ((1 << U.lg) - 1)) == 0) {
    const int32_t i = row * C;
    if (block) {
#pragma unroll
      for (int c = 0; c < C; ++c) s_r[r * C + c] = X[i + c] - P.v[c];
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) X[i + c] = U.assign ? P.v[c] : X[i + c] - P.v[c];
    }
  }
}

template <int C, class T>
__device__ __forceinline__ void lane_update(const WaveBufs &B, const Unit &U, int32_t pass, int lane,
                                            const Slots<T> &L, T *__restrict__ X,
                                            T *__restrict__ s_r, bool block) {
  lane_finish<C, T>(U, pass, lane, L.row, lane_dot<C, T>(B, U, pass, lane, L, X), X, s_r, block);
}

// Synchronisation inside a sweep.  With X in LDS the sweep's threads only
// communicate through LDS (the right-hand side and the factors are read-only
// in global memory), so the barriers fence LDS only and leave the prefetch
// loads in flight; within one wave, LDS operations are performed in order, so
// a wave level only needs a compiler barrier.  With X in global memory both
// wait for the vector-memory counter.
template <bool LDSX>
__device__ __forceinline__ void step_barrier() {
  if constexpr (LDSX) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  } else {
    __syncthreads();
  }
}

template <bool LDSX>
__device__ __forceinline__ void wave_sync() {
  if constexpr (LDSX) {
    __builtin_amdgcn_wave_barrier();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
}

// Wave units (see Packed) are fixed-shape records of 64 lanes, one record
// per unit, interleaved: the lane's four column offsets (16 bytes at 16 l),
// its start and write row offsets (8 bytes at 1024 + 8 l), its four values
// (FP64: two pairs at 1536 + 16 l and 2560 + 16 l; FP32: one quad at
// 1536 + 16 l).  The offsets address the padded vector: zero row, 64 dummy
// rows, then the solution (kWavePadRows); they are for 8-byte rows and are
// scaled for the row size of C directions of T.  With the vector in LDS the
// padded vector starts at LDS address 0 (the LDS kernels have no static LDS),
// so an offset is an LDS address and a gather needs no address arithmetic.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
#define AS3 __attribute__((address_space(3)))

template <class T>
struct WaveRec;
template <>
struct WaveRec<double> {
  static constexpr int bytes = 3584;
};
template <>
struct WaveRec<float> {
  static constexpr int bytes = 2560;
};

template <class T>
__device__ __forceinline__ const char *sw_wrec(const DevSweep AS4 &s);
template <>
__device__ __forceinline__ const char *sw_wrec<double>(const DevSweep AS4 &s) { return s.wrec; }
template <>
__device__ __forceinline__ const char *sw_wrec<float>(const DevSweep AS4 &s) { return s.wrec32; }
template <class T>
__device__ __forceinline__ const char *sw_wrecc(const DevSweep AS4 &s);
template <>
__device__ __forceinline__ const char *sw_wrecc<double>(const DevSweep AS4 &s) { return s.wrecc; }
template <>
__device__ __forceinline__ const char *sw_wrecc<float>(const DevSweep AS4 &s) { return s.wrecc32; }
template <class T>
struct WaveRecC;
template <>
struct WaveRecC<double> {
  static constexpr int bytes = kWaveRecCompact64;
};
template <>
struct WaveRecC<float> {
  static constexpr int bytes = kWaveRecCompact32;
};

// Byte offset of an 8-byte-row offset in a vector whose rows are C values of T.
template <int C, class T>
__device__ __forceinline__ uint32_t row_bytes(uint32_t off) {
  constexpr int rb = C * (int)sizeof(T);
  static_assert(rb == 4 || rb == 8 || rb == 16 || rb == 32, "row size");
  if constexpr (rb == 4) return off >> 1;
  else if constexpr (rb == 8) return off;
  else if constexpr (rb == 16) return off << 1;
  else return off << 2;
}

// Element c of the padded-vector row at 8-byte-row offset off: in LDS the
// padded vector starts at address 0; in global memory at Xpad.
template <int C, class T, bool LDSX>
__device__ __forceinline__ T xget(const T *Xpad, uint32_t off, int c) {
  const uint32_t b = row_bytes<C, T>(off) + (uint32_t)(c * sizeof(T));
  if constexpr (LDSX) return *(const AS3 T *)(size_t)b;
  else return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(Xpad) + b);
}
template <int C, class T, bool LDSX>
__device__ __forceinline__ void xput(T *Xpad, uint32_t off, int c, T v) {
  const uint32_t b = row_bytes<C, T>(off) + (uint32_t)(c * sizeof(T));
  if constexpr (LDSX) *(AS3 T *)(size_t)b = v;
  else *reinterpret_cast<T *>(reinterpret_cast<char *>(Xpad) + b) = v;
}

template <class T>
struct WRing {
  u32x4 col;
  u32x2 row;  // start row, write row
  T val[4];
};

// The record at byte soff of the buffer R (uniform), with per-lane byte
// offsets of the column quad (vc), the row words (vr) and the value pairs
// (vv0, vv1; FP32 reads its quad at vv0).  An out-of-range offset reads
// zeros without a memory access, and so does the whole record past the
// buffer's end: a unit that reads and writes +0 at the zero row.
template <class T>
__device__ __forceinline__ void wrec_load(__amdgpu_buffer_rsrc_t R, int32_t soff, int vc, int vr, int vv0, int vv1,
                                          WRing<T> &W) {
  const int32_t so = __builtin_amdgcn_readfirstlane(soff);
  W.col = __builtin_amdgcn_raw_buffer_load_b128(R, vc, so, 0);
  W.row = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(R, vr, so, 0));
  if constexpr (sizeof(T) == 8) {
    const f64x2 a = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(R, vv0, so, 0));
    const f64x2 b = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(R, vv1, so, 0));
    W.val[0] = a.x;
    W.val[1] = a.y;
    W.val[2] = b.x;
    W.val[3] = b.y;
  } else {
    (void)vv1;
    const f32x4 a = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(R, vv0, so, 0));
    W.val[0] = a.x;
    W.val[1] = a.y;
    W.val[2] = a.z;
    W.val[3] = a.w;
  }
}

// A compact record (see wave_records): one 16-byte header per lane with the
// four column rows, the start and write rows (16-bit row indices) and the
// flags, then the values.  vh, vv0, vv1: per-lane byte offsets of the header
// and the value pairs (FP32 reads its quad at vv0).
template <class T>
struct WRingC {
  u32x4 hdr;
  T val[4];
};

template <class T>
__device__ __forceinline__ void wrecc_load(__amdgpu_buffer_rsrc_t R, int32_t soff, int vh, int vv0, int vv1,
                                           WRingC<T> &W) {
  const int32_t so = __builtin_amdgcn_readfirstlane(soff);
  W.hdr = __builtin_amdgcn_raw_buffer_load_b128(R, vh, so, 0);
  if constexpr (sizeof(T) == 8) {
    const f64x2 a = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(R, vv0, so, 0));
    const f64x2 b = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(R, vv1, so, 0));
    W.val[0] = a.x;
    W.val[1] = a.y;
    W.val[2] = b.x;
    W.val[3] = b.y;
  } else {
    (void)vv1;
    const f32x4 a = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(R, vv0, so, 0));
    W.val[0] = a.x;
    W.val[1] = a.y;
    W.val[2] = a.z;
    W.val[3] = a.w;
  }
}

// The wave walk on compact records with X in LDS (see wave_walk): the same
// unit, its header one load instead of the column quad and the row words.
template <int C, class T>
__device__ __forceinline__ void wave_walk_c(const DevSweep AS4 &s, int32_t u0, int32_t u1, int l64, T *Xpad) {
  const int32_t n = u1 - u0;
  if (n <= 0) return;
  constexpr int RB = WaveRecC<T>::bytes;
  const __amdgpu_buffer_rsrc_t R = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(sw_wrecc<T>(s) + (int64_t)u0 * RB), 0, n * RB, kBufWord3);
  const int vh = l64 * 16, vv0 = l64 * 16 + 1024, vv1 = l64 * 16 + 2048;
  WRingC<T> ring[kWaveAhead];
#pragma unroll
  for (int d = 0; d < kWaveAhead; ++d) {
    wrecc_load<T>(R, d * RB, vh, vv0, vv1, ring[d]);
    __builtin_amdgcn_sched_barrier(0);
  }
  int32_t soff = kWaveAhead * RB;
  for (int32_t j = 0; j < n; j += kWaveAhead) {
#pragma unroll
    for (int d = 0; d < kWaveAhead; ++d) {
      const u32x4 h = ring[d].hdr;
      const uint32_t c0 = (h.x & 0xffffu) << 3, c1 = (h.x >> 16) << 3;
      const uint32_t c2 = (h.y & 0xffffu) << 3, c3 = (h.y >> 16) << 3;
      const uint32_t rs = (h.z & 0xffffu) << 3, rw = (h.z >> 16) << 3;
      const int lg = (int)((uint32_t)__builtin_amdgcn_readfirstlane(h.w) >> 2);
      // loads of the unit kWaveAhead on
      const bool nact = h.w & 1u, ntwo = (h.w >> 1) & 1u;
      const int nv0 = nact ? vv0 : kOffRange, nv1 = ntwo ? vv1 : kOffRange;
      T xv[4][C], xr[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        xv[0][c] = xget<C, T, true>(Xpad, c0, c);
        xv[1][c] = xget<C, T, true>(Xpad, c1, c);
        xv[2][c] = xget<C, T, true>(Xpad, c2, c);
        xv[3][c] = xget<C, T, true>(Xpad, c3, c);
        xr[c] = xget<C, T, true>(Xpad, rs, c);
      }
      T part[C];
#pragma unroll
      for (int c = 0; c < C; ++c) part[c] = T(0);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < C; ++c) part[c] = fma(ring[d].val[e], xv[e][c], part[c]);
      T nv[C];
#pragma unroll
      for (int c = 0; c < C; ++c) nv[c] = xr[c] - group_sum(part[c], lg);
      // every lane writes (lanes without a row to their dummy rows)
#pragma unroll
      for (int c = 0; c < C; ++c) xput<C, T, true>(Xpad, rw, c, nv[c]);
      wave_sync<true>();  // this wave's writes before its next unit's reads
      wrecc_load<T>(R, soff, vh, nv0, nv1, ring[d]);
      soff += RB;
    }
  }
}

// A wave's walk through its units of a wave step, units u0 .. u1 - 1.  Unit
// j runs at step j while the records of units j + 1 .. j + kWaveAhead - 1 are
// in flight, and issues the load of unit j + kWaveAhead's record when it is
// done with its own (so the new record takes the registers of the old).
// Every unit is the same few instructions: five gathers, four FMAs, the group
// sum (its width, lg, is the one per-unit choice, from the write words), one
// subtraction and one write per lane (lanes that own no row write their dummy
// rows).  A unit's start words say which lanes of the unit kWaveAhead on have
// entries, and which have a second value pair: the other lanes skip those
// loads (the vector memory path, not the arithmetic, bounds a wave step, and
// most lanes hold at most two entries).  The buffer resource covers this
// wave's records only, so records past its last unit read as zeros.
template <int C, class T, bool LDSX>
__device__ __forceinline__ void wave_walk(const DevSweep AS4 &s, int32_t u0, int32_t u1, int l64, T *Xpad) {
  const int32_t n = u1 - u0;
  if (n <= 0) return;
  constexpr int RB = WaveRec<T>::bytes;
  const __amdgpu_buffer_rsrc_t R = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(sw_wrec<T>(s) + (int64_t)u0 * RB), 0, n * RB, kBufWord3);
  const int vc = l64 * 16, vr = l64 * 8 + 1024, vv0 = l64 * 16 + 1536, vv1 = l64 * 16 + 2560;
  WRing<T> ring[kWaveAhead];
  // the first records in full, issued in ring order (the loop's wait counts
  // assume the oldest record is the next one used, also on entry)
#pragma unroll
  for (int d = 0; d < kWaveAhead; ++d) {
    wrec_load<T>(R, d * RB, vc, vr, vv0, vv1, ring[d]);
    __builtin_amdgcn_sched_barrier(0);
  }
  int32_t soff = kWaveAhead * RB;
  // every unrolled step runs (a step past the end is the zero unit), so the
  // same loads are in flight on every path through the loop
  for (int32_t j = 0; j < n; j += kWaveAhead) {
#pragma unroll
    for (int d = 0; d < kWaveAhead; ++d) {
      const u32x4 cq = ring[d].col;
      const uint32_t rx = ring[d].row.x, ry = ring[d].row.y;
      const int lg = (int)((uint32_t)__builtin_amdgcn_readfirstlane(ry) >> kWaveLgShift);
      const uint32_t rs = rx & kWaveOffMask, rw = ry & kWaveOffMask;
      // loads of the unit kWaveAhead on
      const bool nact = (rx >> kWaveActBit) & 1u, ntwo = (rx >> kWaveTwoBit) & 1u;
      const int nc = nact ? vc : kOffRange, nv0 = nact ? vv0 : kOffRange, nv1 = ntwo ? vv1 : kOffRange;
      T xv[4][C], xr[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        xv[0][c] = xget<C, T, LDSX>(Xpad, cq.x, c);
        xv[1][c] = xget<C, T, LDSX>(Xpad, cq.y, c);
        xv[2][c] = xget<C, T, LDSX>(Xpad, cq.z, c);
        xv[3][c] = xget<C, T, LDSX>(Xpad, cq.w, c);
        xr[c] = xget<C, T, LDSX>(Xpad, rs, c);
      }
      T part[C];
#pragma unroll
      for (int c = 0; c < C; ++c) part[c] = T(0);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < C; ++c) part[c] = fma(ring[d].val[e], xv[e][c], part[c]);
      T nv[C];
#pragma unroll
      for (int c = 0; c < C; ++c) nv[c] = xr[c] - group_sum(part[c], lg);
      if constexpr (LDSX) {
        // every lane writes (lanes without a row to their dummy rows): no
        // mask, and LDS writes of distinct rows cost little
#pragma unroll
        for (int c = 0; c < C; ++c) xput<C, T, LDSX>(Xpad, rw, c, nv[c]);
      } else if (rw >= (uint32_t)kWavePadRows * 8u) {
        // in global memory only the lanes that own a row store
#pragma unroll
        for (int c = 0; c < C; ++c) xput<C, T, LDSX>(Xpad, rw, c, nv[c]);
      }
      wave_sync<LDSX>();  // this wave's writes before its next unit's reads
      // the record kWaveAhead units on, into the registers this one held
      wrec_load<T>(R, soff, nc, vr, nv0, nv1, ring[d]);
      soff += RB;
    }
  }
}

// Level-scheduled triangular sweep on X (rows of C directions).
//
// Steps: a plain level (independent rows); a block of consecutive narrow
// levels, whose rows first form residuals r = init - (entries to earlier
// steps) and then x = M^{-1} r with the block's dense inverse (the host split
// off the entries inside the block); or a wave step, in which every wave walks
// its own elimination subtrees level by level with wave-local ordering only.
// A workgroup barrier separates steps.
template <int C, int NT, class T, bool LDSX>
__device__ __forceinline__ void sweep(const DevSweep AS4 &s, T *__restrict__ X,
                                      T *__restrict__ s_r, int tid, long long *ss = nullptr) {
  const int32_t ns = s.n_steps;
  if (ns == 0) return;
  if (ss && tid == 0) ss[0] = wall_clock64();
  const WaveBufs B = wave_bufs<T>(s);
  // The next level or block step's first slots and, for a block, its dense
  // inverse entries are loaded a step ahead.  The same loads are issued
  // whatever the next step is (with no rows when it is a wave step, or past
  // the end), so the compiler's wait counts never cover a prefetch early.
  Slots<T> pre;
  DenseRow<T, NT> preD;
  auto prefetch = [&](const int4 nx, bool valid) {
    const bool use = valid && nx.z != 2;
    const Unit Un = use ? unit_at(s, nx.x) : Unit{0, 0, 0, 1, 0, 0, 0, false};
    pre = load_slots<T>(B, Un, 0, tid);
    const Unit Ud = (use && nx.z == 1) ? Un : Unit{0, 0, 0, 1, 0, 0, 0, false};
    preD = load_dense<T, NT>(s, (use && nx.z == 1) ? nx.w : 0, Ud, tid);
  };
  int4 st = step_at(s, 0);
  prefetch(st, true);
  for (int32_t k = 0; k < ns; ++k) {
    const int4 cur = st;
    const Slots<T> first = pre;
    const DenseRow<T, NT> dense = preD;
    if (k + 1 < ns) st = step_at(s, k + 1);
    if (cur.z == 2) {
      // wave step: the wave's units in order (see wave_walk_units); the next
      // step's prefetch is issued once the wave is done.
      // the wave index is uniform in a wave: tell the compiler, so that the
      // walk's control flow and descriptors stay scalar
      const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), l64 = tid & 63;
      const int32_t AS4 *wd = (const int32_t AS4 *)s.wdir;
      const int32_t u0 = wd[cur.x + wv], u1 = wd[cur.x + wv + 1];
      if constexpr (LDSX)
        wave_walk_c<C, T>(s, u0, u1, l64, X - kWavePadRows * C);
      else
        wave_walk<C, T, LDSX>(s, u0, u1, l64, X - kWavePadRows * C);
      prefetch(st, k + 1 < ns);
      step_barrier<LDSX>();
      if (ss && tid == 0 && k + 1 < kMaxStepStamps) ss[k + 1] = wall_clock64();
      continue;
    }
    // level or block step: the arithmetic, then the next step's prefetch
    // (issued after this step's own loads, so waiting for those never waits
    // for it), then the barrier
    const Unit U = unit_at(s, cur.x);
    const bool block = cur.z == 1;
    lane_update<C, T>(B, U, 0, tid, first, X, s_r, block);
    const int32_t passes = (U.rows + U.groups - 1) / U.groups;
    for (int32_t p = 1; p < passes; ++p)
      lane_update<C, T>(B, U, p, tid, load_slots<T>(B, U, p, tid), X, s_r, block);
    prefetch(st, k + 1 < ns);
    step_barrier<LDSX>();
    if (block) {
      dense_apply<C, NT, T>(U, dense, X, s_r, tid);
      step_barrier<LDSX>();
    }
    if (ss && tid == 0 && k + 1 < kMaxStepStamps) ss[k + 1] = wall_clock64();
  }
  __syncthreads();  // full barrier at the end of the sweep
}

// X <- D^{-1} X between the two sweeps of a solve, then a barrier.  A thread
// loads the pivots of several of its rows before it scales any of them (one
// row at a time, each row would wait a full load latency).
template <int C, int NT, class T>
__device__ __forceinline__ void pivot_scale(const T *__restrict__ d, T *__restrict__ X, int32_t n, int tid) {
  constexpr int kRows = C == 4 ? 4 : 8;  // fewer at four directions, where registers are tight
  for (int32_t b = tid; b < n; b += kRows * NT) {
    T v[kRows];
#pragma unroll
    for (int m = 0; m < kRows; ++m) v[m] = b + m * NT < n ? d[b + m * NT] : T(0);
#pragma unroll
    for (int m = 0; m < kRows; ++m) {
      const int32_t i = b + m * NT;
      if (i < n) {
#pragma unroll
        for (int c = 0; c < C; ++c) X[i * C + c] *= v[m];
      }
    }
  }
  __syncthreads();
}

// SpMul: B = -P G_p W into X (rows of C directions, FP64).
template <int C, int NT>
__device__ __forceinline__ void spmul(const NetDesc AS4 &nd, const WorkItem &a, double *__restrict__ X,
                                      int32_t dir0, int tid) {
  if (a.identity_from >= 0) {
    // W = columns of the identity: B is a column of G_p, negated, and -0 in
    // every other row (the values the row products give)
    for (int32_t i = tid; i < nd.n_x * C; i += NT) X[i] = -0.0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (dir0 + c >= a.k) continue;
      const int32_t q = a.identity_from + dir0 + c;
      for (int32_t e = nd.gpt_ptr[q] + tid; e < nd.gpt_ptr[q + 1]; e += NT) X[nd.gpt_col[e] * C + c] = -nd.gpt_val[e];
    }
    return;
  }
  // -0 in every row (what the product of a row without entries gives), then
  // the rows with entries, each from its record: most rows of G_p are empty,
  // and a thread's rows are chains of dependent loads
  for (int32_t i = tid; i < nd.n_x * C; i += NT) X[i] = -0.0;
  __syncthreads();
  for (int32_t j = tid; j < nd.n_gp_rows; j += NT) {
    const int4 r = nd.gp_rows[j];
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    for (int32_t e = r.y; e < r.z; ++e) {
      const double v = nd.gp_val[e];
      const int32_t q = nd.gp_col[e];
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = fma(v, w_at(a, q, dir0 + c), acc[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) X[r.x * C + c] = -acc[c];
  }
}

// The projection records through buffer resources: uniform byte offsets in
// scalar registers, the lane's offset in a vector register, and reads past
// the end return 0 (slots past a pass's slot count read at kOffRange).
struct ProjBufs {
  __amdgpu_buffer_rsrc_t bus, inc;
  int32_t bus_plane, inc_plane;  // plane sizes in bytes
};

__device__ __forceinline__ f64x2 proj_word(__amdgpu_buffer_rsrc_t r, int voff, int32_t soff) {
  return __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, __builtin_amdgcn_readfirstlane(soff), 0));
}

// Incidence slots e0 .. e0 + M - 1 of a lane in a projection pass.
template <int NT, int M>
__device__ __forceinline__ void proj_load_chunk(const ProjBufs &B, int2 pm, int32_t e0, int tid, f64x2 (&r0)[M],
                                                f64x2 (&r1)[M], f64x2 (&r2)[M]) {
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int32_t at = e0 + j < pm.y ? (pm.x + (e0 + j) * NT) * 16 : kOffRange;
    r0[j] = proj_word(B.inc, tid * 16, at);
    r1[j] = proj_word(B.inc, tid * 16, at + B.inc_plane);
    r2[j] = proj_word(B.inc, tid * 16, at + 2 * B.inc_plane);
  }
}

// Tensor projection (Sec. 4.2) with the state tangent Z: the slack-cost
// rank-one scalar, then per bus the branch second-order terms; the x part
// goes negated into Yx, the p part of the voltage parameters into the output
// (the generator parameters' 2 c2 w term is added by spmuladd).  Ends with a
// barrier.
template <int C, int NT>
__device__ __forceinline__ void projection(const NetDesc AS4 &nd, const WorkItem &a,
                                           const double *__restrict__ Z, double *__restrict__ Yx,
                                           double *s_slack, int32_t dir0, int tid) {
  // slack scalar: wave 0 evaluates 64 terms at a time, then every lane adds
  // them in order (the same sum as a serial loop)
  if (tid < 64) {
    double s[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = 0.0;
    for (int32_t q0 = 0; q0 < nd.n_slack; q0 += 64) {
      const int32_t q = q0 + tid;
      double term[C];
#pragma unroll
      for (int c = 0; c < C; ++c) term[c] = 0.0;
      if (q < nd.n_slack) {
        const int32_t tx = nd.slack_thx[q], vs = nd.slack_vs[q];
        const double gth = nd.slack_gth[q], gv = nd.slack_gv[q];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const double dth = tx >= 0 ? Z[tx * C + c] : 0.0;
          const double dv = vs >= 0 ? Z[vs * C + c] : w_at(a, -vs - 1, dir0 + c);
          term[c] = gth * dth + gv * dv;
        }
      }
      const int32_t m = min(64, nd.n_slack - q0);
      for (int32_t j = 0; j < m; ++j) {
#pragma unroll
        for (int c = 0; c < C; ++c) s[c] += __shfl(term[c], j);
      }
    }
    if (tid == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) s_slack[c] = s[c];
    }
  }
  __syncthreads();
  double sl[C];
#pragma unroll
  for (int c = 0; c < C; ++c) sl[c] = s_slack[c];
  constexpr int M = C == 1 ? 4 : 2;  // incidences whose loads are in flight together
  const int32_t AS4 *passes = (const int32_t AS4 *)nd.proj_pass;  // scalar loads
  ProjBufs B;
  B.bus_plane = nd.n_proj_pass * NT * 16;
  B.inc_plane = nd.proj_slots * 16;
  B.bus = __builtin_amdgcn_make_buffer_rsrc((void *)nd.proj_bus, 0, 2 * B.bus_plane, kBufWord3);
  B.inc = __builtin_amdgcn_make_buffer_rsrc((void *)nd.proj_inc, 0, 3 * B.inc_plane, kBufWord3);
  int2 pm_next = make_int2(0, 0);
  if (nd.n_proj_pass > 0) pm_next = make_int2(passes[0], passes[1]);
  for (int32_t p = 0; p < nd.n_proj_pass; ++p) {
    const int2 pm = pm_next;  // loaded a pass ahead
    if (p + 1 < nd.n_proj_pass) pm_next = make_int2(passes[2 * p + 2], passes[2 * p + 3]);
    // lanes past the last bus read padding records (tx = vs = -1, padded
    // incidences) and store nothing: no divergent exit, so the pass index
    // stays uniform
    const bool act = p * NT + tid < nd.n_bus;
    // every load of the bus and of its first M incidences is issued before
    // any of them is used
    const f64x2 b0 = proj_word(B.bus, tid * 16, p * NT * 16);
    const f64x2 b1 = proj_word(B.bus, tid * 16, p * NT * 16 + B.bus_plane);
    f64x2 r0[M], r1[M], r2[M];
    proj_load_chunk<NT, M>(B, pm, 0, tid, r0, r1, r2);
    const int32_t tx = __double2loint(b0.x), vs = __double2hiint(b0.x);
    const double ve = b0.y, sth = b1.x, sv = b1.y;
    double dte[C], dve[C], yth[C], yv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      dte[c] = tx >= 0 ? Z[tx * C + c] : 0.0;
      dve[c] = vs >= 0 ? Z[vs * C + c] : w_at(a, -vs - 1, dir0 + c);
      yth[c] = sth * sl[c];
      yv[c] = sv * sl[c];
    }
    for (int32_t e0 = 0;;) {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const int32_t ot = __double2loint(r2[j].y), ov = __double2hiint(r2[j].y);
        if (e0 + j >= pm.y || ot == kPadInc) continue;
        const double K = r0[j].x, Hps = r0[j].y, H = r1[j].x, A2 = r1[j].y, vo = r2[j].x;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const double dto = ot >= 0 ? Z[ot * C + c] : 0.0;
          const double dvo = ov >= 0 ? Z[ov * C + c] : w_at(a, -ov - 1, dir0 + c);
          const double dd = dte[c] - dto;
          yth[c] += -K * dd + Hps * (vo * dve[c] + ve * dvo);
          yv[c] += Hps * vo * dd + A2 * dve[c] + H * dvo;
        }
      }
      e0 += M;
      if (e0 >= pm.y) break;
      proj_load_chunk<NT, M>(B, pm, e0, tid, r0, r1, r2);
    }
    if (act) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (tx >= 0) Yx[tx * C + c] = -yth[c];
        if (vs >= 0)
          Yx[vs * C + c] = -yv[c];
        else if (dir0 + c < a.k)
          a.HW[(int64_t)(dir0 + c) * a.ldhw + (-vs - 1)] = yv[c];
      }
    }
  }
  __syncthreads();
}

// SpMulAdd: H W = Y_p + G_p^T Psi, Y_p of a generator parameter being its
// 2 c2 w term and that of a voltage parameter the projection's output.
template <int C, int NT>
__device__ __forceinline__ void spmuladd(const NetDesc AS4 &nd, const WorkItem &a,
                                         const double *__restrict__ Psi, int32_t dir0, int tid) {
  // A thread issues the loads of four entries of its row of G_p^T, and its
  // Y_p words, before it waits for any of them; the sum keeps entry order.
  for (int32_t q = tid; q < nd.n_p; q += NT) {
    const double c2x2 = nd.p_c2x2[q];
    double hv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) hv[c] = dir0 + c < a.k ? a.HW[(int64_t)(dir0 + c) * a.ldhw + q] : 0.0;
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    const int32_t e1 = nd.gpt_ptr[q + 1];
    for (int32_t e = nd.gpt_ptr[q]; e < e1; e += 4) {
      double v[4];
      int32_t j[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        v[m] = e + m < e1 ? nd.gpt_val[e + m] : 0.0;
        j[m] = e + m < e1 ? nd.gpt_col[e + m] * C : 0;
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (e + m < e1) {
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] = fma(v[m], Psi[j[m] + c], acc[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (dir0 + c >= a.k) continue;
      const double yp = __builtin_isnan(c2x2) ? hv[c] : __dmul_rn(c2x2, w_at(a, q, dir0 + c));
      a.HW[(int64_t)(dir0 + c) * a.ldhw + q] = yp + acc[c];
    }
  }
}

// dst[0 .. n) = src[0 .. n) with 16-byte accesses, eight per thread in flight
// (src and dst 16-byte aligned).
template <int NT>
__device__ __forceinline__ void copy_to_lds(const double *__restrict__ src, double *__restrict__ dst, int32_t n,
                                            int tid) {
  const int32_t n2 = n / 2;
  const double2 *s2 = reinterpret_cast<const double2 *>(src);
  double2 *d2 = reinterpret_cast<double2 *>(dst);
  for (int32_t b = 0; b < n2; b += 8 * NT) {
    double2 v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = b + m * NT + tid < n2 ? s2[b + m * NT + tid] : make_double2(0.0, 0.0);
#pragma unroll
    for (int m = 0; m < 8; ++m)
      if (b + m * NT + tid < n2) d2[b + m * NT + tid] = v[m];
  }
  if ((n & 1) && tid == 0) dst[n - 1] = src[n - 1];
}

template <int C, int NT, bool LDSX>
__device__ __forceinline__ void reduction(const NetDesc AS4 &nd, const WorkItem &a, double *__restrict__ X,
                                          double *__restrict__ Yx, double *s_slack, double *s_r,
                                          int32_t dir0, long long *stamps, long long *ss = nullptr) {
  const int tid = threadIdx.x;
  // optional phase timestamps (thread 0)
  long long *st = (stamps && tid == 0) ? stamps : nullptr;
  if (st) st[0] = wall_clock64();
  // 1. B' = -P G_p W
  spmul<C, NT>(nd, a, X, dir0, tid);
  __syncthreads();
  if (st) st[1] = wall_clock64();
  // 2. Z' = Uh^{-1} D^{-1} L^{-1} B'
  sweep<C, NT, double, LDSX>(nd.L, X, s_r, tid, ss);
  pivot_scale<C, NT, double>(nd.pivinv, X, nd.n_x, tid);
  if (st) st[2] = wall_clock64();
  sweep<C, NT, double, LDSX>(nd.U, X, s_r, tid, ss ? ss + kSweepStamps : nullptr);
  if (st) st[3] = wall_clock64();
  // 3. tensor projection: -Y_x into Yx, Y_p into the output
  projection<C, NT>(nd, a, X, Yx, s_slack, dir0, tid);
  if (st) st[4] = wall_clock64();
  // 4. Psi' = L^{-T} D^{-1} Uh^{-T} (-P Y_x), in place on the working vector
  // V: X in LDS takes a copy of -P Y_x (Z is no longer needed); with X in
  // global memory the solve runs on Yx itself (so Yx, like X, is the solution
  // part of a padded vector: the wave walk reads its zero row and writes its
  // dummy rows)
  double *V = X;
  if constexpr (LDSX) {
    copy_to_lds<NT>(Yx, X, nd.n_x * C, tid);
    __syncthreads();
  } else {
    V = Yx;
  }
  sweep<C, NT, double, LDSX>(nd.Ut, V, s_r, tid, ss ? ss + 2 * kSweepStamps : nullptr);
  pivot_scale<C, NT, double>(nd.pivinv, V, nd.n_x, tid);
  if (st) st[5] = wall_clock64();
  sweep<C, NT, double, LDSX>(nd.Lt, V, s_r, tid, ss ? ss + 3 * kSweepStamps : nullptr);
  if (st) st[6] = wall_clock64();
  // 5. H W = Y_p + G_p^T Psi
  spmuladd<C, NT>(nd, a, V, dir0, tid);
  __syncthreads();
  if (st) st[7] = wall_clock64();
}

// Workgroup maxima of two non-negative vectors of C values (s_red: kWaves *
// 2 C doubles); every thread receives them.  Ends with a barrier.
template <int C, int NT>
__device__ __forceinline__ void block_max2(double (&a)[C], double (&b)[C], double *s_red, int tid) {
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      a[c] = fmax(a[c], __shfl_xor(a[c], off));
      b[c] = fmax(b[c], __shfl_xor(b[c], off));
    }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      s_red[(tid >> 6) * 2 * C + c] = a[c];
      s_red[(tid >> 6) * 2 * C + C + c] = b[c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < C; ++c) {
    double ma = 0.0, mb = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      ma = fmax(ma, s_red[w * 2 * C + c]);
      mb = fmax(mb, s_red[w * 2 * C + C + c]);
    }
    a[c] = ma;
    b[c] = mb;
  }
  __syncthreads();
}

// One chunk of kEllChunk entries of a lane's row.
struct EllChunkRegs {
  int32_t col[kEllChunk];
  double val[kEllChunk];
};

__device__ __forceinline__ void ell_load(__amdgpu_buffer_rsrc_t bc, __amdgpu_buffer_rsrc_t bv, int32_t first,
                                         int tid, EllChunkRegs &r) {
#pragma unroll
  for (int e = 0; e < kEllChunk; ++e) {
    const int32_t slot = __builtin_amdgcn_readfirstlane(first + e * kThreads);
    r.col[e] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(bc, tid * 4, slot * 4, 0);
    r.val[e] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(bv, tid * 8, slot * 8, 0));
  }
}

// R <- R - A D for the directions with act[c] (rows of C directions; D is the
// FP32 correction just solved for, in LDS or global memory; R the FP64
// residual in global memory), and rmax[c] = max |R_i| over this thread's rows.
// The next chunk's loads are issued before the current one is used.  A row's
// products are summed in slot order, the same for every launch shape.
template <int C, int NT, class T32>
__device__ __forceinline__ void ell_residual(const EllMat AS4 &m, const T32 *__restrict__ D, double *__restrict__ R,
                                             const bool (&act)[C], double (&rmax)[C], int tid) {
  static_assert(NT == kThreads, "row passes are built for the kernel's workgroup");
  const int32_t n = m.n_chunks;
  if (n == 0) return;
  const __amdgpu_buffer_rsrc_t bc = __builtin_amdgcn_make_buffer_rsrc((void *)m.col, 0, m.n_slots * 4, kBufWord3);
  const __amdgpu_buffer_rsrc_t bv = __builtin_amdgcn_make_buffer_rsrc((void *)m.val, 0, m.n_slots * 8, kBufWord3);
  const int32_t AS4 *ch = (const int32_t AS4 *)m.chunks;  // scalar loads
  EllChunkRegs cur, nxt;
  int32_t c_first = ch[0], c_pass = ch[1], c_flags = ch[2];
  ell_load(bc, bv, c_first, tid, cur);
  int32_t row = -1;
  double rv[C], acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) rv[c] = acc[c] = 0.0;
  for (int32_t k = 0; k < n; ++k) {
    int32_t n_first = 0, n_pass = 0, n_flags = 0;
    if (k + 1 < n) {
      n_first = ch[4 * (k + 1)];
      n_pass = ch[4 * (k + 1) + 1];
      n_flags = ch[4 * (k + 1) + 2];
      ell_load(bc, bv, n_first, tid, nxt);
    }
    if (c_flags & 1) {  // first chunk of a pass: the lane's row and its residual
      row = m.rows[c_pass * NT + tid];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        acc[c] = 0.0;
        rv[c] = row >= 0 ? R[row * C + c] : 0.0;
      }
    }
#pragma unroll
    for (int e = 0; e < kEllChunk; ++e)
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = fma(cur.val[e], (double)D[cur.col[e] * C + c], acc[c]);
    if ((c_flags & 2) && row >= 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (!act[c]) continue;
        const double r = rv[c] - acc[c];
        R[row * C + c] = r;
        rmax[c] = fmax(rmax[c], fabs(r));
      }
    }
    cur = nxt;
    c_first = n_first;
    c_pass = n_pass;
    c_flags = n_flags;
  }
}

// Refined mode (FP32 sweeps, FP64 residuals).  Each of the two solves A x = b
// (A = G_x for Z, G_x^T for Psi) runs
//   d_0 = solve32(b), x = d_0, r = b - A d_0;
//   while the direction is not converged and fewer than `refine` corrections
//   were made:  d = solve32(r), x += d, r -= A d
// with x and r in FP64 (global memory) and A d formed in FP64 from the FP32
// correction d where it sits (LDS, or global memory).  A direction has
// converged once ||r||_inf <= tol ||A||_inf ||x||_inf; it then takes no further
// updates, so its result does not depend on the directions it shares the
// workgroup with.  berr[c] = ||r|| / (||A|| ||x||) of the final x, steps[c]
// the corrections made.  V1 holds b on entry (overwritten by r), V2 receives x.
template <int C, int NT, bool TRANS, bool LDSX>
__device__ __forceinline__ void refined_solve(const NetDesc AS4 &nd, double *__restrict__ V1,
                                              double *__restrict__ V2, float *__restrict__ X32,
                                              float *s_r, double *s_red, int refine, double tol, int tid,
                                              double (&berr)[C], int32_t (&steps)[C]) {
  const DevSweep AS4 &s1 = TRANS ? nd.Ut : nd.L;
  const DevSweep AS4 &s2 = TRANS ? nd.Lt : nd.U;
  const EllMat AS4 &A = TRANS ? nd.gxt : nd.gx;
  const int32_t n = nd.n_x;
  bool act[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    act[c] = true;
    steps[c] = 0;
    berr[c] = 0.0;
  }
  for (int it = 0;; ++it) {
    // right-hand side in FP32: b, then the residual
    for (int32_t i = tid; i < n; i += NT) {
#pragma unroll
      for (int c = 0; c < C; ++c) X32[i * C + c] = (float)V1[i * C + c];
    }
    __syncthreads();
    sweep<C, NT, float, LDSX>(s1, X32, s_r, tid);
    pivot_scale<C, NT, float>(nd.pivinv32, X32, n, tid);
    sweep<C, NT, float, LDSX>(s2, X32, s_r, tid);
    double xmax[C], rmax[C];
#pragma unroll
    for (int c = 0; c < C; ++c) xmax[c] = rmax[c] = 0.0;
    for (int32_t i = tid; i < n; i += NT) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (!act[c]) continue;
        const double x = (it ? V2[i * C + c] : 0.0) + (double)X32[i * C + c];
        V2[i * C + c] = x;
        xmax[c] = fmax(xmax[c], fabs(x));
      }
    }
    ell_residual<C, NT, float>(A, X32, V1, act, rmax, tid);
    block_max2<C, NT>(rmax, xmax, s_red, tid);
    bool any = false;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (!act[c]) continue;
      const double scale = A.norm * xmax[c];
      berr[c] = rmax[c] == 0.0 ? 0.0 : rmax[c] / scale;
      steps[c] = it;
      act[c] = !(rmax[c] <= tol * scale) && it < refine;
      any = any || act[c];
    }
    if (!any) break;
  }
}

template <int C, int NT, bool LDSX>
__device__ __forceinline__ void reduction_refined(const NetDesc AS4 &nd, const WorkItem &a,
                                                  float *__restrict__ X32, double *__restrict__ V1,
                                                  double *__restrict__ V2, double *s_slack, float *s_r,
                                                  double *s_red, int refine, double tol, int32_t dir0,
                                                  long long *stamps) {
  const int tid = threadIdx.x;
  long long *st = (stamps && tid == 0) ? stamps : nullptr;
  if (st) st[0] = wall_clock64();
  spmul<C, NT>(nd, a, V1, dir0, tid);
  __syncthreads();
  if (st) st[1] = wall_clock64();
  double bz[C], bp[C];
  int32_t kz[C], kp[C];
  refined_solve<C, NT, false, LDSX>(nd, V1, V2, X32, s_r, s_red, refine, tol, tid, bz, kz);  // Z
  if (st) st[2] = st[3] = wall_clock64();
  projection<C, NT>(nd, a, V2, V1, s_slack, dir0, tid);  // V1 = -Y_x
  if (st) st[4] = wall_clock64();
  refined_solve<C, NT, true, LDSX>(nd, V1, V2, X32, s_r, s_red, refine, tol, tid, bp, kp);  // Psi
  if (st) st[5] = st[6] = wall_clock64();
  spmuladd<C, NT>(nd, a, V2, dir0, tid);
  if (a.rinfo && tid == 0) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (dir0 + c >= a.k) continue;
      double *o = a.rinfo + 4 * (int64_t)(dir0 + c);
      o[0] = bz[c];
      o[1] = (double)kz[c];
      o[2] = bp[c];
      o[3] = (double)kp[c];
    }
  }
  __syncthreads();
  if (st) st[7] = wall_clock64();
}

// X in LDS, Y_x in global scratch.  The kernel uses dynamic LDS only, so
// that the padded vector (zero row, dummy rows, X; pad_rows x C doubles)
// starts at LDS address 0 as the wave walk assumes; the block residuals and
// the slack scalars follow it.
template <int C>
__global__ __launch_bounds__(kThreadsLds) void block_kernel_lds(const LaunchArgs la) {
  extern __shared__ double smem[];
  double *s_r = smem + (int64_t)la.pad_rows * C;
  double *s_slack = s_r + kBlockRows * C;
  double *X = smem + kWavePadRows * C;
  if (threadIdx.x < C) smem[threadIdx.x] = 0.0;  // the zero row (ordered by spmul's barrier)
  double *Yx = la.scratch + (int64_t)blockIdx.x * la.scratch_stride;
  for (int32_t chunk = blockIdx.x; chunk < la.n_chunks; chunk += gridDim.x) {
    const WorkItem it = item_of(la, chunk);
    long long *st = (la.stamps && chunk == (int32_t)blockIdx.x)
                        ? la.stamps + (int64_t)blockIdx.x * kStamps : nullptr;
    reduction<C, kThreadsLds, true>(*(const NetDesc AS4 *)it.nd, it, X, Yx, s_slack, s_r,
                                    (chunk - it.chunk0) * C, st,
                                    (blockIdx.x == 0 && chunk == 0) ? la.step_stamps : nullptr);
  }
}

// X and Y_x in global scratch (networks whose vector does not fit in LDS):
// padded Y_x (the transposed solve runs on it in place), then the padded X.
template <int C>
__global__ __launch_bounds__(kThreads) void block_kernel_global(const LaunchArgs la) {
  __shared__ double s_slack[C];
  __shared__ double s_r[kBlockRows * C];
  double *Ypad = la.scratch + (int64_t)blockIdx.x * la.scratch_stride;
  double *Xpad = Ypad + la.scratch_stride / 2;
  double *Yx = Ypad + kWavePadRows * C;
  double *X = Xpad + kWavePadRows * C;
  if (threadIdx.x < C) {  // the zero rows
    Ypad[threadIdx.x] = 0.0;
    Xpad[threadIdx.x] = 0.0;
  }
  for (int32_t chunk = blockIdx.x; chunk < la.n_chunks; chunk += gridDim.x) {
    const WorkItem it = item_of(la, chunk);
    long long *st = (la.stamps && chunk == (int32_t)blockIdx.x)
                        ? la.stamps + (int64_t)blockIdx.x * kStamps : nullptr;
    reduction<C, kThreads, false>(*(const NetDesc AS4 *)it.nd, it, X, Yx, s_slack, s_r,
                                  (chunk - it.chunk0) * C, st,
                                  (blockIdx.x == 0 && chunk == 0) ? la.step_stamps : nullptr);
  }
}

// Refined mode, padded FP32 correction vector at LDS address 0 (dynamic LDS
// only, as block_kernel_lds), then the block residuals, the slack scalars and
// the workgroup reduction buffer.
template <int C>
__global__ __launch_bounds__(kThreadsLds) void refined_kernel_lds(const LaunchArgs la) {
  extern __shared__ float smem32[];
  float *s_r = smem32 + (int64_t)la.pad_rows * C;
  double *s_slack = reinterpret_cast<double *>(smem32 + (((int64_t)la.pad_rows * C + kBlockRows * C + 1) & ~int64_t(1)));
  double *s_red = s_slack + C;
  float *X32 = smem32 + kWavePadRows * C;
  if (threadIdx.x < C) smem32[threadIdx.x] = 0.f;  // the zero row
  double *V1 = la.scratch + (int64_t)blockIdx.x * la.scratch_stride;
  double *V2 = V1 + la.scratch_stride / 2;
  for (int32_t chunk = blockIdx.x; chunk < la.n_chunks; chunk += gridDim.x) {
    const WorkItem it = item_of(la, chunk);
    long long *st = (la.stamps && chunk == (int32_t)blockIdx.x)
                        ? la.stamps + (int64_t)blockIdx.x * kStamps : nullptr;
    reduction_refined<C, kThreadsLds, true>(*(const NetDesc AS4 *)it.nd, it, X32, V1, V2, s_slack, s_r, s_red,
                                            la.refine, la.refine_tol, (chunk - it.chunk0) * C, st);
  }
}

// Refined mode with every vector in global scratch: V1, V2, the padded FP32
// correction.
template <int C>
__global__ __launch_bounds__(kThreads) void refined_kernel_global(const LaunchArgs la) {
  __shared__ double s_slack[C];
  __shared__ float s_r[kBlockRows * C];
  __shared__ double s_red[kWaves * 2 * C];
  double *V1 = la.scratch + (int64_t)blockIdx.x * la.scratch_stride;
  double *V2 = V1 + la.scratch_stride / 3;
  float *X32pad = reinterpret_cast<float *>(V1 + 2 * (la.scratch_stride / 3));
  float *X32 = X32pad + kWavePadRows * C;
  if (threadIdx.x < C) X32pad[threadIdx.x] = 0.f;  // the zero row
  for (int32_t chunk = blockIdx.x; chunk < la.n_chunks; chunk += gridDim.x) {
    const WorkItem it = item_of(la, chunk);
    long long *st = (la.stamps && chunk == (int32_t)blockIdx.x)
                        ? la.stamps + (int64_t)blockIdx.x * kStamps : nullptr;
    reduction_refined<C, kThreads, false>(*(const NetDesc AS4 *)it.nd, it, X32, V1, V2, s_slack, s_r, s_red,
                                          la.refine, la.refine_tol, (chunk - it.chunk0) * C, st);
  }
}

}  // namespace

// ----------------------------------------------------------------- runtime
namespace {

#define HIP_TRY(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
      return RH_EDEVICE;                                                       \
    }                                                                          \
  } while (0)

struct DeviceInfo {
  int device = -1;
  int cus = 0;
  size_t lds_max = 0;  // dynamic LDS a workgroup may use
  double wall_khz = 0.0;
};

// Launch resources: per-workgroup scratch, timing events, phase stamps and the
// device copy of a work list.  A network owns one (its own calls); a context
// owns one for batched calls.
struct Runner {
  double *scratch = nullptr;
  size_t scratch_bytes = 0;
  std::vector<hipEvent_t> ev;  // start/stop pairs of the launches since the last report
  size_t ev_used = 0;
  long long *stamps = nullptr;
  int32_t stamps_cap = 0, stamps_groups = 0;
  WorkItem *items_dev = nullptr, *items_host = nullptr;
  int32_t items_cap = 0;
  hipEvent_t items_done = nullptr;  // the last launch that read the work list
  int32_t launches = 0, last_c = 0;
  long long *step_stamps = nullptr;  // debug (RH_STEP_STAMPS)
  bool step_stamps_pending = false;
};

rh_status query_info(int device, DeviceInfo &info, std::string &err) {
  int cus = 0, lds_a = 0, lds_b = 0, wkhz = 0;
  HIP_TRY(hipDeviceGetAttribute(&wkhz, hipDeviceAttributeWallClockRate, device));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  HIP_TRY(hipDeviceGetAttribute(&lds_a, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
  HIP_TRY(hipDeviceGetAttribute(&lds_b, hipDeviceAttributeSharedMemPerBlockOptin, device));
  info.device = device;
  info.cus = cus;
  info.wall_khz = wkhz;
  // leave room for the kernels' static LDS (slack scalars and block residuals)
  const size_t lds = (size_t)std::max(lds_a, lds_b);
  const size_t fixed = (size_t)kBlockRows * 8 * sizeof(double) + (size_t)kWaves * 8 * sizeof(double) + 256;
  info.lds_max = lds > fixed ? lds - fixed : 0;
  return RH_OK;
}

void runner_free(Runner &r) {
  if (r.scratch) (void)hipFree(r.scratch);
  for (hipEvent_t e : r.ev) (void)hipEventDestroy(e);
  if (r.stamps) (void)hipFree(r.stamps);
  if (r.items_dev) (void)hipFree(r.items_dev);
  if (r.items_host) (void)hipHostFree(r.items_host);
  if (r.items_done) (void)hipEventDestroy(r.items_done);
  if (r.step_stamps) (void)hipFree(r.step_stamps);
  r = Runner();
}

// Summed launch durations (and mean phase times) since the previous call.
rh_status runner_collect(Runner &r, const DeviceInfo &info, rh_report &rep, std::string &err) {
  rep.last_kernel_ms = -1.0;
  rep.last_launches = r.launches;
  rep.dirs_per_group = r.last_c;
  if (r.stamps_groups > 0 && info.wall_khz > 0) {
    std::vector<long long> st((size_t)r.stamps_groups * kStamps);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(st.data(), r.stamps, st.size() * sizeof(long long), hipMemcpyDeviceToHost));
    for (int p = 0; p < 7; ++p) {
      double sum = 0.0;
      for (int32_t g = 0; g < r.stamps_groups; ++g)
        sum += (double)(st[(size_t)g * kStamps + p + 1] - st[(size_t)g * kStamps + p]);
      rep.phase_us[p] = sum / r.stamps_groups / info.wall_khz * 1e3;
    }
    r.stamps_groups = 0;
  }
  if (r.step_stamps_pending && info.wall_khz > 0) {
    std::vector<long long> st(4 * kSweepStamps);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(st.data(), r.step_stamps, st.size() * sizeof(long long), hipMemcpyDeviceToHost));
    const char *nm[4] = {"L", "U", "Ut", "Lt"};
    const double us = 1e3 / info.wall_khz;
    for (int w = 0; w < 4; ++w) {
      const long long *S = st.data() + (size_t)w * kSweepStamps;
      fprintf(stderr, "steps %s (us):", nm[w]);
      for (int k = 1; k < kMaxStepStamps && S[k] != 0; ++k) fprintf(stderr, " %.2f", (S[k] - S[k - 1]) * us);
      fprintf(stderr, "\n");
    }
    r.step_stamps_pending = false;
  }
  if (r.ev_used > 0) {
    double sum = 0.0;
    for (size_t i = 0; i + 1 < r.ev_used; i += 2) {
      HIP_TRY(hipEventSynchronize(r.ev[i + 1]));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, r.ev[i], r.ev[i + 1]));
      sum += ms;
    }
    rep.last_kernel_ms = sum;
  }
  r.ev_used = 0;
  r.launches = 0;
  return RH_OK;
}

// The LDS kernels address the padded vector from LDS address 0, which holds
// only if they have no static LDS (checked once per kernel; threads that
// race to check it store the same answer).
rh_status no_static_lds(const void *kernel, std::atomic<int> &checked, std::string &err) {
  if (checked.load() == 0) {
    hipFuncAttributes fa{};
    HIP_TRY(hipFuncGetAttributes(&fa, kernel));
    checked.store(fa.sharedSizeBytes == 0 ? 1 : -1);
  }
  if (checked.load() < 0) {
    err = "internal: an LDS kernel has static LDS";
    return RH_EDEVICE;
  }
  return RH_OK;
}

std::mutex g_lds_mu;
std::map<std::pair<int, const void *>, size_t> g_lds_bound;

}  // namespace

rh_status lds_bound(const void *kernel, size_t bytes, std::string &err) {
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  std::lock_guard<std::mutex> lock(g_lds_mu);
  size_t &b = g_lds_bound[{device, kernel}];
  if (bytes > b) {
    HIP_TRY(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    b = bytes;
  }
  return RH_OK;
}

namespace {

// Launch the kernel for C directions per workgroup.  The per-kernel attribute
// calls come first; a launch recorded into a graph makes them beforehand
// (mode kAttrsOnly) and records the launch alone (kLaunchOnly).
enum LaunchMode { kAttrsAndLaunch, kAttrsOnly, kLaunchOnly };

template <int C>
rh_status launch(bool lds, bool refined, int32_t groups, size_t lds_bytes, hipStream_t s,
                 const LaunchArgs &la, std::string &err, LaunchMode mode = kAttrsAndLaunch) {
  static std::atomic<int> checked_b{0}, checked_r{0};
  const bool attrs = mode != kLaunchOnly;
  if (mode == kAttrsOnly) {
    if (!lds) return RH_OK;
    if constexpr (C <= 4) {
      const void *k = refined ? reinterpret_cast<const void *>(&refined_kernel_lds<C>)
                              : reinterpret_cast<const void *>(&block_kernel_lds<C>);
      rh_status st = no_static_lds(k, refined ? checked_r : checked_b, err);
      if (st != RH_OK) return st;
      st = lds_bound(k, lds_bytes, err);
      if (st != RH_OK) return st;
    }
    return RH_OK;
  }
  if (refined) {
    if constexpr (C <= 4) {
      if (lds) {
        if (attrs) {
          rh_status st = no_static_lds(reinterpret_cast<const void *>(&refined_kernel_lds<C>), checked_r, err);
          if (st != RH_OK) return st;
          st = lds_bound(reinterpret_cast<const void *>(&refined_kernel_lds<C>), lds_bytes, err);
          if (st != RH_OK) return st;
        }
        hipLaunchKernelGGL(refined_kernel_lds<C>, dim3(groups), dim3(kThreadsLds), lds_bytes, s, la);
        HIP_TRY(hipGetLastError());
        return RH_OK;
      }
    }
    hipLaunchKernelGGL(refined_kernel_global<C>, dim3(groups), dim3(kThreads), 0, s, la);
    HIP_TRY(hipGetLastError());
    return RH_OK;
  }
  if constexpr (C <= 4) {
    if (lds) {
      if (attrs) {
        rh_status st = no_static_lds(reinterpret_cast<const void *>(&block_kernel_lds<C>), checked_b, err);
        if (st != RH_OK) return st;
        st = lds_bound(reinterpret_cast<const void *>(&block_kernel_lds<C>), lds_bytes, err);
        if (st != RH_OK) return st;
      }
      hipLaunchKernelGGL(block_kernel_lds<C>, dim3(groups), dim3(kThreadsLds), lds_bytes, s, la);
      HIP_TRY(hipGetLastError());
      return RH_OK;
    }
  }
  hipLaunchKernelGGL(block_kernel_global<C>, dim3(groups), dim3(kThreads), 0, s, la);
  HIP_TRY(hipGetLastError());
  return RH_OK;
}

// Directions per workgroup: more share each record load, fewer keep the chip
// busy.  Every kernel runs one 1,024-thread workgroup per CU (its registers
// allow no second one), so take the largest C that still gives every CU a
// workgroup and whose vectors fit the LDS budget.  The choice does not change
// any direction's arithmetic.
int32_t lds_max_c(int64_t n_x, size_t lds_max, bool lds, size_t elem) {
  int32_t c = 4;  // the largest group the kernels are instantiated for
  while (c > 1 && lds && (size_t)n_x * c * elem > lds_max) c >>= 1;
  return c;
}

// force: a count chosen by the tuner (0: none), taken when it fits.
int32_t choose_c(int64_t k, int32_t cus, int64_t n_x, size_t lds_max, bool lds, size_t elem, int32_t force = 0) {
  if (const char *e = std::getenv("RH_DIRS_PER_GROUP")) {
    const int v = std::atoi(e);
    if ((v == 1 || v == 2 || v == 4) && (!lds || (size_t)n_x * v * elem <= lds_max))
      return v;
  }
  if ((force == 1 || force == 2 || force == 4) && (!lds || (size_t)n_x * force * elem <= lds_max)) return force;
  int32_t c = lds_max_c(n_x, lds_max, lds, elem);
  while (c > 1 && k < (int64_t)c * cus) c >>= 1;
  return c;
}

// Launch the reduction over a list of work items (host copies; their nd
// pointers are device descriptors).  max_nx is the largest n_x among them.
// A caller-independent scratch range (the fixed array of the allocation-free
// entry point): the launch runs at most bytes / (workgroup scratch) workgroups
// and records no timing.
struct FixedScratch {
  double *ptr;
  int64_t bytes;
};

// Shape of one batched launch: directions per workgroup, where the working
// vector lives, workgroups and their scratch, dynamic LDS.  Sets the items'
// first chunks.
struct LaunchPlan {
  bool refined = false, lds = false;
  int32_t C = 1, pad_rows = 0, groups = 0;
  int64_t n_chunks = 0, stride = 0;  // stride: doubles of scratch per workgroup
  size_t lds_bytes = 0;
};

rh_status plan_launch(const DeviceInfo &info, int32_t refine, std::vector<WorkItem> &items, int32_t max_nx,
                      LaunchPlan &pl, std::string &err, int32_t force_c = 0) {
  int64_t total_k = 0;
  for (const WorkItem &it : items) total_k += it.k;
  pl = LaunchPlan();
  if (total_k <= 0) return RH_OK;
  pl.refined = refine >= 0;
  const size_t elem = pl.refined ? sizeof(float) : sizeof(double);  // LDS vector element
  pl.pad_rows = max_nx + kWavePadRows;                               // padded working vector
  // X in LDS also means compact wave records (rows as 16-bit indices)
  pl.lds = (size_t)pl.pad_rows * elem <= info.lds_max && pl.pad_rows <= 65536 && !std::getenv("RH_NO_LDS");
  const int32_t C = pl.C = choose_c(total_k, info.cus, pl.pad_rows, info.lds_max, pl.lds, elem, force_c);
  for (WorkItem &it : items) {
    it.chunk0 = (int32_t)pl.n_chunks;
    pl.n_chunks += (it.k + C - 1) / C;
  }
  if (pl.n_chunks > INT32_MAX) {
    err = "too many directions in one launch";
    return RH_EINVAL;
  }
  // per-workgroup scratch, 256-byte aligned: FP64 mode Y_x (+ X when it is
  // not in LDS); refined mode V1, V2 (+ the FP32 correction when not in LDS)
  const int64_t parts = pl.refined ? (pl.lds ? 2 : 3) : (pl.lds ? 1 : 2);
  pl.stride = (parts * (int64_t)pl.pad_rows * C + 31) / 32 * 32;
  const int64_t max_groups_mem = std::max<int64_t>(1, (int64_t(8) << 30) / (pl.stride * 8));
  const int64_t per_cu = pl.lds ? 1 : 2;
  pl.groups = (int32_t)std::min<int64_t>({pl.n_chunks, max_groups_mem, (int64_t)info.cus * 8 * per_cu});
  // dynamic LDS: the padded vector, then the kernels' small buffers (block
  // residuals, slack scalars; the refined kernel's reduction buffer)
  if (pl.lds) {
    if (pl.refined)
      pl.lds_bytes = (((size_t)pl.pad_rows * C + kBlockRows * C + 1) & ~size_t(1)) * sizeof(float) +
                     (size_t)(C + kWaves * 2 * C) * sizeof(double);
    else
      pl.lds_bytes = ((size_t)pl.pad_rows * C + kBlockRows * C + C) * sizeof(double);
  }
  return RH_OK;
}

rh_status launch_plan(const LaunchPlan &pl, int32_t groups, hipStream_t s, const LaunchArgs &la, std::string &err,
                      LaunchMode mode = kAttrsAndLaunch) {
  switch (pl.C) {
    case 1: return launch<1>(pl.lds, pl.refined, groups, pl.lds_bytes, s, la, err, mode);
    case 2: return launch<2>(pl.lds, pl.refined, groups, pl.lds_bytes, s, la, err, mode);
    case 4: return launch<4>(pl.lds, pl.refined, groups, pl.lds_bytes, s, la, err, mode);
    default:
      err = "internal: no kernel for " + std::to_string(pl.C) + " directions per workgroup";
      return RH_EDEVICE;
  }
}

rh_status run_items(const DeviceInfo &info, Runner &r, int32_t timing, int32_t refine, double refine_tol,
                    std::vector<WorkItem> &items, int32_t max_nx, hipStream_t s, std::string &err,
                    const FixedScratch *fixed = nullptr, int32_t force_c = 0) {
  LaunchPlan pl;
  rh_status ps = plan_launch(info, refine, items, max_nx, pl, err, force_c);
  if (ps != RH_OK || pl.n_chunks == 0) return ps;
  const int32_t C = pl.C;
  const int64_t n_chunks = pl.n_chunks, stride = pl.stride;
  const int32_t pad_rows = pl.pad_rows;
  int32_t groups = pl.groups;
  if (fixed) {
    // workgroups take further chunks in turn when the fixed range is short
    const int64_t fit = fixed->bytes / (stride * (int64_t)sizeof(double));
    if (fit < 1) {
      err = "network too large for the fixed scratch: one workgroup needs " +
            std::to_string(stride * (int64_t)sizeof(double)) + " bytes, " + std::to_string(fixed->bytes) +
            " available";
      return RH_EINVAL;
    }
    if (items.size() != 1) {
      err = "internal: the fixed scratch takes one work item";
      return RH_EDEVICE;
    }
    groups = (int32_t)std::min<int64_t>(groups, fit);
    timing = 0;
  }
  const size_t need = (size_t)groups * stride * sizeof(double);
  if (!fixed && need > r.scratch_bytes) {
    HIP_TRY(hipStreamSynchronize(s));  // earlier work on this stream may still use it
    if (r.scratch) HIP_TRY(hipFree(r.scratch));
    r.scratch = nullptr;
    r.scratch_bytes = 0;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, need));
    r.scratch = (double *)p;
    r.scratch_bytes = need;
  }
  LaunchArgs la{};
  la.refine = refine;
  la.refine_tol = refine_tol;
  la.n_items = (int32_t)items.size();
  la.n_chunks = (int32_t)n_chunks;
  la.scratch = fixed ? fixed->ptr : r.scratch;
  la.scratch_stride = stride;
  la.pad_rows = pad_rows;
  if (items.size() == 1) {
    la.items = nullptr;
    la.one = items[0];
  } else {
    if ((int32_t)items.size() > r.items_cap) {
      HIP_TRY(hipStreamSynchronize(s));
      if (r.items_dev) HIP_TRY(hipFree(r.items_dev));
      if (r.items_host) HIP_TRY(hipHostFree(r.items_host));
      r.items_dev = r.items_host = nullptr;
      r.items_cap = 0;
      HIP_TRY(hipMalloc(&r.items_dev, items.size() * sizeof(WorkItem)));
      HIP_TRY(hipHostMalloc(&r.items_host, items.size() * sizeof(WorkItem), hipHostMallocDefault));
      r.items_cap = (int32_t)items.size();
    }
    if (!r.items_done) HIP_TRY(hipEventCreateWithFlags(&r.items_done, hipEventDisableTiming));
    HIP_TRY(hipEventSynchronize(r.items_done));  // the previous list is no longer read
    std::memcpy(r.items_host, items.data(), items.size() * sizeof(WorkItem));
    HIP_TRY(hipMemcpyAsync(r.items_dev, r.items_host, items.size() * sizeof(WorkItem),
                           hipMemcpyHostToDevice, s));
    la.items = r.items_dev;
  }
  la.step_stamps = nullptr;
  if (!fixed && std::getenv("RH_STEP_STAMPS")) {
    if (!r.step_stamps) HIP_TRY(hipMalloc(&r.step_stamps, 4 * kSweepStamps * sizeof(long long)));
    HIP_TRY(hipMemsetAsync(r.step_stamps, 0, 4 * kSweepStamps * sizeof(long long), s));
    la.step_stamps = r.step_stamps;
    r.step_stamps_pending = true;
  }
  la.stamps = nullptr;
  if (timing >= 2) {
    if (r.stamps_cap < groups) {
      HIP_TRY(hipStreamSynchronize(s));
      if (r.stamps) HIP_TRY(hipFree(r.stamps));
      r.stamps = nullptr;
      r.stamps_cap = 0;
      HIP_TRY(hipMalloc(&r.stamps, (size_t)groups * kStamps * sizeof(long long)));
      r.stamps_cap = groups;
    }
    la.stamps = r.stamps;
    r.stamps_groups = groups;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timing >= 1) {
    while (r.ev.size() < r.ev_used + 2) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      r.ev.push_back(e);
    }
    e0 = r.ev[r.ev_used];
    e1 = r.ev[r.ev_used + 1];
    r.ev_used += 2;
    HIP_TRY(hipEventRecord(e0, s));
  }
  const rh_status st = launch_plan(pl, groups, s, la, err);
  if (st != RH_OK) return st;
  if (items.size() > 1) HIP_TRY(hipEventRecord(r.items_done, s));
  if (timing >= 1) HIP_TRY(hipEventRecord(e1, s));
  r.launches += 1;
  r.last_c = C;
  return RH_OK;
}

}  // namespace

struct DeviceNet {
  std::vector<int32_t> sweep_steps;  // barrier steps of the L, U, U^T, L^T sweeps
  std::mutex up_mu;                  // allocs and bytes, while the upload's threads add to them
  double *rinfo = nullptr;           // per-column refinement figures (4 doubles per column)
  int64_t rinfo_cols = 0;
  int64_t bytes = 0;                 // device bytes of the network's own arrays (allocs)
  NetDesc nd{};               // host copy of the descriptor (device pointers)
  NetDesc *nd_dev = nullptr;  // the same descriptor in device memory
  std::vector<void *> allocs;
  std::vector<size_t> alloc_bytes;  // size of each of allocs
  // the previous operating point's allocations while this one is uploaded:
  // the layout depends on the pattern only, so the sizes repeat and each
  // array takes a block of its size instead of a new allocation (the rest
  // is freed at the end of the upload)
  std::multimap<size_t, void *> pool;
  DeviceInfo info;
  Runner run;
};

// A context's resources for batched launches: one runner per stream, since
// launches on one stream are ordered and may share scratch, while launches on
// different streams may overlap.
struct DeviceCtx {
  DeviceInfo info;
  std::vector<std::pair<void *, Runner>> runs;
  Runner &on(void *stream) {
    for (auto &pr : runs)
      if (pr.first == stream) return pr.second;
    runs.emplace_back(stream, Runner());
    return runs.back().second;
  }
};

namespace {

template <class T>
rh_status upload(DeviceNet &dn, const std::vector<T> &v, const T **out, std::string &err) {
  if (v.empty()) {
    *out = nullptr;
    return RH_OK;
  }
  const size_t nb = v.size() * sizeof(T);
  void *p = nullptr;
  {
    std::lock_guard<std::mutex> lk(dn.up_mu);
    auto it = dn.pool.find(nb);
    if (it != dn.pool.end()) {
      p = it->second;
      dn.pool.erase(it);
    }
  }
  if (!p) HIP_TRY(hipMalloc(&p, nb));
  {
    std::lock_guard<std::mutex> lk(dn.up_mu);
    dn.allocs.push_back(p);
    dn.alloc_bytes.push_back(nb);
    dn.bytes += (int64_t)nb;
  }
  HIP_TRY(hipMemcpy(p, v.data(), nb, hipMemcpyHostToDevice));
  *out = static_cast<const T *>(p);
  return RH_OK;
}

#define UP(vec, dst)                                            \
  do {                                                          \
    rh_status s_ = upload(*dn, vec, &(dst), err);               \
    if (s_ != RH_OK) return s_;                                 \
  } while (0)

// Arrays appended to one host staging buffer at 256-byte aligned offsets and
// uploaded as one allocation.
struct Blob {
  std::vector<char> h;
  template <class T>
  int64_t add(const std::vector<T> &v) {
    if (v.empty()) return -1;
    const size_t off = (h.size() + 255) & ~size_t(255);
    h.resize(off + v.size() * sizeof(T));
    std::memcpy(h.data() + off, v.data(), v.size() * sizeof(T));
    return (int64_t)off;
  }
};

template <class T>
const T *at_off(const char *base, int64_t off) {
  return off < 0 ? nullptr : reinterpret_cast<const T *>(base + off);
}

// Host arrays of one sweep's packing: the packed schedule, the four record
// layouts, FP32 copies and the staging buffer.  They are taken from a
// process-wide pool and given back after the upload, so that the next
// upload (the next operating point) fills memory that is already mapped
// instead of faulting in fresh pages; a scratch above kScratchKeep bytes
// is freed instead of kept.
struct SweepScratch {
  Packed pk;
  std::vector<char> rec[4];
  std::vector<float> f32;
  Blob bl;
  size_t bytes() const {
    size_t b = bl.h.capacity() + f32.capacity() * sizeof(float);
    for (const std::vector<char> &r : rec) b += r.capacity();
    for (const std::vector<int32_t> *v : {&pk.steps, &pk.units, &pk.wdir, &pk.scol, &pk.irow, &pk.wlg, &pk.wcol,
                                          &pk.wrow})
      b += v->capacity() * sizeof(int32_t);
    for (const std::vector<double> *v : {&pk.sval, &pk.idinv, &pk.dense, &pk.wval}) b += v->capacity() * sizeof(double);
    return b;
  }
};

// The factors' four sweeps and lu_sweeps' work arrays, pooled the same way.
struct SweepsScratch {
  Sweep sw[4];
  LuSweepsWork lw;
  std::vector<double> pivinv;
  std::vector<float> p32;
  size_t bytes() const {
    size_t b = pivinv.capacity() * sizeof(double) + p32.capacity() * sizeof(float);
    for (const Sweep &s : sw)
      b += (s.lev_ptr.capacity() + s.rows.capacity() + s.ptr.capacity() + s.col.capacity()) * sizeof(int32_t) +
           (s.val.capacity() + s.dinv.capacity()) * sizeof(double);
    for (const std::vector<int32_t> *v : {&lw.tp, &lw.lp, &lw.tc, &lw.lc, &lw.tf, &lw.lf})
      b += v->capacity() * sizeof(int32_t);
    return b + (lw.tv.capacity() + lw.lv.capacity()) * sizeof(double);
  }
};

constexpr size_t kScratchKeep = size_t(256) << 20;
constexpr size_t kScratchPool = 16;

template <class T>
struct ScratchPool {
  std::mutex mu;
  std::vector<std::unique_ptr<T>> free;
  std::unique_ptr<T> take() {
    std::lock_guard<std::mutex> lock(mu);
    if (free.empty()) return std::make_unique<T>();
    std::unique_ptr<T> w = std::move(free.back());
    free.pop_back();
    return w;
  }
  void give(std::unique_ptr<T> w) {
    if (!w || w->bytes() > kScratchKeep) return;
    std::lock_guard<std::mutex> lock(mu);
    if (free.size() < kScratchPool) free.push_back(std::move(w));
  }
};
ScratchPool<SweepScratch> g_sweep_scratch;
ScratchPool<SweepsScratch> g_sweeps_scratch;

// One sweep in one allocation: the layout and entry columns first (read in
// both precisions), then the FP64 values and block inverses, then their FP32
// copies, so that each precision's working set is two contiguous ranges.
// The host part (schedule, packing, records) is prepare_sweep, which touches
// nothing shared, so the four sweeps of a network are prepared on threads of
// their own; commit_sweep uploads.
struct SweepHost {
  SweepScratch *ws = nullptr;
  int64_t o_steps = -1, o_units = -1, o_wdir = -1, o_scol = -1, o_irow = -1, o_sval = -1, o_dense = -1,
          o_wrec = -1, o_sval32 = -1, o_dense32 = -1, o_wrec32 = -1, o_wrecc = -1, o_wrecc32 = -1;
  bool compact = false;
  int32_t n_steps = 0, n_wunits = 0, n_slots = 0, n_irow = 0;
  rh_status st = RH_OK;
  std::string err;
};

void prepare_sweep(const Sweep &s, int32_t n, const std::vector<int32_t> &parent, bool forward,
                   const ScheduleParams &prm, ScheduleCut *cut, SweepHost &h) {
  const Schedule sc = build_schedule(s, n, parent, forward, prm, cut);
  Packed &pk = h.ws->pk;
  pack_schedule(sc, kThreads, pk);
  if (pk.irow.empty()) pk.irow.push_back(0);  // lanes without a row read element 0
  if (!pk.idinv.empty()) {
    h.st = RH_EDEVICE;
    h.err = "internal: device sweeps must have a unit diagonal";
    return;
  }
  // wave-unit records in both precisions, wide and (where the rows fit)
  // compact (layouts: see wave_records)
  const size_t nwu = pk.wlg.size();
  if (nwu * WaveRec<double>::bytes >= (size_t)kOffRange) {
    h.st = RH_EINVAL;
    h.err = "network too large for the wave-unit records";
    return;
  }
  // the four layouts are independent: three of them on threads of their own
  std::vector<char> &rec64 = h.ws->rec[0], &rec32 = h.ws->rec[1], &recc64 = h.ws->rec[2], &recc32 = h.ws->rec[3];
  bool ok64 = false, ok32 = false;
  std::exception_ptr ex[3];
  auto guarded = [&](int k, bool compact, bool fp64, std::vector<char> &out, bool *ok) {
    return std::thread([&, k, compact, fp64, ok] {
      try {
        const bool r = wave_records(pk, compact, fp64, out);
        if (ok) *ok = r;
      } catch (...) {
        ex[k] = std::current_exception();
      }
    });
  };
  std::thread t0 = guarded(0, false, false, rec32, nullptr);
  std::thread t1 = guarded(1, true, true, recc64, &ok64);
  std::thread t2 = guarded(2, true, false, recc32, &ok32);
  (void)wave_records(pk, false, true, rec64);
  t0.join();
  t1.join();
  t2.join();
  for (const std::exception_ptr &e : ex)
    if (e) std::rethrow_exception(e);
  h.compact = ok64 && ok32;
  Blob &bl = h.ws->bl;
  bl.h.clear();
  std::vector<float> &f32 = h.ws->f32;
  h.o_steps = bl.add(pk.steps);
  h.o_units = bl.add(pk.units);
  h.o_wdir = bl.add(pk.wdir);
  h.o_scol = bl.add(pk.scol);
  h.o_irow = bl.add(pk.irow);
  h.o_sval = bl.add(pk.sval);
  h.o_dense = bl.add(pk.dense);
  h.o_wrec = bl.add(rec64);
  f32.assign(pk.sval.begin(), pk.sval.end());
  h.o_sval32 = bl.add(f32);
  f32.assign(pk.dense.begin(), pk.dense.end());
  h.o_dense32 = bl.add(f32);
  h.o_wrec32 = bl.add(rec32);
  h.o_wrecc = h.compact ? bl.add(recc64) : -1;
  h.o_wrecc32 = h.compact ? bl.add(recc32) : -1;
  h.n_steps = (int32_t)(pk.steps.size() / 4);
  h.n_wunits = (int32_t)nwu;
  h.n_slots = (int32_t)pk.scol.size();
  h.n_irow = (int32_t)pk.irow.size();
}

rh_status commit_sweep(DeviceNet *dn, const SweepHost &h, DevSweep &o, std::string &err) {
  if (h.st != RH_OK) {
    err = h.err;
    return h.st;
  }
  const char *base = nullptr;
  UP(h.ws->bl.h, base);
  o.n_steps = h.n_steps;
  o.steps = at_off<int4>(base, h.o_steps);
  o.units = at_off<int4>(base, h.o_units);
  o.wdir = at_off<int32_t>(base, h.o_wdir);
  o.scol = at_off<int32_t>(base, h.o_scol);
  o.irow = at_off<int32_t>(base, h.o_irow);
  o.sval = at_off<double>(base, h.o_sval);
  o.dense = at_off<double>(base, h.o_dense);
  o.sval32 = at_off<float>(base, h.o_sval32);
  o.dense32 = at_off<float>(base, h.o_dense32);
  o.n_wunits = h.n_wunits;
  o.wrec = at_off<char>(base, h.o_wrec);
  o.wrec32 = at_off<char>(base, h.o_wrec32);
  o.wrecc = h.compact ? at_off<char>(base, h.o_wrecc) : nullptr;
  o.wrecc32 = h.compact ? at_off<char>(base, h.o_wrecc32) : nullptr;
  o.n_slots = h.n_slots;
  o.n_irow = h.n_irow;
  return RH_OK;
}

// The four sweeps (L, U, U^T, L^T), each prepared and uploaded on a thread of
// its own (the device is current per thread).  An exception on a thread is
// raised again here.
rh_status upload_sweeps(DeviceNet *dn, int device, const Sweep *const sw[4], int32_t n,
                        const std::vector<int32_t> &parent, const ScheduleParams &prm, DevSweep *const out[4],
                        ScheduleCut *cuts, std::string &err) {
  SweepHost hs[4];
  std::unique_ptr<SweepScratch> ws[4];
  for (int k = 0; k < 4; ++k) {
    ws[k] = g_sweep_scratch.take();
    hs[k].ws = ws[k].get();
  }
  rh_status st[4] = {RH_OK, RH_OK, RH_OK, RH_OK};
  std::string errs[4];
  std::exception_ptr ex[4];
  {
    std::vector<std::thread> th;
    for (int k = 0; k < 4; ++k)
      th.emplace_back([&, k] {
        try {
          if (hipSetDevice(device) != hipSuccess) {
            st[k] = RH_EDEVICE;
            errs[k] = "hipSetDevice failed on an upload thread";
            return;
          }
          prepare_sweep(*sw[k], n, parent, k % 2 == 0, prm, &cuts[k], hs[k]);
          st[k] = commit_sweep(dn, hs[k], *out[k], errs[k]);
        } catch (...) {
          ex[k] = std::current_exception();
        }
      });
    for (std::thread &t : th) t.join();
  }
  for (int k = 0; k < 4; ++k) g_sweep_scratch.give(std::move(ws[k]));
  for (int k = 0; k < 4; ++k)
    if (ex[k]) std::rethrow_exception(ex[k]);
  for (int k = 0; k < 4; ++k)
    if (st[k] != RH_OK) {
      err = errs[k];
      return st[k];
    }
  for (int k = 0; k < 4; ++k) dn->sweep_steps.push_back(out[k]->n_steps);
  return RH_OK;
}

// A matrix in the row-pass layout of EllMat: rows by decreasing length,
// kThreads per pass, every pass padded to a multiple of kEllChunk entries.
rh_status upload_ell(DeviceNet *dn, std::vector<std::vector<std::pair<int32_t, double>>> &R, EllMat &m,
                     std::string &err) {
  const int32_t n = (int32_t)R.size();
  std::vector<int32_t> order(n);
  double norm = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    order[i] = i;
    std::sort(R[i].begin(), R[i].end());
    double s = 0.0;
    for (auto &pr : R[i]) s += std::fabs(pr.second);
    norm = std::max(norm, s);
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return R[a].size() > R[b].size(); });
  const int32_t npass = (n + kThreads - 1) / kThreads;
  std::vector<int32_t> rows((size_t)npass * kThreads, -1), chunks;
  std::vector<int32_t> first(npass), width(npass);
  int64_t slots = 0;
  for (int32_t p = 0; p < npass; ++p) {
    const int32_t longest = (int32_t)R[order[(size_t)p * kThreads]].size();
    const int32_t E = std::max(kEllChunk, (longest + kEllChunk - 1) / kEllChunk * kEllChunk);
    first[p] = (int32_t)slots;
    width[p] = E;
    for (int32_t e0 = 0; e0 < E; e0 += kEllChunk) {
      chunks.push_back((int32_t)(slots + (int64_t)e0 * kThreads));
      chunks.push_back(p);
      chunks.push_back((e0 == 0 ? 1 : 0) | (e0 + kEllChunk >= E ? 2 : 0));
      chunks.push_back(0);
    }
    slots += (int64_t)E * kThreads;
  }
  if (slots * 8 >= 0x7fffffff) {
    err = "network too large for the residual layout";
    return RH_EINVAL;
  }
  std::vector<int32_t> col((size_t)slots, 0);
  std::vector<double> val((size_t)slots, 0.0);
  for (int32_t p = 0; p < npass; ++p)
    for (int32_t t = 0; t < kThreads && (int64_t)p * kThreads + t < n; ++t) {
      const int32_t i = order[(size_t)p * kThreads + t];
      rows[(size_t)p * kThreads + t] = i;
      for (size_t e = 0; e < R[i].size(); ++e) {
        const size_t k = (size_t)first[p] + e * kThreads + t;
        col[k] = R[i][e].first;
        val[k] = R[i][e].second;
      }
    }
  Blob bl;
  const int64_t o_ch = bl.add(chunks), o_rows = bl.add(rows), o_col = bl.add(col), o_val = bl.add(val);
  const char *base = nullptr;
  UP(bl.h, base);
  m.n_chunks = (int32_t)(chunks.size() / 4);
  m.n_slots = (int32_t)slots;
  m.chunks = at_off<int4>(base, o_ch);
  m.rows = at_off<int32_t>(base, o_rows);
  m.col = at_off<int32_t>(base, o_col);
  m.val = at_off<double>(base, o_val);
  m.norm = norm;
  return RH_OK;
}

}  // namespace

rh_status device_set(int32_t device, std::string &err) {
  HIP_TRY(hipSetDevice(device));
  return RH_OK;
}

namespace {
// Device address of the fixed scratch array, per device (taken once, with
// that device current).
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void *g_fixed_ptr[kMaxDevices] = {};

void *fixed_scratch_of(int32_t device) {
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  return device >= 0 && device < kMaxDevices ? g_fixed_ptr[device] : nullptr;
}
}  // namespace

rh_status device_fixed_scratch_init(int32_t device, std::string &err) {
  if (device < 0 || device >= kMaxDevices) {
    err = "device index beyond the fixed scratch table";
    return RH_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (g_fixed_ptr[device]) return RH_OK;
  HIP_TRY(hipSetDevice(device));
  void *p = nullptr;
  HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) {
    err = "hipGetSymbolAddress returned no address for the fixed scratch";
    return RH_EDEVICE;
  }
  g_fixed_ptr[device] = p;
  return RH_OK;
}

void device_free(Network &net) {
  if (!net.dev) return;
  (void)hipDeviceSynchronize();
  for (void *p : net.dev->allocs) (void)hipFree(p);
  for (auto &pr : net.dev->pool) (void)hipFree(pr.second);  // an upload that stopped half-way
  if (net.dev->rinfo) (void)hipFree(net.dev->rinfo);
  runner_free(net.dev->run);
  delete net.dev;
  net.dev = nullptr;
}

void device_ctx_free(Context &ctx) {
  if (!ctx.dev) return;
  (void)hipDeviceSynchronize();
  for (auto &pr : ctx.dev->runs) runner_free(pr.second);
  delete ctx.dev;
  ctx.dev = nullptr;
}

rh_status device_collect(Network &net, std::string &err) {
  if (!net.dev) return RH_OK;
  return runner_collect(net.dev->run, net.dev->info, net.report, err);
}

rh_status device_ctx_collect(Context &ctx, rh_report &rep, std::string &err) {
  rep.last_kernel_ms = -1.0;
  if (!ctx.dev) return RH_OK;
  // sum over the streams' runners
  rh_report total = rep;
  total.last_launches = 0;
  double ms = 0.0;
  bool any_ms = false;
  for (auto &pr : ctx.dev->runs) {
    rh_report r = rep;
    rh_status s = runner_collect(pr.second, ctx.dev->info, r, err);
    if (s != RH_OK) return s;
    total.last_launches += r.last_launches;
    if (r.last_kernel_ms >= 0) {
      ms += r.last_kernel_ms;
      any_ms = true;
    }
    if (r.last_launches > 0) {
      total.dirs_per_group = r.dirs_per_group;
      for (int p = 0; p < 7; ++p) total.phase_us[p] = r.phase_us[p];
    }
  }
  total.last_kernel_ms = any_ms ? ms : -1.0;
  rep = total;
  return RH_OK;
}

rh_status device_upload(Network &net, std::string &err, const std::function<rh_status(std::string &)> &accept) {
  HIP_TRY(hipSetDevice(net.ctx->device));
  Runner keep;  // keep the launch resources across operating points
  double *keep_rinfo = nullptr;
  int64_t keep_cols = 0;
  std::multimap<size_t, void *> pool;  // and the arrays' device memory (see DeviceNet::pool)
  if (net.dev) {
    keep = net.dev->run;
    net.dev->run = Runner();
    keep_rinfo = net.dev->rinfo;
    keep_cols = net.dev->rinfo_cols;
    net.dev->rinfo = nullptr;
    (void)hipDeviceSynchronize();  // no kernel uses them any more
    for (size_t q = 0; q < net.dev->allocs.size(); ++q)
      pool.emplace(net.dev->alloc_bytes[q], net.dev->allocs[q]);
    net.dev->allocs.clear();
    net.dev->alloc_bytes.clear();
    device_free(net);
  }
  DeviceNet *dn = new DeviceNet();
  net.dev = dn;
  ++net.dev_gen;
  dn->run = keep;
  dn->rinfo = keep_rinfo;
  dn->rinfo_cols = keep_cols;
  dn->pool = std::move(pool);
  rh_status qs = query_info(net.ctx->device, dn->info, err);
  if (qs != RH_OK) return qs;

  NetDesc &nd = dn->nd;
  const LuPlan &lu = net.lu;
  nd.n_x = net.n_x;
  nd.n_p = net.n_p;
  nd.n_bus = net.n_bus;

  // The factors' sweeps read the factors only: they are prepared and
  // uploaded on a thread of their own while `accept` finishes the host side
  // of the solve.  On every way out of this function the guard joins the
  // thread (it is destroyed first) and the scratch goes back to the pool.
  struct Joiner {
    std::thread t;
    ~Joiner() {
      if (t.joinable()) t.join();
    }
  };
  struct SweepsGuard {
    std::unique_ptr<SweepsScratch> w = g_sweeps_scratch.take();
    ~SweepsGuard() { g_sweeps_scratch.give(std::move(w)); }
  } sg;
  ScheduleParams prm;
  prm.bmax = kBlockRows;
  prm.block_rows = kBlockRows;
  prm.lane_budget = kLaneBudget;
  prm.n_waves = kWaves;
  if (const char *e = std::getenv("RH_BLOCK_ROWS")) prm.bmax = std::min(kBlockRows, std::max(0, std::atoi(e)));
  if (const char *e = std::getenv("RH_WAVE_STEPS")) prm.wave_mode = std::atoi(e) != 0;
  if (net.sched_bmax >= 0) prm.bmax = std::min(kBlockRows, net.sched_bmax);  // the tuner's choice
  if (net.sched_wave >= 0) prm.wave_mode = net.sched_wave != 0;
  // the sweeps' cuts depend on the pattern and these parameters only
  if (net.cut_params[0] != prm.bmax || net.cut_params[1] != prm.wave_mode) {
    for (ScheduleCut &c : net.cuts) c = ScheduleCut();
    net.cut_params[0] = prm.bmax;
    net.cut_params[1] = prm.wave_mode;
  }
  rh_status sw_st = RH_OK;
  std::string sw_err;
  std::exception_ptr sw_ex;
  Joiner sweeps;
  sweeps.t = std::thread([&] {
    try {
      if (hipSetDevice(net.ctx->device) != hipSuccess) {
        sw_st = RH_EDEVICE;
        sw_err = "hipSetDevice failed on an upload thread";
        return;
      }
      sw_st = [&]() -> rh_status {
        std::string &err = sw_err;
        Sweep &sl = sg.w->sw[0], &su = sg.w->sw[1], &sut = sg.w->sw[2], &slt = sg.w->sw[3];
        std::vector<double> &pivinv = sg.w->pivinv;
        lu_sweeps(lu, sl, su, sut, slt, pivinv, &sg.w->lw);
        UP(pivinv, nd.pivinv);
        std::vector<float> &p32 = sg.w->p32;
        p32.assign(pivinv.begin(), pivinv.end());
        UP(p32, nd.pivinv32);
        const std::vector<int32_t> parent = etree_parent(lu);
        const Sweep *const sw[4] = {&sl, &su, &sut, &slt};
        DevSweep *const out[4] = {&nd.L, &nd.U, &nd.Ut, &nd.Lt};
        return upload_sweeps(dn, net.ctx->device, sw, net.n_x, parent, prm, out, net.cuts, err);
      }();
    } catch (...) {
      sw_ex = std::current_exception();
    }
  });
  if (accept) {
    const rh_status s = accept(err);
    if (s != RH_OK) return s;
  }

  // G_x and G_x^T in permuted numbering (residuals of the refined mode), each
  // built and uploaded on a thread of its own while the sweeps are; the
  // guard joins them on every way out of this function
  rh_status ell_st[2] = {RH_OK, RH_OK};
  std::string ell_err[2];
  std::exception_ptr ell_ex[2];
  Joiner ell[2];
  for (int k = 0; k < 2; ++k)
    ell[k].t = std::thread([&, k] {
      try {
        if (hipSetDevice(net.ctx->device) != hipSuccess) {
          ell_st[k] = RH_EDEVICE;
          ell_err[k] = "hipSetDevice failed on an upload thread";
          return;
        }
        const int32_t nx = net.n_x;
        std::vector<std::vector<std::pair<int32_t, double>>> rows(nx);
        for (int32_t r = 0; r < nx; ++r)
          for (int32_t e = net.gx.ptr[r]; e < net.gx.ptr[r + 1]; ++e) {
            const int32_t ip = lu.iperm[r], jp = lu.iperm[net.gx.col[e]];
            if (k == 0)
              rows[ip].push_back({jp, net.gx.val[e]});
            else
              rows[jp].push_back({ip, net.gx.val[e]});
          }
        ell_st[k] = upload_ell(dn, rows, k == 0 ? nd.gx : nd.gxt, ell_err[k]);
      } catch (...) {
        ell_ex[k] = std::current_exception();
      }
    });

  // G_p with rows in permuted order, and G_p^T with permuted columns
  {
    std::vector<int4> grows;
    std::vector<int32_t> col;
    std::vector<double> val;
    for (int32_t ip = 0; ip < net.n_x; ++ip) {
      const int32_t r = lu.perm[ip], e0 = (int32_t)col.size();
      for (int32_t e = net.gp.ptr[r]; e < net.gp.ptr[r + 1]; ++e) {
        col.push_back(net.gp.col[e]);
        val.push_back(net.gp.val[e]);
      }
      if ((int32_t)col.size() > e0) grows.push_back(make_int4(ip, e0, (int32_t)col.size(), 0));
    }
    nd.n_gp_rows = (int32_t)grows.size();
    UP(grows, nd.gp_rows);
    UP(col, nd.gp_col);
    UP(val, nd.gp_val);
    std::vector<std::vector<std::pair<int32_t, double>>> rows(net.n_p);
    for (int32_t r = 0; r < net.n_x; ++r)
      for (int32_t e = net.gp.ptr[r]; e < net.gp.ptr[r + 1]; ++e)
        rows[net.gp.col[e]].push_back({lu.iperm[r], net.gp.val[e]});
    std::vector<int32_t> tptr(net.n_p + 1, 0), tcol;
    std::vector<double> tval;
    for (int32_t q = 0; q < net.n_p; ++q) {
      std::sort(rows[q].begin(), rows[q].end());
      for (auto &pr : rows[q]) {
        tcol.push_back(pr.first);
        tval.push_back(pr.second);
      }
      tptr[q + 1] = (int32_t)tcol.size();
    }
    std::vector<double> c2(net.n_p, std::numeric_limits<double>::quiet_NaN());
    for (int32_t b : net.pv) c2[net.pg_p[b]] = 2.0 * net.c2[net.gen_of_bus[b]];
    std::vector<double> lam_p(net.n_x);
    for (int32_t ip = 0; ip < net.n_x; ++ip) lam_p[ip] = net.lam[lu.perm[ip]];
    Blob bl;
    const int64_t o_ptr = bl.add(tptr), o_col = bl.add(tcol), o_val = bl.add(tval), o_c2 = bl.add(c2);
    const int64_t o_lam = bl.add(lam_p), o_fp = bl.add(net.fp);
    const char *base = nullptr;
    UP(bl.h, base);
    nd.gpt_ptr = at_off<int32_t>(base, o_ptr);
    nd.gpt_col = at_off<int32_t>(base, o_col);
    nd.gpt_val = at_off<double>(base, o_val);
    nd.p_c2x2 = at_off<double>(base, o_c2);
    nd.lam = at_off<double>(base, o_lam);
    nd.fp = at_off<double>(base, o_fp);
  }
  // tangent sources per bus in permuted numbering: theta from X[thx] (-1 at
  // the reference bus); v from X[vs] at PQ buses, else from W[-vs - 1]
  std::vector<int32_t> thx(net.n_bus), vs(net.n_bus);
  for (int32_t b = 0; b < net.n_bus; ++b) {
    thx[b] = net.th_x[b] >= 0 ? lu.iperm[net.th_x[b]] : -1;
    vs[b] = net.v_x[b] >= 0 ? lu.iperm[net.v_x[b]] : -net.v_p[b] - 1;
  }
  const Tape &tp = net.tape;
  // tensor projection records: buses by decreasing degree (ties by index),
  // kThreads per pass, incidences in tape order
  {
    const int32_t nb = net.n_bus;
    std::vector<int32_t> order(nb);
    for (int32_t b = 0; b < nb; ++b) order[b] = b;
    auto deg = [&](int32_t b) { return tp.inc_ptr[b + 1] - tp.inc_ptr[b]; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return deg(x) > deg(y); });
    const int32_t npass = (nb + kThreads - 1) / kThreads;
    // the two int32 halves of a record word
    auto bits = [](int32_t lo, int32_t hi) {
      const uint64_t u = (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32);
      double d;
      std::memcpy(&d, &u, sizeof d);
      return d;
    };
    std::vector<int2> pm(npass);
    int64_t slots = 0;
    for (int32_t p = 0; p < npass; ++p) {
      const int32_t E = deg(order[p * kThreads]);
      pm[p] = make_int2((int32_t)slots, E);
      slots += (int64_t)E * kThreads;
      if (slots * 3 * 16 >= kProjMaxBytes) {
        err = "network too large for the projection records";
        return RH_EINVAL;
      }
    }
    const size_t S = (size_t)slots;
    const size_t NB = (size_t)npass * kThreads;  // bus planes padded to whole passes
    if ((int64_t)NB * 2 * 16 >= kProjMaxBytes) {
      err = "network too large for the projection records";
      return RH_EINVAL;
    }
    std::vector<double> pb(4 * NB, 0.0), pi(6 * S, 0.0);  // double2 planes
    for (size_t i = 0; i < NB; ++i) pb[2 * i] = bits(-1, -1);
    for (size_t k = 0; k < S; ++k) pi[2 * (2 * S + k) + 1] = bits(kPadInc, 0);
    for (int32_t p = 0; p < npass; ++p) {
      const int32_t first = p * kThreads;
      for (int32_t t = 0; t < kThreads && first + t < nb; ++t) {
        const int32_t b = order[first + t];
        const size_t i = (size_t)(first + t);
        pb[2 * i] = bits(thx[b], vs[b]);
        pb[2 * i + 1] = tp.bus_v[b];
        pb[2 * (NB + i)] = tp.bus_sth[b];
        pb[2 * (NB + i) + 1] = tp.bus_sv[b];
        for (int32_t e = 0; e < deg(b); ++e) {
          const int32_t q = tp.inc_ptr[b] + e, o = tp.inc_other[q];
          const size_t k = (size_t)pm[p].x + (size_t)e * kThreads + t;
          pi[2 * k] = tp.inc_K[q];
          pi[2 * k + 1] = tp.inc_Hps[q];
          pi[2 * (S + k)] = tp.inc_H[q];
          pi[2 * (S + k) + 1] = tp.inc_A2[q];
          pi[2 * (2 * S + k)] = tp.inc_vo[q];
          pi[2 * (2 * S + k) + 1] = bits(thx[o], vs[o]);
        }
      }
    }
    nd.n_proj_pass = npass;
    nd.proj_slots = (int32_t)S;
    Blob bl;
    const int64_t o_pass = bl.add(pm), o_bus = bl.add(pb), o_inc = bl.add(pi);
    const char *base = nullptr;
    UP(bl.h, base);
    nd.proj_pass = at_off<int2>(base, o_pass);
    nd.proj_bus = at_off<double2>(base, o_bus);
    nd.proj_inc = at_off<double2>(base, o_inc);
  }
  nd.n_slack = (int32_t)tp.slack_bus.size();
  {
    std::vector<int32_t> sth(tp.slack_bus.size()), svs(tp.slack_bus.size());
    for (size_t q = 0; q < tp.slack_bus.size(); ++q) {
      sth[q] = thx[tp.slack_bus[q]];
      svs[q] = vs[tp.slack_bus[q]];
    }
    UP(sth, nd.slack_thx);
    UP(svs, nd.slack_vs);
  }
  UP(tp.slack_gth, nd.slack_gth);
  UP(tp.slack_gv, nd.slack_gv);
  // the sweeps, then G_x and G_x^T (built on their threads meanwhile)
  sweeps.t.join();
  if (sw_ex) std::rethrow_exception(sw_ex);
  if (sw_st != RH_OK) {
    err = sw_err;
    return sw_st;
  }
  net.report.steps_l = nd.L.n_steps;
  net.report.steps_u = nd.U.n_steps;
  for (int k = 0; k < 2; ++k) ell[k].t.join();
  for (int k = 0; k < 2; ++k)
    if (ell_ex[k]) std::rethrow_exception(ell_ex[k]);
  for (int k = 0; k < 2; ++k)
    if (ell_st[k] != RH_OK) {
      err = ell_err[k];
      return ell_st[k];
    }
  {
    const NetDesc *p = nullptr;
    const std::vector<NetDesc> one(1, dn->nd);
    UP(one, p);
    dn->nd_dev = const_cast<NetDesc *>(p);
  }
  // what the previous operating point left unused
  for (auto &pr : dn->pool) (void)hipFree(pr.second);
  dn->pool.clear();
  HIP_TRY(hipDeviceSynchronize());
  return RH_OK;
}

namespace {
// grad F = grad_p f + G_p^T lambda (eq. (reduced_gradient)), one parameter
// per thread over the rows of G_p^T.
__global__ __launch_bounds__(256) void reduced_gradient_kernel(const NetDesc *nd, double *grad) {
  const int32_t q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nd->n_p) return;
  double acc = nd->fp[q];
  for (int32_t e = nd->gpt_ptr[q]; e < nd->gpt_ptr[q + 1]; ++e) acc = fma(nd->gpt_val[e], nd->lam[nd->gpt_col[e]], acc);
  grad[q] = acc;
}
}  // namespace

rh_status device_reduced_gradient(Network &net, double *dgrad, void *stream, std::string &err) {
  if (!net.dev) {
    err = "the operating point is not on the device";
    return RH_ESTATE;
  }
  HIP_TRY(hipSetDevice(net.ctx->device));
  const int32_t n_p = net.n_p;
  if (n_p > 0)
    hipLaunchKernelGGL(reduced_gradient_kernel, dim3((n_p + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), (const NetDesc *)net.dev->nd_dev, dgrad);
  HIP_TRY(hipGetLastError());
  return RH_OK;
}

rh_status device_hvp(Network &net, int32_t k, const double *dW, int64_t ldw, double *dHW,
                     int64_t ldhw, int32_t identity_from, rh_precision prec, void *stream,
                     std::string &err) {
  DeviceNet *dn = net.dev;
  if (!dn) {
    err = "network has no device data (solve first)";
    return RH_ESTATE;
  }
  if (k <= 0 || ldhw < net.n_p || (identity_from < 0 && (ldw < net.n_p || !dW)) || !dHW) {
    err = "bad block arguments";
    return RH_EINVAL;
  }
  if (identity_from >= 0 && (int64_t)identity_from + k > net.n_p) {
    err = "identity block exceeds n_p";
    return RH_EINVAL;
  }
  HIP_TRY(hipSetDevice(net.ctx->device));
  std::vector<WorkItem> items(1);
  WorkItem &it = items[0];
  it.nd = dn->nd_dev;
  it.W = dW;
  it.HW = dHW;
  it.ldw = ldw;
  it.ldhw = ldhw;
  it.k = k;
  it.identity_from = identity_from;
  it.rinfo = nullptr;
  const int32_t refine = prec == RH_FP32_REFINED ? net.ctx->refine : -1;
  if (refine >= 0) {
    // per-column refinement figures: columns 0 .. k - 1 of the call, or the
    // identity block's own columns of the full Hessian
    const int64_t cols = identity_from >= 0 ? (int64_t)net.n_p : (int64_t)k;
    if (cols > dn->rinfo_cols) {
      HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
      if (dn->rinfo) HIP_TRY(hipFree(dn->rinfo));
      dn->rinfo = nullptr;
      dn->rinfo_cols = 0;
      HIP_TRY(hipMalloc(&dn->rinfo, (size_t)cols * 4 * sizeof(double)));
      dn->rinfo_cols = cols;
    }
    it.rinfo = dn->rinfo + 4 * (int64_t)(identity_from >= 0 ? identity_from : 0);
  }
  const rh_tile &t = net.tile[prec == RH_FP32_REFINED ? 1 : 0];
  rh_status s = run_items(dn->info, dn->run, net.ctx->timing, refine, net.ctx->refine_tol, items, net.n_x,
                          (hipStream_t)stream, err, nullptr, t.k > 0 ? t.dirs_per_group : 0);
  net.report.dirs_per_group = dn->run.last_c;
  return s;
}

rh_status device_hvp_noalloc(Network &net, int32_t k, const double *dW, int64_t ldw, double *dHW, int64_t ldhw,
                             rh_precision prec, void *stream, std::string &err) {
  DeviceNet *dn = net.dev;
  if (!dn) {
    err = "network has no device data (solve first)";
    return RH_ESTATE;
  }
  if (k <= 0 || ldhw < net.n_p || ldw < net.n_p || !dW || !dHW) {
    err = "bad block arguments";
    return RH_EINVAL;
  }
  void *fp = fixed_scratch_of(net.ctx->device);
  if (!fp) {
    err = "no fixed scratch on this device (context not created on it)";
    return RH_ESTATE;
  }
  HIP_TRY(hipSetDevice(net.ctx->device));
  std::vector<WorkItem> items(1);
  WorkItem &it = items[0];
  it = WorkItem{};
  it.nd = dn->nd_dev;
  it.W = dW;
  it.HW = dHW;
  it.ldw = ldw;
  it.ldhw = ldhw;
  it.k = k;
  it.identity_from = -1;
  it.rinfo = nullptr;  // no per-column refinement figures
  const FixedScratch fx{static_cast<double *>(fp), (int64_t)RH_NOALLOC_SCRATCH_BYTES};
  const int32_t refine = prec == RH_FP32_REFINED ? net.ctx->refine : -1;
  const rh_tile &t = net.tile[prec == RH_FP32_REFINED ? 1 : 0];
  return run_items(dn->info, dn->run, 0, refine, net.ctx->refine_tol, items, net.n_x, (hipStream_t)stream, err,
                   &fx, t.k > 0 ? t.dirs_per_group : 0);
}

rh_status device_hvp_batch(Context &ctx, int32_t n, Network *const *nets, const int32_t *k,
                           const double *const *dW, const int64_t *ldw, double *const *dHW,
                           const int64_t *ldhw, const int32_t *identity_from, rh_precision prec,
                           void *stream, std::string &err) {
  HIP_TRY(hipSetDevice(ctx.device));
  if (!ctx.dev) {
    ctx.dev = new DeviceCtx();
    rh_status qs = query_info(ctx.device, ctx.dev->info, err);
    if (qs != RH_OK) return qs;
  }
  std::vector<WorkItem> items;
  int32_t max_nx = 0;
  for (int32_t i = 0; i < n; ++i) {
    Network &net = *nets[i];
    if (k[i] == 0) continue;
    WorkItem it{};
    it.nd = net.dev->nd_dev;
    it.W = dW[i];
    it.HW = dHW[i];
    it.ldw = ldw[i];
    it.ldhw = ldhw[i];
    it.k = k[i];
    it.identity_from = identity_from ? identity_from[i] : -1;
    it.rinfo = nullptr;  // batched calls record no per-column refinement figures
    items.push_back(it);
    max_nx = std::max(max_nx, net.n_x);
  }
  if (items.empty()) return RH_OK;
  const int32_t refine = prec == RH_FP32_REFINED ? ctx.refine : -1;
  return run_items(ctx.dev->info, ctx.dev->on(stream), ctx.timing, refine, ctx.refine_tol, items, max_nx,
                   (hipStream_t)stream, err);
}

int32_t device_max_c(const Network &net, rh_precision prec) {
  const DeviceNet *dn = net.dev;
  if (!dn) return 1;
  const size_t elem = prec == RH_FP32_REFINED ? sizeof(float) : sizeof(double);
  const int64_t pad_rows = (int64_t)net.n_x + kWavePadRows;
  const bool lds = (size_t)pad_rows * elem <= dn->info.lds_max && !std::getenv("RH_NO_LDS");
  return lds_max_c(pad_rows, dn->info.lds_max, lds, elem);
}

std::string device_key(int32_t device) {
  hipDeviceProp_t p{};
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string k = std::string(p.gcnArchName) + "/" + std::to_string(p.multiProcessorCount) + "cu";
  for (char &c : k)
    if (c == ' ' || c == '|' || c == '\n') c = '_';
  return k;
}

int32_t device_launch_dirs(const Network &net, rh_precision prec) {
  const DeviceNet *dn = net.dev;
  if (!dn) return 1;
  const rh_tile &t = net.tile[prec == RH_FP32_REFINED ? 1 : 0];
  if (t.k > 0) return t.dirs_per_group * dn->info.cus;  // the tuner's count
  const bool refined = prec == RH_FP32_REFINED;
  const size_t elem = refined ? sizeof(float) : sizeof(double);
  const int64_t pad_rows = (int64_t)net.n_x + kWavePadRows;
  const bool lds = (size_t)pad_rows * elem <= dn->info.lds_max && !std::getenv("RH_NO_LDS");
  return lds_max_c(pad_rows, dn->info.lds_max, lds, elem) * dn->info.cus;
}

struct DeviceBatch {
  int device = -1;
  std::vector<const Network *> nets;
  std::vector<uint64_t> gens;
  WorkItem *items_dev = nullptr;
  double *scratch = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t C = 0, groups = 0, dirs = 0;
};

void device_batch_free(DeviceBatch *b) {
  if (!b) return;
  if (b->device >= 0) {
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();  // replays may still be in flight on the callers' streams
  }
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->items_dev) (void)hipFree(b->items_dev);
  if (b->scratch) (void)hipFree(b->scratch);
  delete b;
}

namespace {
rh_status batch_build(DeviceBatch &b, const DeviceInfo &info, int32_t refine, double refine_tol,
                      std::vector<WorkItem> &items, int32_t max_nx, std::string &err) {
  LaunchPlan pl;
  rh_status ps = plan_launch(info, refine, items, max_nx, pl, err);
  if (ps != RH_OK) return ps;
  b.C = pl.C;
  b.groups = pl.groups;
  HIP_TRY(hipMalloc(&b.scratch, std::max<size_t>(256, (size_t)pl.groups * pl.stride * sizeof(double))));
  LaunchArgs la{};
  la.refine = refine;
  la.refine_tol = refine_tol;
  la.n_items = (int32_t)items.size();
  la.n_chunks = (int32_t)pl.n_chunks;
  la.scratch = b.scratch;
  la.scratch_stride = pl.stride;
  la.pad_rows = pl.pad_rows;
  if (items.size() == 1) {
    la.one = items[0];
  } else {
    HIP_TRY(hipMalloc(&b.items_dev, items.size() * sizeof(WorkItem)));
    HIP_TRY(hipMemcpy(b.items_dev, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    la.items = b.items_dev;
  }
  if (pl.n_chunks == 0) return RH_OK;  // nothing to record: replays do nothing
  // kernel attributes first (not stream work), then the launch alone in the graph
  std::string e2;
  rh_status as = launch_plan(pl, pl.groups, nullptr, la, err, kAttrsOnly);
  if (as != RH_OK) return as;
  HIP_TRY(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
  rh_status ls = launch_plan(pl, pl.groups, b.cap, la, e2, kLaunchOnly);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(b.cap, &g);
  b.graph = g;
  if (ls != RH_OK) {
    err = e2;
    return ls;
  }
  HIP_TRY(ce);
  HIP_TRY(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
  return RH_OK;
}
}  // namespace

rh_status device_batch_create(Context &ctx, int32_t n, Network *const *nets, const int32_t *k,
                              const double *const *dW, const int64_t *ldw, double *const *dHW,
                              const int64_t *ldhw, const int32_t *identity_from, rh_precision prec,
                              DeviceBatch **out, std::string &err) {
  *out = nullptr;
  HIP_TRY(hipSetDevice(ctx.device));
  if (!ctx.dev) {
    ctx.dev = new DeviceCtx();
    rh_status qs = query_info(ctx.device, ctx.dev->info, err);
    if (qs != RH_OK) return qs;
  }
  DeviceBatch *b = new DeviceBatch();
  b->device = ctx.device;
  std::vector<WorkItem> items;
  int32_t max_nx = 0;
  for (int32_t i = 0; i < n; ++i) {
    Network &net = *nets[i];
    b->nets.push_back(&net);
    b->gens.push_back(net.dev_gen);
    if (k[i] == 0) continue;
    WorkItem it{};
    it.nd = net.dev->nd_dev;
    it.W = dW[i];
    it.HW = dHW[i];
    it.ldw = ldw[i];
    it.ldhw = ldhw[i];
    it.k = k[i];
    it.identity_from = identity_from ? identity_from[i] : -1;
    it.rinfo = nullptr;
    items.push_back(it);
    b->dirs += k[i];
    max_nx = std::max(max_nx, net.n_x);
  }
  const int32_t refine = prec == RH_FP32_REFINED ? ctx.refine : -1;
  rh_status s = batch_build(*b, ctx.dev->info, refine, ctx.refine_tol, items, max_nx, err);
  if (s != RH_OK) {
    device_batch_free(b);
    return s;
  }
  *out = b;
  return RH_OK;
}

rh_status device_batch_launch(DeviceBatch *b, void *stream, std::string &err) {
  for (size_t i = 0; i < b->nets.size(); ++i)
    if (!b->nets[i]->dev || b->nets[i]->dev_gen != b->gens[i] || !b->nets[i]->solved) {
      err = "batch item " + std::to_string(i) + ": the network was re-uploaded or invalidated since the batch was recorded";
      return RH_ESTATE;
    }
  if (!b->exec) return RH_OK;
  HIP_TRY(hipSetDevice(b->device));
  HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
  return RH_OK;
}

void device_batch_info(const DeviceBatch *b, int32_t *dirs_per_group, int32_t *workgroups, int32_t *directions) {
  if (dirs_per_group) *dirs_per_group = b->C;
  if (workgroups) *workgroups = b->groups;
  if (directions) *directions = b->dirs;
}

rh_status device_refinement_report(Network &net, int32_t n, std::vector<double> &out, std::string &err) {
  DeviceNet *dn = net.dev;
  if (!dn || !dn->rinfo || n > dn->rinfo_cols) {
    err = "no refined product recorded for these columns";
    return RH_ESTATE;
  }
  out.assign((size_t)n * 4, 0.0);
  if (n == 0) return RH_OK;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out.data(), dn->rinfo, out.size() * sizeof(double), hipMemcpyDeviceToHost));
  return RH_OK;
}

int64_t device_network_bytes(const Network &net) {
  const DeviceNet *dn = net.dev;
  if (!dn) return 0;
  return dn->bytes + dn->rinfo_cols * 4 * (int64_t)sizeof(double) + (int64_t)dn->run.scratch_bytes;
}

int64_t device_scratch_per_direction(int32_t n_x, rh_precision prec) {
  // per-workgroup scratch of run_items, per direction it owns, with the
  // vector in global memory (the larger case): FP64 Y_x and X; refined V1,
  // V2 and the FP32 correction
  return (prec == RH_FP32_REFINED ? 3 * 8 : 2 * 8) * ((int64_t)n_x + kWavePadRows);
}

rh_status device_alloc(void **p, size_t bytes, std::string &err) {
  HIP_TRY(hipMalloc(p, bytes));
  return RH_OK;
}

void device_release(void *p) {
  if (p) (void)hipFree(p);
}

rh_status device_memcpy_h2d(void *dst, const void *src, size_t bytes, std::string &err) {
  HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
  return RH_OK;
}

rh_status device_memcpy_d2h(void *dst, const void *src, size_t bytes, std::string &err) {
  HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  return RH_OK;
}

rh_status device_memcpy_2d(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width,
                           size_t rows, int to_device, std::string &err) {
  HIP_TRY(hipMemcpy2D(dst, dpitch, src, spitch, width, rows,
                      to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost));
  return RH_OK;
}

rh_status device_sync(void *stream, std::string &err) {
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return RH_OK;
}

}  // namespace rh
