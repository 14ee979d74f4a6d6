// Device-resident Newton-Raphson on g(x, p) = 0 (Sec. 3.2) with a
// fixed-pattern numeric LU refactorisation of G_x on the GPU (Sec. 5.2: the
// pattern and the ordering are analysed once on the host; only the numeric
// factorisation is repeated for every operating point).
//
// Per Newton step, on the device:
//   1. bus voltages from x and p; per branch the four end flows of eq.
//      (powerflow) and their 16 partial derivatives w.r.t. (theta_f, theta_t,
//      v_f, v_t);
//   2. the mismatch g (per bus, its incident branches summed in branch
//      order) and max |g|, the one number the host reads per step;
//   3. the values of G_x on its fixed pattern (per entry, its branch
//      partials summed in branch order: no atomics);
//   4. P G_x P^T = L U with static diagonal pivots: row by row, the rows of
//      one elimination level at a time (one wave per row, the row's values
//      in LDS), except the last rows (the top of the elimination tree, where
//      the factors are nearly dense), which after their steps with earlier
//      rows are factored as one dense block by one workgroup, in registers;
//   5. the Newton step from the two triangular solves (the rows below the
//      dense block by levels, the block by dense substitution), and
//      x -= step.
// After convergence the state and the factors are copied to the host, which
// forms the first-order adjoint and the branch coefficients from them (it
// does not factorise) and uploads the product path as after a host solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <cstring>
#include <vector>

#include "rh_internal.h"

namespace rh {

namespace {

#define HIP_TRY(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
      return RH_EDEVICE;                                                       \
    }                                                                          \
  } while (0)

constexpr int kNtThreads = 1024;
constexpr int kNtWaves = kNtThreads / 64;

// Device arrays of one network (pattern and topology: built once).
struct NtArrays {
  int32_t n_bus, n_br, n_x, n_p, nnz_gx, nnz_lu, maxpat;
  // branches
  const int32_t *br_f, *br_t;
  const double *gs, *bs, *bsh;
  // buses: state maps and incidences (branch order)
  const int32_t *th_x, *v_x, *v_p, *pg_p;
  const int32_t *inc_ptr, *inc_code;  // code = 4 * branch + 2 * end (end 0 from, 1 to)
  // G_x: contributions of branch partials per pattern entry, in branch order
  const int32_t *gxc_ptr, *gxc_src;  // src = 16 * branch + 4 * flow + variable
  // LU (permuted numbering): row i holds its L part (|lrow|) then its U part
  // (diagonal first); lucol = column of every position
  const int32_t *row_ptr, *nl, *lucol, *perm;
  const int32_t *a_ptr, *a_src;  // G_x entries of permuted row i: G_x value index
  const uint16_t *a_dst;         // ... and position in the row
  const int64_t *upd_ptr;        // per row: first target of its updates
  const uint16_t *tgt;           // targets (position in the row) of every update, row by row
  const int4 *step;              // per L position: {U part of the pivot row: start, length; first target; row}
  // the dense top block: rows b0 .. n_x - 1 (m_blk of them); levels of the
  // rows below it; per block row its steps with pivot rows below b0 and the
  // position of every block column in it (-1: none)
  int32_t b0, m_blk;
  const int32_t *lev_ptr_f, *lev_rows_f, *ns, *dmap;
  const int32_t *lev_ptr_uf, *lev_rows_uf;  // U levels of the rows below b0
  // per entry of lev_rows_f / lev_rows_uf: {row, first entry, entries, diagonal
  // position} of the row in the L (U) sweep (entries past the diagonal for U)
  const int4 *sdesc_l, *sdesc_u;
  // per entry of lev_rows_f: {row, first position, positions, L positions}
  // and {first, end} of its G_x entries (a row's set-up in one load)
  const int4 *fdesc;
  const int2 *fdesc_a;
};

// Per-solve device vectors.
struct NtVectors {
  double *x, *p, *Pd, *Qd, *th, *v, *flows, *dG, *g, *gx, *lu, *y;
  double *rinv;  // 1 / u_ii of every finished row
  double *S;     // the dense block after the steps with pivot rows below b0, then its factors
                 // (m_blk x m_blk, row-major: L below the diagonal, U on and above)
  double *amax;  // largest |G_x entry| of every block row (the pivot test)
  double *stat;  // [0] max |g|, [1] non-finite flag, [2] singular pivot row + 1
};

struct NtArgs {
  NtArrays a;
  NtVectors w;
};

// ---- kernels: states, flows, residual, Jacobian values -----------------

__global__ void nt_state(const NtArgs A) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= A.a.n_bus) return;
  const int32_t tx = A.a.th_x[b], vx = A.a.v_x[b], vp = A.a.v_p[b];
  A.w.th[b] = tx >= 0 ? A.w.x[tx] : 0.0;
  A.w.v[b] = vx >= 0 ? A.w.x[vx] : (vp >= 0 ? A.w.p[vp] : 0.0);
}

// End flows alpha v_e^2 + v_f v_t h(a) of one branch and their partials.
__global__ void nt_flows(const NtArgs A, int want_grad) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= A.a.n_br) return;
  const int32_t f = A.a.br_f[b], t = A.a.br_t[b];
  const double gs = A.a.gs[b], bs = A.a.bs[b], bh = A.a.bsh[b];
  const double a = A.w.th[f] - A.w.th[t];
  double s, c;
  sincos(a, &s, &c);
  const double alpha[4] = {gs, -(bs + bh), gs, -(bs + bh)};
  const double h[4] = {-(gs * c + bs * s), -(gs * s - bs * c), -(gs * c - bs * s), gs * s + bs * c};
  const double hp[4] = {gs * s - bs * c, -(gs * c + bs * s), gs * s + bs * c, gs * c - bs * s};
  const double vf = A.w.v[f], vt = A.w.v[t], K = vf * vt;
  A.w.flows[4 * b + 0] = alpha[0] * vf * vf + K * h[0];
  A.w.flows[4 * b + 1] = alpha[1] * vf * vf + K * h[1];
  A.w.flows[4 * b + 2] = alpha[2] * vt * vt + K * h[2];
  A.w.flows[4 * b + 3] = alpha[3] * vt * vt + K * h[3];
  if (!want_grad) return;
  for (int k = 0; k < 4; ++k) {
    double *d = A.w.dG + 16 * (int64_t)b + 4 * k;
    d[0] = K * hp[k];
    d[1] = -K * hp[k];
    d[2] = vt * h[k] + (k < 2 ? 2.0 * alpha[k] * vf : 0.0);
    d[3] = vf * h[k] + (k >= 2 ? 2.0 * alpha[k] * vt : 0.0);
  }
}

// g at the x rows of every bus: P (theta rows) and Q (v rows) mismatch.
__global__ void nt_residual(const NtArgs A) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= A.a.n_bus) return;
  double P = 0.0, Q = 0.0;
  for (int32_t e = A.a.inc_ptr[b]; e < A.a.inc_ptr[b + 1]; ++e) {
    const int32_t code = A.a.inc_code[e];
    P += A.w.flows[code];
    Q += A.w.flows[code + 1];
  }
  const int32_t tx = A.a.th_x[b], vx = A.a.v_x[b], pg = A.a.pg_p[b];
  if (tx >= 0) {
    double r = P + A.w.Pd[b];
    if (pg >= 0) r -= A.w.p[pg];
    A.w.g[tx] = r;
  }
  if (vx >= 0) A.w.g[vx] = Q + A.w.Qd[b];
}

// max |g| and a non-finite flag (one workgroup); clears the pivot status.
__global__ __launch_bounds__(kNtThreads) void nt_norm(const NtArgs A) {
  __shared__ double s_max[kNtWaves];
  __shared__ int s_bad[kNtWaves];
  double m = 0.0;
  int bad = 0;
  for (int32_t i = threadIdx.x; i < A.a.n_x; i += kNtThreads) {
    const double gi = A.w.g[i];
    if (!isfinite(gi)) bad = 1;
    m = fmax(m, fabs(gi));
  }
  for (int off = 32; off >= 1; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off));
    bad |= __shfl_xor(bad, off);
  }
  if ((threadIdx.x & 63) == 0) {
    s_max[threadIdx.x >> 6] = m;
    s_bad[threadIdx.x >> 6] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0;
    int bb = 0;
    for (int w = 0; w < kNtWaves; ++w) {
      mm = fmax(mm, s_max[w]);
      bb |= s_bad[w];
    }
    A.w.stat[0] = mm;
    A.w.stat[1] = bb;
    A.w.stat[2] = 0.0;
  }
}

// Values of G_x: every pattern entry sums its branch partials in branch order.
__global__ void nt_gx(const NtArgs A) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.a.nnz_gx) return;
  double acc = 0.0;
  for (int32_t e = A.a.gxc_ptr[s]; e < A.a.gxc_ptr[s + 1]; ++e) acc += A.w.dG[A.a.gxc_src[e]];
  A.w.gx[s] = acc;
}

// ---- refactorisation ----------------------------------------------------

// P G_x P^T = L U, one elimination level of rows at a time (rows of a level
// depend only on rows of earlier levels), one wave per row.  A row is
// scattered into the wave's LDS buffer; then, for every entry of its L part
// in ascending order (pivot row k), l = w_q / u_kk and the U part of row k
// (final: an earlier level) is subtracted, l times, at precomputed
// positions; then the row is written back with the reciprocal of its pivot.
// The elimination steps form the critical path (about ten thousand at 10k
// buses, below the dense block), so a step waits for nothing in global memory:
// the step descriptors are loaded 64 at a time into a lane register and read
// by readlane, the pivot reciprocal, U values and targets of a step are
// loaded four steps ahead into a statically indexed ring, and l takes the
// stored reciprocal instead of a division.  A pivot below 1e-13 times the
// row's largest entry (or not finite) marks the row.
struct NtOp {
  double uv, rk;
  int32_t tg, ul, kb, us;
};

// A row of the factors: its first position and positions, and the range of
// its G_x entries.
struct NtRow {
  int32_t base, len, a0, a1;
};

__device__ __forceinline__ NtRow nt_row(const NtArgs &A, int32_t i) {
  return NtRow{A.a.row_ptr[i], A.a.row_ptr[i + 1] - A.a.row_ptr[i], A.a.a_ptr[i], A.a.a_ptr[i + 1]};
}

// A row scattered into W and its first nl elimination steps taken; returns
// the largest |entry| of the row before elimination.
__device__ __forceinline__ double nt_eliminate(const NtArgs &A, const NtRow &R, int32_t nl, double *W, int l64) {
  const NtArrays &a = A.a;
  const double *LU = A.w.lu;
  const int32_t base = R.base, len = R.len;
  for (int32_t t = l64; t < len; t += 64) W[t] = 0.0;
  double amax = 0.0;
  for (int32_t t = R.a0 + l64; t < R.a1; t += 64) {
    const double val = A.w.gx[a.a_src[t]];
    W[a.a_dst[t]] = val;
    amax = fmax(amax, fabs(val));
  }
  for (int off = 32; off >= 1; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  __builtin_amdgcn_wave_barrier();
  const int4 *SI = a.step + base;
  const int4 z4 = make_int4(0, 0, 0, 0);
  // the descriptors in chunks of 64 steps: lane j of cur holds step c + j,
  // lane j of nxt step c + 64 + j
  int4 cur = l64 < nl ? SI[l64] : z4, nxt = 64 + l64 < nl ? SI[64 + l64] : z4;
  // the update targets of consecutive steps follow each other (ul - 1 per
  // step), so only the first step's start is read
  int32_t us_run = __builtin_amdgcn_readlane(cur.z, 0);
  // step q's descriptor from lane j of src, its loads into o
  auto load_op = [&](int32_t q, const int4 &src, int j, NtOp &o) {
    const bool in = q < nl;
    o.kb = __builtin_amdgcn_readlane(src.x, j);
    o.ul = in ? __builtin_amdgcn_readlane(src.y, j) : 0;
    o.us = us_run;
    us_run += in ? o.ul - 1 : 0;
    const int32_t k = __builtin_amdgcn_readlane(src.w, j);
    // every lane issues the same three loads on every path (an address of
    // 0 where it has no entry; such values are never used), so the
    // compiler's wait before a step counts only that step's own loads
    // instead of draining the whole ring
    const bool ok = in && 1 + l64 < o.ul;
    o.uv = LU[ok ? o.kb + 1 + l64 : 0];
    o.tg = a.tgt[ok ? o.us + l64 : 0];
    o.rk = A.w.rinv[in ? k : 0];
  };
  constexpr int kD = 4;
  static_assert(64 % kD == 0, "whole groups of steps per chunk");
  NtOp ring[kD];
#pragma unroll
  for (int d = 0; d < kD; ++d) load_op(d, cur, d, ring[d]);
  auto step = [&](int32_t q, const NtOp &o) {
    const double l = W[q] * o.rk;
    __builtin_amdgcn_wave_barrier();  // every lane has read w_q
    if (l64 == 0) W[q] = l;
    if (1 + l64 < o.ul) W[o.tg] -= l * o.uv;
    if (o.ul > 65)  // a pivot row longer than a wave: the rest of it
      for (int32_t s2 = 65 + l64; s2 < o.ul; s2 += 64) W[a.tgt[o.us + s2 - 1]] -= l * LU[o.kb + s2];
    __builtin_amdgcn_wave_barrier();  // this step's writes before the next step's reads
  };
  for (int32_t c = 0; c < nl; c += 64) {
    // groups of kD steps; the ring's loads for the steps kD on read this
    // chunk's descriptors, in the chunk's last group the next chunk's
    int32_t g = 0;
    for (; g < 64 - kD && c + g < nl; g += kD) {
#pragma unroll
      for (int d = 0; d < kD; ++d) {
        const int32_t q = c + g + d;
        if (q < nl) step(q, ring[d]);
        load_op(q + kD, cur, g + d + kD, ring[d]);
      }
    }
    if (c + g < nl) {
#pragma unroll
      for (int d = 0; d < kD; ++d) {
        const int32_t q = c + g + d;
        if (q < nl) step(q, ring[d]);
        load_op(q + kD, nxt, g + d + kD - 64, ring[d]);
      }
    }
    cur = nxt;
    nxt = c + 128 + l64 < nl ? SI[c + 128 + l64] : z4;
  }
  __builtin_amdgcn_wave_barrier();
  return amax;
}

// A pivot below 1e-13 times its row's largest entry (or not finite) marks
// the row as singular.
__device__ __forceinline__ void nt_check_pivot(const NtArgs &A, int32_t i, double d, double amax) {
  if (!isfinite(d) || !(fabs(d) > 1e-13 * amax) || amax == 0.0) A.w.stat[2] = (double)(i + 1);
}

// Row idx of the levels below the dense block, its set-up from one
// descriptor.
__device__ __forceinline__ void nt_factor_row(const NtArgs &A, int32_t idx, double *W, int l64) {
  const int4 d = A.a.fdesc[idx];
  const int2 ar = A.a.fdesc_a[idx];
  const int32_t i = d.x, base = d.y, len = d.z, nl = d.w;
  const double amax = nt_eliminate(A, NtRow{base, len, ar.x, ar.y}, nl, W, l64);
  for (int32_t t = l64; t < len; t += 64) A.w.lu[base + t] = W[t];
  if (l64 == 0) {
    const double d = W[nl];
    A.w.rinv[i] = 1.0 / d;
    nt_check_pivot(A, i, d, amax);
  }
}

// Block row r: its steps with pivot rows below b0; the finished L entries
// go to the factors, the rest (columns b0 and up) into row r of S.
__device__ __forceinline__ void nt_block_row(const NtArgs &A, int32_t r, double *W, int l64) {
  const int32_t m = A.a.m_blk, i = A.a.b0 + r, ns = A.a.ns[r];
  const NtRow R = nt_row(A, i);
  const int32_t base = R.base;
  const double amax = nt_eliminate(A, R, ns, W, l64);
  for (int32_t t = l64; t < ns; t += 64) A.w.lu[base + t] = W[t];
  for (int32_t c = l64; c < m; c += 64) {
    const int32_t p = A.a.dmap[(int64_t)r * m + c];
    A.w.S[(int64_t)r * m + c] = p >= 0 ? W[p] : 0.0;
  }
  if (l64 == 0) A.w.amax[r] = amax;
}

// One wide level of the rows below b0: a wave per row over many workgroups
// of four waves.
constexpr int kNtWideWaves = 4;
__global__ __launch_bounds__(64 * kNtWideWaves) void nt_refactor_level(const NtArgs A, int32_t lev) {
  extern __shared__ double s_w[];
  const int wv = threadIdx.x >> 6, l64 = threadIdx.x & 63;
  const int32_t idx = A.a.lev_ptr_f[lev] + blockIdx.x * kNtWideWaves + wv;
  if (idx < A.a.lev_ptr_f[lev + 1]) nt_factor_row(A, idx, s_w + (int64_t)wv * A.a.maxpat, l64);
}

// Levels lev0 .. lev1 - 1 of the rows below b0 by one workgroup, a barrier
// between levels.
__global__ __launch_bounds__(kNtThreads) void nt_refactor_run(const NtArgs A, int32_t lev0, int32_t lev1) {
  extern __shared__ double s_w[];
  const int wv = threadIdx.x >> 6, l64 = threadIdx.x & 63;
  double *W = s_w + (int64_t)wv * A.a.maxpat;
  for (int32_t lev = lev0; lev < lev1; ++lev) {
    for (int32_t idx = A.a.lev_ptr_f[lev] + wv; idx < A.a.lev_ptr_f[lev + 1]; idx += kNtWaves)
      nt_factor_row(A, idx, W, l64);
    __syncthreads();
  }
}

// The block rows' steps with pivot rows below b0 (all final), a wave per row.
__global__ __launch_bounds__(64 * kNtWideWaves) void nt_block_rows(const NtArgs A) {
  extern __shared__ double s_w[];
  const int wv = threadIdx.x >> 6, l64 = threadIdx.x & 63;
  const int32_t r = blockIdx.x * kNtWideWaves + wv;
  if (r < A.a.m_blk) nt_block_row(A, r, s_w + (int64_t)wv * A.a.maxpat, l64);
}

// The dense block S = L_b U_b by one workgroup, right-looking with static
// pivots: at column c, every entry (r, j) with r, j > c loses
// (s_rc / s_cc) s_cj.  Each entry thus receives its updates in ascending
// pivot order with l = s_rc * (1 / s_cc), as in the row-by-row elimination,
// so the factors agree with it.  The block stays in registers: thread
// (column j, row group g) holds rows g, g + 8, ..., g + 120 of column j.  Before
// step c the threads of column c publish its entries below the diagonal,
// the threads holding row c its entries right of the diagonal and the
// reciprocal of the pivot, into one of two LDS buffers (zeros elsewhere, so
// every thread updates all its entries with no test: a zero multiplier or
// pivot-row entry leaves an entry unchanged); one barrier per step.  Column
// c of L is scaled at the write-back (the unscaled s_rc is what step c
// publishes).  The results go to the factors through dmap, with the pivot
// reciprocals.
constexpr int kNtDenseCols = 128;                         // threads along a row
constexpr int kNtDenseGroups = kNtThreads / kNtDenseCols;  // row groups
constexpr int kNtDenseRows = kNtDenseCols / kNtDenseGroups;  // rows per thread
static_assert(kNtDenseCols >= kNtDenseTop, "one thread per block column");
static_assert(kNtDenseCols == 128 && kNtThreads == 1024, "the wave layout below");
struct NtDenseLds {
  double col[2][kNtDenseCols];  // pivot column, row g + 8 k at g * kNtDenseRows + k
  double row[2][kNtDenseCols];  // pivot row, by column
  double rinv[kNtDenseCols];    // pivot reciprocals
};

__device__ __forceinline__ void nt_dense_publish(NtDenseLds &L, const double (&t)[kNtDenseRows], int32_t c,
                                                 int32_t m, int j, int g) {
  const int b = c & 1;
  if (j == c) {
#pragma unroll
    for (int k = 0; k < kNtDenseRows; ++k) {
      const int32_t r = g + k * kNtDenseGroups;
      L.col[b][g * kNtDenseRows + k] = r > c && r < m ? t[k] : 0.0;
    }
  }
  if (g == c % kNtDenseGroups) {
    const int kc = c / kNtDenseGroups;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kNtDenseRows; ++k) v = k == kc ? t[k] : v;
    L.row[b][j] = j > c && j < m ? v : 0.0;
    if (j == c) L.rinv[c] = 1.0 / v;
  }
}

__global__ __launch_bounds__(kNtThreads) void nt_dense_lu(const NtArgs A) {
  __shared__ NtDenseLds L;
  const int32_t m = A.a.m_blk, b0 = A.a.b0;
  // Wave w takes the column half (w / 4) mod 2 and the row group
  // w mod 4 + 4 (w / 8): the four waves that share a SIMD (w mod 4) hold
  // both halves, so the SIMDs stay evenly loaded once the first half's
  // columns are finished.  The row group is the same for a whole wave.
  const int tid = threadIdx.x, w = tid >> 6;
  const int j = (tid & 63) + 64 * ((w >> 2) & 1);
  const int g = __builtin_amdgcn_readfirstlane((w & 3) + 4 * (w >> 3));
  // the block, and (for the write-back, loaded now so that their latency
  // hides behind the steps) each entry's factor position and the row
  // maximum of this column's diagonal entry
  // (every load from a clamped address, so that none waits for another;
  // the entries outside the block are masked afterwards)
  double t[kNtDenseRows];
  int32_t pos[kNtDenseRows], base[kNtDenseRows];
  uint32_t in = 0;
#pragma unroll
  for (int k = 0; k < kNtDenseRows; ++k) {
    const int32_t r = g + k * kNtDenseGroups;
    const bool ok = r < m && j < m;
    in |= (uint32_t)ok << k;
    const int64_t e = ok ? (int64_t)r * m + j : 0;
    t[k] = A.w.S[e];
    pos[k] = A.a.dmap[e];
    base[k] = A.a.row_ptr[b0 + (r < m ? r : m - 1)];
  }
  const double amax = A.w.amax[j < m ? j : 0];
#pragma unroll
  for (int k = 0; k < kNtDenseRows; ++k) t[k] = (in >> k) & 1 ? t[k] : 0.0;
  nt_dense_publish(L, t, 0, m, j, g);
  __syncthreads();
  for (int32_t c = 0; c < m; ++c) {
    const int b = c & 1;
    // a wave whose columns are all finished has nothing to update, nor a
    // wave's finished rows (tests uniform over the wave)
    if ((j | 63) > c) {
      const double rp = L.rinv[c], u = L.row[b][j];
      const double *cb = &L.col[b][g * kNtDenseRows];
#pragma unroll
      for (int k = 0; k < kNtDenseRows; ++k)
        if (g + k * kNtDenseGroups > c) t[k] -= (cb[k] * rp) * u;
    }
    if (c + 1 < m) nt_dense_publish(L, t, c + 1, m, j, g);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kNtDenseRows; ++k) {
    const int32_t r = g + k * kNtDenseGroups;
    if (!((in >> k) & 1)) continue;
    if (j == r) {
      nt_check_pivot(A, b0 + r, t[k], amax);
      A.w.rinv[b0 + r] = L.rinv[r];
    }
    const double v = j < r ? t[k] * L.rinv[j] : t[k];
    A.w.S[(int64_t)r * m + j] = v;  // the dense block's factors, for the Newton step's solves
    if (pos[k] >= 0) A.w.lu[base[k] + pos[k]] = v;
  }
}

// ---- Newton step: y = P g; L y; U y; x -= P^T y ---------------------------
// One wave per row: lanes take the row's entries in turn and the wave sums.
// Y is the vector being solved (global memory, or its copy in LDS).

__device__ __forceinline__ void nt_lrow(const NtArgs &A, double *Y, int32_t i, int l64) {
  const NtArrays &a = A.a;
  const int32_t base = a.row_ptr[i], nl = a.nl[i];
  double s = 0.0;
  for (int32_t q = l64; q < nl; q += 64) s += A.w.lu[base + q] * Y[a.lucol[base + q]];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (l64 == 0) Y[i] -= s;
}

__device__ __forceinline__ void nt_urow(const NtArgs &A, double *Y, int32_t i, int l64) {
  const NtArrays &a = A.a;
  const int32_t ub = a.row_ptr[i] + a.nl[i], ue = a.row_ptr[i + 1];
  double s = 0.0;
  for (int32_t q = ub + 1 + l64; q < ue; q += 64) s += A.w.lu[q] * Y[a.lucol[q]];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (l64 == 0) Y[i] = (Y[i] - s) / A.w.lu[ub];
}

__global__ void nt_permute_in(const NtArgs A) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < A.a.n_x) A.w.y[i] = A.w.g[A.a.perm[i]];
}

__global__ void nt_update_x(const NtArgs A) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < A.a.n_x) A.w.x[A.a.perm[i]] -= A.w.y[i];
}

// One wide level of the L (upper = 0) or U (upper = 1) sweep over the rows
// below the dense block, a wave per row.
__global__ __launch_bounds__(256) void nt_solve_level(const NtArgs A, int32_t lev, int32_t upper) {
  const int wv = threadIdx.x >> 6, l64 = threadIdx.x & 63;
  const int32_t *lp = upper ? A.a.lev_ptr_uf : A.a.lev_ptr_f;
  const int32_t *lr = upper ? A.a.lev_rows_uf : A.a.lev_rows_f;
  const int32_t idx = lp[lev] + blockIdx.x * 4 + wv;
  if (idx >= lp[lev + 1]) return;
  if (upper)
    nt_urow(A, A.w.y, lr[idx], l64);
  else
    nt_lrow(A, A.w.y, lr[idx], l64);
}

// Levels lev0 .. lev1 - 1 of one sweep over the rows below the dense block by
// one workgroup, a barrier between levels.  A row takes a group of eight
// lanes (lane j of the group its entries j, j + 8, ...; the rows of a level
// hold few entries), so one pass covers 128 rows of a level.  With LDSY the
// whole vector is copied into LDS first (the rows' reads then wait for LDS
// instead of the L2), and the rows of these levels are written back at the
// end.  A level's rows depend on the vector only through its gathers, so
// each lane loads the descriptor of its first row two levels ahead and that
// row's first entry and column (and, for U, its diagonal) one level ahead:
// every load from a clamped address, so that each level issues the same
// loads and waits only for loads issued a level before.
constexpr int kNtGroup = 8;                                   // lanes per row
constexpr int kNtPassRows = kNtThreads / kNtGroup;            // rows per pass
struct NtRowPre {
  int4 d;   // {row, first entry, entries, diagonal}
  bool ok;  // the lane's group has a row there
  double v, dg;
  int32_t c;
};

template <bool LDSY>
__global__ __launch_bounds__(kNtThreads) void nt_solve_run(const NtArgs A, int32_t lev0, int32_t lev1,
                                                           int32_t upper) {
  extern __shared__ double s_y[];
  const int tid = threadIdx.x, slot = tid / kNtGroup, j = tid % kNtGroup;
  const int32_t *lp = upper ? A.a.lev_ptr_uf : A.a.lev_ptr_f;
  const int4 *D = upper ? A.a.sdesc_u : A.a.sdesc_l;
  double *Y = A.w.y;
  if constexpr (LDSY) {
    for (int32_t i = tid; i < A.a.n_x; i += kNtThreads) s_y[i] = A.w.y[i];
    __syncthreads();
    Y = s_y;
  }
  // the group's row at position first + slot of a level: the descriptor
  auto desc_at = [&](int32_t lev, int32_t first, NtRowPre &p) {
    const int32_t lc = lev < lev1 ? lev : lev1 - 1;
    const int32_t idx = lp[lc] + first + slot;
    p.ok = lev < lev1 && idx < lp[lc + 1];
    p.d = D[p.ok ? idx : lp[lev0]];
  };
  // ... and the lane's first entry (the descriptor loaded before)
  auto vals_of = [&](NtRowPre &p) {
    const bool in = p.ok && j < p.d.z;
    p.v = A.w.lu[in ? p.d.y + j : 0];
    p.c = A.a.lucol[in ? p.d.y + j : 0];
    p.dg = A.w.lu[p.ok && upper ? p.d.w : 0];
  };
  // one row per group: the lane's first entry, then any further ones, the
  // group sum, and the group's first lane writes (every lane takes part)
  auto row = [&](const NtRowPre &p) {
    const int32_t ne = p.ok ? p.d.z : 0;
    double s = j < ne ? p.v * Y[p.c] : 0.0;
    for (int32_t q = kNtGroup + j; q < ne; q += kNtGroup) s += A.w.lu[p.d.y + q] * Y[A.a.lucol[p.d.y + q]];
#pragma unroll
    for (int off = kNtGroup / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (j == 0 && p.ok) Y[p.d.x] = upper ? (Y[p.d.x] - s) / p.dg : Y[p.d.x] - s;
  };
  NtRowPre cur, nxt, nx2;
  desc_at(lev0, 0, cur);
  desc_at(lev0 + 1, 0, nxt);
  vals_of(cur);
  for (int32_t lev = lev0; lev < lev1; ++lev) {
    const NtRowPre p = cur;
    cur = nxt;
    desc_at(lev + 2, 0, nx2);
    vals_of(cur);
    nxt = nx2;
    row(p);
    // further passes of a level with more than a pass of rows, not prefetched
    for (int32_t first = kNtPassRows; lp[lev] + first < lp[lev + 1]; first += kNtPassRows) {
      NtRowPre q;
      desc_at(lev, first, q);
      vals_of(q);
      row(q);
    }
    __syncthreads();
  }
  if constexpr (LDSY) {
    const int32_t *lr = upper ? A.a.lev_rows_uf : A.a.lev_rows_f;
    for (int32_t idx = lp[lev0] + tid; idx < lp[lev1]; idx += kNtThreads) A.w.y[lr[idx]] = s_y[lr[idx]];
  }
}

// The L sweep's block rows, their entries with columns below b0 (the first
// ns of the row; the rest is the dense block's), a wave per row.
__global__ __launch_bounds__(256) void nt_block_lres(const NtArgs A) {
  const int wv = threadIdx.x >> 6, l64 = threadIdx.x & 63;
  const int32_t r = blockIdx.x * 4 + wv;
  if (r >= A.a.m_blk) return;
  const int32_t i = A.a.b0 + r, base = A.a.row_ptr[i], ns = A.a.ns[r];
  double s = 0.0;
  for (int32_t q = l64; q < ns; q += 64) s += A.w.lu[base + q] * A.w.y[A.a.lucol[base + q]];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (l64 == 0) A.w.y[i] -= s;
}

// The dense block's two triangular solves, which follow each other in the
// Newton step: the factors are staged in LDS by the workgroup, then one wave
// substitutes, lane l holding rows l and l + 64, forward with the unit lower
// factor, then backward with the upper factor.  The solved value of each
// step is broadcast by readlane, so the steps wait for no barrier and no
// memory; the backward steps multiply by the stored pivot reciprocals.
static_assert(kNtDenseTop <= 128, "two rows per lane in the dense solve");
__device__ __forceinline__ double nt_lane_bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(kNtThreads) void nt_dense_solve(const NtArgs A) {
  extern __shared__ double s_t[];
  const int32_t m = A.a.m_blk, b0 = A.a.b0, ld = m + 1;
  double *s_rinv = s_t + (int64_t)m * ld;  // the pivot reciprocals
  for (int32_t e = threadIdx.x; e < m * m; e += kNtThreads) s_t[(e / m) * ld + e % m] = A.w.S[e];
  for (int32_t r = threadIdx.x; r < m; r += kNtThreads) s_rinv[r] = A.w.rinv[b0 + r];
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const int l = threadIdx.x;
  const int32_t r0 = l, r1 = l + 64;
  double y0 = r0 < m ? A.w.y[b0 + r0] : 0.0, y1 = r1 < m ? A.w.y[b0 + r1] : 0.0;
  for (int32_t c = 0; c < m; ++c) {
    const double yc = nt_lane_bcast(c < 64 ? y0 : y1, c & 63);
    if (r0 > c && r0 < m) y0 -= s_t[r0 * ld + c] * yc;
    if (r1 > c && r1 < m) y1 -= s_t[r1 * ld + c] * yc;
  }
  for (int32_t c = m - 1; c >= 0; --c) {
    const double xc = nt_lane_bcast(c < 64 ? y0 : y1, c & 63) * s_rinv[c];
    if (r0 == c) y0 = xc;
    if (r1 == c) y1 = xc;
    if (r0 < c) y0 -= s_t[r0 * ld + c] * xc;
    if (r1 < c) y1 -= s_t[r1 * ld + c] * xc;
  }
  if (r0 < m) A.w.y[b0 + r0] = y0;
  if (r1 < m) A.w.y[b0 + r1] = y1;
}

}  // namespace

// ---- host side --------------------------------------------------------------

struct DevNewton {
  int device = -1;
  std::vector<void *> allocs;
  NtArgs args{};
  size_t lds_bytes = 0;
  std::vector<int32_t> row_ptr;  // host copy (unpacking the factors)
  // levels with many rows run as launches of their own over many workgroups,
  // every run of the other levels as one launch of one workgroup
  std::vector<int32_t> lev_rows_f, lev_rows_uf;  // rows per level below the dense block (L, U)
  size_t lds_solve = 0;                          // the dense solve's staged block
  size_t lds_y = 0;  // the vector in LDS for the solves' runs of levels (0: too large, global memory)
};

// A level is wide with at least this many rows: it gets a launch of its own
// (a wave per row over many workgroups) instead of rounds of the one
// workgroup's 16 waves, each row a round.  Below that the launch costs more
// than the rounds: from 64 rows for the refactorisation, whose rows take
// many elimination steps, from 256 for the solves, whose rows take one
// short dot product.
constexpr int32_t kWideRows = 64;
constexpr int32_t kWideSolveRows = 256;
// Largest vector the solves' runs of levels keep in LDS.
constexpr size_t kNtLdsY = 156 * 1024;

namespace {

template <class T>
rh_status nt_up(DevNewton &d, const std::vector<T> &v, const T **out, std::string &err) {
  void *p = nullptr;
  HIP_TRY(hipMalloc(&p, std::max<size_t>(sizeof(T), v.size() * sizeof(T))));
  d.allocs.push_back(p);
  if (!v.empty()) HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<const T *>(p);
  return RH_OK;
}

rh_status nt_alloc(DevNewton &d, size_t n, double **out, std::string &err) {
  void *p = nullptr;
  HIP_TRY(hipMalloc(&p, std::max<size_t>(8, n * sizeof(double))));
  d.allocs.push_back(p);
  *out = static_cast<double *>(p);
  return RH_OK;
}

#define NT_UP(vec, dst)                                  \
  do {                                                   \
    rh_status s_ = nt_up(d, vec, &(dst), err);           \
    if (s_ != RH_OK) return s_;                          \
  } while (0)

rh_status nt_build(Network &net, DevNewton &d, std::string &err) {
  const LuPlan &lu = net.lu;
  const int32_t n = lu.n, m = net.n_br, nb = net.n_bus;
  NtArrays &a = d.args.a;
  a.n_bus = nb;
  a.n_br = m;
  a.n_x = net.n_x;
  a.n_p = net.n_p;
  a.nnz_gx = (int32_t)net.gx.nnz();
  NT_UP(net.br_f, a.br_f);
  NT_UP(net.br_t, a.br_t);
  NT_UP(net.gs, a.gs);
  NT_UP(net.bs, a.bs);
  NT_UP(net.bsh, a.bsh);
  NT_UP(net.th_x, a.th_x);
  NT_UP(net.v_x, a.v_x);
  NT_UP(net.v_p, a.v_p);
  NT_UP(net.pg_p, a.pg_p);
  {
    std::vector<int32_t> ptr(nb + 1, 0), code(2 * (size_t)m);
    for (int32_t b = 0; b < m; ++b) {
      ptr[net.br_f[b] + 1]++;
      ptr[net.br_t[b] + 1]++;
    }
    for (int32_t b = 0; b < nb; ++b) ptr[b + 1] += ptr[b];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int32_t b = 0; b < m; ++b) {
      code[fill[net.br_f[b]]++] = 4 * b;
      code[fill[net.br_t[b]]++] = 4 * b + 2;
    }
    NT_UP(ptr, a.inc_ptr);
    NT_UP(code, a.inc_code);
  }
  {
    // contributions of branch partials to G_x entries, in branch order
    const int64_t nnz = net.gx.nnz();
    std::vector<int32_t> cnt(nnz + 1, 0), src;
    for (size_t q = 0; q < net.gx_slot.size(); ++q)
      if (net.gx_slot[q] >= 0) cnt[net.gx_slot[q] + 1]++;
    for (int64_t s = 0; s < nnz; ++s) cnt[s + 1] += cnt[s];
    src.assign(cnt[nnz], 0);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (size_t q = 0; q < net.gx_slot.size(); ++q)  // q = 16 b + 4 k + var: branch order
      if (net.gx_slot[q] >= 0) src[fill[net.gx_slot[q]]++] = (int32_t)q;
    NT_UP(cnt, a.gxc_ptr);
    NT_UP(src, a.gxc_src);
  }
  {
    LuMaps mp;
    if (!lu_device_maps(lu, net.gx, mp, err)) return RH_EDEVICE;
    if ((size_t)mp.maxpat * sizeof(double) * kNtWaves > 150 * 1024) {
      err = "LU row pattern too wide for the device refactorisation (" + std::to_string(mp.maxpat) + ")";
      return RH_EINVAL;
    }
    a.maxpat = mp.maxpat;
    a.nnz_lu = mp.row_ptr[n];
    NT_UP(mp.row_ptr, a.row_ptr);
    NT_UP(mp.nl, a.nl);
    NT_UP(mp.lucol, a.lucol);
    NT_UP(lu.perm, a.perm);
    NT_UP(mp.a_ptr, a.a_ptr);
    NT_UP(mp.a_src, a.a_src);
    NT_UP(mp.a_dst, a.a_dst);
    NT_UP(mp.upd_ptr, a.upd_ptr);
    NT_UP(mp.tgt, a.tgt);
    {
      std::vector<int4> st(mp.step.size() / 4);
      std::memcpy(st.data(), mp.step.data(), mp.step.size() * sizeof(int32_t));
      NT_UP(st, a.step);
    }
    for (size_t l = 0; l + 1 < mp.lev_ptr_f.size(); ++l) d.lev_rows_f.push_back(mp.lev_ptr_f[l + 1] - mp.lev_ptr_f[l]);
    for (size_t l = 0; l + 1 < mp.lev_ptr_uf.size(); ++l)
      d.lev_rows_uf.push_back(mp.lev_ptr_uf[l + 1] - mp.lev_ptr_uf[l]);
    d.row_ptr = mp.row_ptr;
    a.b0 = mp.b0;
    a.m_blk = n - mp.b0;
    NT_UP(mp.lev_ptr_f, a.lev_ptr_f);
    NT_UP(mp.lev_rows_f, a.lev_rows_f);
    NT_UP(mp.ns, a.ns);
    NT_UP(mp.dmap, a.dmap);
    NT_UP(mp.lev_ptr_uf, a.lev_ptr_uf);
    NT_UP(mp.lev_rows_uf, a.lev_rows_uf);
    {
      // row descriptors of the solves' levels below the dense block
      std::vector<int4> dl(mp.lev_rows_f.size()), du(mp.lev_rows_uf.size());
      for (size_t q = 0; q < dl.size(); ++q) {
        const int32_t i = mp.lev_rows_f[q];
        dl[q] = make_int4(i, mp.row_ptr[i], mp.nl[i], 0);
      }
      for (size_t q = 0; q < du.size(); ++q) {
        const int32_t i = mp.lev_rows_uf[q], ub = mp.row_ptr[i] + mp.nl[i];
        du[q] = make_int4(i, ub + 1, mp.row_ptr[i + 1] - ub - 1, ub);
      }
      if (dl.empty()) dl.push_back(make_int4(0, 0, 0, 0));
      if (du.empty()) du.push_back(make_int4(0, 0, 0, 0));
      NT_UP(dl, a.sdesc_l);
      NT_UP(du, a.sdesc_u);
      // the refactorisation's rows below the dense block
      std::vector<int4> fd(mp.lev_rows_f.size());
      std::vector<int2> fa(mp.lev_rows_f.size());
      for (size_t q = 0; q < fd.size(); ++q) {
        const int32_t i = mp.lev_rows_f[q];
        fd[q] = make_int4(i, mp.row_ptr[i], mp.row_ptr[i + 1] - mp.row_ptr[i], mp.nl[i]);
        fa[q] = make_int2(mp.a_ptr[i], mp.a_ptr[i + 1]);
      }
      if (fd.empty()) {
        fd.push_back(make_int4(0, 0, 0, 0));
        fa.push_back(make_int2(0, 0));
      }
      NT_UP(fd, a.fdesc);
      NT_UP(fa, a.fdesc_a);
    }
    d.lds_solve = ((size_t)a.m_blk * (a.m_blk + 1) + a.m_blk) * sizeof(double);
    d.lds_bytes = (size_t)mp.maxpat * sizeof(double) * kNtWaves;
  }
  NtVectors &w = d.args.w;
  rh_status s;
  if ((s = nt_alloc(d, net.n_x, &w.x, err)) != RH_OK || (s = nt_alloc(d, net.n_p, &w.p, err)) != RH_OK ||
      (s = nt_alloc(d, nb, &w.Pd, err)) != RH_OK || (s = nt_alloc(d, nb, &w.Qd, err)) != RH_OK ||
      (s = nt_alloc(d, nb, &w.th, err)) != RH_OK || (s = nt_alloc(d, nb, &w.v, err)) != RH_OK ||
      (s = nt_alloc(d, 4 * (size_t)m, &w.flows, err)) != RH_OK ||
      (s = nt_alloc(d, 16 * (size_t)m, &w.dG, err)) != RH_OK || (s = nt_alloc(d, net.n_x, &w.g, err)) != RH_OK ||
      (s = nt_alloc(d, a.nnz_gx, &w.gx, err)) != RH_OK || (s = nt_alloc(d, a.nnz_lu, &w.lu, err)) != RH_OK ||
      (s = nt_alloc(d, net.n_x, &w.y, err)) != RH_OK || (s = nt_alloc(d, 4, &w.stat, err)) != RH_OK ||
      (s = nt_alloc(d, net.n_x, &w.rinv, err)) != RH_OK ||
      (s = nt_alloc(d, (size_t)a.m_blk * a.m_blk, &w.S, err)) != RH_OK ||
      (s = nt_alloc(d, a.m_blk, &w.amax, err)) != RH_OK)
    return s;
  if ((s = lds_bound(reinterpret_cast<const void *>(&nt_refactor_run), d.lds_bytes, err)) != RH_OK ||
      (s = lds_bound(reinterpret_cast<const void *>(&nt_dense_solve), d.lds_solve, err)) != RH_OK)
    return s;
  if ((size_t)net.n_x * sizeof(double) <= kNtLdsY) {
    d.lds_y = (size_t)net.n_x * sizeof(double);
    if ((s = lds_bound(reinterpret_cast<const void *>(&nt_solve_run<true>), d.lds_y, err)) != RH_OK) return s;
  }

  return RH_OK;
}

rh_status nt_step_kernels(DevNewton &d, int32_t m, int32_t nb, int32_t nnz_gx, bool jacobian, std::string &err) {
  const int T = 256;
  hipLaunchKernelGGL(nt_state, dim3((nb + T - 1) / T), dim3(T), 0, nullptr, d.args);
  hipLaunchKernelGGL(nt_flows, dim3((m + T - 1) / T), dim3(T), 0, nullptr, d.args, jacobian ? 1 : 0);
  hipLaunchKernelGGL(nt_residual, dim3((nb + T - 1) / T), dim3(T), 0, nullptr, d.args);
  hipLaunchKernelGGL(nt_norm, dim3(1), dim3(kNtThreads), 0, nullptr, d.args);
  if (jacobian) {
    hipLaunchKernelGGL(nt_gx, dim3((nnz_gx + T - 1) / T), dim3(T), 0, nullptr, d.args);
    const size_t lds_w = (size_t)d.args.a.maxpat * sizeof(double) * kNtWideWaves;
    const std::vector<int32_t> &rows = d.lev_rows_f;
    const int32_t nlev = (int32_t)rows.size();
    for (int32_t l = 0; l < nlev;) {
      if (rows[l] >= kWideRows) {
        hipLaunchKernelGGL(nt_refactor_level, dim3((rows[l] + kNtWideWaves - 1) / kNtWideWaves),
                           dim3(64 * kNtWideWaves), lds_w, nullptr, d.args, l);
        ++l;
        continue;
      }
      int32_t l1 = l;
      while (l1 < nlev && rows[l1] < kWideRows) ++l1;
      hipLaunchKernelGGL(nt_refactor_run, dim3(1), dim3(kNtThreads), d.lds_bytes, nullptr, d.args, l, l1);
      l = l1;
    }
    const int32_t mb = d.args.a.m_blk;
    if (mb > 0) {
      hipLaunchKernelGGL(nt_block_rows, dim3((mb + kNtWideWaves - 1) / kNtWideWaves), dim3(64 * kNtWideWaves),
                         lds_w, nullptr, d.args);
      hipLaunchKernelGGL(nt_dense_lu, dim3(1), dim3(kNtThreads), 0, nullptr, d.args);
    }
  }
  HIP_TRY(hipGetLastError());
  return RH_OK;
}

// The Newton step: y = P g, the two sweeps, x -= P^T y.  The L sweep takes
// the rows below the dense block by levels, then the block rows' entries
// with earlier rows, then the block; the U sweep the block first (one kernel
// for the block's two solves), then the rows below it by levels.
rh_status nt_solve_kernels(DevNewton &d, std::string &err) {
  const int T = 256;
  const int32_t n = d.args.a.n_x, mb = d.args.a.m_blk;
  auto levels = [&](const std::vector<int32_t> &rows, int32_t upper) {
    const int32_t nlev = (int32_t)rows.size();
    for (int32_t l = 0; l < nlev;) {
      if (rows[l] >= kWideSolveRows) {
        hipLaunchKernelGGL(nt_solve_level, dim3((rows[l] + 3) / 4), dim3(256), 0, nullptr, d.args, l, upper);
        ++l;
        continue;
      }
      int32_t l1 = l;
      while (l1 < nlev && rows[l1] < kWideSolveRows) ++l1;
      if (d.lds_y)
        hipLaunchKernelGGL(nt_solve_run<true>, dim3(1), dim3(kNtThreads), d.lds_y, nullptr, d.args, l, l1, upper);
      else
        hipLaunchKernelGGL(nt_solve_run<false>, dim3(1), dim3(kNtThreads), 0, nullptr, d.args, l, l1, upper);
      l = l1;
    }
  };
  hipLaunchKernelGGL(nt_permute_in, dim3((n + T - 1) / T), dim3(T), 0, nullptr, d.args);
  levels(d.lev_rows_f, 0);
  if (mb > 0) {
    hipLaunchKernelGGL(nt_block_lres, dim3((mb + 3) / 4), dim3(256), 0, nullptr, d.args);
    hipLaunchKernelGGL(nt_dense_solve, dim3(1), dim3(kNtThreads), d.lds_solve, nullptr, d.args);
  }
  levels(d.lev_rows_uf, 1);
  hipLaunchKernelGGL(nt_update_x, dim3((n + T - 1) / T), dim3(T), 0, nullptr, d.args);
  HIP_TRY(hipGetLastError());
  return RH_OK;
}

}  // namespace

void device_newton_free(Network &net) {
  DevNewton *d = net.dnewton;
  if (!d) return;
  (void)hipSetDevice(d->device);
  (void)hipDeviceSynchronize();
  for (void *p : d->allocs) (void)hipFree(p);
  delete d;
  net.dnewton = nullptr;
}

rh_status device_newton(Network &net, double tol, int32_t max_iter, NewtonResult &res, std::string &err) {
  HIP_TRY(hipSetDevice(net.ctx->device));
  if (!net.dnewton) {
    DevNewton *d = new DevNewton();
    d->device = net.ctx->device;
    net.dnewton = d;
    rh_status s = nt_build(net, *d, err);
    if (s != RH_OK) {
      device_newton_free(net);
      return s;
    }
  }
  DevNewton &d = *net.dnewton;
  NtVectors &w = d.args.w;
  std::vector<double> x(net.n_x, 0.0);
  if ((int32_t)net.x0.size() == net.n_x)
    x = net.x0;
  else
    for (int32_t b : net.pq) x[net.v_x[b]] = 1.0;
  HIP_TRY(hipMemcpy(w.x, x.data(), x.size() * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.p, net.p.data(), net.p.size() * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.Pd, net.Pd.data(), net.Pd.size() * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w.Qd, net.Qd.data(), net.Qd.size() * sizeof(double), hipMemcpyHostToDevice));
  const int32_t m = net.n_br, nb = net.n_bus, nnz_gx = (int32_t)net.gx.nnz();
  double stat[3] = {0.0, 0.0, 0.0};
  double r_prev = std::numeric_limits<double>::infinity();
  int32_t it = 0;
  for (;; ++it) {
    // mismatch at x; with the Jacobian and its factors unless this is the end
    rh_status s = nt_step_kernels(d, m, nb, nnz_gx, true, err);
    if (s != RH_OK) return s;
    HIP_TRY(hipMemcpy(stat, w.stat, sizeof stat, hipMemcpyDeviceToHost));
    res.iters = it;
    res.resid = stat[0];
    if (stat[1] != 0.0) {
      err = "Newton produced a non-finite residual";
      return RH_ENOCONV;
    }
    if (stat[2] != 0.0) {
      err = "G_x is singular to working precision (pivot " + std::to_string((int64_t)stat[2] - 1) + ")";
      return RH_ESINGULAR;
    }
    if (stat[0] <= tol || newton_stalled(it, stat[0], r_prev)) break;
    if (it >= max_iter) {
      err = "Newton did not reach the tolerance in max_iter steps";
      return RH_ENOCONV;
    }
    r_prev = stat[0];
    if ((s = nt_solve_kernels(d, err)) != RH_OK) return s;
  }
  // the accepted state and the factors of G_x there (from the last step's
  // kernels, which ran at this x)
  res.x.resize(net.n_x);
  HIP_TRY(hipMemcpy(res.x.data(), w.x, net.n_x * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> luv(d.row_ptr.back());
  HIP_TRY(hipMemcpy(luv.data(), w.lu, luv.size() * sizeof(double), hipMemcpyDeviceToHost));
  LuPlan &lu = net.lu;
  for (int32_t i = 0; i < lu.n; ++i) {
    const double *r = luv.data() + d.row_ptr[i];
    const size_t nl = lu.lrow[i].size();
    lu.lval[i].assign(r, r + nl);
    lu.uval[i].assign(r + nl, r + nl + lu.urow[i].size());
  }
  return RH_OK;
}

}  // namespace rh
