// Dense FP64 Cholesky factorisation and solves on the device: the dense
// linear system H_t d_t = -g_t of the real-time tracking update (Sec. 6.3,
// eq. (qp_rto)), whose matrix is the reduced Hessian that stays resident in
// HBM after Algorithm 2.
//
// A is column-major, n x n, leading dimension lda; only its lower triangle
// (diagonal included) is read and it is overwritten by L with A = L L^T.
// Right-looking, in panels of kNB columns:
//   chol_panel:  every wave factors the kNB x kNB diagonal block in
//                registers (lanes 0 .. kNB - 1 hold its rows, the pivot
//                column broadcast by readlane) and, with the same
//                broadcasts, solves L_ij L_jj^T = A_ij for 64 - kNB rows of
//                the panel below it (a row on each of the other lanes);
//   chol_update: A_ik -= L_i L_k^T on the lower triangle of the trailing
//                matrix in 64 x 64 tiles, with FP64 MFMA (16 x 16 x 4), in
//                two launches: the tile column that holds the next panel,
//                then the rest together with the next panel's factorisation
//                in workgroups of the same launch (a lookahead of one panel).
// A failed pivot (not positive, or not finite) stores its column + 1 in a
// status word; every later kernel reads it first and does nothing.
// The forward sweep L Y = B rides along: the right-hand sides are extra rows
// of the augmented matrix [A; B^T], substituted in the panels like the rows
// of A and updated by a matrix-vector product per panel, so that at the end
// B holds Y.  chol_back_block then solves L^T X = Y a block of 64 unknowns
// per launch, from the last.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "rh_internal.h"

namespace rh {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kNB = 32;    // panel width
constexpr int kTile = 64;  // trailing-update tile

__device__ __forceinline__ double rdlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1 / sqrt(d) for a pivot d: the hardware reciprocal square root refined by
// two Newton-Raphson steps on f(r) = 1 / r^2 - d (each squares the relative
// error), a shorter dependency chain than a square root and a division.
// Pivots below 2^-900 are scaled by 2^1000 first (exactly, a power of two)
// and the result by 2^500, so that the estimate never sees a denormal.
__device__ __forceinline__ double pivot_rsqrt(double d) {
  const bool tiny = d < 0x1p-900;
  const double ds = tiny ? d * 0x1p+1000 : d;
  double ri = __builtin_amdgcn_rsq(ds);
  for (int it = 0; it < 2; ++it) {
    const double h = ds * ri;
    ri = fma(0.5 * ri, fma(-h, ri, 1.0), ri);
  }
  return tiny ? ri * 0x1p+500 : ri;
}

// Step C of the right-looking factorisation of the diagonal block, whose
// rows lanes 0 .. NB - 1 hold, and of the substitution of the rows the
// other lanes hold, with the same broadcasts: v[c] is entry c of the lane's
// row.  Steps unrolled by recursion so that every index is a compile-time
// constant.  The empty asm statements materialise v[k] at the end of the
// step: the compiler would otherwise sink each chain of updates down to
// step k and keep every broadcast factor entry alive until then (hundreds
// of scalar registers, spilled).
template <int NB, int C>
__device__ __forceinline__ void chol_step(double (&v)[NB], int32_t &bad) {
  if constexpr (C < NB) {
    const double dcc = rdlane(v[C], C);
    if (bad < 0 && !(dcc > 0.0 && dcc <= 1.7976931348623157e308)) bad = C;
    // column C scaled by 1 / sqrt(d_CC); on lane C this gives the pivot
    // d_CC / sqrt(d_CC) itself (within an ulp of sqrt(d_CC))
    v[C] *= pivot_rsqrt(dcc);
#pragma unroll
    for (int k = C + 1; k < NB; ++k) {
      const double lkc = rdlane(v[C], k);  // L(k, C)
      v[k] = fma(-v[C], lkc, v[k]);
    }
#pragma unroll
    for (int k = C + 1; k < NB; ++k) asm volatile("" : "+v"(v[k]));
    chol_step<NB, C + 1>(v, bad);
  }
}

__global__ void dense_clear(int32_t *info) {
  if (threadIdx.x == 0) *info = 0;
}

// F = A (lower triangle) with tau added on the diagonal; columns per block.
__global__ __launch_bounds__(256) void dense_shift_copy(const double *A, int64_t lda, double *F, int64_t ldf,
                                                        int32_t n, double tau) {
  const int32_t j = blockIdx.x;
  for (int32_t i = j + threadIdx.x; i < n; i += 256) {
    const double v = A[i + (int64_t)j * lda];
    F[i + (int64_t)j * ldf] = i == j ? v + tau : v;
  }
}

__global__ __launch_bounds__(256) void dense_diag(const double *A, int64_t lda, int32_t n, double *out) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = A[i + (int64_t)i * lda];
}

__global__ __launch_bounds__(256) void dense_neg(const double *a, double *b, int32_t n) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = -a[i];
}

// Row r of the augmented matrix [A; B^T]: a row of A (r < n) or right-hand
// side r - n, whose entry c is B[c + (r - n) ldb].
__device__ __forceinline__ double *aug_row(double *A, int64_t lda, double *B, int64_t ldb, int32_t n, int32_t r,
                                           int32_t c) {
  return r < n ? A + r + (int64_t)c * lda : B + c + (int64_t)(r - n) * ldb;
}

// Panel j0 for workgroup blk of the panel's launch: every wave factors the
// diagonal block and solves x L^T = row for 64 - NB rows below it (rows of
// A, then the right-hand sides).
template <int NB>
__device__ __forceinline__ void panel_rows(double *A, int64_t lda, int32_t n, double *B, int64_t ldb, int32_t nrhs,
                                           int32_t j0, int32_t blk, int32_t *info) {
  static_assert(NB <= 32, "the diagonal block and the panel rows share a wave");
  if (*info) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t nb = min(NB, n - j0);
  // lanes 0 .. NB - 1: the diagonal block's rows (rows and columns past nb
  // completed by the identity); the other lanes: rows of the panel below it
  const bool dg = lane < NB;
  const int32_t r = j0 + nb + (blk * 4 + wave) * (64 - NB) + (lane - NB);
  const bool has = !dg && r < n + nrhs;
  double v[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    double t = 0.0;
    if (has && c < nb) t = *aug_row(A, lda, B, ldb, n, r, j0 + c);
    if (dg && lane < nb && c < nb && c <= lane) t = A[(j0 + lane) + (int64_t)(j0 + c) * lda];
    if (dg && lane >= nb && c == lane) t = 1.0;
    v[c] = t;
  }
  // The diagonal lanes above the diagonal (lane < column) run the same
  // updates on entries of the upper part, which are never read as L and
  // never stored: no per-lane predicates, whose masks would stay live
  // across the unrolled loop.
  int32_t bad = -1;
  chol_step<NB, 0>(v, bad);
  if (bad >= 0) {
    if (blk == 0 && threadIdx.x == 0) *info = j0 + bad + 1;
    return;
  }
  if (blk == 0 && wave == 0 && dg && lane < nb) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c <= lane) A[(j0 + lane) + (int64_t)(j0 + c) * lda] = v[c];
  }
  if (has) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) *aug_row(A, lda, B, ldb, n, r, j0 + c) = v[c];
  }
}

// Tile (ti, tk), ti >= tk, of the trailing matrix from a linear index.
__device__ __forceinline__ void tri_tile(int32_t b, int32_t &ti, int32_t &tk) {
  int32_t t = (int32_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((int64_t)(t + 1) * (t + 2) / 2 <= b) ++t;
  while ((int64_t)t * (t + 1) / 2 > b) --t;
  ti = t;
  tk = b - (int32_t)((int64_t)t * (t + 1) / 2);
}

// Four waves per 64 x 64 tile, a 32 x 32 quadrant each (2 x 2 MFMA blocks).
// The MFMA forms D = S_k S_i^T from 16 x 4 slabs of the panel, S_k over the
// tile's columns and S_i over its rows, so that D[a][b] is the update of
// A(row b, column a): a lane's four outputs then lie along one column of A
// and 16 lanes store 16 consecutive rows.  Operand layout of
// v_mfma_f64_16x16x4f64 (measured on gfx950): lane l holds A-operand
// (l % 16, l / 16) and B-operand (l / 16, l % 16); output register q of lane
// l is D[4 q + l / 16][l % 16].
// Tiles of workgroup blk: with part kUpdFirst, the first tile column (which
// holds the next panel) and then the right-hand sides; with kUpdRest, the
// tiles right of that column.  Each entry gets the same update either way.
constexpr int kUpdFirst = 1, kUpdRest = 2;

template <int NB>
__device__ __forceinline__ void update_tiles(double *A, int64_t lda, int32_t n, double *B, int64_t ldb,
                                             int32_t nrhs, int32_t j0, int32_t blk, int32_t tiles, int32_t part,
                                             const int32_t *info) {
  if (*info) return;
  if (blk >= tiles) {
    // right-hand-side rows of the augmented matrix: b_col -= sum_c y_c L(col, c)
    // over the trailing columns, y = the panel's entries of the solved rows
    const int32_t col = j0 + NB + (blk - tiles) * 256 + threadIdx.x;
    if (col >= n) return;
    for (int32_t q = 0; q < nrhs; ++q) {
      const double *y = B + (int64_t)q * ldb + j0;
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) acc = fma(A[col + (int64_t)(j0 + c) * lda], y[c], acc);
      B[col + (int64_t)q * ldb] -= acc;
    }
    return;
  }
  int32_t ti, tk;
  if (part == kUpdFirst) {
    ti = blk;
    tk = 0;
  } else {
    tri_tile(blk, ti, tk);
    ++ti, ++tk;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int qi = wave >> 1, qk = wave & 1;
  if (ti == tk && qk > qi) return;  // above the diagonal
  const int32_t j1 = j0 + NB;
  const int32_t r0 = j1 + ti * kTile + qi * 32, c0 = j1 + tk * kTile + qk * 32;
  if (r0 >= n || c0 >= n) return;
  const int li = lane & 15, lk = lane >> 4;
  // the entries this lane updates, loaded with the panel so that the two
  // loads overlap
  double cur[2][2][4];
#pragma unroll
  for (int hk = 0; hk < 2; ++hk)
#pragma unroll
    for (int hi = 0; hi < 2; ++hi)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int32_t row = r0 + 16 * hi + li, col = c0 + 16 * hk + 4 * q + lk;
        cur[hk][hi][q] = (row < n && col < n && row >= col) ? A[row + (int64_t)col * lda] : 0.0;
      }
  v4d acc[2][2];
#pragma unroll
  for (int hk = 0; hk < 2; ++hk)
#pragma unroll
    for (int hi = 0; hi < 2; ++hi) acc[hk][hi] = v4d{0.0, 0.0, 0.0, 0.0};
  double sk[NB / 4][2], si[NB / 4][2];
#pragma unroll
  for (int s = 0; s < NB / 4; ++s) {
    const int64_t col = (int64_t)(j0 + 4 * s + lk) * lda;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t rk = c0 + 16 * h + li, ri = r0 + 16 * h + li;
      sk[s][h] = rk < n ? A[rk + col] : 0.0;
      si[s][h] = ri < n ? A[ri + col] : 0.0;
    }
  }
#pragma unroll
  for (int s = 0; s < NB / 4; ++s)
#pragma unroll
    for (int hk = 0; hk < 2; ++hk)
#pragma unroll
      for (int hi = 0; hi < 2; ++hi)
        acc[hk][hi] = __builtin_amdgcn_mfma_f64_16x16x4f64(sk[s][hk], si[s][hi], acc[hk][hi], 0, 0, 0);
#pragma unroll
  for (int hk = 0; hk < 2; ++hk)
#pragma unroll
    for (int hi = 0; hi < 2; ++hi)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int32_t row = r0 + 16 * hi + li, col = c0 + 16 * hk + 4 * q + lk;
        if (row < n && col < n && row >= col) A[row + (int64_t)col * lda] = cur[hk][hi][q] - acc[hk][hi][q];
      }
}

template <int NB>
__global__ __launch_bounds__(256) void chol_panel(double *A, int64_t lda, int32_t n, double *B, int64_t ldb,
                                                  int32_t nrhs, int32_t j0, int32_t *info) {
  panel_rows<NB>(A, lda, n, B, ldb, nrhs, j0, blockIdx.x, info);
}

// The first tile column of the update of panel j0 and the right-hand sides.
template <int NB>
__global__ __launch_bounds__(256) void chol_update_first(double *A, int64_t lda, int32_t n, double *B, int64_t ldb,
                                                         int32_t nrhs, int32_t j0, int32_t tiles,
                                                         const int32_t *info) {
  update_tiles<NB>(A, lda, n, B, ldb, nrhs, j0, blockIdx.x, tiles, kUpdFirst, info);
}

// The lookahead: panel j0 + NB (whose columns the first tile column has
// made final) in the first pblocks workgroups, and the rest of the update
// of panel j0 in the others, which touch none of its columns.
template <int NB>
__global__ __launch_bounds__(256) void chol_panel_update(double *A, int64_t lda, int32_t n, double *B, int64_t ldb,
                                                         int32_t nrhs, int32_t j0, int32_t pblocks, int32_t tiles,
                                                         int32_t *info) {
  if ((int32_t)blockIdx.x < pblocks)
    panel_rows<NB>(A, lda, n, B, ldb, nrhs, j0 + NB, blockIdx.x, info);
  else
    update_tiles<NB>(A, lda, n, B, ldb, nrhs, j0, (int32_t)blockIdx.x - pblocks, tiles, kUpdRest, info);
}

// L^T x = y, one launch per block of 64 unknowns from the last (the rows of
// B above the block already hold z = y - contributions of the later
// blocks).  Every workgroup solves the block's triangle (staged in LDS,
// wave 0) and then updates its slice of the rows above, right-looking:
// z_r -= sum_c L(j0 + c, r) x_c, whose 64 entries are contiguous in column r.
// Workgroup 0 stores the block's x in X (not in B, whose block rows the
// other workgroups may still be reading).  Columns of B: grid y.
__global__ __launch_bounds__(256) void chol_back_block(const double *A, int64_t lda, int32_t n, double *B,
                                                       int64_t ldb, double *X, int32_t j0, const int32_t *info) {
  if (*info) return;
  __shared__ double s_L[64][65];
  __shared__ double s_rinv[64];
  __shared__ double s_x[64];
  double *z = B + (int64_t)blockIdx.y * ldb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t bs = min(64, n - j0);
  for (int t = threadIdx.x; t < 64 * 64; t += 256) {
    const int i = t & 63, c = t >> 6;  // consecutive threads: consecutive rows of a column
    s_L[i][c] = (i < bs && c < i) ? A[(j0 + i) + (int64_t)(j0 + c) * lda] : 0.0;
  }
  if (threadIdx.x < 64) {
    const int c = threadIdx.x;
    s_rinv[c] = c < bs ? 1.0 / A[(j0 + c) + (int64_t)(j0 + c) * lda] : 0.0;
  }
  __syncthreads();
  if (wave == 0) {
    // lane i: z_i and column i of the strictly lower triangle; right-looking
    // from the last unknown: x_c = z_c / L(c, c) (z_c broadcast), then
    // z_i -= L(c, i) x_c on every lane.  Lane i's z stops changing once c
    // passes i (L(c, i) = 0 for c <= i here), so x_i = z_i / L(i, i) at the end.
    double col[64];
#pragma unroll
    for (int c = 0; c < 64; ++c) col[c] = s_L[c][lane];
    double zv = lane < bs ? z[j0 + lane] : 0.0;
#pragma unroll
    for (int c = 63; c >= 0; --c) {
      const double xc = rdlane(zv, c) * s_rinv[c];
      zv = fma(-col[c], xc, zv);
    }
    const double xv = zv * s_rinv[lane];
    s_x[lane] = xv;
    if (blockIdx.x == 0 && lane < bs) X[(int64_t)blockIdx.y * n + j0 + lane] = xv;
  }
  __syncthreads();
  const int32_t r = (int32_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= j0) return;
  const double *colr = A + j0 + (int64_t)r * lda;  // L(j0 .., r)
  double acc0 = 0.0, acc1 = 0.0;
  int c = 0;
  for (; c + 1 < bs; c += 2) {
    acc0 = fma(colr[c], s_x[c], acc0);
    acc1 = fma(colr[c + 1], s_x[c + 1], acc1);
  }
  if (c < bs) acc0 = fma(colr[c], s_x[c], acc0);
  z[r] -= acc0 + acc1;
}

__global__ __launch_bounds__(256) void dense_copy_cols(const double *X, int32_t n, double *B, int64_t ldb,
                                                       int32_t nrhs) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * nrhs) return;
  const int32_t q = (int32_t)(t / n), i = (int32_t)(t % n);
  B[i + (int64_t)q * ldb] = X[t];
}

}  // namespace

// ---- host side --------------------------------------------------------------

#define DENSE_TRY(expr)                                   \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) {                               \
      err = std::string(#expr) + ": " + hipGetErrorString(e_); \
      return RH_EDEVICE;                                  \
    }                                                     \
  } while (0)

// Right-looking with a lookahead of one panel, two launches per panel
// after the first: the tile column of the trailing update that holds panel
// j0 + kNB (with the right-hand sides), then that panel together with the
// rest of the update, so that the panel's latency overlaps the update.
rh_status dense_cholesky(int32_t n, double *A, int64_t lda, double *B, int64_t ldb, int32_t nrhs, int32_t *dinfo,
                         void *stream, std::string &err) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!B) nrhs = 0;
  auto panel_blocks = [&](int32_t j0) {  // 4 waves of 64 - kNB rows
    const int32_t below = n - j0 - std::min(kNB, n - j0), per = 4 * (64 - kNB);
    return std::max(1, (below + nrhs + per - 1) / per);
  };
  hipLaunchKernelGGL(dense_clear, dim3(1), dim3(64), 0, st, dinfo);
  if (n > 0)
    hipLaunchKernelGGL(chol_panel<kNB>, dim3(panel_blocks(0)), dim3(256), 0, st, A, lda, n, B, ldb, nrhs, 0, dinfo);
  for (int32_t j0 = 0; j0 < n; j0 += kNB) {
    const int32_t below = n - j0 - std::min(kNB, n - j0);
    if (below <= 0) break;  // j0 + kNB exists below
    const int64_t T = (below + kTile - 1) / kTile;
    const int64_t rhs_groups = nrhs > 0 ? (below + 255) / 256 : 0;
    hipLaunchKernelGGL(chol_update_first<kNB>, dim3((uint32_t)(T + rhs_groups)), dim3(256), 0, st, A, lda, n, B,
                       ldb, nrhs, j0, (int32_t)T, (const int32_t *)dinfo);
    const int32_t pb = panel_blocks(j0 + kNB);
    const int64_t rest = (T - 1) * T / 2;
    hipLaunchKernelGGL(chol_panel_update<kNB>, dim3((uint32_t)(pb + rest)), dim3(256), 0, st, A, lda, n, B, ldb,
                       nrhs, j0, pb, (int32_t)rest, dinfo);
  }
  DENSE_TRY(hipGetLastError());
  return RH_OK;
}

rh_status dense_back_solve(int32_t n, const double *L, int64_t ldl, double *B, int64_t ldb, int32_t nrhs,
                           double *work, const int32_t *dinfo, void *stream, std::string &err) {
  if (nrhs <= 0 || n <= 0) return RH_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int32_t j0 = ((n - 1) / 64) * 64; j0 >= 0; j0 -= 64) {
    const uint32_t groups = (uint32_t)std::max(1, (j0 + 255) / 256);
    hipLaunchKernelGGL(chol_back_block, dim3(groups, (uint32_t)nrhs), dim3(256), 0, st, L, ldl, n, B, ldb, work, j0,
                       dinfo);
  }
  const int64_t total = (int64_t)n * nrhs;
  hipLaunchKernelGGL(dense_copy_cols, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, (const double *)work,
                     n, B, ldb, nrhs);
  DENSE_TRY(hipGetLastError());
  return RH_OK;
}

rh_status dense_shift_copy(int32_t n, const double *A, int64_t lda, double *F, int64_t ldf, double tau, void *stream,
                           std::string &err) {
  if (n <= 0) return RH_OK;
  hipLaunchKernelGGL(dense_shift_copy, dim3(n), dim3(256), 0, static_cast<hipStream_t>(stream), A, lda, F, ldf, n,
                     tau);
  DENSE_TRY(hipGetLastError());
  return RH_OK;
}

rh_status dense_diagonal(int32_t n, const double *A, int64_t lda, double *out, void *stream, std::string &err) {
  if (n <= 0) return RH_OK;
  hipLaunchKernelGGL(dense_diag, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), A, lda, n,
                     out);
  DENSE_TRY(hipGetLastError());
  return RH_OK;
}

rh_status dense_negate(int32_t n, const double *a, double *b, void *stream, std::string &err) {
  if (n <= 0) return RH_OK;
  hipLaunchKernelGGL(dense_neg, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), a, b, n);
  DENSE_TRY(hipGetLastError());
  return RH_OK;
}

}  // namespace rh
