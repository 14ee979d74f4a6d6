// Dense FP64 Cholesky factorisation and solves on the device: the dense
// linear system H_t d_t = -g_t of the real-time tracking update (Sec. 6.3,
// eq. (qp_rto)), whose matrix is the reduced Hessian that stays resident in
// HBM after Algorithm 2.
//
// A is column-major, n x n, leading dimension lda; only its lower triangle
// (diagonal included) is read and it is overwritten by L with A = L L^T.
// Right-looking, in panels of kNB columns:
//   chol_panel:  one wave factors the kNB x kNB diagonal block in registers
//                (lane i holds row i, the pivot column broadcast by readlane)
//                into LDS; then every wave solves L_ij L_jj^T = A_ij for 64
//                rows of the panel below it (one row per lane, the factor's
//                entries read from LDS at one address per wave);
//   chol_update: A_ik -= L_i L_k^T on the lower triangle of the trailing
//                matrix in 64 x 64 tiles, with FP64 MFMA (16 x 16 x 4).
// A failed pivot (not positive, or not finite) stores its column + 1 in a
// status word; every later kernel reads it first and does nothing.
// chol_solve then solves L L^T X = B for the columns of B (one workgroup per
// column): the forward sweep right-looking (the update of the rows below a
// block reads columns of L, contiguous), the backward sweep left-looking (a
// block's unknowns take dot products of columns of L with the finished part).
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

// Optimisation barrier: the values v[c + 1 ..] are materialised here.  In
// the unrolled right-looking steps below, the compiler would otherwise sink
// each v[k]'s chain of updates down to step k and keep every broadcast
// factor entry alive until then (hundreds of scalar registers, spilled).
template <int NB>
__device__ __forceinline__ void pin_after(double (&v)[NB], int c) {
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (k > c) asm volatile("" : "+v"(v[k]));
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

template <int NB>
__global__ __launch_bounds__(256) void chol_panel(double *A, int64_t lda, int32_t n, int32_t j0, int32_t *info) {
  if (*info) return;
  __shared__ double s_L[NB][NB + 1];
  __shared__ double s_rinv[NB];
  __shared__ int32_t s_bad;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t nb = min(NB, n - j0);
  if (wave == 0) {
    // the diagonal block, rows and columns past nb completed by the identity
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double v = 0.0;
      if (lane < nb && c < nb && c <= lane) v = A[(j0 + lane) + (int64_t)(j0 + c) * lda];
      if (lane >= nb && lane < NB && c == lane) v = 1.0;
      a[c] = v;
    }
    // Lanes above the diagonal (lane < column) run the same updates on
    // entries of the upper part, which are never read as L and are zeroed
    // below: no per-lane predicates, whose masks would otherwise stay live
    // across the whole unrolled loop.
    int32_t bad = -1;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const double dcc = rdlane(a[c], c);
      if (bad < 0 && !(dcc > 0.0 && dcc <= 1.7976931348623157e308)) bad = c;
      // column c scaled by 1 / sqrt(d_cc); on lane c this gives the pivot
      // d_cc / sqrt(d_cc) itself (within an ulp of sqrt(d_cc))
      const double ri = 1.0 / sqrt(dcc);
      a[c] *= ri;
      if (lane == 0) s_rinv[c] = ri;
#pragma unroll
      for (int k = c + 1; k < NB; ++k) a[k] = fma(-a[c], rdlane(a[c], k), a[k]);  // L(k, c)
      pin_after<NB>(a, c);
    }
    if (lane < NB) {
#pragma unroll
      for (int c = 0; c < NB; ++c) s_L[lane][c] = c <= lane ? a[c] : 0.0;
    }
    if (lane == 0) s_bad = bad;
    if (blockIdx.x == 0) {
      if (bad >= 0) {
        if (lane == 0) *info = j0 + bad + 1;
      } else if (lane < nb) {
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c <= lane) A[(j0 + lane) + (int64_t)(j0 + c) * lda] = a[c];
      }
    }
  }
  __syncthreads();
  if (s_bad >= 0) return;
  const int32_t r = j0 + nb + (blockIdx.x * 4 + wave) * 64 + lane;
  if (r >= n) return;
  double x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = c < nb ? A[r + (int64_t)(j0 + c) * lda] : 0.0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    x[c] *= s_rinv[c];
#pragma unroll
    for (int k = c + 1; k < NB; ++k) x[k] = fma(-x[c], s_L[k][c], x[k]);
    pin_after<NB>(x, c);
  }
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c < nb) A[r + (int64_t)(j0 + c) * lda] = x[c];
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
template <int NB>
__global__ __launch_bounds__(256) void chol_update(double *A, int64_t lda, int32_t n, int32_t j0,
                                                   const int32_t *info) {
  if (*info) return;
  int32_t ti, tk;
  tri_tile(blockIdx.x, ti, tk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int qi = wave >> 1, qk = wave & 1;
  if (ti == tk && qk > qi) return;  // above the diagonal
  const int32_t j1 = j0 + NB;
  const int32_t r0 = j1 + ti * kTile + qi * 32, c0 = j1 + tk * kTile + qk * 32;
  if (r0 >= n || c0 >= n) return;
  const int li = lane & 15, lk = lane >> 4;
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
        if (row < n && col < n && row >= col) A[row + (int64_t)col * lda] -= acc[hk][hi][q];
      }
}

// L L^T x = b for one column of B per workgroup (1024 threads).  The 64 x 64
// diagonal blocks are staged in LDS and solved by wave 0, a row per lane.
constexpr int kSolveThreads = 1024;
constexpr int kSolveWaves = kSolveThreads / 64;

__device__ __forceinline__ void stage_block(const double *A, int64_t lda, int32_t j0, int32_t bs,
                                            double (*s_L)[65]) {
  for (int t = threadIdx.x; t < 64 * 64; t += kSolveThreads) {
    const int i = t & 63, c = t >> 6;  // consecutive threads: consecutive rows of a column
    s_L[i][c] = (i < bs && c <= i) ? A[(j0 + i) + (int64_t)(j0 + c) * lda] : 0.0;
  }
}

__global__ __launch_bounds__(kSolveThreads) void chol_solve(const double *A, int64_t lda, int32_t n, double *B,
                                                            int64_t ldb, const int32_t *info) {
  if (*info) return;
  double *y = B + (int64_t)blockIdx.x * ldb;
  __shared__ double s_L[64][65];
  __shared__ double s_blk[64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // forward: L y = b
  for (int32_t j0 = 0; j0 < n; j0 += 64) {
    const int32_t bs = min(64, n - j0);
    stage_block(A, lda, j0, bs, s_L);
    __syncthreads();
    if (wave == 0) {
      double v = lane < bs ? y[j0 + lane] : 0.0;
      for (int c = 0; c < bs; ++c) {
        if (lane == c) v = v / s_L[c][c];
        const double vc = __shfl(v, c);
        if (lane > c) v = fma(-s_L[lane][c], vc, v);
      }
      if (lane < bs) {
        y[j0 + lane] = v;
        s_blk[lane] = v;
      }
    }
    __syncthreads();
    // rows below: y_r -= sum_c L(r, j0 + c) y_{j0 + c}
    for (int32_t r = j0 + bs + threadIdx.x; r < n; r += kSolveThreads) {
      double acc = 0.0;
      for (int c = 0; c < bs; ++c) acc = fma(A[r + (int64_t)(j0 + c) * lda], s_blk[c], acc);
      y[r] -= acc;
    }
    __syncthreads();
  }
  // backward: L^T x = y, blocks from the last
  const int32_t nblk = (n + 63) / 64;
  for (int32_t bk = nblk - 1; bk >= 0; --bk) {
    const int32_t j0 = bk * 64, bs = min(64, n - j0), j1 = j0 + bs;
    stage_block(A, lda, j0, bs, s_L);
    // z_c = y_c - sum_{r >= j1} L(r, c) x_r for the block's columns c: wave w
    // takes columns w, w + 16, ...; lanes stride the rows
    for (int c = wave; c < bs; c += kSolveWaves) {
      double acc = 0.0;
      const double *col = A + (int64_t)(j0 + c) * lda;
      for (int32_t r = j1 + lane; r < n; r += 64) acc = fma(col[r], y[r], acc);
      for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
      if (lane == 0) s_blk[c] = acc;
    }
    __syncthreads();
    if (wave == 0) {
      const double z = lane < bs ? y[j0 + lane] - s_blk[lane] : 0.0;
      double xv = 0.0;
      // x_c = (z_c - sum_{i > c} L(i, c) x_i) / L(c, c), c descending
      for (int c = bs - 1; c >= 0; --c) {
        double t = lane > c ? s_L[lane][c] * xv : 0.0;
        for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
        if (lane == c) xv = (z - t) / s_L[c][c];
      }
      if (lane < bs) y[j0 + lane] = xv;
    }
    __syncthreads();
  }
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

rh_status dense_cholesky(int32_t n, double *A, int64_t lda, int32_t *dinfo, void *stream, std::string &err) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(dense_clear, dim3(1), dim3(64), 0, st, dinfo);
  for (int32_t j0 = 0; j0 < n; j0 += kNB) {
    const int32_t nb = std::min(kNB, n - j0), below = n - j0 - nb;
    const int32_t blocks = std::max(1, (below + 255) / 256);
    hipLaunchKernelGGL(chol_panel<kNB>, dim3(blocks), dim3(256), 0, st, A, lda, n, j0, dinfo);
    if (below > 0) {
      const int64_t T = (below + kTile - 1) / kTile, tiles = T * (T + 1) / 2;
      hipLaunchKernelGGL(chol_update<kNB>, dim3((uint32_t)tiles), dim3(256), 0, st, A, lda, n, j0,
                         (const int32_t *)dinfo);
    }
  }
  DENSE_TRY(hipGetLastError());
  return RH_OK;
}

rh_status dense_solve(int32_t n, const double *L, int64_t ldl, double *B, int64_t ldb, int32_t nrhs,
                      const int32_t *dinfo, void *stream, std::string &err) {
  if (nrhs <= 0 || n <= 0) return RH_OK;
  hipLaunchKernelGGL(chol_solve, dim3(nrhs), dim3(kSolveThreads), 0, static_cast<hipStream_t>(stream), L, ldl, n,
                     B, ldb, dinfo);
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
