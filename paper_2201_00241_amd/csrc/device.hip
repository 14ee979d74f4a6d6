// Device path of librh: the batched adjoint-adjoint reduction on gfx950.
//
// One launch processes a block of k directions W (Sec. 4.3, Algorithm 2).
// The directions are independent, so each workgroup owns C of them and runs
// every step of the reduction for its directions ("direction-owned" scheme):
//
//   1. SpMul            B' = -P G_p W                        (row-parallel)
//   2. BatchSparseSolve Z' = U^{-1} L^{-1} B'                (level-scheduled)
//   3. BatchTensorProjection (Sec. 4.2, forward-over-reverse of the branch
//      flows): every bus sums the second-order terms of its incident branches
//      (gather form of the "edges, then nodes" accumulation: no atomics), plus
//      the slack-cost rank-one term and the 2 c2 diagonal of the generator
//      costs.  The x part is written negated as the right-hand side of
//      step 4, the p part straight into the output.
//   4. BatchSparseSolve (transposed)  Psi' = L^{-T} U^{-T} (-P Y_x)
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
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "rh_internal.h"

namespace rh {

namespace {

constexpr int kThreads = 512;      // global-vector variant (several workgroups per CU)
constexpr int kThreadsLds = 1024;  // LDS variant (one workgroup per CU at 10k buses)
// lanes x rows budget used to pick a level's lane-group size (fixed, so the
// schedule never depends on the launch shape)
constexpr int kLaneBudget = 512;

constexpr int kBlockRows = 64;  // rows of a merged block of narrow levels (one wave)

struct DevSweep {
  int32_t n_levels;  // steps
  // per step: first position, row count, log2 lanes per row, offset of the
  // block's dense inverse (-1: a plain level)
  const int4 *lev;
  const int32_t *rows, *ptr, *col;
  const double *val, *dinv;  // dinv == nullptr: unit diagonal
  const double *dense;       // block inverses
};

struct NetDesc {
  int32_t n_x, n_p, n_bus, n_pg, n_slack;
  DevSweep L, U, Ut, Lt;
  const int32_t *gp_ptr, *gp_col;  // G_p, rows in permuted x order
  const double *gp_val;
  const int32_t *gpt_ptr, *gpt_col;  // G_p^T, columns in permuted x order
  const double *gpt_val;
  // bus tangent sources: theta from X[thx] (-1: reference, zero tangent);
  // v from X[vs] if vs >= 0, else from W[-vs - 1] (generator magnitude)
  const int32_t *bus_thx, *bus_vs;
  const int32_t *inc_ptr, *inc_othx, *inc_ovs;  // incidences, other end's sources
  const double *inc_K, *inc_Hps, *inc_H, *inc_A2, *inc_vo;
  const double *bus_v, *bus_sth, *bus_sv;
  const int32_t *slack_thx, *slack_vs;
  const double *slack_gth, *slack_gv;
  const int32_t *pg_idx;
  const double *pg_c2x2;
};

struct BlockArgs {
  int32_t k;              // directions in this launch
  int32_t identity_from;  // >= 0: W is columns identity_from.. of the identity
  const double *W;
  int64_t ldw;
  double *HW;
  int64_t ldhw;
  double *scratch;
  int64_t scratch_stride;  // doubles per workgroup
  long long *stamps;       // kStamps wall-clock stamps per workgroup, or nullptr
};

constexpr int kStamps = 8;

__device__ __forceinline__ double w_at(const BlockArgs &a, int32_t q, int32_t dir) {
  if (dir >= a.k) return 0.0;
  if (a.identity_from >= 0) return (q == a.identity_from + dir) ? 1.0 : 0.0;
  return a.W[(int64_t)dir * a.ldw + q];
}

// Registers holding one row of a level: its position, entry range, the first
// kPre entries of this lane, the matrix row and the reciprocal pivot.  Loaded
// one level ahead, so that the dependent global loads leave the critical path
// of the sweep (they do not depend on the solution vector).
constexpr int kPre = 4;
struct RowPre {
  int32_t pos, q0, q1, row;
  int32_t col[kPre];
  double val[kPre];
  double dinv;
};

__device__ __forceinline__ RowPre prefetch_row(const DevSweep &s, const int4 m, int32_t r, int lane,
                                               int width) {
  RowPre p;
  p.pos = -1;
  if (r < m.y) {
    p.pos = m.x + r;
    p.q0 = s.ptr[p.pos];
    p.q1 = s.ptr[p.pos + 1];
    p.row = s.rows[p.pos];
    p.dinv = s.dinv ? s.dinv[p.pos] : 1.0;
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
      const int32_t q = p.q0 + lane + i * width;
      p.col[i] = q < p.q1 ? s.col[q] : 0;
      p.val[i] = q < p.q1 ? s.val[q] : 0.0;
    }
  }
  return p;
}

// One row: new value = (init - sum_j val_j X_j) * dinv, summed by a lane
// group of `width` lanes and combined by a shuffle butterfly.  Rows of a block
// step only form the residual (no pivot) into s_r at their place in the block.
template <int C, int NT>
__device__ __forceinline__ void row_update(const DevSweep &s, const RowPre &p, double *__restrict__ X,
                                           const double *__restrict__ init, double *__restrict__ s_r,
                                           int32_t first, bool block, int lane, int width) {
  double part[C];
#pragma unroll
  for (int c = 0; c < C; ++c) part[c] = 0.0;
#pragma unroll
  for (int i = 0; i < kPre; ++i) {
    const int32_t j = p.col[i] * C;
#pragma unroll
    for (int c = 0; c < C; ++c) part[c] = fma(p.val[i], X[j + c], part[c]);
  }
  for (int32_t q = p.q0 + lane + kPre * width; q < p.q1; q += width) {
    const double v = s.val[q];
    const int32_t j = s.col[q] * C;
#pragma unroll
    for (int c = 0; c < C; ++c) part[c] = fma(v, X[j + c], part[c]);
  }
  for (int off = width >> 1; off > 0; off >>= 1) {
#pragma unroll
    for (int c = 0; c < C; ++c) part[c] += __shfl_xor(part[c], off);
  }
  if (lane == 0) {
    const int32_t i = p.row * C;
    if (block) {
      const int32_t a = (p.pos - first) * C;
#pragma unroll
      for (int c = 0; c < C; ++c) s_r[a + c] = (init ? init[i + c] : X[i + c]) - part[c];
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double v = (init ? init[i + c] : X[i + c]) - part[c];
        if (s.dinv) v *= p.dinv;
        X[i + c] = v;
      }
    }
  }
}

// Level-scheduled triangular sweep on X (rows of C directions).
//
// A step is either one dependency level (its rows are independent) or a block
// of consecutive narrow levels (at most kBlockRows rows in all).  For a block
// the host has split each row's entries into those reaching rows solved in
// earlier steps (kept in the CSR arrays) and those inside the block, and
// stored the dense inverse M^{-1} of the block's own triangular system
// (column-major, kBlockRows x kBlockRows at most).  A block is then solved in
// two parallel phases: residuals r = init - (external part), then x = M^{-1} r.
template <int C, int NT>
__device__ __forceinline__ void sweep(const DevSweep &s, double *__restrict__ X,
                                      const double *__restrict__ init, double *__restrict__ s_r,
                                      int tid) {
  const int32_t nl = s.n_levels;
  if (nl == 0) return;
  int4 m = s.lev[0];
  int lg = m.z;
  RowPre pre = prefetch_row(s, m, tid >> lg, tid & ((1 << lg) - 1), 1 << lg);
  for (int32_t lev = 0; lev < nl; ++lev) {
    const int4 cur = m;
    const int width = 1 << lg;
    const int lane = tid & (width - 1);
    const RowPre first = pre;
    if (lev + 1 < nl) {  // next step's first rows, issued before this step's work
      m = s.lev[lev + 1];
      lg = m.z;
      pre = prefetch_row(s, m, tid >> lg, tid & ((1 << lg) - 1), 1 << lg);
    }
    const bool block = cur.w >= 0;
    if (first.pos >= 0) {
      row_update<C, NT>(s, first, X, init, s_r, cur.x, block, lane, width);
      for (int32_t r = (tid >> cur.z) + (NT >> cur.z); r < cur.y; r += (NT >> cur.z)) {
        const RowPre p = prefetch_row(s, cur, r, lane, width);
        row_update<C, NT>(s, p, X, init, s_r, cur.x, block, lane, width);
      }
    }
    __syncthreads();
    if (block) {
      if (tid < cur.y) {
        const double *__restrict__ Mi = s.dense + cur.w;
        double acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0.0;
        for (int32_t b = 0; b <= tid; ++b) {
          const double v = Mi[tid + b * cur.y];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] = fma(v, s_r[b * C + c], acc[c]);
        }
        const int32_t i = s.rows[cur.x + tid] * C;
#pragma unroll
        for (int c = 0; c < C; ++c) X[i + c] = acc[c];
      }
      __syncthreads();
    }
  }
}

template <int C, int NT>
__device__ __forceinline__ void reduction(const NetDesc &nd, const BlockArgs &a, double *__restrict__ X,
                                          double *__restrict__ Yx, double *s_slack, double *s_r,
                                          int32_t dir0) {
  const int tid = threadIdx.x;
  // optional phase timestamps (first chunk of each workgroup, thread 0)
  long long *st = (a.stamps && dir0 == (int32_t)blockIdx.x * C && tid == 0)
                      ? a.stamps + (int64_t)blockIdx.x * kStamps : nullptr;
  if (st) st[0] = wall_clock64();
  // 1. B' = -P G_p W
  for (int32_t i = tid; i < nd.n_x; i += NT) {
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    for (int32_t e = nd.gp_ptr[i]; e < nd.gp_ptr[i + 1]; ++e) {
      const double v = nd.gp_val[e];
      const int32_t q = nd.gp_col[e];
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = fma(v, w_at(a, q, dir0 + c), acc[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) X[i * C + c] = -acc[c];
  }
  __syncthreads();
  if (st) st[1] = wall_clock64();
  // 2. Z' = U^{-1} L^{-1} B'
  sweep<C, NT>(nd.L, X, nullptr, s_r, tid);
  if (st) st[2] = wall_clock64();
  sweep<C, NT>(nd.U, X, nullptr, s_r, tid);
  if (st) st[3] = wall_clock64();
  // 3a. slack-cost rank-one term: s = grad P_ref . tangent
  if (tid < C) {
    const int c = tid;
    double s = 0.0;
    for (int32_t q = 0; q < nd.n_slack; ++q) {
      const int32_t tx = nd.slack_thx[q], vs = nd.slack_vs[q];
      const double dth = tx >= 0 ? X[tx * C + c] : 0.0;
      const double dv = vs >= 0 ? X[vs * C + c] : w_at(a, -vs - 1, dir0 + c);
      s += nd.slack_gth[q] * dth + nd.slack_gv[q] * dv;
    }
    s_slack[c] = s;
  }
  __syncthreads();
  // 3b. per-bus gather of the branch second-order terms
  for (int32_t e = tid; e < nd.n_bus; e += NT) {
    const int32_t tx = nd.bus_thx[e], vs = nd.bus_vs[e];
    const double ve = nd.bus_v[e], sth = nd.bus_sth[e], sv = nd.bus_sv[e];
    double dte[C], dve[C], yth[C], yv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      dte[c] = tx >= 0 ? X[tx * C + c] : 0.0;
      dve[c] = vs >= 0 ? X[vs * C + c] : w_at(a, -vs - 1, dir0 + c);
      yth[c] = sth * s_slack[c];
      yv[c] = sv * s_slack[c];
    }
    for (int32_t q = nd.inc_ptr[e]; q < nd.inc_ptr[e + 1]; ++q) {
      const int32_t ot = nd.inc_othx[q], ov = nd.inc_ovs[q];
      const double K = nd.inc_K[q], hps = nd.inc_Hps[q], H = nd.inc_H[q], A2 = nd.inc_A2[q];
      const double vo = nd.inc_vo[q];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const double dto = ot >= 0 ? X[ot * C + c] : 0.0;
        const double dvo = ov >= 0 ? X[ov * C + c] : w_at(a, -ov - 1, dir0 + c);
        const double dd = dte[c] - dto;
        yth[c] += -K * dd + hps * (vo * dve[c] + ve * dvo);
        yv[c] += hps * vo * dd + A2 * dve[c] + H * dvo;
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (tx >= 0) Yx[tx * C + c] = -yth[c];
      if (vs >= 0)
        Yx[vs * C + c] = -yv[c];
      else if (dir0 + c < a.k)
        a.HW[(int64_t)(dir0 + c) * a.ldhw + (-vs - 1)] = yv[c];
    }
  }
  for (int32_t g = tid; g < nd.n_pg; g += NT) {
    const int32_t q = nd.pg_idx[g];
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (dir0 + c < a.k) a.HW[(int64_t)(dir0 + c) * a.ldhw + q] = nd.pg_c2x2[g] * w_at(a, q, dir0 + c);
  }
  __syncthreads();
  if (st) st[4] = wall_clock64();
  // 4. Psi' = L^{-T} U^{-T} (-P Y_x)
  sweep<C, NT>(nd.Ut, X, Yx, s_r, tid);
  if (st) st[5] = wall_clock64();
  sweep<C, NT>(nd.Lt, X, nullptr, s_r, tid);
  if (st) st[6] = wall_clock64();
  // 5. H W = Y_p + G_p^T Psi
  for (int32_t q = tid; q < nd.n_p; q += NT) {
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    for (int32_t e = nd.gpt_ptr[q]; e < nd.gpt_ptr[q + 1]; ++e) {
      const double v = nd.gpt_val[e];
      const int32_t j = nd.gpt_col[e] * C;
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = fma(v, X[j + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (dir0 + c < a.k) a.HW[(int64_t)(dir0 + c) * a.ldhw + q] += acc[c];
  }
  __syncthreads();
  if (st) st[7] = wall_clock64();
}

// X in LDS (dynamic shared memory of n_x * C doubles); Y_x in global scratch.
template <int C>
__global__ __launch_bounds__(kThreadsLds) void block_kernel_lds(const NetDesc nd, const BlockArgs a) {
  extern __shared__ double smem[];
  __shared__ double s_slack[C];
  __shared__ double s_r[kBlockRows * C];
  double *Yx = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;
  const int32_t n_chunks = (a.k + C - 1) / C;
  for (int32_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x)
    reduction<C, kThreadsLds>(nd, a, smem, Yx, s_slack, s_r, chunk * C);
}

// X and Y_x in global scratch (networks whose vector does not fit in LDS).
template <int C>
__global__ __launch_bounds__(kThreads) void block_kernel_global(const NetDesc nd, const BlockArgs a) {
  __shared__ double s_slack[C];
  __shared__ double s_r[kBlockRows * C];
  double *Yx = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;
  double *X = Yx + (int64_t)nd.n_x * C;
  const int32_t n_chunks = (a.k + C - 1) / C;
  for (int32_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x)
    reduction<C, kThreads>(nd, a, X, Yx, s_slack, s_r, chunk * C);
}

}  // namespace

// ----------------------------------------------------------------- device net
struct DeviceNet {
  NetDesc nd{};
  std::vector<void *> allocs;
  double *scratch = nullptr;
  size_t scratch_bytes = 0;
  int32_t n_sms = 0;
  size_t lds_max = 0;  // dynamic LDS a workgroup may use
  // start/stop events of the launches of the current call (timing on)
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  // in-kernel phase stamps of the last launch (timing level 2)
  long long *stamps = nullptr;
  int32_t stamps_cap = 0, stamps_groups = 0;
  double wall_khz = 0.0;
};

namespace {

#define HIP_TRY(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
      return RH_EDEVICE;                                                       \
    }                                                                          \
  } while (0)

template <class T>
rh_status upload(DeviceNet &dn, const std::vector<T> &v, const T **out, std::string &err) {
  if (v.empty()) {
    *out = nullptr;
    return RH_OK;
  }
  void *p = nullptr;
  HIP_TRY(hipMalloc(&p, v.size() * sizeof(T)));
  dn.allocs.push_back(p);
  HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<const T *>(p);
  return RH_OK;
}

#define UP(vec, dst)                                            \
  do {                                                          \
    rh_status s_ = upload(*dn, vec, &(dst), err);               \
    if (s_ != RH_OK) return s_;                                 \
  } while (0)

rh_status upload_sweep(DeviceNet *dn, const Sweep &s, int32_t n, int bmax, DevSweep &o,
                       std::string &err) {
  const Schedule sc = build_schedule(s, n, bmax, kBlockRows, kLaneBudget);
  o.n_levels = (int32_t)(sc.meta.size() / 4);
  const int32_t *mp = nullptr;
  UP(sc.meta, mp);
  o.lev = reinterpret_cast<const int4 *>(mp);
  UP(sc.s.rows, o.rows);
  UP(sc.s.ptr, o.ptr);
  UP(sc.s.col, o.col);
  UP(sc.s.val, o.val);
  o.dinv = nullptr;
  if (!sc.s.dinv.empty()) UP(sc.s.dinv, o.dinv);
  o.dense = nullptr;
  if (!sc.dense.empty()) UP(sc.dense, o.dense);
  return RH_OK;
}

}  // namespace

rh_status device_set(int32_t device, std::string &err) {
  HIP_TRY(hipSetDevice(device));
  return RH_OK;
}

void device_free(Network &net) {
  if (!net.dev) return;
  (void)hipDeviceSynchronize();
  for (void *p : net.dev->allocs) (void)hipFree(p);
  if (net.dev->scratch) (void)hipFree(net.dev->scratch);
  for (hipEvent_t e : net.dev->ev) (void)hipEventDestroy(e);
  if (net.dev->stamps) (void)hipFree(net.dev->stamps);
  delete net.dev;
  net.dev = nullptr;
}

void device_take_timing(Network &net) {
  if (net.dev) net.dev->ev_used = 0;
  net.report.last_launches = 0;
}

rh_status device_kernel_ms(Network &net, double *ms_out, std::string &err) {
  *ms_out = -1.0;
  DeviceNet *dn = net.dev;
  if (!dn) return RH_OK;
  if (dn->stamps_groups > 0 && dn->wall_khz > 0) {
    std::vector<long long> st((size_t)dn->stamps_groups * kStamps);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(st.data(), dn->stamps, st.size() * sizeof(long long), hipMemcpyDeviceToHost));
    for (int p = 0; p < 7; ++p) {
      double sum = 0.0;
      for (int32_t g = 0; g < dn->stamps_groups; ++g)
        sum += (double)(st[(size_t)g * kStamps + p + 1] - st[(size_t)g * kStamps + p]);
      net.report.phase_us[p] = sum / dn->stamps_groups / dn->wall_khz * 1e3;
    }
    dn->stamps_groups = 0;
  }
  if (dn->ev_used == 0) return RH_OK;
  double sum = 0.0;
  for (size_t i = 0; i + 1 < dn->ev_used; i += 2) {
    HIP_TRY(hipEventSynchronize(dn->ev[i + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, dn->ev[i], dn->ev[i + 1]));
    sum += ms;
  }
  *ms_out = sum;
  return RH_OK;
}

rh_status device_upload(Network &net, std::string &err) {
  HIP_TRY(hipSetDevice(net.ctx->device));
  size_t keep_bytes = 0;
  double *keep = nullptr;
  if (net.dev) {  // keep the scratch buffer across operating points
    keep = net.dev->scratch;
    keep_bytes = net.dev->scratch_bytes;
    net.dev->scratch = nullptr;
    device_free(net);
  }
  DeviceNet *dn = new DeviceNet();
  net.dev = dn;
  dn->scratch = keep;
  dn->scratch_bytes = keep_bytes;
  int cus = 0, lds_a = 0, lds_b = 0, wkhz = 0;
  HIP_TRY(hipDeviceGetAttribute(&wkhz, hipDeviceAttributeWallClockRate, net.ctx->device));
  dn->wall_khz = wkhz;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, net.ctx->device));
  HIP_TRY(hipDeviceGetAttribute(&lds_a, hipDeviceAttributeMaxSharedMemoryPerBlock, net.ctx->device));
  HIP_TRY(hipDeviceGetAttribute(&lds_b, hipDeviceAttributeSharedMemPerBlockOptin, net.ctx->device));
  dn->n_sms = cus;
  // leave room for the kernel's static LDS (the slack scalars)
  dn->lds_max = (size_t)std::max(lds_a, lds_b) > 256 ? (size_t)std::max(lds_a, lds_b) - 256 : 0;

  NetDesc &nd = dn->nd;
  const LuPlan &lu = net.lu;
  nd.n_x = net.n_x;
  nd.n_p = net.n_p;
  nd.n_bus = net.n_bus;

  Sweep sl, su, sut, slt;
  lu_sweeps(lu, sl, su, sut, slt);
  int bmax = kBlockRows;
  if (const char *e = std::getenv("RH_BLOCK_ROWS")) bmax = std::min(kBlockRows, std::max(0, std::atoi(e)));
  const int32_t n = net.n_x;
  if (upload_sweep(dn, sl, n, bmax, nd.L, err) != RH_OK ||
      upload_sweep(dn, su, n, bmax, nd.U, err) != RH_OK ||
      upload_sweep(dn, sut, n, bmax, nd.Ut, err) != RH_OK ||
      upload_sweep(dn, slt, n, bmax, nd.Lt, err) != RH_OK)
    return RH_EDEVICE;
  net.report.steps_l = nd.L.n_levels;
  net.report.steps_u = nd.U.n_levels;

  // G_p with rows in permuted order, and G_p^T with permuted columns
  {
    std::vector<int32_t> ptr(net.n_x + 1, 0), col;
    std::vector<double> val;
    for (int32_t ip = 0; ip < net.n_x; ++ip) {
      const int32_t r = lu.perm[ip];
      for (int32_t e = net.gp.ptr[r]; e < net.gp.ptr[r + 1]; ++e) {
        col.push_back(net.gp.col[e]);
        val.push_back(net.gp.val[e]);
      }
      ptr[ip + 1] = (int32_t)col.size();
    }
    UP(ptr, nd.gp_ptr);
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
    UP(tptr, nd.gpt_ptr);
    UP(tcol, nd.gpt_col);
    UP(tval, nd.gpt_val);
  }
  // tangent sources per bus in permuted numbering: theta from X[thx] (-1 at
  // the reference bus); v from X[vs] at PQ buses, else from W[-vs - 1]
  std::vector<int32_t> thx(net.n_bus), vs(net.n_bus);
  for (int32_t b = 0; b < net.n_bus; ++b) {
    thx[b] = net.th_x[b] >= 0 ? lu.iperm[net.th_x[b]] : -1;
    vs[b] = net.v_x[b] >= 0 ? lu.iperm[net.v_x[b]] : -net.v_p[b] - 1;
  }
  UP(thx, nd.bus_thx);
  UP(vs, nd.bus_vs);
  const Tape &tp = net.tape;
  {
    std::vector<int32_t> oth(tp.inc_other.size()), ovs(tp.inc_other.size());
    for (size_t q = 0; q < tp.inc_other.size(); ++q) {
      oth[q] = thx[tp.inc_other[q]];
      ovs[q] = vs[tp.inc_other[q]];
    }
    UP(oth, nd.inc_othx);
    UP(ovs, nd.inc_ovs);
  }
  UP(tp.inc_ptr, nd.inc_ptr);
  UP(tp.inc_K, nd.inc_K);
  UP(tp.inc_Hps, nd.inc_Hps);
  UP(tp.inc_H, nd.inc_H);
  UP(tp.inc_A2, nd.inc_A2);
  UP(tp.inc_vo, nd.inc_vo);
  UP(tp.bus_v, nd.bus_v);
  UP(tp.bus_sth, nd.bus_sth);
  UP(tp.bus_sv, nd.bus_sv);
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
  {
    std::vector<int32_t> idx;
    std::vector<double> c2;
    for (int32_t b : net.pv) {
      idx.push_back(net.pg_p[b]);
      c2.push_back(2.0 * net.c2[net.gen_of_bus[b]]);
    }
    nd.n_pg = (int32_t)idx.size();
    UP(idx, nd.pg_idx);
    UP(c2, nd.pg_c2x2);
  }
  HIP_TRY(hipDeviceSynchronize());
  return RH_OK;
}

namespace {

template <int C>
rh_status launch(bool lds, int32_t groups, size_t lds_bytes, hipStream_t s, const NetDesc &nd,
                 const BlockArgs &a, std::string &err) {
  if constexpr (C <= 4) {
    if (lds) {
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&block_kernel_lds<C>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
      hipLaunchKernelGGL(block_kernel_lds<C>, dim3(groups), dim3(kThreadsLds), lds_bytes, s, nd, a);
      HIP_TRY(hipGetLastError());
      return RH_OK;
    }
  }
  hipLaunchKernelGGL(block_kernel_global<C>, dim3(groups), dim3(kThreads), 0, s, nd, a);
  HIP_TRY(hipGetLastError());
  return RH_OK;
}

// Directions per workgroup: more share each factor entry, fewer keep the chip
// busy.  Take the largest C (<= 8) that still gives two workgroups per CU
// and whose vector fits the LDS budget (the LDS variant).  The result does
// not change any direction's arithmetic.
int32_t choose_c(int32_t k, int32_t cus, int64_t n_x, size_t lds_max, bool lds) {
  if (const char *e = std::getenv("RH_DIRS_PER_GROUP")) {
    const int v = std::atoi(e);
    if ((v == 1 || v == 2 || v == 4 || (v == 8 && !lds)) && (!lds || (size_t)n_x * v * 8 <= lds_max))
      return v;
  }
  int32_t c = lds ? 4 : 8;  // (8 directions x 1024 threads would spill registers)
  while (c > 1 && ((int64_t)k < (int64_t)c * 2 * cus || (lds && (size_t)n_x * c * 8 > lds_max)))
    c >>= 1;
  return c;
}

}  // namespace

rh_status device_hvp(Network &net, int32_t k, const double *dW, int64_t ldw, double *dHW,
                     int64_t ldhw, int32_t identity_from, void *stream, std::string &err) {
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
  const bool lds = (size_t)net.n_x * 8 <= dn->lds_max && !std::getenv("RH_NO_LDS");
  const int32_t C = choose_c(k, dn->n_sms, net.n_x, dn->lds_max, lds);
  const int32_t n_chunks = (k + C - 1) / C;
  // per-workgroup scratch: Y_x (and X when it is not in LDS), 256-byte aligned
  const int64_t stride = ((lds ? 1LL : 2LL) * net.n_x * C + 31) / 32 * 32;
  const int64_t max_groups_mem = std::max<int64_t>(1, (int64_t(8) << 30) / (stride * 8));
  const int64_t per_cu = lds ? 1 : 4;
  const int32_t groups = (int32_t)std::min<int64_t>({(int64_t)n_chunks, max_groups_mem,
                                                     (int64_t)dn->n_sms * 8 * per_cu});
  const size_t need = (size_t)groups * stride * sizeof(double);
  if (need > dn->scratch_bytes) {
    // the buffer may still be in use by earlier work on the same stream
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    if (dn->scratch) HIP_TRY(hipFree(dn->scratch));
    dn->scratch = nullptr;
    dn->scratch_bytes = 0;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, need));
    dn->scratch = (double *)p;
    dn->scratch_bytes = need;
  }
  BlockArgs a;
  a.k = k;
  a.identity_from = identity_from;
  a.W = dW;
  a.ldw = ldw;
  a.HW = dHW;
  a.ldhw = ldhw;
  a.scratch = dn->scratch;
  a.scratch_stride = stride;
  a.stamps = nullptr;
  if (net.ctx->timing >= 2) {
    if (dn->stamps_cap < groups) {
      HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
      if (dn->stamps) HIP_TRY(hipFree(dn->stamps));
      dn->stamps = nullptr;
      dn->stamps_cap = 0;
      HIP_TRY(hipMalloc(&dn->stamps, (size_t)groups * kStamps * sizeof(long long)));
      dn->stamps_cap = groups;
    }
    a.stamps = dn->stamps;
    dn->stamps_groups = groups;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (net.ctx->timing) {
    while (dn->ev.size() < dn->ev_used + 2) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      dn->ev.push_back(e);
    }
    e0 = dn->ev[dn->ev_used];
    e1 = dn->ev[dn->ev_used + 1];
    dn->ev_used += 2;
    HIP_TRY(hipEventRecord(e0, s));
  }
  const size_t lds_bytes = lds ? (size_t)net.n_x * C * sizeof(double) : 0;
  rh_status st;
  switch (C) {
    case 1: st = launch<1>(lds, groups, lds_bytes, s, dn->nd, a, err); break;
    case 2: st = launch<2>(lds, groups, lds_bytes, s, dn->nd, a, err); break;
    case 4: st = launch<4>(lds, groups, lds_bytes, s, dn->nd, a, err); break;
    default: st = launch<8>(lds, groups, lds_bytes, s, dn->nd, a, err); break;
  }
  if (st != RH_OK) return st;
  net.report.last_launches += 1;
  net.report.dirs_per_group = C;
  if (net.ctx->timing) HIP_TRY(hipEventRecord(e1, s));
  return RH_OK;
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
