// Device path of librh: the batched adjoint-adjoint reduction on gfx950.
//
// One launch processes a block of k directions W (Sec. 4.3, Algorithm 2).
// The directions are independent, so the launch hands each workgroup C of
// them ("direction-owned" scheme) and the workgroup runs every step of the
// reduction for its directions:
//
//   1. SpMul            B' = -P G_p W                        (row-parallel)
//   2. BatchSparseSolve Z' = U^{-1} L^{-1} B'                (level-scheduled)
//   3. BatchTensorProjection (Sec. 4.2, forward-over-reverse of the branch
//      flows): tangents are gathered into bus space, every bus sums the
//      second-order terms of its incident branches (gather form of the
//      "edges, then nodes" accumulation: no atomics), plus the slack-cost
//      rank-one term and the 2 c2 diagonal of the generator costs.  The x
//      part is written negated as the right-hand side of step 4, the p part
//      straight into the output.
//   4. BatchSparseSolve (transposed)  Psi' = L^{-T} U^{-T} (-P Y_x)
//   5. SpMulAdd         H W = Y_p + G_p^T Psi
//
// Vectors in x space live in the permuted (factor) numbering, so no
// permutation pass is needed.  Dependencies between triangular-sweep levels
// only ever cross threads of the same workgroup, so a workgroup barrier is the
// only synchronisation: no inter-workgroup flags, no grid barrier, and the
// arithmetic of a direction does not depend on k, C or the workgroup it lands
// on (bitwise block-size invariance).
//
// Per-workgroup scratch (global memory, L2/MALL resident): X1 and X2 (n_x x C)
// and the bus-space tangents (2 n_bus x C), each row holding the C directions
// contiguously.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "rh_internal.h"

namespace rh {

namespace {

constexpr int kThreads = 256;

struct DevSweep {
  int32_t n_levels;
  const int32_t *lev_ptr, *rows, *ptr, *col;
  const double *val, *dinv;  // dinv == nullptr: unit diagonal
};

struct NetDesc {
  int32_t n_x, n_p, n_bus, n_pg, n_slack;
  DevSweep L, U, Ut, Lt;
  const int32_t *gp_ptr, *gp_col;  // G_p, rows in permuted x order
  const double *gp_val;
  const int32_t *gpt_ptr, *gpt_col;  // G_p^T, columns in permuted x order
  const double *gpt_val;
  const int32_t *bus_thx, *bus_vx, *bus_vp;  // bus -> permuted x index / p index (-1 none)
  const int32_t *inc_ptr, *inc_other;
  const double *inc_K, *inc_Hps, *inc_H, *inc_A2, *inc_vo;
  const double *bus_v, *bus_sth, *bus_sv;
  const int32_t *slack_bus;
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
};

template <int C>
__device__ __forceinline__ double w_at(const BlockArgs &a, int32_t q, int32_t dir) {
  if (a.identity_from >= 0) return (q == a.identity_from + dir) ? 1.0 : 0.0;
  return a.W[(int64_t)dir * a.ldw + q];
}

// Level-scheduled triangular sweep, in place on X (rows of C directions).
template <int C>
__device__ __forceinline__ void sweep(const DevSweep &s, double *__restrict__ X, int slot, int d,
                                      bool active) {
  for (int32_t lev = 0; lev < s.n_levels; ++lev) {
    const int32_t b = s.lev_ptr[lev], e = s.lev_ptr[lev + 1];
    if (active) {
      for (int32_t pos = b + slot; pos < e; pos += kThreads / C) {
        const int32_t i = s.rows[pos];
        double acc = X[i * C + d];
        const int32_t q0 = s.ptr[pos], q1 = s.ptr[pos + 1];
        for (int32_t q = q0; q < q1; ++q) acc -= s.val[q] * X[s.col[q] * C + d];
        if (s.dinv) acc *= s.dinv[pos];
        X[i * C + d] = acc;
      }
    }
    __syncthreads();
  }
}

template <int C>
__global__ __launch_bounds__(kThreads) void block_kernel(const NetDesc nd, const BlockArgs a) {
  const int tid = threadIdx.x;
  const int d = tid % C;
  const int slot = tid / C;
  constexpr int kRowsPerPass = kThreads / C;
  __shared__ double s_slack[C];
  double *__restrict__ X1 = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;
  double *__restrict__ X2 = X1 + (int64_t)nd.n_x * C;
  double *__restrict__ Dth = X2 + (int64_t)nd.n_x * C;
  double *__restrict__ Dv = Dth + (int64_t)nd.n_bus * C;
  const int32_t n_chunks = (a.k + C - 1) / C;

  for (int32_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    const int32_t dir = chunk * C + d;
    const bool active = dir < a.k;
    double *__restrict__ hw = a.HW + (int64_t)(active ? dir : 0) * a.ldhw;

    // 1. B' = -P G_p W
    if (active) {
      for (int32_t i = slot; i < nd.n_x; i += kRowsPerPass) {
        double acc = 0.0;
        for (int32_t e = nd.gp_ptr[i]; e < nd.gp_ptr[i + 1]; ++e)
          acc -= nd.gp_val[e] * w_at<C>(a, nd.gp_col[e], dir);
        X1[i * C + d] = acc;
      }
    }
    __syncthreads();
    // 2. Z' = U^{-1} L^{-1} B'
    sweep<C>(nd.L, X1, slot, d, active);
    sweep<C>(nd.U, X1, slot, d, active);
    // 3a. tangents in bus space
    if (active) {
      for (int32_t b = slot; b < nd.n_bus; b += kRowsPerPass) {
        const int32_t tx = nd.bus_thx[b], vx = nd.bus_vx[b];
        Dth[b * C + d] = tx >= 0 ? X1[tx * C + d] : 0.0;
        Dv[b * C + d] = vx >= 0 ? X1[vx * C + d] : w_at<C>(a, nd.bus_vp[b], dir);
      }
    }
    __syncthreads();
    // 3b. slack-cost rank-one term: s = grad P_ref . tangent
    if (tid < C) {
      double s = 0.0;
      if (chunk * C + tid < a.k) {
        for (int32_t q = 0; q < nd.n_slack; ++q) {
          const int32_t b = nd.slack_bus[q];
          s += nd.slack_gth[q] * Dth[b * C + tid] + nd.slack_gv[q] * Dv[b * C + tid];
        }
      }
      s_slack[tid] = s;
    }
    __syncthreads();
    // 3c. per-bus gather of the branch second-order terms
    if (active) {
      const double s = s_slack[d];
      for (int32_t e = slot; e < nd.n_bus; e += kRowsPerPass) {
        const double dte = Dth[e * C + d], dve = Dv[e * C + d], ve = nd.bus_v[e];
        double yth = nd.bus_sth[e] * s, yv = nd.bus_sv[e] * s;
        for (int32_t q = nd.inc_ptr[e]; q < nd.inc_ptr[e + 1]; ++q) {
          const int32_t o = nd.inc_other[q];
          const double dd = dte - Dth[o * C + d];
          const double dvo = Dv[o * C + d];
          const double vo = nd.inc_vo[q], hps = nd.inc_Hps[q];
          yth += -nd.inc_K[q] * dd + hps * (vo * dve + ve * dvo);
          yv += hps * vo * dd + nd.inc_A2[q] * dve + nd.inc_H[q] * dvo;
        }
        const int32_t tx = nd.bus_thx[e], vx = nd.bus_vx[e];
        if (tx >= 0) X2[tx * C + d] = -yth;
        if (vx >= 0)
          X2[vx * C + d] = -yv;
        else
          hw[nd.bus_vp[e]] = yv;
      }
      for (int32_t g = slot; g < nd.n_pg; g += kRowsPerPass) {
        const int32_t q = nd.pg_idx[g];
        hw[q] = nd.pg_c2x2[g] * w_at<C>(a, q, dir);
      }
    }
    __syncthreads();
    // 4. Psi' = L^{-T} U^{-T} (-P Y_x)
    sweep<C>(nd.Ut, X2, slot, d, active);
    sweep<C>(nd.Lt, X2, slot, d, active);
    // 5. H W = Y_p + G_p^T Psi
    if (active) {
      for (int32_t q = slot; q < nd.n_p; q += kRowsPerPass) {
        double acc = 0.0;
        for (int32_t e = nd.gpt_ptr[q]; e < nd.gpt_ptr[q + 1]; ++e)
          acc += nd.gpt_val[e] * X2[nd.gpt_col[e] * C + d];
        hw[q] += acc;
      }
    }
    __syncthreads();
  }
}

}  // namespace

// ----------------------------------------------------------------- device net
struct DeviceNet {
  NetDesc nd{};
  std::vector<void *> allocs;
  double *scratch = nullptr;
  size_t scratch_bytes = 0;
  int32_t n_sms = 0;
  // start/stop events of the launches of the current call (timing on)
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
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

rh_status upload_sweep(DeviceNet *dn, const Sweep &s, DevSweep &o, std::string &err) {
  o.n_levels = s.n_levels();
  UP(s.lev_ptr, o.lev_ptr);
  UP(s.rows, o.rows);
  UP(s.ptr, o.ptr);
  UP(s.col, o.col);
  UP(s.val, o.val);
  o.dinv = nullptr;
  if (!s.dinv.empty()) UP(s.dinv, o.dinv);
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
  if (!dn || dn->ev_used == 0) return RH_OK;
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
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, net.ctx->device));
  dn->n_sms = cus;

  NetDesc &nd = dn->nd;
  const LuPlan &lu = net.lu;
  nd.n_x = net.n_x;
  nd.n_p = net.n_p;
  nd.n_bus = net.n_bus;

  Sweep sl, su, sut, slt;
  lu_sweeps(lu, sl, su, sut, slt);
  if (upload_sweep(dn, sl, nd.L, err) != RH_OK || upload_sweep(dn, su, nd.U, err) != RH_OK ||
      upload_sweep(dn, sut, nd.Ut, err) != RH_OK || upload_sweep(dn, slt, nd.Lt, err) != RH_OK)
    return RH_EDEVICE;

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
  // bus maps in permuted numbering
  {
    std::vector<int32_t> thx(net.n_bus), vx(net.n_bus);
    for (int32_t b = 0; b < net.n_bus; ++b) {
      thx[b] = net.th_x[b] >= 0 ? lu.iperm[net.th_x[b]] : -1;
      vx[b] = net.v_x[b] >= 0 ? lu.iperm[net.v_x[b]] : -1;
    }
    UP(thx, nd.bus_thx);
    UP(vx, nd.bus_vx);
    UP(net.v_p, nd.bus_vp);
  }
  const Tape &tp = net.tape;
  UP(tp.inc_ptr, nd.inc_ptr);
  UP(tp.inc_other, nd.inc_other);
  UP(tp.inc_K, nd.inc_K);
  UP(tp.inc_Hps, nd.inc_Hps);
  UP(tp.inc_H, nd.inc_H);
  UP(tp.inc_A2, nd.inc_A2);
  UP(tp.inc_vo, nd.inc_vo);
  UP(tp.bus_v, nd.bus_v);
  UP(tp.bus_sth, nd.bus_sth);
  UP(tp.bus_sv, nd.bus_sv);
  nd.n_slack = (int32_t)tp.slack_bus.size();
  UP(tp.slack_bus, nd.slack_bus);
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

// Directions per workgroup: more directions share each factor entry, fewer
// workgroups share the chip.  Keep at least two workgroups per CU when k allows.
int32_t choose_c(int32_t k, int32_t cus) {
  if (const char *e = std::getenv("RH_DIRS_PER_GROUP")) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4 || v == 8) return v;
  }
  if (k >= 8 * 2 * cus) return 8;
  if (k >= 4 * 2 * cus) return 4;
  if (k >= 2 * 2 * cus) return 2;
  return 1;
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
  const int32_t C = choose_c(k, dn->n_sms);
  const int32_t n_chunks = (k + C - 1) / C;
  // scratch per workgroup, padded to 256 bytes
  const int64_t stride = ((2LL * net.n_x + 2LL * net.n_bus) * C + 31) / 32 * 32;
  const int64_t max_groups_mem = std::max<int64_t>(1, (int64_t(8) << 30) / (stride * 8));
  const int32_t groups = (int32_t)std::min<int64_t>({(int64_t)n_chunks, max_groups_mem,
                                                     (int64_t)dn->n_sms * 16});
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
  switch (C) {
    case 1: hipLaunchKernelGGL(block_kernel<1>, dim3(groups), dim3(kThreads), 0, s, dn->nd, a); break;
    case 2: hipLaunchKernelGGL(block_kernel<2>, dim3(groups), dim3(kThreads), 0, s, dn->nd, a); break;
    case 4: hipLaunchKernelGGL(block_kernel<4>, dim3(groups), dim3(kThreads), 0, s, dn->nd, a); break;
    default: hipLaunchKernelGGL(block_kernel<8>, dim3(groups), dim3(kThreads), 0, s, dn->nd, a); break;
  }
  HIP_TRY(hipGetLastError());
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
