// Real-time tracking update on the device (Sec. 6.3, eq.
// (nonlinearoptreduced_time) and eq. (qp_rto)), and the dense SPD solve it
// is built on.
//
// With the network solved at (p_t, w_t):
//   Step 1: g_t = grad_p F (eq. (reduced_gradient)) and H_t = d2 F by
//           Algorithm 2 on the columns of the identity, both into device
//           workspace owned by the network;
//   Step 2: (H_t + tau I) d_t = -g_t by the dense Cholesky factorisation on
//           the device, tau = 0 whenever H_t is positive definite (the
//           paper's step); otherwise the smallest tau of a doubling sequence
//           whose factorisation succeeds (Cholesky with an added multiple of
//           the identity, Nocedal and Wright, Numerical Optimization,
//           Algorithm 3.3);
//   then p_{t+1} = p_t + d_t, projected on the caller's bounds and ramp
//   limits.
// H_t never leaves the device; the host reads the diagonal (for tau), the
// pivot status, g_t and d_t (n_p values each).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "rh_internal.h"

namespace rh {

struct DevTrack {
  int device = -1;
  int32_t n_p = 0;
  double *H = nullptr, *F = nullptr, *g = nullptr, *d = nullptr, *diag = nullptr;
  int32_t *info = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

#define TR_TRY(expr)                                                           \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
      return RH_EDEVICE;                                                       \
    }                                                                          \
  } while (0)

#define TR_OK(expr)                  \
  do {                               \
    rh_status s_ = (expr);           \
    if (s_ != RH_OK) return s_;      \
  } while (0)

// Factorisations tried before the shift is given up.
constexpr int kMaxTries = 64;
// beta of the shift sequence, relative to max_i |H_ii|.
constexpr double kBetaRel = 1e-3;

rh_status track_alloc(Network &net, DevTrack *&t, std::string &err) {
  if (net.dtrack && net.dtrack->n_p == net.n_p && net.dtrack->device == net.ctx->device) {
    t = net.dtrack;
    return RH_OK;
  }
  device_track_free(net);
  t = new DevTrack();
  net.dtrack = t;
  t->device = net.ctx->device;
  t->n_p = net.n_p;
  const size_t n = (size_t)std::max(1, net.n_p);
  TR_TRY(hipMalloc(&t->H, n * n * sizeof(double)));
  TR_TRY(hipMalloc(&t->F, n * n * sizeof(double)));
  TR_TRY(hipMalloc(&t->g, n * sizeof(double)));
  TR_TRY(hipMalloc(&t->d, n * sizeof(double)));
  TR_TRY(hipMalloc(&t->diag, n * sizeof(double)));
  TR_TRY(hipMalloc(&t->info, sizeof(int32_t)));
  for (hipEvent_t &e : t->ev) TR_TRY(hipEventCreate(&e));
  return RH_OK;
}

}  // namespace

void device_track_free(Network &net) {
  DevTrack *t = net.dtrack;
  if (!t) return;
  (void)hipSetDevice(t->device);
  (void)hipDeviceSynchronize();
  for (void *p : {(void *)t->H, (void *)t->F, (void *)t->g, (void *)t->d, (void *)t->diag, (void *)t->info})
    if (p) (void)hipFree(p);
  for (hipEvent_t e : t->ev)
    if (e) (void)hipEventDestroy(e);
  delete t;
  net.dtrack = nullptr;
}

rh_status dense_spd_solve(int device, int32_t n, double *A, int64_t lda, double *B, int64_t ldb, int32_t nrhs,
                          void *stream, int32_t &failed_col, std::string &err) {
  TR_TRY(hipSetDevice(device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t *info = nullptr;
  double *work = nullptr;
  TR_TRY(hipMalloc(&info, sizeof(int32_t)));
  {
    hipError_t e = hipMalloc(&work, std::max<size_t>(1, (size_t)n * std::max(1, nrhs)) * sizeof(double));
    if (e != hipSuccess) {
      (void)hipFree(info);
      err = std::string("dense solve workspace: ") + hipGetErrorString(e);
      return RH_ENOMEM;
    }
  }
  rh_status s = dense_cholesky(n, A, lda, B, ldb, nrhs, info, stream, err);
  if (s == RH_OK) s = dense_back_solve(n, A, lda, B, ldb, nrhs, work, info, stream, err);
  int32_t h = 0;
  if (s == RH_OK) {
    hipError_t e = hipMemcpyAsync(&h, info, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      err = std::string("dense solve: ") + hipGetErrorString(e);
      s = RH_EDEVICE;
    }
  }
  if (s != RH_OK) (void)hipStreamSynchronize(st);  // the launches may still use the buffers
  (void)hipFree(info);
  (void)hipFree(work);
  failed_col = h > 0 ? h - 1 : -1;
  return s;
}

rh_status tracking_step(Network &net, int32_t k_block, double shift, const double *lo, const double *hi,
                        const double *ramp, double *dd, void *stream, rh_tracking_info &out, std::string &err) {
  TR_TRY(hipSetDevice(net.ctx->device));
  DevTrack *t = nullptr;
  TR_OK(track_alloc(net, t, err));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t n = net.n_p;
  TR_TRY(hipEventRecord(t->ev[0], st));
  TR_OK(device_reduced_gradient(net, t->g, stream, err));
  TR_TRY(hipEventRecord(t->ev[1], st));
  TR_OK(reduced_hessian_into(net, t->H, n, k_block, RH_FP64, stream, err));
  TR_TRY(hipEventRecord(t->ev[2], st));
  // tau_0 from the diagonal
  TR_OK(dense_diagonal(n, t->H, n, t->diag, stream, err));
  std::vector<double> dg(n), gh(n), dh(n);
  TR_TRY(hipMemcpyAsync(dg.data(), t->diag, n * sizeof(double), hipMemcpyDeviceToHost, st));
  TR_TRY(hipMemcpyAsync(gh.data(), t->g, n * sizeof(double), hipMemcpyDeviceToHost, st));
  TR_TRY(hipStreamSynchronize(st));
  double dmin = std::numeric_limits<double>::infinity(), dmax = 0.0, ginf = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    if (!std::isfinite(dg[i]) || !std::isfinite(gh[i])) {
      err = "non-finite reduced Hessian or gradient";
      return RH_ENOCONV;
    }
    dmin = std::min(dmin, dg[i]);
    dmax = std::max(dmax, std::fabs(dg[i]));
    ginf = std::max(ginf, std::fabs(gh[i]));
  }
  double beta = kBetaRel * dmax;
  if (beta == 0.0) beta = kBetaRel;
  double tau = (n == 0 || dmin + shift > 0.0) ? shift : -dmin + beta;
  int32_t tries = 0, bad = 0;
  for (;;) {
    ++tries;
    TR_OK(dense_shift_copy(n, t->H, n, t->F, n, tau, stream, err));
    TR_OK(dense_negate(n, t->g, t->d, stream, err));
    TR_OK(dense_cholesky(n, t->F, n, t->d, n, 1, t->info, stream, err));
    TR_TRY(hipMemcpyAsync(&bad, t->info, sizeof bad, hipMemcpyDeviceToHost, st));
    TR_TRY(hipStreamSynchronize(st));
    if (bad == 0) break;
    if (tries >= kMaxTries) {
      err = "no diagonal shift made the reduced Hessian positive definite";
      return RH_ESINGULAR;
    }
    tau = std::max(2.0 * tau, beta);
  }
  TR_OK(dense_back_solve(n, t->F, n, t->d, n, 1, t->diag, t->info, stream, err));
  TR_TRY(hipEventRecord(t->ev[3], st));
  if (dd && n > 0) TR_TRY(hipMemcpyAsync(dd, t->d, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  TR_TRY(hipMemcpyAsync(dh.data(), t->d, n * sizeof(double), hipMemcpyDeviceToHost, st));
  TR_TRY(hipStreamSynchronize(st));
  float ms[3] = {0.f, 0.f, 0.f};
  for (int i = 0; i < 3; ++i) TR_TRY(hipEventElapsedTime(&ms[i], t->ev[i], t->ev[i + 1]));
  double dinf = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    if (!std::isfinite(dh[i])) {
      err = "non-finite tracking step";
      return RH_ENOCONV;
    }
    dinf = std::max(dinf, std::fabs(dh[i]));
  }
  out.tau = tau;
  out.tries = tries;
  out.pad = 0;
  out.grad_inf = ginf;
  out.step_inf = dinf;
  out.ms_gradient = ms[0];
  out.ms_hessian = ms[1];
  out.ms_solve = ms[2];
  // p_{t+1}: p_t + d_t within the ramp limits and the bounds
  for (int32_t q = 0; q < n; ++q) {
    double v = net.p[q] + dh[q];
    if (ramp) v = std::min(std::max(v, net.p[q] - ramp[q]), net.p[q] + ramp[q]);
    if (lo) v = std::max(v, lo[q]);
    if (hi) v = std::min(v, hi[q]);
    net.p[q] = v;
  }
  // the next solve starts from this operating point's state
  net.x0 = net.x;
  net.solved = false;
  return RH_OK;
}

}  // namespace rh
