// C ABI entry points of librh (declared in include/rh.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "rh_internal.h"

using namespace rh;

namespace {

thread_local std::string g_err;

rh_status fail(rh_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

#define GUARD_BEGIN try {
#define GUARD_END                                             \
  }                                                           \
  catch (const std::bad_alloc &) {                            \
    return fail(RH_ENOMEM, "host allocation failed");         \
  }                                                           \
  catch (const std::exception &ex) {                          \
    return fail(RH_EINVAL, std::string("exception: ") + ex.what()); \
  }                                                           \
  catch (...) {                                               \
    return fail(RH_EINVAL, "unknown exception");              \
  }

bool finite_n(const double *a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

rh_status need_solved(const rh_network *net) {
  if (!net) return fail(RH_EINVAL, "null network");
  if (!net->n.solved) return fail(RH_ESTATE, "no converged power flow for the current parameters");
  return RH_OK;
}

rh_status need_device(rh_network *net) {
  if (net->n.ctx->device < 0) return fail(RH_EDEVICE, "host-only context");
  return RH_OK;
}

void invalidate(Network &n) {
  n.solved = false;
}

}  // namespace

namespace rh {
rh_status reduced_hessian_into(Network &n, double *H, int64_t ldh, int32_t k_block, rh_precision prec,
                               void *hip_stream, std::string &err) {
  const int32_t n_p = n.n_p;
  rh_status s = RH_OK;
  int32_t k = k_block > n_p ? n_p : k_block;
  int32_t group = 1;
  if (k_block == 0) {
    // the tuned shape: its k is the launch size
    rh_tile &t = n.tile[prec == RH_FP64 ? 0 : 1];
    if (t.k == 0) {
      rh_tile tt{};
      if ((s = autotune(n, prec, 0, tt, err)) != RH_OK) return s;
    }
    k = std::min(t.k, n_p);
  } else {
    // consecutive blocks share a launch when one block leaves CUs idle at
    // the directions per workgroup the network allows (a direction's product
    // does not depend on the launch it runs in)
    const int32_t want = device_launch_dirs(n, prec);
    group = std::max(1, std::min((want + k - 1) / k, (n_p + k - 1) / k));
  }
  n.report.last_k = k;
  for (int32_t j0 = 0; j0 < n_p; j0 += group * k) {
    const int32_t kb = std::min(group * k, n_p - j0);
    s = device_hvp(n, kb, nullptr, 0, H + (int64_t)j0 * ldh, ldh, j0, prec, hip_stream, err);
    if (s != RH_OK) return s;
  }
  if (prec == RH_FP32_REFINED) n.refined_cols = n_p;
  return RH_OK;
}
}  // namespace rh

extern "C" {

const char *rh_status_string(rh_status s) {
  switch (s) {
    case RH_OK: return "ok";
    case RH_EINVAL: return "invalid argument";
    case RH_ENOMEM: return "out of memory";
    case RH_ENOCONV: return "Newton did not converge";
    case RH_ESINGULAR: return "singular Jacobian";
    case RH_ESTATE: return "call out of order";
    case RH_EDEVICE: return "device error";
    case RH_EBUSY: return "busy";
  }
  return "unknown status";
}

const char *rh_last_error(void) { return g_err.c_str(); }

rh_status rh_context_create(int32_t device, rh_context **out) {
  GUARD_BEGIN
  if (!out) return fail(RH_EINVAL, "null out");
  *out = nullptr;
  if (device < -1) return fail(RH_EINVAL, "device must be >= -1");
  if (device >= 0) {
    std::string err;
    rh_status s = device_set(device, err);
    if (s == RH_OK) s = device_fixed_scratch_init(device, err);
    if (s != RH_OK) return fail(s, err);
  }
  rh_context *c = new rh_context();
  c->c.device = device;
  *out = c;
  return RH_OK;
  GUARD_END
}

rh_status rh_context_destroy(rh_context *ctx) {
  if (!ctx) return RH_OK;
  device_ctx_free(ctx->c);
  delete ctx;
  return RH_OK;
}

rh_status rh_context_set_timing(rh_context *ctx, int32_t on) {
  if (!ctx) return fail(RH_EINVAL, "null context");
  if (on < 0 || on > 2) return fail(RH_EINVAL, "timing level must be 0, 1 or 2");
  ctx->c.timing = on;
  return RH_OK;
}

rh_status rh_context_set_refinement(rh_context *ctx, int32_t steps) {
  if (!ctx) return fail(RH_EINVAL, "null context");
  if (steps < 0 || steps > 16) return fail(RH_EINVAL, "refinement steps must be in 0..16");
  ctx->c.refine = steps;
  return RH_OK;
}

rh_status rh_context_set_refinement_tol(rh_context *ctx, double tol) {
  if (!ctx) return fail(RH_EINVAL, "null context");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(RH_EINVAL, "tolerance must be finite and >= 0");
  ctx->c.refine_tol = tol;
  return RH_OK;
}

rh_status rh_network_create(rh_context *ctx, const rh_network_desc *desc, rh_network **out) {
  GUARD_BEGIN
  if (!ctx || !desc || !out) return fail(RH_EINVAL, "null argument");
  *out = nullptr;
  rh_network *net = new rh_network();
  net->n.ctx = &ctx->c;
  std::string err;
  rh_status s = network_build(net->n, *desc, err);
  if (s != RH_OK) {
    delete net;
    return fail(s, err);
  }
  net->n.report.last_kernel_ms = -1.0;
  *out = net;
  return RH_OK;
  GUARD_END
}

rh_status rh_network_destroy(rh_network *net) {
  if (!net) return RH_OK;
  device_newton_free(net->n);
  device_track_free(net->n);
  device_free(net->n);
  delete net;
  return RH_OK;
}

rh_status rh_network_dims(const rh_network *net, int32_t *n_x, int32_t *n_p) {
  if (!net) return fail(RH_EINVAL, "null network");
  if (n_x) *n_x = net->n.n_x;
  if (n_p) *n_p = net->n.n_p;
  return RH_OK;
}

rh_status rh_network_index_maps(const rh_network *net, int32_t *x_bus, int32_t *x_kind,
                                int32_t *p_bus, int32_t *p_kind) {
  if (!net) return fail(RH_EINVAL, "null network");
  const Network &n = net->n;
  for (int32_t b = 0; b < n.n_bus; ++b) {
    if (n.th_x[b] >= 0) {
      if (x_bus) x_bus[n.th_x[b]] = b;
      if (x_kind) x_kind[n.th_x[b]] = 0;
    }
    if (n.v_x[b] >= 0) {
      if (x_bus) x_bus[n.v_x[b]] = b;
      if (x_kind) x_kind[n.v_x[b]] = 1;
    }
    if (n.v_p[b] >= 0) {
      if (p_bus) p_bus[n.v_p[b]] = b;
      if (p_kind) p_kind[n.v_p[b]] = 1;
    }
    if (n.pg_p[b] >= 0) {
      if (p_bus) p_bus[n.pg_p[b]] = b;
      if (p_kind) p_kind[n.pg_p[b]] = 2;
    }
  }
  return RH_OK;
}

rh_status rh_set_parameters(rh_network *net, const double *p) {
  if (!net || !p) return fail(RH_EINVAL, "null argument");
  if (!finite_n(p, net->n.n_p)) return fail(RH_EINVAL, "NaN or Inf in parameters");
  net->n.p.assign(p, p + net->n.n_p);
  invalidate(net->n);
  return RH_OK;
}

rh_status rh_get_parameters(const rh_network *net, double *p) {
  if (!net || !p) return fail(RH_EINVAL, "null argument");
  std::memcpy(p, net->n.p.data(), sizeof(double) * net->n.n_p);
  return RH_OK;
}

rh_status rh_set_loads(rh_network *net, const double *Pd, const double *Qd) {
  if (!net || !Pd || !Qd) return fail(RH_EINVAL, "null argument");
  if (!finite_n(Pd, net->n.n_bus) || !finite_n(Qd, net->n.n_bus))
    return fail(RH_EINVAL, "NaN or Inf in loads");
  net->n.Pd.assign(Pd, Pd + net->n.n_bus);
  net->n.Qd.assign(Qd, Qd + net->n.n_bus);
  invalidate(net->n);
  return RH_OK;
}

rh_status rh_set_initial_state(rh_network *net, const double *x0) {
  if (!net) return fail(RH_EINVAL, "null network");
  if (!x0) {
    net->n.x0.clear();
    return RH_OK;
  }
  if (!finite_n(x0, net->n.n_x)) return fail(RH_EINVAL, "NaN or Inf in initial state");
  net->n.x0.assign(x0, x0 + net->n.n_x);
  return RH_OK;
}

rh_status rh_solve_powerflow(rh_network *net, double tol, int32_t max_iter, int32_t *iters,
                             double *resid_inf) {
  GUARD_BEGIN
  if (!net) return fail(RH_EINVAL, "null network");
  std::string err;
  rh_status s = network_solve(net->n, tol, max_iter, err);
  if (iters) *iters = net->n.newton_iters;
  if (resid_inf) *resid_inf = net->n.newton_resid;
  if (s != RH_OK) return fail(s, err);
  if (net->n.ctx->device >= 0) {
    s = device_upload(net->n, err);
    if (s != RH_OK) {
      net->n.solved = false;
      return fail(s, err);
    }
  }
  return RH_OK;
  GUARD_END
}

rh_status rh_solve_powerflow_device(rh_network *net, double tol, int32_t max_iter, int32_t *iters,
                                    double *resid_inf) {
  GUARD_BEGIN
  if (!net) return fail(RH_EINVAL, "null network");
  if (net->n.ctx->device < 0) return fail(RH_EDEVICE, "host-only context");
  Network &n = net->n;
  n.solved = false;
  if (n.islanded) return fail(RH_ESINGULAR, "some bus is not connected to the reference bus: G_x is singular");
  if (!(tol > 0.0) || max_iter < 0) return fail(RH_EINVAL, "tol must be > 0 and max_iter >= 0");
  std::string err;
  NewtonResult res;
  rh_status s = device_newton(n, tol, max_iter, res, err);
  if (iters) *iters = res.iters;
  if (resid_inf) *resid_inf = res.resid;
  n.newton_iters = res.iters;
  n.newton_resid = res.resid;
  if (s != RH_OK) return fail(s, err);
  // the host side of the solve (Jacobians, adjoint, tape) runs while the
  // upload prepares the factors' sweeps
  s = device_upload(n, err, [&](std::string &e) { return network_accept(n, res.x, res.iters, res.resid, true, e); });
  if (s != RH_OK) {
    n.solved = false;
    return fail(s, err);
  }
  return RH_OK;
  GUARD_END
}

rh_status rh_get_factors(const rh_network *net, double *l, double *u) {
  if (!net) return fail(RH_EINVAL, "null network");
  if (!net->n.solved) return fail(RH_ESTATE, "no converged power flow for the current parameters");
  const LuPlan &lu = net->n.lu;
  int64_t ql = 0, qu = 0;
  for (int32_t i = 0; i < lu.n; ++i) {
    if (l)
      for (double v : lu.lval[i]) l[ql++] = v;
    if (u)
      for (double v : lu.uval[i]) u[qu++] = v;
  }
  return RH_OK;
}

rh_status rh_get_state(const rh_network *net, double *x) {
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if (!x) return fail(RH_EINVAL, "null x");
  std::memcpy(x, net->n.x.data(), sizeof(double) * net->n.n_x);
  return RH_OK;
}

rh_status rh_objective(const rh_network *net, double *F) {
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if (!F) return fail(RH_EINVAL, "null F");
  *F = net->n.objective;
  return RH_OK;
}

rh_status rh_condition_estimate(const rh_network *net, double *cond1) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if (!cond1) return fail(RH_EINVAL, "null cond1");
  *cond1 = condest_1(net->n);
  return RH_OK;
  GUARD_END
}

rh_status rh_reduced_gradient(rh_network *net, double *grad) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if (!grad) return fail(RH_EINVAL, "null grad");
  std::vector<double> g;
  reduced_gradient(net->n, g);
  std::memcpy(grad, g.data(), sizeof(double) * net->n.n_p);
  return RH_OK;
  GUARD_END
}

rh_status rh_hvp_device(rh_network *net, int32_t k, const void *dW, int64_t ldw, void *dHW,
                        int64_t ldhw, rh_precision prec, void *hip_stream) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if ((s = need_device(net)) != RH_OK) return s;
  if (prec != RH_FP64 && prec != RH_FP32_REFINED) return fail(RH_EINVAL, "unknown precision");
  if (k < 0 || !dW || !dHW || ldw < net->n.n_p || ldhw < net->n.n_p)
    return fail(RH_EINVAL, "bad product arguments");
  net->n.report.last_k = k;
  if (k == 0) return RH_OK;
  std::string err;
  s = device_hvp(net->n, k, static_cast<const double *>(dW), ldw, static_cast<double *>(dHW), ldhw,
                 -1, prec, hip_stream, err);
  if (s != RH_OK) return fail(s, err);
  if (prec == RH_FP32_REFINED) net->n.refined_cols = k;
  return RH_OK;
  GUARD_END
}

rh_status rh_hvp_device_noalloc(rh_network *net, int32_t k, const void *dW, int64_t ldw, void *dHW,
                                int64_t ldhw, rh_precision prec, void *hip_stream) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if ((s = need_device(net)) != RH_OK) return s;
  if (prec != RH_FP64 && prec != RH_FP32_REFINED) return fail(RH_EINVAL, "unknown precision");
  if (k < 0 || !dW || !dHW || ldw < net->n.n_p || ldhw < net->n.n_p)
    return fail(RH_EINVAL, "bad product arguments");
  net->n.report.last_k = k;
  if (k == 0) return RH_OK;
  std::string err;
  s = device_hvp_noalloc(net->n, k, static_cast<const double *>(dW), ldw, static_cast<double *>(dHW), ldhw,
                         prec, hip_stream, err);
  if (s != RH_OK) return fail(s, err);
  return RH_OK;
  GUARD_END
}

rh_status rh_autotune(rh_network *net, rh_precision prec, int32_t flags, rh_tile *out) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if ((s = need_device(net)) != RH_OK) return s;
  if (prec != RH_FP64 && prec != RH_FP32_REFINED) return fail(RH_EINVAL, "unknown precision");
  if (flags & ~(RH_TUNE_MEASURE | RH_TUNE_NO_CACHE)) return fail(RH_EINVAL, "unknown tuner flags");
  std::string err;
  rh_tile t{};
  s = autotune(net->n, prec, flags, t, err);
  if (s != RH_OK) return fail(s, err);
  if (out) *out = t;
  return RH_OK;
  GUARD_END
}

rh_status rh_get_tile(const rh_network *net, rh_precision prec, rh_tile *out) {
  if (!net || !out) return fail(RH_EINVAL, "null argument");
  if (prec != RH_FP64 && prec != RH_FP32_REFINED) return fail(RH_EINVAL, "unknown precision");
  *out = net->n.tile[prec == RH_FP32_REFINED ? 1 : 0];
  return RH_OK;
}


rh_status rh_reduced_hessian_device(rh_network *net, void *dH, int64_t ldh, int32_t k_block,
                                    rh_precision prec, void *hip_stream) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if ((s = need_device(net)) != RH_OK) return s;
  if (prec != RH_FP64 && prec != RH_FP32_REFINED) return fail(RH_EINVAL, "unknown precision");
  const int32_t n_p = net->n.n_p;
  if (!dH || ldh < n_p || k_block < 0) return fail(RH_EINVAL, "bad Hessian arguments");
  std::string err;
  s = reduced_hessian_into(net->n, static_cast<double *>(dH), ldh, k_block, prec, hip_stream, err);
  if (s != RH_OK) return fail(s, err);
  return RH_OK;
  GUARD_END
}

rh_status rh_hvp(rh_network *net, int32_t k, const double *W, int64_t ldw, double *HW, int64_t ldhw,
                 rh_precision prec) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if ((s = need_device(net)) != RH_OK) return s;
  const int32_t n_p = net->n.n_p;
  if (k < 0 || !W || !HW || ldw < n_p || ldhw < n_p) return fail(RH_EINVAL, "bad product arguments");
  if (k == 0) return RH_OK;
  for (int32_t j = 0; j < k; ++j)
    if (!finite_n(W + (int64_t)j * ldw, n_p)) return fail(RH_EINVAL, "NaN or Inf in W");
  std::string err;
  void *dW = nullptr, *dHW = nullptr;
  const size_t bytes = sizeof(double) * (size_t)n_p * k;
  if ((s = device_alloc(&dW, bytes, err)) != RH_OK) return fail(s, err);
  if ((s = device_alloc(&dHW, bytes, err)) != RH_OK) {
    device_release(dW);
    return fail(s, err);
  }
  s = device_memcpy_2d(dW, sizeof(double) * n_p, W, sizeof(double) * ldw, sizeof(double) * n_p, k, 1,
                       err);
  if (s == RH_OK) {
    s = rh_hvp_device(net, k, dW, n_p, dHW, n_p, prec, nullptr);
    if (s != RH_OK) err = g_err;
  }
  if (s == RH_OK) s = device_sync(nullptr, err);
  if (s == RH_OK)
    s = device_memcpy_2d(HW, sizeof(double) * ldhw, dHW, sizeof(double) * n_p, sizeof(double) * n_p,
                         k, 0, err);
  device_release(dW);
  device_release(dHW);
  if (s != RH_OK) return fail(s, err);
  return RH_OK;
  GUARD_END
}

rh_status rh_reduced_hessian(rh_network *net, double *H, int64_t ldh, int32_t k_block,
                             rh_precision prec) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if ((s = need_device(net)) != RH_OK) return s;
  const int32_t n_p = net->n.n_p;
  if (!H || ldh < n_p) return fail(RH_EINVAL, "bad Hessian arguments");
  std::string err;
  void *dH = nullptr;
  if ((s = device_alloc(&dH, sizeof(double) * (size_t)n_p * n_p, err)) != RH_OK) return fail(s, err);
  s = rh_reduced_hessian_device(net, dH, n_p, k_block, prec, nullptr);
  if (s != RH_OK) err = g_err;
  if (s == RH_OK) s = device_sync(nullptr, err);
  if (s == RH_OK)
    s = device_memcpy_2d(H, sizeof(double) * ldh, dH, sizeof(double) * n_p, sizeof(double) * n_p,
                         n_p, 0, err);
  device_release(dH);
  if (s != RH_OK) return fail(s, err);
  return RH_OK;
  GUARD_END
}

rh_status rh_reduced_gradient_device(rh_network *net, void *dgrad, void *hip_stream) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if ((s = need_device(net)) != RH_OK) return s;
  if (!dgrad) return fail(RH_EINVAL, "null gradient buffer");
  std::string err;
  if ((s = device_reduced_gradient(net->n, static_cast<double *>(dgrad), hip_stream, err)) != RH_OK)
    return fail(s, err);
  return RH_OK;
  GUARD_END
}

rh_status rh_cholesky_solve_device(rh_context *ctx, int32_t n, void *dA, int64_t lda, void *dB, int64_t ldb,
                                   int32_t nrhs, void *hip_stream, int32_t *failed_col) {
  GUARD_BEGIN
  if (failed_col) *failed_col = -1;
  if (!ctx) return fail(RH_EINVAL, "null context");
  if (ctx->c.device < 0) return fail(RH_EDEVICE, "host-only context");
  if (n < 0 || nrhs < 0 || lda < std::max(1, n) || ldb < std::max(1, n)) return fail(RH_EINVAL, "bad dimensions");
  if (n > 0 && (!dA || (nrhs > 0 && !dB))) return fail(RH_EINVAL, "null buffer");
  if (n == 0) return RH_OK;
  std::string err;
  int32_t bad = -1;
  rh_status s = dense_spd_solve(ctx->c.device, n, static_cast<double *>(dA), lda, static_cast<double *>(dB), ldb,
                                nrhs, hip_stream, bad, err);
  if (s != RH_OK) return fail(s, err);
  if (failed_col) *failed_col = bad;
  if (bad >= 0) return fail(RH_ESINGULAR, "leading minor " + std::to_string(bad + 1) + " is not positive definite");
  return RH_OK;
  GUARD_END
}

rh_status rh_tracking_step_device(rh_network *net, int32_t k_block, double shift, const double *lo, const double *hi,
                                  const double *ramp, void *dd, void *hip_stream, rh_tracking_info *info) {
  GUARD_BEGIN
  rh_status s = need_solved(net);
  if (s != RH_OK) return s;
  if ((s = need_device(net)) != RH_OK) return s;
  const int32_t n_p = net->n.n_p;
  if (k_block < 0 || !(shift >= 0.0) || !std::isfinite(shift)) return fail(RH_EINVAL, "bad k_block or shift");
  if ((lo && !finite_n(lo, n_p)) || (hi && !finite_n(hi, n_p)) || (ramp && !finite_n(ramp, n_p)))
    return fail(RH_EINVAL, "NaN or Inf in bounds or ramp limits");
  for (int32_t q = 0; q < n_p; ++q)
    if ((lo && hi && lo[q] > hi[q]) || (ramp && ramp[q] < 0.0)) return fail(RH_EINVAL, "empty bounds or negative ramp");
  std::string err;
  rh_tracking_info r{};
  if ((s = tracking_step(net->n, k_block, shift, lo, hi, ramp, static_cast<double *>(dd), hip_stream, r, err)) !=
      RH_OK)
    return fail(s, err);
  if (info) *info = r;
  return RH_OK;
  GUARD_END
}

rh_status rh_last_report(const rh_network *net, rh_report *out) {
  if (!net || !out) return fail(RH_EINVAL, "null argument");
  rh_network *mnet = const_cast<rh_network *>(net);
  std::string err;
  if (mnet->n.ctx->device >= 0) {
    rh_status s = device_collect(mnet->n, err);
    if (s != RH_OK) return fail(s, err);
  }
  *out = net->n.report;
  out->tile[0] = net->n.tile[0];
  out->tile[1] = net->n.tile[1];
  return RH_OK;
}

rh_status rh_network_device_bytes(const rh_network *net, rh_precision prec, int64_t *resident,
                                  int64_t *scratch_per_direction) {
  if (!net) return fail(RH_EINVAL, "null network");
  if (prec != RH_FP64 && prec != RH_FP32_REFINED) return fail(RH_EINVAL, "unknown precision");
  if (resident) *resident = device_network_bytes(net->n);
  if (scratch_per_direction) *scratch_per_direction = device_scratch_per_direction(net->n.n_x, prec);
  return RH_OK;
}

rh_status rh_refinement_report(const rh_network *net, int32_t n, double *berr_z, int32_t *steps_z,
                               double *berr_psi, int32_t *steps_psi) {
  GUARD_BEGIN
  if (!net) return fail(RH_EINVAL, "null network");
  rh_network *mnet = const_cast<rh_network *>(net);
  if (mnet->n.refined_cols < 0) return fail(RH_ESTATE, "no refined product call on this network");
  if (n < 0 || n > mnet->n.refined_cols)
    return fail(RH_EINVAL, "column count exceeds that of the last refined call");
  std::vector<double> v;
  std::string err;
  rh_status s = device_refinement_report(mnet->n, n, v, err);
  if (s != RH_OK) return fail(s, err);
  for (int32_t j = 0; j < n; ++j) {
    if (berr_z) berr_z[j] = v[4 * (size_t)j];
    if (steps_z) steps_z[j] = (int32_t)v[4 * (size_t)j + 1];
    if (berr_psi) berr_psi[j] = v[4 * (size_t)j + 2];
    if (steps_psi) steps_psi[j] = (int32_t)v[4 * (size_t)j + 3];
  }
  return RH_OK;
  GUARD_END
}

}  // extern "C"

namespace {
// Checks of a batch (rh_hvp_batch_device, rh_batch_create); fills ns.
rh_status check_batch(rh_context *ctx, int32_t n, rh_network *const *nets, const int32_t *k, const void *const *dW,
                      const int64_t *ldw, void *const *dHW, const int64_t *ldhw, const int32_t *identity_from,
                      rh_precision prec, std::vector<Network *> &ns) {
  if (!ctx) return fail(RH_EINVAL, "null context");
  if (ctx->c.device < 0) return fail(RH_EDEVICE, "host-only context");
  if (prec != RH_FP64 && prec != RH_FP32_REFINED) return fail(RH_EINVAL, "unknown precision");
  if (n < 0 || (n > 0 && (!nets || !k || !dW || !ldw || !dHW || !ldhw)))
    return fail(RH_EINVAL, "bad batch arguments");
  ns.assign(n, nullptr);
  for (int32_t i = 0; i < n; ++i) {
    if (!nets[i]) return fail(RH_EINVAL, "null network in batch");
    Network &net = nets[i]->n;
    if (net.ctx != &ctx->c) return fail(RH_EINVAL, "network of another context in batch");
    if (!net.solved || !net.dev) return fail(RH_ESTATE, "unsolved network in batch");
    const int32_t idf = identity_from ? identity_from[i] : -1;
    const std::string where = "batch item " + std::to_string(i) + " (k " + std::to_string(k[i]) +
                              ", n_p " + std::to_string(net.n_p) + ", ldw " + std::to_string(ldw[i]) +
                              ", ldhw " + std::to_string(ldhw[i]) + ", identity_from " +
                              std::to_string(idf) + ")";
    if (k[i] < 0 || (k[i] > 0 && (!dHW[i] || ldhw[i] < net.n_p)))
      return fail(RH_EINVAL, "bad output of " + where);
    if (k[i] > 0 && idf < 0 && (!dW[i] || ldw[i] < net.n_p)) return fail(RH_EINVAL, "bad input of " + where);
    if (idf >= 0 && (int64_t)idf + k[i] > net.n_p) return fail(RH_EINVAL, "identity block exceeds n_p in " + where);
    ns[i] = &net;
  }
  return RH_OK;
}
}  // namespace

struct rh_batch {
  DeviceBatch *b = nullptr;
};

extern "C" {

rh_status rh_hvp_batch_device(rh_context *ctx, int32_t n, rh_network *const *nets, const int32_t *k,
                              const void *const *dW, const int64_t *ldw, void *const *dHW,
                              const int64_t *ldhw, const int32_t *identity_from, rh_precision prec,
                              void *hip_stream) {
  GUARD_BEGIN
  std::vector<Network *> ns;
  rh_status s = check_batch(ctx, n, nets, k, dW, ldw, dHW, ldhw, identity_from, prec, ns);
  if (s != RH_OK) return s;
  std::string err;
  s = device_hvp_batch(ctx->c, n, ns.data(), k, reinterpret_cast<const double *const *>(dW), ldw,
                       reinterpret_cast<double *const *>(dHW), ldhw, identity_from, prec, hip_stream, err);
  if (s != RH_OK) return fail(s, err);
  return RH_OK;
  GUARD_END
}

rh_status rh_batch_create(rh_context *ctx, int32_t n, rh_network *const *nets, const int32_t *k,
                          const void *const *dW, const int64_t *ldw, void *const *dHW, const int64_t *ldhw,
                          const int32_t *identity_from, rh_precision prec, rh_batch **out) {
  GUARD_BEGIN
  if (!out) return fail(RH_EINVAL, "null out");
  *out = nullptr;
  std::vector<Network *> ns;
  rh_status s = check_batch(ctx, n, nets, k, dW, ldw, dHW, ldhw, identity_from, prec, ns);
  if (s != RH_OK) return s;
  std::string err;
  DeviceBatch *db = nullptr;
  s = device_batch_create(ctx->c, n, ns.data(), k, reinterpret_cast<const double *const *>(dW), ldw,
                          reinterpret_cast<double *const *>(dHW), ldhw, identity_from, prec, &db, err);
  if (s != RH_OK) return fail(s, err);
  rh_batch *b = new rh_batch();
  b->b = db;
  *out = b;
  return RH_OK;
  GUARD_END
}

rh_status rh_batch_launch(rh_batch *b, void *hip_stream) {
  GUARD_BEGIN
  if (!b || !b->b) return fail(RH_EINVAL, "null batch");
  std::string err;
  rh_status s = device_batch_launch(b->b, hip_stream, err);
  if (s != RH_OK) return fail(s, err);
  return RH_OK;
  GUARD_END
}

rh_status rh_batch_info(const rh_batch *b, int32_t *dirs_per_group, int32_t *workgroups, int32_t *directions) {
  if (!b || !b->b) return fail(RH_EINVAL, "null batch");
  device_batch_info(b->b, dirs_per_group, workgroups, directions);
  return RH_OK;
}

rh_status rh_batch_destroy(rh_batch *b) {
  if (!b) return RH_OK;
  device_batch_free(b->b);
  delete b;
  return RH_OK;
}

rh_status rh_context_report(rh_context *ctx, rh_report *out) {
  if (!ctx || !out) return fail(RH_EINVAL, "null argument");
  *out = rh_report{};
  std::string err;
  if (ctx->c.device >= 0) {
    rh_status s = device_ctx_collect(ctx->c, *out, err);
    if (s != RH_OK) return fail(s, err);
  }
  return RH_OK;
}

}  // extern "C"
