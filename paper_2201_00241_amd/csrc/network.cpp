// Host planner: network ingest, state/parameter bookkeeping, branch-wise
// flows and Jacobians, Newton-Raphson, first-order adjoint, reduced gradient
// and the per-incidence second-order coefficients used by the device path.
//
// Power flow model: Sec. 3.1, eq. (powerflow) written per branch.  For a
// branch (f, t) with series admittance g_s + j b_s = 1/(r + j x), half line
// charging b_h = b/2 at each end, and a = theta_f - theta_t, every end flow
// has the form  F = alpha v_e^2 + v_f v_t h(a)  with
//   P_f: alpha = g_s,          h = -(g_s cos a + b_s sin a)
//   Q_f: alpha = -(b_s + b_h), h = -(g_s sin a - b_s cos a)
//   P_t: alpha = g_s,          h = -(g_s cos a - b_s sin a)
//   Q_t: alpha = -(b_s + b_h), h =  (g_s sin a + b_s cos a)
// and a bus injection is the sum of the end flows at that bus.
#include <algorithm>
#include <cmath>
#include <limits>
#include <cstring>
#include <numeric>
#include <queue>

#include "rh_internal.h"

namespace rh {
namespace {

// Per-flow coefficient alpha, h and dh/da of one branch.
struct FlowTerms {
  double alpha[4], h[4], hp[4];
};

inline FlowTerms flow_terms(double gs, double bs, double bh, double a) {
  const double c = std::cos(a), s = std::sin(a);
  FlowTerms t;
  t.alpha[0] = gs;
  t.h[0] = -(gs * c + bs * s);
  t.hp[0] = gs * s - bs * c;
  t.alpha[1] = -(bs + bh);
  t.h[1] = -(gs * s - bs * c);
  t.hp[1] = -(gs * c + bs * s);
  t.alpha[2] = gs;
  t.h[2] = -(gs * c - bs * s);
  t.hp[2] = gs * s + bs * c;
  t.alpha[3] = -(bs + bh);
  t.h[3] = gs * s + bs * c;
  t.hp[3] = gs * c - bs * s;
  return t;
}

// Gradient of flow k of a branch w.r.t. (theta_f, theta_t, v_f, v_t).
inline void flow_grad(const FlowTerms &t, int k, double vf, double vt, double g[4]) {
  const double K = vf * vt;
  g[0] = K * t.hp[k];
  g[1] = -K * t.hp[k];
  g[2] = vt * t.h[k] + (k < 2 ? 2.0 * t.alpha[k] * vf : 0.0);
  g[3] = vf * t.h[k] + (k >= 2 ? 2.0 * t.alpha[k] * vt : 0.0);
}

bool finite_all(const double *a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// Assemble G_x and G_p values at (th, v) into net.gx / net.gp (fixed patterns).
void assemble_jacobians(Network &net, const std::vector<double> &th, const std::vector<double> &v,
                        const std::vector<int64_t> &gx_slot, const std::vector<int64_t> &gp_slot) {
  std::fill(net.gx.val.begin(), net.gx.val.end(), 0.0);
  std::fill(net.gp.val.begin(), net.gp.val.end(), 0.0);
  for (int32_t b = 0; b < net.n_br; ++b) {
    const int32_t f = net.br_f[b], t = net.br_t[b];
    const FlowTerms ft = flow_terms(net.gs[b], net.bs[b], net.bsh[b], th[f] - th[t]);
    for (int k = 0; k < 4; ++k) {
      double g[4];
      flow_grad(ft, k, v[f], v[t], g);
      for (int q = 0; q < 4; ++q) {
        const int64_t s = gx_slot[(int64_t)b * 16 + k * 4 + q];
        if (s >= 0) net.gx.val[s] += g[q];
      }
      for (int q = 0; q < 2; ++q) {
        const int64_t s = gp_slot[(int64_t)b * 8 + k * 2 + q];
        if (s >= 0) net.gp.val[s] += g[2 + q];
      }
    }
  }
  for (int32_t i : net.pv) net.gp.val[gp_slot[(int64_t)net.n_br * 8 + i]] = -1.0;
}

// Build a CSR pattern from (row, col) pairs; returns the position of each pair.
void pattern_from_pairs(Csr &m, int32_t n_rows, int32_t n_cols,
                        const std::vector<std::pair<int32_t, int32_t>> &pairs,
                        std::vector<int64_t> &pos_of_pair) {
  std::vector<std::pair<int32_t, int32_t>> u;
  u.reserve(pairs.size());
  for (auto &pr : pairs)
    if (pr.first >= 0 && pr.second >= 0) u.push_back(pr);
  std::sort(u.begin(), u.end());
  u.erase(std::unique(u.begin(), u.end()), u.end());
  m.n_rows = n_rows;
  m.n_cols = n_cols;
  m.ptr.assign(n_rows + 1, 0);
  m.col.resize(u.size());
  for (size_t e = 0; e < u.size(); ++e) {
    m.ptr[u[e].first + 1]++;
    m.col[e] = u[e].second;
  }
  for (int32_t r = 0; r < n_rows; ++r) m.ptr[r + 1] += m.ptr[r];
  m.val.assign(u.size(), 0.0);
  pos_of_pair.resize(pairs.size());
  for (size_t q = 0; q < pairs.size(); ++q) {
    const auto &pr = pairs[q];
    if (pr.first < 0 || pr.second < 0) {
      pos_of_pair[q] = -1;
      continue;
    }
    const int32_t *b = m.col.data() + m.ptr[pr.first];
    const int32_t *e = m.col.data() + m.ptr[pr.first + 1];
    pos_of_pair[q] = std::lower_bound(b, e, pr.second) - m.col.data();
  }
}

}  // namespace

void unpack_state(const Network &net, const std::vector<double> &x, const std::vector<double> &p,
                  std::vector<double> &th, std::vector<double> &v) {
  th.assign(net.n_bus, 0.0);
  v.assign(net.n_bus, 0.0);
  for (int32_t b = 0; b < net.n_bus; ++b) {
    if (net.th_x[b] >= 0) th[b] = x[net.th_x[b]];
    if (net.v_x[b] >= 0) v[b] = x[net.v_x[b]];
    if (net.v_p[b] >= 0) v[b] = p[net.v_p[b]];
  }
}

void flows_inject(const Network &net, const std::vector<double> &th, const std::vector<double> &v,
                  std::vector<double> &P, std::vector<double> &Q) {
  P.assign(net.n_bus, 0.0);
  Q.assign(net.n_bus, 0.0);
  for (int32_t b = 0; b < net.n_br; ++b) {
    const int32_t f = net.br_f[b], t = net.br_t[b];
    const FlowTerms ft = flow_terms(net.gs[b], net.bs[b], net.bsh[b], th[f] - th[t]);
    const double K = v[f] * v[t];
    P[f] += ft.alpha[0] * v[f] * v[f] + K * ft.h[0];
    Q[f] += ft.alpha[1] * v[f] * v[f] + K * ft.h[1];
    P[t] += ft.alpha[2] * v[t] * v[t] + K * ft.h[2];
    Q[t] += ft.alpha[3] * v[t] * v[t] + K * ft.h[3];
  }
}

namespace {

// g(x, p) of eq. (powerflowvec): P rows at PV and PQ buses, Q rows at PQ buses,
// each stored at the x index of the matching unknown.
void residual(const Network &net, const std::vector<double> &th, const std::vector<double> &v,
              const std::vector<double> &p, std::vector<double> &g) {
  std::vector<double> P, Q;
  flows_inject(net, th, v, P, Q);
  g.assign(net.n_x, 0.0);
  for (int32_t b = 0; b < net.n_bus; ++b) {
    if (net.th_x[b] >= 0) {
      double r = P[b] + net.Pd[b];
      if (net.pg_p[b] >= 0) r -= p[net.pg_p[b]];
      g[net.th_x[b]] = r;
    }
    if (net.v_x[b] >= 0) g[net.v_x[b]] = Q[b] + net.Qd[b];
  }
}

// Gradient of P^inj at the reference bus, as (bus, d/dtheta_b, d/dv_b) triples.
void slack_gradient(const Network &net, const std::vector<double> &th, const std::vector<double> &v,
                    std::vector<int32_t> &bus, std::vector<double> &gth, std::vector<double> &gv) {
  std::vector<double> dth(net.n_bus, 0.0), dv(net.n_bus, 0.0);
  std::vector<char> touched(net.n_bus, 0);
  for (int32_t b = 0; b < net.n_br; ++b) {
    const int32_t f = net.br_f[b], t = net.br_t[b];
    int k;
    if (f == net.ref)
      k = 0;
    else if (t == net.ref)
      k = 2;
    else
      continue;
    const FlowTerms ft = flow_terms(net.gs[b], net.bs[b], net.bsh[b], th[f] - th[t]);
    double g[4];
    flow_grad(ft, k, v[f], v[t], g);
    dth[f] += g[0];
    dth[t] += g[1];
    dv[f] += g[2];
    dv[t] += g[3];
    touched[f] = touched[t] = 1;
  }
  bus.clear();
  gth.clear();
  gv.clear();
  for (int32_t b = 0; b < net.n_bus; ++b)
    if (touched[b]) {
      bus.push_back(b);
      gth.push_back(dth[b]);
      gv.push_back(dv[b]);
    }
}

double slack_power(const Network &net, const std::vector<double> &th, const std::vector<double> &v) {
  std::vector<double> P, Q;
  flows_inject(net, th, v, P, Q);
  return P[net.ref] + net.Pd[net.ref];
}

}  // namespace

rh_status network_build(Network &net, const rh_network_desc &d, std::string &err) {
  if (d.n_bus < 2 || d.n_branch < 1 || d.n_gen < 1) {
    err = "network needs at least 2 buses, 1 branch and 1 generator";
    return RH_EINVAL;
  }
  if (!d.br_from || !d.br_to || !d.br_r || !d.br_x || !d.br_b || !d.bus_type || !d.Pd || !d.Qd ||
      !d.gen_bus || !d.Pg || !d.Vg || !d.c2 || !d.c1 || !d.c0) {
    err = "null array in network description";
    return RH_EINVAL;
  }
  const int32_t n = d.n_bus, m = d.n_branch, ng = d.n_gen;
  if (!finite_all(d.br_r, m) || !finite_all(d.br_x, m) || !finite_all(d.br_b, m) ||
      !finite_all(d.Pd, n) || !finite_all(d.Qd, n) || !finite_all(d.Pg, ng) ||
      !finite_all(d.Vg, ng) || !finite_all(d.c2, ng) || !finite_all(d.c1, ng) ||
      !finite_all(d.c0, ng)) {
    err = "NaN or Inf in network description";
    return RH_EINVAL;
  }
  net.n_bus = n;
  net.n_br = m;
  net.n_gen = ng;
  net.br_f.assign(d.br_from, d.br_from + m);
  net.br_t.assign(d.br_to, d.br_to + m);
  net.br_r.assign(d.br_r, d.br_r + m);
  net.br_x.assign(d.br_x, d.br_x + m);
  net.br_b.assign(d.br_b, d.br_b + m);
  net.bus_type.assign(d.bus_type, d.bus_type + n);
  net.Pd.assign(d.Pd, d.Pd + n);
  net.Qd.assign(d.Qd, d.Qd + n);
  net.gen_bus.assign(d.gen_bus, d.gen_bus + ng);
  net.Pg.assign(d.Pg, d.Pg + ng);
  net.Vg.assign(d.Vg, d.Vg + ng);
  net.c2.assign(d.c2, d.c2 + ng);
  net.c1.assign(d.c1, d.c1 + ng);
  net.c0.assign(d.c0, d.c0 + ng);

  for (int32_t b = 0; b < m; ++b) {
    const int32_t f = net.br_f[b], t = net.br_t[b];
    if (f < 0 || f >= n || t < 0 || t >= n) {
      err = "branch endpoint out of range";
      return RH_EINVAL;
    }
    if (f == t) {
      err = "self-loop branch";
      return RH_EINVAL;
    }
    const double zr = net.br_r[b], zx = net.br_x[b];
    const double den = zr * zr + zx * zx;
    if (!(den > 0.0)) {
      err = "branch with zero impedance";
      return RH_EINVAL;
    }
  }
  net.ref = -1;
  for (int32_t b = 0; b < n; ++b) {
    const int32_t t = net.bus_type[b];
    if (t != kPQ && t != kPV && t != kRef) {
      err = "bus_type must be 1 (PQ), 2 (PV) or 3 (reference)";
      return RH_EINVAL;
    }
    if (t == kRef) {
      if (net.ref >= 0) {
        err = "more than one reference bus";
        return RH_EINVAL;
      }
      net.ref = b;
    }
  }
  if (net.ref < 0) {
    err = "no reference bus";
    return RH_EINVAL;
  }
  net.gen_of_bus.assign(n, -1);
  for (int32_t g = 0; g < ng; ++g) {
    const int32_t b = net.gen_bus[g];
    if (b < 0 || b >= n) {
      err = "generator bus out of range";
      return RH_EINVAL;
    }
    if (net.gen_of_bus[b] >= 0) {
      err = "two generators on one bus";
      return RH_EINVAL;
    }
    if (net.bus_type[b] == kPQ) {
      err = "generator on a PQ bus";
      return RH_EINVAL;
    }
    net.gen_of_bus[b] = g;
  }
  for (int32_t b = 0; b < n; ++b)
    if (net.bus_type[b] != kPQ && net.gen_of_bus[b] < 0) {
      err = "PV or reference bus without a generator";
      return RH_EINVAL;
    }

  // series admittance and half charging per branch
  net.gs.resize(m);
  net.bs.resize(m);
  net.bsh.resize(m);
  for (int32_t b = 0; b < m; ++b) {
    const double zr = net.br_r[b], zx = net.br_x[b], den = zr * zr + zx * zx;
    net.gs[b] = zr / den;
    net.bs[b] = -zx / den;
    net.bsh[b] = 0.5 * net.br_b[b];
  }

  // bookkeeping: x = [theta_pv; theta_pq; v_pq], p = [Pg_pv; v_ref; v_pv]
  net.pv.clear();
  net.pq.clear();
  for (int32_t b = 0; b < n; ++b) {
    if (net.bus_type[b] == kPV) net.pv.push_back(b);
    if (net.bus_type[b] == kPQ) net.pq.push_back(b);
  }
  net.n_pv = (int32_t)net.pv.size();
  net.n_pq = (int32_t)net.pq.size();
  net.n_x = net.n_pv + 2 * net.n_pq;
  net.n_p = 2 * net.n_pv + 1;
  net.th_x.assign(n, -1);
  net.v_x.assign(n, -1);
  net.v_p.assign(n, -1);
  net.pg_p.assign(n, -1);
  for (int32_t i = 0; i < net.n_pv; ++i) {
    net.th_x[net.pv[i]] = i;
    net.pg_p[net.pv[i]] = i;
    net.v_p[net.pv[i]] = net.n_pv + 1 + i;
  }
  for (int32_t i = 0; i < net.n_pq; ++i) {
    net.th_x[net.pq[i]] = net.n_pv + i;
    net.v_x[net.pq[i]] = net.n_pv + net.n_pq + i;
  }
  net.v_p[net.ref] = net.n_pv;

  // connectivity to the reference bus (an island makes G_x singular)
  {
    std::vector<std::vector<int32_t>> adj(n);
    for (int32_t b = 0; b < m; ++b) {
      adj[net.br_f[b]].push_back(net.br_t[b]);
      adj[net.br_t[b]].push_back(net.br_f[b]);
    }
    std::vector<char> seen(n, 0);
    std::queue<int32_t> q;
    q.push(net.ref);
    seen[net.ref] = 1;
    int32_t cnt = 1;
    while (!q.empty()) {
      const int32_t u = q.front();
      q.pop();
      for (int32_t w : adj[u])
        if (!seen[w]) {
          seen[w] = 1;
          ++cnt;
          q.push(w);
        }
    }
    net.islanded = (cnt != n);
  }

  // patterns of G_x and G_p and the scatter maps of the branch gradients
  std::vector<std::pair<int32_t, int32_t>> gx_pairs((size_t)m * 16), gp_pairs((size_t)m * 8 + n);
  for (int32_t b = 0; b < m; ++b) {
    const int32_t f = net.br_f[b], t = net.br_t[b];
    const int32_t rows[4] = {net.th_x[f], net.v_x[f], net.th_x[t], net.v_x[t]};
    const int32_t cols[4] = {net.th_x[f], net.th_x[t], net.v_x[f], net.v_x[t]};
    const int32_t pcols[2] = {net.v_p[f], net.v_p[t]};
    for (int k = 0; k < 4; ++k) {
      for (int q = 0; q < 4; ++q)
        gx_pairs[(size_t)b * 16 + k * 4 + q] = {rows[k] >= 0 && cols[q] >= 0 ? rows[k] : -1,
                                                rows[k] >= 0 && cols[q] >= 0 ? cols[q] : -1};
      for (int q = 0; q < 2; ++q)
        gp_pairs[(size_t)b * 8 + k * 2 + q] = {rows[k] >= 0 && pcols[q] >= 0 ? rows[k] : -1,
                                               rows[k] >= 0 && pcols[q] >= 0 ? pcols[q] : -1};
    }
  }
  for (int32_t b = 0; b < n; ++b)
    gp_pairs[(size_t)m * 8 + b] = net.pg_p[b] >= 0 ? std::make_pair(net.th_x[b], net.pg_p[b])
                                                   : std::make_pair(-1, -1);
  pattern_from_pairs(net.gx, net.n_x, net.n_x, gx_pairs, net.gx_slot);
  pattern_from_pairs(net.gp, net.n_x, net.n_p, gp_pairs, net.gp_slot);
  // the pattern of G_x must hold its diagonal (every x unknown touches a branch)
  for (int32_t r = 0; r < net.n_x; ++r) {
    const int32_t *b = net.gx.col.data() + net.gx.ptr[r];
    const int32_t *e = net.gx.col.data() + net.gx.ptr[r + 1];
    if (!std::binary_search(b, e, r)) {
      err = "bus without branches";
      return RH_EINVAL;
    }
  }
  net.report.n_x = net.n_x;
  net.report.n_p = net.n_p;

  lu_analyse(net.lu, net.gx);
  net.report.nnz_gx = net.gx.nnz();
  net.report.nnz_l = net.lu.nnz_l;
  net.report.nnz_u = net.lu.nnz_u;
  net.report.levels_l = net.lu.n_levels_l;
  net.report.levels_u = net.lu.n_levels_u;

  net.p.assign(net.n_p, 0.0);
  for (int32_t i = 0; i < net.n_pv; ++i) {
    const int32_t g = net.gen_of_bus[net.pv[i]];
    net.p[i] = net.Pg[g];
    net.p[net.n_pv + 1 + i] = net.Vg[g];
  }
  net.p[net.n_pv] = net.Vg[net.gen_of_bus[net.ref]];
  net.solved = false;
  return RH_OK;
}

namespace {

// Second-order coefficients of the Lagrangian per bus incidence (Sec. 4.2).
//
// With multipliers mu on the injections (lambda on the balance rows and the
// slack generator's marginal cost 2 c2 Pg_ref + c1 on P_ref), the Lagrangian
// restricted to one branch is
//   phi = a_f v_f^2 + a_t v_t^2 + v_f v_t H(a),
//   a_f = mu^P_f g_s - mu^Q_f (b_s + b_h),  a_t likewise,
//   H   = sum over the four flows of mu times their h(a),
// so its Hessian in (theta_f, theta_t, v_f, v_t) only needs K = v_f v_t H,
// H, H' = dH/da, 2 a_f, 2 a_t and the voltages.  For the end e of a branch
// whose other end is o, with s_e = +1 at the from end and -1 at the to end,
// the product with a tangent (dtheta, dv) contributes
//   y_theta_e += -K (dtheta_e - dtheta_o) + s_e H' (v_o dv_e + v_e dv_o)
//   y_v_e     +=  s_e H' v_o (dtheta_e - dtheta_o) + 2 a_e dv_e + H dv_o.
void build_tape(Network &net, const std::vector<double> &th, const std::vector<double> &v) {
  Tape &tp = net.tape;
  const int32_t n = net.n_bus;
  std::vector<double> muP(n, 0.0), muQ(n, 0.0);
  for (int32_t b = 0; b < n; ++b) {
    if (net.th_x[b] >= 0) muP[b] = net.lam[net.th_x[b]];
    if (net.v_x[b] >= 0) muQ[b] = net.lam[net.v_x[b]];
  }
  const int32_t gr = net.gen_of_bus[net.ref];
  const double Pr = slack_power(net, th, v);
  muP[net.ref] = 2.0 * net.c2[gr] * Pr + net.c1[gr];

  tp.inc_ptr.assign(n + 1, 0);
  for (int32_t b = 0; b < net.n_br; ++b) {
    tp.inc_ptr[net.br_f[b] + 1]++;
    tp.inc_ptr[net.br_t[b] + 1]++;
  }
  for (int32_t b = 0; b < n; ++b) tp.inc_ptr[b + 1] += tp.inc_ptr[b];
  const int32_t ninc = tp.inc_ptr[n];
  tp.inc_other.assign(ninc, 0);
  tp.inc_K.assign(ninc, 0.0);
  tp.inc_Hps.assign(ninc, 0.0);
  tp.inc_H.assign(ninc, 0.0);
  tp.inc_A2.assign(ninc, 0.0);
  tp.inc_vo.assign(ninc, 0.0);
  std::vector<int32_t> fill(tp.inc_ptr.begin(), tp.inc_ptr.end() - 1);
  for (int32_t b = 0; b < net.n_br; ++b) {
    const int32_t f = net.br_f[b], t = net.br_t[b];
    const double gs = net.gs[b], bs = net.bs[b], bh = net.bsh[b];
    const double a = th[f] - th[t], c = std::cos(a), s = std::sin(a);
    const double af = muP[f] * gs - muQ[f] * (bs + bh);
    const double at = muP[t] * gs - muQ[t] * (bs + bh);
    const double H = -muP[f] * (gs * c + bs * s) - muQ[f] * (gs * s - bs * c) -
                     muP[t] * (gs * c - bs * s) + muQ[t] * (gs * s + bs * c);
    const double Hp = -muP[f] * (-gs * s + bs * c) - muQ[f] * (gs * c + bs * s) -
                      muP[t] * (-gs * s - bs * c) + muQ[t] * (gs * c - bs * s);
    const double K = v[f] * v[t] * H;
    // the incidences of a bus follow branch order, which keeps the summation
    // order fixed
    int32_t q = fill[f]++;
    tp.inc_other[q] = t;
    tp.inc_K[q] = K;
    tp.inc_Hps[q] = Hp;
    tp.inc_H[q] = H;
    tp.inc_A2[q] = 2.0 * af;
    tp.inc_vo[q] = v[t];
    q = fill[t]++;
    tp.inc_other[q] = f;
    tp.inc_K[q] = K;
    tp.inc_Hps[q] = -Hp;
    tp.inc_H[q] = H;
    tp.inc_A2[q] = 2.0 * at;
    tp.inc_vo[q] = v[f];
  }
  tp.bus_v = v;
  slack_gradient(net, th, v, tp.slack_bus, tp.slack_gth, tp.slack_gv);
  tp.slack_c2x2 = 2.0 * net.c2[gr];
  tp.bus_sth.assign(n, 0.0);
  tp.bus_sv.assign(n, 0.0);
  for (size_t i = 0; i < tp.slack_bus.size(); ++i) {
    tp.bus_sth[tp.slack_bus[i]] = tp.slack_c2x2 * tp.slack_gth[i];
    tp.bus_sv[tp.slack_bus[i]] = tp.slack_c2x2 * tp.slack_gv[i];
  }
}

// grad_x f and grad_p f of the cost.
void cost_gradient(const Network &net, const std::vector<double> &th, const std::vector<double> &v,
                   std::vector<double> &fx, std::vector<double> &fp) {
  fx.assign(net.n_x, 0.0);
  fp.assign(net.n_p, 0.0);
  const int32_t gr = net.gen_of_bus[net.ref];
  const double Pr = slack_power(net, th, v);
  const double m = 2.0 * net.c2[gr] * Pr + net.c1[gr];
  std::vector<int32_t> bus;
  std::vector<double> gth, gv;
  slack_gradient(net, th, v, bus, gth, gv);
  for (size_t i = 0; i < bus.size(); ++i) {
    const int32_t b = bus[i];
    if (net.th_x[b] >= 0) fx[net.th_x[b]] += m * gth[i];
    if (net.v_x[b] >= 0) fx[net.v_x[b]] += m * gv[i];
    if (net.v_p[b] >= 0) fp[net.v_p[b]] += m * gv[i];
  }
  for (int32_t i = 0; i < net.n_pv; ++i) {
    const int32_t g = net.gen_of_bus[net.pv[i]];
    fp[i] += 2.0 * net.c2[g] * net.p[i] + net.c1[g];
  }
}

double cost(const Network &net, const std::vector<double> &th, const std::vector<double> &v) {
  double F = 0.0;
  for (int32_t i = 0; i < net.n_pv; ++i) {
    const int32_t g = net.gen_of_bus[net.pv[i]];
    const double P = net.p[i];
    F += net.c2[g] * P * P + net.c1[g] * P + net.c0[g];
  }
  const int32_t gr = net.gen_of_bus[net.ref];
  const double Pr = slack_power(net, th, v);
  return F + net.c2[gr] * Pr * Pr + net.c1[gr] * Pr + net.c0[gr];
}

}  // namespace

rh_status network_solve(Network &net, double tol, int32_t max_iter, std::string &err) {
  net.solved = false;
  if (net.islanded) {
    err = "some bus is not connected to the reference bus: G_x is singular";
    return RH_ESINGULAR;
  }
  if (!(tol > 0.0) || max_iter < 0) {
    err = "tol must be > 0 and max_iter >= 0";
    return RH_EINVAL;
  }
  // initial state: the caller's guess, else a flat start
  std::vector<double> x(net.n_x, 0.0);
  if ((int32_t)net.x0.size() == net.n_x)
    x = net.x0;
  else
    for (int32_t b : net.pq) x[net.v_x[b]] = 1.0;
  std::vector<double> th, v, g;
  int32_t it = 0;
  double r = 0.0, r_prev = std::numeric_limits<double>::infinity();
  for (;; ++it) {
    unpack_state(net, x, net.p, th, v);
    residual(net, th, v, net.p, g);
    r = 0.0;
    bool finite = true;
    for (double e : g) {
      if (!std::isfinite(e)) finite = false;
      r = std::max(r, std::fabs(e));
    }
    if (!finite) {
      err = "Newton produced a non-finite residual";
      net.newton_iters = it;
      return RH_ENOCONV;
    }
    if (r <= tol || newton_stalled(it, r, r_prev)) break;
    if (it >= max_iter) {
      err = "Newton did not reach the tolerance in max_iter steps";
      net.newton_iters = it;
      net.newton_resid = r;
      return RH_ENOCONV;
    }
    r_prev = r;
    assemble_jacobians(net, th, v, net.gx_slot, net.gp_slot);
    if (!lu_factor(net.lu, net.gx, err)) return RH_ESINGULAR;
    lu_solve(net.lu, g);
    for (int32_t i = 0; i < net.n_x; ++i) x[i] -= g[i];
  }
  return network_accept(net, x, it, r, false, err);
}

rh_status network_accept(Network &net, const std::vector<double> &x, int32_t it, double r, bool factors_given,
                         std::string &err) {
  net.solved = false;
  std::vector<double> th, v;
  unpack_state(net, x, net.p, th, v);
  net.x = x;
  net.newton_iters = it;
  net.newton_resid = r;
  // Jacobians and factors at the accepted state
  assemble_jacobians(net, th, v, net.gx_slot, net.gp_slot);
  if (!factors_given && !lu_factor(net.lu, net.gx, err)) return RH_ESINGULAR;
  // first-order adjoint: G_x^T lambda = -grad_x f^T
  std::vector<double> fx, fp;
  cost_gradient(net, th, v, fx, fp);
  net.fp = fp;
  net.lam.resize(net.n_x);
  for (int32_t i = 0; i < net.n_x; ++i) net.lam[i] = -fx[i];
  lu_solve_t(net.lu, net.lam);
  net.objective = cost(net, th, v);
  build_tape(net, th, v);
  net.report.newton_iters = it;
  net.report.newton_resid = r;
  net.solved = true;
  return RH_OK;
}

double condest_1(const Network &net) {
  const int32_t n = net.n_x;
  if (n == 0) return 0.0;
  const Csr &A = net.gx;
  std::vector<double> colsum(n, 0.0);
  for (int32_t r = 0; r < A.n_rows; ++r)
    for (int32_t e = A.ptr[r]; e < A.ptr[r + 1]; ++e) colsum[A.col[e]] += std::fabs(A.val[e]);
  const double anorm = *std::max_element(colsum.begin(), colsum.end());
  auto norm1 = [](const std::vector<double> &v) {
    double t = 0.0;
    for (double e : v) t += std::fabs(e);
    return t;
  };
  auto sgn = [](double v) { return v >= 0.0 ? 1.0 : -1.0; };
  auto argmax_abs = [](const std::vector<double> &v) {
    size_t j = 0;
    for (size_t i = 1; i < v.size(); ++i)
      if (std::fabs(v[i]) > std::fabs(v[j])) j = i;
    return j;
  };
  // Hager's method with Higham's refinements (LAPACK's xLACON): a lower
  // bound of ||A^{-1}||_1 from at most five solves with A and A^T
  std::vector<double> x(n, 1.0 / n), xi(n), z;
  lu_solve(net.lu, x);
  double est = norm1(x);
  if (n > 1) {
    for (int32_t i = 0; i < n; ++i) xi[i] = sgn(x[i]);
    z = xi;
    lu_solve_t(net.lu, z);
    size_t j = argmax_abs(z);
    for (int iter = 2; iter <= 5; ++iter) {
      std::fill(x.begin(), x.end(), 0.0);
      x[j] = 1.0;
      lu_solve(net.lu, x);
      const double prev = est;
      est = norm1(x);
      bool same = true;
      for (int32_t i = 0; i < n && same; ++i) same = sgn(x[i]) == xi[i];
      if (same || est <= prev) {
        est = std::max(est, prev);
        break;
      }
      for (int32_t i = 0; i < n; ++i) xi[i] = sgn(x[i]);
      z = xi;
      lu_solve_t(net.lu, z);
      const size_t jl = j;
      j = argmax_abs(z);
      if (std::fabs(z[jl]) == std::fabs(z[j])) break;
    }
    // the alternating vector, against cancellation in the estimate above
    for (int32_t i = 0; i < n; ++i) x[i] = (i % 2 ? -1.0 : 1.0) * (1.0 + (double)i / (double)(n - 1));
    lu_solve(net.lu, x);
    est = std::max(est, 2.0 * norm1(x) / (3.0 * n));
  }
  return anorm * est;
}

void reduced_gradient(const Network &net, std::vector<double> &grad) {
  std::vector<double> th, v, fx;
  unpack_state(net, net.x, net.p, th, v);
  cost_gradient(net, th, v, fx, grad);
  // grad F = grad_p f + G_p^T lambda
  for (int32_t r = 0; r < net.gp.n_rows; ++r)
    for (int32_t e = net.gp.ptr[r]; e < net.gp.ptr[r + 1]; ++e)
      grad[net.gp.col[e]] += net.gp.val[e] * net.lam[r];
}

}  // namespace rh
