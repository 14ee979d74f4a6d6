// Fixed-pattern sparse LU of G_x with a symmetric fill-reducing ordering.
//
// The paper factorises G_x once on the host and re-uses the pattern for every
// refactorisation and for the batched forward/backward solves (Sec. 5.2).
// Here the host computes a minimum-degree ordering on the (structurally
// symmetric) pattern of G_x, the symbolic factor by simulating the
// elimination, and the numeric factor P A P^T = L U row by row with diagonal
// pivots (the power-flow Jacobian has a dominant diagonal in the natural
// pairing of angle/active-power and magnitude/reactive-power).  Rows of the
// triangular factors are then grouped into dependency levels for the device
// sweeps.
#include <algorithm>
#include <cstring>
#include <climits>
#include <cmath>
#include <queue>
#include <exception>
#include <stdexcept>
#include <thread>

#include "rh_internal.h"

namespace rh {

void lu_analyse(LuPlan &lu, const Csr &pat) {
  const int32_t n = pat.n_rows;
  lu.n = n;
  // adjacency of the symmetric pattern, without the diagonal
  std::vector<std::vector<int32_t>> adj(n);
  for (int32_t r = 0; r < n; ++r)
    for (int32_t e = pat.ptr[r]; e < pat.ptr[r + 1]; ++e) {
      const int32_t c = pat.col[e];
      if (c != r) {
        adj[r].push_back(c);
        adj[c].push_back(r);
      }
    }
  std::vector<int32_t> mark(n, -1);
  for (int32_t r = 0; r < n; ++r) {
    auto &a = adj[r];
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  // minimum degree by explicit elimination-graph updates (ties: lower index)
  using Item = std::pair<int32_t, int32_t>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int32_t r = 0; r < n; ++r) heap.push({(int32_t)adj[r].size(), r});
  std::vector<char> gone(n, 0);
  std::vector<std::vector<int32_t>> nbrs(n);  // eliminated k-th: its neighbours
  lu.perm.assign(n, -1);
  lu.iperm.assign(n, -1);
  std::vector<int32_t> merged;
  for (int32_t k = 0; k < n; ++k) {
    int32_t v;
    for (;;) {
      const Item it = heap.top();
      heap.pop();
      if (!gone[it.second] && (int32_t)adj[it.second].size() == it.first) {
        v = it.second;
        break;
      }
    }
    gone[v] = 1;
    lu.perm[k] = v;
    lu.iperm[v] = k;
    const std::vector<int32_t> nb = adj[v];
    nbrs[k] = nb;
    for (int32_t u : nb) {
      // adj[u] <- adj[u] \ {v}  union  nb \ {u}
      merged.clear();
      for (int32_t w : adj[u])
        if (w != v && mark[w] != u) {
          mark[w] = u;
          merged.push_back(w);
        }
      for (int32_t w : nb)
        if (w != u && mark[w] != u) {
          mark[w] = u;
          merged.push_back(w);
        }
      for (int32_t w : merged) mark[w] = -1;
      adj[u].assign(merged.begin(), merged.end());
      heap.push({(int32_t)adj[u].size(), u});
    }
    adj[v].clear();
    adj[v].shrink_to_fit();
  }
  // symbolic factor in permuted numbering
  lu.urow.assign(n, {});
  lu.lrow.assign(n, {});
  lu.nnz_l = lu.nnz_u = 0;
  for (int32_t k = 0; k < n; ++k) {
    auto &u = lu.urow[k];
    u.reserve(nbrs[k].size() + 1);
    u.push_back(k);
    std::vector<int32_t> cols;
    cols.reserve(nbrs[k].size());
    for (int32_t w : nbrs[k]) cols.push_back(lu.iperm[w]);
    std::sort(cols.begin(), cols.end());
    u.insert(u.end(), cols.begin(), cols.end());
    for (int32_t c : cols) lu.lrow[c].push_back(k);  // ascending k
    lu.nnz_u += (int64_t)u.size();
    lu.nnz_l += (int64_t)cols.size();
  }
  lu.lval.assign(n, {});
  lu.uval.assign(n, {});
  for (int32_t i = 0; i < n; ++i) {
    lu.lval[i].assign(lu.lrow[i].size(), 0.0);
    lu.uval[i].assign(lu.urow[i].size(), 0.0);
  }
  // dependency levels: forward sweeps (L, U^T) and backward sweeps (U, L^T)
  lu.level_l.assign(n, 0);
  lu.n_levels_l = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t lv = 0;
    for (int32_t k : lu.lrow[i]) lv = std::max(lv, lu.level_l[k] + 1);
    lu.level_l[i] = lv;
    lu.n_levels_l = std::max(lu.n_levels_l, lv + 1);
  }
  lu.level_u.assign(n, 0);
  lu.n_levels_u = 0;
  for (int32_t i = n - 1; i >= 0; --i) {
    int32_t lv = 0;
    for (size_t q = 1; q < lu.urow[i].size(); ++q) lv = std::max(lv, lu.level_u[lu.urow[i][q]] + 1);
    lu.level_u[i] = lv;
    lu.n_levels_u = std::max(lu.n_levels_u, lv + 1);
  }
}

bool lu_factor(LuPlan &lu, const Csr &a, std::string &err) {
  const int32_t n = lu.n;
  std::vector<double> w(n, 0.0);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t r = lu.perm[i];
    double rowmax = 0.0;
    for (int32_t e = a.ptr[r]; e < a.ptr[r + 1]; ++e) {
      w[lu.iperm[a.col[e]]] = a.val[e];
      rowmax = std::max(rowmax, std::fabs(a.val[e]));
    }
    const auto &lr = lu.lrow[i];
    auto &lv = lu.lval[i];
    for (size_t q = 0; q < lr.size(); ++q) {
      const int32_t k = lr[q];
      const double l = w[k] / lu.uval[k][0];
      lv[q] = l;
      w[k] = 0.0;
      const auto &ur = lu.urow[k];
      const auto &uv = lu.uval[k];
      for (size_t s = 1; s < ur.size(); ++s) w[ur[s]] -= l * uv[s];
    }
    const auto &ur = lu.urow[i];
    auto &uv = lu.uval[i];
    for (size_t s = 0; s < ur.size(); ++s) {
      uv[s] = w[ur[s]];
      w[ur[s]] = 0.0;
    }
    if (!std::isfinite(uv[0]) || std::fabs(uv[0]) <= 1e-13 * rowmax || rowmax == 0.0) {
      err = "G_x is singular to working precision (pivot " + std::to_string(i) + ")";
      return false;
    }
  }
  return true;
}

void lu_solve(const LuPlan &lu, std::vector<double> &b) {
  const int32_t n = lu.n;
  std::vector<double> y(n);
  for (int32_t i = 0; i < n; ++i) y[i] = b[lu.perm[i]];
  for (int32_t i = 0; i < n; ++i) {
    double s = y[i];
    const auto &lr = lu.lrow[i];
    const auto &lv = lu.lval[i];
    for (size_t q = 0; q < lr.size(); ++q) s -= lv[q] * y[lr[q]];
    y[i] = s;
  }
  for (int32_t i = n - 1; i >= 0; --i) {
    const auto &ur = lu.urow[i];
    const auto &uv = lu.uval[i];
    double s = y[i];
    for (size_t q = 1; q < ur.size(); ++q) s -= uv[q] * y[ur[q]];
    y[i] = s / uv[0];
  }
  for (int32_t i = 0; i < n; ++i) b[lu.perm[i]] = y[i];
}

void lu_solve_t(const LuPlan &lu, std::vector<double> &b) {
  // A^T = P^T U^T L^T P
  const int32_t n = lu.n;
  std::vector<double> y(n);
  for (int32_t i = 0; i < n; ++i) y[i] = b[lu.perm[i]];
  for (int32_t k = 0; k < n; ++k) {  // U^T z = y, by columns of U^T (rows of U)
    const auto &ur = lu.urow[k];
    const auto &uv = lu.uval[k];
    const double z = y[k] / uv[0];
    y[k] = z;
    for (size_t q = 1; q < ur.size(); ++q) y[ur[q]] -= uv[q] * z;
  }
  for (int32_t i = n - 1; i >= 0; --i) {  // L^T w = z, by columns of L^T (rows of L)
    const auto &lr = lu.lrow[i];
    const auto &lv = lu.lval[i];
    const double z = y[i];
    for (size_t q = 0; q < lr.size(); ++q) y[lr[q]] -= lv[q] * z;
  }
  for (int32_t i = 0; i < n; ++i) b[lu.perm[i]] = y[i];
}

namespace {

// Group rows by level; `row_entries(i, cols, vals)` appends row i's entries.
template <class F>
void make_sweep(Sweep &s, int32_t n, const std::vector<int32_t> &level, int32_t n_levels,
                F row_entries, const std::vector<double> *diag) {
  s.lev_ptr.assign(n_levels + 1, 0);
  for (int32_t i = 0; i < n; ++i) s.lev_ptr[level[i] + 1]++;
  for (int32_t l = 0; l < n_levels; ++l) s.lev_ptr[l + 1] += s.lev_ptr[l];
  s.rows.assign(n, 0);
  std::vector<int32_t> fill(s.lev_ptr.begin(), s.lev_ptr.end() - 1);
  for (int32_t i = 0; i < n; ++i) s.rows[fill[level[i]]++] = i;  // ascending within a level
  s.ptr.assign(n + 1, 0);
  s.col.clear();
  s.val.clear();
  s.dinv.clear();
  for (int32_t pos = 0; pos < n; ++pos) {
    const int32_t i = s.rows[pos];
    row_entries(i, s.col, s.val);
    s.ptr[pos + 1] = (int32_t)s.col.size();
    if (diag) s.dinv.push_back(1.0 / (*diag)[i]);
  }
}

}  // namespace

void lu_sweeps(const LuPlan &lu, Sweep &sl, Sweep &su, Sweep &sut, Sweep &slt, std::vector<double> &pivinv,
               LuSweepsWork *work) {
  const int32_t n = lu.n;
  LuSweepsWork local;
  LuSweepsWork &w = work ? *work : local;
  // U = D Uh with Uh unit upper triangular: U^{-1} = Uh^{-1} D^{-1} and
  // U^{-T} = D^{-1} Uh^{-T}, so every sweep has a unit diagonal and each solve
  // scales by D^{-1} between its two sweeps.
  pivinv.assign(n, 0.0);
  for (int32_t k = 0; k < n; ++k) pivinv[k] = 1.0 / lu.uval[k][0];
  // rows of Uh^T and L^T in flat arrays, each row in ascending column order
  // (rows of U and L visited in ascending order)
  std::vector<int32_t> &tp = w.tp, &lp = w.lp, &tc = w.tc, &lc = w.lc, &tf = w.tf, &lf = w.lf;
  std::vector<double> &tv = w.tv, &lv = w.lv;
  tp.assign(n + 1, 0);
  lp.assign(n + 1, 0);
  for (int32_t k = 0; k < n; ++k) {
    for (size_t q = 1; q < lu.urow[k].size(); ++q) tp[lu.urow[k][q] + 1]++;
    for (int32_t c : lu.lrow[k]) lp[c + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) {
    tp[i + 1] += tp[i];
    lp[i + 1] += lp[i];
  }
  tc.resize(tp[n]);  // every entry is written below
  lc.resize(lp[n]);
  tv.resize(tp[n]);
  lv.resize(lp[n]);
  tf.assign(tp.begin(), tp.end() - 1);
  lf.assign(lp.begin(), lp.end() - 1);
  for (int32_t k = 0; k < n; ++k) {
    const double d = lu.uval[k][0];
    for (size_t q = 1; q < lu.urow[k].size(); ++q) {
      const int32_t e = tf[lu.urow[k][q]]++;
      tc[e] = k;
      tv[e] = lu.uval[k][q] / d;
    }
    for (size_t q = 0; q < lu.lrow[k].size(); ++q) {
      const int32_t e = lf[lu.lrow[k][q]]++;
      lc[e] = k;
      lv[e] = lu.lval[k][q];
    }
  }
  // the four sweeps are independent: one thread each (an exception on a
  // thread is raised again here)
  std::exception_ptr ex[3];
  auto guarded = [&](int k, auto body) {
    return std::thread([&ex, k, body] {
      try {
        body();
      } catch (...) {
        ex[k] = std::current_exception();
      }
    });
  };
  std::thread t0 = guarded(0, [&] {
    make_sweep(sl, n, lu.level_l, lu.n_levels_l,
               [&](int32_t i, std::vector<int32_t> &c, std::vector<double> &v) {
                 c.insert(c.end(), lu.lrow[i].begin(), lu.lrow[i].end());
                 v.insert(v.end(), lu.lval[i].begin(), lu.lval[i].end());
               },
               nullptr);
  });
  std::thread t1 = guarded(1, [&] {
    make_sweep(su, n, lu.level_u, lu.n_levels_u,
               [&](int32_t i, std::vector<int32_t> &c, std::vector<double> &v) {
                 c.insert(c.end(), lu.urow[i].begin() + 1, lu.urow[i].end());
                 const double d = lu.uval[i][0];
                 for (size_t q = 1; q < lu.uval[i].size(); ++q) v.push_back(lu.uval[i][q] / d);
               },
               nullptr);
  });
  std::thread t2 = guarded(2, [&] {
    make_sweep(sut, n, lu.level_l, lu.n_levels_l,
               [&](int32_t i, std::vector<int32_t> &c, std::vector<double> &v) {
                 c.insert(c.end(), tc.begin() + tp[i], tc.begin() + tp[i + 1]);
                 v.insert(v.end(), tv.begin() + tp[i], tv.begin() + tp[i + 1]);
               },
               nullptr);
  });
  make_sweep(slt, n, lu.level_u, lu.n_levels_u,
             [&](int32_t i, std::vector<int32_t> &c, std::vector<double> &v) {
               c.insert(c.end(), lc.begin() + lp[i], lc.begin() + lp[i + 1]);
               v.insert(v.end(), lv.begin() + lp[i], lv.begin() + lp[i + 1]);
             },
             nullptr);
  t0.join();
  t1.join();
  t2.join();
  for (const std::exception_ptr &e : ex)
    if (e) std::rethrow_exception(e);
}

// log2 of the lane group per row of a step: about four entries of the
// step's longest row per lane, as long as rows x lanes stays within the
// lane budget.
int lane_log2(int32_t rows, int32_t longest, int lane_budget) {
  int lg = 0;
  while (lg < 6 && (1 << lg) * 4 < longest) ++lg;
  while (lg > 0 && (int64_t)rows << lg > lane_budget) --lg;
  return lg;
}

namespace {

// Append rows (positions of `in`) as one step of the output: a plain level,
// or (block = true) a block with its internal entries folded into the dense
// inverse of its triangular system.
void emit_rows(const Sweep &in, const std::vector<int32_t> &pos, bool block, int lane_budget,
               std::vector<int32_t> &local, Schedule &out) {
  Sweep &o = out.s;
  const int32_t b = (int32_t)o.rows.size(), rows = (int32_t)pos.size();
  if (block)
    for (int32_t a = 0; a < rows; ++a) local[in.rows[pos[a]]] = a;
  int32_t longest = 0;
  std::vector<long double> M;
  if (block) M.assign((size_t)rows * rows, 0.0L);
  for (int32_t a = 0; a < rows; ++a) {
    const int32_t p = pos[a];
    o.rows.push_back(in.rows[p]);
    if (!in.dinv.empty()) o.dinv.push_back(in.dinv[p]);
    const int32_t start = (int32_t)o.col.size();
    for (int32_t q = in.ptr[p]; q < in.ptr[p + 1]; ++q) {
      const int32_t c = in.col[q];
      if (block && local[c] >= 0) {
        M[(size_t)a + (size_t)local[c] * rows] = in.val[q];
      } else {
        o.col.push_back(c);
        o.val.push_back(in.val[q]);
      }
    }
    o.ptr.push_back((int32_t)o.col.size());
    longest = std::max(longest, (int32_t)o.col.size() - start);
    if (block) M[(size_t)a * (rows + 1)] = in.dinv.empty() ? 1.0L : 1.0L / in.dinv[p];
  }
  int32_t off = -1;
  if (block) {
    // column j of M^{-1} by forward substitution on e_j (extended precision)
    off = (int32_t)out.dense.size();
    out.dense.resize(out.dense.size() + (size_t)rows * rows, 0.0);
    std::vector<long double> y(rows);
    for (int32_t j = 0; j < rows; ++j) {
      for (int32_t a = 0; a < rows; ++a) {
        long double acc = (a == j) ? 1.0L : 0.0L;
        for (int32_t c = j; c < a; ++c) acc -= M[(size_t)a + (size_t)c * rows] * y[c];
        y[a] = a < j ? 0.0L : acc / M[(size_t)a * (rows + 1)];
      }
      for (int32_t a = j; a < rows; ++a) out.dense[off + (size_t)a + (size_t)j * rows] = (double)y[a];
    }
    for (int32_t a = 0; a < rows; ++a) local[in.rows[pos[a]]] = -1;
  }
  out.meta.insert(out.meta.end(), {b, rows, lane_log2(rows, longest, lane_budget), off});
}

// Level steps for the rows `order` (positions of `in`, a valid sweep order),
// levels counted among these rows only; runs of narrow levels with at most
// `bmax` rows in all become blocks.  Returns the number of steps.
int32_t emit_levels(const Sweep &in, const std::vector<int32_t> &order, std::vector<int32_t> &lvl_of_row,
                    int bmax, int lane_budget, std::vector<int32_t> &local, Schedule *out) {
  // level among `order` rows (dependencies outside are already solved)
  int32_t nl = 0;
  for (int32_t p : order) lvl_of_row[in.rows[p]] = 0;
  for (int32_t p : order) {
    int32_t lv = 0;
    for (int32_t q = in.ptr[p]; q < in.ptr[p + 1]; ++q) {
      const int32_t d = lvl_of_row[in.col[q]];
      if (d >= 0) lv = std::max(lv, d + 1);
    }
    lvl_of_row[in.rows[p]] = lv;
    nl = std::max(nl, lv + 1);
  }
  std::vector<std::vector<int32_t>> levels(nl);
  for (int32_t p : order) levels[lvl_of_row[in.rows[p]]].push_back(p);
  for (int32_t p : order) lvl_of_row[in.rows[p]] = -1;
  int32_t steps = 0, l = 0;
  while (l < nl) {
    int32_t l2 = l + 1, rows = (int32_t)levels[l].size();
    if (bmax > 1 && rows <= bmax)
      while (l2 < nl && rows + (int32_t)levels[l2].size() <= bmax) rows += (int32_t)levels[l2++].size();
    const bool block = (l2 - l) >= 2;
    std::vector<int32_t> pos;
    for (int32_t k = l; k < l2; ++k) pos.insert(pos.end(), levels[k].begin(), levels[k].end());
    if (out) emit_rows(in, pos, block, lane_budget, local, *out);
    ++steps;
    l = l2;
  }
  return steps;
}

}  // namespace

namespace {

// The cut of a sweep (see build_schedule): for the cut factors f = 1 .. 32,
// subtrees of at most total / (waves f) work go to the waves by
// longest-processing-time-first and single-subtree moves, and the cut with
// the lowest modelled cost wins.  Returns the factor chosen (0: no wave step)
// and the owner of every row.
int choose_cut(const Sweep &in, int32_t n, const std::vector<int32_t> &parent, const ScheduleParams &prm, int bmax,
               std::vector<int32_t> &lvl, std::vector<int32_t> &local, std::vector<int32_t> &owner) {
  const int32_t npos = (int32_t)in.rows.size();
  const int nw = prm.n_waves;
  std::vector<int32_t> all(npos);
  for (int32_t p = 0; p < npos; ++p) all[p] = p;
  // subtree work (rows + entries) in the elimination tree (parent > child)
  std::vector<double> wk(n, 0.0), sub(n, 0.0);
  double total = 0.0;
  for (int32_t p = 0; p < npos; ++p) {
    wk[in.rows[p]] = 1.0 + (in.ptr[p + 1] - in.ptr[p]);
    total += wk[in.rows[p]];
  }
  std::vector<std::vector<int32_t>> kids(n);
  std::vector<int32_t> roots;
  for (int32_t v = 0; v < n; ++v) {
    sub[v] += wk[v];
    if (parent[v] >= 0) {
      sub[parent[v]] += sub[v];
      kids[parent[v]].push_back(v);
    } else {
      roots.push_back(v);
    }
  }
  // costs in wave-unit times: a workgroup barrier step ~ 5 units
  const double kBarrier = 5.0, kUnit = 1.0;
  const double plain_cost = kBarrier * emit_levels(in, all, lvl, bmax, prm.lane_budget, local, nullptr);
  double best = plain_cost;
  int best_f = 0;
  std::vector<int32_t> best_owner;
  for (int f : {1, 2, 4, 8, 16, 32}) {
    const double target = total / (nw * f);
    std::vector<int32_t> stack(roots), subroots;
    std::vector<char> top(n, 0);
    while (!stack.empty()) {
      const int32_t v = stack.back();
      stack.pop_back();
      if (sub[v] <= target) {
        subroots.push_back(v);
      } else {
        top[v] = 1;
        stack.insert(stack.end(), kids[v].begin(), kids[v].end());
      }
    }
    std::sort(subroots.begin(), subroots.end(),
              [&](int32_t a, int32_t b) { return sub[a] > sub[b] || (sub[a] == sub[b] && a < b); });
    // subtree of every row below the cut, and the level of each row within
    // its subtree (subtrees are independent, so a wave's levels are the
    // union of its subtrees' levels)
    const int32_t ns = (int32_t)subroots.size();
    std::vector<int32_t> sid(n, -1);
    for (int32_t i = 0; i < ns; ++i) {
      std::vector<int32_t> st{subroots[i]};
      while (!st.empty()) {
        const int32_t v = st.back();
        st.pop_back();
        sid[v] = i;
        st.insert(st.end(), kids[v].begin(), kids[v].end());
      }
    }
    // per subtree and level: rows and longest row
    std::vector<std::vector<std::pair<int32_t, int32_t>>> prof(ns);
    {
      std::vector<int32_t> wl(n, -1);
      for (int32_t p = 0; p < npos; ++p) {
        const int32_t r = in.rows[p];
        if (sid[r] < 0) continue;
        int32_t lv = 0;
        for (int32_t q = in.ptr[p]; q < in.ptr[p + 1]; ++q)
          if (sid[in.col[q]] == sid[r]) lv = std::max(lv, wl[in.col[q]] + 1);
        wl[r] = lv;
        auto &P = prof[sid[r]];
        if ((int32_t)P.size() <= lv) P.resize(lv + 1, {0, 0});
        P[lv].first += 1;
        P[lv].second = std::max(P[lv].second, in.ptr[p + 1] - in.ptr[p]);
      }
    }
    // units a wave emits for a set of subtrees: merged levels, runs of
    // narrow levels as wave blocks (two units), others split into units
    // of 64 >> lg rows (lg: lanes per row so the longest fits in
    // kSlotsAhead slots), as emit_wave_step and pack_schedule do
    auto wave_units = [&](const std::vector<int32_t> &set) {
      std::vector<std::pair<int32_t, int32_t>> M;
      for (int32_t i : set) {
        if (M.size() < prof[i].size()) M.resize(prof[i].size(), {0, 0});
        for (size_t l = 0; l < prof[i].size(); ++l) {
          M[l].first += prof[i][l].first;
          M[l].second = std::max(M[l].second, prof[i][l].second);
        }
      }
      auto split = [](int32_t rows, int32_t longest) {
        int lg = 0;
        while (lg < 6 && (1 << lg) * kSlotsAhead < longest) ++lg;
        const int32_t per = std::max(1, 64 >> lg);
        return (rows + per - 1) / per;
      };
      int64_t units = 0;
      for (size_t l = 0, L = M.size(); l < L;) {
        size_t l2 = l;
        int32_t rows = 0, longest = 0;
        if (in.dinv.empty())
          while (l2 < L && rows + M[l2].first <= kWaveBlockRows) {
            rows += M[l2].first;
            longest = std::max(longest, M[l2].second);
            ++l2;
          }
        if (l2 - l >= 3) {
          units += 1 + split(rows, longest);
          l = l2;
        } else {
          units += split(M[l].first, M[l].second);
          ++l;
        }
      }
      return units;
    };
    // longest-processing-time-first by subtree work, then moves of single
    // subtrees off the wave with the most units while that lowers the most
    std::vector<double> load(nw, 0.0);
    std::vector<std::vector<int32_t>> sets(nw);
    for (int32_t i = 0; i < ns; ++i) {
      const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[w] += sub[subroots[i]];
      sets[w].push_back(i);
    }
    std::vector<int64_t> units(nw);
    for (int w = 0; w < nw; ++w) units[w] = wave_units(sets[w]);
    for (int it = 0; it < 4 * ns; ++it) {
      const int wm = (int)(std::max_element(units.begin(), units.end()) - units.begin());
      int64_t best_m = units[wm], best_a = 0, best_b = 0;
      int best_j = -1, best_w = -1;
      for (size_t j = 0; j < sets[wm].size(); ++j) {
        std::vector<int32_t> rest = sets[wm];
        rest.erase(rest.begin() + (long)j);
        const int64_t a = wave_units(rest);
        if (a >= best_m) continue;
        for (int w2 = 0; w2 < nw; ++w2) {
          if (w2 == wm) continue;
          std::vector<int32_t> more = sets[w2];
          more.push_back(sets[wm][j]);
          const int64_t b = wave_units(more);
          if (std::max(a, b) < best_m) {
            best_m = std::max(a, b);
            best_a = a;
            best_b = b;
            best_j = (int)j;
            best_w = w2;
          }
        }
      }
      if (best_j < 0) break;
      sets[best_w].push_back(sets[wm][best_j]);
      sets[wm].erase(sets[wm].begin() + best_j);
      units[wm] = best_a;
      units[best_w] = best_b;
    }
    std::fill(owner.begin(), owner.end(), -1);
    for (int w = 0; w < nw; ++w)
      for (int32_t i : sets[w]) {
        std::vector<int32_t> st{subroots[i]};
        while (!st.empty()) {
          const int32_t v = st.back();
          st.pop_back();
          owner[v] = w;
          st.insert(st.end(), kids[v].begin(), kids[v].end());
        }
      }
    // wave makespan: the most units on one wave
    const double makespan = kUnit * (double)*std::max_element(units.begin(), units.end());
    std::vector<int32_t> order;
    for (int32_t p = 0; p < npos; ++p)
      if (owner[in.rows[p]] < 0) order.push_back(p);
    const double cost =
        kBarrier * (1 + emit_levels(in, order, lvl, bmax, prm.lane_budget, local, nullptr)) + makespan;
    if (cost < best) {
      best = cost;
      best_f = f;
      best_owner = owner;
    }
  }
  if (best_f != 0) owner = best_owner;
  return best_f;
}

}  // namespace

// Sweep schedule.  Steps are plain levels, dense-inverse blocks of merged
// narrow levels, or one wave step: the elimination tree is cut into disjoint
// subtrees (each subtree's rows depend only on the subtree and on rows outside
// it that are solved before), the subtrees are assigned to the workgroup's
// waves (longest-processing-time-first, then single-subtree moves that lower
// the largest number of units on one wave), and every wave walks its
// subtrees level by level with wave-local ordering only.  The cut is chosen
// by a small cost model (a workgroup barrier step ~ 5 wave units); the wave
// step comes first in forward sweeps (leaves first) and last in backward
// sweeps.
// The cut (the search above, the costly part) is taken from `cut` when it
// holds one, and stored there otherwise.
Schedule build_schedule(const Sweep &in, int32_t n, const std::vector<int32_t> &parent, bool forward,
                        const ScheduleParams &prm, ScheduleCut *cut) {
  const int bmax = std::min(prm.bmax, prm.block_rows);
  Schedule out;
  std::vector<int32_t> local(n, -1), lvl(n, -1);
  const int32_t npos = (int32_t)in.rows.size();
  std::vector<int32_t> pos_of(n, -1);
  for (int32_t p = 0; p < npos; ++p) pos_of[in.rows[p]] = p;
  std::vector<int32_t> all(npos);
  for (int32_t p = 0; p < npos; ++p) all[p] = p;

  out.s.ptr.assign(1, 0);
  const int nw = prm.n_waves;
  if (prm.wave_mode == 0 || nw < 2 || (int32_t)parent.size() != n ||
      (cut && cut->valid && cut->plain)) {
    emit_levels(in, all, lvl, bmax, prm.lane_budget, local, &out);
    return out;
  }
  std::vector<int32_t> owner(n, -1);  // wave of a subtree row, -1 = top part
  if (cut && cut->valid && (int32_t)cut->owner.size() == n) {
    owner = cut->owner;
  } else {
    int best_f = choose_cut(in, n, parent, prm, bmax, lvl, local, owner);
    if (cut) {
      cut->valid = true;
      cut->plain = best_f == 0;
      cut->owner = owner;
    }
    if (best_f == 0) {
      emit_levels(in, all, lvl, bmax, prm.lane_budget, local, &out);
      return out;
    }
  }
  std::vector<int32_t> top_order;
  for (int32_t p = 0; p < npos; ++p)
    if (owner[in.rows[p]] < 0) top_order.push_back(p);
  auto emit_wave_step = [&]() {
    // wave levels within each wave (dependencies inside the same wave only)
    std::vector<int32_t> wl(n, -1);
    std::vector<std::vector<std::vector<int32_t>>> W(nw);
    for (int32_t p = 0; p < npos; ++p) {
      const int32_t r = in.rows[p];
      const int32_t w = owner[r];
      if (w < 0) continue;
      int32_t lv = 0;
      for (int32_t q = in.ptr[p]; q < in.ptr[p + 1]; ++q)
        if (owner[in.col[q]] == w) lv = std::max(lv, wl[in.col[q]] + 1);
      wl[r] = lv;
      if ((int32_t)W[w].size() <= lv) W[w].resize(lv + 1);
      W[w][lv].push_back(p);
    }
    const int32_t dir0 = (int32_t)out.wdir.size();
    const int32_t b = (int32_t)out.s.rows.size();
    int32_t rows_total = 0;
    // rows at positions `ps` of `in` as one wave unit; entries to columns with
    // local[c] >= 0 (inside a wave block) are left out
    auto emit_unit = [&](const std::vector<int32_t> &ps) {
      const int32_t first = (int32_t)out.s.rows.size();
      int32_t longest = 0;
      for (int32_t p : ps) {
        out.s.rows.push_back(in.rows[p]);
        if (!in.dinv.empty()) out.s.dinv.push_back(in.dinv[p]);
        const int32_t start = (int32_t)out.s.col.size();
        for (int32_t q = in.ptr[p]; q < in.ptr[p + 1]; ++q)
          if (local[in.col[q]] < 0) {
            out.s.col.push_back(in.col[q]);
            out.s.val.push_back(in.val[q]);
          }
        out.s.ptr.push_back((int32_t)out.s.col.size());
        longest = std::max(longest, (int32_t)out.s.col.size() - start);
      }
      out.wlev.insert(out.wlev.end(), {first, (int32_t)ps.size(), lane_log2((int32_t)ps.size(), longest, 64), 0});
      rows_total += (int32_t)ps.size();
    };
    // a run of narrow wave levels with at most kWaveBlockRows rows in all:
    // a residual unit (entries to earlier rows) and an assigning unit that
    // applies the inverse of the run's unit lower-triangular block, whose
    // "entries" are the inverse's row (columns = the run's rows, diagonal 1)
    auto emit_wave_block = [&](const std::vector<int32_t> &ps) {
      const int32_t R = (int32_t)ps.size();
      for (int32_t a = 0; a < R; ++a) local[in.rows[ps[a]]] = a;
      std::vector<long double> M((size_t)R * R, 0.0L);  // column-major
      for (int32_t a = 0; a < R; ++a) {
        M[(size_t)a * (R + 1)] = 1.0L;
        for (int32_t q = in.ptr[ps[a]]; q < in.ptr[ps[a] + 1]; ++q)
          if (local[in.col[q]] >= 0) M[(size_t)a + (size_t)local[in.col[q]] * R] = in.val[q];
      }
      emit_unit(ps);
      // inverse by forward substitution on the unit vectors (extended precision)
      std::vector<long double> inv((size_t)R * R, 0.0L), y(R);
      for (int32_t j = 0; j < R; ++j) {
        for (int32_t a = 0; a < R; ++a) {
          long double acc = (a == j) ? 1.0L : 0.0L;
          for (int32_t c = j; c < a; ++c) acc -= M[(size_t)a + (size_t)c * R] * y[c];
          y[a] = a < j ? 0.0L : acc;
        }
        for (int32_t a = j; a < R; ++a) inv[(size_t)a + (size_t)j * R] = y[a];
      }
      const int32_t first = (int32_t)out.s.rows.size();
      for (int32_t a = 0; a < R; ++a) {
        out.s.rows.push_back(in.rows[ps[a]]);
        for (int32_t c = 0; c <= a; ++c) {
          out.s.col.push_back(in.rows[ps[c]]);
          out.s.val.push_back((double)inv[(size_t)a + (size_t)c * R]);
        }
        out.s.ptr.push_back((int32_t)out.s.col.size());
      }
      out.wlev.insert(out.wlev.end(), {first, R, lane_log2(R, R, 64), 1});
      for (int32_t a = 0; a < R; ++a) local[in.rows[ps[a]]] = -1;
    };
    for (int w = 0; w < nw; ++w) {
      out.wdir.push_back((int32_t)(out.wlev.size() / 4));
      const size_t L = W[w].size();
      size_t l = 0;
      while (l < L) {
        size_t l2 = l;
        int32_t rows = 0;
        if (in.dinv.empty())
          while (l2 < L && rows + (int32_t)W[w][l2].size() <= kWaveBlockRows) rows += (int32_t)W[w][l2++].size();
        if (l2 - l >= 3) {
          std::vector<int32_t> ps;
          for (size_t x = l; x < l2; ++x) ps.insert(ps.end(), W[w][x].begin(), W[w][x].end());
          emit_wave_block(ps);
          l = l2;
        } else {
          emit_unit(W[w][l]);
          ++l;
        }
      }
    }
    out.wdir.push_back((int32_t)(out.wlev.size() / 4));
    out.meta.insert(out.meta.end(), {b, rows_total, 0, -2 - dir0});
  };
  if (forward) {
    emit_wave_step();
    emit_levels(in, top_order, lvl, bmax, prm.lane_budget, local, &out);
  } else {
    emit_levels(in, top_order, lvl, bmax, prm.lane_budget, local, &out);
    emit_wave_step();
  }
  return out;
}

namespace {
// Rows grouped by level (ascending), as {level pointer, rows}.
void group_levels(const std::vector<int32_t> &level, int32_t n_lev, std::vector<int32_t> &ptr,
                  std::vector<int32_t> &rows) {
  ptr.assign(n_lev + 1, 0);
  for (int32_t l : level) ptr[l + 1]++;
  for (int32_t l = 0; l < n_lev; ++l) ptr[l + 1] += ptr[l];
  rows.assign(level.size(), 0);
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (int32_t i = 0; i < (int32_t)level.size(); ++i) rows[fill[level[i]]++] = i;
}
}  // namespace

bool lu_device_maps(const LuPlan &lu, const Csr &gx, LuMaps &mp, std::string &err) {
  const int32_t n = lu.n;
  mp = LuMaps();
  mp.row_ptr.assign(n + 1, 0);
  mp.nl.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    mp.nl[i] = (int32_t)lu.lrow[i].size();
    const int32_t len = mp.nl[i] + (int32_t)lu.urow[i].size();
    mp.row_ptr[i + 1] = mp.row_ptr[i] + len;
    mp.maxpat = std::max(mp.maxpat, len);
    mp.lucol.insert(mp.lucol.end(), lu.lrow[i].begin(), lu.lrow[i].end());
    mp.lucol.insert(mp.lucol.end(), lu.urow[i].begin(), lu.urow[i].end());
  }
  if (mp.maxpat > 65535) {
    err = "LU row pattern too wide for 16-bit positions";
    return false;
  }
  // position of column c within row i (the L part and the U part are each
  // ascending, and every L column is below every U column)
  auto pos_in = [&](int32_t i, int32_t c) -> int32_t {
    const int32_t *b = mp.lucol.data() + mp.row_ptr[i], *e = mp.lucol.data() + mp.row_ptr[i + 1];
    const int32_t *p = std::lower_bound(b, e, c);
    return (p != e && *p == c) ? (int32_t)(p - b) : -1;
  };
  mp.a_ptr.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t r = lu.perm[i];
    for (int32_t e = gx.ptr[r]; e < gx.ptr[r + 1]; ++e) {
      const int32_t p = pos_in(i, lu.iperm[gx.col[e]]);
      if (p < 0) {
        err = "internal: G_x entry outside the LU pattern";
        return false;
      }
      mp.a_src.push_back(e);
      mp.a_dst.push_back((uint16_t)p);
    }
    mp.a_ptr[i + 1] = (int32_t)mp.a_src.size();
  }
  mp.upd_ptr.assign(n + 1, 0);
  mp.step.assign(4 * (size_t)mp.row_ptr[n], 0);
  for (int32_t i = 0; i < n; ++i) {
    for (size_t q = 0; q < lu.lrow[i].size(); ++q) {
      const int32_t k = lu.lrow[i][q];
      int32_t *st = &mp.step[4 * ((size_t)mp.row_ptr[i] + q)];
      st[0] = mp.row_ptr[k] + (int32_t)lu.lrow[k].size();
      st[1] = (int32_t)lu.urow[k].size();
      if (mp.tgt.size() > (size_t)INT32_MAX) {
        err = "too many factor updates for 32-bit offsets";
        return false;
      }
      st[2] = (int32_t)mp.tgt.size();
      st[3] = k;
      for (size_t s = 1; s < lu.urow[k].size(); ++s) {
        const int32_t p = pos_in(i, lu.urow[k][s]);
        if (p < 0) {
          err = "internal: fill outside the LU pattern";
          return false;
        }
        mp.tgt.push_back((uint16_t)p);
      }
    }
    mp.upd_ptr[i + 1] = (int64_t)mp.tgt.size();
  }
  // the dense top block and the levels of the rows below it (a row below b0
  // depends only on earlier rows, so its level stands; levels left empty are
  // dropped)
  const int32_t b0 = n - std::min<int32_t>(kNtDenseTop, n), mb = n - b0;
  mp.b0 = b0;
  auto below = [&](const std::vector<int32_t> &level, int32_t n_levels, std::vector<int32_t> &ptr,
                   std::vector<int32_t> &rows) {
    std::vector<int32_t> renum(n_levels, -1), lvf(b0);
    for (int32_t i = 0; i < b0; ++i) renum[level[i]] = 0;
    int32_t nf = 0;
    for (int32_t l = 0; l < n_levels; ++l)
      if (renum[l] == 0) renum[l] = nf++;
    for (int32_t i = 0; i < b0; ++i) lvf[i] = renum[level[i]];
    group_levels(lvf, nf, ptr, rows);
  };
  below(lu.level_l, lu.n_levels_l, mp.lev_ptr_f, mp.lev_rows_f);
  below(lu.level_u, lu.n_levels_u, mp.lev_ptr_uf, mp.lev_rows_uf);
  mp.ns.assign(mb, 0);
  mp.dmap.assign((size_t)mb * mb, -1);
  for (int32_t r = 0; r < mb; ++r) {
    const int32_t i = b0 + r, base = mp.row_ptr[i], len = mp.row_ptr[i + 1] - base;
    int32_t q = 0;
    while (q < mp.nl[i] && mp.lucol[base + q] < b0) ++q;
    mp.ns[r] = q;
    for (; q < len; ++q) mp.dmap[(size_t)r * mb + (mp.lucol[base + q] - b0)] = q;
  }
  return true;
}

std::vector<int32_t> etree_parent(const LuPlan &lu) {
  std::vector<int32_t> parent(lu.n, -1);
  for (int32_t k = 0; k < lu.n; ++k)
    if (lu.urow[k].size() > 1) parent[k] = lu.urow[k][1];
  return parent;
}

namespace {

// One level or block unit: rows at positions [b, b + rows) of sc.s with lane
// groups of 2^lg.
int32_t pack_unit(const Schedule &sc, int32_t b, int32_t rows, int lg, int max_lanes, Packed &pk) {
  const Sweep &s = sc.s;
  const int32_t w = 1 << lg;
  const int32_t groups = std::max<int32_t>(1, std::min<int32_t>(rows, max_lanes / w));
  const int32_t lanes = groups * w;
  const int32_t passes = rows > 0 ? (rows + groups - 1) / groups : 0;
  int32_t longest = 0;
  for (int32_t r = 0; r < rows; ++r) longest = std::max(longest, s.ptr[b + r + 1] - s.ptr[b + r]);
  const int32_t E0 = (longest + w - 1) / w;
  const int32_t E = (E0 + 3) & ~3;  // whole column quads
  const int32_t slot_base = (int32_t)pk.scol.size(), info_base = (int32_t)pk.irow.size();
  pk.scol.resize(pk.scol.size() + (size_t)passes * E * lanes, 0);
  pk.sval.resize(pk.sval.size() + (size_t)passes * E * lanes, 0.0);
  for (int32_t r = 0; r < rows; ++r) {
    const int32_t p = r / groups, g = r % groups, pos = b + r;
    const int32_t q0 = s.ptr[pos], len = s.ptr[pos + 1] - q0;
    for (int32_t j = 0; j < w; ++j)
      for (int32_t e = 0; e < E; ++e) {
        const int32_t q = j + e * w;
        if (q >= len) continue;
        // a lane's columns in quads, its values in pairs, pass after pass
        const size_t lane = (size_t)g * w + j, base = (size_t)slot_base + (size_t)p * E * lanes;
        const size_t ac = base + (size_t)(e >> 2) * 4 * lanes + 4 * lane + (e & 3);
        const size_t av = base + (size_t)(e >> 1) * 2 * lanes + 2 * lane + (e & 1);
        pk.scol[ac] = s.col[q0 + q];
        pk.sval[av] = s.val[q0 + q];
      }
    pk.irow.push_back(s.rows[pos]);
    if (!s.dinv.empty()) pk.idinv.push_back(s.dinv[pos]);
  }
  const int32_t u = (int32_t)(pk.units.size() / 8);
  pk.units.insert(pk.units.end(), {slot_base, info_base, rows, groups, lg, E, lanes, -1});
  return u;
}

// Byte offset of padded-vector row r (8-byte rows), see Packed.
int32_t wave_off(int32_t r) { return r * 8; }

// One fixed-shape wave unit (see Packed): part k of each listed row (entries
// 256 k .. 256 k + 255 of its entries at positions `pos` of sc.s), lane
// groups of 2^lg.
struct WaveRow {
  int32_t pos, first, end;  // position in sc.s and the entry range of this part
};

// Returns the entry count of each lane in `cnt` (64 per unit).
void pack_wave_unit(const Schedule &sc, const std::vector<WaveRow> &rows, int lg, bool assign, Packed &pk,
                    std::vector<uint8_t> &cnt) {
  const Sweep &s = sc.s;
  const int32_t w = 1 << lg;
  if ((int32_t)rows.size() * w > 64) throw std::runtime_error("internal: wave unit wider than a wave");
  const size_t c0 = pk.wcol.size(), r0 = pk.wrow.size(), v0 = pk.wval.size();
  pk.wcol.resize(c0 + 256, wave_off(0));
  pk.wrow.resize(r0 + 128, wave_off(0));
  pk.wval.resize(v0 + 256, 0.0);
  for (int32_t l = 0; l < 64; ++l) pk.wrow[r0 + 2 * l + 1] = wave_off(1 + l);  // dummy rows
  const int32_t lgbits = (int32_t)((uint32_t)lg << kWaveLgShift);
  const size_t k0 = cnt.size();
  cnt.resize(k0 + 64, 0);
  for (size_t r = 0; r < rows.size(); ++r) {
    const WaveRow &R = rows[r];
    const int32_t row = s.rows[R.pos] + kWavePadRows, len = R.end - R.first;
    if (len > 4 * w) throw std::runtime_error("internal: wave row part longer than its lanes' slots");
    for (int32_t j = 0; j < w; ++j) {
      const int32_t l = (int32_t)r * w + j;
      pk.wrow[r0 + 2 * l] = assign ? wave_off(0) : wave_off(row);
      if ((uint32_t)wave_off(row) > kWaveOffMask) throw std::runtime_error("network too large for wave offsets");
      if (j == 0) pk.wrow[r0 + 2 * l + 1] = wave_off(row);
      for (int32_t e = 0; e < 4; ++e) {
        const int32_t q = j + e * w;
        if (q >= len) continue;
        pk.wcol[c0 + 4 * l + e] = wave_off(s.col[R.first + q] + kWavePadRows);
        const double v = s.val[R.first + q];
        pk.wval[v0 + 128 * (e >> 1) + 2 * l + (e & 1)] = assign ? -v : v;
        cnt[k0 + l] = (uint8_t)(e + 1);
      }
    }
  }
  for (int32_t l = 0; l < 64; ++l) pk.wrow[r0 + 2 * l + 1] |= lgbits;
  pk.wlg.push_back(lg);
}

// Load flags of a wave's units u0 .. u1 - 1 (see Packed): unit u carries in
// its start words which lanes of unit u + kWaveAhead have entries, and which
// have entries 2 or 3.
void set_wave_flags(Packed &pk, const std::vector<uint8_t> &cnt, int32_t u0, int32_t u1) {
  for (int32_t u = u0; u + kWaveAhead < u1; ++u)
    for (int32_t l = 0; l < 64; ++l) {
      const uint8_t c = cnt[64 * (size_t)(u + kWaveAhead) + l];
      uint32_t w = (uint32_t)pk.wrow[128 * (size_t)u + 2 * l];
      if (c >= 1) w |= 1u << kWaveActBit;
      if (c >= 3) w |= 1u << kWaveTwoBit;
      pk.wrow[128 * (size_t)u + 2 * l] = (int32_t)w;
    }
}

// Lanes per row (log2) so that `longest` entries fit in four slots per lane.
int wave_lg(int32_t longest) {
  int lg = 0;
  while (lg < 6 && (1 << lg) * kSlotsAhead < longest) ++lg;
  return lg;
}

}  // namespace

Packed pack_schedule(const Schedule &sc, int lanes) {
  Packed pk;
  pack_schedule(sc, lanes, pk);
  return pk;
}

void pack_schedule(const Schedule &sc, int lanes, Packed &pk) {
  for (std::vector<int32_t> *v : {&pk.steps, &pk.units, &pk.wdir, &pk.irow, &pk.wlg, &pk.wcol, &pk.wrow}) v->clear();
  for (std::vector<double> *v : {&pk.idinv, &pk.wval}) v->clear();
  // element 0 of the slots and of the block inverses is a zero that lanes
  // without an entry read
  pk.scol.assign(1, 0);
  pk.sval.assign(1, 0.0);
  pk.dense.assign(1, 0.0);
  pk.dense.insert(pk.dense.end(), sc.dense.begin(), sc.dense.end());
  constexpr int32_t kPart = 64 * kSlotsAhead;  // entries of one row in one wave unit
  const size_t ns = sc.meta.size() / 4;
  for (size_t st = 0; st < ns; ++st) {
    const int32_t b = sc.meta[4 * st], rows = sc.meta[4 * st + 1], lg = sc.meta[4 * st + 2];
    const int32_t kind = sc.meta[4 * st + 3];
    if (kind <= -2) {
      if (!sc.s.dinv.empty()) throw std::runtime_error("internal: wave steps need a unit diagonal");
      const int32_t d = -2 - kind;
      const int32_t off = (int32_t)pk.wdir.size();
      const int32_t nw = lanes / 64;
      std::vector<uint8_t> cnt;  // entries per lane of every wave unit
      for (int32_t w = 0; w < nw; ++w) {
        const int32_t wu0 = (int32_t)pk.wlg.size();
        cnt.resize(64 * (size_t)wu0, 0);
        pk.wdir.push_back(wu0);
        for (int32_t j = sc.wdir[d + w]; j < sc.wdir[d + w + 1]; ++j) {
          const int32_t b = sc.wlev[4 * j], rows = sc.wlev[4 * j + 1], assign = sc.wlev[4 * j + 3];
          if (assign) {
            // the second unit of a wave block reads all its rows before it
            // writes any: one unit
            int32_t longest = 0;
            std::vector<WaveRow> rs;
            for (int32_t r = 0; r < rows; ++r) {
              rs.push_back({b + r, sc.s.ptr[b + r], sc.s.ptr[b + r + 1]});
              longest = std::max(longest, sc.s.ptr[b + r + 1] - sc.s.ptr[b + r]);
            }
            pack_wave_unit(sc, rs, wave_lg(longest), true, pk, cnt);
            continue;
          }
          // a subtracting unit's rows are independent: split it into units
          // of 64 >> lg rows with lanes enough for each row's first 256
          // entries; longer rows continue in further units
          int32_t longest = 0, parts = 1;
          for (int32_t r = 0; r < rows; ++r) {
            const int32_t len = sc.s.ptr[b + r + 1] - sc.s.ptr[b + r];
            longest = std::max(longest, std::min(len, kPart));
            parts = std::max(parts, (len + kPart - 1) / kPart);
          }
          for (int32_t k = 0; k < parts; ++k) {
            std::vector<WaveRow> rs;
            int32_t lk = 0;
            for (int32_t r = 0; r < rows; ++r) {
              const int32_t q0 = sc.s.ptr[b + r] + k * kPart, q1 = std::min(sc.s.ptr[b + r + 1], q0 + kPart);
              if (k > 0 && q0 >= q1) continue;
              rs.push_back({b + r, q0, std::max(q0, q1)});
              lk = std::max(lk, q1 - q0);
            }
            const int ul = wave_lg(k == 0 ? longest : lk);
            const size_t per = (size_t)std::max(1, 64 >> ul);
            for (size_t r0 = 0; r0 < rs.size(); r0 += per)
              pack_wave_unit(sc, std::vector<WaveRow>(rs.begin() + r0, rs.begin() + std::min(rs.size(), r0 + per)),
                             ul, false, pk, cnt);
          }
        }
        set_wave_flags(pk, cnt, wu0, (int32_t)pk.wlg.size());
      }
      pk.wdir.push_back((int32_t)pk.wlg.size());
      pk.steps.insert(pk.steps.end(), {off, 0, 2, 0});
    } else {
      const int32_t u = pack_unit(sc, b, rows, lg, lanes, pk);
      pk.steps.insert(pk.steps.end(), {u, 0, kind >= 0 ? 1 : 0, kind >= 0 ? kind + 1 : 0});
      if (kind >= 0) {
        // the block's inverse row-major (the lanes of a row read consecutive
        // columns: whole cache lines)
        double *M = pk.dense.data() + kind + 1;
        for (int32_t a = 0; a < rows; ++a)
          for (int32_t c = 0; c < a; ++c) std::swap(M[(size_t)a + (size_t)c * rows], M[(size_t)a * rows + c]);
      }
    }
  }
}

bool wave_records(const Packed &pk, bool compact, bool fp64, std::vector<char> &out) {
  const size_t nu = pk.wlg.size();
  const int rb = compact ? (fp64 ? kWaveRecCompact64 : kWaveRecCompact32) : (fp64 ? kWaveRecWide64 : kWaveRecWide32);
  out.assign(nu * rb, 0);
  const int vbase = compact ? 1024 : 1536;
  for (size_t u = 0; u < nu; ++u) {
    char *r = out.data() + u * rb;
    for (int l = 0; l < 64; ++l) {
      const int32_t *wc = &pk.wcol[256 * u + 4 * l];
      const uint32_t ws = (uint32_t)pk.wrow[128 * u + 2 * l], ww = (uint32_t)pk.wrow[128 * u + 2 * l + 1];
      if (compact) {
        uint32_t rows[6];
        for (int e = 0; e < 4; ++e) rows[e] = (uint32_t)wc[e] >> 3;
        rows[4] = (ws & kWaveOffMask) >> 3;
        rows[5] = (ww & kWaveOffMask) >> 3;
        for (uint32_t v : rows)
          if (v > 0xffffu) {
            out.clear();
            return false;
          }
        const uint32_t h[4] = {rows[0] | rows[1] << 16, rows[2] | rows[3] << 16, rows[4] | rows[5] << 16,
                               ((ws >> kWaveActBit) & 1u) | ((ws >> kWaveTwoBit) & 1u) << 1 |
                                   (ww >> kWaveLgShift) << 2};
        std::memcpy(r + 16 * l, h, 16);
      } else {
        std::memcpy(r + 16 * l, wc, 16);
        const uint32_t w2[2] = {ws, ww};
        std::memcpy(r + 1024 + 8 * l, w2, 8);
      }
      for (int e = 0; e < 4; ++e) {
        const double v = pk.wval[256 * u + 128 * (e >> 1) + 2 * l + (e & 1)];
        if (fp64) {
          std::memcpy(r + vbase + 1024 * (e >> 1) + 16 * l + 8 * (e & 1), &v, 8);
        } else {
          const float f = (float)v;
          std::memcpy(r + vbase + 16 * l + 4 * e, &f, 4);
        }
      }
    }
  }
  return true;
}

}  // namespace rh
