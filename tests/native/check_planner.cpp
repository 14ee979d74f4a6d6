// CPU check of the host planner of librh (compiled and run by
// tests/test_native.py).  Reads a network from a binary file, then checks
//  1. the fixed-pattern LU: A x = b and A^T x = b solves against a dense
//     Gaussian elimination of the same G_x (small networks only);
//  2. the device sweep schedules: a host emulation of the kernel's step
//     structure (plain levels and dense-inverse blocks) against a plain
//     row-by-row sweep, for block sizes 0, 16 and 64.
// Prints "max_err <name> <value>" lines; exit status 0 unless it fails to run.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2201_00241_amd/csrc/rh_internal.h"

using namespace rh;

template <class T>
static std::vector<T> rd(FILE *f, size_t n) {
  std::vector<T> v(n);
  if (fread(v.data(), sizeof(T), n, f) != n) v.clear();
  return v;
}

// Emulates the kernel's step structure.  In a wave step the waves run one
// after the other in reverse order, each level by level, and every row first
// checks that the rows it reads are final (solved in an earlier step, or
// earlier in its own wave); `ok` turns false otherwise.
static void emulate(const Schedule &sc, std::vector<double> &X, bool &ok) {
  const Sweep &s = sc.s;
  const size_t ns = sc.meta.size() / 4;
  std::vector<char> done(X.size(), 0);
  for (size_t p = 0; p < s.rows.size(); ++p) done[s.rows[p]] = 0;
  std::vector<char> pending(X.size(), 0);
  for (size_t p = 0; p < s.rows.size(); ++p) pending[s.rows[p]] = 1;
  auto row = [&](int p) {
    double part = 0;
    for (int q = s.ptr[p]; q < s.ptr[p + 1]; ++q) {
      if (pending[s.col[q]]) ok = false;
      part += s.val[q] * X[s.col[q]];
    }
    double v = X[s.rows[p]] - part;
    if (!s.dinv.empty()) v *= s.dinv[p];
    X[s.rows[p]] = v;
    pending[s.rows[p]] = 0;
  };
  for (size_t st = 0; st < ns; ++st) {
    const int b = sc.meta[4 * st], rows = sc.meta[4 * st + 1], off = sc.meta[4 * st + 3];
    if (off <= -2) {
      const int d = -2 - off;
      const int nw = 16;
      for (int w = nw - 1; w >= 0; --w)
        for (int j = sc.wdir[d + w]; j < sc.wdir[d + w + 1]; ++j) {
          const int first = sc.wlev[4 * j], nr = sc.wlev[4 * j + 1];
          if (sc.wlev[4 * j + 3] == 0) {
            for (int r = 0; r < nr; ++r) row(first + r);
          } else {
            // assigning unit of a wave block: all reads, then all writes
            std::vector<double> v(nr, 0.0);
            for (int r = 0; r < nr; ++r)
              for (int q = s.ptr[first + r]; q < s.ptr[first + r + 1]; ++q) {
                if (pending[s.col[q]]) ok = false;
                v[r] += s.val[q] * X[s.col[q]];
              }
            for (int r = 0; r < nr; ++r) X[s.rows[first + r]] = v[r];
          }
        }
      continue;
    }
    if (off < 0) {
      // rows of a level are independent: all read before any is written
      for (int a = 0; a < rows; ++a)
        for (int q = s.ptr[b + a]; q < s.ptr[b + a + 1]; ++q)
          if (pending[s.col[q]]) ok = false;
    }
    std::vector<double> r(rows);
    for (int a = 0; a < rows; ++a) {
      const int p = b + a;
      double part = 0;
      for (int q = s.ptr[p]; q < s.ptr[p + 1]; ++q) {
        if (off >= 0 && pending[s.col[q]]) ok = false;  // external entries only
        part += s.val[q] * X[s.col[q]];
      }
      double v = X[s.rows[p]] - part;
      if (off < 0) {
        if (!s.dinv.empty()) v *= s.dinv[p];
        X[s.rows[p]] = v;
        pending[s.rows[p]] = 0;
      } else {
        r[a] = v;
      }
    }
    if (off >= 0)
      for (int a = 0; a < rows; ++a) {
        double acc = 0;
        for (int c = 0; c <= a; ++c) acc += sc.dense[off + a + (size_t)c * rows] * r[c];
        X[s.rows[b + a]] = acc;
        pending[s.rows[b + a]] = 0;
      }
  }
  for (size_t i = 0; i < X.size(); ++i)
    if (pending[i]) ok = false;
  (void)done;
}

// The wave-unit arrays the kernel walks: whole 64-lane records, unit ranges
// of the waves in order, every offset a whole 8-byte row of the padded
// vector (n rows behind kWavePadRows) and lg within a wave.  Returns false
// on any inconsistency.
static bool check_wave_walk(const Packed &pk, int n) {
  const size_t nu = pk.wlg.size();
  if (pk.wcol.size() != 256 * nu || pk.wrow.size() != 128 * nu || pk.wval.size() != 256 * nu) return false;
  const long lim = 8L * (n + kWavePadRows);
  for (int32_t o : pk.wcol)
    if (o < 0 || o % 8 || o >= lim) return false;
  for (size_t k = 0; k < pk.wrow.size(); ++k) {
    const long o = (long)((uint32_t)pk.wrow[k] & kWaveOffMask);
    if (o % 8 || o >= lim) return false;
    if (k % 2 == 1 && (int)((uint32_t)pk.wrow[k] >> kWaveLgShift) != pk.wlg[k / 128]) return false;
    if (k % 2 == 0 && ((uint32_t)pk.wrow[k] >> kWaveLgShift & 1u)) return false;  // unused bit
  }
  for (int32_t lg : pk.wlg)
    if (lg < 0 || lg > 6) return false;
  int prev = 0;
  for (size_t st = 0; st < pk.steps.size() / 4; ++st) {
    if (pk.steps[4 * st + 2] != 2) continue;
    const int a = pk.steps[4 * st];
    for (int w = 0; w <= 16; ++w) {
      const int u = pk.wdir[a + w];
      if (u < prev || u > (int)nu) return false;
      prev = u;
    }
  }
  return true;
}

// The device records of the wave units (wave_records) decoded back, field by
// field, against the packed arrays: wide and compact, FP64 and FP32.
static bool check_records(const Packed &pk) {
  std::vector<char> w64, w32, c64, c32;
  if (!wave_records(pk, false, true, w64) || !wave_records(pk, false, false, w32)) return false;
  if (!wave_records(pk, true, true, c64) || !wave_records(pk, true, false, c32)) return false;
  const size_t nu = pk.wlg.size();
  if (w64.size() != nu * kWaveRecWide64 || w32.size() != nu * kWaveRecWide32 ||
      c64.size() != nu * kWaveRecCompact64 || c32.size() != nu * kWaveRecCompact32)
    return false;
  auto u32 = [](const char *p) {
    uint32_t v;
    std::memcpy(&v, p, 4);
    return v;
  };
  for (size_t u = 0; u < nu; ++u)
    for (int l = 0; l < 64; ++l) {
      const uint32_t ws = (uint32_t)pk.wrow[128 * u + 2 * l], ww = (uint32_t)pk.wrow[128 * u + 2 * l + 1];
      const char *hw = w64.data() + u * kWaveRecWide64, *hw32 = w32.data() + u * kWaveRecWide32;
      const char *hc = c64.data() + u * kWaveRecCompact64, *hc32 = c32.data() + u * kWaveRecCompact32;
      for (int e = 0; e < 4; ++e) {
        const uint32_t col = (uint32_t)pk.wcol[256 * u + 4 * l + e];
        if (u32(hw + 16 * l + 4 * e) != col || u32(hw32 + 16 * l + 4 * e) != col) return false;
        const uint32_t hword = u32(hc + 16 * l + 4 * (e >> 1)), hword32 = u32(hc32 + 16 * l + 4 * (e >> 1));
        const uint32_t row = (e & 1) ? hword >> 16 : hword & 0xffffu;
        if (hword != hword32 || row * 8u != col) return false;
        const double v = pk.wval[256 * u + 128 * (e >> 1) + 2 * l + (e & 1)];
        double a, b;
        float f, g;
        std::memcpy(&a, hw + 1536 + 1024 * (e >> 1) + 16 * l + 8 * (e & 1), 8);
        std::memcpy(&b, hc + 1024 + 1024 * (e >> 1) + 16 * l + 8 * (e & 1), 8);
        std::memcpy(&f, hw32 + 1536 + 16 * l + 4 * e, 4);
        std::memcpy(&g, hc32 + 1024 + 16 * l + 4 * e, 4);
        if (std::memcmp(&a, &v, 8) || std::memcmp(&b, &v, 8) || f != (float)v || g != (float)v) return false;
      }
      if (u32(hw + 1024 + 8 * l) != ws || u32(hw + 1028 + 8 * l) != ww) return false;
      const uint32_t rows = u32(hc + 16 * l + 8), fl = u32(hc + 16 * l + 12);
      if ((rows & 0xffffu) * 8u != (ws & kWaveOffMask) || (rows >> 16) * 8u != (ww & kWaveOffMask)) return false;
      if ((fl & 1u) != ((ws >> kWaveActBit) & 1u) || ((fl >> 1) & 1u) != ((ws >> kWaveTwoBit) & 1u) ||
          (fl >> 2) != (ww >> kWaveLgShift) || (int)(fl >> 2) != pk.wlg[u])
        return false;
      if (rows != u32(hc32 + 16 * l + 8) || fl != u32(hc32 + 16 * l + 12)) return false;
    }
  return true;
}

// One fixed-shape wave unit on the padded vector Xp: every lane sums its four
// slots, lane groups combine, and every lane writes X[start] - sum to its
// write row (all reads before any write, as in one wave).  Reads of rows not
// yet final clear `ok`; so does a change of the zero row, or a row written
// by more than one lane.
// `act`/`two`: which lanes load their column quad and first value pair, and
// their second value pair (the flags carried kWaveAhead units earlier; all
// for a wave's first units); a skipped load reads zeros.  A lane with an
// entry its flags skip clears `ok`.
static void wave_unit(const Packed &pk, int u, const bool *act, const bool *two, std::vector<double> &Xp,
                      std::vector<char> &pend, bool &ok) {
  const int w = 1 << pk.wlg[u];
  double part[64], nv[64];
  for (int l = 0; l < 64; ++l) {
    part[l] = 0.0;
    for (int e = 0; e < 4; ++e) {
      const bool loaded = act[l] && (e < 2 || two[l]);
      const double v0 = pk.wval[256 * u + 128 * (e >> 1) + 2 * l + (e & 1)];
      if (!loaded && v0 != 0.0) ok = false;
      const int c = loaded ? pk.wcol[256 * u + 4 * l + e] / 8 : 0;
      const double v = loaded ? v0 : 0.0;
      if (v != 0.0 && pend[c]) ok = false;
      part[l] += v * Xp[c];
    }
  }
  for (int l = 0; l < 64; ++l) {
    double t = 0.0;
    for (int j = (l / w) * w; j < (l / w + 1) * w; ++j) t += part[j];
    nv[l] = Xp[(pk.wrow[128 * u + 2 * l] & kWaveOffMask) / 8] - t;
  }
  std::vector<int> hits(Xp.size(), 0);
  for (int l = 0; l < 64; ++l) {
    const int r = (int)(((uint32_t)pk.wrow[128 * u + 2 * l + 1] & kWaveOffMask) / 8);
    if (r == 0 && nv[l] != 0.0) ok = false;
    if (r >= kWavePadRows && ++hits[r] > 1) ok = false;
    Xp[r] = nv[l];
    if (r >= kWavePadRows) pend[r] = 0;
  }
  if (Xp[0] != 0.0) ok = false;
}

// Emulates the kernel on the packed (per-lane slot) form: every lane sums its
// slots, lane groups combine, the group's row is written.  Wave steps run
// waves in reverse order; reads of rows not yet final clear `ok`.
static void emulate_packed(const Packed &pk, std::vector<double> &X, std::vector<char> pending, bool &ok) {
  auto unit = [&](int u, bool block, std::vector<double> &r) {
    const int *U = &pk.units[8 * u];
    const int slot_base = U[0], info_base = U[1], rows = U[2], groups = U[3], lg = U[4], E = U[5],
              lanes = U[6];
    const bool assign = false;
    const int w = 1 << lg;
    r.assign(rows, 0.0);
    std::vector<double> part(rows, 0.0);
    const int passes = rows ? (rows + groups - 1) / groups : 0;
    for (int p = 0; p < passes; ++p)
      for (int lane = 0; lane < lanes; ++lane) {
        const int row = p * groups + lane / w;
        if (row >= rows) continue;
        for (int e = 0; e < E; ++e) {
          // a lane's columns in quads and its values in pairs, pass by pass
          const size_t base = (size_t)slot_base + (size_t)p * E * lanes;
          const size_t ac = base + (size_t)(e / 4) * 4 * lanes + 4 * (size_t)lane + e % 4;
          const size_t av = base + (size_t)(e / 2) * 2 * lanes + 2 * (size_t)lane + e % 2;
          if (pk.sval[av] != 0.0 && pending[pk.scol[ac]]) ok = false;
          part[row] += pk.sval[av] * X[pk.scol[ac]];
        }
      }
    for (int a = 0; a < rows; ++a) {
      const int i = pk.irow[info_base + a];
      double v = assign ? part[a] : X[i] - part[a];
      if (block) {
        r[a] = v;
      } else {
        if (!pk.idinv.empty()) v *= pk.idinv[info_base + a];
        X[i] = v;
        pending[i] = 0;
      }
    }
  };
  std::vector<double> r;
  // the padded vector of the wave units: zero row, dummy rows, then X
  const size_t n = X.size();
  std::vector<double> Xp(n + kWavePadRows, 0.0);
  std::vector<char> pp(n + kWavePadRows, 0);
  for (size_t st = 0; st < pk.steps.size() / 4; ++st) {
    const int a = pk.steps[4 * st], kind = pk.steps[4 * st + 2], off = pk.steps[4 * st + 3];
    if (kind == 2) {
      for (size_t i = 0; i < n; ++i) {
        Xp[i + kWavePadRows] = X[i];
        pp[i + kWavePadRows] = pending[i];
      }
      const int nw = 16;
      for (int w = nw - 1; w >= 0; --w)
        for (int u = pk.wdir[a + w]; u < pk.wdir[a + w + 1]; ++u) {
          bool act[64], two[64];
          for (int l = 0; l < 64; ++l) {
            const uint32_t f = u - kWaveAhead >= pk.wdir[a + w] ? (uint32_t)pk.wrow[128 * (u - kWaveAhead) + 2 * l] : ~0u;
            act[l] = (f >> kWaveActBit) & 1u;
            two[l] = (f >> kWaveTwoBit) & 1u;
          }
          wave_unit(pk, u, act, two, Xp, pp, ok);
        }
      for (size_t i = 0; i < n; ++i) {
        X[i] = Xp[i + kWavePadRows];
        pending[i] = pp[i + kWavePadRows];
      }
    } else if (kind == 0) {
      unit(a, false, r);
    } else {
      unit(a, true, r);
      const int *U = &pk.units[8 * a];
      const int rows = U[2], info_base = U[1];
      for (int x = 0; x < rows; ++x) {
        double acc = 0;
        for (int c = 0; c <= x; ++c) acc += pk.dense[off + (size_t)x * rows + c] * r[c];
        X[pk.irow[info_base + x]] = acc;
        pending[pk.irow[info_base + x]] = 0;
      }
    }
  }
  for (char c : pending)
    if (c) ok = false;
}

static void plain(const Sweep &s, std::vector<double> &X) {
  for (size_t p = 0; p < s.rows.size(); ++p) {
    double v = X[s.rows[p]];
    for (int q = s.ptr[p]; q < s.ptr[p + 1]; ++q) v -= s.val[q] * X[s.col[q]];
    if (!s.dinv.empty()) v *= s.dinv[p];
    X[s.rows[p]] = v;
  }
}

static double relerr(const std::vector<double> &a, const std::vector<double> &b) {
  double e = 0, m = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    e = std::max(e, std::fabs(a[i] - b[i]));
    m = std::max(m, std::fabs(b[i]));
  }
  return e / m;
}

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  auto hdr = rd<int32_t>(f, 3);
  const int n = hdr[0], m = hdr[1], g = hdr[2];
  auto bf = rd<int32_t>(f, m), bt = rd<int32_t>(f, m);
  auto r = rd<double>(f, m), x = rd<double>(f, m), b = rd<double>(f, m);
  auto ty = rd<int32_t>(f, n);
  auto pd = rd<double>(f, n), qd = rd<double>(f, n);
  auto gb = rd<int32_t>(f, g);
  auto pg = rd<double>(f, g), vg = rd<double>(f, g), c2 = rd<double>(f, g), c1 = rd<double>(f, g),
       c0 = rd<double>(f, g);
  auto v0 = rd<double>(f, n);
  fclose(f);
  rh_network_desc d{n, m, g, bf.data(), bt.data(), r.data(), x.data(), b.data(), ty.data(), pd.data(),
                    qd.data(), gb.data(), pg.data(), vg.data(), c2.data(), c1.data(), c0.data()};
  Context ctx;
  Network net;
  net.ctx = &ctx;
  std::string err;
  if (network_build(net, d, err) != RH_OK) {
    printf("build error %s\n", err.c_str());
    return 1;
  }
  if (v0.size() == (size_t)n) {
    net.x0.assign(net.n_x, 0.0);
    for (int bb = 0; bb < n; ++bb)
      if (net.v_x[bb] >= 0) net.x0[net.v_x[bb]] = v0[bb];
  }
  if (network_solve(net, 1e-13, 30, err) != RH_OK) {
    printf("solve error %s\n", err.c_str());
    return 1;
  }
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  const int nx = net.n_x;
  if (nx <= 400) {  // dense Gaussian elimination with partial pivoting
    std::vector<double> A((size_t)nx * nx, 0.0);
    for (int i = 0; i < nx; ++i)
      for (int e = net.gx.ptr[i]; e < net.gx.ptr[i + 1]; ++e) A[(size_t)i * nx + net.gx.col[e]] = net.gx.val[e];
    for (int trans = 0; trans < 2; ++trans) {
      std::vector<double> M(A), rhs(nx), sol;
      if (trans)
        for (int i = 0; i < nx; ++i)
          for (int j = 0; j < nx; ++j) M[(size_t)i * nx + j] = A[(size_t)j * nx + i];
      for (auto &v : rhs) v = nd(rng);
      sol = rhs;
      if (trans)
        lu_solve_t(net.lu, sol);
      else
        lu_solve(net.lu, sol);
      std::vector<double> bvec(rhs);
      for (int k = 0; k < nx; ++k) {
        int p = k;
        for (int i = k + 1; i < nx; ++i)
          if (std::fabs(M[(size_t)i * nx + k]) > std::fabs(M[(size_t)p * nx + k])) p = i;
        for (int j = 0; j < nx; ++j) std::swap(M[(size_t)k * nx + j], M[(size_t)p * nx + j]);
        std::swap(bvec[k], bvec[p]);
        for (int i = k + 1; i < nx; ++i) {
          const double l = M[(size_t)i * nx + k] / M[(size_t)k * nx + k];
          for (int j = k; j < nx; ++j) M[(size_t)i * nx + j] -= l * M[(size_t)k * nx + j];
          bvec[i] -= l * bvec[k];
        }
      }
      std::vector<double> xs(nx);
      for (int i = nx - 1; i >= 0; --i) {
        double s = bvec[i];
        for (int j = i + 1; j < nx; ++j) s -= M[(size_t)i * nx + j] * xs[j];
        xs[i] = s / M[(size_t)i * nx + i];
      }
      printf("max_err lu_solve%s %.3e\n", trans ? "_t" : "", relerr(sol, xs));
    }
  }
  Sweep sw[4];
  std::vector<double> pivinv;
  lu_sweeps(net.lu, sw[0], sw[1], sw[2], sw[3], pivinv);
  const char *nm[4] = {"L", "U", "Ut", "Lt"};
  const bool fwd[4] = {true, false, true, false};
  const std::vector<int32_t> parent = etree_parent(net.lu);
  int bad = 0;
  {
    // the sweeps built again into the same objects and work arrays
    Sweep rs[4];
    std::vector<double> rp;
    LuSweepsWork lw;
    for (int rep = 0; rep < 2; ++rep) lu_sweeps(net.lu, rs[0], rs[1], rs[2], rs[3], rp, &lw);
    bool same = rp == pivinv;
    for (int k = 0; k < 4; ++k)
      same = same && rs[k].lev_ptr == sw[k].lev_ptr && rs[k].rows == sw[k].rows && rs[k].ptr == sw[k].ptr &&
             rs[k].col == sw[k].col && rs[k].val == sw[k].val && rs[k].dinv == sw[k].dinv;
    if (!same) {
      printf("sweeps_reuse_mismatch\n");
      ++bad;
    }
  }
  Packed reused;  // packed again in place after every other schedule
  for (int k = 0; k < 4; ++k)
    for (int wave : {0, 1})
      for (int bmax : {0, 16, 64}) {
        ScheduleParams prm;
        prm.bmax = bmax;
        prm.wave_mode = wave;
        const Schedule sc = build_schedule(sw[k], nx, parent, fwd[k], prm);
        std::vector<double> X(nx);
        for (auto &v : X) v = nd(rng);
        std::vector<double> Y = X;
        bool ok = true;
        emulate(sc, X, ok);
        plain(sw[k], Y);
        if (!ok) ++bad;
        int waves = 0;
        for (size_t q = 0; q < sc.meta.size() / 4; ++q) waves += sc.meta[4 * q + 3] <= -2;
        // the packed form the kernel reads
        {
          const Packed pk = pack_schedule(sc, 1024);
          pack_schedule(sc, 1024, reused);
          if (reused.steps != pk.steps || reused.units != pk.units || reused.wdir != pk.wdir ||
              reused.scol != pk.scol || reused.irow != pk.irow || reused.sval != pk.sval ||
              reused.idinv != pk.idinv || reused.dense != pk.dense || reused.wlg != pk.wlg ||
              reused.wcol != pk.wcol || reused.wrow != pk.wrow || reused.wval != pk.wval) {
            printf("pack_reuse_mismatch %s_w%d_b%d\n", nm[k], wave, bmax);
            ++bad;
          }
          std::vector<double> Xp = Y;
          for (size_t p = 0; p < Xp.size(); ++p) Xp[p] = 0;
          std::vector<double> X0(nx);
          std::mt19937_64 r2(99 + k);
          for (auto &v : X0) v = nd(r2);
          std::vector<double> Xa = X0, Xb = X0;
          std::vector<char> pend(nx, 0);
          for (int32_t rr : sw[k].rows) pend[rr] = 1;
          bool okp = true;
          emulate_packed(pk, Xa, pend, okp);
          if (!check_wave_walk(pk, nx)) {
            printf("wave_walk_mismatch %s_w%d_b%d\n", nm[k], wave, bmax);
            okp = false;
          }
          if (!check_records(pk)) {
            printf("record_mismatch %s_w%d_b%d\n", nm[k], wave, bmax);
            okp = false;
          }
          plain(sw[k], Xb);
          if (!okp) ++bad;
          printf("max_err packed_%s_w%d_b%d %.3e order_ok %d slots %zu\n", nm[k], wave, bmax,
                 relerr(Xa, Xb), okp ? 1 : 0, pk.scol.size());
        }
        printf("max_err sweep_%s_w%d_b%d %.3e steps %zu wave_steps %d order_ok %d\n", nm[k], wave, bmax,
               relerr(X, Y), sc.meta.size() / 4, waves, ok ? 1 : 0);
      }
  printf("order_violations %d\n", bad);
  // the device refactorisation's maps, replayed on the host in the kernels'
  // order (levels of the rows below the dense block, each row in a buffer:
  // scatter G_x, eliminate with the L part's rows in ascending order at the
  // mapped positions; then the block rows' steps with rows below it into the
  // dense block; then its dense right-looking LU, written back through the
  // block's position map), against the host factorisation of the same G_x
  {
    LuMaps mp;
    std::string e2;
    if (!lu_device_maps(net.lu, net.gx, mp, e2)) {
      printf("maps error %s\n", e2.c_str());
      return 1;
    }
    const LuPlan &lu = net.lu;
    std::vector<double> LU(mp.row_ptr[nx], std::nan("")), W(mp.maxpat);
    std::vector<char> done(nx, 0);
    int level_bad = 0;
    // row i into W with its first ns steps
    auto eliminate = [&](int32_t i, int32_t ns) {
      const int32_t base = mp.row_ptr[i], len = mp.row_ptr[i + 1] - base;
      std::fill(W.begin(), W.begin() + len, 0.0);
      for (int32_t t = mp.a_ptr[i]; t < mp.a_ptr[i + 1]; ++t) W[mp.a_dst[t]] = net.gx.val[mp.a_src[t]];
      int64_t u = mp.upd_ptr[i];
      for (int32_t q = 0; q < ns; ++q) {
        const int32_t k = mp.lucol[base + q];
        if (!done[k]) ++level_bad;  // row k must be final (an earlier level)
        const int32_t kb = mp.row_ptr[k] + mp.nl[k], ul = mp.row_ptr[k + 1] - kb;
        const double l = W[q] / LU[kb];
        W[q] = l;
        for (int32_t s2 = 1; s2 < ul; ++s2) W[mp.tgt[u + s2 - 1]] -= l * LU[kb + s2];
        u += ul - 1;
      }
      if (ns == mp.nl[i] && u != mp.upd_ptr[i + 1]) ++level_bad;
    };
    const int32_t b0 = mp.b0, mb = nx - b0;
    if (mb < 1 || mb > kNtDenseTop || (int32_t)mp.ns.size() != mb) ++level_bad;
    int32_t nf = 0;
    for (size_t lev = 0; lev + 1 < mp.lev_ptr_f.size(); ++lev) {
      if (mp.lev_ptr_f[lev + 1] == mp.lev_ptr_f[lev]) ++level_bad;  // empty levels are dropped
      for (int32_t idx = mp.lev_ptr_f[lev]; idx < mp.lev_ptr_f[lev + 1]; ++idx) {
        const int32_t i = mp.lev_rows_f[idx], base = mp.row_ptr[i], len = mp.row_ptr[i + 1] - base;
        if (i >= b0 || done[i]) ++level_bad;
        eliminate(i, mp.nl[i]);
        for (int32_t t = 0; t < len; ++t) LU[base + t] = W[t];
        ++nf;
      }
      for (int32_t idx = mp.lev_ptr_f[lev]; idx < mp.lev_ptr_f[lev + 1]; ++idx) done[mp.lev_rows_f[idx]] = 1;
    }
    if (nf != b0) ++level_bad;  // every row below the block exactly once
    // the block rows: steps with rows below b0, the rest into S
    std::vector<double> S((size_t)mb * mb, 0.0);
    for (int32_t r = 0; r < mb; ++r) {
      const int32_t i = b0 + r, base = mp.row_ptr[i], len = mp.row_ptr[i + 1] - base, ns = mp.ns[r];
      eliminate(i, ns);
      for (int32_t t = 0; t < ns; ++t) LU[base + t] = W[t];
      int32_t mapped = 0;
      for (int32_t c = 0; c < mb; ++c) {
        const int32_t q = mp.dmap[(size_t)r * mb + c];
        if (q < 0) continue;
        if (q < ns || q >= len || mp.lucol[base + q] != b0 + c) ++level_bad;
        S[(size_t)r * mb + c] = W[q];
        ++mapped;
      }
      if (mapped != len - ns) ++level_bad;  // the map covers the rest of the row
      for (int32_t q = ns; q < mp.nl[i]; ++q)
        if (mp.lucol[base + q] < b0) ++level_bad;
    }
    // the dense block, right-looking, then written back
    for (int32_t c = 0; c < mb; ++c)
      for (int32_t r = c + 1; r < mb; ++r) {
        const double l = S[(size_t)r * mb + c] / S[(size_t)c * mb + c];
        for (int32_t j = c + 1; j < mb; ++j) S[(size_t)r * mb + j] -= l * S[(size_t)c * mb + j];
      }
    for (int32_t r = 0; r < mb; ++r)
      for (int32_t c = 0; c < mb; ++c) {
        const int32_t q = mp.dmap[(size_t)r * mb + c];
        const double v = S[(size_t)r * mb + c];
        if (q < 0) {
          if (v != 0.0) ++level_bad;  // no fill outside the pattern
          continue;
        }
        LU[mp.row_ptr[b0 + r] + q] = c < r ? v / S[(size_t)c * mb + c] : v;
      }
    double e = 0.0, mx = 0.0;
    for (int32_t i = 0; i < nx; ++i) {
      const int32_t base = mp.row_ptr[i];
      for (size_t q = 0; q < lu.lval[i].size(); ++q) {
        e = std::max(e, std::fabs(LU[base + q] - lu.lval[i][q]));
        mx = std::max(mx, std::fabs(lu.lval[i][q]));
      }
      for (size_t q = 0; q < lu.uval[i].size(); ++q) {
        e = std::max(e, std::fabs(LU[base + mp.nl[i] + q] - lu.uval[i][q]));
        mx = std::max(mx, std::fabs(lu.uval[i][q]));
      }
    }
    printf("max_err device_refactor %.3e\n", e / mx);
    // the Newton step's solve in the kernels' order with these factors: the
    // L sweep over the rows below the block by levels, the block rows'
    // entries with earlier rows, the block forward; the block backward, then
    // the U sweep over the rows below it by levels; against the host solve
    {
      std::vector<double> rhs(nx), y(nx), ref(nx);
      for (auto &v : rhs) v = nd(rng);
      for (int32_t i = 0; i < nx; ++i) y[i] = rhs[lu.perm[i]];
      std::vector<char> fin(nx, 0);
      for (size_t lev = 0; lev + 1 < mp.lev_ptr_f.size(); ++lev) {
        for (int32_t idx = mp.lev_ptr_f[lev]; idx < mp.lev_ptr_f[lev + 1]; ++idx) {
          const int32_t i = mp.lev_rows_f[idx], base = mp.row_ptr[i];
          double acc = 0.0;
          for (int32_t q = 0; q < mp.nl[i]; ++q) {
            if (!fin[mp.lucol[base + q]]) ++level_bad;
            acc += LU[base + q] * y[mp.lucol[base + q]];
          }
          y[i] -= acc;
        }
        for (int32_t idx = mp.lev_ptr_f[lev]; idx < mp.lev_ptr_f[lev + 1]; ++idx) fin[mp.lev_rows_f[idx]] = 1;
      }
      for (int32_t r = 0; r < mb; ++r) {
        const int32_t i = b0 + r, base = mp.row_ptr[i];
        for (int32_t q = 0; q < mp.ns[r]; ++q) {
          if (!fin[mp.lucol[base + q]]) ++level_bad;
          y[i] -= LU[base + q] * y[mp.lucol[base + q]];
        }
      }
      for (int32_t c = 0; c < mb; ++c)
        for (int32_t r = c + 1; r < mb; ++r) y[b0 + r] -= S[(size_t)r * mb + c] / S[(size_t)c * mb + c] * y[b0 + c];
      for (int32_t c = mb - 1; c >= 0; --c) {
        y[b0 + c] /= S[(size_t)c * mb + c];
        for (int32_t r = 0; r < c; ++r) y[b0 + r] -= S[(size_t)r * mb + c] * y[b0 + c];
      }
      std::fill(fin.begin(), fin.end(), 0);
      for (int32_t i = b0; i < nx; ++i) fin[i] = 1;
      int32_t nuf = 0;
      for (size_t lev = 0; lev + 1 < mp.lev_ptr_uf.size(); ++lev) {
        for (int32_t idx = mp.lev_ptr_uf[lev]; idx < mp.lev_ptr_uf[lev + 1]; ++idx) {
          const int32_t i = mp.lev_rows_uf[idx], ub = mp.row_ptr[i] + mp.nl[i], ue = mp.row_ptr[i + 1];
          if (i >= b0) ++level_bad;
          double acc = 0.0;
          for (int32_t q = ub + 1; q < ue; ++q) {
            if (!fin[mp.lucol[q]]) ++level_bad;
            acc += LU[q] * y[mp.lucol[q]];
          }
          y[i] = (y[i] - acc) / LU[ub];
          ++nuf;
        }
        for (int32_t idx = mp.lev_ptr_uf[lev]; idx < mp.lev_ptr_uf[lev + 1]; ++idx) fin[mp.lev_rows_uf[idx]] = 1;
      }
      if (nuf != b0) ++level_bad;
      std::vector<double> sol(nx);
      for (int32_t i = 0; i < nx; ++i) sol[lu.perm[i]] = y[i];
      ref = rhs;
      lu_solve(net.lu, ref);
      printf("max_err device_solve %.3e\n", relerr(sol, ref));
    }
    printf("refactor_level_violations %d\n", level_bad);
  }
  // the four sweeps compose to the two solves: U^-1 L^-1 (P b) and L^-T U^-T (P b)
  {
    std::vector<double> bb(nx);
    for (auto &v : bb) v = nd(rng);
    std::vector<double> ref = bb, X(nx);
    lu_solve(net.lu, ref);
    for (int i = 0; i < nx; ++i) X[net.lu.iperm[i]] = bb[i];
    ScheduleParams prm;
    bool ok = true;
    emulate(build_schedule(sw[0], nx, parent, true, prm), X, ok);
    for (int i = 0; i < nx; ++i) X[i] *= pivinv[i];
    emulate(build_schedule(sw[1], nx, parent, false, prm), X, ok);
    std::vector<double> sol(nx);
    for (int i = 0; i < nx; ++i) sol[i] = X[net.lu.iperm[i]];
    printf("max_err solve_via_sweeps %.3e\n", relerr(sol, ref));
    ref = bb;
    lu_solve_t(net.lu, ref);
    for (int i = 0; i < nx; ++i) X[net.lu.iperm[i]] = bb[i];
    emulate(build_schedule(sw[2], nx, parent, true, prm), X, ok);
    for (int i = 0; i < nx; ++i) X[i] *= pivinv[i];
    emulate(build_schedule(sw[3], nx, parent, false, prm), X, ok);
    if (!ok) printf("order_violations_composed 1\n");
    for (int i = 0; i < nx; ++i) sol[i] = X[net.lu.iperm[i]];
    printf("max_err solve_t_via_sweeps %.3e\n", relerr(sol, ref));
  }
  return 0;
}
