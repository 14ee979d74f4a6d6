// Launch-shape tuner of librh (rh_autotune): times the candidate shapes of a
// network's products on the device and keeps the fastest, with a cache file
// so that a grid is measured once per device and precision.
//
// A shape is the full Hessian's launch size k (Sec. 5.3 evaluates the
// Hessian in blocks of directions), the directions each workgroup owns, and
// the two parameters of the triangular-sweep schedule.  The schedule depends
// only on the sparsity pattern of the LU factors, which the grid topology
// fixes (the ordering is computed from the pattern and the pivots are
// static), so the cache key is a hash of the topology, not of the operating
// point.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "rh_internal.h"

namespace rh {

namespace {

// Bump when the planner or the kernels change in a way that invalidates
// cached shapes.
constexpr const char *kCacheVersion = "v1";

uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
  const unsigned char *c = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

template <class T>
uint64_t hash_vec(uint64_t h, const std::vector<T> &v) {
  const uint64_t n = v.size();
  h = fnv1a(h, &n, sizeof n);
  return v.empty() ? h : fnv1a(h, v.data(), v.size() * sizeof(T));
}

uint64_t topology_hash(const Network &net) {
  uint64_t h = 1469598103934665603ull;
  const int32_t dims[3] = {net.n_bus, net.n_br, net.n_gen};
  h = fnv1a(h, dims, sizeof dims);
  h = hash_vec(h, net.br_f);
  h = hash_vec(h, net.br_t);
  h = hash_vec(h, net.bus_type);
  h = hash_vec(h, net.gen_bus);
  return h;
}

std::string cache_path() {
  if (const char *p = std::getenv("RH_TUNE_CACHE")) return p;
  const char *home = std::getenv("HOME");
  if (!home || !*home) return "";
  return std::string(home) + "/.cache/librh/tiles.txt";
}

std::string cache_key(const Network &net, rh_precision prec) {
  char hx[17];
  std::snprintf(hx, sizeof hx, "%016llx", (unsigned long long)topology_hash(net));
  return std::string(kCacheVersion) + " " + hx + " " + device_key(net.ctx->device) + " " +
         (prec == RH_FP32_REFINED ? "refined" : "fp64");
}

// Networks tuned on several threads read and append the cache one at a time.
std::mutex g_cache_mu;

// The last line of the cache with this key, if any.
bool cache_read(const std::string &key, rh_tile &t) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  const std::string path = cache_path();
  if (path.empty()) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() || line[key.size()] != ' ') continue;
    std::istringstream is(line.substr(key.size()));
    rh_tile r{};
    if (is >> r.k >> r.dirs_per_group >> r.block_rows >> r.wave_steps >> r.ms_per_hessian && r.k > 0 &&
        (r.dirs_per_group == 1 || r.dirs_per_group == 2 || r.dirs_per_group == 4) && r.block_rows >= 0 &&
        r.block_rows <= 64 && (r.wave_steps == 0 || r.wave_steps == 1)) {
      t = r;
      found = true;
    }
  }
  return found;
}

void cache_write(const std::string &key, const rh_tile &t) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  const std::string path = cache_path();
  if (path.empty()) return;
  // create the directories on the way (best effort: a failure only skips the cache)
  for (size_t i = path.find('/', 1); i != std::string::npos; i = path.find('/', i + 1))
    (void)mkdir(path.substr(0, i).c_str(), 0755);
  std::ofstream f(path, std::ios::app);
  if (!f) return;
  f << key << ' ' << t.k << ' ' << t.dirs_per_group << ' ' << t.block_rows << ' ' << t.wave_steps << ' '
    << t.ms_per_hessian << '\n';
}

}  // namespace

rh_status autotune(Network &net, rh_precision prec, int32_t flags, rh_tile &out, std::string &err) {
  const int pi = prec == RH_FP32_REFINED ? 1 : 0;
  const std::string key = cache_key(net, prec);
  rh_tile best{};
  const bool use_cache = !(flags & RH_TUNE_NO_CACHE);
  if (use_cache && !(flags & RH_TUNE_MEASURE) && cache_read(key, best)) {
    best.source = 2;
  } else {
    const int32_t n_p = net.n_p;
    std::vector<int32_t> ks;
    for (int32_t k : {128, 256, 512, 1024})
      if (k < n_p) ks.push_back(k);
    if (n_p <= 1024) ks.push_back(n_p);
    const int32_t kmax = *std::max_element(ks.begin(), ks.end());
    void *dH = nullptr;
    rh_status s = device_alloc(&dH, sizeof(double) * (size_t)n_p * kmax, err);
    if (s != RH_OK) return s;
    double *H = static_cast<double *>(dH);
    const std::pair<int32_t, int32_t> scheds[4] = {{64, 1}, {32, 1}, {16, 1}, {64, 0}};
    double best_ms = 0.0;
    for (const auto &sc : scheds) {
      net.sched_bmax = sc.first;
      net.sched_wave = sc.second;
      if ((s = device_upload(net, err)) != RH_OK) break;
      for (int32_t c = 1; c <= device_max_c(net, prec) && s == RH_OK; c *= 2)
        for (int32_t k : ks) {
          net.tile[pi] = rh_tile{k, c, sc.first, sc.second, 0.0, 1};
          double t_min = 0.0;
          for (int rep = 0; rep < 3 && s == RH_OK; ++rep) {
            const auto t0 = std::chrono::steady_clock::now();
            s = device_hvp(net, k, nullptr, 0, H, n_p, 0, prec, nullptr, err);
            if (s == RH_OK) s = device_sync(nullptr, err);
            const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (rep == 1 || (rep > 1 && t < t_min)) t_min = t;  // the first run is untimed
          }
          if (s != RH_OK) break;
          const double ms = t_min * ((n_p + k - 1) / k);
          if (best.k == 0 || ms < best_ms) {
            best = rh_tile{k, c, sc.first, sc.second, ms, 1};
            best_ms = ms;
          }
        }
      if (s != RH_OK) break;
    }
    device_release(dH);
    if (s != RH_OK) {
      net.tile[pi] = rh_tile{};
      net.sched_bmax = net.sched_wave = -1;
      std::string e2;
      (void)device_upload(net, e2);
      return s;
    }
    if (use_cache) cache_write(key, best);
  }
  // apply: the schedule (re-uploaded when it differs from the current one)
  // and the launch shape
  if (net.sched_bmax != best.block_rows || net.sched_wave != best.wave_steps) {
    net.sched_bmax = best.block_rows;
    net.sched_wave = best.wave_steps;
    rh_status s = device_upload(net, err);
    if (s != RH_OK) return s;
  }
  net.tile[pi] = best;
  // the other precision's shape assumed the schedule it was chosen with
  rh_tile &other = net.tile[1 - pi];
  if (other.k > 0 && (other.block_rows != best.block_rows || other.wave_steps != best.wave_steps)) other = rh_tile{};
  out = best;
  return RH_OK;
}

}  // namespace rh
