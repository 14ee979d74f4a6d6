// Internal structures of librh (host planner + device path).
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/rh.h"

namespace rh {

enum BusType : int32_t { kPQ = 1, kPV = 2, kRef = 3 };

// Row-compressed sparse matrix (ascending columns within each row).
struct Csr {
  int32_t n_rows = 0, n_cols = 0;
  std::vector<int32_t> ptr, col;
  std::vector<double> val;
  int64_t nnz() const { return static_cast<int64_t>(col.size()); }
};

// One triangular sweep, rows grouped by dependency level.  Entry `pos` of the
// level-ordered arrays is matrix row rows[pos]; its off-diagonal entries are
// col/val[ptr[pos] .. ptr[pos+1]); dinv[pos] is the reciprocal pivot (empty for
// unit-diagonal factors).
struct Sweep {
  std::vector<int32_t> lev_ptr, rows, ptr, col;
  std::vector<double> val, dinv;
  int32_t n_levels() const { return static_cast<int32_t>(lev_ptr.size()) - 1; }
};

// Fixed-pattern LU of a structurally symmetric matrix, P A P^T = L U, with a
// fill-reducing symmetric ordering and diagonal pivots.
struct LuPlan {
  int32_t n = 0;
  std::vector<int32_t> perm;   // perm[k] = original index eliminated k-th
  std::vector<int32_t> iperm;  // iperm[perm[k]] = k
  // Patterns in permuted numbering, ascending.
  std::vector<std::vector<int32_t>> lrow;  // strictly lower part of row i
  std::vector<std::vector<int32_t>> urow;  // upper part of row i, diagonal first
  // Values, aligned with the patterns.
  std::vector<std::vector<double>> lval, uval;
  int64_t nnz_l = 0, nnz_u = 0;
  std::vector<int32_t> level_l, level_u;
  int32_t n_levels_l = 0, n_levels_u = 0;
};

// Device sweep schedule: the sweep's rows in step order, with the entries of
// merged blocks split off into dense block inverses; per step
// {first position, rows, log2 lanes per row, kind}, kind = dense offset of a
// block, -1 for a plain level, or -2 - d for a wave step whose waves' level
// lists are wlev[wdir[d + w] .. wdir[d + w + 1]) (4 ints per wave unit:
// first position, rows, log2 lanes per row, assign).  A wave unit is one wave
// level, or one half of a wave block (see kWaveBlockRows): its residual unit
// (assign 0, entries to rows outside the block) followed by the assigning
// unit (assign 1) whose entries are the rows of the block's inverse.
struct Schedule {
  Sweep s;  // rows, ptr, col, val, dinv (lev_ptr unused)
  std::vector<int32_t> meta;
  std::vector<double> dense;
  std::vector<int32_t> wdir, wlev;
};

// Rows of a wave block: a run of narrow wave levels solved with the inverse of
// its unit lower-triangular block (one lane group of 4 per row, one pass).
constexpr int32_t kWaveBlockRows = 16;

// Device form of a schedule.
//
// Level and block steps: every unit (a level step or the rows of a block)
// stores its entries in per-lane slots: rows are spread over groups of 2^lg
// lanes, `groups` rows per pass, and lane j of a group holds entries j,
// j + 2^lg, ... of its row, `E` slots per lane and pass (E a multiple of 4),
// padded with (column 0, value 0).  A pass occupies slots slot_base + pass *
// E * lanes onwards and keeps a lane's columns in quads and its values in
// pairs: the column of slot (e, lane) sits at + (e >> 2) * 4 lanes + 4 lane +
// (e & 3), its value at + (e >> 1) * 2 lanes + 2 lane + (e & 1), so a lane
// reads four columns, or two values, with one access, and the quads (pairs)
// of a pass's lanes are contiguous.
// units: 8 ints each {slot_base, info_base, rows, groups, lg, E, lanes, -1};
// irow/idinv give each row's matrix row and reciprocal pivot (unit order).
// Slot 0 and dense[0] are a zero padding entry (offsets start at 1) that
// lanes without an entry read.
// steps: 4 ints each {unit or wave directory offset, 0, kind, dense offset},
// kind 0 = level, 1 = block (dense inverse at the offset, rows x rows,
// row-major), 2 = wave step
// (its waves' wave-unit ranges are wdir[off + w] .. wdir[off + w + 1]).
//
// Wave steps: fixed-shape wave units (one wave, one pass, 64 lanes, four
// entry slots per lane), so that a wave walks them with no per-unit decode:
// rows of 2^wlg[u] lanes each; lane j of a row's group holds entries j,
// j + 2^lg, j + 2 * 2^lg, j + 3 * 2^lg.  Every position is a byte offset into
// a padded vector whose first kWavePadRows rows are not the solution's: row 0
// is a zero that is never changed (padding reads it), rows 1 .. 64 take the
// writes of lanes that own no row (lane l writes row 1 + l), and solution row
// i sits at row i + kWavePadRows; offsets are for 8-byte rows (the kernel
// scales them for other row sizes).  Record of unit u, per lane l:
//   wcol[256 u + 4 l + e]  offset of entry e's column (padding: row 0)
//   wrow[128 u + 2 l]      offset of the row the lane's update starts from:
//                          its own row, or row 0 (the second unit of a
//                          wave block, and lanes without a row); bit
//                          kWaveActBit: lane l has entries in the unit
//                          kWaveAhead units later on the same wave (its
//                          column quad and first value pair are loaded),
//                          bit kWaveTwoBit: it has entries 2 or 3 there (its
//                          second value pair is loaded); lanes whose loads
//                          are skipped read zeros (column row 0, value 0)
//   wrow[128 u + 2 l + 1]  offset the lane writes: its row for the first lane
//                          of a group, else its dummy row 1 + l; bits
//                          kWaveLgShift and up hold the unit's lg
//   wval[256 u + 128 (e >> 1) + 2 l + (e & 1)]  entry e's value (negated in the
//                          second unit of a wave block, so that every lane
//                          computes x = X[start] - sum of value * X[column])
// A row of a wave level with more than 256 entries is continued by further
// units right after the level's first (each adds 256 more entries of the
// row to its partial value).
constexpr int kSlotsAhead = 4;
constexpr int32_t kWavePadRows = 65;
constexpr int kWaveLgShift = 29;
constexpr int kWaveActBit = 30, kWaveTwoBit = 31;
constexpr uint32_t kWaveOffMask = (1u << kWaveLgShift) - 1;
// Records a wave has in flight while it walks its units (the distance of
// the load flags above).
constexpr int kWaveAhead = 2;

struct Packed {
  std::vector<int32_t> steps, units, wdir;
  std::vector<int32_t> scol, irow;
  std::vector<double> sval, idinv, dense;
  std::vector<int32_t> wlg, wcol, wrow;
  std::vector<double> wval;
};

// The cut of a sweep into a wave step and the steps above it: the wave that
// owns each row below the cut (-1 above it), or no wave step at all.  It
// depends only on the sweep's pattern and the schedule parameters, so a
// network reuses it for every operating point.
struct ScheduleCut {
  bool valid = false, plain = false;
  std::vector<int32_t> owner;
};
struct ScheduleParams {
  int bmax = 64;          // rows of a merged block (0: no blocks)
  int block_rows = 64;    // the kernel's block capacity
  int lane_budget = 1024;  // rows x lanes of a level step
  int n_waves = 16;       // waves of the kernel's workgroup
  int wave_mode = 1;      // 0: no wave step
};

struct DeviceNet;  // defined by the device translation unit
struct DeviceCtx;  // likewise: a context's resources for batched launches
struct DeviceBatch;  // likewise: a batched launch recorded as a graph
struct DevNewton;    // the device Newton's arrays (newton.hip)
struct DevTrack;     // the tracking update's device workspace (track.hip)

struct Context {
  int32_t device = -1;  // -1: host only
  int32_t timing = 0;  // 0 off, 1 launch events, 2 also in-kernel phase stamps
  int32_t refine = 4;  // refined mode: at most this many corrections after the first FP32 solve
  double refine_tol = 1e-13;  // refined mode: a direction stops once its backward error is <= this
  DeviceCtx *dev = nullptr;
};

// Per-bus-incidence coefficients of the branch-wise Lagrangian Hessian.
struct Tape {
  // incidence list by bus: branches touching bus e, other end o
  std::vector<int32_t> inc_ptr, inc_other;
  std::vector<double> inc_K, inc_Hps, inc_H, inc_A2, inc_vo;
  std::vector<double> bus_v, bus_sth, bus_sv;  // voltage, slack-term coefficients
  std::vector<int32_t> slack_bus;              // buses with a nonzero slack coefficient
  std::vector<double> slack_gth, slack_gv;     // d P_ref / d theta_b, d v_b
  double slack_c2x2 = 0.0;                     // 2 c2 of the reference generator
};

struct Network {
  Context *ctx = nullptr;
  // ---- description (copied)
  int32_t n_bus = 0, n_br = 0, n_gen = 0;
  std::vector<int32_t> br_f, br_t, bus_type, gen_bus;
  std::vector<double> br_r, br_x, br_b, Pd, Qd, Pg, Vg, c2, c1, c0;
  // ---- per-branch series admittance and shunt
  std::vector<double> gs, bs, bsh;  // g_s, b_s, b_c / 2
  // ---- bookkeeping (eq. (powerflowvec), Table 1 counts)
  int32_t ref = -1, n_pv = 0, n_pq = 0, n_x = 0, n_p = 0;
  std::vector<int32_t> pv, pq;           // ascending bus ids
  std::vector<int32_t> gen_of_bus;       // -1 if none
  std::vector<int32_t> th_x, v_x, v_p;   // bus -> x index of theta / v, p index of v (-1 none)
  std::vector<int32_t> pg_p;             // bus -> p index of Pg (-1 none)
  // ---- Jacobian patterns (original numbering) and scatter maps
  Csr gx;                                 // G_x pattern/values, rows = x order
  Csr gp;                                 // G_p, n_x x n_p
  std::vector<int64_t> gx_slot, gp_slot;  // branch-gradient slot -> value position (-1: none)
  bool islanded = false;                  // some bus is not connected to the reference
  // ---- factorisation
  LuPlan lu;
  // ---- state
  std::vector<double> p, x, lam;
  std::vector<double> fp;  // grad_p f at the operating point
  std::vector<double> x0;  // Newton start (empty: flat start)
  bool solved = false;
  int32_t newton_iters = 0;
  double newton_resid = 0.0;
  double objective = 0.0;
  Tape tape;
  rh_report report{};
  DeviceNet *dev = nullptr;
  DevNewton *dnewton = nullptr;  // device Newton arrays (rh_solve_powerflow_device)
  DevTrack *dtrack = nullptr;    // tracking workspace (rh_tracking_step_device)
  uint64_t dev_gen = 0;  // device uploads so far (a recorded launch checks it is unchanged)
  // launch shape per precision (0 FP64, 1 refined) chosen by the tuner
  // (tune.cpp); k == 0: not chosen, the library's defaults apply
  rh_tile tile[2] = {};
  // schedule parameters of the uploaded sweeps (-1: the defaults)
  int32_t sched_bmax = -1, sched_wave = -1;
  // the cuts of the four sweeps (L, U, U^T, L^T) for the parameters
  // cut_params = {bmax, wave mode} (reused across operating points)
  ScheduleCut cuts[4];
  int32_t cut_params[2] = {-1, -1};
  int32_t refined_cols = -1;    // columns of the last refined product call (-1: none)
};

// ---- host planner (network.cpp)
rh_status network_build(Network &net, const rh_network_desc &d, std::string &err);
rh_status network_solve(Network &net, double tol, int32_t max_iter, std::string &err);
// The state x is accepted after `it` Newton steps with residual r: the
// Jacobians at x, the factors of G_x (factored here unless factors_given:
// net.lu already holds them), the first-order adjoint, the objective and the
// branch coefficients.
rh_status network_accept(Network &net, const std::vector<double> &x, int32_t it, double r, bool factors_given,
                         std::string &err);
// Maps of the device refactorisation (P G_x P^T = L U on the fixed pattern):
// row i of the factors occupies row_ptr[i] .. row_ptr[i + 1] - 1, its L part
// (nl[i] entries) then its U part (diagonal first), with column lucol[] of
// every position; the G_x entries a_src[a_ptr[i] ..] of permuted row i go to
// positions a_dst[..] of the row; eliminating with row k (every entry of row
// i's L part in turn) updates the positions tgt[upd_ptr[i] ..] of row i, one
// per entry of row k's U part after its diagonal.  Update targets are
// numbered below 2^31.
struct LuMaps {
  std::vector<int32_t> row_ptr, nl, lucol, a_ptr, a_src;
  std::vector<uint16_t> a_dst, tgt;
  std::vector<int64_t> upd_ptr;
  // per L position of a row (the elimination with row k = its column): the
  // start and length of row k's U part, the first of its update targets,
  // and k
  std::vector<int32_t> step;  // 4 per factor position (only L positions used)
  int32_t maxpat = 0;
  // The refactorisation treats the last n - b0 rows (the top of the
  // elimination tree, nearly dense) as one dense block: rows below b0 are
  // factored level by level (lev_ptr_f, lev_rows_f: the L levels restricted
  // to them, empty levels dropped); a block row first takes its ns steps
  // with pivot rows below b0, then the block is factored densely.  dmap[r m
  // + c] is the position of column b0 + c in row b0 + r, or -1.
  int32_t b0 = 0;
  std::vector<int32_t> lev_ptr_f, lev_rows_f, ns, dmap;
  // the U levels restricted to the rows below b0 (the backward solve takes
  // the block first), empty levels dropped
  std::vector<int32_t> lev_ptr_uf, lev_rows_uf;
};
// Rows in the dense top block of the device refactorisation (at most).
constexpr int32_t kNtDenseTop = 128;
bool lu_device_maps(const LuPlan &lu, const Csr &gx, LuMaps &mp, std::string &err);
// Newton on the device (newton.hip): the state and the factors of G_x at it
// are returned (x in res, the factor values in net.lu).
struct NewtonResult {
  int32_t iters = 0;
  double resid = 0.0;
  std::vector<double> x;
};
rh_status device_newton(Network &net, double tol, int32_t max_iter, NewtonResult &res, std::string &err);
void device_newton_free(Network &net);
// Newton at rounding level: after three steps, a residual below 1e-11 that
// no longer halves is accepted (the tolerance may lie below what the
// arithmetic can reach for a large grid).
inline bool newton_stalled(int32_t it, double r, double r_prev) {
  return it >= 3 && r < 1e-11 && r >= 0.5 * r_prev;
}

// ---- dense FP64 Cholesky (dense.hip) and the tracking update (track.hip)
// A = L L^T in place on the lower triangle (column-major), and L Y = B in
// place for the nrhs columns of B (B may be null); *dinfo = 0, or the first
// failed column + 1.  Enqueued on `stream`.
rh_status dense_cholesky(int32_t n, double *A, int64_t lda, double *B, int64_t ldb, int32_t nrhs, int32_t *dinfo,
                         void *stream, std::string &err);
// L^T X = Y in place for nrhs columns (nothing if *dinfo != 0); work holds
// n * nrhs doubles.
rh_status dense_back_solve(int32_t n, const double *L, int64_t ldl, double *B, int64_t ldb, int32_t nrhs,
                           double *work, const int32_t *dinfo, void *stream, std::string &err);
// F = lower triangle of A with tau added on the diagonal.
rh_status dense_shift_copy(int32_t n, const double *A, int64_t lda, double *F, int64_t ldf, double tau, void *stream,
                           std::string &err);
rh_status dense_diagonal(int32_t n, const double *A, int64_t lda, double *out, void *stream, std::string &err);
rh_status dense_negate(int32_t n, const double *a, double *b, void *stream, std::string &err);
// Factorise and solve, synchronously; failed_col = -1 or the failed column.
rh_status dense_spd_solve(int device, int32_t n, double *A, int64_t lda, double *B, int64_t ldb, int32_t nrhs,
                          void *stream, int32_t &failed_col, std::string &err);
rh_status tracking_step(Network &net, int32_t k_block, double shift, const double *lo, const double *hi,
                        const double *ramp, double *dd, void *stream, rh_tracking_info &out, std::string &err);
void device_track_free(Network &net);
// grad F = grad_p f + G_p^T lambda of the uploaded operating point (device.hip).
rh_status device_reduced_gradient(Network &net, double *dgrad, void *stream, std::string &err);
// The full reduced Hessian into device memory in blocks of k_block
// directions (0: the tuned launch size) (api.cpp).
rh_status reduced_hessian_into(Network &n, double *H, int64_t ldh, int32_t k_block, rh_precision prec,
                               void *hip_stream, std::string &err);
void flows_inject(const Network &net, const std::vector<double> &th, const std::vector<double> &v,
                  std::vector<double> &P, std::vector<double> &Q);
void unpack_state(const Network &net, const std::vector<double> &x, const std::vector<double> &p,
                  std::vector<double> &th, std::vector<double> &v);
void reduced_gradient(const Network &net, std::vector<double> &grad);
// 1-norm condition estimate of G_x from its factors (a lower bound that is
// usually exact or within a small factor).
double condest_1(const Network &net);

// ---- sparse LU (sparse_lu.cpp)
void lu_analyse(LuPlan &lu, const Csr &pattern);
bool lu_factor(LuPlan &lu, const Csr &a, std::string &err);
void lu_solve(const LuPlan &lu, std::vector<double> &b);        // A x = b in place
void lu_solve_t(const LuPlan &lu, std::vector<double> &b);      // A^T x = b in place
// The four unit-diagonal sweeps of the two solves with A = P^T L D Uh P:
// A^{-1} b = P^T Uh^{-1} D^{-1} L^{-1} P b and A^{-T} b = P^T L^{-T} D^{-1}
// Uh^{-T} P b; pivinv = D^{-1} (reciprocal pivots, factor numbering).
// `work` (may be null) holds the transposed rows of Uh and L between calls,
// so that a caller that keeps it (and the four sweeps) reuses their memory.
struct LuSweepsWork {
  std::vector<int32_t> tp, lp, tc, lc, tf, lf;
  std::vector<double> tv, lv;
};
void lu_sweeps(const LuPlan &lu, Sweep &sl, Sweep &su, Sweep &sut, Sweep &slt, std::vector<double> &pivinv,
               LuSweepsWork *work = nullptr);
int lane_log2(int32_t rows, int32_t longest, int lane_budget);
// `cut` (may be null): reused if valid, else filled with the cut chosen.
Schedule build_schedule(const Sweep &in, int32_t n, const std::vector<int32_t> &parent, bool forward,
                        const ScheduleParams &prm, ScheduleCut *cut = nullptr);
std::vector<int32_t> etree_parent(const LuPlan &lu);
// Pack a schedule into per-lane slots; `lanes` = workgroup size, wave steps use
// 64 lanes per wave.  The second form fills `pk` in place, reusing the
// capacity of its arrays.
Packed pack_schedule(const Schedule &sc, int lanes);
void pack_schedule(const Schedule &sc, int lanes, Packed &pk);
// Device records of the wave units, one fixed-size record per unit, read
// by the kernel's wave walk with one 16-byte load per lane for each part.
//  wide (any network), per lane l:
//    [16 l]          the four column offsets (u32, as wcol)
//    [1024 + 8 l]    the start and write words (as wrow)
//    values          FP64: entries 0-1 at [1536 + 16 l], 2-3 at [2560 + 16 l];
//                    FP32: entries 0-3 at [1536 + 16 l]
//  compact (padded vectors of at most 65,536 rows), per lane l:
//    [16 l]          {col 0 | col 1 << 16, col 2 | col 3 << 16,
//                     start | write << 16, act | two << 1 | lg << 2}, all
//                     rows as indices (offset / 8)
//    values          FP64: entries 0-1 at [1024 + 16 l], 2-3 at [2048 + 16 l];
//                    FP32: entries 0-3 at [1024 + 16 l]
// Returns false (and no records) if a compact record cannot hold the rows.
constexpr int kWaveRecWide64 = 3584, kWaveRecWide32 = 2560;
constexpr int kWaveRecCompact64 = 3072, kWaveRecCompact32 = 2048;
bool wave_records(const Packed &pk, bool compact, bool fp64, std::vector<char> &out);

// ---- device path (device.hip)
// Uploads the solved operating point.  `accept` (may be empty) finishes the
// host side of the solve (network_accept); the upload calls it while the
// factors' sweeps are prepared on other threads, and reads the Jacobians,
// adjoint and tape only after it returns.
rh_status device_upload(Network &net, std::string &err,
                        const std::function<rh_status(std::string &)> &accept = nullptr);
void device_free(Network &net);
void device_ctx_free(Context &ctx);
// Fill the report's launch count, summed kernel time and phase times of the
// launches since the previous collection, and start a new window.
rh_status device_collect(Network &net, std::string &err);
rh_status device_ctx_collect(Context &ctx, rh_report &rep, std::string &err);
rh_status device_hvp(Network &net, int32_t k, const double *dW, int64_t ldw, double *dHW,
                     int64_t ldhw, int32_t identity_from, rh_precision prec, void *stream,
                     std::string &err);
rh_status device_hvp_batch(Context &ctx, int32_t n, Network *const *nets, const int32_t *k,
                           const double *const *dW, const int64_t *ldw, double *const *dHW,
                           const int64_t *ldhw, const int32_t *identity_from, rh_precision prec,
                           void *stream, std::string &err);
rh_status device_set(int32_t device, std::string &err);
// Raises the dynamic-LDS bound of `kernel` on the current device to `bytes`
// if it is lower.  The bound belongs to the kernel, not to a network, so it
// only grows: a network that needs less never cuts the bound another one
// (on another thread, say) launches with.
rh_status lds_bound(const void *kernel, size_t bytes, std::string &err);
// Takes the device address of the fixed scratch array of the allocation-free
// entry point on `device` (once per device; that device becomes current).
rh_status device_fixed_scratch_init(int32_t device, std::string &err);
// rh_hvp_device with the fixed scratch: no allocation, no timing, no
// per-column refinement figures.
rh_status device_hvp_noalloc(Network &net, int32_t k, const double *dW, int64_t ldw, double *dHW, int64_t ldhw,
                             rh_precision prec, void *stream, std::string &err);
rh_status device_memcpy_h2d(void *dst, const void *src, size_t bytes, std::string &err);
rh_status device_memcpy_d2h(void *dst, const void *src, size_t bytes, std::string &err);
rh_status device_memcpy_2d(void *dst, size_t dpitch, const void *src, size_t spitch,
                           size_t width, size_t rows, int to_device, std::string &err);
// A batched launch (as device_hvp_batch) recorded once as a HIP graph: the
// work list is uploaded and the launch scratch allocated at creation, then
// every replay is one graph launch.  The batch keeps the networks' upload
// generations and refuses to replay once one has changed.
rh_status device_batch_create(Context &ctx, int32_t n, Network *const *nets, const int32_t *k,
                              const double *const *dW, const int64_t *ldw, double *const *dHW,
                              const int64_t *ldhw, const int32_t *identity_from, rh_precision prec,
                              DeviceBatch **out, std::string &err);
rh_status device_batch_launch(DeviceBatch *b, void *stream, std::string &err);
void device_batch_info(const DeviceBatch *b, int32_t *dirs_per_group, int32_t *workgroups, int32_t *directions);
void device_batch_free(DeviceBatch *b);
// The most directions per workgroup the network's vectors allow (LDS), and
// a name of the device for the tuner's cache.
int32_t device_max_c(const Network &net, rh_precision prec);
std::string device_key(int32_t device);
// ---- launch-shape tuner (tune.cpp): rh_autotune on a solved network
rh_status autotune(Network &net, rh_precision prec, int32_t flags, rh_tile &out, std::string &err);
// Directions one launch needs to give every CU a workgroup at the largest
// number of directions per workgroup that the network's vectors allow.
int32_t device_launch_dirs(const Network &net, rh_precision prec);
// Per-column figures of the last refined product call: 4 doubles per column
// {backward error of Z, corrections of Z, backward error of Psi, corrections of Psi}.
rh_status device_refinement_report(Network &net, int32_t n, std::vector<double> &out, std::string &err);
// Device bytes held by the network (factors, schedules, coefficients,
// descriptors, its launch scratch and report buffers), and the launch
// scratch a direction of a network with n_x states may take.
int64_t device_network_bytes(const Network &net);
int64_t device_scratch_per_direction(int32_t n_x, rh_precision prec);
rh_status device_alloc(void **p, size_t bytes, std::string &err);
void device_release(void *p);
rh_status device_sync(void *stream, std::string &err);

}  // namespace rh

struct rh_context {
  rh::Context c;
};
struct rh_network {
  rh::Network n;
};
