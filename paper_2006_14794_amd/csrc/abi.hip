// C ABI of libsigkernel: argument validation, workspace layout, launches.
// Declarations and contracts: include/sigkernel.h.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "../../include/sigkernel.h"
#include "corrector.h"
#include "internal.h"
#include "tune.h"

namespace {

using sk::Batch;

// Dyadic orders the sweep kernels are compiled for; beyond them the batch is
// refined (split_order) and swept at the highest compiled order.
constexpr int32_t kMaxKernelOrder = 3;
// Workspace of the allocation-free Gram (sigkernel_gram_noalloc).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// Fine rows or columns of one pair: 2^lambda (len - 1) <= 2^20.
constexpr int64_t kMaxFineSide = int64_t(1) << 20;

// A dyadic order lambda > kMaxKernelOrder runs as order k = kMaxKernelOrder on
// the increments split into rep = 2^(lambda - k) equal parts: each coarse cell
// of P_lambda is then rep x rep cells of the refined batch, whose fine cells
// and coefficients G0 2^-2lambda are exactly those of P_lambda (the parts are
// the increment times an exact power of two).
struct Order {
  int32_t k;
  int32_t rep;
};

Order split_order(int32_t lam) {
  if (lam <= kMaxKernelOrder) return Order{lam, 1};
  return Order{kMaxKernelOrder, 1 << (lam - kMaxKernelOrder)};
}

// The batch as the kernels see it after refinement (len - 1 increments become
// rep (len - 1)); the points pointer is unchanged.
sk_paths refined(const sk_paths* p, int32_t rep) {
  sk_paths r = *p;
  if (r.len > 1) r.len = (int32_t)((int64_t)(r.len - 1) * rep + 1);
  return r;
}

// lambda >= 0 and every pair's fine grid within kMaxFineSide on each side.
bool order_ok(int32_t lam, const sk_paths* X, const sk_paths* Y, int32_t max_order) {
  if (lam < 0 || lam > max_order) return false;
  for (const sk_paths* p : {X, Y})
    if (((int64_t)(p->len > 1 ? p->len - 1 : 0) << lam) > kMaxFineSide) return false;
  return true;
}
constexpr int32_t kMaxDyadicOrder = 20;

bool valid_batch(const sk_paths* p) {
  if (!p) return false;
  if (p->n_paths < 0 || p->dim < 1 || p->len < 1) return false;
  return true;
}

Batch to_batch(const sk_paths* p) {
  return Batch{p->points, p->offsets, p->n_paths, p->len, p->dim};
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// rows of the dense increment buffer of a batch (upper bound when ragged),
// plus kStreamPad rows on each side that the streaming sweep may read
size_t inc_rows(const sk_paths* p) {
  return (size_t)p->n_paths * (size_t)(p->len - 1) + 2 * (size_t)sk::kStreamPad;
}

// Workspace of the forward call, in this order: dense increments of X and of
// Y, then (ragged batches only) the per-path plan of X and of Y.
struct ForwardLayout {
  size_t incx, incy, planx_n, planx_start, plany_n, plany_start, total;
};

size_t plan_bytes_n(const sk_paths* p) {
  return p->offsets ? align256((size_t)p->n_paths * sizeof(int32_t)) : 0;
}
size_t plan_bytes_start(const sk_paths* p) {
  return p->offsets ? align256((size_t)p->n_paths * sizeof(int64_t)) : 0;
}

ForwardLayout forward_layout(const sk_paths* X, const sk_paths* Y) {
  const size_t dp = (size_t)sk::padded_dim(X->dim);
  ForwardLayout L{};
  size_t off = 0;
  L.incx = off;
  off += align256(inc_rows(X) * dp * sizeof(float));
  L.incy = off;
  off += align256(inc_rows(Y) * dp * sizeof(float));
  L.planx_n = off;
  off += plan_bytes_n(X);
  L.planx_start = off;
  off += plan_bytes_start(X);
  L.plany_n = off;
  off += plan_bytes_n(Y);
  L.plany_start = off;
  off += plan_bytes_start(Y);
  L.total = off;
  return L;
}

size_t forward_ws(const sk_paths* X, const sk_paths* Y) { return forward_layout(X, Y).total; }

// Pairs streamed through one wave for a Gram with a uniform y batch: the
// tuned value, else enough waves to fill every SIMD about four times, at
// most 64 pairs per run.
int64_t choose_run(int64_t nx, int64_t ny, int32_t tuned) {
  if (tuned > 0) return tuned < ny ? tuned : (ny > 0 ? ny : 1);
  const int64_t target_waves = 256 * 4 * 4;
  int64_t run = (nx * ny) / target_waves;
  if (run < 1) run = 1;
  if (run > 64) run = 64;
  if (run > ny) run = ny;
  return run;
}

// SIMDs of the current device (four per compute unit); 1024 if unknown.
int64_t device_simds() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    return 1024;
  return 4 * (int64_t)cus;
}

// Pairs streamed through one wave of a one-wave forward Gram sweep: the tuned
// value, else the run that minimises the busiest SIMD's time.  A run of k
// pairs over `cols` fine columns each takes about k + 64 / cols pair times
// (the wavefront fills once per run); the busiest SIMD holds
// ceil(waves / SIMDs) waves, and a SIMD with one, two or three waves issues
// at 0.73, 0.93 or 0.97 of its rate with four or more (measured on the
// sweep).  A symmetric Gram counts only its upper triangle's runs (without
// the diagonal when that is zeroed).  At most
// 64 pairs per run; ties go to the shorter run.
int64_t choose_sweep_run(int64_t nx, int64_t ny, int64_t cols, bool sym, int32_t tuned,
                         bool no_diag = false) {
  if (tuned > 0 || ny <= 1 || cols <= 0) return choose_run(nx, ny, tuned);
  const int64_t simds = device_simds();
  const double fill = 64.0 / (double)cols;
  const int64_t cap = ny < 64 ? ny : 64;
  int64_t best = 1;
  double best_cost = 0.0;
  for (int64_t run = 1; run <= cap; ++run) {
    const int64_t rpr = (ny + run - 1) / run;
    const int64_t s = sym && no_diag ? 1 : 0;
    const int64_t waves = sym ? sk::tri_runs(nx - s, rpr, run, s) : nx * rpr;
    const int64_t per_simd = (waves + simds - 1) / simds;
    const double rate = per_simd >= 4 ? 1.0 : per_simd == 3 ? 0.97 : per_simd == 2 ? 0.93 : 0.73;
    const double cost = (double)per_simd * ((double)run + fill) / rate;
    if (run == 1 || cost < best_cost) {
      best = run;
      best_cost = cost;
    }
  }
  return best;
}

// Independent pairs: the forward layout (increments not scaled), the pair
// plan (order, class counts, queue counters) and one band buffer per
// persistent wave slot.
constexpr int64_t kPairSlots = 4096;

// Pipelined bands (pair_band_kernel) for batches whose grids need several
// bands, when every band task's slot buffer fits this budget.
constexpr size_t kPipeCapBytes = size_t(1) << 30;
// SIMDs of the target (256 compute units of 4): the band-height model's
// notion of a full chip (a constant, so that workspace sizes do not depend
// on the device queried)
constexpr int64_t kSimds = 1024;

struct PairLayout {
  int rows_lo, rows_hi;
  int64_t slots, band_stride;  // doubles per slot
  bool pipe;                   // long class as pipelined band tasks
  int64_t tasks_max;           // upper bound of the band tasks
  size_t order, counts, bands, task_base, tbuf, total;
};

PairLayout pair_layout(const sk_paths* X0, const sk_paths* Y0, int32_t lam0, bool gram) {
  const Order o = split_order(lam0);
  const sk_paths Xr = refined(X0, o.rep), Yr = refined(Y0, o.rep);
  const sk_paths* X = &Xr;
  const sk_paths* Y = &Yr;
  const int32_t lam = o.k;
  PairLayout L{};
  const int64_t npairs = gram ? X->n_paths * Y->n_paths : X->n_paths;
  const int d = X->dim;
  // rows of the longest possible pair (its shorter path on the rows)
  const int64_t shorter = (X->len < Y->len ? X->len : Y->len) - 1;
  const int64_t rows = (shorter < 1 ? 1 : shorter) << lam;
  int rmax = 0;
  for (int R = 1; R <= sk::kMaxRowsPerLane; R *= 2)
    if (sk::sweep_fn(sk::kKernelPair, lam, R, d)) rmax = R;
  int rhi = 1;
  while (rhi < rmax && 64 * (int64_t)rhi < rows) rhi *= 2;
  // Few long pairs of equal length: lower bands (fewer rows per lane) keep
  // more SIMDs busy and make each step cheaper, at the price of more
  // hand-overs, each band lagging the one above by about a pipeline fill plus
  // a staging chunk (80 steps).  Modelled time of a pair: (columns + 63 +
  // (bands - 1) 80) steps of cost R + 20, times the waves per SIMD beyond one.
  // The 20 rows stand for the part of a step that does not shrink with R: a
  // wave alone on its SIMD waits on latencies (DPP hand-off, loads, the
  // cells' dependency chain) more than it issues.  Fitted to five pairs of
  // 2000 points at order 4 (8.05, 6.98, 7.60, 10.77 ms at R = 32, 16, 8, 4).
  if (rmax && rhi == rmax && !X0->offsets && !Y0->offsets && rows > 64 * (int64_t)rmax) {
    const int64_t cols = (X->len > Y->len ? X->len : Y->len) - 1;
    auto cost = [&](int R) {
      const int64_t nb = (rows + 64 * (int64_t)R - 1) / (64 * (int64_t)R);
      const double share = (double)(nb * npairs) / kSimds;
      return (double)(cols + 63 + (nb - 1) * 80) * (R + 20) * (share > 1.0 ? share : 1.0);
    };
    // a height whose band tasks' slot buffers exceed the budget would lose
    // the pipeline: not a candidate
    const int64_t stride = (X->len > Y->len ? X->len : Y->len) + 2 * sk::kStreamPad;
    auto fits = [&](int R) {
      const int64_t nb = (rows + 64 * (int64_t)R - 1) / (64 * (int64_t)R);
      return (size_t)(nb * npairs) * (size_t)(stride << lam) * sizeof(double) <= kPipeCapBytes;
    };
    double best = cost(rmax);
    for (int R = rmax / 2; R >= 1; R /= 2) {
      if (!sk::sweep_fn(sk::kKernelPairBandFull, lam, R, d) || !fits(R)) continue;
      const double c = cost(R);
      if (c < best) {
        best = c;
        rhi = R;
      }
    }
  }
  L.rows_hi = rmax ? rhi : 0;
  L.rows_lo = rhi > 1 ? rhi / 2 : rhi;
  // wave slots: a whole number of 4-wave workgroups
  L.slots = npairs < kPairSlots ? npairs : kPairSlots;
  L.slots = ((L.slots < 1 ? 1 : L.slots) + 3) & ~int64_t(3);
  const int64_t longer = (X->len > Y->len ? X->len : Y->len);
  L.band_stride = (longer + 2 * sk::kStreamPad) << lam;
  const int64_t nb_max = L.rows_hi ? (rows + 64 * (int64_t)L.rows_hi - 1) / (64 * L.rows_hi) : 1;
  L.tasks_max = npairs * nb_max;
  L.pipe = L.rows_hi > 0 && nb_max > 1 && npairs <= INT32_MAX &&
           (size_t)L.tasks_max * (size_t)L.band_stride * sizeof(double) <= kPipeCapBytes;
  size_t off = forward_ws(X, Y);
  L.order = off;
  off += align256((size_t)(npairs > 0 ? npairs : 1) * sizeof(int32_t));
  L.counts = off;
  off += 256;  // counts[2], counters[2], the band-task counter
  L.bands = off;
  off += align256((size_t)L.slots * (size_t)L.band_stride * sizeof(double));
  L.task_base = off;
  L.tbuf = off;
  if (L.pipe) {
    off += align256((size_t)(npairs + 1) * sizeof(int32_t));
    L.tbuf = off;
    off += align256((size_t)L.tasks_max * (size_t)L.band_stride * sizeof(double));
  }
  L.total = off;
  return L;
}

// Channels beyond which the fused sweeps are not compiled: wider batches run
// the coefficient sweep (coef.hip) with the increment Gram formed first.
constexpr int32_t kMaxFusedDim = 16;
// Coefficient slots held at once (waves are launched in chunks within it).
constexpr size_t kCoefCapBytes = size_t(1) << 30;

struct CoefPlan {
  int R;
  int32_t lam, rep;
  int32_t run;
  int64_t runs_per_row, n_waves;
  int64_t stride;  // floats per wave
  int64_t chunk;   // waves per producer / sweep launch pair
  size_t coef_off, total;
};

// mode 0: pairs; 1, 2: Gram (2: upper triangle)
CoefPlan coef_plan(const sk_paths* X, const sk_paths* Y, int32_t lam0, int mode) {
  CoefPlan P{};
  const Order o = split_order(lam0);
  const sk_paths Xr = refined(X, o.rep), Yr = refined(Y, o.rep);
  P.lam = o.k;
  P.rep = o.rep;
  const int64_t fine_rows = (int64_t)(Xr.len > 1 ? Xr.len - 1 : 1) << o.k;
  P.R = sk::coef_rows_per_lane(fine_rows, o.k);
  P.coef_off = forward_ws(X, Y);  // unrefined increments and plans
  P.total = P.coef_off;
  if (P.R == 0) return P;
  if (mode == 0) {
    P.run = 1;
    P.runs_per_row = 1;
    P.n_waves = X->n_paths;
  } else {
    P.run = Y->offsets ? 1 : (int32_t)choose_run(X->n_paths, Y->n_paths, 0);
    P.runs_per_row = (Y->n_paths + P.run - 1) / P.run;
    P.n_waves = X->n_paths * P.runs_per_row;
  }
  const int64_t cols = (int64_t)P.run * (Yr.len > 1 ? Yr.len - 1 : 1);
  P.stride = sk::coef_wave_floats(cols, P.R, o.k);
  P.chunk = (int64_t)(kCoefCapBytes / ((size_t)P.stride * sizeof(float)));
  if (P.chunk < 1) P.chunk = 1;
  if (P.chunk > P.n_waves) P.chunk = P.n_waves > 0 ? P.n_waves : 1;
  P.total = P.coef_off + align256((size_t)P.chunk * (size_t)P.stride * sizeof(float));
  return P;
}

// Workspace of a Gram call: the one-wave sweep's layout or, for x paths too
// tall for it, the persistent pair kernel's; the coefficient sweep's for
// batches wider than the fused sweeps.
size_t gram_ws(const sk_paths* X, const sk_paths* Y, int32_t lam) {
  if (X->dim > kMaxFusedDim && X->dim == Y->dim) return coef_plan(X, Y, lam, 1).total;
  const Order o = split_order(lam);
  const sk_paths Xr = refined(X, o.rep), Yr = refined(Y, o.rep);
  const size_t f = forward_ws(&Xr, &Yr);
  if (X->dim != Y->dim) return f;
  const size_t g = pair_layout(X, Y, lam, true).total;
  return f > g ? f : g;
}

// Gram gradient workspace: the forward layout (increments, and the plans of
// ragged batches), the task order of a ragged batch, counters, one scratch
// slot per persistent wave (checkpoints and band hand-overs), and the x-side
// and y-side increment gradients in double.  The persistent waves are a
// constant number (two per SIMD of the target), so that the workspace size
// does not depend on the device queried.
constexpr int64_t kGradSlots = 2048;

struct GradPlan {
  int lam, rep;
  bool ragged;
  int64_t run, runs_per_row, n_tasks, slots;
  int nb_max, nseg_max;
  int64_t cols_max;
  int32_t mrows, nrows;
  int64_t slot_stride;  // doubles
  size_t order, counts, scratch, partx, party, total;
};

// Pairs per gradient task for a uniform y batch: the tuned value, else about
// one task with pairs per persistent wave (kGradSlots; a symmetric Gram's
// tasks below the diagonal are empty), at most 64 pairs per task.  Longer
// tasks pay the wavefront's fill once per run of pairs instead of per pair.
int64_t choose_grad_run(int64_t nx, int64_t ny, bool sym, int32_t tuned) {
  if (tuned > 0) return tuned < ny ? tuned : (ny > 0 ? ny : 1);
  const int64_t pairs = sym ? nx * (nx + 1) / 2 : nx * ny;
  int64_t run = pairs / kGradSlots;
  if (run < 1) run = 1;
  if (run > 64) run = 64;
  if (run > ny) run = ny;
  return run;
}

GradPlan grad_plan(const sk_paths* X0, const sk_paths* Y0, int32_t lam0, uint32_t flags) {
  const Order o = split_order(lam0);
  const sk_paths Xr = refined(X0, o.rep), Yr = refined(Y0, o.rep);
  GradPlan P{};
  P.lam = o.k;
  P.rep = o.rep;
  P.ragged = X0->offsets || Y0->offsets;
  const int64_t m = Xr.len > 1 ? Xr.len - 1 : 0, n = Yr.len > 1 ? Yr.len - 1 : 0;
  const int d = X0->dim;
  P.mrows = (int32_t)m;
  P.nrows = (int32_t)n;
  if (P.ragged) {
    P.run = 1;
    P.runs_per_row = Y0->n_paths;
  } else {
    const sk_tune t = sk::tuning_for(SK_OP_GRAM_BACKWARD, X0, Y0, lam0, flags);
    P.run = choose_grad_run(X0->n_paths, Y0->n_paths, (flags & SK_SYMMETRIC) != 0, t.run);
    P.runs_per_row = (Y0->n_paths + P.run - 1) / P.run;
  }
  P.n_tasks = X0->n_paths * P.runs_per_row;
  P.slots = P.n_tasks < kGradSlots ? P.n_tasks : kGradSlots;
  if (P.slots < 1) P.slots = 1;
  const int64_t M = m << P.lam;
  const int64_t band_rows = 64 * (int64_t)sk::kGradRows;
  P.nb_max = (int)(M > 0 ? (M + band_rows - 1) / band_rows : 1);
  P.cols_max = P.run * (n > 0 ? n : 1);
  const int C = sk::grad_segment(P.lam, d);
  P.nseg_max = (int)((P.cols_max + 63 + C - 1) / C);
  P.slot_stride = sk::grad_slot_layout(P.lam, P.nb_max, P.nseg_max, P.cols_max).stride;
  size_t off = forward_ws(&Xr, &Yr);
  P.order = off;
  if (P.ragged) off += align256((size_t)(P.n_tasks > 0 ? P.n_tasks : 1) * sizeof(int32_t));
  P.counts = off;
  off += 256;  // the pair plan's counts and counters, the gradient queue head
  P.scratch = off;
  off += align256((size_t)P.slots * (size_t)P.slot_stride * sizeof(double));
  P.partx = off;
  off += align256((size_t)X0->n_paths * (size_t)P.runs_per_row * (size_t)m * d * sizeof(double));
  P.party = off;
  off += align256((size_t)X0->n_paths * Y0->n_paths * (size_t)n * d * sizeof(double));
  P.total = off;
  return P;
}

int rounding_of(uint32_t flags) {
  if (flags & SK_GRAM_BF16) return sk::kRoundBf16;
  if (flags & SK_GRAM_F16) return sk::kRoundF16;
  return sk::kRoundNone;
}

sk_status check_flags(uint32_t flags, uint32_t allowed) {
  if ((flags & SK_GRAM_BF16) && (flags & SK_GRAM_F16)) return SK_ERR_FLAGS;
  if (flags & ~allowed) return SK_ERR_FLAGS;
  if ((flags & SK_NO_DIAG) && !(flags & SK_SYMMETRIC)) return SK_ERR_FLAGS;
  return SK_OK;
}

// gram: every (a, b) of the two batches, out[a * ny + b]; else pairs (x_k, y_k)
sk_status run_pairs(const sk_paths* X, const sk_paths* Y, int32_t lam0, float* out, void* ws,
                    size_t ws_bytes, hipStream_t stream, bool gram, int rounding,
                    const sk_tune& tune, bool implicit) {
  const int d = X->dim;
  const int dp = sk::padded_dim(d);
  const PairLayout PL = pair_layout(X, Y, lam0, gram);
  const int64_t npairs = gram ? X->n_paths * Y->n_paths : X->n_paths;
  if (npairs > INT32_MAX) return SK_ERR_UNSUPPORTED;
  if (PL.rows_hi == 0) return SK_ERR_UNSUPPORTED;
  if (ws_bytes < PL.total) return SK_ERR_WORKSPACE;
  const Order o = split_order(lam0);
  const int32_t lam = o.k;
  const sk_paths Xr = refined(X, o.rep), Yr = refined(Y, o.rep);
  const ForwardLayout L = forward_layout(&Xr, &Yr);
  char* base = static_cast<char*>(ws);
  float* incx = reinterpret_cast<float*>(base + L.incx) + sk::kStreamPad * dp;
  float* incy = reinterpret_cast<float*>(base + L.incy) + sk::kStreamPad * dp;
  sk::PathPlan px{reinterpret_cast<int32_t*>(base + L.planx_n),
                  reinterpret_cast<int64_t*>(base + L.planx_start)};
  sk::PathPlan py{reinterpret_cast<int32_t*>(base + L.plany_n),
                  reinterpret_cast<int64_t*>(base + L.plany_start)};
  const sk::Batch bx = to_batch(X), by = to_batch(Y);
  if (X->offsets && sk::launch_plan(bx, px, stream) != hipSuccess) return SK_ERR_HIP;
  if (Y->offsets && sk::launch_plan(by, py, stream) != hipSuccess) return SK_ERR_HIP;
  if (sk::launch_increments_xy(bx, X->offsets ? &px : nullptr, 1.0f, by,
                               Y->offsets ? &py : nullptr, 1.0f, dp, incx, incy, stream, rounding,
                               o.rep) != hipSuccess)
    return SK_ERR_HIP;
  if (X->offsets && sk::launch_scale_plan(px, X->n_paths, o.rep, stream) != hipSuccess)
    return SK_ERR_HIP;
  if (Y->offsets && sk::launch_scale_plan(py, Y->n_paths, o.rep, stream) != hipSuccess)
    return SK_ERR_HIP;
  int32_t* order = reinterpret_cast<int32_t*>(base + PL.order);
  int32_t* counts = reinterpret_cast<int32_t*>(base + PL.counts);
  sk::PairPlanArgs pp{};
  pp.x_n = X->offsets ? px.n : nullptr;
  pp.x_len = Xr.len;
  pp.y_n = Y->offsets ? py.n : nullptr;
  pp.y_len = Yr.len;
  pp.npairs = (int32_t)npairs;
  pp.gram_ny = gram ? Y->n_paths : 0;
  pp.lam = lam;
  // pipelined bands: every pair joins the band-task queue (a short pair, or
  // one without cells, is one task at the end of it) and there is no short
  // class
  const bool pipe = PL.pipe && tune.pair_bands != 1;
  pp.rows_lo = pipe ? 0 : PL.rows_lo;
  pp.rows_hi = PL.rows_hi;
  pp.order = order;
  pp.counts = counts;
  pp.counters = counts + 2;
  if (sk::launch_pair_plan(pp, stream) != hipSuccess) return SK_ERR_HIP;

  sk::PairArgs a{};
  a.incx = incx;
  a.incy = incy;
  a.x_n = pp.x_n;
  a.x_start = X->offsets ? px.start : nullptr;
  a.y_n = pp.y_n;
  a.y_start = Y->offsets ? py.start : nullptr;
  a.x_len = Xr.len;
  a.y_len = Yr.len;
  a.scale = ldexp(1.0, -(2 * lam + 1));
  a.implicit = implicit ? 1 : 0;
  a.bandbuf = reinterpret_cast<double*>(base + PL.bands);
  a.band_stride = PL.band_stride;
  a.out = out;
  a.gram_ny = pp.gram_ny;
  // long-row class first (it holds the longest pairs), then the short class
  a.order = order;
  a.count = counts;
  a.counter = counts + 2;
  hipError_t e = hipSuccess;
  if (pipe) {
    // long class: every band of a pair at once (pipelined band tasks)
    int32_t* task_base = reinterpret_cast<int32_t*>(base + PL.task_base);
    double* tbuf = reinterpret_cast<double*>(base + PL.tbuf);
    if (sk::launch_band_plan(pp, PL.rows_hi, task_base, counts + 4, stream) != hipSuccess)
      return SK_ERR_HIP;
    if (sk::launch_fill_task_slots(reinterpret_cast<uint64_t*>(tbuf), pp, task_base,
                                   PL.band_stride, PL.tasks_max, sk::kBandSlotSentinel,
                                   stream) != hipSuccess)
      return SK_ERR_HIP;
    sk::PairArgs b = a;
    b.task_base = task_base;
    b.task_counter = counts + 4;
    b.tbuf = tbuf;
    b.tstride = PL.band_stride;
    // a batch of equal lengths has one top band for all its pairs: when it
    // needs all R rows per lane, the kernel with bands of one height runs
    // (the fitted kernel exists at the largest fitting height only)
    bool fit_top = sk::sweep_fn(sk::kKernelPairBand, lam, PL.rows_hi, d) != nullptr;
    if (fit_top && !X->offsets && !Y->offsets) {
      const int64_t band_rows = 64 * (int64_t)PL.rows_hi;
      const int64_t M = (int64_t)((Xr.len < Yr.len ? Xr.len : Yr.len) - 1) << lam;
      const int64_t top_rows = M - (M - 1) / band_rows * band_rows;
      fit_top = 2 * top_rows <= band_rows;
    }
    e = sk::launch_pair_bands(b, lam, PL.rows_hi, d, (PL.tasks_max + 3) & ~int64_t(3), stream,
                              tune.pair_blocks_per_cu, fit_top);
  } else {
    e = sk::launch_pairs(a, lam, PL.rows_hi, d, PL.slots, stream, tune.pair_blocks_per_cu);
  }
  if (e == hipSuccess && !pipe) {
    // the short class follows the long one in `order`; its offset (the long
    // class's count) is only known on the device, where the kernel reads it
    a.order = order;
    a.count = counts + 1;
    a.counter = counts + 3;
    a.order_base = counts;  // start of the short class: order[counts[0]]
    e = sk::launch_pairs(a, lam, PL.rows_lo, d, PL.slots, stream, tune.pair_blocks_per_cu);
  }
  if (e == hipErrorInvalidValue) return SK_ERR_UNSUPPORTED;
  return e == hipSuccess ? SK_OK : SK_ERR_HIP;
}

// Any channel count: the increment Gram on the matrix cores, then the
// coefficient sweep, wave chunk by wave chunk (coef.hip).
sk_status run_coef(const sk_paths* X, const sk_paths* Y, int32_t lam0, uint32_t flags,
                   float* out, void* ws, size_t ws_bytes, hipStream_t stream, int mode) {
  const CoefPlan P = coef_plan(X, Y, lam0, mode);
  if (P.R == 0) return SK_ERR_UNSUPPORTED;
  if (ws_bytes < P.total) return SK_ERR_WORKSPACE;
  const int d = X->dim;
  const int dp = sk::padded_dim(d);
  const ForwardLayout L = forward_layout(X, Y);
  char* base = static_cast<char*>(ws);
  float* incx = reinterpret_cast<float*>(base + L.incx) + sk::kStreamPad * dp;
  float* incy = reinterpret_cast<float*>(base + L.incy) + sk::kStreamPad * dp;
  float* coef = reinterpret_cast<float*>(base + P.coef_off);
  sk::PathPlan px{reinterpret_cast<int32_t*>(base + L.planx_n),
                  reinterpret_cast<int64_t*>(base + L.planx_start)};
  sk::PathPlan py{reinterpret_cast<int32_t*>(base + L.plany_n),
                  reinterpret_cast<int64_t*>(base + L.plany_start)};
  const sk::Batch bx = to_batch(X), by = to_batch(Y);
  if (X->offsets && sk::launch_plan(bx, px, stream) != hipSuccess) return SK_ERR_HIP;
  if (Y->offsets && sk::launch_plan(by, py, stream) != hipSuccess) return SK_ERR_HIP;
  const int rounding = rounding_of(flags);
  if (sk::launch_increments_xy(bx, X->offsets ? &px : nullptr, 1.0f, by,
                               Y->offsets ? &py : nullptr, 1.0f, dp, incx, incy, stream,
                               rounding) != hipSuccess)
    return SK_ERR_HIP;
  // both kernels see the refined counts (the producer divides them back)
  if (X->offsets && sk::launch_scale_plan(px, X->n_paths, P.rep, stream) != hipSuccess)
    return SK_ERR_HIP;
  if (Y->offsets && sk::launch_scale_plan(py, Y->n_paths, P.rep, stream) != hipSuccess)
    return SK_ERR_HIP;
  const sk_paths Xr = refined(X, P.rep), Yr = refined(Y, P.rep);

  sk::CoefArgs c{};
  c.incx = incx;
  c.incy = incy;
  c.x_n = X->offsets ? px.n : nullptr;
  c.x_start = X->offsets ? px.start : nullptr;
  c.y_n = Y->offsets ? py.n : nullptr;
  c.y_start = Y->offsets ? py.start : nullptr;
  c.x_len = Xr.len;
  c.y_len = Yr.len;
  c.nx = X->n_paths;
  c.ny = Y->n_paths;
  c.mode = mode;
  c.run = P.run;
  c.runs_per_row = P.runs_per_row;
  c.d = d;
  c.dpad = dp;
  c.R = P.R;
  c.lam = P.lam;
  c.rep = P.rep;
  c.scale = ldexpf(1.0f, -(2 * P.lam + 1)) / ((float)P.rep * (float)P.rep);
  c.coef = coef;
  c.coef_stride = P.stride;

  sk::SweepArgs a{};
  a.x_n = c.x_n;
  a.x_start = c.x_start;
  a.y_n = c.y_n;
  a.y_start = c.y_start;
  a.x_len = Xr.len;
  a.y_len = Yr.len;
  a.nx = X->n_paths;
  a.ny = Y->n_paths;
  a.mode = mode;
  a.no_diag = (flags & SK_NO_DIAG) ? 1 : 0;
  a.implicit = (flags & SK_IMPLICIT) ? 1 : 0;
  a.run = P.run;
  a.runs_per_row = P.runs_per_row;
  a.out = out;
  a.out_ld = Y->n_paths;
  a.coef = coef;
  a.coef_stride = P.stride;
  for (int64_t w0 = 0; w0 < P.n_waves; w0 += P.chunk) {
    const int64_t nw = (P.n_waves - w0) < P.chunk ? (P.n_waves - w0) : P.chunk;
    c.wave0 = w0;
    c.n_waves = nw;
    if (sk::launch_coef(c, rounding, X->len - 1, Y->len - 1, stream) != hipSuccess)
      return SK_ERR_HIP;
    a.wave0 = w0;
    a.n_waves = nw;
    const hipError_t e = sk::launch_coef_sweep(a, P.lam, P.R, a.implicit != 0, stream);
    if (e == hipErrorInvalidValue) return SK_ERR_UNSUPPORTED;
    if (e != hipSuccess) return SK_ERR_HIP;
  }
  return SK_OK;
}

// A symmetric Gram's waves enumerate only the runs of its upper triangle; an
// unbiased one (diagonal zeroed) leaves the diagonal out of them, and
// zero_skipped_diagonal writes it.
void set_triangle(sk::SweepArgs& a, int mode) {
  if (mode != 2) return;
  const int64_t s = a.no_diag ? 1 : 0;
  a.tri = (int32_t)(1 + s);
  a.n_waves = a.nx > s ? sk::tri_runs(a.nx - s, a.runs_per_row, a.run, s) : 0;
}

sk_status zero_skipped_diagonal(const sk::SweepArgs& a, hipStream_t stream) {
  if (a.tri != 2 || !a.out) return SK_OK;
  return sk::launch_zero_diag(a.out, a.nx, stream) == hipSuccess ? SK_OK : SK_ERR_HIP;
}

sk_status run_forward(const sk_paths* X, const sk_paths* Y, int32_t lam0, uint32_t flags,
                      float* out, void* ws, size_t ws_bytes, hipStream_t stream, int mode) {
  if (X->dim > kMaxFusedDim)
    return run_coef(X, Y, lam0, flags, out, ws, ws_bytes, stream, mode);
  const int rounding = rounding_of(flags);
  const sk_tune tune = sk::tuning_for(mode == 0 ? SK_OP_PAIR : SK_OP_GRAM, X, Y, lam0, flags);
  const bool implicit = (flags & SK_IMPLICIT) != 0;
  if (mode == 0)
    return run_pairs(X, Y, lam0, out, ws, ws_bytes, stream, false, rounding, tune, implicit);
  const Order o = split_order(lam0);
  const int32_t lam = o.k;
  const sk_paths Xr = refined(X, o.rep), Yr = refined(Y, o.rep);
  const int d = X->dim;
  const int dp = sk::padded_dim(d);
  const int64_t fine_rows = (int64_t)(Xr.len - 1) << lam;
  const int R = sk::choose_rows_per_lane(fine_rows < 1 ? 1 : fine_rows, lam, d);
  if (R == 0) {
    // x paths taller than one wave's strips: every (a, b) through the
    // persistent pair kernel with row bands (a symmetric Gram is filled in
    // both halves by solving both)
    const sk_status st =
        run_pairs(X, Y, lam0, out, ws, ws_bytes, stream, true, rounding, tune, implicit);
    if (st == SK_OK && mode == 2 && (flags & SK_NO_DIAG) &&
        sk::launch_zero_diag(out, X->n_paths, stream) != hipSuccess)
      return SK_ERR_HIP;
    return st;
  }
  const ForwardLayout L = forward_layout(&Xr, &Yr);
  if (ws_bytes < L.total) return SK_ERR_WORKSPACE;

  char* base = static_cast<char*>(ws);
  float* incx = reinterpret_cast<float*>(base + L.incx) + sk::kStreamPad * dp;
  float* incy = reinterpret_cast<float*>(base + L.incy) + sk::kStreamPad * dp;
  sk::PathPlan px{reinterpret_cast<int32_t*>(base + L.planx_n),
                  reinterpret_cast<int64_t*>(base + L.planx_start)};
  sk::PathPlan py{reinterpret_cast<int32_t*>(base + L.plany_n),
                  reinterpret_cast<int64_t*>(base + L.plany_start)};
  const sk::Batch bx = to_batch(X), by = to_batch(Y);
  if (X->offsets && sk::launch_plan(bx, px, stream) != hipSuccess) return SK_ERR_HIP;
  if (Y->offsets && sk::launch_plan(by, py, stream) != hipSuccess) return SK_ERR_HIP;
  // h = G0 / 2^(2 lam + 1): fold the exact power-of-two scale into the x side
  const float scale = ldexpf(1.0f, -(2 * lam + 1));
  if (sk::launch_increments_xy(bx, X->offsets ? &px : nullptr, scale, by,
                               Y->offsets ? &py : nullptr, 1.0f, dp, incx, incy, stream, rounding,
                               o.rep) != hipSuccess)
    return SK_ERR_HIP;
  if (X->offsets && sk::launch_scale_plan(px, X->n_paths, o.rep, stream) != hipSuccess)
    return SK_ERR_HIP;
  if (Y->offsets && sk::launch_scale_plan(py, Y->n_paths, o.rep, stream) != hipSuccess)
    return SK_ERR_HIP;

  sk::SweepArgs a{};
  a.incx = incx;
  a.incy = incy;
  a.x_n = X->offsets ? px.n : nullptr;
  a.x_start = X->offsets ? px.start : nullptr;
  a.y_n = Y->offsets ? py.n : nullptr;
  a.y_start = Y->offsets ? py.start : nullptr;
  a.x_len = Xr.len;
  a.y_len = Yr.len;
  a.nx = X->n_paths;
  a.ny = Y->n_paths;
  a.mode = mode;
  a.no_diag = (flags & SK_NO_DIAG) ? 1 : 0;
  a.implicit = implicit ? 1 : 0;
  a.out = out;
  a.out_ld = Y->n_paths;
  if (mode == 0) {
    a.run = 1;
    a.runs_per_row = 1;
    a.n_waves = X->n_paths;
  } else {
    a.run = Y->offsets ? 1
                       : (int32_t)choose_sweep_run(X->n_paths, Y->n_paths,
                                                   (int64_t)(Y->len - 1) << lam, mode == 2,
                                                   tune.run, a.no_diag != 0);
    a.runs_per_row = (Y->n_paths + a.run - 1) / a.run;
    a.n_waves = X->n_paths * a.runs_per_row;
    set_triangle(a, mode);
  }
  const hipError_t e = sk::launch_sweep(a, lam, R, d, stream, tune.waves_per_block);
  if (e == hipErrorInvalidValue) return SK_ERR_UNSUPPORTED;
  if (e != hipSuccess) return SK_ERR_HIP;
  return zero_skipped_diagonal(a, stream);
}

// MMD^2 workspace: the three Gram blocks, the two upstream weight matrices,
// then the largest workspace of the calls it makes
// (they run one after the other on the stream and share it).
struct Mmd2Layout {
  size_t kxx, kyy, kxy, wxx, wxy, sub, sub_bytes, total;
};

Mmd2Layout mmd2_layout(const sk_paths* X, const sk_paths* Y, int32_t lam, uint32_t flags) {
  const size_t n = (size_t)X->n_paths, m = (size_t)Y->n_paths;
  Mmd2Layout L{};
  size_t off = 0;
  L.kxx = off;
  off += align256(n * n * sizeof(float));
  L.kyy = off;
  off += align256(m * m * sizeof(float));
  L.kxy = off;
  off += align256(n * m * sizeof(float));
  L.wxx = off;
  off += align256(n * n * sizeof(float));
  L.wxy = off;
  off += align256(n * m * sizeof(float));
  size_t sub = gram_ws(X, X, lam);
  const size_t c[] = {gram_ws(Y, Y, lam), gram_ws(X, Y, lam)};
  for (size_t v : c) sub = v > sub ? v : sub;
  if (flags & SK_MMD2_GRAD) {
    const size_t b1 = grad_plan(X, X, lam, SK_SYMMETRIC | SK_NO_DIAG).total;
    const size_t b2 = grad_plan(X, Y, lam, 0).total;
    sub = b1 > sub ? b1 : sub;
    sub = b2 > sub ? b2 : sub;
  }
  L.sub = off;
  L.sub_bytes = sub;
  off += align256(sub);
  L.total = off;
  return L;
}

// ---- learned corrector ----------------------------------------------------
sk_status check_corrector_batches(const sk_paths* X, const sk_paths* Y) {
  if (!X || !Y) return SK_ERR_NULL;
  if (!valid_batch(X) || !valid_batch(Y)) return SK_ERR_SHAPE;
  if (X->dim != Y->dim || X->n_paths != Y->n_paths) return SK_ERR_SHAPE;
  if (X->offsets || Y->offsets) return SK_ERR_UNSUPPORTED;
  // the feature map holds 64 x 64 blocks of 4 x 4 coarse cells
  if (X->len > 257 || Y->len > 257 || X->dim > 16) return SK_ERR_UNSUPPORTED;
  if (X->n_paths > 0 && (!X->points || !Y->points)) return SK_ERR_NULL;
  return SK_OK;
}

struct DwPlan {
  int nblocks;
  int64_t per_block;
};

// weight-gradient partials of layer l: at most 256 workgroups, whole chunks
// of 16 output positions each
DwPlan dw_plan(int l, int64_t n) {
  const int64_t ho = sk::corr::kLayerHi[l] / 2;
  const int64_t T = n * ho * ho;
  if (T == 0) return DwPlan{0, 16};
  int64_t nb = (T + 63) / 64;
  if (nb > 256) nb = 256;
  int64_t per = (T + nb - 1) / nb;
  per = (per + 15) & ~int64_t(15);
  return DwPlan{(int)((T + per - 1) / per), per};
}

size_t corrector_bwd_ws(int64_t n) {
  size_t part = 0;
  for (int l = 0; l < sk::corr::kLayers; ++l) {
    const size_t w = (size_t)sk::corr::layer_params(l) * sizeof(float);
    const size_t v = (size_t)dw_plan(l, n).nblocks * w;
    part = v > part ? v : part;
  }
  return 2 * align256((size_t)n * sk::corr::kFeatFloats * sizeof(float)) + align256(part) + 256;
}

struct PredictLayout {
  PairLayout pl;
  size_t wb, feats, y, k0, total;
};

PredictLayout predict_layout(const sk_paths* X, const sk_paths* Y, int32_t lam) {
  PredictLayout L{};
  L.pl = pair_layout(X, Y, lam, false);
  const size_t n = (size_t)X->n_paths;
  size_t off = L.pl.total;
  L.wb = off;
  off += align256((size_t)sk::corr::kHeadOffset * sizeof(uint16_t));
  L.feats = off;
  off += align256(n * sk::corr::kFeatFloats * sizeof(uint16_t));
  L.y = off;
  off += align256(n * 2 * sizeof(float));
  L.k0 = off;
  off += align256(n * sizeof(float));
  L.total = off;
  return L;
}

// Dense unscaled increments of both batches of a corrector call.
sk_status corrector_increments(const sk_paths* X, const sk_paths* Y, char* base, float** incx,
                               float** incy, hipStream_t st) {
  const int dp = sk::padded_dim(X->dim);
  const ForwardLayout L = forward_layout(X, Y);
  *incx = reinterpret_cast<float*>(base + L.incx) + sk::kStreamPad * dp;
  *incy = reinterpret_cast<float*>(base + L.incy) + sk::kStreamPad * dp;
  if (sk::launch_increments_xy(to_batch(X), nullptr, 1.0f, to_batch(Y), nullptr, 1.0f, dp, *incx,
                               *incy, st) != hipSuccess)
    return SK_ERR_HIP;
  return SK_OK;
}

sk_status corrector_forward(const float* params, const sk::corr::bf16* feats, int64_t n,
                            sk::corr::bf16* acts, float* y, hipStream_t st) {
  using namespace sk::corr;
  const bf16* in = feats;
  for (int l = 0; l < kLayers; ++l) {
    ConvArgs a{};
    a.in = in;
    a.w = params + param_offset(l);
    a.b = a.w + (int64_t)kCout * 9 * kLayerCin[l];
    a.out = acts + act_offset(l) * n;
    a.n = n;
    if (launch_conv_fwd(l, a, st) != hipSuccess) return SK_ERR_HIP;
    in = a.out;
  }
  if (launch_head_fwd(in, params + kHeadOffset, params + kHeadOffset + 2 * kHeadIn, n, y, st) !=
      hipSuccess)
    return SK_ERR_HIP;
  return SK_OK;
}

// ---- static-kernel lift ------------------------------------------------------
// Workspace of the lifted sweep: dense node rows of X and of Y (kStreamPad
// rows on each side), then the ragged plans.
struct LiftedLayout {
  size_t nodex, nodey, planx_n, planx_start, plany_n, plany_start, total;
};

size_t node_rows(const sk_paths* p) {
  return (size_t)p->n_paths * (size_t)p->len + 2 * (size_t)sk::kStreamPad;
}

LiftedLayout lifted_layout(const sk_paths* X, const sk_paths* Y) {
  const size_t dp = (size_t)sk::padded_dim(X->dim);
  LiftedLayout L{};
  size_t off = 0;
  L.nodex = off;
  off += align256(node_rows(X) * dp * sizeof(float));
  L.nodey = off;
  off += align256(node_rows(Y) * dp * sizeof(float));
  L.planx_n = off;
  off += plan_bytes_n(X);
  L.planx_start = off;
  off += plan_bytes_start(X);
  L.plany_n = off;
  off += plan_bytes_n(Y);
  L.plany_start = off;
  off += plan_bytes_start(Y);
  L.total = off;
  return L;
}

sk_status check_static_kernel(const sk_static_kernel* k) {
  if (!k) return SK_ERR_NULL;
  if (k->kind == SK_STATIC_LINEAR) return SK_OK;
  if (k->kind != SK_STATIC_RBF) return SK_ERR_VALUE;
  return (k->sigma > 0.0 && isfinite(k->sigma) && isfinite(1.0 / (2.0 * k->sigma * k->sigma)))
             ? SK_OK
             : SK_ERR_VALUE;
}

// mode 0: pairs (x_k, y_k); 1: Gram; 2: symmetric Gram (upper triangle, mirrored)
sk_status run_lifted(const sk_paths* X, const sk_paths* Y, int32_t lam, uint32_t flags,
                     const sk_static_kernel* kernel, float* out, void* ws, size_t ws_bytes,
                     hipStream_t stream, int mode) {
  // the linear kernel's lift is the path itself: the plain scheme
  if (kernel->kind == SK_STATIC_LINEAR)
    return run_forward(X, Y, lam, flags, out, ws, ws_bytes, stream, mode);
  const int d = X->dim;
  const int dp = sk::padded_dim(d);
  const int64_t fine_rows = (int64_t)(X->len - 1) << lam;
  const int R = sk::choose_rows_for(sk::kKernelLifted, fine_rows < 1 ? 1 : fine_rows, lam, d);
  if (R == 0) return SK_ERR_UNSUPPORTED;
  const LiftedLayout L = lifted_layout(X, Y);
  if (ws_bytes < L.total) return SK_ERR_WORKSPACE;
  char* base = static_cast<char*>(ws);
  float* nx = reinterpret_cast<float*>(base + L.nodex) + sk::kStreamPad * dp;
  float* ny = reinterpret_cast<float*>(base + L.nodey) + sk::kStreamPad * dp;
  sk::PathPlan px{reinterpret_cast<int32_t*>(base + L.planx_n),
                  reinterpret_cast<int64_t*>(base + L.planx_start)};
  sk::PathPlan py{reinterpret_cast<int32_t*>(base + L.plany_n),
                  reinterpret_cast<int64_t*>(base + L.plany_start)};
  const sk::Batch bx = to_batch(X), by = to_batch(Y);
  if (X->offsets && sk::launch_plan(bx, px, stream) != hipSuccess) return SK_ERR_HIP;
  if (Y->offsets && sk::launch_plan(by, py, stream) != hipSuccess) return SK_ERR_HIP;
  if (sk::launch_nodes(bx, X->offsets ? &px : nullptr, dp, nx, stream) != hipSuccess)
    return SK_ERR_HIP;
  if (sk::launch_nodes(by, Y->offsets ? &py : nullptr, dp, ny, stream) != hipSuccess)
    return SK_ERR_HIP;

  sk::SweepArgs a{};
  a.incx = nx;
  a.incy = ny;
  a.x_n = X->offsets ? px.n : nullptr;
  a.x_start = X->offsets ? px.start : nullptr;
  a.y_n = Y->offsets ? py.n : nullptr;
  a.y_start = Y->offsets ? py.start : nullptr;
  a.x_len = X->len;
  a.y_len = Y->len;
  a.nx = X->n_paths;
  a.ny = Y->n_paths;
  a.mode = mode;
  a.no_diag = (flags & SK_NO_DIAG) ? 1 : 0;
  a.implicit = (flags & SK_IMPLICIT) ? 1 : 0;
  a.lift_inv = 1.0 / (2.0 * kernel->sigma * kernel->sigma);
  a.lift_scale = ldexp(1.0, -(2 * lam + 1));
  a.out = out;
  a.out_ld = Y->n_paths;
  if (mode == 0) {
    a.run = 1;
    a.runs_per_row = 1;
    a.n_waves = X->n_paths;
  } else {
    a.run = Y->offsets ? 1
                       : (int32_t)choose_sweep_run(X->n_paths, Y->n_paths,
                                                   (int64_t)(Y->len - 1) << lam, mode == 2, 0,
                                                   a.no_diag != 0);
    a.runs_per_row = (Y->n_paths + a.run - 1) / a.run;
    a.n_waves = X->n_paths * a.runs_per_row;
    set_triangle(a, mode);
  }
  const hipError_t e = sk::launch_lifted(a, lam, R, d, stream, 0);
  if (e == hipErrorInvalidValue) return SK_ERR_UNSUPPORTED;
  if (e != hipSuccess) return SK_ERR_HIP;
  return zero_skipped_diagonal(a, stream);
}

}  // namespace

// ---- the allocation-free Gram ------------------------------------------------
// Its workspace is this file-scope array (each GPU that runs the library
// holds one copy until the process ends).  In host code `scratch` names a
// host-side stand-in, not the device array: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (nullptr on failure).
void* scratch_address() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

const char* sigkernel_version(void) { return "0.1.0"; }

const char* sigkernel_status_string(sk_status s) {
  switch (s) {
    case SK_OK: return "ok";
    case SK_ERR_NULL: return "null pointer argument";
    case SK_ERR_SHAPE: return "inconsistent shapes";
    case SK_ERR_ORDER: return "unsupported dyadic order";
    case SK_ERR_WORKSPACE: return "workspace missing or too small";
    case SK_ERR_FLAGS: return "invalid flags";
    case SK_ERR_HIP: return "HIP launch error";
    case SK_ERR_UNSUPPORTED: return "shape outside the compiled configurations";
    case SK_ERR_STATE: return "not allowed while the stream is being captured";
    case SK_ERR_VALUE: return "parameter outside its domain";
    default: return "unknown status";
  }
}

size_t sigkernel_workspace_bytes(int32_t op, const sk_paths* X, const sk_paths* Y,
                                 int32_t dyadic_order, uint32_t flags) {
  (void)dyadic_order;
  (void)flags;
  if (!valid_batch(X) || !valid_batch(Y)) return 0;
  switch (op) {
    case SK_OP_PAIR:
      if (X->dim != Y->dim) return 0;
      if (X->dim > kMaxFusedDim) return coef_plan(X, Y, dyadic_order, 0).total;
      return pair_layout(X, Y, dyadic_order, false).total;
    case SK_OP_GRAM:
      return gram_ws(X, Y, dyadic_order);
    case SK_OP_GRAM_BACKWARD:
      if (X->dim != Y->dim) return 0;
      return grad_plan(X, Y, dyadic_order, flags).total;
    case SK_OP_MMD2:
      if (X->dim != Y->dim) return 0;
      return mmd2_layout(X, Y, dyadic_order, flags).total;
    case SK_OP_CORRECTOR_FEATURES:
      if (check_corrector_batches(X, Y) == SK_ERR_SHAPE) return 0;
      return forward_ws(X, Y);
    case SK_OP_CORRECTOR_BACKWARD:
      return corrector_bwd_ws(X->n_paths);
    case SK_OP_CORRECTOR_PREDICT:
      if (check_corrector_batches(X, Y) == SK_ERR_SHAPE) return 0;
      return predict_layout(X, Y, dyadic_order).total;
    case SK_OP_PAIR_LIFTED:
    case SK_OP_GRAM_LIFTED: {
      // the linear static kernel runs the plain calls: room for either
      const size_t f = lifted_layout(X, Y).total;
      const size_t g = sigkernel_workspace_bytes(op == SK_OP_PAIR_LIFTED ? SK_OP_PAIR : SK_OP_GRAM,
                                                 X, Y, dyadic_order, flags);
      return f > g ? f : g;
    }
    default:
      return 0;
  }
}

sk_status sigkernel_pair(const sk_paths* x, const sk_paths* y, int32_t dyadic_order,
                         uint32_t flags, float* out, void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y) return SK_ERR_NULL;
  if (!valid_batch(x) || !valid_batch(y)) return SK_ERR_SHAPE;
  if (!out && x->n_paths > 0) return SK_ERR_NULL;
  if ((x->n_paths > 0 && !x->points) || (y->n_paths > 0 && !y->points)) return SK_ERR_NULL;
  if (x->dim != y->dim || x->n_paths != y->n_paths) return SK_ERR_SHAPE;
  if (!order_ok(dyadic_order, x, y, kMaxDyadicOrder)) return SK_ERR_ORDER;
  if (sk_status f = check_flags(flags, SK_GRAM_BF16 | SK_GRAM_F16 | SK_IMPLICIT)) return f;
  if (x->n_paths == 0) return SK_OK;
  if (!ws) return SK_ERR_WORKSPACE;
  return run_forward(x, y, dyadic_order, flags, out, ws, ws_bytes,
                     static_cast<hipStream_t>(stream), 0);
}

sk_status sigkernel_gram(const sk_paths* X, const sk_paths* Y, int32_t dyadic_order,
                         uint32_t flags, float* K, void* ws, size_t ws_bytes, void* stream) {
  if (!X || !Y) return SK_ERR_NULL;
  if (!valid_batch(X) || !valid_batch(Y)) return SK_ERR_SHAPE;
  if (!K && X->n_paths > 0 && Y->n_paths > 0) return SK_ERR_NULL;
  if ((X->n_paths > 0 && !X->points) || (Y->n_paths > 0 && !Y->points)) return SK_ERR_NULL;
  if (X->dim != Y->dim) return SK_ERR_SHAPE;
  if (!order_ok(dyadic_order, X, Y, kMaxDyadicOrder)) return SK_ERR_ORDER;
  if (sk_status f = check_flags(
          flags, SK_SYMMETRIC | SK_NO_DIAG | SK_GRAM_BF16 | SK_GRAM_F16 | SK_IMPLICIT))
    return f;
  if ((flags & SK_SYMMETRIC) &&
      (X->points != Y->points || X->offsets != Y->offsets || X->n_paths != Y->n_paths ||
       X->len != Y->len))
    return SK_ERR_SHAPE;
  if (X->n_paths == 0 || Y->n_paths == 0) return SK_OK;
  if (!ws) return SK_ERR_WORKSPACE;
  return run_forward(X, Y, dyadic_order, flags, K, ws, ws_bytes,
                     static_cast<hipStream_t>(stream), (flags & SK_SYMMETRIC) ? 2 : 1);
}

sk_status sigkernel_gram_noalloc(const sk_paths* X, const sk_paths* Y, int32_t dyadic_order,
                                 uint32_t flags, float* K, void* stream) {
  // every check that sigkernel_gram makes before touching the workspace, then
  // the size check, all before any HIP call
  if (!X || !Y) return SK_ERR_NULL;
  if (!valid_batch(X) || !valid_batch(Y)) return SK_ERR_SHAPE;
  if (!K && X->n_paths > 0 && Y->n_paths > 0) return SK_ERR_NULL;
  if ((X->n_paths > 0 && !X->points) || (Y->n_paths > 0 && !Y->points)) return SK_ERR_NULL;
  if (X->dim != Y->dim) return SK_ERR_SHAPE;
  if (!order_ok(dyadic_order, X, Y, kMaxDyadicOrder)) return SK_ERR_ORDER;
  if (sk_status f = check_flags(
          flags, SK_SYMMETRIC | SK_NO_DIAG | SK_GRAM_BF16 | SK_GRAM_F16 | SK_IMPLICIT))
    return f;
  if (X->n_paths == 0 || Y->n_paths == 0) return SK_OK;
  if (gram_ws(X, Y, dyadic_order) > kNoAllocScratchBytes) return SK_ERR_WORKSPACE;
  void* ws = scratch_address();
  if (!ws) return SK_ERR_HIP;
  return sigkernel_gram(X, Y, dyadic_order, flags, K, ws, kNoAllocScratchBytes, stream);
}

size_t sigkernel_gram_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

sk_status sigkernel_pair_lifted(const sk_paths* x, const sk_paths* y, int32_t dyadic_order,
                                uint32_t flags, const sk_static_kernel* kernel, float* out,
                                void* ws, size_t ws_bytes, void* stream) {
  if (!x || !y) return SK_ERR_NULL;
  if (!valid_batch(x) || !valid_batch(y)) return SK_ERR_SHAPE;
  if (!out && x->n_paths > 0) return SK_ERR_NULL;
  if ((x->n_paths > 0 && !x->points) || (y->n_paths > 0 && !y->points)) return SK_ERR_NULL;
  if (x->dim != y->dim || x->n_paths != y->n_paths) return SK_ERR_SHAPE;
  if (!order_ok(dyadic_order, x, y, kMaxKernelOrder)) return SK_ERR_ORDER;
  if (sk_status k = check_static_kernel(kernel)) return k;
  const uint32_t allowed = kernel->kind == SK_STATIC_LINEAR ? SK_IMPLICIT | SK_GRAM_BF16 |
                                                                  SK_GRAM_F16
                                                            : SK_IMPLICIT;
  if (sk_status f = check_flags(flags, allowed)) return f;
  if (x->n_paths == 0) return SK_OK;
  if (!ws) return SK_ERR_WORKSPACE;
  return run_lifted(x, y, dyadic_order, flags, kernel, out, ws, ws_bytes,
                    static_cast<hipStream_t>(stream), 0);
}

sk_status sigkernel_gram_lifted(const sk_paths* X, const sk_paths* Y, int32_t dyadic_order,
                                uint32_t flags, const sk_static_kernel* kernel, float* K,
                                void* ws, size_t ws_bytes, void* stream) {
  if (!X || !Y) return SK_ERR_NULL;
  if (!valid_batch(X) || !valid_batch(Y)) return SK_ERR_SHAPE;
  if (!K && X->n_paths > 0 && Y->n_paths > 0) return SK_ERR_NULL;
  if ((X->n_paths > 0 && !X->points) || (Y->n_paths > 0 && !Y->points)) return SK_ERR_NULL;
  if (X->dim != Y->dim) return SK_ERR_SHAPE;
  if (!order_ok(dyadic_order, X, Y, kMaxKernelOrder)) return SK_ERR_ORDER;
  if (sk_status k = check_static_kernel(kernel)) return k;
  const uint32_t allowed =
      SK_SYMMETRIC | SK_NO_DIAG | SK_IMPLICIT |
      (kernel->kind == SK_STATIC_LINEAR ? SK_GRAM_BF16 | SK_GRAM_F16 : 0u);
  if (sk_status f = check_flags(flags, allowed)) return f;
  if ((flags & SK_SYMMETRIC) &&
      (X->points != Y->points || X->offsets != Y->offsets || X->n_paths != Y->n_paths ||
       X->len != Y->len))
    return SK_ERR_SHAPE;
  if (X->n_paths == 0 || Y->n_paths == 0) return SK_OK;
  if (!ws) return SK_ERR_WORKSPACE;
  return run_lifted(X, Y, dyadic_order, flags, kernel, K, ws, ws_bytes,
                    static_cast<hipStream_t>(stream), (flags & SK_SYMMETRIC) ? 2 : 1);
}

sk_status sigkernel_reduced_measure(const float* K, const float* alpha, int32_t n, double lam,
                                    double step, int32_t iters, double* beta, double* loss,
                                    double* step_out, void* stream) {
  if (!K || !alpha || !beta) return SK_ERR_NULL;
  if (n < 1 || n > sk::kMaxReduceN || iters < 0) return SK_ERR_SHAPE;
  if (!(lam >= 0.0) || !isfinite(lam) || !(step >= 0.0) || !isfinite(step)) return SK_ERR_VALUE;
  sk::ReduceArgs a{};
  a.K = K;
  a.ld = n;
  a.alpha = alpha;
  a.n = n;
  a.lam = lam;
  a.step = step;
  a.iters = iters;
  a.beta = beta;
  a.loss = loss;
  a.step_out = step_out;
  return sk::launch_reduce(a, static_cast<hipStream_t>(stream)) == hipSuccess ? SK_OK
                                                                               : SK_ERR_HIP;
}

sk_status sigkernel_reduced_measure_support(const float* K, const float* alpha, int32_t n,
                                            int32_t support, int32_t iters, int32_t rounds,
                                            double step, double* beta, double* lam_out,
                                            double* step_out, void* stream) {
  if (!K || !alpha || !beta || !lam_out) return SK_ERR_NULL;
  if (n < 1 || n > sk::kMaxReduceN || iters < 0) return SK_ERR_SHAPE;
  if (support < 1 || support > n || rounds < 1) return SK_ERR_VALUE;
  if (!(step >= 0.0) || !isfinite(step)) return SK_ERR_VALUE;
  sk::ReduceArgs a{};
  a.K = K;
  a.ld = n;
  a.alpha = alpha;
  a.n = n;
  a.step = step;
  a.iters = iters;
  a.support = support;
  a.rounds = rounds;
  a.beta = beta;
  a.lam_out = lam_out;
  a.step_out = step_out;
  return sk::launch_reduce(a, static_cast<hipStream_t>(stream)) == hipSuccess ? SK_OK
                                                                               : SK_ERR_HIP;
}

sk_status sigkernel_increment_gram(const sk_paths* X, const sk_paths* Y, int32_t gram,
                                  uint32_t flags, float* G0, int64_t ldg, void* stream) {
  if (!X || !Y) return SK_ERR_NULL;
  if (!valid_batch(X) || !valid_batch(Y) || X->dim != Y->dim) return SK_ERR_SHAPE;
  if (gram != 0 && gram != 1) return SK_ERR_FLAGS;
  if (!gram && X->n_paths != Y->n_paths) return SK_ERR_SHAPE;
  if (sk_status f = check_flags(flags, SK_GRAM_BF16 | SK_GRAM_F16)) return f;
  if (X->offsets || Y->offsets) return SK_ERR_UNSUPPORTED;
  if (ldg != 0 && ldg < (int64_t)Y->len - 1) return SK_ERR_SHAPE;
  const int64_t pairs = gram ? X->n_paths * Y->n_paths : X->n_paths;
  if (pairs == 0 || X->len < 2 || Y->len < 2) return SK_OK;
  if (!G0 || !X->points || !Y->points) return SK_ERR_NULL;
  if (X->dim > sk::kGramMfmaMaxDim) return SK_ERR_UNSUPPORTED;
  sk::GramArgs a{};
  a.x = X->points;
  a.y = Y->points;
  a.x_len = X->len;
  a.y_len = Y->len;
  a.d = X->dim;
  a.nx = X->n_paths;
  a.ny = Y->n_paths;
  a.gram = gram;
  a.g0 = G0;
  a.ld = ldg ? ldg : (int64_t)Y->len - 1;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = X->dim <= sk::kGramRowsMaxDim ? sk::launch_gram_rows(a, rounding_of(flags), st)
                                                     : sk::launch_gram_mfma(a, rounding_of(flags), st);
  if (e == hipErrorInvalidValue) return SK_ERR_UNSUPPORTED;
  return e == hipSuccess ? SK_OK : SK_ERR_HIP;
}

static sk_status gram_backward(const sk_paths* X, const sk_paths* Y, int32_t dyadic_order,
                               uint32_t flags, const float* dK, float* dX, float* dY, float* K,
                               bool accumulate, void* ws, size_t ws_bytes, void* stream);

sk_status sigkernel_mmd2(const sk_paths* X, const sk_paths* Y, int32_t dyadic_order,
                         uint32_t flags, float* mmd2, float* dX, void* ws, size_t ws_bytes,
                         void* stream) {
  if (!X || !Y || !mmd2) return SK_ERR_NULL;
  if (!valid_batch(X) || !valid_batch(Y)) return SK_ERR_SHAPE;
  if (X->dim != Y->dim || X->n_paths < 2 || Y->n_paths < 2) return SK_ERR_SHAPE;
  if (!order_ok(dyadic_order, X, Y, kMaxDyadicOrder)) return SK_ERR_ORDER;
  if (sk_status f = check_flags(flags, SK_MMD2_GRAD)) return f;
  if ((flags & SK_MMD2_GRAD) && !dX) return SK_ERR_NULL;
  if (!X->points || !Y->points) return SK_ERR_NULL;
  if (!ws) return SK_ERR_WORKSPACE;
  const Mmd2Layout L = mmd2_layout(X, Y, dyadic_order, flags);
  if (ws_bytes < L.total) return SK_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  float* kxx = reinterpret_cast<float*>(base + L.kxx);
  float* kyy = reinterpret_cast<float*>(base + L.kyy);
  float* kxy = reinterpret_cast<float*>(base + L.kxy);
  void* sub = base + L.sub;
  const uint32_t unb = SK_SYMMETRIC | SK_NO_DIAG;
  const bool grad = (flags & SK_MMD2_GRAD) != 0;
  // with the gradient, Kxx and Kxy come from the gradient launches' forward
  // passes (which a uniform batch of one-point paths skips)
  const bool ragged = X->offsets || Y->offsets;
  const bool fused = grad && (ragged || (X->len >= 2 && Y->len >= 2));
  sk_status r;
  if (!fused && (r = sigkernel_gram(X, X, dyadic_order, unb, kxx, sub, L.sub_bytes, stream)))
    return r;
  if ((r = sigkernel_gram(Y, Y, dyadic_order, unb, kyy, sub, L.sub_bytes, stream))) return r;
  if (!fused && (r = sigkernel_gram(X, Y, dyadic_order, 0, kxy, sub, L.sub_bytes, stream)))
    return r;
  if (grad) {
    const int64_t n = X->n_paths, m = Y->n_paths;
    float* wxx = reinterpret_cast<float*>(base + L.wxx);
    float* wxy = reinterpret_cast<float*>(base + L.wxy);
    // d MMD^2 / d Kxx[a][b] = 1 / (n (n - 1)) off the diagonal (the symmetric
    // backward ignores the diagonal); d MMD^2 / d Kxy[a][b] = -2 / (n m)
    if (sk::launch_fill(wxx, n * n, (float)(1.0 / ((double)n * (double)(n - 1))), st) !=
        hipSuccess)
      return SK_ERR_HIP;
    if (sk::launch_fill(wxy, n * m, (float)(-2.0 / ((double)n * (double)m)), st) != hipSuccess)
      return SK_ERR_HIP;
    if ((r = gram_backward(X, X, dyadic_order, unb, wxx, dX, nullptr, fused ? kxx : nullptr,
                           false, sub, L.sub_bytes, stream)))
      return r;
    // the cross term's gradient is added to dX by its point-gradient launch
    if ((r = gram_backward(X, Y, dyadic_order, 0, wxy, dX, nullptr, fused ? kxy : nullptr, true,
                           sub, L.sub_bytes, stream)))
      return r;
  }
  if (sk::launch_mmd2_reduce(kxx, X->n_paths, kyy, Y->n_paths, kxy, mmd2, st) != hipSuccess)
    return SK_ERR_HIP;
  return SK_OK;
}

// The Gram backward; K (optional) receives the forward values of the same
// pairs, as sigkernel_gram with the same flags would write them (the
// gradient launch's forward pass computes them anyway); accumulate: dX +=
// instead of dX = (the MMD's cross term).
static sk_status gram_backward(const sk_paths* X, const sk_paths* Y, int32_t dyadic_order,
                               uint32_t flags, const float* dK, float* dX, float* dY, float* K,
                               bool accumulate, void* ws, size_t ws_bytes, void* stream) {
  if (!X || !Y) return SK_ERR_NULL;
  if (!valid_batch(X) || !valid_batch(Y)) return SK_ERR_SHAPE;
  if (X->dim != Y->dim) return SK_ERR_SHAPE;
  if (!order_ok(dyadic_order, X, Y, kMaxDyadicOrder)) return SK_ERR_ORDER;
  if (sk_status f = check_flags(flags, SK_SYMMETRIC | SK_NO_DIAG)) return f;
  const bool sym = (flags & SK_SYMMETRIC) != 0;
  if (sym && (X->points != Y->points || X->offsets != Y->offsets || X->n_paths != Y->n_paths ||
              X->len != Y->len))
    return SK_ERR_SHAPE;
  if (sym && dY) return SK_ERR_SHAPE;  // one batch: its gradient goes to dX
  if (X->n_paths == 0 || Y->n_paths == 0) return SK_OK;
  if (!dK || (!dX && !dY)) return SK_ERR_NULL;
  if (!X->points || !Y->points) return SK_ERR_NULL;
  if (X->n_paths * Y->n_paths > INT32_MAX) return SK_ERR_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Order o = split_order(dyadic_order);
  const int lam = o.k;
  const sk_paths Xr = refined(X, o.rep), Yr = refined(Y, o.rep);
  const int d = X->dim;
  const bool ragged = X->offsets || Y->offsets;
  // uniform batches of one-point paths: the kernel is the constant 1, every
  // gradient is 0
  if (!ragged && (X->len < 2 || Y->len < 2)) {
    if (accumulate) return SK_OK;
    if (dX && sk::launch_fill(dX, X->n_paths * X->len * d, 0.0f, st) != hipSuccess)
      return SK_ERR_HIP;
    if (dY && sk::launch_fill(dY, Y->n_paths * Y->len * d, 0.0f, st) != hipSuccess)
      return SK_ERR_HIP;
    return SK_OK;
  }
  if (!sk::grad_supported(lam, d)) return SK_ERR_UNSUPPORTED;
  const GradPlan P = grad_plan(X, Y, dyadic_order, flags);
  // the kernel addresses a task's scratch slot, y rows and y-side sums with
  // 32-bit byte offsets
  const uint64_t k4G = 1ull << 32;
  if ((uint64_t)P.slot_stride * sizeof(double) >= k4G ||
      (uint64_t)P.cols_max * sk::padded_dim(d) * sizeof(float) >= k4G ||
      (uint64_t)P.cols_max * d * sizeof(double) >= k4G)
    return SK_ERR_UNSUPPORTED;
  if (!ws) return SK_ERR_WORKSPACE;
  if (ws_bytes < P.total) return SK_ERR_WORKSPACE;

  const int dp = sk::padded_dim(d);
  const ForwardLayout L = forward_layout(&Xr, &Yr);
  char* base = static_cast<char*>(ws);
  float* incx = reinterpret_cast<float*>(base + L.incx) + sk::kStreamPad * dp;
  float* incy = reinterpret_cast<float*>(base + L.incy) + sk::kStreamPad * dp;
  sk::PathPlan px{reinterpret_cast<int32_t*>(base + L.planx_n),
                  reinterpret_cast<int64_t*>(base + L.planx_start)};
  sk::PathPlan py{reinterpret_cast<int32_t*>(base + L.plany_n),
                  reinterpret_cast<int64_t*>(base + L.plany_start)};
  const sk::Batch bx = to_batch(X), by = to_batch(Y);
  const float scale = ldexpf(1.0f, -(2 * lam + 1));
  if (X->offsets && sk::launch_plan(bx, px, st) != hipSuccess) return SK_ERR_HIP;
  if (Y->offsets && sk::launch_plan(by, py, st) != hipSuccess) return SK_ERR_HIP;
  if (sk::launch_increments_xy(bx, X->offsets ? &px : nullptr, scale, by,
                               Y->offsets ? &py : nullptr, 1.0f, dp, incx, incy, st, sk::kRoundNone,
                               o.rep) != hipSuccess)
    return SK_ERR_HIP;
  if (X->offsets && sk::launch_scale_plan(px, X->n_paths, o.rep, st) != hipSuccess)
    return SK_ERR_HIP;
  if (Y->offsets && sk::launch_scale_plan(py, Y->n_paths, o.rep, st) != hipSuccess)
    return SK_ERR_HIP;

  int32_t* counts = reinterpret_cast<int32_t*>(base + P.counts);
  int32_t* order = nullptr;
  if (ragged) {
    // one task per pair, costliest first (the ordering only steers scheduling)
    order = reinterpret_cast<int32_t*>(base + P.order);
    sk::PairPlanArgs pp{};
    pp.x_n = X->offsets ? px.n : nullptr;
    pp.x_len = Xr.len;
    pp.y_n = Y->offsets ? py.n : nullptr;
    pp.y_len = Yr.len;
    pp.npairs = (int32_t)P.n_tasks;
    pp.gram_ny = Y->n_paths;
    pp.lam = lam;
    pp.rows_lo = 0;  // one class
    pp.rows_hi = sk::kGradRows;
    pp.order = order;
    pp.counts = counts;
    pp.counters = counts + 2;
    if (sk::launch_pair_plan(pp, st) != hipSuccess) return SK_ERR_HIP;
  }

  sk::GradArgs ga{};
  ga.incx = incx;
  ga.incy = incy;
  ga.x_n = X->offsets ? px.n : nullptr;
  ga.x_start = X->offsets ? px.start : nullptr;
  ga.y_n = Y->offsets ? py.n : nullptr;
  ga.y_start = Y->offsets ? py.start : nullptr;
  ga.x_len = Xr.len;
  ga.y_len = Yr.len;
  ga.nx = X->n_paths;
  ga.ny = Y->n_paths;
  ga.mode = sym ? 2 : 1;
  ga.no_diag = (flags & SK_NO_DIAG) ? 1 : 0;
  ga.run = (int32_t)P.run;
  ga.runs_per_row = P.runs_per_row;
  ga.n_tasks = (int32_t)P.n_tasks;
  ga.order = order;
  ga.counter = counts + 4;
  ga.dK = dK;
  ga.K = K;
  ga.scratch = reinterpret_cast<double*>(base + P.scratch);
  ga.slot_stride = P.slot_stride;
  ga.nb_max = P.nb_max;
  ga.nseg_max = P.nseg_max;
  ga.cols_max = P.cols_max;
  ga.part_x = reinterpret_cast<double*>(base + P.partx);
  // the y-side sums only when a y gradient is asked for (the y batch's, or
  // the second argument of a symmetric Gram's pairs)
  const bool ys = sym || dY != nullptr;
  ga.part_y = ys ? reinterpret_cast<double*>(base + P.party) : nullptr;
  ga.mrows = P.mrows;
  ga.nrows = P.nrows;
  if (sk::launch_grad(ga, lam, d, ys, P.slots, st) != hipSuccess) return SK_ERR_HIP;

  // the parts of a refined increment are the increment over rep: their
  // gradients sum, times 1 / rep, to the increment's
  const double inv_rep = 1.0 / (double)o.rep;
  auto points = [&](const sk_paths* B, const sk::PathPlan& plan, bool x_side, float* out,
                    bool acc) -> hipError_t {
    sk::GradPointArgs g{};
    g.part_x = x_side ? ga.part_x : nullptr;
    g.runs_per_row = P.runs_per_row;
    g.mrows = P.mrows;
    g.part_y = (!x_side || sym) ? ga.part_y : nullptr;
    g.py_rows = X->n_paths;
    g.py_ld = Y->n_paths;
    g.nrows = P.nrows;
    g.col_upper = sym ? 1 : 0;
    g.xscale = (double)scale * inv_rep;
    g.yscale = inv_rep;
    g.rep = o.rep;
    g.offsets = B->offsets;
    g.plan_n = B->offsets ? plan.n : nullptr;
    g.n_paths = B->n_paths;
    g.len = B->len;
    g.d = d;
    g.rows_bound = B->n_paths * (int64_t)B->len;
    g.accumulate = acc ? 1 : 0;
    g.out = out;
    return sk::launch_grad_points(g, st);
  };
  if (dX && points(X, px, true, dX, accumulate) != hipSuccess) return SK_ERR_HIP;
  if (dY && points(Y, py, false, dY, false) != hipSuccess) return SK_ERR_HIP;
  return SK_OK;
}

sk_status sigkernel_gram_backward(const sk_paths* X, const sk_paths* Y, int32_t dyadic_order,
                                  uint32_t flags, const float* dK, float* dX, float* dY, void* ws,
                                  size_t ws_bytes, void* stream) {
  return gram_backward(X, Y, dyadic_order, flags, dK, dX, dY, nullptr, false, ws, ws_bytes,
                       stream);
}

// ---- learned corrector ----------------------------------------------------
int64_t sigkernel_corrector_param_count(void) { return sk::corr::kParams; }
int64_t sigkernel_corrector_act_elems(void) { return sk::corr::kActFloats; }

sk_status sigkernel_corrector_features(const sk_paths* X, const sk_paths* Y, const float* norm,
                                       uint16_t* feats, float* k0, void* ws, size_t ws_bytes,
                                       void* stream) {
  if (sk_status c = check_corrector_batches(X, Y)) return c;
  if (X->n_paths == 0) return SK_OK;
  if (!feats || !k0) return SK_ERR_NULL;
  if (!ws || ws_bytes < forward_ws(X, Y)) return SK_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  sk::corr::FeatArgs fa{};
  float *incx, *incy;
  if (sk_status c = corrector_increments(X, Y, static_cast<char*>(ws), &incx, &incy, st)) return c;
  fa.incx = incx;
  fa.incy = incy;
  fa.m = X->len - 1;
  fa.n = Y->len - 1;
  fa.npairs = X->n_paths;
  fa.norm = norm;
  fa.feats = reinterpret_cast<sk::corr::bf16*>(feats);
  fa.k0 = k0;
  return sk::corr::launch_features(fa, X->dim, st) == hipSuccess ? SK_OK : SK_ERR_HIP;
}

sk_status sigkernel_corrector_forward(const float* params, const uint16_t* feats, int64_t n,
                                      uint16_t* acts, float* y, void* stream) {
  if (n < 0) return SK_ERR_SHAPE;
  if (n == 0) return SK_OK;
  if (!params || !feats || !acts || !y) return SK_ERR_NULL;
  return corrector_forward(params, reinterpret_cast<const sk::corr::bf16*>(feats), n,
                           reinterpret_cast<sk::corr::bf16*>(acts), y,
                           static_cast<hipStream_t>(stream));
}

sk_status sigkernel_corrector_backward(const float* params, const uint16_t* feats_bits,
                                       const uint16_t* acts_bits, const float* dy, int64_t n,
                                       float* grads, void* ws, size_t ws_bytes, void* stream) {
  using namespace sk::corr;
  const bf16* feats = reinterpret_cast<const bf16*>(feats_bits);
  const bf16* acts = reinterpret_cast<const bf16*>(acts_bits);
  if (n < 0) return SK_ERR_SHAPE;
  if (!params || !grads || (n > 0 && (!feats || !acts || !dy))) return SK_ERR_NULL;
  const size_t need = corrector_bwd_ws(n);
  if (!ws || ws_bytes < need) return SK_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const size_t act_bytes = align256((size_t)n * kFeatFloats * sizeof(float));
  float* dA = reinterpret_cast<float*>(base);
  float* dB = reinterpret_cast<float*>(base + act_bytes);
  float* partial = reinterpret_cast<float*>(base + 2 * act_bytes);
  if (launch_head_bwd(dy, acts + act_offset(3) * n, params + kHeadOffset, n, dA,
                      grads + kHeadOffset, st) != hipSuccess)
    return SK_ERR_HIP;
  for (int l = kLayers - 1; l >= 0; --l) {
    const DwPlan P = dw_plan(l, n);
    ConvBwdArgs a{};
    a.in = l == 0 ? feats : acts + act_offset(l - 1) * n;
    a.w = params + param_offset(l);
    a.out = acts + act_offset(l) * n;
    a.dout = dA;
    a.din = dB;
    a.partial = partial;
    a.n = n;
    a.nblocks = P.nblocks;
    a.per_block = P.per_block;
    if (launch_conv_dw(l, a, grads + param_offset(l), st) != hipSuccess) return SK_ERR_HIP;
    if (l > 0) {
      if (launch_conv_dx(l, a, st) != hipSuccess) return SK_ERR_HIP;
      float* t = dA;
      dA = dB;
      dB = t;
    }
  }
  return SK_OK;
}

sk_status sigkernel_corrector_loss(const float* y, const float* k_target, const float* k0,
                                   const float* target_norm, int64_t n, float* loss, float* dy,
                                   void* stream) {
  if (n < 1) return SK_ERR_SHAPE;
  if (!y || !k_target || !k0 || !target_norm || !loss || !dy) return SK_ERR_NULL;
  return sk::corr::launch_loss(y, k_target, k0, target_norm, n, loss, dy,
                               static_cast<hipStream_t>(stream)) == hipSuccess
             ? SK_OK
             : SK_ERR_HIP;
}

sk_status sigkernel_adam_step(float* params, const float* grads, float* m, float* v, int64_t n,
                              int32_t* step, float lr, float beta1, float beta2, float eps,
                              void* stream) {
  if (n < 0) return SK_ERR_SHAPE;
  if (!step || (n > 0 && (!params || !grads || !m || !v))) return SK_ERR_NULL;
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f))
    return SK_ERR_FLAGS;
  return sk::corr::launch_adam(params, grads, m, v, n, step, lr, beta1, beta2, eps,
                               static_cast<hipStream_t>(stream)) == hipSuccess
             ? SK_OK
             : SK_ERR_HIP;
}

sk_status sigkernel_channel_stats(const void* x, int32_t x_dtype, const float* sub, int64_t rows,
                                  int32_t channels, float* mean, float* rstd, void* ws,
                                  size_t ws_bytes, void* stream) {
  if (x_dtype != 0 && x_dtype != 1) return SK_ERR_FLAGS;
  if (rows < 1 || channels < 1 || channels > sk::corr::kMaxStatChannels) return SK_ERR_SHAPE;
  if (!x || !mean || !rstd) return SK_ERR_NULL;
  if (!ws || ws_bytes < sk::corr::kStatsWorkspaceBytes) return SK_ERR_WORKSPACE;
  return sk::corr::launch_channel_stats(x, x_dtype == 1, sub, rows, channels, mean, rstd,
                                        static_cast<double*>(ws),
                                        static_cast<hipStream_t>(stream)) == hipSuccess
             ? SK_OK
             : SK_ERR_HIP;
}

sk_status sigkernel_corrector_predict(const sk_paths* X, const sk_paths* Y, int32_t fallback_order,
                                      const float* params, const float* norm,
                                      const float* target_norm, float kappa, float tol, float* out,
                                      float* err, int32_t* fallback, void* ws, size_t ws_bytes,
                                      void* stream) {
  if (sk_status c = check_corrector_batches(X, Y)) return c;
  if (fallback_order < 0 || fallback_order > kMaxKernelOrder) return SK_ERR_ORDER;
  if (!(kappa >= 0.0f) || !(tol >= 0.0f)) return SK_ERR_FLAGS;
  const int64_t n = X->n_paths;
  if (n == 0) return SK_OK;
  if (!params || !norm || !target_norm || !out) return SK_ERR_NULL;
  if (n > INT32_MAX) return SK_ERR_UNSUPPORTED;
  const PredictLayout L = predict_layout(X, Y, fallback_order);
  if (L.pl.rows_hi == 0) return SK_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < L.total) return SK_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  float *incx, *incy;
  if (sk_status c = corrector_increments(X, Y, base, &incx, &incy, st)) return c;
  sk::corr::bf16* wb = reinterpret_cast<sk::corr::bf16*>(base + L.wb);
  sk::corr::bf16* feats = reinterpret_cast<sk::corr::bf16*>(base + L.feats);
  float* y = reinterpret_cast<float*>(base + L.y);
  float* k0 = reinterpret_cast<float*>(base + L.k0);
  sk::corr::FeatArgs fa{};
  fa.incx = incx;
  fa.incy = incy;
  fa.m = X->len - 1;
  fa.n = Y->len - 1;
  fa.npairs = n;
  fa.norm = norm;
  fa.feats = feats;
  fa.k0 = k0;
  if (sk::corr::launch_features(fa, X->dim, st) != hipSuccess) return SK_ERR_HIP;
  // weights to bf16 once per call, then the whole network per pair on chip
  if (sk::corr::launch_to_bf16(params, sk::corr::kHeadOffset, wb, st) != hipSuccess)
    return SK_ERR_HIP;
  sk::corr::NetArgs na{};
  na.feats = feats;
  na.wb = wb;
  na.params = params;
  na.n = n;
  na.y = y;
  if (sk::corr::launch_net_fused(na, st) != hipSuccess) return SK_ERR_HIP;
  int32_t* order = reinterpret_cast<int32_t*>(base + L.pl.order);
  int32_t* counts = reinterpret_cast<int32_t*>(base + L.pl.counts);
  sk::corr::DecideArgs da{};
  da.k0 = k0;
  da.y = y;
  da.tnorm = target_norm;
  da.kappa = kappa;
  da.tol = tol;
  da.n = n;
  da.out = out;
  da.err = err;
  da.fallback = fallback;
  da.order = order;
  da.count = counts;
  if (sk::corr::launch_decide(da, st) != hipSuccess) return SK_ERR_HIP;
  // the plain solve at the fallback order for the compacted pairs only: the
  // persistent pair kernel reads their number from the device
  sk::PairArgs a{};
  a.incx = incx;
  a.incy = incy;
  a.x_len = X->len;
  a.y_len = Y->len;
  a.scale = ldexp(1.0, -(2 * fallback_order + 1));
  a.order = order;
  a.count = counts;
  a.counter = counts + 2;
  a.bandbuf = reinterpret_cast<double*>(base + L.pl.bands);
  a.band_stride = L.pl.band_stride;
  a.out = out;
  const hipError_t e =
      sk::launch_pairs(a, fallback_order, L.pl.rows_hi, X->dim, L.pl.slots, st, 0);
  if (e == hipErrorInvalidValue) return SK_ERR_UNSUPPORTED;
  return e == hipSuccess ? SK_OK : SK_ERR_HIP;
}

}  // extern "C"
