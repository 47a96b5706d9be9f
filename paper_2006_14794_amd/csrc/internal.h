// Internal declarations shared by the HIP translation units of libsigkernel.
// Not part of the public ABI (see include/sigkernel.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

// Row pitch (floats) of the padded increment arrays: channels rounded up to a
// multiple of 4 so that one row is a whole number of 16-byte loads.
inline int padded_dim(int d) { return (d + 3) & ~3; }

// A batch as the kernels see it: either uniform (offsets == nullptr, every path
// has `len` points) or ragged (device offsets, `len` an upper bound).
struct Batch {
  const float* points;
  const int64_t* offsets;
  int64_t n_paths;
  int32_t len;
  int32_t dim;
};

// Per-path layout of the dense increment array of a ragged batch: n[k] is the
// number of increments of path k (points - 1), or -1 when the path breaks the
// batch contract; start[k] is its first row.  Rows of consecutive valid paths
// are contiguous (start is the exclusive prefix sum of max(n, 0)).
// Uniform batches use the closed form n = len - 1, start = k (len - 1).
struct PathPlan {
  int32_t* n;
  int64_t* start;
};

hipError_t launch_plan(const Batch& b, PathPlan plan, hipStream_t stream);

// p[0 .. n) = v (a kernel rather than a memset node, so that captured graphs
// replay it like any other launch)
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t stream);

// Dense padded increments of both batches of a call, in one launch: row
// start[k] + p of a batch's buffer holds scale * (x_{p+1} - x_p), p < n[k],
// zero-padded to `dpad` channels (scalex for X, scaley for Y; powers of two).
// With rounding kRoundBf16 / kRoundF16 each increment is first rounded to
// that 16-bit format (the inner products then see 16-bit inputs, float32
// sums).  With rep > 1 (a power of two) every increment fills rep
// consecutive rows, each scale * (x_{p+1} - x_p) / rep: the batch refined rep
// times, exactly (rows start[k] rep + p rep + j).
enum { kRoundNone = 0, kRoundBf16 = 1, kRoundF16 = 2 };
hipError_t launch_increments_xy(const Batch& bx, const PathPlan* planx, float scalex,
                                const Batch& by, const PathPlan* plany, float scaley, int dpad,
                                float* incx, float* incy, hipStream_t stream,
                                int rounding = kRoundNone, int rep = 1);
// The plan of a batch refined rep times: n[k] -> n[k] rep (for n[k] > 0),
// start[k] -> start[k] rep.  Run after the increments have read the plan.
hipError_t launch_scale_plan(PathPlan plan, int64_t n_paths, int rep, hipStream_t stream);

// Dense padded node rows (the points themselves): path k occupies rows
// [start[k] + k, start[k] + k + n[k] + 1) of a ragged batch, [k len, (k + 1)
// len) of a uniform one; channels beyond d are zero.  Paths with n[k] < 0 are
// skipped.
hipError_t launch_nodes(const Batch& b, const PathPlan* plan, int dpad, float* nodes,
                        hipStream_t stream);

}  // namespace sk

#include "grad_args.h"
#include "sweep_args.h"

namespace sk {

// Largest number of fine rows per lane of the one-wave sweep.
constexpr int kMaxRowsPerLane = 32;

// Rows per lane for `fine_rows` rows on a 64-lane wave (0 if none is compiled).
int choose_rows_per_lane(int64_t fine_rows, int lam, int dim);

// Returns hipErrorInvalidValue when no compiled configuration covers the shape.
// waves_per_block: 1, 2 or 4 one-wave sweeps per workgroup (0: 4).
hipError_t launch_sweep(const SweepArgs& a, int lam, int rows_per_lane, int dim,
                        hipStream_t stream, int waves_per_block = 0);
// The sweep of the Gaussian-lifted kernel (lifted_kernel.h): incx / incy hold
// node rows, lift_inv and lift_scale are set.
hipError_t launch_lifted(const SweepArgs& a, int lam, int rows_per_lane, int dim,
                         hipStream_t stream, int waves_per_block = 0);
// Rows per lane of a compiled sweep kernel of the given kind for `fine_rows`
// rows (0 if none).
int choose_rows_for(int kind, int64_t fine_rows, int lam, int dim);

// Gradient of weighted Gram entries (grad_kernel.h, grad.hip): persistent
// waves over the tasks of a GradArgs, `slots` of them, each with its own
// scratch slot (the queue counter is zeroed by a kernel first); ys: form the
// y-side gradients (a.part_y), else the x side only.
hipError_t launch_grad(const GradArgs& a, int lam, int dim, bool ys, int64_t slots,
                       hipStream_t stream);
bool grad_supported(int lam, int dim);

// Point gradients of one batch from a gradient launch's increment gradients
// (grad.hip): see grad_points_kernel.
struct GradPointArgs {
  const double* part_x;     // [n_paths][runs_per_row][mrows][d] or nullptr
  int64_t runs_per_row;
  int32_t mrows;
  const double* part_y;     // [py_rows][py_ld][nrows][d] or nullptr; path k is column k
  int64_t py_rows, py_ld;
  int32_t nrows;
  int32_t col_upper;        // symmetric Gram: rows a <= k only
  double xscale, yscale;
  int32_t rep;
  const int64_t* offsets;   // ragged batch (device) or nullptr
  const int32_t* plan_n;    // ragged: increments per path (-1: broken)
  int64_t n_paths;
  int32_t len;              // uniform: points per path
  int32_t d;
  int64_t rows_bound;       // point rows covered by the launch (uniform: all; ragged: a bound)
  int32_t accumulate;       // 1: out += the gradient; 0: out = the gradient
  float* out;               // [rows][d]
};
hipError_t launch_grad_points(const GradPointArgs& a, hipStream_t stream);

hipError_t launch_mmd2_reduce(const float* kxx, int64_t n, const float* kyy, int64_t m,
                              const float* kxy, float* out, hipStream_t stream);
hipError_t launch_add(float* dst, const float* src, int64_t n, hipStream_t stream);
hipError_t launch_zero_diag(float* k, int64_t n, hipStream_t stream);  // k[i][i] = 0, k is n x n

// Independent pairs, persistent and length-sorted (pair_kernel.h, pairs.hip).
struct PairArgs {
  const float* incx;        // dense increments of both batches, not scaled
  const float* incy;
  const int32_t* x_n;       // ragged plans (nullptr for a uniform batch)
  const int64_t* x_start;
  const int32_t* y_n;
  const int64_t* y_start;
  int32_t x_len, y_len;
  double scale;             // 2^-(2 lam + 1)
  const int32_t* order;     // pair ids, long class first, each class longest first
  const int32_t* order_base;  // device: offset of this class in `order` (nullptr: 0)
  const int32_t* count;     // device: pairs in this class
  int32_t* counter;         // device queue head (zeroed by the plan kernel)
  double* bandbuf;          // per wave slot: band_stride doubles
  int64_t band_stride;
  float* out;               // out[pid]
  int64_t gram_ny;          // 0: pair pid is (x_pid, y_pid); else (x_{pid / gram_ny}, y_{pid % gram_ny})
  int32_t implicit;         // 1: the implicit scheme's cell factor (2 + h) / (2 - h)
  // pipelined bands (pair_band_kernel): band tasks of the class in `order`
  const int32_t* task_base; // device [count + 1]: first task of each pair, total at [count]
  int32_t* task_counter;    // device queue head over the tasks
  double* tbuf;             // per task: tstride doubles (its bottom row), sentinel-filled
  int64_t tstride;
};

struct PairPlanArgs {
  const int32_t* x_n;
  int32_t x_len;
  const int32_t* y_n;
  int32_t y_len;
  int32_t npairs, lam, rows_lo, rows_hi;
  int64_t gram_ny;          // as in PairArgs
  int32_t* order;           // [npairs]: long-row class first
  int32_t* counts;          // [2]: long class, short class
  int32_t* counters;        // [2]
};

hipError_t launch_pair_plan(const PairPlanArgs& p, hipStream_t stream);
// Band tasks of the long class (order[0 .. counts[0])): task_base[k] = sum of
// the band counts (rows / (64 R), rounded up) of the pairs before k, the total
// at task_base[counts[0]]; zeroes *task_counter.  One workgroup, any count.
hipError_t launch_band_plan(const PairPlanArgs& p, int rows_per_lane, int32_t* task_base,
                            int32_t* task_counter, hipStream_t stream);
// The pipelined band kernel over those tasks (persistent, like launch_pairs),
// compiled only at the largest rows per lane that fits.  fit_top: each pair's
// top band takes R/4, R/2 or R rows per lane by its rows; else every band
// takes R.
hipError_t launch_pair_bands(const PairArgs& a, int lam, int rows_per_lane, int dim,
                             int64_t max_waves, hipStream_t stream, int blocks_per_cu,
                             bool fit_top);
// p[0 .. n) = v (64-bit pattern), as a kernel
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t stream);
// v (kBandSlotSentinel) into the slots the band tasks of a band plan will
// write: the first (columns << lam) doubles of every task but each pair's
// last, tasks below t_max only (reads the plan on the device).
hipError_t launch_fill_task_slots(uint64_t* tbuf, const PairPlanArgs& p,
                                  const int32_t* task_base, int64_t stride, int64_t t_max,
                                  uint64_t v, hipStream_t stream);
// The sentinel of the pipelined bands' slots (a signalling NaN arithmetic never yields).
constexpr uint64_t kBandSlotSentinel = 0x7FF40000DEAD5EB0ull;
// Persistent launch: min(max_waves, blocks_per_cu 4-wave workgroups per CU)
// wavefronts; blocks_per_cu 0 takes the occupancy limit.  Waves never wait on
// one another, so any count is correct; it only changes the balance.
hipError_t launch_pairs(const PairArgs& a, int lam, int rows_per_lane, int dim,
                        int64_t max_waves, hipStream_t stream, int blocks_per_cu = 0);

// Coefficient-driven sweep for any number of channels (coef.hip).
// coef_kernel writes the pre-scaled coarse coefficients of the launched
// waves in the order coef_sweep_kernel reads them; see coef.hip.
struct CoefArgs {
  const float* incx;        // dense unscaled increments (not refined)
  const float* incy;
  const int32_t* x_n;       // plans of the batch as swept (refined: n rep, start rep)
  const int64_t* x_start;
  const int32_t* y_n;
  const int64_t* y_start;
  int32_t x_len, y_len;     // points per path as swept (refined)
  int64_t nx, ny;
  int32_t mode;             // as SweepArgs
  int32_t run;
  int64_t runs_per_row;
  int64_t wave0, n_waves;   // waves of this launch
  int32_t d, dpad;
  int32_t R, lam, rep;      // the consuming sweep's rows per lane and order; refinement
  float scale;              // 2^-(2 lam + 1) / rep^2
  float* coef;              // per launched wave: coef_stride floats
  int64_t coef_stride;
};
// Rows per lane of the coefficient sweep (R >= 2^lam; 0 if none fits).
int coef_rows_per_lane(int64_t fine_rows, int lam);
// Floats of one wave's coefficient slots for a run of total_cols columns.
int64_t coef_wave_floats(int64_t total_cols, int R, int lam);
// max_m, max_n: unrefined increment counts (upper bounds) of the batches.
hipError_t launch_coef(const CoefArgs& a, int precision, int64_t max_m, int64_t max_n,
                       hipStream_t stream);
hipError_t launch_coef_sweep(const SweepArgs& a, int lam, int rows_per_lane, bool implicit,
                             hipStream_t stream, int waves_per_block = 0);

// Reduced measure by proximal gradient (reduce.hip): one workgroup.
constexpr int kMaxReduceN = 4096;
struct ReduceArgs {
  const float* K;           // [n][ld] Gram, row-major
  int64_t ld;
  const float* alpha;       // [n] weights of the measure
  int32_t n;
  double lam, step;         // penalty (fixed-penalty mode); step <= 0: automatic
  int32_t iters;            // iterations (per bisection round in support mode)
  int32_t support, rounds;  // support > 0: bisection on the penalty for this support size
  double* beta;             // [n] out
  double* loss;             // [iters + 1] out (fixed-penalty mode; nullable)
  double* lam_out;          // [1] out (support mode)
  double* step_out;         // [1] out, nullable
};
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t stream);

// Increment Gram of uniform batches.
struct GramArgs {
  const float* x;           // points [nx][x_len][d]
  const float* y;           // points [ny][y_len][d]
  int32_t x_len, y_len, d;
  int64_t nx, ny;
  int32_t gram;             // 1: every (a, b), pair index a ny + b; 0: pairs (x_k, y_k)
  float* g0;                // [pairs][x_len - 1][ld], columns < y_len - 1 written
  int64_t ld;               // row stride of g0 in floats, >= y_len - 1
};
// precision: kRoundNone (float32 inputs), kRoundBf16, kRoundF16
constexpr int kGramRowsMaxDim = 16;
hipError_t launch_gram_rows(const GramArgs& a, int precision, hipStream_t stream);
// The same on the matrix cores for kGramRowsMaxDim < d <= kGramMfmaMaxDim
// (gram_mfma.hip).
constexpr int kGramMfmaMaxDim = 64;
hipError_t launch_gram_mfma(const GramArgs& a, int precision, hipStream_t stream);

// Compiled sweep kernels by kind, dyadic order, rows per lane and channels
// (nullptr when the configuration is not compiled).
enum { kKernelForward = 0, kKernelPair = 3, kKernelLifted = 4, kKernelForwardImplicit = 5,
       kKernelPairBand = 6, kKernelPairBandFull = 7 };
void* sweep_fn(int kind, int lam, int rows_per_lane, int dim);

}  // namespace sk
