// Independent pairs (x_k, y_k) of uneven lengths: the explicit scheme of
// Section 3.1, eq. (explicit_finite_diff), on P_lambda, one pair at a time per
// wavefront, with a persistent grid that takes pairs from a length-sorted
// device queue (longest first).
//
// Per pair the shorter path is put on the rows (the scheme is symmetric in
// its two arguments), so the wave streams the longer path's columns.  When
// the rows exceed one wave's strips (64 lanes x R), the grid is processed in
// row bands from the top: lane 63 of band b writes its bottom row (one
// double per fine column) to a per-wave buffer, and lane 0 of band b+1
// reads it as its upper neighbour instead of the boundary value 1.  Within a
// band the mapping is the forward sweep's: lane strips, one coarse column per
// step, DPP wave_shr:1 between lanes, coarse coefficients on the fly.
#pragma once
#include <math.h>

#include "internal.h"
#include "sweep_fwd_kernel.h"

namespace sk {
namespace pairk {

using fwd::first_row;
using fwd::from_prev_lane;
using fwd::load_row;
using fwd::n_inc;

template <int R, int LAM, int D>
__global__ __launch_bounds__(256) void pair_kernel(const PairArgs a) {
  constexpr int DP = (D + 3) & ~3;
  constexpr int S = 1 << LAM;
  constexpr int CR = (R >> LAM) > 0 ? (R >> LAM) : 1;

  const int lane = threadIdx.x & 63;
  const int64_t slot = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  double* __restrict__ bb = a.bandbuf + slot * a.band_stride;
  const int32_t count = *a.count;
  const int32_t* __restrict__ order = a.order + (a.order_base ? *a.order_base : 0);

  for (;;) {
    // next pair of this class (one vector atomic per wave)
    int32_t k = 0;
    if (lane == 0) k = atomicAdd(a.counter, 1);
    k = __builtin_amdgcn_readlane(k, 0);  // scalar: the task loop's control flow is uniform
    if (k >= count) break;
    const int32_t pid = order[k];
    const int64_t ix = a.gram_ny ? pid / a.gram_ny : pid;
    const int64_t iy = a.gram_ny ? pid - ix * a.gram_ny : pid;
    const int32_t mx = n_inc(a.x_n, a.x_len, ix), my = n_inc(a.y_n, a.y_len, iy);
    if (mx < 0 || my < 0 || mx == 0 || my == 0) {
      // every lane stores the same value: no lane-dependent branch may precede
      // a back-edge of this loop.  With a lane-0-only store here the compiler
      // sent lanes 1..63 straight from that store back to the queue-index
      // broadcast with the atomic skipped (they cannot be lane 0), so they ran
      // a second loop header without lane 0 and read lane 0's stale index:
      // part of the wave swept the previous task again.
      a.out[pid] = (mx < 0 || my < 0) ? __builtin_nanf("") : 1.0f;
      continue;
    }
    const bool swap = mx > my;
    const int32_t m = swap ? my : mx, n = swap ? mx : my;
    const float* __restrict__ rinc =
        swap ? a.incy + first_row(a.y_start, a.y_len, iy) * DP
             : a.incx + first_row(a.x_start, a.x_len, ix) * DP;
    const float* __restrict__ cinc =
        swap ? a.incx + first_row(a.x_start, a.x_len, ix) * DP
             : a.incy + first_row(a.y_start, a.y_len, iy) * DP;
    const int M = m << LAM;
    const int nb = (M + 64 * R - 1) / (64 * R);
    const int off = nb * 64 * R - M;  // virtual rows above row 0, in the top band
    const int32_t nsteps = (int32_t)sweep_steps(n);
    double result = 1.0;

    for (int band = 0; band < nb; ++band) {
      // the previous band's bottom row (written by lane 63) must be visible
      if (band > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const bool top = (band == 0), last = (band == nb - 1);
      const int row0 = (band * 64 + lane) * R - off;
      const int p0 = row0 >> LAM;
      float dx[CR][D];
#pragma unroll
      for (int c = 0; c < CR; ++c) {
        float t[DP];
        if (p0 + c >= 0 && p0 + c < m) {
          load_row<DP>(rinc + (int64_t)(p0 + c) * DP, t);
        } else {
#pragma unroll
          for (int q = 0; q < DP; ++q) t[q] = 0.0f;
        }
#pragma unroll
        for (int q = 0; q < D; ++q) dx[c][q] = t[q];
      }

      double u[R];
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = 1.0;
      double pub[S];
#pragma unroll
      for (int cc = 0; cc < S; ++cc) pub[cc] = 1.0;
      double up_last = 1.0;
      // The top band's first off / R lanes hold only virtual rows: zero
      // increments and the boundary value 1 whatever the step, so the band
      // starts at the first real lane's first column (lane l at column
      // t0 - l), saving those steps of pipeline fill.
      const int32_t t0 = top ? off / R : 0;
      int32_t g = t0 - lane;
      const float* __restrict__ yp = cinc + (int64_t)g * DP;
      // upper neighbours of lane 0: the boundary (top band) or the band above
      auto bnd_load = [&](int32_t t, double (&v)[S]) {
#pragma unroll
        for (int cc = 0; cc < S; ++cc) v[cc] = top ? 1.0 : bb[(int64_t)t * S + cc];
      };

      float dyA[DP], dyB[DP], dyC[DP];
      double bA[S], bB[S], bC[S];
      load_row<DP>(yp, dyA);
      load_row<DP>(yp + DP, dyB);
      bnd_load(0, bA);
      bnd_load(1, bB);

      auto step = [&](int32_t t, float (&dy)[DP], float (&refill)[DP], double (&bv)[S],
                      double (&brefill)[S]) {
        load_row<DP>(yp + 2 * DP, refill);
        bnd_load(t + 2, brefill);
        float h32[CR];
#pragma unroll
        for (int c = 0; c < CR; ++c) {
          float s = 0.0f;
#pragma unroll
          for (int q = 0; q < D; ++q) s = __builtin_fmaf(dx[c][q], dy[q], s);
          h32[c] = s;
        }
        double up[S];
#pragma unroll
        for (int cc = 0; cc < S; ++cc) up[cc] = from_prev_lane(pub[cc], bv[cc]);

        if ((uint32_t)g < (uint32_t)n) {
          double gk[CR];
          if (a.implicit) {
            double h[CR];
#pragma unroll
            for (int c = 0; c < CR; ++c) h[c] = (double)h32[c] * a.scale;  // exact: 2^-k
            fwd::implicit_factors<CR>(h, gk);
          } else {
#pragma unroll
            for (int c = 0; c < CR; ++c) gk[c] = __builtin_fma((double)h32[c], a.scale, 1.0);
          }
          double v[R][S];
#pragma unroll
          for (int dgl = 0; dgl < R + S - 1; ++dgl) {
#pragma unroll
            for (int cc = 0; cc < S; ++cc) {
              const int r = dgl - cc;
              if (r < 0 || r >= R) continue;
              const double A = (cc == 0) ? u[r] : v[r][cc - 1];
              const double B = (r == 0) ? up[cc] : v[r - 1][cc];
              const double C = (r == 0) ? ((cc == 0) ? up_last : up[cc - 1])
                                        : ((cc == 0) ? u[r - 1] : v[r - 1][cc - 1]);
              v[r][cc] = __builtin_fma(gk[(R >= S) ? (r >> LAM) : 0], A + B, -C);
            }
          }
#pragma unroll
          for (int r = 0; r < R; ++r) u[r] = v[r][S - 1];
#pragma unroll
          for (int cc = 0; cc < S; ++cc) pub[cc] = v[R - 1][cc];
          up_last = up[S - 1];
          if (lane == 63) {
            if (!last) {
#pragma unroll
              for (int cc = 0; cc < S; ++cc) bb[(int64_t)g * S + cc] = pub[cc];
            } else if (g == n - 1) {
              result = u[R - 1];
            }
          }
        }
        ++g;
        yp += DP;
      };

      // (from t0 the last iteration may run up to two steps past nsteps:
      // inactive for every lane, rows within the stream padding)
      for (int32_t t = t0; t < nsteps; t += 3) {
        step(t, dyA, dyC, bA, bC);
        step(t + 1, dyB, dyA, bB, bA);
        step(t + 2, dyC, dyB, bC, bB);
      }
      if (!last) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    // lane 63 holds the value; every lane stores it (no lane-dependent branch
    // before the back-edge, see above)
    a.out[pid] = (float)fwd::lane_value(result, 63);
  }
}

// Pipelined row bands.  The queue holds band tasks in
// pair order, band by band (task_base[k] = first task of the k-th pair of the
// class); a wave takes one task, i.e. one band of one pair, so all bands of a
// pair are swept at the same time, each one lagging the band above by a
// little over one wave's pipeline fill.
//   * Band b writes its bottom row (one double per fine column) into the
//     task's own slot buffer with agent-scope atomic stores, once per value.
//   * The slot buffers are filled with a signalling-NaN sentinel beforehand
//     (arithmetic never produces it), so a value is ready when it differs from
//     the sentinel: band b+1 polls the slots of task tau - 1 with agent-scope
//     atomic loads, kChunk coarse columns at a time, one chunk ahead, staging
//     them in LDS for lane 0.
//   * A task only waits on the task taken just before it (same pair), whose
//     wave is running, so the chain always advances; the wait is bounded all
//     the same, and on expiry the missing values become NaN, which flows to
//     the pair's output and releases the bands below.
constexpr int kChunk = 16;         // coarse columns staged per chunk
constexpr int kSpinMax = 1 << 18;  // polls per value before giving up

__device__ __forceinline__ bool is_sentinel(double v) {
  return (uint64_t)__double_as_longlong(v) == kBandSlotSentinel;
}

// One band task: the band's lanes hold RT fine rows each, lane l's first row
// being row0 (rows above row 0 are virtual: zero increments, value 1).  top:
// the band's upper neighbours are the boundary; last: it ends the pair and
// lane 63 writes the pair's value.
template <int RT, int LAM, int D>
__device__ __forceinline__ void band_sweep(const PairArgs& a,
                                           double (&stage)[2][kChunk << LAM], int lane,
                                           int32_t tau, bool top, bool last, int row0,
                                           int32_t pid, int32_t m, int32_t n,
                                           const float* __restrict__ rinc,
                                           const float* __restrict__ cinc) {
  constexpr int DP = (D + 3) & ~3;
  constexpr int S = 1 << LAM;
  constexpr int CR = (RT >> LAM) > 0 ? (RT >> LAM) : 1;
  constexpr int CHS = kChunk * S;        // doubles per chunk
  constexpr int PER = (CHS + 63) / 64;   // doubles per lane per chunk
  const int32_t nsteps = (int32_t)sweep_steps(n);
  double* __restrict__ own = a.tbuf + (int64_t)tau * a.tstride;
  const double* __restrict__ above = a.tbuf + (int64_t)(tau - 1) * a.tstride;

  const int p0 = row0 >> LAM;
  float dx[CR][D];
#pragma unroll
  for (int c = 0; c < CR; ++c) {
    float t[DP];
    if (p0 + c >= 0 && p0 + c < m) {
      load_row<DP>(rinc + (int64_t)(p0 + c) * DP, t);
    } else {
#pragma unroll
      for (int q = 0; q < DP; ++q) t[q] = 0.0f;
    }
#pragma unroll
    for (int q = 0; q < D; ++q) dx[c][q] = t[q];
  }

  // upper neighbours of lane 0, staged chunk by chunk from the band above
  bool failed = false;  // wave-uniform
  double pf[PER];
  auto fetch = [&](int32_t chunk) {  // issue the loads of a chunk
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = lane + 64 * i;
      const int32_t col = chunk * kChunk + e / S;
      pf[i] = 0.0;
      if (!top && e < CHS && col < n)
        pf[i] = __hip_atomic_load(above + (int64_t)col * S + (e % S), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  auto commit = [&](int32_t chunk) {  // wait for a chunk's values, then stage them
    bool missing = false;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = lane + 64 * i;
      const int32_t col = chunk * kChunk + e / S;
      double v = pf[i];
      if (!top && e < CHS && col < n) {
        int spins = 0;
        while (!failed && is_sentinel(v) && spins < kSpinMax) {
          ++spins;
          __builtin_amdgcn_s_sleep(2);
          v = __hip_atomic_load(above + (int64_t)col * S + (e % S), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
        }
        if (is_sentinel(v)) {
          v = __builtin_nan("");
          missing = true;
        }
      }
      if (e < CHS) stage[chunk & 1][e] = top ? 1.0 : v;
    }
    // a value that never came poisons the rest of this band (no more waits)
    failed = failed || __ballot(missing) != 0;
  };

  double u[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) u[r] = 1.0;
  double pub[S];
#pragma unroll
  for (int cc = 0; cc < S; ++cc) pub[cc] = 1.0;
  double up_last = 1.0;
  int32_t g = -lane;
  const float* __restrict__ yp = cinc + (int64_t)g * DP;
  auto bnd_load = [&](int32_t t, double (&v)[S]) {
#pragma unroll
    for (int cc = 0; cc < S; ++cc) v[cc] = stage[(t / kChunk) & 1][(t % kChunk) * S + cc];
  };

  fetch(0);
  commit(0);
  fetch(1);
  float dyA[DP], dyB[DP], dyC[DP];
  double bA[S], bB[S], bC[S];
  load_row<DP>(yp, dyA);
  load_row<DP>(yp + DP, dyB);
  bnd_load(0, bA);
  bnd_load(1, bB);
  double result = 1.0;

  auto step = [&](int32_t t, float (&dy)[DP], float (&refill)[DP], double (&bv)[S],
                  double (&brefill)[S]) {
    load_row<DP>(yp + 2 * DP, refill);
    if ((t + 2) % kChunk == 0) {  // the next chunk is read from step t on
      const int32_t c = (t + 2) / kChunk;
      commit(c);
      fetch(c + 1);
    }
    bnd_load(t + 2, brefill);
    float h32[CR];
#pragma unroll
    for (int c = 0; c < CR; ++c) {
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < D; ++q) s = __builtin_fmaf(dx[c][q], dy[q], s);
      h32[c] = s;
    }
    double up[S];
#pragma unroll
    for (int cc = 0; cc < S; ++cc) up[cc] = from_prev_lane(pub[cc], bv[cc]);

    if ((uint32_t)g < (uint32_t)n) {
      double gk[CR];
      if (a.implicit) {
        double h[CR];
#pragma unroll
        for (int c = 0; c < CR; ++c) h[c] = (double)h32[c] * a.scale;  // exact: 2^-k
        fwd::implicit_factors<CR>(h, gk);
      } else {
#pragma unroll
        for (int c = 0; c < CR; ++c) gk[c] = __builtin_fma((double)h32[c], a.scale, 1.0);
      }
      double v[RT][S];
      float sv[1];
      fwd::cell_block<RT, LAM, CR, false>(v, sv, u, up, up_last, gk);
#pragma unroll
      for (int r = 0; r < RT; ++r) u[r] = v[r][S - 1];
#pragma unroll
      for (int cc = 0; cc < S; ++cc) pub[cc] = v[RT - 1][cc];
      up_last = up[S - 1];
      if (lane == 63) {
        if (!last) {
#pragma unroll
          for (int cc = 0; cc < S; ++cc)
            __hip_atomic_store(own + (int64_t)g * S + cc, pub[cc], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else if (g == n - 1) {
          result = u[RT - 1];
        }
      }
    }
    ++g;
    yp += DP;
  };

  for (int32_t t = 0; t < nsteps; t += 3) {
    step(t, dyA, dyC, bA, bC);
    step(t + 1, dyB, dyA, bB, bA);
    step(t + 2, dyC, dyB, bC, bB);
  }
  // lane 63 holds the value; every lane stores it (see pair_kernel)
  result = fwd::lane_value(result, 63);
  if (last) a.out[pid] = (float)result;
}

// Full bands hold R fine rows per lane (64 R rows).  The pair's rows are cut
// from the bottom, so only the top band is partial.  FIT_TOP: the top band
// takes the smallest of R/4, R/2 and R rows per lane that covers its rows,
// which saves the issue slots of lanes that would only hold virtual rows; the
// band plan counts the bands at R rows per lane, which this split keeps.
// Without FIT_TOP every band has R rows per lane: the kernel holds one sweep
// body, which the compiler schedules a little better (about 4% on a chain of
// bands), for batches whose top bands need all R rows anyway.
template <int R, int LAM, int D, bool FIT_TOP>
__global__ __launch_bounds__(256) void pair_band_kernel(const PairArgs a) {
  constexpr int DP = (D + 3) & ~3;
  __shared__ double stage[4][2][kChunk << LAM];

  const int lane = threadIdx.x & 63;
  const int wl = threadIdx.x >> 6;
  const int32_t count = *a.count;
  const int32_t* __restrict__ order = a.order;
  const int32_t total_tasks = a.task_base[count];

  for (;;) {
    int32_t tau = 0;
    if (lane == 0) tau = atomicAdd(a.task_counter, 1);
    tau = __builtin_amdgcn_readlane(tau, 0);  // scalar (see pair_kernel)
    if (tau >= total_tasks) break;
    // the pair of this task: the last k with task_base[k] <= tau
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (a.task_base[mid] <= tau) lo = mid; else hi = mid - 1;
    }
    const int32_t band = tau - a.task_base[lo];
    const int32_t pid = order[lo];
    const int64_t ix = a.gram_ny ? pid / a.gram_ny : pid;
    const int64_t iy = a.gram_ny ? pid - ix * a.gram_ny : pid;
    const int32_t mx = n_inc(a.x_n, a.x_len, ix), my = n_inc(a.y_n, a.y_len, iy);
    if (mx <= 0 || my <= 0) {  // one task for such a pair
      // every lane stores the same value (see pair_kernel)
      a.out[pid] = (mx < 0 || my < 0) ? __builtin_nanf("") : 1.0f;
      continue;
    }
    const bool swap = mx > my;
    const int32_t m = swap ? my : mx, n = swap ? mx : my;
    const float* __restrict__ rinc =
        swap ? a.incy + first_row(a.y_start, a.y_len, iy) * DP
             : a.incx + first_row(a.x_start, a.x_len, ix) * DP;
    const float* __restrict__ cinc =
        swap ? a.incx + first_row(a.x_start, a.x_len, ix) * DP
             : a.incy + first_row(a.y_start, a.y_len, iy) * DP;
    const int M = m << LAM;
    const int nb = (M + 64 * R - 1) / (64 * R);
    const int top_rows = M - (nb - 1) * 64 * R;  // 1 .. 64 R
    const bool last = band == nb - 1;
    // rows per lane of this band: R / 4, R / 2 or R (one if-else chain, no
    // continue after a sweep)
    const int quarter = R >= 4 ? R / 4 : R, half = R >= 2 ? R / 2 : R;
    const int rt = (!FIT_TOP || band > 0)      ? R
                   : 64 * quarter >= top_rows ? quarter
                   : 64 * half >= top_rows    ? half
                                              : R;
    if (rt == R) {
      const int row0 = band > 0 ? top_rows + ((band - 1) * 64 + lane) * R
                                : lane * R - (64 * R - top_rows);
      band_sweep<R, LAM, D>(a, stage[wl], lane, tau, band == 0, last, row0, pid, m, n, rinc,
                            cinc);
    } else if (rt == half) {
      band_sweep<(R >= 2 ? R / 2 : R), LAM, D>(a, stage[wl], lane, tau, true, last,
                                               lane * half - (64 * half - top_rows), pid, m,
                                               n, rinc, cinc);
    } else {
      band_sweep<(R >= 4 ? R / 4 : R), LAM, D>(a, stage[wl], lane, tau, true, last,
                                               lane * quarter - (64 * quarter - top_rows),
                                               pid, m, n, rinc, cinc);
    }
  }
}

}  // namespace pairk
}  // namespace sk
