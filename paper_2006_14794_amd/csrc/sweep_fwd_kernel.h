// Forward sweep of the explicit Goursat scheme, Section 3.1,
// eq. (explicit_finite_diff), on the dyadic grid P_lambda, with the coarse
// increment inner products computed on the fly.
//
// Mapping (one 64-lane wavefront per run of pairs that share the x path):
//   * lane l owns the R consecutive fine cell rows [l R, l R + R) of the grid
//     (rows follow x) and keeps their current values in registers;
//   * the wave advances one coarse column (2^lambda fine columns) per step,
//     lane l lagging lane l-1 by one step, so that the cells being updated lie
//     on one block antidiagonal (the antidiagonal independence noted in
//     Section 3.1.1);
//   * lane l-1's bottom-row values at the current coarse column arrive through
//     one DPP wave_shr:1 move per fine column (two 32-bit moves per double);
//   * the y increments of consecutive pairs are consecutive rows, so a wave
//     streams the columns of several pairs (x_a, y_b), (x_a, y_{b+1}), ...
//     back to back and pays the 63-step pipeline fill once per run; a lane
//     that reaches the first column of the next pair resets its rows to the
//     boundary value 1;
//   * the coarse coefficient G0[p][q] = <dx_p, dy_q> is recomputed per step
//     from the lane's dx rows (registers, pre-scaled by 2^-(2 lambda + 1)) and
//     the coarse column's dy row (loaded two steps ahead), and reused for the
//     4^lambda fine cells it covers (remark after eq. (explicit_finite_diff)).
//
// Cell update, in double: with A = left, B = up, C = up-left node and
// g = 1 + G0 / 2^(2 lambda + 1),
//     K' = fma(g, A + B, -C)  ==  A + B - C + (g - 1)(A + B),
// two double operations per cell.  g is formed in double, where the rounding
// of 1 + h perturbs h by at most 2^-53 in absolute value.  The implicit scheme
// of the remark after eq. (explicit_finite_diff) quadratures the cell with all
// four corners; solved for the new corner it is the same update with
// g = (1 + h/2) / (1 - h/2) = (2 + h) / (2 - h), formed once per coarse cell.
#pragma once
#include <math.h>

#include "sweep_args.h"

namespace sk {
namespace fwd {

// lane l receives lane l-1's value; lane 0 keeps `keep` (wave_shr:1 with the
// bound control off leaves the out-of-range lane's destination untouched).
__device__ __forceinline__ double from_prev_lane(double v, double keep) {
  const unsigned long long bv = (unsigned long long)__double_as_longlong(v);
  const unsigned long long bk = (unsigned long long)__double_as_longlong(keep);
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)bk, (int)(unsigned)bv, 0x138, 0xF,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(bk >> 32),
                                             (int)(unsigned)(bv >> 32), 0x138, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}

// The value of lane `l`, in scalar registers (uniform for the compiler).
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1 / den: the hardware reciprocal refined by two Newton-Raphson steps (each
// at least squares the relative error), within a few ulp at about half the
// cost of an IEEE division; 0 gives NaN.
__device__ __forceinline__ double refined_reciprocal(double den) {
  double r = __builtin_amdgcn_rcp(den);
  double e = __builtin_fma(-den, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-den, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Cell factors of the implicit scheme, g = (2 + h) / (2 - h) = 4 / (2 - h) - 1,
// for a lane's CR coarse rows.  The reciprocals of each group of up to four
// d = 2 - h come from one reciprocal of their product and back-multiplication
// (batch inversion: with q_i = d_0 ... d_i, 1/d_i = q_{i-1} / q_i), which
// replaces three quarter-rate reciprocals and their Newton steps by six
// products.  Each reciprocal is within a few ulp; g is formed with one fused
// multiply-add.  For h that are floats times a power of two, |d| is 0 or at
// least 2^-23, so the product of four stays inside the double range; h = 2
// gives NaN factors for its group (the scheme has no solution there).
template <int CR>
__device__ __forceinline__ void implicit_factors(const double (&h)[CR], double (&g)[CR]) {
#pragma unroll
  for (int c0 = 0; c0 < CR; c0 += 4) {
    constexpr int kGroup = 4;
    const int n = CR - c0 < kGroup ? CR - c0 : kGroup;
    double d[kGroup], q[kGroup];
#pragma unroll
    for (int i = 0; i < kGroup; ++i) {
      if (i < n) {
        d[i] = 2.0 - h[c0 + i];
        q[i] = i ? q[i - 1] * d[i] : d[i];
      }
    }
    double r = refined_reciprocal(q[n - 1]);  // 1 / q_{n-1}
#pragma unroll
    for (int i = kGroup - 1; i >= 1; --i) {
      if (i < n) {
        g[c0 + i] = __builtin_fma(4.0, r * q[i - 1], -1.0);  // 1/d_i = q_{i-1} / q_i
        r *= d[i];                                          // 1 / q_{i-1}
      }
    }
    g[c0] = __builtin_fma(4.0, r, -1.0);
  }
}

template <int DP>
__device__ __forceinline__ void load_row(const float* __restrict__ p, float (&v)[DP]) {
  const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int c = 0; c < DP / 4; ++c) {
    const float4 t = p4[c];
    v[4 * c + 0] = t.x;
    v[4 * c + 1] = t.y;
    v[4 * c + 2] = t.z;
    v[4 * c + 3] = t.w;
  }
}

__device__ __forceinline__ int32_t n_inc(const int32_t* plan, int32_t len, int64_t k) {
  return plan ? plan[k] : len - 1;
}
__device__ __forceinline__ int64_t first_row(const int64_t* plan, int32_t len, int64_t k) {
  return plan ? plan[k] : k * (int64_t)(len - 1);
}

__device__ __forceinline__ void store_out(const SweepArgs& a, int64_t ia, int64_t ib, float v) {
  if (!a.out) return;
  if (a.mode == 0) {
    a.out[ia] = v;
  } else {
    a.out[ia * a.out_ld + ib] = v;
    if (a.mode == 2 && ia != ib) a.out[ib * a.out_ld + ia] = v;
  }
}

// Resolves the run of pairs (x_ia, y_b), b in [b0, b1), of wave w, writes the
// value of every pair with nothing to sweep (a broken path: NaN; a one-point
// path: the boundary value 1; 0 on the diagonal of a symmetric Gram without
// its diagonal, as for swept pairs), and returns false when the wave has no
// columns to stream.  m: increments of x_ia; total: columns of the run.
// Runs longer than one pair are only formed for uniform y batches, so every
// pair of a run has the same width.
__device__ __forceinline__ bool wave_run(const SweepArgs& a, int64_t w, int lane, int rows,
                                         int lam, int64_t& ia, int64_t& b0, int64_t& b1,
                                         int32_t& m, int64_t& total) {
  if (a.mode == 0) {
    ia = w;
    b0 = w;
    b1 = w + 1;
  } else if (a.tri) {
    // s = 1: the triangle without its diagonal (the host zeroes it)
    const int64_t s = a.tri - 1;
    // the last row whose runs start at or before wave w (binary search on
    // the increasing run counts; the values are uniform over the wave)
    int64_t lo = 0, hi = a.nx - s;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (tri_runs(mid, a.runs_per_row, a.run, s) <= w) lo = mid; else hi = mid;
    }
    ia = lo;
    const int64_t start =
        ((ia + s) / a.run + (w - tri_runs(ia, a.runs_per_row, a.run, s))) * a.run;
    b0 = start > ia + s ? start : ia + s;  // the row's first run begins at column ia + s
    b1 = start + a.run < a.ny ? start + a.run : a.ny;
  } else {
    ia = w / a.runs_per_row;
    b0 = (w - ia * a.runs_per_row) * a.run;
    b1 = b0 + a.run < a.ny ? b0 + a.run : a.ny;
    if (a.mode == 2 && b0 < ia) b0 = ia;
    if (b0 >= b1) return false;
  }
  m = n_inc(a.x_n, a.x_len, ia);
  total = 0;
  for (int64_t b = b0; b < b1; ++b) {
    const int32_t nb = n_inc(a.y_n, a.y_len, b);
    float v = 0.0f;
    bool trivial = true;
    if (m < 0 || nb < 0)
      v = __builtin_nanf("");
    else if (m == 0 || nb == 0)
      v = 1.0f;
    else
      trivial = false;
    if (!trivial) {
      total += nb;
    } else if (lane == 0) {
      store_out(a, ia, b, (a.mode == 2 && a.no_diag && b == ia) ? 0.0f : v);
    }
  }
  if (m <= 0 || total == 0) return false;
  if (((int64_t)m << lam) > rows) {  // excluded by the host; never read past the lane rows
    for (int64_t b = b0 + lane; b < b1; b += 64) store_out(a, ia, b, __builtin_nanf(""));
    return false;
  }
  return true;
}

// One step of a lane: its R x S block of fine cells (R rows, the S = 2^LAM
// fine columns of one coarse column), in antidiagonal order so that the S
// columns form independent dependency chains for the scheduler.
//   v[r][cc]  out: the block's new values
//   sv        STORE: the R*S cell sums A + B (row-major, rounded to float)
//   u[r]      the lane's values at the previous fine column
//   up[cc]    the row above the strip (from lane l-1) at fine column cc
//   up_last   the row above at the previous fine column (C of the corner cell)
//   gk[c]     cell factor of coarse row c of the strip
// The caller then shifts u, pub and up_last to the block's last column/row
// (kept outside: the same statements inside the helper cost the Gram sweep
// eleven registers with this compiler).
template <int R, int LAM, int CR, bool STORE>
__device__ __forceinline__ void cell_block(double (&v)[R][1 << LAM],
                                           float (&sv)[STORE ? R * (1 << LAM) : 1],
                                           const double (&u)[R], const double (&up)[1 << LAM],
                                           double up_last, const double (&gk)[CR]) {
  constexpr int S = 1 << LAM;
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
      const double AB = A + B;
      if constexpr (STORE) sv[r * S + cc] = (float)AB;
      v[r][cc] = __builtin_fma(gk[(R >= S) ? (r >> LAM) : 0], AB, -C);
    }
  }
}

// IMPL: the implicit scheme's cell factor (a separate instantiation, so that
// the explicit kernel carries none of its registers).
template <int R, int LAM, int D, bool IMPL>
__global__ __launch_bounds__(256) void sweep_kernel(const SweepArgs a) {
  constexpr int DP = (D + 3) & ~3;
  constexpr int S = 1 << LAM;                          // fine columns per coarse column
  constexpr int CR = (R >> LAM) > 0 ? (R >> LAM) : 1;  // coarse rows per lane

  const int lane = threadIdx.x & 63;
  const int64_t w = a.wave0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= a.wave0 + a.n_waves) return;  // uniform per wave

  int64_t ia, b0, b1, total;
  int32_t m;
  if (!wave_run(a, w, lane, 64 * R, LAM, ia, b0, b1, m, total)) return;
  const int M = m << LAM;

  // Lane strips are aligned to the bottom of the grid: cell row M - 1 is the
  // last row of lane 63, and the rows above row 0 that the top strip covers
  // are virtual (zero increments, values identically 1 -- the boundary row).
  const int row0 = lane * R - (64 * R - M);
  const int p0 = row0 >> LAM;  // floor division; negative for virtual rows
  const int64_t xrow = first_row(a.x_start, a.x_len, ia);
  float dx[CR][D];
#pragma unroll
  for (int c = 0; c < CR; ++c) {
    float t[DP];
    if (p0 + c >= 0 && p0 + c < m) {
      load_row<DP>(a.incx + (xrow + p0 + c) * DP, t);
    } else {
#pragma unroll
      for (int k = 0; k < DP; ++k) t[k] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) dx[c][k] = t[k];
  }

  // y stream: global column g of the run is dense row first_row(b0) + g.  The
  // increment buffers carry kStreamPad rows before and after the data, so
  // rows g in [-63, total + 3] can be read without clamping (rows outside
  // the run only feed lanes that are inactive at that step).
  const int32_t total32 = (int32_t)total;
  int32_t g = -lane;
  const float* __restrict__ yp = a.incy + (first_row(a.y_start, a.y_len, b0) + g) * DP;
  // every pair of a run has the same width (runs longer than one pair are
  // only formed for uniform y batches)
  const int32_t cn = n_inc(a.y_n, a.y_len, b0);
  int32_t q = 0;  // column of the current pair

  double u[R];
#pragma unroll
  for (int r = 0; r < R; ++r) u[r] = 1.0;
  double pub[S], up[S];
#pragma unroll
  for (int cc = 0; cc < S; ++cc) {
    pub[cc] = 1.0;
    up[cc] = 1.0;  // lane 0 keeps the boundary value for the whole run
  }
  double up_last = 1.0;

  float dyA[DP], dyB[DP], dyC[DP];
  load_row<DP>(yp, dyA);
  load_row<DP>(yp + DP, dyB);
  // a multiple of 3 steps; the extra steps are inactive for every lane
  const int32_t nsteps = (int32_t)sweep_steps(total);

  // Three y-row buffers: step t reads buffer t % 3 and refills buffer
  // (t + 2) % 3, which step t - 1 has finished with, so the two-step-ahead
  // load never overlaps a live row wherever the compiler places it.
  auto step = [&](float (&dy)[DP], float (&refill)[DP]) {
    load_row<DP>(yp + 2 * DP, refill);
    float h32[CR];
#pragma unroll
    for (int c = 0; c < CR; ++c) {
      float s = 0.0f;
#pragma unroll
      for (int k = 0; k < D; ++k) s = __builtin_fmaf(dx[c][k], dy[k], s);
      h32[c] = s;
    }

#pragma unroll
    for (int cc = 0; cc < S; ++cc) up[cc] = from_prev_lane(pub[cc], up[cc]);

    if ((uint32_t)g < (uint32_t)total32) {
      double gk[CR];
      if constexpr (IMPL) {
        double h[CR];
#pragma unroll
        for (int c = 0; c < CR; ++c) h[c] = (double)h32[c];
        implicit_factors<CR>(h, gk);
      } else {
#pragma unroll
        for (int c = 0; c < CR; ++c) gk[c] = 1.0 + (double)h32[c];
      }
      double v[R][S];
      float sv[1];
      cell_block<R, LAM, CR, false>(v, sv, u, up, up_last, gk);
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[r][S - 1];
#pragma unroll
      for (int cc = 0; cc < S; ++cc) pub[cc] = v[R - 1][cc];
      up_last = up[S - 1];
      if (++q == cn) {
        // last column of a pair: emit its terminal value, then the left
        // boundary (value 1) of the next pair of the run
        if (lane == 63) {
          const int64_t cb = b0 + g / cn;
          store_out(a, ia, cb, (a.mode == 2 && a.no_diag && cb == ia) ? 0.0f : (float)u[R - 1]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = 1.0;
        up_last = 1.0;
        q = 0;
      }
    }
    ++g;
    yp += DP;
  };

  for (int32_t t = 0; t < nsteps; t += 3) {
    step(dyA, dyC);
    step(dyB, dyA);
    step(dyC, dyB);
  }
}

}  // namespace fwd
}  // namespace sk
