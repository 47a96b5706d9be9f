// Forward sweep of the signature kernel of lifted paths (the static-kernel
// lift of eq. (PDE_lifted)) with the Gaussian static kernel
//     kappa(a, b) = exp(-|a - b|^2 / (2 sigma^2)).
// By the finite-difference form that follows eq. (PDE_lifted), the coarse
// coefficient of the cell between nodes p, p+1 of x and q, q+1 of y is the
// second difference
//     G[p][q] = kappa(x_{p+1}, y_{q+1}) - kappa(x_p, y_{q+1})
//               - kappa(x_{p+1}, y_q) + kappa(x_p, y_q)
// (the printed second term has x_t where the pairing needs y_t), in place of
// <dx_p, dy_q>; the scheme on P_lambda is otherwise the plain one.
//
// Mapping: the lane strips, DPP exchange, runs of pairs and cell update of
// the plain sweep (sweep_fwd_kernel.h).  What changes is the coefficient:
//   * lane l keeps the x NODES of its coarse rows, x_{p0} .. x_{p0+CR}
//     (float registers; nodes above the grid repeat x_0, which makes their
//     coefficients exactly 0);
//   * the wave streams y node rows; at node y_t a lane evaluates
//     kappa(x_{p0+c}, y_t) for its nodes c = 1 .. CR in double (the
//     differences of float coordinates are exact in double); with at least
//     2^lambda rows per lane its node 0 is lane l-1's node CR, which that
//     lane evaluated at the previous step (one column ahead) with the same
//     inputs and instructions, and arrives by DPP (with fewer rows, lanes
//     share coarse rows and node 0 is evaluated too); then the row differences
//     d_t[c] = kappa(x_{p0+c+1}, y_t) - kappa(x_{p0+c}, y_t) and
//     G[p0+c][t-1] = d_t[c] - d_{t-1}[c];
//   * each pair's stream starts with its node y_0, a priming step that only
//     records d_0 (so a run of n_b-increment pairs takes sum (n_b + 1) steps).
// The coefficient is a second difference of values near 1; forming it in
// double keeps its relative error near 2^-50 |kappa| / |G| rather than the
// 2^-24 |kappa| / |G| of float.
#pragma once
#include <math.h>

#include "sweep_fwd_kernel.h"

namespace sk {
namespace lift {

using fwd::cell_block;
using fwd::first_row;
using fwd::from_prev_lane;
using fwd::implicit_factors;
using fwd::load_row;
using fwd::n_inc;
using fwd::store_out;
using fwd::wave_run;

// First node row of path k in a dense node buffer: paths are consecutive,
// each with n_k + 1 rows (uniform: len rows).
__device__ __forceinline__ int64_t first_node(const int64_t* start, int32_t len, int64_t k) {
  return start ? start[k] + k : k * (int64_t)len;
}

template <int R, int LAM, int D>
__global__ __launch_bounds__(256) void lifted_sweep_kernel(const SweepArgs a) {
  constexpr int DP = (D + 3) & ~3;
  constexpr int S = 1 << LAM;
  constexpr int CR = (R >> LAM) > 0 ? (R >> LAM) : 1;

  const int lane = threadIdx.x & 63;
  const int64_t w = a.wave0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= a.wave0 + a.n_waves) return;  // uniform per wave

  int64_t ia, b0, b1, total;
  int32_t m;
  if (!wave_run(a, w, lane, 64 * R, LAM, ia, b0, b1, m, total)) return;
  const int M = m << LAM;

  // strips aligned to the bottom of the grid, as in the plain sweep
  const int off = 64 * R - M;  // virtual rows above row 0 (uniform)
  const int row0 = lane * R - off;
  const int p0 = row0 >> LAM;
  const int64_t xnode = first_node(a.x_start, a.x_len, ia);
  float xn[CR + 1][D];
#pragma unroll
  for (int c = 0; c <= CR; ++c) {
    const int p = p0 + c < 0 ? 0 : p0 + c;  // p0 + CR <= m always
    float t[DP];
    load_row<DP>(a.incx + (xnode + p) * DP, t);
#pragma unroll
    for (int k = 0; k < D; ++k) xn[c][k] = t[k];
  }

  // y stream: stream row g of the run is node row first_node(b0) + g; every
  // pair of a run has cn increments, so cn + 1 rows
  const int32_t cn = n_inc(a.y_n, a.y_len, b0);
  const int32_t rows32 = (int32_t)(total + total / cn);
  int32_t g = -lane;
  const float* __restrict__ yp = a.incy + (first_node(a.y_start, a.y_len, b0) + g) * DP;
  int32_t q = -1;  // column of the current pair; -1: its priming node
  const double inv = a.lift_inv;
  const double scale = a.lift_scale;

  double u[R];
#pragma unroll
  for (int r = 0; r < R; ++r) u[r] = 1.0;
  double pub[S], up[S];
#pragma unroll
  for (int cc = 0; cc < S; ++cc) {
    pub[cc] = 1.0;
    up[cc] = 1.0;
  }
  double up_last = 1.0;
  double dprev[CR];
#pragma unroll
  for (int c = 0; c < CR; ++c) dprev[c] = 0.0;
  // this lane's node-CR kernel value at the previous step, for lane l+1
  // (R >= 2^lambda: lane l's first coarse row is lane l-1's last plus one)
  double kpub = 0.0;
  // Lane 0 has no lane above: when its strip starts above the grid (off > 0)
  // its nodes 0 and 1 are both x_0 and node 1's value serves; when the grid
  // fills the wave exactly, node 0 is evaluated as well (a uniform branch).
  const bool own_top = off == 0;

  float yA[DP], yB[DP], yC[DP];
  load_row<DP>(yp, yA);
  load_row<DP>(yp + DP, yB);
  const int32_t nsteps = (int32_t)sweep_steps(rows32);

  auto step = [&](float (&yn)[DP], float (&refill)[DP]) {
    load_row<DP>(yp + 2 * DP, refill);
    double yd[D];
#pragma unroll
    for (int k = 0; k < D; ++k) yd[k] = (double)yn[k];
    auto kappa = [&](int c) {
      double r = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double t = (double)xn[c][k] - yd[k];
        r = __builtin_fma(t, t, r);
      }
      return exp(-r * inv);
    };
    double kap[CR + 1];
#pragma unroll
    for (int c = 1; c <= CR; ++c) kap[c] = kappa(c);
    if constexpr (R >= S) {
      double keep0 = kap[1];
      if (own_top) keep0 = kappa(0);
      kap[0] = from_prev_lane(kpub, keep0);
      kpub = kap[CR];
    } else {
      kap[0] = kappa(0);  // lanes share coarse rows: no lane above holds node 0
    }

#pragma unroll
    for (int cc = 0; cc < S; ++cc) up[cc] = from_prev_lane(pub[cc], up[cc]);

    if ((uint32_t)g < (uint32_t)rows32) {
      double dn[CR];
#pragma unroll
      for (int c = 0; c < CR; ++c) dn[c] = kap[c + 1] - kap[c];
      if (q < 0) {
        q = 0;
      } else {
        double gk[CR], h[CR];
#pragma unroll
        for (int c = 0; c < CR; ++c) h[c] = (dn[c] - dprev[c]) * scale;
        if (a.implicit) {
          implicit_factors<CR>(h, gk);
        } else {
#pragma unroll
          for (int c = 0; c < CR; ++c) gk[c] = 1.0 + h[c];
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
          if (lane == 63) {
            const int64_t cb = b0 + g / (cn + 1);
            store_out(a, ia, cb,
                      (a.mode == 2 && a.no_diag && cb == ia) ? 0.0f : (float)u[R - 1]);
          }
#pragma unroll
          for (int r = 0; r < R; ++r) u[r] = 1.0;
          up_last = 1.0;
          q = -1;
        }
      }
#pragma unroll
      for (int c = 0; c < CR; ++c) dprev[c] = dn[c];
    }
    ++g;
    yp += DP;
  };

  for (int32_t t = 0; t < nsteps; t += 3) {
    step(yA, yC);
    step(yB, yA);
    step(yC, yB);
  }
}

}  // namespace lift
}  // namespace sk
