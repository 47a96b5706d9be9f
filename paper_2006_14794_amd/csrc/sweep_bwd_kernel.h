// Adjoint (reverse) sweep of the explicit Goursat scheme, Section 3.1,
// eq. (explicit_finite_diff), and the gradient of the terminal values with
// respect to the path increments.
//
// The forward scheme computes, for every cell (i, j) of P_lambda,
//     K[i+1][j+1] = g_ij (K[i+1][j] + K[i][j+1]) - K[i][j],
//     g_ij = 1 + G0[p][q] / 2^(2 lambda + 1),   (p, q) the coarse cell of (i, j).
// With a_ij the derivative of the weighted terminal value w K[M][N] with
// respect to K[i+1][j+1] (the cell's output node), reverse accumulation of
// that loop gives, cell by cell from the terminal corner,
//     a_ij = g_{i,j+1} a_{i,j+1} + g_{i+1,j} a_{i+1,j} - a_{i+1,j+1},
//     a_{M-1,N-1} = w,  a = 0 outside the grid,
// and d(w K[M][N]) / d g_ij = a_ij (K[i+1][j] + K[i][j+1]).  The second
// factor is stored per cell by the forward pass (sweep_fwd_store.hip).
// Summing over the 4^lambda fine cells of a coarse cell gives the
// derivative with respect to G0[p][q] / 2^(2 lambda + 1), which is contracted
// with the increments: x side sum_q dG[p][q] dy_q (per lane, registers),
// y side sum_p dG[p][q] dx_p (summed across the 64 lanes by a DPP chain that
// follows the reverse wavefront).
//
// Mapping: the forward's lane strips (bottom-aligned, R rows per lane) and
// runs of pairs, traversed backwards: lane 63 leads, lane l follows lane l+1
// one coarse column later, and values flow upwards through wave_shl:1.
#pragma once
#include <math.h>

#include "internal.h"

namespace sk {
namespace bwd {

// lane l receives lane l+1's value; lane 63 keeps `keep` (wave_shl:1 with the
// bound control off leaves the out-of-range lane's destination untouched).
__device__ __forceinline__ double from_next_lane(double v, double keep) {
  const unsigned long long bv = (unsigned long long)__double_as_longlong(v);
  const unsigned long long bk = (unsigned long long)__double_as_longlong(keep);
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)bk, (int)(unsigned)bv, 0x130, 0xF,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(bk >> 32),
                                             (int)(unsigned)(bv >> 32), 0x130, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}
__device__ __forceinline__ float from_next_lane(float v, float keep) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(keep), __float_as_int(v), 0x130, 0xF, 0xF, false));
}

template <int N>
__device__ __forceinline__ void load_vec(const float* __restrict__ p, float (&v)[N]) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      const float4 t = *reinterpret_cast<const float4*>(p + i);
      v[i] = t.x;
      v[i + 1] = t.y;
      v[i + 2] = t.z;
      v[i + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = p[i];
  }
}

template <int R, int LAM, int D>
__global__ __launch_bounds__(256) void adjoint_kernel(const BwdArgs a) {
  constexpr int DP = (D + 3) & ~3;
  constexpr int S = 1 << LAM;
  constexpr int CR = (R >> LAM) > 0 ? (R >> LAM) : 1;
  constexpr int RS = R * S;

  const int lane = threadIdx.x & 63;
  const int64_t w = a.wave0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= a.wave0 + a.n_waves) return;  // uniform per wave

  const int32_t m = a.x_len - 1, n = a.y_len - 1;  // both >= 1 (checked by the host)
  const int64_t ia = w / a.runs_per_row;
  int64_t b0 = (w - ia * a.runs_per_row) * a.run;
  const int64_t b1 = b0 + a.run < a.ny ? b0 + a.run : a.ny;
  if (a.mode == 2 && b0 < ia) b0 = ia;
  float* __restrict__ px = a.part_x + w * (int64_t)m * D;
  if (b0 >= b1) {  // an empty run of the upper triangle: no contribution
    for (int64_t e = lane; e < (int64_t)m * D; e += 64) px[e] = 0.0f;
    return;
  }

  const int M = m << LAM;
  const int row0 = lane * R - (64 * R - M);  // bottom-aligned strip (virtual rows < 0)
  const int p0 = row0 >> LAM;
  const int cb_below = ((row0 + R) >> LAM) - p0;  // coarse row of the cell row below the strip

  // x increments (pre-scaled) of coarse rows p0 .. p0 + CR; the last one is
  // the row of the cells below the strip
  float dx[CR + 1][D];
#pragma unroll
  for (int c = 0; c <= CR; ++c) {
    float t[DP];
    if (p0 + c >= 0 && p0 + c < m) {
      load_vec<DP>(a.incx + ((int64_t)ia * m + p0 + c) * DP, t);
    } else {
#pragma unroll
      for (int k = 0; k < DP; ++k) t[k] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) dx[c][k] = t[k];
  }
  float dxacc[CR][D];
#pragma unroll
  for (int c = 0; c < CR; ++c)
#pragma unroll
    for (int k = 0; k < D; ++k) dxacc[c][k] = 0.0f;

  const int32_t total = (int32_t)((b1 - b0) * n);
  const int32_t nsteps = (int32_t)sweep_steps(total);
  // global column of this lane at backward step t: total + 62 - lane - t; the
  // forward handled it at its step gcol + lane
  int32_t gcol = total + 62 - lane;
  const float* __restrict__ yp = a.incy + ((int64_t)b0 * n + gcol) * DP;
  const float* __restrict__ sbase = a.store + (w - a.wave0) * a.store_stride + (int64_t)lane * 4;
  auto srow = [&](int32_t tf) -> const float* {  // clamped: inactive steps read in bounds
    const int32_t c = tf < 0 ? 0 : (tf >= nsteps ? nsteps - 1 : tf);
    return sbase + (int64_t)c * 64 * cell_group_floats(RS);
  };

  double ar[R];     // a of this strip's cells at the first fine column of the next coarse column
  double gr[CR];    // coefficients of that column (own coarse rows)
#pragma unroll
  for (int r = 0; r < R; ++r) ar[r] = 0.0;
#pragma unroll
  for (int c = 0; c < CR; ++c) gr[c] = 1.0;
  double pub[S], ab[S];  // published top-row a / received lane l+1 top-row a
#pragma unroll
  for (int cc = 0; cc < S; ++cc) {
    pub[cc] = 0.0;
    ab[cc] = 0.0;  // lane 63 keeps 0: nothing below the grid
  }
  double prev_ab0 = 0.0;  // lane l+1's top-row a at the first fine column of the next coarse column
  float ypub[D], ych[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    ypub[k] = 0.0f;
    ych[k] = 0.0f;
  }

  int32_t q = n - 1;  // column of the current pair (counting down)
  int64_t cbp = b1 - 1;
  auto weight = [&](int64_t b) -> float {
    if (a.mode == 2 && b == ia) return a.no_diag ? 0.0f : a.dK[ia * a.ny + b];
    float wt = a.dK[ia * a.ny + b];
    if (a.mode == 2) wt += a.dK[b * a.ny + ia];  // K[a][b] and K[b][a] are one solve
    return wt;
  };
  float wcur = (lane == 63) ? weight(cbp) : 0.0f;

  float dyA[DP], dyB[DP];
  float sA[RS], sB[RS];
  load_vec<DP>(yp, dyA);
  get_cells<RS>(srow(gcol + lane), sA);

  auto step = [&](float (&dy)[DP], float (&dyn)[DP], float (&sv)[RS], float (&svn)[RS]) {
    // refill the other buffers for the next step (consumed by the previous one)
    load_vec<DP>(yp - DP, dyn);
    get_cells<RS>(srow(gcol + lane - 1), svn);

    float h32[CR + 1];
#pragma unroll
    for (int c = 0; c <= CR; ++c) {
      float s = 0.0f;
#pragma unroll
      for (int k = 0; k < D; ++k) s = __builtin_fmaf(dx[c][k], dy[k], s);
      h32[c] = s;
    }
#pragma unroll
    for (int cc = 0; cc < S; ++cc) ab[cc] = from_next_lane(pub[cc], ab[cc]);
#pragma unroll
    for (int k = 0; k < D; ++k) ych[k] = from_next_lane(ypub[k], ych[k]);

    if ((uint32_t)gcol < (uint32_t)total) {
      if (q == n - 1) {  // last column of a pair: nothing to the right
#pragma unroll
        for (int r = 0; r < R; ++r) ar[r] = 0.0;
        // the terminal cell (lane 63, last row) receives the seed through its
        // below-right neighbour: a = 0 + 0 - (-w)
        prev_ab0 = (lane == 63) ? -(double)wcur : 0.0;
      }
      double gk[CR + 1];
#pragma unroll
      for (int c = 0; c <= CR; ++c) gk[c] = 1.0 + (double)h32[c];
      const double gbelow = (R >= S) ? gk[CR] : (cb_below ? gk[1] : gk[0]);

      double v[R][S];
#pragma unroll
      for (int dgl = R + S - 2; dgl >= 0; --dgl) {
#pragma unroll
        for (int cc = S - 1; cc >= 0; --cc) {
          const int r = dgl - cc;
          if (r < 0 || r >= R) continue;
          const int cr = (R >= S) ? (r >> LAM) : 0;
          const double right = (cc == S - 1) ? ar[r] : v[r][cc + 1];
          const double gR = (cc == S - 1) ? gr[cr] : gk[cr];
          const double below = (r == R - 1) ? ab[cc] : v[r + 1][cc];
          const double gB = (r == R - 1) ? gbelow : gk[(R >= S) ? ((r + 1) >> LAM) : 0];
          const double diag = (r == R - 1) ? ((cc == S - 1) ? prev_ab0 : ab[cc + 1])
                                           : ((cc == S - 1) ? ar[r + 1] : v[r + 1][cc + 1]);
          v[r][cc] = __builtin_fma(gR, right, __builtin_fma(gB, below, -diag));
        }
      }
      // coefficient gradient per coarse cell of the strip
      double dg[CR];
#pragma unroll
      for (int c = 0; c < CR; ++c) dg[c] = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cc = 0; cc < S; ++cc)
          dg[(R >= S) ? (r >> LAM) : 0] =
              __builtin_fma(v[r][cc], (double)sv[r * S + cc], dg[(R >= S) ? (r >> LAM) : 0]);
      float ypart[D];
#pragma unroll
      for (int k = 0; k < D; ++k) ypart[k] = 0.0f;
#pragma unroll
      for (int c = 0; c < CR; ++c) {
        const float g = (float)dg[c];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          dxacc[c][k] = __builtin_fmaf(g, dy[k], dxacc[c][k]);
          ypart[k] = __builtin_fmaf(g, dx[c][k], ypart[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < D; ++k) ypub[k] = ych[k] + ypart[k];
      if (lane == 0) {  // the chain has summed all 64 strips of this column
        float* __restrict__ py = a.part_y + ((ia * a.ny + cbp) * n + q) * D;
#pragma unroll
        for (int k = 0; k < D; ++k) py[k] = ypub[k];
      }
#pragma unroll
      for (int cc = 0; cc < S; ++cc) pub[cc] = v[0][cc];
      prev_ab0 = ab[0];
#pragma unroll
      for (int r = 0; r < R; ++r) ar[r] = v[r][0];
#pragma unroll
      for (int c = 0; c < CR; ++c) gr[c] = gk[c];
      if (--q < 0) {  // first column of the pair done: move to the pair on the left
        q = n - 1;
        --cbp;
        if (lane == 63 && cbp >= b0) wcur = weight(cbp);
      }
    }
    --gcol;
    yp -= DP;
  };

  for (int32_t t = 0; t < nsteps; t += 2) {
    step(dyA, dyB, sA, sB);
    step(dyB, dyA, sB, sA);
  }

  if constexpr (R < S) {
    // S / R consecutive lanes (aligned groups) share one coarse row: sum
    // their parts; the first lane of the group writes
    constexpr int G = S / R;
#pragma unroll
    for (int o = 1; o < G; o <<= 1)
#pragma unroll
      for (int k = 0; k < D; ++k) dxacc[0][k] += __shfl_xor(dxacc[0][k], o, 64);
    if (lane % G != 0) return;
  }
#pragma unroll
  for (int c = 0; c < CR; ++c) {
    const int p = p0 + c;
    if (p >= 0 && p < m) {
#pragma unroll
      for (int k = 0; k < D; ++k) px[(int64_t)p * D + k] = dxacc[c][k];
    }
  }
}

}  // namespace bwd
}  // namespace sk
