// Gradient of a weighted sum of Gram entries, L = sum_ab w_ab k(x_a, y_b),
// through the explicit scheme of Section 3.1, eq. (explicit_finite_diff), on
// P_lambda: the discrete adjoint of the cell recurrence, with the forward
// values recomputed from checkpoints instead of stored.
//
// The forward scheme computes, for every cell (i, j),
//     K[i+1][j+1] = g_ij (K[i+1][j] + K[i][j+1]) - K[i][j],
//     g_ij = 1 + G0[p][q] / 2^(2 lambda + 1),   (p, q) the coarse cell of (i, j).
// With a_ij the derivative of w K[M][N] with respect to the cell's output node
// K[i+1][j+1], reverse accumulation of that loop gives, from the terminal corner,
//     a_ij = g_{i,j+1} a_{i,j+1} + g_{i+1,j} a_{i+1,j} - a_{i+1,j+1},
//     a_{M-1,N-1} = w,  a = 0 outside the grid,
// and dL / dg_ij = a_ij (K[i+1][j] + K[i][j+1]).  Summed over the 4^lambda fine
// cells of a coarse cell this is the derivative with respect to
// G0[p][q] / 2^(2 lambda + 1), contracted with the increments: the x side
// sum_q dG[p][q] dy_q stays in the lane's registers, the y side
// sum_p dG[p][q] dx_p is summed across the lanes by a DPP chain that follows
// the reverse wavefront.  Every gradient sum is formed in double.
//
// Mapping: one wave per task (a run of pairs sharing the x path, or one pair),
// lane l owning R fine rows of a band of 64 R rows; the bands of a task are
// swept one after another.
//  * Forward pass, bands top to bottom: the forward sweep's wavefront (one
//    coarse column per step, lane l lagging lane l-1 by one step, DPP
//    wave_shr:1 between lanes).  A band's bottom row goes to `hand_f` for the
//    band below; every C steps each lane saves its state (R + 2^lambda
//    doubles) as a checkpoint; the last band writes the terminal values.
//  * Adjoint pass, bands bottom to top.  Lane l handles coarse column t - l
//    at forward step t, and the reverse wavefront (lane 63 leading) reaches
//    the same column at reverse step T - t for every lane: the adjoint runs
//    the forward program backwards in time.  So the C forward steps of a
//    segment are recomputed from its checkpoint (the same state and the same
//    operations: bitwise the forward's values), their cell sums A + B are kept
//    on chip, and the segment's C reverse steps consume them in the opposite
//    order.  A band's top-row adjoint values go to `hand_a` and its y-side
//    partial sums to the y-gradient rows, for the band above.
//  * Every lane steps at every step.  Outside the task's columns (before a
//    lane's first column and after its last) the staged y rows are zero, so
//    the forward values there stay the boundary value 1 before the run and
//    are never read after it, and the adjoint values stay 0 after the run
//    (in reverse order: before it) and are never read before it; gradients
//    only collect products with zero increments there.  No step branches on
//    the lane's column, except for the bookkeeping of pair ends.
//  * Inputs of a segment (y rows, the neighbouring bands' rows) are staged
//    in LDS one segment ahead; outputs for the neighbouring bands are staged
//    in LDS and written out once per segment.
// HBM traffic per fine cell: the checkpoints, 8 (R + 2^lambda) /
// (R 2^lambda C) bytes written once and read once, instead of a stored cell
// sum per fine cell.
#pragma once
#include <math.h>

#include <type_traits>

#include "grad_args.h"
#include "sweep_fwd_kernel.h"

namespace sk {
namespace grad {

using fwd::first_row;
using fwd::from_prev_lane;
using fwd::load_row;
using fwd::n_inc;

// lane l receives lane l+1's value; lane 63 keeps `keep` (wave_shl:1 with the
// bound control off leaves the out-of-range lane's destination untouched).
__device__ __forceinline__ float from_next_lane(float v, float keep) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(keep), __float_as_int(v), 0x130, 0xF, 0xF, false));
}
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

// base[i] with a 32-bit byte offset (a uniform base and one offset register:
// the addressing of the staging loads and stores of a task, whose buffers are
// far below 4 GB)
template <class T>
__device__ __forceinline__ T& at(T* base, uint32_t i) {
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return *reinterpret_cast<T*>(reinterpret_cast<C*>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
}

// s_waitcnt operand of vmcnt(0) alone (expcnt and lgkmcnt at their maxima)
constexpr int kWaitVmcnt0 = 0x0F70;

// Upstream weight of the solve (x_ia, y_b): in the upper triangle of a
// symmetric Gram, K[a][b] and K[b][a] are one solve.
__device__ __forceinline__ double pair_weight(const GradArgs& a, int64_t ia, int64_t b) {
  const double w = (double)a.dK[ia * a.ny + b];
  if (a.mode != 2) return w;
  if (b == ia) return a.no_diag ? 0.0 : w;
  return w + (double)a.dK[b * a.ny + ia];
}

__device__ __forceinline__ void store_value(const GradArgs& a, int64_t ia, int64_t b, float v) {
  a.K[ia * a.ny + b] = v;
  if (a.mode == 2 && b != ia) a.K[b * a.ny + ia] = v;
}

// Every lane of the wave writes the same values to rows [0, n) of p (a fill
// without lane-dependent branches around it).
__device__ __forceinline__ void fill_rows(double* __restrict__ p, int64_t n, double v, int lane) {
  for (int64_t e0 = 0; e0 < n; e0 += 64)
    if (e0 + lane < n) p[e0 + lane] = v;
}

// CL steps of a segment keep their cell sums in LDS, the next CG in registers.
// Two waves per SIMD (at most 256 registers) up to 4 channels below order 3;
// otherwise one or two, as the registers allow: wider increments and
// accumulators, or the eight fine columns of order 3, would spill to memory.
// YS: the y-side gradients are formed (the gradient of the y batch, or of a
// symmetric Gram); without them the kernel forms the x side only.
template <int R, int LAM, int D, int CL, int CG, bool YS>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(D <= 4 && LAM < 3 ? 2 : 1, 2))) void grad_kernel(
    const GradArgs a) {
  constexpr int DP = (D + 3) & ~3;
  constexpr int DY = YS ? D : 0;          // y-side sums per column
  constexpr int DYA = YS ? D : 1;         // (their array extent)
  constexpr int S = 1 << LAM;
  constexpr int CR = (R >> LAM) > 0 ? (R >> LAM) : 1;
  constexpr int RS = R * S;
  constexpr int KS = R + S;               // checkpoint doubles per lane
  constexpr int C = CL + CG;
  constexpr int G4 = RS / 4;              // float4 groups of one lane's cell sums per step
  constexpr int Y4 = (C + 63) * DP / 4;   // float4s of a segment's y rows
  constexpr int PY = (Y4 + 63) / 64;      // ... per lane
  constexpr int NB = C * S;               // lane 0's upper neighbours per segment
  constexpr int PB = (NB + 63) / 64;
  constexpr int LW = S + 1 + DY;          // a band's hand-over per column: S a values,
                                          // one coefficient, D y-side sums
  constexpr int NL = C * LW;              // lane 63's lower neighbours per segment
  constexpr int PL = (NL + 63) / 64;
  static_assert(KS == grad_state_doubles(LAM) && R == kGradRows && RS % 4 == 0,
                "scratch geometry");
  // cell sums: [step][group][lane], each 16-byte access of the wave covers 1 KB,
  // no bank conflicts
  __shared__ float4 lds[CL * G4 * 64];
  __shared__ float4 sy[Y4];    // the segment's y rows: row g - (t0 - 63), zero outside the task
  __shared__ double sb[NB];    // [step][fine column]: lane 0's upper neighbours
  __shared__ double sl[NL];    // [step][LW]: lane 63's lower neighbours, zero outside the task
  __shared__ double sw[NL];    // outputs of the segment for the neighbouring bands

  const int lane = threadIdx.x;
  const GradSlot L = grad_slot_layout(LAM, a.nb_max, a.nseg_max, a.cols_max);
  double* __restrict__ scr = a.scratch + (int64_t)blockIdx.x * a.slot_stride;
  double* __restrict__ ckpt = scr + L.ckpt;
  double* __restrict__ hand_f = scr + L.hand_f;
  double* __restrict__ hand_a = scr + L.hand_a;
  const int64_t ck_band = (int64_t)(a.nseg_max - 1) * KS * 64;
  const int64_t hf_band = a.cols_max * S;
  const int64_t ha_buf = (a.cols_max + 1) * (S + 1);

  for (;;) {
    int32_t task = 0;
    if (lane == 0) task = atomicAdd(a.counter, 1);
    task = __builtin_amdgcn_readlane(task, 0);  // scalar: uniform loop control
    if (task >= a.n_tasks) break;
    int64_t ia, b0, b1, jslot;
    if (a.order) {
      const int64_t pid = a.order[task];
      ia = pid / a.ny;
      b0 = pid - ia * a.ny;
      b1 = b0 + 1;
      jslot = b0;
    } else {
      ia = task / a.runs_per_row;
      jslot = task - ia * a.runs_per_row;
      b0 = jslot * a.run;
      b1 = b0 + a.run < a.ny ? b0 + a.run : a.ny;
    }
    if (a.mode == 2 && b0 < ia) b0 = ia;  // below the diagonal: nothing (b0 >= b1 there)
    const int32_t m = n_inc(a.x_n, a.x_len, ia);
    double* __restrict__ px = a.part_x + ((int64_t)ia * a.runs_per_row + jslot) * a.mrows * D;
    if (a.mode == 2 && a.no_diag && b0 == ia && b0 < b1) {
      // the diagonal of a symmetric Gram without it: the constant 0, no
      // gradient (every lane stores the same values)
      if (YS)
        fill_rows(a.part_y + ((int64_t)ia * a.ny + ia) * a.nrows * D, (int64_t)a.nrows * D,
                  m < 0 ? __builtin_nan("") : 0.0, lane);
      if (a.K) a.K[ia * a.ny + ia] = 0.0f;
      ++b0;
    }
    const int32_t n = b0 < b1 ? n_inc(a.y_n, a.y_len, b0) : 0;
    double* __restrict__ pyt = YS ? a.part_y + ((int64_t)ia * a.ny + b0) * a.nrows * D : nullptr;

    if (!(b0 < b1 && m > 0 && n > 0)) {
      // Nothing to sweep.  Values: a broken path NaN, a one-point path 1;
      // gradients 0 (NaN for a broken pair).  Every lane stores the same values.
      const bool broken = m < 0 || (b0 < b1 && n < 0);
      fill_rows(px, (int64_t)a.mrows * D, broken ? __builtin_nan("") : 0.0, lane);
      for (int64_t b = b0; b < b1; ++b) {
        const int32_t nb_ = n_inc(a.y_n, a.y_len, b);
        const bool bad = m < 0 || nb_ < 0;
        if (YS)
          fill_rows(a.part_y + ((int64_t)ia * a.ny + b) * a.nrows * D, (int64_t)a.nrows * D,
                    bad ? __builtin_nan("") : 0.0, lane);
        if (a.K) store_value(a, ia, b, bad ? __builtin_nanf("") : 1.0f);
      }
      continue;
    }

    const int32_t total = (int32_t)((b1 - b0) * n);  // coarse columns of the task
    const int32_t nseg = (total + 63 + C - 1) / C;
    const int M = m << LAM;
    const int nb = (M + 64 * R - 1) / (64 * R);
    const int off = nb * 64 * R - M;  // virtual rows above row 0, in the top band
    const float* __restrict__ xinc = a.incx + first_row(a.x_start, a.x_len, ia) * DP;
    const float* __restrict__ ycol = a.incy + first_row(a.y_start, a.y_len, b0) * DP;

    // ---- staging of a segment's inputs (registers one segment ahead, then LDS)
    auto fetch_y = [&](int32_t seg, float4 (&py)[PY]) {
      const int32_t t0 = seg * C;
#pragma unroll
      for (int i = 0; i < PY; ++i) {
        const int e = lane + 64 * i;
        py[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const int32_t g = t0 - 63 + e / (DP / 4);
        if (e < Y4 && (uint32_t)g < (uint32_t)total)
          py[i] = at(reinterpret_cast<const float4*>(ycol), (uint32_t)(g * (DP / 4) + e % (DP / 4)));
      }
    };
    auto put_y = [&](const float4 (&py)[PY]) {
#pragma unroll
      for (int i = 0; i < PY; ++i) {
        const int e = lane + 64 * i;
        if (e < Y4) sy[e] = py[i];
      }
    };
    // lane 0's upper neighbours at steps t0 .. t0 + C - 1 (columns t0 + j;
    // beyond the task: the last column's, never used for a real cell)
    auto fetch_up = [&](int32_t seg, bool top, const double* __restrict__ above,
                        double (&pb)[PB]) {
      const int32_t t0 = seg * C;
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const int e = lane + 64 * i;
        pb[i] = 1.0;
        if (!top && e < NB) {
          int32_t col = t0 + e / S;
          col = col < total ? col : total - 1;
          pb[i] = at(above, (uint32_t)(col * S + e % S));
        }
      }
    };
    auto put_up = [&](const double (&pb)[PB]) {
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const int e = lane + 64 * i;
        if (e < NB) sb[e] = pb[i];
      }
    };
    // the y row of a lane at step t0 + j
    auto get_dy = [&](int j, float (&dy)[DP]) {
      const float4* r = &sy[(j - lane + 63) * (DP / 4)];
#pragma unroll
      for (int c = 0; c < DP / 4; ++c) {
        const float4 f = r[c];
        dy[4 * c] = f.x;
        dy[4 * c + 1] = f.y;
        dy[4 * c + 2] = f.z;
        dy[4 * c + 3] = f.w;
      }
    };
    auto load_dx = [&](int p0, float (&dx)[CR][D]) {
#pragma unroll
      for (int c = 0; c < CR; ++c) {
        float tr[DP];
        if (p0 + c >= 0 && p0 + c < m) {
          load_row<DP>(xinc + (int64_t)(p0 + c) * DP, tr);
        } else {
#pragma unroll
          for (int k = 0; k < DP; ++k) tr[k] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < D; ++k) dx[c][k] = tr[k];
      }
    };
    // Steps j (bit j) at which a lane whose column at the segment's first step
    // is g0 is at the last column of a pair (k n - 1 for some k >= 1) of the
    // task: the forward values restart there, the adjoint receives its seed.
    auto pair_end_mask = [&](int32_t g0) -> uint32_t {
      const int32_t c0 = g0 > 0 ? g0 : 0;
      const int32_t cend = g0 + C - 1 < total - 1 ? g0 + C - 1 : total - 1;
      uint32_t mask = 0;
      for (int32_t e = (c0 / n) * n + n - 1; e <= cend; e += n) mask |= 1u << (e - g0);
      return mask;
    };
    // The LDS inputs of a step are read one step ahead (during the previous
    // step's arithmetic), so that their latency is hidden; each step is
    // scheduled on its own (sched_barrier before the read of the next step's
    // inputs): interleaving the unrolled steps would keep several steps'
    // values live and spill registers.
    // forward step inputs: the lane's y row, lane 0's upper neighbours
    struct FwdIn {
      float dy[DP];
      double up[S];
    };
    auto read_fwd = [&](int j, FwdIn& in) {
      get_dy(j, in.dy);
#pragma unroll
      for (int cc = 0; cc < S; ++cc) in.up[cc] = sb[j * S + cc];
    };
    // one forward step of the wavefront at step t0 + j; st: the cell sums
    // (when it holds R S floats)
    auto forward_step = [&](const FwdIn& in, const float (&dx)[CR][D], double (&u)[R],
                            double (&pub)[S], double& up_last, auto& st) {
      float h32[CR];
#pragma unroll
      for (int c = 0; c < CR; ++c) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) s = __builtin_fmaf(dx[c][k], in.dy[k], s);
        h32[c] = s;
      }
      double up[S];
#pragma unroll
      for (int cc = 0; cc < S; ++cc) up[cc] = from_prev_lane(pub[cc], in.up[cc]);
      double gk[CR];
#pragma unroll
      for (int c = 0; c < CR; ++c) gk[c] = 1.0 + (double)h32[c];
      double v[R][S];
      constexpr bool kStore = sizeof(st) == sizeof(float) * RS;
      fwd::cell_block<R, LAM, CR, kStore>(v, st, u, up, up_last, gk);
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[r][S - 1];
#pragma unroll
      for (int cc = 0; cc < S; ++cc) pub[cc] = v[R - 1][cc];
      up_last = up[S - 1];
    };

    // ---------------- forward pass: bands top to bottom ----------------
    for (int band = 0; band < nb; ++band) {
      if (band > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // hand_f of the band above
      const bool top = band == 0, last = band == nb - 1;
      const int p0 = ((band * 64 + lane) * R - off) >> LAM;  // floor; < 0 for virtual rows
      float dx[CR][D];
      load_dx(p0, dx);
      // the band's increments have arrived before the segment loop starts:
      // otherwise the compiler's wait for them can land at the head of a step
      // loop and cover the staging loads in flight there too (vmcnt(0))
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      const double* __restrict__ above = hand_f + (int64_t)(band > 0 ? band - 1 : 0) * hf_band;
      double* __restrict__ below = hand_f + (int64_t)band * hf_band;
      double* __restrict__ ck = ckpt + (int64_t)band * ck_band;
      double u[R], pub[S], up_last = 1.0;
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = 1.0;
#pragma unroll
      for (int cc = 0; cc < S; ++cc) pub[cc] = 1.0;
      float4 py[PY];
      double pb[PB];
      fetch_y(0, py);
      fetch_up(0, top, above, pb);
      for (int32_t seg = 0; seg < nseg; ++seg) {
        const int32_t t0 = seg * C;
        __syncthreads();  // the previous segment's reads of the staging are done
        put_y(py);
        put_up(pb);
        __syncthreads();
        if (seg + 1 < nseg) {
          fetch_y(seg + 1, py);
          fetch_up(seg + 1, top, above, pb);
        }
        const uint32_t pe = pair_end_mask(t0 - lane);
        auto fwd_pass_step = [&](const int j, const FwdIn& in) {
          float st[1];
          forward_step(in, dx, u, pub, up_last, st);
          // lane 63's bottom row: for the band below, or in the last band the
          // Gram value at the last column of a pair (its last entry)
          if (lane == 63) {
#pragma unroll
            for (int cc = 0; cc < S; ++cc) sw[j * S + cc] = pub[cc];
          }
          if ((pe >> j) & 1u) {
            // last column of a pair: the left boundary of the next pair
#pragma unroll
            for (int r = 0; r < R; ++r) u[r] = 1.0;
            up_last = 1.0;
          }
        };
        // two steps per iteration, alternating two input buffers (the read
        // past the segment's last step re-reads that step)
        FwdIn fa, fb;
        read_fwd(0, fa);
#pragma unroll 1
        for (int j = 0; j + 1 < C; j += 2) {
          __builtin_amdgcn_sched_barrier(0);
          read_fwd(j + 1, fb);
          fwd_pass_step(j, fa);
          __builtin_amdgcn_sched_barrier(0);
          read_fwd(j + 2 < C ? j + 2 : j + 1, fa);
          fwd_pass_step(j + 1, fb);
        }
        if constexpr (C & 1) {
          __builtin_amdgcn_sched_barrier(0);
          fwd_pass_step(C - 1, fa);
        }
        // (global stores stay out of the step loop: a loop with stores makes
        // the compiler wait for the staging loads in flight before entering it)
        if (!last) {  // the band's bottom row at columns t0 - 63 .. t0 + C - 64
          __syncthreads();
          for (int e = lane; e < C * S; e += 64) {
            const int32_t col = t0 + e / S - 63;
            if ((uint32_t)col < (uint32_t)total) at(below, (uint32_t)(col * S + e % S)) = sw[e];
          }
        } else if (a.K) {  // the values of the pairs that end in this segment
          __syncthreads();
          for (int j = lane; j < C; j += 64) {
            const int32_t col = t0 + j - 63;
            if ((uint32_t)col < (uint32_t)total && (col + 1) % n == 0)
              store_value(a, ia, b0 + col / n, (float)sw[j * S + S - 1]);
          }
        }
        // the checkpoint of the next segment: the state before its first step.
        // (Stored at the end of the segment, before the next staging loads:
        // the next step loop overwrites these registers, and a wait for the
        // stores then leaves the later loads in flight.)
        if (seg + 1 < nseg) {
          const uint32_t c0 = (uint32_t)(seg * KS * 64 + lane);
#pragma unroll
          for (int r = 0; r < R - 1; ++r) at(ck, c0 + r * 64) = u[r];
#pragma unroll
          for (int cc = 0; cc < S; ++cc) at(ck, c0 + (R - 1 + cc) * 64) = pub[cc];
          at(ck, c0 + (R - 1 + S) * 64) = up_last;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }

    // ---------------- adjoint pass: bands bottom to top ----------------
    for (int band = nb - 1; band >= 0; --band) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // checkpoints, hand_f, hand_a, part_y
      const bool top = band == 0, last = band == nb - 1;
      const int row0 = (band * 64 + lane) * R - off;
      const int p0 = row0 >> LAM;
      const int cb_below = ((row0 + R) >> LAM) - p0;  // coarse row of the cell row below, relative
      float dx[CR][D];
      load_dx(p0, dx);
      double dxd[CR][DYA];  // the same increments in double, for the y-side products
#pragma unroll
      for (int c = 0; c < CR; ++c)
#pragma unroll
        for (int k = 0; k < DY; ++k) dxd[c][k] = (double)dx[c][k];
      double dxacc[CR][D];
#pragma unroll
      for (int c = 0; c < CR; ++c)
#pragma unroll
        for (int k = 0; k < D; ++k) dxacc[c][k] = 0.0;
      const double* __restrict__ above = hand_f + (int64_t)(band > 0 ? band - 1 : 0) * hf_band;
      const double* __restrict__ abl = hand_a + (int64_t)((band + 1) & 1) * ha_buf;
      double* __restrict__ abw = hand_a + (int64_t)(band & 1) * ha_buf;
      const double* __restrict__ ck = ckpt + (int64_t)band * ck_band;

      // lane 63's lower neighbours at steps t0 .. t0 + C - 1 (columns
      // t0 + j - 63; zero outside the task and below the last band)
      auto fetch_low = [&](int32_t seg, double (&pl)[PL]) {
        const int32_t t0 = seg * C;
#pragma unroll
        for (int i = 0; i < PL; ++i) {
          const int e = lane + 64 * i;
          pl[i] = 0.0;
          const int j = e / LW, f = e - j * LW;
          const int32_t col = t0 + j - 63;
          if (!last && e < NL && (uint32_t)col < (uint32_t)total) {
            if (!YS || f <= S) {
              pl[i] = at(abl, (uint32_t)(col * (S + 1) + f));
            } else {
              const int32_t bq = col / n, qq = col - bq * n;
              pl[i] = at(pyt, (uint32_t)((bq * a.nrows + qq) * D + (f - S - 1)));
            }
          }
        }
      };
      auto put_low = [&](const double (&pl)[PL]) {
#pragma unroll
        for (int i = 0; i < PL; ++i) {
          const int e = lane + 64 * i;
          if (e < NL) sl[e] = pl[i];
        }
      };
      auto fetch_ck = [&](int32_t seg, double (&pk)[KS]) {
        if (seg > 0) {
          const uint32_t c0 = (uint32_t)((seg - 1) * KS * 64 + lane);
#pragma unroll
          for (int i = 0; i < KS; ++i) pk[i] = at(ck, c0 + i * 64);
        } else {
#pragma unroll
          for (int i = 0; i < KS; ++i) pk[i] = 1.0;
        }
      };

      double ar[R];   // a of the strip's cells at the first fine column of the next coarse column
      double gr[CR];  // cell factors of that column
#pragma unroll
      for (int r = 0; r < R; ++r) ar[r] = 0.0;
#pragma unroll
      for (int c = 0; c < CR; ++c) gr[c] = 1.0;
      double pubA[S];  // published top-row a
#pragma unroll
      for (int cc = 0; cc < S; ++cc) pubA[cc] = 0.0;
      double prev_ab0 = 0.0;  // lane l+1's top-row a at the next column's first fine column
      float hpub = 0.0f;      // published coefficient (first coarse row)
      double ypub[DYA];       // published y-side partial sums
#pragma unroll
      for (int k = 0; k < DY; ++k) ypub[k] = 0.0;

      float4 py[PY];
      double pb[PB], pl[PL], pk[KS];
      fetch_y(nseg - 1, py);
      fetch_up(nseg - 1, top, above, pb);
      fetch_low(nseg - 1, pl);
      fetch_ck(nseg - 1, pk);
      for (int32_t seg = nseg - 1; seg >= 0; --seg) {
        const int32_t t0 = seg * C;
        const int32_t g0 = t0 - lane;  // column of this lane at step t0
        __syncthreads();  // the previous segment's reads of the staging are done
        put_y(py);
        put_up(pb);
        put_low(pl);
        __syncthreads();
        // recompute the segment's forward steps from its checkpoint
        double u[R], pub[S], up_last;
#pragma unroll
        for (int r = 0; r < R - 1; ++r) u[r] = pk[r];
#pragma unroll
        for (int cc = 0; cc < S; ++cc) pub[cc] = pk[R - 1 + cc];
        up_last = pk[R - 1 + S];
        {  // the last value: the bottom row's last entry, or 1 after a pair's end
          const int32_t cl = g0 - 1;
          u[R - 1] = ((uint32_t)cl < (uint32_t)total && (cl + 1) % n == 0) ? 1.0 : pub[S - 1];
        }
        const uint32_t pe = pair_end_mask(g0);
        auto recompute_step = [&](const int j, const FwdIn& in, float (&st)[RS]) {
          forward_step(in, dx, u, pub, up_last, st);
          if ((pe >> j) & 1u) {
#pragma unroll
            for (int r = 0; r < R; ++r) u[r] = 1.0;
            up_last = 1.0;
          }
        };
        auto put_sums = [&](const int j, const float (&st)[RS]) {
#pragma unroll
          for (int e = 0; e < G4; ++e)
            lds[(j * G4 + e) * 64 + lane] =
                make_float4(st[4 * e], st[4 * e + 1], st[4 * e + 2], st[4 * e + 3]);
        };
        // the first CL steps keep their cell sums in LDS, the last CG in
        // registers; inputs read one step ahead, alternating two buffers
        float sv[CG][RS];
        FwdIn fi[2];
        read_fwd(0, fi[0]);
#pragma unroll 1
        for (int j = 0; j < CL; j += 2) {
          float st[RS];
          __builtin_amdgcn_sched_barrier(0);
          read_fwd(j + 1, fi[1]);
          recompute_step(j, fi[0], st);
          put_sums(j, st);
          __builtin_amdgcn_sched_barrier(0);
          read_fwd(j + 2, fi[0]);  // j + 2 <= CL < C
          recompute_step(j + 1, fi[1], st);
          put_sums(j + 1, st);
        }
#pragma unroll
        for (int j = CL; j < C; ++j) {
          __builtin_amdgcn_sched_barrier(0);
          if (j + 1 < C) read_fwd(j + 1, fi[(j + 1 - CL) & 1]);
          recompute_step(j, fi[(j - CL) & 1], sv[j - CL]);
        }

        // the segment's reverse steps
        // reverse step inputs: the lane's y row, lane 63's lower neighbours
        // and, for the steps whose cell sums sit in LDS, those sums
        struct RevIn {
          float dy[DP];
          double lo[LW];
        };
        auto read_rev = [&](int j, RevIn& in) {
          get_dy(j, in.dy);
#pragma unroll
          for (int f = 0; f < LW; ++f) in.lo[f] = sl[j * LW + f];
        };
        auto read_sums = [&](int j, float (&sj)[RS]) {
#pragma unroll
          for (int e = 0; e < G4; ++e) {
            const float4 f = lds[(j * G4 + e) * 64 + lane];
            sj[4 * e] = f.x;
            sj[4 * e + 1] = f.y;
            sj[4 * e + 2] = f.z;
            sj[4 * e + 3] = f.w;
          }
        };
        auto rev_step = [&](const int j, const RevIn& in, const float(&sj)[RS]) {
          const float(&dy)[DP] = in.dy;
          const double(&lo)[LW] = in.lo;
          float h32[CR];
#pragma unroll
          for (int c = 0; c < CR; ++c) {
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) s = __builtin_fmaf(dx[c][k], dy[k], s);
            h32[c] = s;
          }
          double ab[S];  // lane l+1's top-row a (lane 63: the band below's)
#pragma unroll
          for (int cc = 0; cc < S; ++cc) ab[cc] = from_next_lane(pubA[cc], lo[cc]);
          // the coarse row below the strip is lane l+1's first one (R >= S), or
          // with R < S the lane's own or the next lane's (cb_below)
          const float hb = from_next_lane(hpub, (float)lo[S]);
          double ych[DYA];
#pragma unroll
          for (int k = 0; k < DY; ++k) ych[k] = from_next_lane(ypub[k], lo[S + 1 + k]);
          if ((pe >> j) & 1u) {  // last column of a pair: nothing to the right
#pragma unroll
            for (int r = 0; r < R; ++r) ar[r] = 0.0;
            // the terminal cell (lane 63 of the last band, last row) receives
            // the seed through its below-right neighbour: a = 0 + 0 - (-w)
            prev_ab0 = (last && lane == 63) ? -pair_weight(a, ia, b0 + (g0 + j) / n) : 0.0;
          }
          double gk[CR];
#pragma unroll
          for (int c = 0; c < CR; ++c) gk[c] = 1.0 + (double)h32[c];
          const double gbelow = (R >= S || cb_below) ? 1.0 + (double)hb : gk[0];
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
              const double belowv = (r == R - 1) ? ab[cc] : v[r + 1][cc];
              const double gB = (r == R - 1) ? gbelow : gk[(R >= S) ? ((r + 1) >> LAM) : 0];
              const double diag = (r == R - 1) ? ((cc == S - 1) ? prev_ab0 : ab[cc + 1])
                                               : ((cc == S - 1) ? ar[r + 1] : v[r + 1][cc + 1]);
              v[r][cc] = __builtin_fma(gR, right, __builtin_fma(gB, belowv, -diag));
            }
          }
          // coefficient gradients of the strip's coarse cells, contracted
          double dg[CR];
#pragma unroll
          for (int c = 0; c < CR; ++c) dg[c] = 0.0;
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int cc = 0; cc < S; ++cc) {
              const int c = (R >= S) ? (r >> LAM) : 0;
              dg[c] = __builtin_fma(v[r][cc], (double)sj[r * S + cc], dg[c]);
            }
          double ypart[DYA];
#pragma unroll
          for (int k = 0; k < DY; ++k) ypart[k] = 0.0;
#pragma unroll
          for (int c = 0; c < CR; ++c) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
              dxacc[c][k] = __builtin_fma(dg[c], (double)dy[k], dxacc[c][k]);
              if (k < DY) ypart[k] = __builtin_fma(dg[c], dxd[c][k], ypart[k]);
            }
          }
#pragma unroll
          for (int k = 0; k < DY; ++k) ypub[k] = ych[k] + ypart[k];
          // lane 0's outputs: for the band above, and the y-side sums
          if (lane == 0) {
#pragma unroll
            for (int cc = 0; cc < S; ++cc) sw[j * LW + cc] = v[0][cc];
            sw[j * LW + S] = (double)h32[0];
#pragma unroll
            for (int k = 0; k < DY; ++k) sw[j * LW + S + 1 + k] = ypub[k];
          }
          hpub = h32[0];
#pragma unroll
          for (int cc = 0; cc < S; ++cc) pubA[cc] = v[0][cc];
          prev_ab0 = ab[0];
#pragma unroll
          for (int r = 0; r < R; ++r) ar[r] = v[r][0];
#pragma unroll
          for (int c = 0; c < CR; ++c) gr[c] = gk[c];
        };
        // inputs read one step ahead, alternating two buffers
        RevIn ri[2];
        float sr[2][RS];
        read_rev(C - 1, ri[0]);
#pragma unroll
        for (int j = C - 1; j >= CL; --j) {
          const int b = (C - 1 - j) & 1;
          __builtin_amdgcn_sched_barrier(0);
          read_rev(j - 1, ri[b ^ 1]);
          if (j == CL) read_sums(j - 1, sr[b ^ 1]);
          rev_step(j, ri[b], sv[j - CL]);
        }
        // the next segment's staging and checkpoint, loaded while the steps
        // whose cell sums sit in LDS run (the registers are free by now)
        if (seg > 0) {
          fetch_y(seg - 1, py);
          fetch_up(seg - 1, top, above, pb);
          fetch_low(seg - 1, pl);
          fetch_ck(seg - 1, pk);
        }
        // steps CL - 1 .. 0, two per iteration; the first one's inputs are in
        // buffer (C - CL) & 1, the read before step 0 re-reads step 0
        {
          constexpr int kb = (C - CL) & 1;
#pragma unroll 1
          for (int j = CL - 1; j >= 1; j -= 2) {
            __builtin_amdgcn_sched_barrier(0);
            read_rev(j - 1, ri[kb ^ 1]);
            read_sums(j - 1, sr[kb ^ 1]);
            rev_step(j, ri[kb], sr[kb]);
            __builtin_amdgcn_sched_barrier(0);
            const int jn = j >= 2 ? j - 2 : 0;
            read_rev(jn, ri[kb]);
            read_sums(jn, sr[kb]);
            rev_step(j - 1, ri[kb ^ 1], sr[kb ^ 1]);
          }
          if constexpr (CL & 1) {
            __builtin_amdgcn_sched_barrier(0);
            rev_step(0, ri[kb], sr[kb]);
          }
        }
        // lane 0's outputs at columns t0 .. t0 + C - 1: the y-side sums of the
        // band's rows (final for the top band) and, for the band above, the
        // top-row a values and coefficients
        __syncthreads();
        for (int e = lane; e < NL; e += 64) {
          const int j = e / LW, f = e - j * LW;
          const int32_t col = t0 + j;
          if ((uint32_t)col < (uint32_t)total) {
            if (!YS || f <= S) {
              if (!top) at(abw, (uint32_t)(col * (S + 1) + f)) = sw[e];
            } else {
              const int32_t bq = col / n, qq = col - bq * n;
              at(pyt, (uint32_t)((bq * a.nrows + qq) * D + (f - S - 1))) = sw[e];
            }
          }
        }
      }

      // x-side increment gradients of the band's coarse rows
      if constexpr (R < S) {
        // S / R consecutive lanes (aligned groups) share one coarse row
        constexpr int G = S / R;
#pragma unroll
        for (int o = 1; o < G; o <<= 1)
#pragma unroll
          for (int k = 0; k < D; ++k) dxacc[0][k] += __shfl_xor(dxacc[0][k], o, 64);
      }
      const bool writer = (R >= S) || (lane % ((R < S) ? (S / R) : 1) == 0);
#pragma unroll
      for (int c = 0; c < CR; ++c) {
        const int p = p0 + c;
        if (writer && p >= 0 && p < m) {
#pragma unroll
          for (int k = 0; k < D; ++k) px[(int64_t)p * D + k] = dxacc[c][k];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    // rows of px beyond this path's increments (ragged batches) are never read
  }
}

}  // namespace grad
}  // namespace sk
