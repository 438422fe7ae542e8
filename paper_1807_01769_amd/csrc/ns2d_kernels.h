// ns2d_kernels.h -- kernels of the 2D vorticity-form step.
//
// State: w_hat[N][N/2+1] (ky, kx).  Velocity from vorticity through the
// stream function (w = -lap psi, u = d psi/dy, v = -d psi/dx):
//   u_hat = i ky w_hat / |k|^2,  v_hat = -i kx w_hat / |k|^2  (0 at k = 0),
// tendency in conservative form N = -div(u w):
//   N_hat = -i kx (u w)^ - i ky (v w)^,  N_hat(0) = 0, 2/3-rule cube mask.
// One tendency evaluation is two passes over memory:
//   Y (fwd + inv)  forward y transforms of (u w, v w) -> N -> Lawson RK4
//                  combine -> next stage input -> (u, v, w) -> three inverse
//                  y transforms                               [k2_y]
//   X (c2r / r2c)  three C2R, products, two R2C               [k2_x]
// With NF = 2 the state also holds the buoyancy b_hat (Boussinesq flow in
// the vertical plane, gravity along -y, N2 the squared Brunt-Vaisala
// frequency):  N_w += -div(u w) + i kx b_hat,  N_b = -div(u b) - N2 v_hat;
// the passes then carry (u, v, w, b) and (u w, v w, u b, v b), and the y pass
// keeps every stage input in `a.sin` for the linear coupling terms.
//
// Every kernel works on a batch of equal-size runs: block b handles part
// b % bpr of local run b / bpr; the run's state sits at state_off[run] in
// a packed array (offset 0 without a table) and its workspace at
// run * stride.  A single plan is the batch of one run.
//
// Y passes use LB lines (kx columns) per block, LB * N/8 threads, line
// mx = part * LB + b of the padded kx range [0, 16 XT); X passes use RP row
// pairs per block, RP * N/8 threads.
#pragma once
#include <type_traits>

#include "ns_common.h"

namespace fs {

struct Batch {
  const long long* state_off;  // per-run state offsets (complex elements) or null
  size_t in_stride, out_stride, acc_stride;  // per-run workspace strides
  int bpr;                     // blocks per run
};

// inverse y transforms of (u, v, w[, b]) derived from the stage input held
// as w[0][e] (and b = w[1][e]) at y-position t + e*P of line b (kx = mx);
// writes Wn[3 or 4][XT][N][16]
template <typename T, int N, int LB, int NF, class TW>
__device__ __forceinline__ void y_inverse_fields(cx<T> (&w)[NF][8], int t, int b, int mx, T kb,
                                                 cx<T>* __restrict__ w1, cx<T>* lds,
                                                 const TW& tw) {
  using G = Geo<N, false>;
  constexpr int P = G::P;
  const size_t fstride = (size_t)G::XT * N * kTile;
  cx<T>* dst0 = w1 + (size_t)(mx >> 4) * N * kTile + (mx & 15);
  auto lidx = [=](int, int pos) { return pos * LB + b; };
  const T kx = kb * (T)mx;
#pragma unroll
  for (int f = 0; f < 2 + NF; f++) {
    cx<T> v[1][8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int iy = t + e * P;
      const T ky = kb * (T)(iy <= N / 2 ? iy : iy - N);
      const T k2 = kx * kx + ky * ky;
      const T ik2 = k2 > (T)0 ? (T)1 / k2 : (T)0;
      if (f == 0) v[0][e] = mul_i(cscale(w[0][e], ky * ik2));
      else if (f == 1) v[0][e] = mul_i(cscale(w[0][e], -kx * ik2));
      else v[0][e] = w[f - 2][e];
    }
    fft_lines<T, N, +1, 1>(v, t, lds, lidx, tw);
    cx<T>* dst = dst0 + f * fstride;
#pragma unroll
    for (int e = 0; e < 8; e++) dst[(size_t)(t + e * P) * kTile] = v[0][e];
  }
}

// First pass of a stage from the state: W1 = inverse y transforms of
// (u, v, w).  Grid: runs * bpr, bpr = 16 XT / LB.
template <typename T, int N, int LB, int NF = 1>
__global__ void __launch_bounds__(LB * N / 8)
    k2_p1(const cx<T>* __restrict__ state, cx<T>* __restrict__ w1, StageArgs<T> a, Batch bt) {
  using G = Geo<N, false>;
  constexpr int P = G::P, NH = N / 2 + 1;
  __shared__ cx<T> lds[LB * N];
  const int b = threadIdx.x % LB, t = threadIdx.x / LB;
  const Twiddles<T, N> twr(a.tw, t);
  const int run = blockIdx.x / bt.bpr, part = blockIdx.x % bt.bpr;
  state += bt.state_off ? bt.state_off[run] : 0;
  w1 += run * bt.out_stride;
  const int mx = part * LB + b;
  cx<T> w[NF][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int iy = t + e * P;
    const int jy = G::i2j(iy);
    const bool kept = mx < G::H && jy >= 0;
#pragma unroll
    for (int f = 0; f < NF; f++) {
      w[f][e] = kept ? state[(size_t)f * N * NH + (size_t)iy * NH + mx] : cx<T>{0, 0};
      if (NF > 1 && kept)
        a.sin[((size_t)f * G::XT * G::M + (size_t)(mx >> 4) * G::M + jy) * kTile + (mx & 15)] =
            w[f][e];
    }
  }
  y_inverse_fields<T, N, LB, NF>(w, t, b, mx, a.kb, w1, lds, twr);
}

// X pass: rows (y0, y0+1); in Wn[3 or 4][XT][N][16] (u, v, w[, b]), out
// Wn[2 or 4][XT][N][16] ((u w), (v w)[, (u b), (v b)]) scaled by `scale`.
// With umax, the largest |u|, |v| is max-reduced into *umax.
// Grid: runs * bpr, bpr = N/2/RP.
template <typename T, int N, int RP, int NF = 1>
__global__ void __launch_bounds__(RP * N / 8)
    k2_x(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ tw,
         T scale, Batch bt, unsigned long long* __restrict__ umax) {
  using G = Geo<N, false>;
  using R = RowPairs<N>;
  constexpr int P = G::P;
  constexpr int NL = 2 + NF;  // inverse lines: (u, v) of each row, (w[, b]) of both rows
  // plain flow transforms one line at a time (one line of LDS per row pair,
  // fewer registers, more waves per CU); with buoyancy the lines go together
  constexpr int NLDS = NF == 1 ? 1 : NL;
  __shared__ cx<T> lds[RP * NLDS * R::NPAD];
  __shared__ cx<T> stage[NF == 1 ? RP * 6 * G::XT * kTile : 1];
  const int rp = threadIdx.x / P, t = threadIdx.x % P;
  const Twiddles<T, N> twr(tw, t);
  const int run = blockIdx.x / bt.bpr, part = blockIdx.x % bt.bpr;
  in += run * bt.in_stride;
  out += run * bt.out_stride;
  const int y0 = 2 * (part * RP + rp);
  cx<T>* my_lds = lds + rp * NLDS * R::NPAD;
  auto lidx = [=](int f, int pos) { return f * R::NPAD + R::pad(pos); };
  const size_t fstride = (size_t)G::XT * N * kTile;
  auto at = [=](int f, int y, int m) -> cx<T> {
    return in[f * fstride + ((size_t)(m >> 4) * N + y) * kTile + (m & 15)];
  };
  if constexpr (NF == 1) {
    // The pair's kept coefficients of u, v, w (for each field, row and tile
    // 16 contiguous values) are staged in LDS with 16-byte loads, all in
    // flight; then (w(y0) + i w(y1)), and per row (u + i v) and its products
    // (u w, v w) forward-transformed as one line and untangled.
    constexpr int SROW = G::XT * kTile;  // one field of one row
    cx<T>* stg = stage + rp * 6 * SROW;
    {
      constexpr int PER = 16 / (int)sizeof(cx<T>);
      constexpr int LOADS = 6 * SROW / PER;
      const uint4* src4 = reinterpret_cast<const uint4*>(in);
      uint4* st4 = reinterpret_cast<uint4*>(stg);
#pragma unroll
      for (int i0 = 0; i0 < LOADS; i0 += P) {
        const int i = i0 + t;
        if (i < LOADS) {
          const int c = i / (kTile / PER), lo = i % (kTile / PER);
          const int fr = c / G::XT, xt = c % G::XT;  // fr = 2 f + r
          const size_t g = (fr / 2) * fstride + ((size_t)xt * N + y0 + fr % 2) * kTile;
          st4[c * (kTile / PER) + lo] = src4[g / PER + lo];
        }
      }
      __syncthreads();
    }
    auto sat = [=](int f, int r) { return stg + (2 * f + r) * SROW; };
    cx<T> v[1][8];
#pragma unroll
    for (int e = 0; e < 8; e++)
      v[0][e] = c2r_pair_at<T, N, false>(t + e * P, [&](int m) { return sat(2, 0)[m]; },
                                         [&](int m) { return sat(2, 1)[m]; });
    fft_lines<T, N, +1, 1>(v, t, my_lds, lidx, twr);
    T ws[2][8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
      ws[0][e] = v[0][e].re * scale;
      ws[1][e] = v[0][e].im * scale;
    }
    double um = 0.0;
#pragma unroll
    for (int r = 0; r < 2; r++) {
#pragma unroll
      for (int e = 0; e < 8; e++)
        v[0][e] = c2r_pair_at<T, N, false>(t + e * P, [&](int m) { return sat(0, r)[m]; },
                                           [&](int m) { return sat(1, r)[m]; });
      fft_lines<T, N, +1, 1>(v, t, my_lds, lidx, twr);
#pragma unroll
      for (int e = 0; e < 8; e++) {
        if (umax) um = fmax(um, (double)fmax(fabs(v[0][e].re), fabs(v[0][e].im)));
        v[0][e] = {v[0][e].re * ws[r][e], v[0][e].im * ws[r][e]};
      }
      fft_lines<T, N, -1, 1>(v, t, my_lds, lidx, twr);
#pragma unroll
      for (int e = 0; e < 8; e++) my_lds[lidx(0, t + e * P)] = v[0][e];
      __syncthreads();
      for (int m = t; m < G::XT * kTile; m += P) {
        const size_t o = ((size_t)(m >> 4) * N + (y0 + r)) * kTile + (m & 15);
        cx<T> A = {0, 0}, B = {0, 0};
        if (m < G::H) r2c_untangle(my_lds[lidx(0, m)], my_lds[lidx(0, (N - m) & (N - 1))], A, B);
        out[o] = A;
        out[fstride + o] = B;
      }
      __syncthreads();
    }
    if (umax) umax_wave(umax, um);
    return;
  }
  cx<T> v[NL][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int k = t + e * P;
    v[0][e] = c2r_pair_at<T, N, false>(k, [&](int m) { return at(0, y0, m); },
                                       [&](int m) { return at(1, y0, m); });
    v[1][e] = c2r_pair_at<T, N, false>(k, [&](int m) { return at(0, y0 + 1, m); },
                                       [&](int m) { return at(1, y0 + 1, m); });
#pragma unroll
    for (int f = 0; f < NF; f++)
      v[2 + f][e] = c2r_pair_at<T, N, false>(k, [&](int m) { return at(2 + f, y0, m); },
                                             [&](int m) { return at(2 + f, y0 + 1, m); });
  }
  fft_lines<T, N, +1, NL>(v, t, my_lds, lidx, twr);
  if (umax) {
    double um = 0.0;
#pragma unroll
    for (int e = 0; e < 8; e++)
      um = fmax(um, (double)fmax(fmax(fabs(v[0][e].re), fabs(v[0][e].im)),
                                 fmax(fabs(v[1][e].re), fabs(v[1][e].im))));
    umax_wave(umax, um);
  }
  // product lines: (u s, v s) of row y0 and of row y1 for s = w[, b]
  cx<T> q[2 * NF][8];
#pragma unroll
  for (int f = 0; f < NF; f++)
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const T s0 = v[2 + f][e].re * scale, s1 = v[2 + f][e].im * scale;
      q[2 * f][e] = {v[0][e].re * s0, v[0][e].im * s0};
      q[2 * f + 1][e] = {v[1][e].re * s1, v[1][e].im * s1};
    }
  fft_lines<T, N, -1, 2 * NF>(q, t, my_lds, lidx, twr);
#pragma unroll
  for (int f = 0; f < 2 * NF; f++)
#pragma unroll
    for (int e = 0; e < 8; e++) my_lds[lidx(f, t + e * P)] = q[f][e];
  __syncthreads();
  for (int m = t; m < G::XT * kTile; m += P) {
    const size_t o = ((size_t)(m >> 4) * N) * kTile + (m & 15);
#pragma unroll
    for (int l = 0; l < 2 * NF; l++) {
      const int r = l & 1, fo = 2 * (l >> 1);  // row, first output field of the line
      cx<T> A = {0, 0}, B = {0, 0};
      if (m < G::H) r2c_untangle(my_lds[lidx(l, m)], my_lds[lidx(l, (N - m) & (N - 1))], A, B);
      out[fo * fstride + o + (size_t)(y0 + r) * kTile] = A;
      out[(fo + 1) * fstride + o + (size_t)(y0 + r) * kTile] = B;
    }
  }
}

// Y pass: forward y transforms of the products, tendency, Lawson combine and
// the next stage's inverse transforms.  acc: [NF][XT][M][16] per run; with
// NF = 2, a.sin [2][XT][M][16] holds the stage input (read for the coupling
// terms, then replaced by the next stage input).
// Grid: runs * bpr, bpr = 16 XT / LB.
template <typename T, int N, int LB, int MODE, int NF = 1>
__global__ void __launch_bounds__(LB * N / 8)
    k2_y(const cx<T>* __restrict__ w2, cx<T>* __restrict__ w1, StageArgs<T> a, Batch bt,
         int do_p1) {
  using G = Geo<N, false>;
  constexpr int P = G::P, NH = N / 2 + 1;
  constexpr size_t kField = (size_t)G::XT * G::M * kTile;  // one compact field
  __shared__ cx<T> lds[LB * N];
  const int b = threadIdx.x % LB, t = threadIdx.x / LB;
  const Twiddles<T, N> twr(a.tw, t);
  const int run = blockIdx.x / bt.bpr, part = blockIdx.x % bt.bpr;
  w2 += run * bt.in_stride;
  w1 += run * bt.out_stride;
  const size_t soff = bt.state_off ? bt.state_off[run] : 0;
  const int mx = part * LB + b;
  auto lidx = [=](int, int pos) { return pos * LB + b; };
  const size_t fstride = (size_t)G::XT * N * kTile;
  const cx<T>* src = w2 + (size_t)(mx >> 4) * N * kTile + (mx & 15);
  cx<T> f[2 * NF][1][8];
#pragma unroll
  for (int c = 0; c < 2 * NF; c++)
#pragma unroll
    for (int e = 0; e < 8; e++) f[c][0][e] = src[c * fstride + (size_t)(t + e * P) * kTile];
#pragma unroll
  for (int c = 0; c < 2 * NF; c++) fft_lines<T, N, -1, 1>(f[c], t, lds, lidx, twr);

  const T kx = a.kb * (T)mx;
  const T dt = stage_dt(a);
  cx<T> w[NF][8];
  bool bad = false;  // a non-finite value written to the state
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int iy = t + e * P;
    const int jy = G::i2j(iy);
    if (!(mx < G::H && jy >= 0)) {
#pragma unroll
      for (int c = 0; c < NF; c++) w[c][e] = {0, 0};
      continue;
    }
    const int my = iy <= N / 2 ? iy : iy - N;
    const T ky = a.kb * (T)my;
    const size_t ci = ((size_t)(mx >> 4) * G::M + jy) * kTile + (mx & 15);
    cx<T> nl[NF];
#pragma unroll
    for (int c = 0; c < NF; c++) nl[c] = {0, 0};
    if (mx != 0 || my != 0) {
#pragma unroll
      for (int c = 0; c < NF; c++)
        nl[c] = mul_i(cscale(f[2 * c][0][e], -kx) - cscale(f[2 * c + 1][0][e], ky));
      if constexpr (NF == 2) {
        const cx<T> ws = a.sin[ci], bs = a.sin[kField + ci];
        const T k2 = kx * kx + ky * ky;
        nl[0] = nl[0] + mul_i(cscale(bs, kx));                // + d b / dx
        nl[1] = nl[1] + mul_i(cscale(ws, a.n2 * kx / k2));    // - N2 v
      }
    }
    const size_t so = soff + (size_t)iy * NH + mx;
    if constexpr (MODE == kModeTend) {
#pragma unroll
      for (int c = 0; c < NF; c++) a.tend[(size_t)c * N * NH + so] = nl[c];
    } else {
      const T E = a.e1[mx] * a.e1[iy];
      const T Eh = a.eh1[mx] * a.eh1[iy];
      const size_t ao = run * bt.acc_stride + ci;
#pragma unroll
      for (int c = 0; c < NF; c++) {
        cx<T> acc = {0, 0}, u = {0, 0};
        if constexpr (mode_reads_state(MODE)) u = a.state[(size_t)c * N * NH + so];
        if constexpr (mode_reads_acc(MODE)) acc = a.acc[c * kField + ao];
        const cx<T> nxt = rk4_combine<MODE>(u, acc, nl[c], E, Eh, dt);
        if constexpr (mode_writes_state(MODE)) {
          a.state[(size_t)c * N * NH + so] = nxt;
          bad |= nonfinite(nxt);
        }
        if constexpr (mode_writes_acc(MODE)) a.acc[c * kField + ao] = acc;
        if constexpr (NF == 2) a.sin[c * kField + ci] = nxt;
        w[c][e] = nxt;
      }
    }
  }
  if constexpr (mode_writes_state(MODE)) {
    if (a.nonfin) flag_wave(a.nonfin, bad);
  }
  if constexpr (MODE != kModeTend) {
    if (do_p1) y_inverse_fields<T, N, LB, NF>(w, t, b, mx, a.kb, w1, lds, twr);
  }
}

// ---------------------------------------------------------------------------
// Block-resident steps of small plain-flow runs (an ensemble's small size
// classes).  Up to N = 128 the (kx, y) intermediate of a run -- u, v, w at the
// kept kx, 3 x N x H complex values (132 KB at 128) -- fits in LDS next to one
// transform line per lane group, so one block advances one run through all
// the steps of a call and goes to HBM only for the state and the accumulator
// (29 KB each at 128, which stay in L2).  Each stage is the x pass and the y
// pass of k2_x / k2_y done in turn on the block's LDS:
//   x phase: per row pair, C2R of (w(y0) + i w(y1)) and of (u + i v) of each
//            row, the products, R2C of (u w + i v w), untangled and written
//            over u and v of that row;
//   y phase: per kx column, forward y of (u w, v w), tendency, Lawson combine,
//            and the inverse y transforms of the next input's u, v, w, each
//            line using its own column slot as its exchange space.
// The operations of the two kernels, in their order: the runs end where the
// class-batched passes leave them up to rounding (the compiler may contract
// multiply-adds differently in the two kernels).
// LDS rows have an odd stride S >= H (column accesses of a wave's 16
// positions then fall in distinct banks).  Grid: one block per run.
// ---------------------------------------------------------------------------
template <int N>
struct Resident {
  static constexpr int P = N / 8;
  static constexpr int H = Geo<N, false>::H;
  static constexpr int S = H | 1;
  // line groups: as many as the intermediate leaves LDS for (one padded
  // exchange line each)
  static constexpr int GROUPS = N == 128 ? 24 : 32;
  static constexpr int THREADS = GROUPS * P;
  static constexpr int NPAD = RowPairs<N>::NPAD;
  static constexpr size_t kLds = (size_t)(3 * N * S + GROUPS * NPAD) * sizeof(cx<float>);
  static constexpr bool kFits = N <= 128 && kLds <= 163840;
};

template <int N>
__global__ void __launch_bounds__((Resident<N>::THREADS))
    k2_resident(StageArgs<float> a, Batch bt, int steps) {
  using T = float;
  using G = Geo<N, false>;
  using RS = Resident<N>;
  static_assert(RS::kFits, "a run does not fit one block's LDS");
  constexpr int P = G::P, NH = N / 2 + 1, S = RS::S, H = G::H;
  // [field u v w][y][kx < S], then one exchange line per group: one array,
  // so that a transform can take either as its exchange space through its
  // index map alone (no branch around the barriers inside)
  constexpr int kX = 3 * N * S;
  __shared__ cx<T> buf[kX + RS::GROUPS * RS::NPAD];
  const int g = threadIdx.x / P;
  // t and kb are laundered at the start of every phase (relaunder): what
  // derives from them is then recomputed per phase instead of being hoisted
  // out of the step loop and held in registers through all of it
  int t = threadIdx.x % P;
  T kb = a.kb;
  auto relaunder = [&]() { asm volatile("" : "+v"(t), "+s"(kb)); };
  const Twiddles<T, N> twr(a.tw, t);
  const int run = blockIdx.x;
  const size_t soff = bt.state_off ? bt.state_off[run] : 0;
  const int xo = kX + g * RS::NPAD;  // this group's exchange line
  cx<T>* const myx = buf + xo;
  auto row = [&](int f, int y) { return buf + (f * N + y) * S; };
  // exchange space of line f of column mx: its own slot in the intermediate
  // (act) or the group's exchange line
  auto col_idx = [=](int f, int mx, bool act) {
    return [=](int, int pos) { return act ? (f * N + pos) * S + mx : xo + RowPairs<N>::pad(pos); };
  };
  const T scale = (T)(1.0 / ((double)N * N));
  const T dt = stage_dt(a);

  // inverse y transforms of (u, v, w) of the stage input w0 at column mx into
  // the column's slots (or, for a group past the last column, through its
  // exchange line with nothing stored)
  auto y_inverse = [&](const cx<T> (&w0)[8], int mx, bool act) {
    const T kx = kb * (T)mx;
#pragma unroll
    for (int f = 0; f < 3; f++) {
      cx<T> v[1][8];
#pragma unroll
      for (int e = 0; e < 8; e++) {
        const int iy = t + e * P;
        const T ky = kb * (T)(iy <= N / 2 ? iy : iy - N);
        const T k2 = kx * kx + ky * ky;
        const T ik2 = k2 > (T)0 ? (T)1 / k2 : (T)0;
        if (f == 0) v[0][e] = mul_i(cscale(w0[e], ky * ik2));
        else if (f == 1) v[0][e] = mul_i(cscale(w0[e], -kx * ik2));
        else v[0][e] = w0[e];
      }
      fft_lines<T, N, +1, 1>(v, t, buf, col_idx(f, mx, act), twr);
      if (act) {
#pragma unroll
        for (int e = 0; e < 8; e++) row(f, t + e * P)[mx] = v[0][e];
      }
    }
  };

  // first inverse pass of the call, from the state
  for (int c0 = 0; c0 < H; c0 += RS::GROUPS) {
    const int mx = c0 + g;
    const bool act = mx < H;
    cx<T> w0[8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int iy = t + e * P;
      w0[e] = act && G::i2j(iy) >= 0 ? a.state[soff + (size_t)iy * NH + mx] : cx<T>{0, 0};
    }
    y_inverse(w0, mx, act);
  }
  __syncthreads();

  auto x_phase = [&]() {
    relaunder();
    auto lidx = [=](int, int pos) { return RowPairs<N>::pad(pos); };
    for (int p0 = 0; p0 < N / 2; p0 += RS::GROUPS) {
      const int p = p0 + g;
      const bool act = p < N / 2;
      const int y0 = act ? 2 * p : 0;  // a spare group transforms rows 0, 1 and stores nothing
      cx<T> v[1][8];
#pragma unroll
      for (int e = 0; e < 8; e++)
        v[0][e] = c2r_pair_at<T, N, false>(t + e * P, [&](int m) { return row(2, y0)[m]; },
                                           [&](int m) { return row(2, y0 + 1)[m]; });
      fft_lines<T, N, +1, 1>(v, t, myx, lidx, twr);
      T ws[2][8];
#pragma unroll
      for (int e = 0; e < 8; e++) {
        ws[0][e] = v[0][e].re * scale;
        ws[1][e] = v[0][e].im * scale;
      }
#pragma unroll
      for (int r = 0; r < 2; r++) {
#pragma unroll
        for (int e = 0; e < 8; e++)
          v[0][e] = c2r_pair_at<T, N, false>(t + e * P, [&](int m) { return row(0, y0 + r)[m]; },
                                             [&](int m) { return row(1, y0 + r)[m]; });
        fft_lines<T, N, +1, 1>(v, t, myx, lidx, twr);
#pragma unroll
        for (int e = 0; e < 8; e++) v[0][e] = {v[0][e].re * ws[r][e], v[0][e].im * ws[r][e]};
        fft_lines<T, N, -1, 1>(v, t, myx, lidx, twr);
#pragma unroll
        for (int e = 0; e < 8; e++) myx[lidx(0, t + e * P)] = v[0][e];
        __syncthreads();
        if (act) {
          for (int m = t; m < H; m += P) {
            cx<T> A, B;
            r2c_untangle(myx[lidx(0, m)], myx[lidx(0, (N - m) & (N - 1))], A, B);
            row(0, y0 + r)[m] = A;
            row(1, y0 + r)[m] = B;
          }
        }
        __syncthreads();
      }
    }
  };

  auto y_phase = [&](auto mode_c, bool do_inv) {
    constexpr int MODE = decltype(mode_c)::value;
    relaunder();
    bool bad = false;  // a non-finite value written to the state
    for (int c0 = 0; c0 < H; c0 += RS::GROUPS) {
      const int mx = c0 + g;
      const bool act = mx < H;
      const int ml = act ? mx : 0;
      cx<T> f[2][1][8];
#pragma unroll
      for (int c = 0; c < 2; c++)
#pragma unroll
        for (int e = 0; e < 8; e++) f[c][0][e] = row(c, t + e * P)[ml];
#pragma unroll
      for (int c = 0; c < 2; c++) fft_lines<T, N, -1, 1>(f[c], t, buf, col_idx(c, mx, act), twr);
      const T kx = kb * (T)mx;
      cx<T> w0[8];
#pragma unroll
      for (int e = 0; e < 8; e++) {
        const int iy = t + e * P;
        const int jy = G::i2j(iy);
        if (!(act && jy >= 0)) {
          w0[e] = {0, 0};
          continue;
        }
        const int my = iy <= N / 2 ? iy : iy - N;
        const T ky = kb * (T)my;
        const size_t ci = ((size_t)(mx >> 4) * G::M + jy) * kTile + (mx & 15);
        cx<T> nl = {0, 0};
        if (mx != 0 || my != 0) nl = mul_i(cscale(f[0][0][e], -kx) - cscale(f[1][0][e], ky));
        const size_t so = soff + (size_t)iy * NH + mx;
        const T E = a.e1[mx] * a.e1[iy];
        const T Eh = a.eh1[mx] * a.eh1[iy];
        const size_t ao = run * bt.acc_stride + ci;
        cx<T> acc = {0, 0}, u = {0, 0};
        if constexpr (mode_reads_state(MODE)) u = a.state[so];
        if constexpr (mode_reads_acc(MODE)) acc = a.acc[ao];
        const cx<T> nxt = rk4_combine<MODE>(u, acc, nl, E, Eh, dt);
        if constexpr (mode_writes_state(MODE)) {
          a.state[so] = nxt;
          bad |= nonfinite(nxt);
        }
        if constexpr (mode_writes_acc(MODE)) a.acc[ao] = acc;
        w0[e] = nxt;
      }
      if (do_inv) y_inverse(w0, mx, act);
    }
    if constexpr (mode_writes_state(MODE)) {
      if (a.nonfin) flag_wave(a.nonfin, bad);
    }
  };

  for (int k = 0; k < steps; k++) {
    const bool more = k + 1 < steps;
    x_phase();
    y_phase(std::integral_constant<int, kStage1>{}, true);
    __syncthreads();
    x_phase();
    y_phase(std::integral_constant<int, kStage2>{}, true);
    __syncthreads();
    x_phase();
    y_phase(std::integral_constant<int, kStage3>{}, true);
    __syncthreads();
    x_phase();
    y_phase(std::integral_constant<int, kStage4>{}, more);
    __syncthreads();
  }
}

// Plain 2D transforms for the FFT entry points.
// spec [N][N/2+1] -> Wn(FULL)[XT][N][16] (inverse y); grid XT * SUB
template <typename T, int N>
__global__ void __launch_bounds__((Strided<T, N>::THREADS))
    k2f_y_inv(const cx<T>* __restrict__ spec, cx<T>* __restrict__ w, const cx<T>* __restrict__ tw) {
  using G = Geo<N, true>;
  using C = Strided<T, N>;
  constexpr int P = G::P, NH = N / 2 + 1;
  __shared__ cx<T> lds[C::LB * N];
  const int b = threadIdx.x % C::LB, t = threadIdx.x / C::LB;
  const Twiddles<T, N, false> twr(tw, t);
  const int sub = blockIdx.x % C::SUB, xt = blockIdx.x / C::SUB;
  const int mx = xt * kTile + sub * C::LB + b;
  cx<T> v[1][8];
#pragma unroll
  for (int e = 0; e < 8; e++)
    v[0][e] = mx < G::H ? spec[(size_t)(t + e * P) * NH + mx] : cx<T>{0, 0};
  fft_lines<T, N, +1, 1>(v, t, lds, [=](int, int pos) { return pos * C::LB + b; }, twr);
  cx<T>* dst = w + (size_t)xt * N * kTile + sub * C::LB + b;
#pragma unroll
  for (int e = 0; e < 8; e++) dst[(size_t)(t + e * P) * kTile] = v[0][e];
}

// Wn(FULL)[XT][N][16] -> spec [N][N/2+1] (forward y); grid XT * SUB
template <typename T, int N>
__global__ void __launch_bounds__((Strided<T, N>::THREADS))
    k2f_y_fwd(const cx<T>* __restrict__ w, cx<T>* __restrict__ spec, const cx<T>* __restrict__ tw) {
  using G = Geo<N, true>;
  using C = Strided<T, N>;
  constexpr int P = G::P, NH = N / 2 + 1;
  __shared__ cx<T> lds[C::LB * N];
  const int b = threadIdx.x % C::LB, t = threadIdx.x / C::LB;
  const Twiddles<T, N, false> twr(tw, t);
  const int sub = blockIdx.x % C::SUB, xt = blockIdx.x / C::SUB;
  const int mx = xt * kTile + sub * C::LB + b;
  const cx<T>* src = w + (size_t)xt * N * kTile + sub * C::LB + b;
  cx<T> v[1][8];
#pragma unroll
  for (int e = 0; e < 8; e++) v[0][e] = src[(size_t)(t + e * P) * kTile];
  fft_lines<T, N, -1, 1>(v, t, lds, [=](int, int pos) { return pos * C::LB + b; }, twr);
  if (mx < G::H) {
#pragma unroll
    for (int e = 0; e < 8; e++) spec[(size_t)(t + e * P) * NH + mx] = v[0][e];
  }
}

}  // namespace fs
