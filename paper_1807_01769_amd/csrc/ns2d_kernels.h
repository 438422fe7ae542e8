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
#include "ns_common.h"

namespace fs {

struct Batch {
  const long long* state_off;  // per-run state offsets (complex elements) or null
  size_t in_stride, out_stride, acc_stride;  // per-run workspace strides
  int bpr;                     // blocks per run
};

// three inverse y transforms of (u, v, w) derived from w_hat held as w[e]
// at y-position t + e*P of line b (kx = mx); writes Wn[3][XT][N][16]
template <typename T, int N, int LB, class TW>
__device__ __forceinline__ void y_inverse_three(cx<T> (&w)[8], int t, int b, int mx, T kb,
                                                cx<T>* __restrict__ w1, cx<T>* lds,
                                                const TW& tw) {
  using G = Geo<N, false>;
  constexpr int P = G::P;
  const size_t fstride = (size_t)G::XT * N * kTile;
  cx<T>* dst0 = w1 + (size_t)(mx >> 4) * N * kTile + (mx & 15);
  auto lidx = [=](int, int pos) { return pos * LB + b; };
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
      if (f == 0) v[0][e] = mul_i(cscale(w[e], ky * ik2));
      else if (f == 1) v[0][e] = mul_i(cscale(w[e], -kx * ik2));
      else v[0][e] = w[e];
    }
    fft_lines<T, N, +1, 1>(v, t, lds, lidx, tw);
    cx<T>* dst = dst0 + f * fstride;
#pragma unroll
    for (int e = 0; e < 8; e++) dst[(size_t)(t + e * P) * kTile] = v[0][e];
  }
}

// First pass of a stage from the state: W1 = inverse y transforms of
// (u, v, w).  Grid: runs * bpr, bpr = 16 XT / LB.
template <typename T, int N, int LB>
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
  cx<T> w[8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int iy = t + e * P;
    const bool kept = mx < G::H && G::i2j(iy) >= 0;
    w[e] = kept ? state[(size_t)iy * NH + mx] : cx<T>{0, 0};
  }
  y_inverse_three<T, N, LB>(w, t, b, mx, a.kb, w1, lds, twr);
}

// X pass: rows (y0, y0+1); in Wn[3][XT][N][16] (u, v, w), out Wn[2][XT][N][16]
// ((u w), (v w)) scaled by `scale`.  Grid: runs * bpr, bpr = N/2/RP.
template <typename T, int N, int RP>
__global__ void __launch_bounds__(RP * N / 8)
    k2_x(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ tw,
         T scale, Batch bt, unsigned long long* __restrict__ umax) {
  using G = Geo<N, false>;
  using R = RowPairs<N>;
  constexpr int P = G::P;
  __shared__ cx<T> lds[RP * 3 * R::NPAD];
  const int rp = threadIdx.x / P, t = threadIdx.x % P;
  const Twiddles<T, N> twr(tw, t);
  const int run = blockIdx.x / bt.bpr, part = blockIdx.x % bt.bpr;
  in += run * bt.in_stride;
  out += run * bt.out_stride;
  const int y0 = 2 * (part * RP + rp);
  cx<T>* my_lds = lds + rp * 3 * R::NPAD;
  auto lidx = [=](int f, int pos) { return f * R::NPAD + R::pad(pos); };
  const size_t fstride = (size_t)G::XT * N * kTile;
  auto at = [=](int f, int y, int m) -> cx<T> {
    return in[f * fstride + ((size_t)(m >> 4) * N + y) * kTile + (m & 15)];
  };
  cx<T> v[3][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int k = t + e * P;
    v[0][e] = c2r_pair_at<T, N, false>(k, [&](int m) { return at(0, y0, m); },
                                       [&](int m) { return at(1, y0, m); });
    v[1][e] = c2r_pair_at<T, N, false>(k, [&](int m) { return at(0, y0 + 1, m); },
                                       [&](int m) { return at(1, y0 + 1, m); });
    v[2][e] = c2r_pair_at<T, N, false>(k, [&](int m) { return at(2, y0, m); },
                                       [&](int m) { return at(2, y0 + 1, m); });
  }
  fft_lines<T, N, +1, 3>(v, t, my_lds, lidx, twr);
  if (umax) {
    double um = 0.0;
#pragma unroll
    for (int e = 0; e < 8; e++)
      um = fmax(um, (double)fmax(fmax(fabs(v[0][e].re), fabs(v[0][e].im)),
                                 fmax(fabs(v[1][e].re), fabs(v[1][e].im))));
    umax_wave(umax, um);
  }
  cx<T> q[2][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const T w0 = v[2][e].re * scale, w1 = v[2][e].im * scale;
    q[0][e] = {v[0][e].re * w0, v[0][e].im * w0};
    q[1][e] = {v[1][e].re * w1, v[1][e].im * w1};
  }
  fft_lines<T, N, -1, 2>(q, t, my_lds, lidx, twr);
#pragma unroll
  for (int f = 0; f < 2; f++)
#pragma unroll
    for (int e = 0; e < 8; e++) my_lds[lidx(f, t + e * P)] = q[f][e];
  __syncthreads();
  for (int m = t; m < G::XT * kTile; m += P) {
    const size_t o = ((size_t)(m >> 4) * N) * kTile + (m & 15);
#pragma unroll
    for (int r = 0; r < 2; r++) {
      cx<T> A = {0, 0}, B = {0, 0};
      if (m < G::H) r2c_untangle(my_lds[lidx(r, m)], my_lds[lidx(r, (N - m) & (N - 1))], A, B);
      out[o + (size_t)(y0 + r) * kTile] = A;
      out[fstride + o + (size_t)(y0 + r) * kTile] = B;
    }
  }
}

// Y pass: forward y transforms of (u w, v w), tendency, Lawson combine and the
// next stage's inverse transforms.  acc: [XT][M][16] per run.
// Grid: runs * bpr, bpr = 16 XT / LB.
template <typename T, int N, int LB, int MODE>
__global__ void __launch_bounds__(LB * N / 8)
    k2_y(const cx<T>* __restrict__ w2, cx<T>* __restrict__ w1, StageArgs<T> a, Batch bt,
         int do_p1) {
  using G = Geo<N, false>;
  constexpr int P = G::P, NH = N / 2 + 1;
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
  cx<T> f1[1][8], f2[1][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    f1[0][e] = src[(size_t)(t + e * P) * kTile];
    f2[0][e] = src[fstride + (size_t)(t + e * P) * kTile];
  }
  fft_lines<T, N, -1, 1>(f1, t, lds, lidx, twr);
  fft_lines<T, N, -1, 1>(f2, t, lds, lidx, twr);

  const T kx = a.kb * (T)mx;
  const T dt = stage_dt(a);
  cx<T> w[8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int iy = t + e * P;
    const int jy = G::i2j(iy);
    if (!(mx < G::H && jy >= 0)) {
      w[e] = {0, 0};
      continue;
    }
    const int my = iy <= N / 2 ? iy : iy - N;
    const T ky = a.kb * (T)my;
    cx<T> nl = {0, 0};
    if (mx != 0 || my != 0) nl = mul_i(cscale(f1[0][e], -kx) - cscale(f2[0][e], ky));
    const size_t so = soff + (size_t)iy * NH + mx;
    if constexpr (MODE == kModeTend) {
      a.tend[so] = nl;
    } else {
      const T E = a.e1[mx] * a.e1[iy];
      const T Eh = a.eh1[mx] * a.eh1[iy];
      const size_t ao = run * bt.acc_stride + ((size_t)(mx >> 4) * G::M + jy) * kTile + (mx & 15);
      cx<T> acc = {0, 0}, u = {0, 0};
      if constexpr (mode_reads_state(MODE)) u = a.state[so];
      if constexpr (mode_reads_acc(MODE)) acc = a.acc[ao];
      const cx<T> nxt = rk4_combine<MODE>(u, acc, nl, E, Eh, dt);
      if constexpr (mode_writes_state(MODE)) a.state[so] = nxt;
      if constexpr (mode_writes_acc(MODE)) a.acc[ao] = acc;
      w[e] = nxt;
    }
  }
  if constexpr (MODE != kModeTend) {
    if (do_p1) y_inverse_three<T, N, LB>(w, t, b, mx, a.kb, w1, lds, twr);
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
