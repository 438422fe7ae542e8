// ns3d_kernels.h -- kernels of the 3D velocity-form step.
//
// One tendency evaluation N(u) = P[(u x w)^] (w = curl u, P the projection
// onto divergence-free fields, 2/3-rule cube truncation) is four passes over
// HBM, each a batch of 1D transforms with the pointwise work fused in:
//
//   Z  (z, fwd + inv)  previous stage's products -> forward z transform ->
//                      projection, forcing, Lawson RK4 combine -> next stage
//                      input -> curl -> five inverse z transforms
//                      (u, wx, wy)                                [k3_z]
//   Yi (y, inverse)    five fields in, wz formed, six out         [k_y_inv_step]
//   X  (x, c2r / r2c)  six C2R, u x w, three R2C                  [k3_x]
//   Yf (y, forward)    three fields                               [k_y_fwd]
//
// Only kept modes are ever moved: the z passes touch the M x H kept
// (ky, kx) columns, the y passes the H kept kx planes, and the x pass reads
// and writes the H kept kx values of every row.
//
// Stratified (Boussinesq) flow carries a buoyancy field b as a fourth state
// component: the inverse passes move six and seven fields (u, w, b), the x pass also
// forms the buoyancy flux u b, and the forward passes move six (u x w, u b).
#pragma once
#include <type_traits>

#include "ns_common.h"

namespace fs {

// ---------------------------------------------------------------------------
// X pass: for each row pair (y0, y0+1) at height z, inverse-transform
// (ux,uy) and (wx,wy) of each row and (uz(y0),uz(y1)), (wz(y0),wz(y1)),
// form p = (u x w) * scale, forward transform (px + i py) of each row and
// (pz(y0) + i pz(y1)), store kept kx.
// One transform line is in flight at a time and the cross product is built
// as its factors arrive (u kept, partial products accumulated).  The kept
// coefficients of one row (six fields) are staged in LDS with 16-byte loads
// before its transforms, so a 64-lane block needs 13 KB of LDS at N = 512
// and twelve blocks fit a CU.  With umax, the largest |u_c| of the physical
// velocity is max-reduced into *umax.
// in : Wn[6][N][XT][N][16]   out: Wn[3][N][XT][N][16]
// STRAT: in Wn[7] (+ b), out Wn[6] (+ u b, v b, w b); b of the two rows is
// one complex line, the flux (fx + i fy) of each row and (fz(y0) + i fz(y1))
// three more forward lines.
// Grid: (N/2/RP, N) with RP = XRows<T, N, STRAT>::RP.
// ---------------------------------------------------------------------------
// Row pairs of a block: the seven staged fields of a double-precision
// stratified pass take half as many row pairs per block (LDS).
template <typename T, int N, bool STRAT>
using XRows = RowPairs<N, (STRAT && sizeof(T) == 8) ? 32 : 64>;

template <typename T, int N, bool STRAT = false>
__global__ void __launch_bounds__((XRows<T, N, STRAT>::THREADS),
                                  (sizeof(T) == 4 && !STRAT ? 3 : 1))
    k3_x(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ tw,
         T scale, unsigned long long* __restrict__ umax) {
  using G = Geo<N, false>;
  using R = XRows<T, N, STRAT>;
  constexpr int P = G::P;
  constexpr int FIN = STRAT ? 7 : 6;  // input fields
  // staging: kept coefficients [field][xt][16] of one row at a time (the
  // second row's fields of the cross-row lines come from HBM directly)
  constexpr int SROW = FIN * G::XT * kTile;
  static_assert(STRAT == false || N > 512 || sizeof(T) == 4 ||
                    (size_t)R::RP * (SROW + R::NPAD) * sizeof(cx<T>) <= 65536,
                "x-pass staging exceeds 64 KiB of LDS");
  __shared__ cx<T> stage[R::RP * SROW];
  __shared__ cx<T> lds[R::RP * R::NPAD];
  const int rp = threadIdx.x / P, t = threadIdx.x % P;
  const Twiddles<T, N> twr(tw, t);
  const int z = blockIdx.y;
  const int y0 = 2 * (blockIdx.x * R::RP + rp);
  cx<T>* line = lds + rp * R::NPAD;
  cx<T>* st = stage + rp * SROW;
  auto lidx = [=](int, int pos) { return R::pad(pos); };
  const size_t fstride = (size_t)N * G::XT * N * kTile;  // one field

  // staging of row y0 + r: for each (field, tile) the row is 16 contiguous
  // coefficients; 16-byte loads, all in flight.  With SKIP, the fields of
  // the cross-row lines (uz, wz; b) are left out: the second row's are read
  // for those lines before its staging.
  auto stage_row = [&](int r, auto skip) {
    constexpr bool SKIP = decltype(skip)::value;
    constexpr int PER = 16 / (int)sizeof(cx<T>);  // coefficients per load
    constexpr int NF = SKIP ? 4 : FIN;            // fields staged: 0, 1, 4, 5 with SKIP
    constexpr int LOADS = NF * G::XT * kTile / PER;
    const uint4* src4 = reinterpret_cast<const uint4*>(in);
    uint4* st4 = reinterpret_cast<uint4*>(st);
#pragma unroll
    for (int i0 = 0; i0 < LOADS; i0 += P) {
      const int i = i0 + t;
      if (i < LOADS) {
        const int c = i / (kTile / PER), lo = i % (kTile / PER);
        const int fs = c / G::XT, xt = c % G::XT;
        const int f = SKIP && fs >= 2 ? fs + 2 : fs;
        const size_t g = ((((size_t)f * N + z) * G::XT + xt) * N + y0 + r) * kTile;
        st4[(f * G::XT + xt) * (kTile / PER) + lo] = src4[g / PER + lo];
      }
    }
  };
  // Register e holds position k = t + e*P of the complex line a + i b; it
  // needs coefficient m = k (k <= K) or the conjugate mirror m = N - k
  // (k >= N - K) of both half spectra.
  int off[8], kind[8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int k = t + e * P;
    const int m = k <= G::K ? k : (k >= N - G::K ? N - k : 0);
    kind[e] = k <= G::K ? (k == 0 ? 2 : 1) : (k >= N - G::K ? -1 : 0);
    off[e] = m;
  }
  // the second row's field f at every register position, from HBM (off[e]
  // = 0 where nothing is kept: a valid element, loaded unconditionally so
  // that all loads are in flight together)
  auto row1_field = [&](int f, cx<T> (&bv)[8]) {
    const cx<T>* src = in + (((size_t)f * N + z) * G::XT * N + (y0 + 1)) * kTile;
#pragma unroll
    for (int e = 0; e < 8; e++) bv[e] = src[(size_t)(off[e] >> 4) * N * kTile + (off[e] & 15)];
  };
  // the second row's wz, uz (and b) for the cross lines below are loaded
  // with the staging of the first row and have arrived by its barrier
  cx<T> bw[8], bu[8], bb[STRAT ? 8 : 1];
  row1_field(3, bw);
  row1_field(2, bu);
  if constexpr (STRAT) row1_field(6, bb);
  stage_row(0, std::false_type{});
  // held here, before the barrier: not sunk below it into the transforms
#pragma unroll
  for (int e = 0; e < 8; e++) {
    asm volatile("" : "+v"(bw[e].re), "+v"(bw[e].im), "+v"(bu[e].re), "+v"(bu[e].im));
    if constexpr (STRAT) asm volatile("" : "+v"(bb[e].re), "+v"(bb[e].im));
  }
  __syncthreads();

  // inverse transform of the complex line A + i B: half spectrum A staged at
  // ba, B given at each register position (bv)
  auto inverse_line_v = [&](const cx<T>* ba, const cx<T> (&bv)[8], cx<T> (&v)[1][8]) {
#pragma unroll
    for (int e = 0; e < 8; e++) {
      cx<T> res = {0, 0};
      if (kind[e] != 0) {
        cx<T> A = ba[off[e]], B = bv[e];
        if (kind[e] == 2) A.im = B.im = 0;
        res = kind[e] > 0 ? cx<T>{A.re - B.im, A.im + B.re} : cx<T>{A.re + B.im, B.re - A.im};
      }
      v[0][e] = res;
    }
    fft_lines<T, N, +1, 1>(v, t, line, lidx, twr);
  };
  auto inverse_line = [&](const cx<T>* ba, const cx<T>* bb, cx<T> (&v)[1][8]) {
    cx<T> bv[8];
#pragma unroll
    for (int e = 0; e < 8; e++) bv[e] = bb[off[e]];
    inverse_line_v(ba, bv, v);
  };

  cx<T>* outz = out + (size_t)z * G::XT * N * kTile;
  // forward transform of v, untangled into kept kx of the two real lines
  // (field fa, row ya) and (field fb, row yb)
  auto forward_store = [&](cx<T> (&v)[1][8], int fa, int ya, int fb, int yb) {
    fft_lines<T, N, -1, 1>(v, t, line, lidx, twr);
#pragma unroll
    for (int e = 0; e < 8; e++) line[lidx(0, t + e * P)] = v[0][e];
    __syncthreads();
    for (int m = t; m < G::XT * kTile; m += P) {
      cx<T> A = {0, 0}, B = {0, 0};
      if (m < G::H) r2c_untangle(line[lidx(0, m)], line[lidx(0, (N - m) & (N - 1))], A, B);
      const size_t o = ((size_t)(m >> 4) * N) * kTile + (m & 15);
      st_nt(&outz[fa * fstride + o + (size_t)ya * kTile], A);
      st_nt(&outz[fb * fstride + o + (size_t)yb * kTile], B);
    }
    __syncthreads();
  };

  // Lines: (ux + i uy) and (wx + i wy) of each row, and across the pair
  // (uz(y0) + i uz(y1)), (wz(y0) + i wz(y1)): like with like.  A velocity and
  // a vorticity component in one line would leave the vorticity's rounding,
  // about |k| times larger, on the velocity (the single-precision error of
  // the tendency then grows with N).  Row by row the cross product is built
  // as its factors arrive; (px + i py) of each row is transformed at once,
  // pz of the first row waits to be paired with pz of the second.  The two
  // cross lines (and b's) come first; the second row's fields of them are
  // read from HBM directly (16 lanes per 128-byte row), in flight with the
  // staging loads of the first row.
  auto row_ptr = [&](int f) -> const cx<T>* { return st + f * G::XT * kTile; };  // staged row
  T pz0[8], uz1[8], wz1[8], wz0[8];
  double um = 0.0;  // largest |u_c| seen (only when umax is requested)
  // buoyancy of both rows (b(y0) + i b(y1)) and the first row's fz
  T bq[2][8], fz0[8];
  if constexpr (STRAT) {
    cx<T> v[1][8];
    inverse_line_v(row_ptr(6), bb, v);
#pragma unroll
    for (int e = 0; e < 8; e++) {
      bq[0][e] = v[0][e].re * scale;
      bq[1][e] = v[0][e].im * scale;
    }
  }
  T uz0[8];
  {
    cx<T> v[1][8];
    inverse_line_v(row_ptr(3), bw, v);
#pragma unroll
    for (int e = 0; e < 8; e++) {
      wz0[e] = v[0][e].re;
      wz1[e] = v[0][e].im;
    }
    inverse_line_v(row_ptr(2), bu, v);
#pragma unroll
    for (int e = 0; e < 8; e++) {
      uz0[e] = v[0][e].re;
      uz1[e] = v[0][e].im;
    }
  }
#pragma unroll
  for (int r = 0; r < 2; r++) {
    if (r == 1) {
      // every read of row 0 ended before the last barrier of its stores
      stage_row(1, std::true_type{});
      __syncthreads();
    }
    T ux[8], uy[8], uz[8], qx[8], qy[8];
    cx<T> v[1][8];
    inverse_line(row_ptr(0), row_ptr(1), v);
#pragma unroll
    for (int e = 0; e < 8; e++) {
      ux[e] = v[0][e].re;
      uy[e] = v[0][e].im;
      const T wz = r == 0 ? wz0[e] : wz1[e];
      qx[e] = uy[e] * wz;   // px = uy wz - uz wy
      qy[e] = -ux[e] * wz;  // py = uz wx - ux wz
    }
#pragma unroll
    for (int e = 0; e < 8; e++) uz[e] = r == 0 ? uz0[e] : uz1[e];
    if (umax) {
#pragma unroll
      for (int e = 0; e < 8; e++)
        um = fmax(um, (double)fmax(fmax(fabs(ux[e]), fabs(uy[e])), fabs(uz[e])));
    }
    if constexpr (STRAT) {
      // buoyancy flux u b (b carries the scale): (fx + i fy) now, fz paired
#pragma unroll
      for (int e = 0; e < 8; e++) {
        v[0][e] = {ux[e] * bq[r][e], uy[e] * bq[r][e]};
        if (r == 0) fz0[e] = uz[e] * bq[0][e];
      }
      forward_store(v, 3, y0 + r, 4, y0 + r);
      if (r == 1) {
#pragma unroll
        for (int e = 0; e < 8; e++) v[0][e] = {fz0[e], uz[e] * bq[1][e]};
        forward_store(v, 5, y0, 5, y0 + 1);
      }
    }
    inverse_line(row_ptr(4), row_ptr(5), v);
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const T wx = v[0][e].re, wy = v[0][e].im;
      const T pz = (ux[e] * wy - uy[e] * wx) * scale;
      v[0][e] = {(qx[e] - uz[e] * wy) * scale, (qy[e] + uz[e] * wx) * scale};
      if (r == 0) pz0[e] = pz;
      else qx[e] = pz;
    }
    forward_store(v, 0, y0 + r, 1, y0 + r);
    if (r == 1) {
#pragma unroll
      for (int e = 0; e < 8; e++) v[0][e] = {pz0[e], qx[e]};
      forward_store(v, 2, y0, 2, y0 + 1);
    }
  }
  if (umax) umax_wave(umax, um);
}

// The fused z passes keep three components plus a transform line in registers.
// Lines per block: a block of 1024 threads covers a whole 128-byte row of the
// tile-blocked layout (16 lines) at N = 512 in single precision (velocity
// only: one block per CU, 132 KB of LDS with the stash, 4 waves per SIMD);
// otherwise at most 512 threads below N = 1024 (two blocks per CU, each
// covering part of each row, merged in L2), and 1024-thread blocks of eight
// lines at N = 1024.  Full-row blocks measured 913 -> 840 us per 512^3 launch.
// In single precision their twiddles come from a copy of the table in LDS and
// the compiler is asked for 4 waves per SIMD (2 with buoyancy, whose pass
// needs twice the registers); double precision keeps the register budget.
// NC: state components (4 with buoyancy).
template <typename T, int N, int NC = 3>
using ZCfg = Strided<T, N, cmin(kTile, cmax(1, ((N >= 1024 || (N == 512 && sizeof(T) == 4 &&
                                                                  NC == 3))
                                                     ? 1024
                                                     : 512) /
                                                    (N / 8)))>;
// linear propagator of a fused z pass
enum LinearProp : int { kPropVisc = 0, kPropRot = 1, kPropStrat = 2, kPropStratRot = 3 };
// the propagators of Boussinesq flow, whose state carries the buoyancy too
constexpr bool prop_boussinesq(int prop) { return prop >= kPropStrat; }
template <typename T, int PROP = kPropVisc>
constexpr int zpass_waves() {
  return sizeof(T) == 4 ? (prop_boussinesq(PROP) ? 2 : 4) : 1;
}
// modes per lane whose u_n and accumulator a z pass loads at once (the
// propagators of rotation and buoyancy, double precision and the longer
// transforms need their registers for themselves)
template <typename T, int N, int PROP>
constexpr int kZChunk = PROP == kPropVisc && sizeof(T) == 4 && N <= 512 ? 2 : 1;

// twiddle table of a z pass: the LDS copy `twl` (filled by the block) in single
// precision, the global table otherwise
template <typename T, int N, int THREADS>
__device__ __forceinline__ const cx<T>* zpass_twiddles(const cx<T>* __restrict__ tw, cx<T>* twl) {
  if constexpr (sizeof(T) == 4) {
    for (int i = threadIdx.x; i < N; i += THREADS) twl[i] = tw[i];
    __syncthreads();
    return twl;
  } else {
    return tw;
  }
}

// ---------------------------------------------------------------------------
// Inverse z transforms of a stage input v held in registers as v[c][e] at
// z-position t + e*P of line b: the velocity and the horizontal vorticity
// (wx, wy; w = i k x v), written to the compact workspace Wm (Geo::wm_row) as
// ux uy uz wx wy.
// The vertical vorticity needs no kz and is formed by the inverse y pass.
// NC = 4 adds the buoyancy v[3] as field 5.
// ---------------------------------------------------------------------------
template <typename T, int N, int NC, class TW>
__device__ __forceinline__ void z_inverse(cx<T> (&v)[NC][8], int t, int b, int jy, int xt,
                                          int sub, int mx, int my, T kb,
                                          cx<T>* __restrict__ w1, cx<T>* lds, const TW& tw) {
  using G = Geo<N, false>;
  using C = ZCfg<T, N, NC>;
  constexpr int P = G::P;
  const size_t fstride = G::wm_row(1, 0, 0);
  cx<T>* dst0 = w1 + G::wm_row(0, xt, 0) + (size_t)jy * kTile + sub * C::LB + b;
  const size_t zstride = G::kWmZ;
  auto lidx = [=](int, int pos) { return pos * C::LB + b; };
  const T kx = kb * (T)mx, ky = kb * (T)my;
  // vorticity first (needs v), then velocity in place
#pragma unroll
  for (int c = 0; c < 2; c++) {
    cx<T> w[1][8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int iz = t + e * P;
      const T kz = kb * (T)(iz <= N / 2 ? iz : iz - N);
      w[0][e] = c == 0 ? mul_i(cscale(v[2][e], ky) - cscale(v[1][e], kz))
                       : mul_i(cscale(v[0][e], kz) - cscale(v[2][e], kx));
    }
    fft_lines<T, N, +1, 1>(w, t, lds, lidx, tw);
    cx<T>* dst = dst0 + (3 + c) * fstride;  // wx, wy in fields 3, 4
#pragma unroll
    for (int e = 0; e < 8; e++) dst[(size_t)(t + e * P) * zstride] = w[0][e];
  }
#pragma unroll
  for (int c = 0; c < NC; c++) {
    cx<T> w[1][8];
#pragma unroll
    for (int e = 0; e < 8; e++) w[0][e] = v[c][e];
    fft_lines<T, N, +1, 1>(w, t, lds, lidx, tw);
    cx<T>* dst = dst0 + (c < 3 ? c : 5) * fstride;
#pragma unroll
    for (int e = 0; e < 8; e++) dst[(size_t)(t + e * P) * zstride] = w[0][e];
  }
}

template <typename T>
__device__ __forceinline__ int band_index(int mx, int my, int mz, int bw) {
  return ((mz + bw) * (2 * bw + 1) + (my + bw)) * (bw + 1) + mx;
}

// Forcing band test split into the part fixed for a lane's column (mx, my):
// band_column gives mx^2 + my^2 when the column can meet the band, else -1;
// in_band then checks one mz of that column.
template <typename T>
__device__ __forceinline__ int band_column(const StageArgs<T>& a, int mx, int my) {
  if (a.m2max < 0 || mx > a.bw || my > a.bw || my < -a.bw) return -1;
  return mx * mx + my * my;
}
template <typename T>
__device__ __forceinline__ bool in_band(const StageArgs<T>& a, int m2xy, int mz) {
  if (m2xy < 0 || mz > a.bw || mz < -a.bw) return false;
  const int m2 = m2xy + mz * mz;
  return m2 >= a.m2min && m2 <= a.m2max;
}

// 1/x for the projection: the hardware reciprocal (1 ulp) in single
// precision, a division in double precision
template <typename T>
__device__ __forceinline__ T recip(T x) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(x);
  else return (T)1 / x;
}

// ---------------------------------------------------------------------------
// First inverse pass of a stage, from the caller's state (ABI layout
// [NC][N][N][N/2+1]): masks to the kept set, records the band values, and
// writes the five (NC = 4: six) inverse-z-transformed fields.
// Grid: M * XT * SUB.
// ---------------------------------------------------------------------------
template <typename T, int N, int NC = 3>
__global__ void __launch_bounds__((ZCfg<T, N, NC>::THREADS))
    k3_p1(const cx<T>* __restrict__ state, cx<T>* __restrict__ w1, StageArgs<T> a) {
  using G = Geo<N, false>;
  using C = ZCfg<T, N, NC>;
  constexpr int P = G::P;
  constexpr int NH = N / 2 + 1;
  __shared__ cx<T> lds[C::LB * N];
  const int b = threadIdx.x % C::LB, t = threadIdx.x / C::LB;
  __shared__ cx<T> twl[sizeof(T) == 4 ? N : 1];
  const Twiddles<T, N, false> twr(zpass_twiddles<T, N, C::THREADS>(a.tw, twl), t);
  int jy, rem;
  if (!xcd_row_block(G::M, G::XT * C::SUB, jy, rem)) return;  // whole block
  const int xt = rem / C::SUB, sub = rem % C::SUB;
  const int mx = xt * kTile + sub * C::LB + b;
  const int iy = G::j2i(jy), my = G::jmode(jy);
  const bool col = mx < G::H;
  const int m2xy = band_column(a, mx, my);
  const size_t cstride = (size_t)N * N * NH;
  cx<T> v[NC][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int iz = t + e * P;
    const bool kept = col && G::i2j(iz) >= 0;
    const size_t o = ((size_t)iz * N + iy) * NH + mx;
#pragma unroll
    for (int c = 0; c < NC; c++) v[c][e] = kept ? state[c * cstride + o] : cx<T>{0, 0};
    if (kept) {
      const int mz = iz <= N / 2 ? iz : iz - N;
      if (in_band(a, m2xy, mz)) {
        const int bi = band_index<T>(mx, my, mz, a.bw);
        const int bn = (2 * a.bw + 1) * (2 * a.bw + 1) * (a.bw + 1);
#pragma unroll
        for (int c = 0; c < 3; c++) a.vband[c * bn + bi] = v[c][e];
      }
    }
  }
  z_inverse<T, N, NC>(v, t, b, jy, xt, sub, mx, my, a.kb, w1, lds, twr);
}

// ---------------------------------------------------------------------------
// Z pass: forward z transforms of the stage's products (Wm[3], Geo::wm_row),
// projection + forcing -> tendency of this stage, Lawson RK4 combine, and
// (do_p1) the next stage's five (six) inverse z transforms into w1.
// MODE kModeTend writes the tendency to a.tend instead.  PROP selects the
// linear propagator of the combine: viscosity, + rotation (about z), or
// + buoyancy force and stratification (kPropStrat, and with rotation too
// kPropStratRot: products Wm[6], the
// flux u b giving the buoyancy tendency -i k.(u b)^, four state components,
// six inverse transforms).  Grid: M * XT * SUB.
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE, int PROP = kPropVisc>
__global__ void __launch_bounds__((ZCfg<T, N, prop_boussinesq(PROP) ? 4 : 3>::THREADS),
                                  (zpass_waves<T, PROP>()))
    k3_z(const cx<T>* __restrict__ w4, cx<T>* __restrict__ w1, StageArgs<T> a, int do_p1) {
  using G = Geo<N, false>;
  using C = ZCfg<T, N, prop_boussinesq(PROP) ? 4 : 3>;
  constexpr int P = G::P;
  constexpr int NH = N / 2 + 1;
  constexpr int NC = prop_boussinesq(PROP) ? 4 : 3;
  __shared__ cx<T> lds[C::LB * N];
  const int b = threadIdx.x % C::LB, t = threadIdx.x / C::LB;
  __shared__ cx<T> twl[sizeof(T) == 4 ? N : 1];
  const Twiddles<T, N, false> twr(zpass_twiddles<T, N, C::THREADS>(a.tw, twl), t);
  int jy, rem;
  if (!xcd_row_block(G::M, G::XT * C::SUB, jy, rem)) return;  // whole block
  const int xt = rem / C::SUB, sub = rem % C::SUB;
  const int mx = xt * kTile + sub * C::LB + b;
  const int iy = G::j2i(jy), my = G::jmode(jy);
  const bool col = mx < G::H;
  auto lidx = [=](int, int pos) { return pos * C::LB + b; };

  // forward z transforms of the three product components
  const size_t fstride = G::wm_row(1, 0, 0);
  const size_t zstride = G::kWmZ;
  const cx<T>* src0 = w4 + G::wm_row(0, xt, 0) + (size_t)jy * kTile + sub * C::LB + b;
  // all three components' loads are issued before the first transform
  cx<T> v[NC][8];
#pragma unroll
  for (int c = 0; c < 3; c++)
#pragma unroll
    for (int e = 0; e < 8; e++) v[c][e] = src0[c * fstride + (size_t)(t + e * P) * zstride];
  // up to 512: the first component's transformed lines wait in an LDS stash
  // (each lane reads back only what it wrote, so no barrier) while the other
  // two are transformed; held in registers they spilled to scratch (single
  // precision at two blocks per CU, double precision at one)
  constexpr bool kStash = N <= 512 && !prop_boussinesq(PROP);
  __shared__ cx<T> stash[kStash ? C::LB * N : 1];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    fft_lines<T, N, -1, 1>(reinterpret_cast<cx<T>(&)[1][8]>(v[c]), t, lds, lidx, twr);
    if constexpr (kStash) {
      if (c == 0) {
#pragma unroll
        for (int e = 0; e < 8; e++) stash[lidx(0, t + e * P)] = v[0][e];
      }
    }
  }
  const T kx = a.kb * (T)mx, ky = a.kb * (T)my;
  if constexpr (prop_boussinesq(PROP)) {
    // buoyancy tendency -i k.(u b)^, one flux component at a time
#pragma unroll
    for (int e = 0; e < 8; e++) v[3][e] = {0, 0};
#pragma unroll
    for (int c = 0; c < 3; c++) {
      cx<T> f[1][8];
#pragma unroll
      for (int e = 0; e < 8; e++) f[0][e] = src0[(3 + c) * fstride + (size_t)(t + e * P) * zstride];
      fft_lines<T, N, -1, 1>(f, t, lds, lidx, twr);
#pragma unroll
      for (int e = 0; e < 8; e++) {
        const int iz = t + e * P;
        const T kc = c == 0 ? kx : (c == 1 ? ky : a.kb * (T)(iz <= N / 2 ? iz : iz - N));
        v[3][e] = v[3][e] - mul_i(cscale(f[0][e], kc));
      }
    }
  }

  const size_t cstride = (size_t)N * N * NH;
  const size_t acstride = (size_t)G::XT * G::M * G::M * kTile;
  const int bn = (2 * a.bw + 1) * (2 * a.bw + 1) * (a.bw + 1);
  const T alpha = a.m2max >= 0 ? a.alpha[0] : (T)0;
  const T dt = stage_dt(a);
  // forcing-band modes exist only in blocks whose kx range starts within the
  // band and whose ky is in it: a block-uniform test, so that the per-mode
  // test below stays out of every other block's register budget
  const bool blk_band = a.m2max >= 0 && xt * kTile + sub * C::LB <= a.bw && my <= a.bw &&
                        my >= -a.bw;
  bool bad = false;  // a non-finite value written to the state
  // u_n and the accumulator of CH modes are loaded before any of them is
  // combined and stored: the stores could alias later loads as far as the
  // compiler knows, so loads issued mode by mode would wait out one memory
  // round trip per mode
  auto combine = [&](cx<T>* state, cx<T>* accp) {
    constexpr int CH = kZChunk<T, N, PROP>;
    const T exy = a.e1[mx] * a.e1[iy], ehxy = a.eh1[mx] * a.eh1[iy];
#pragma unroll
    for (int e0 = 0; e0 < 8; e0 += CH) {
      cx<T> us[NC][CH], as[NC][CH];
      T ez[CH], ehz[CH];
#pragma unroll
      for (int q = 0; q < CH; q++) {
        const int iz = t + (e0 + q) * P;
        const int jz = G::i2j(iz);
        const size_t so = ((size_t)iz * N + iy) * NH + mx;
        const size_t ao = (((size_t)xt * G::M + jy) * G::M + jz) * kTile + sub * C::LB + b;
        const bool kept = col && jz >= 0;
#pragma unroll
        for (int c = 0; c < NC; c++) {
          us[c][q] = as[c][q] = cx<T>{0, 0};
          if (kept && mode_reads_state(MODE)) us[c][q] = state[c * cstride + so];
          if (kept && mode_reads_acc(MODE)) as[c][q] = accp[c * acstride + ao];
        }
        ez[q] = ehz[q] = (T)0;
        if (kept && MODE != kModeTend) {
          ez[q] = a.e1[iz];
          ehz[q] = a.eh1[iz];
        }
      }
#pragma unroll
      for (int q = 0; q < CH; q++) {
        const int e = e0 + q;
        const int iz = t + e * P;
        const int jz = G::i2j(iz);
        const bool kept = col && jz >= 0;
        if (!kept) {
#pragma unroll
          for (int c = 0; c < NC; c++) v[c][e] = {0, 0};
          continue;
        }
        const int mz = iz <= N / 2 ? iz : iz - N;
        const T kz = a.kb * (T)mz;
        const T k2 = kx * kx + ky * ky + kz * kz;
        cx<T> nl[NC];
        if constexpr (kStash) v[0][e] = stash[lidx(0, t + e * P)];
        if (k2 > (T)0) {
          const T ik2 = recip(k2);
          const cx<T> kp =
              cscale(cscale(v[0][e], kx) + cscale(v[1][e], ky) + cscale(v[2][e], kz), ik2);
          nl[0] = v[0][e] - cscale(kp, kx);
          nl[1] = v[1][e] - cscale(kp, ky);
          nl[2] = v[2][e] - cscale(kp, kz);
          if constexpr (NC == 4) nl[3] = v[3][e];
        } else {
#pragma unroll
          for (int c = 0; c < NC; c++) nl[c] = {0, 0};
        }
        bool band = false;
        int bi = 0;
        if (blk_band) {
          band = in_band(a, band_column(a, mx, my), mz);
          if (band) {
            bi = band_index<T>(mx, my, mz, a.bw);
#pragma unroll
            for (int c = 0; c < 3; c++) nl[c] = nl[c] + cscale(a.vband[c * bn + bi], alpha);
          }
        }
        const size_t so = ((size_t)iz * N + iy) * NH + mx;
        if constexpr (MODE == kModeTend) {
#pragma unroll
          for (int c = 0; c < NC; c++) a.tend[c * cstride + so] = nl[c];
        } else {
          const T E = exy * ez[q];
          const T Eh = ehxy * ehz[q];
          const size_t ao = (((size_t)xt * G::M + jy) * G::M + jz) * kTile + sub * C::LB + b;
          if constexpr (PROP != kPropVisc) {
            // the combination acts on the mode's NC-vectors
            cx<T> u[NC], acc[NC], nxt[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) {
              u[c] = us[c][q];
              acc[c] = as[c][q];
            }
            if (k2 == (T)0) {
              // the mean mode: the unprojected linear terms (rotation of the
              // horizontal mean, buoyancy oscillation of the vertical mean)
              MeanProp<T, NC> R;
              R.set(a.rotf, prop_boussinesq(PROP) ? a.n2 : (T)0, dt);
              prop_combine<MODE>(u, acc, nl, E, Eh, dt, R, nxt);
            } else if constexpr (PROP == kPropRot) {
              RotProp<T> R;
              const T ikn = k2 > (T)0 ? (T)1 / sqrt(k2) : (T)0;
              R.kh[0] = kx * ikn;
              R.kh[1] = ky * ikn;
              R.kh[2] = kz * ikn;
              const T sg = a.rotf * kz * ikn;
              R.s1 = sin(sg * dt);
              R.c1 = cos(sg * dt);
              R.s2 = sin(sg * dt * (T)0.5);
              R.c2 = cos(sg * dt * (T)0.5);
              prop_combine<MODE>(u, acc, nl, E, Eh, dt, R, nxt);
            } else if constexpr (PROP == kPropStrat) {
              StratProp<T> R;
              R.set(kx, ky, kz, a.n2, dt);
              prop_combine<MODE>(u, acc, nl, E, Eh, dt, R, nxt);
            } else {
              StratRotProp<T> R;
              R.set(kx, ky, kz, a.n2, a.rotf, dt);
              prop_combine<MODE>(u, acc, nl, E, Eh, dt, R, nxt);
            }
#pragma unroll
            for (int c = 0; c < NC; c++) {
              if constexpr (mode_writes_state(MODE)) {
                state[c * cstride + so] = nxt[c];
                bad |= nonfinite(nxt[c]);
              }
              if constexpr (mode_writes_acc(MODE)) accp[c * acstride + ao] = acc[c];
              v[c][e] = nxt[c];
            }
          } else {
#pragma unroll
            for (int c = 0; c < 3; c++) {
              cx<T> acc = as[c][q];
              const cx<T> nxt = rk4_combine<MODE>(us[c][q], acc, nl[c], E, Eh, dt);
              if constexpr (mode_writes_state(MODE)) {
                state[c * cstride + so] = nxt;
                bad |= nonfinite(nxt);
              }
              if constexpr (mode_writes_acc(MODE)) accp[c * acstride + ao] = acc;
              v[c][e] = nxt;
            }
          }
          if (band && do_p1) {
#pragma unroll
            for (int c = 0; c < 3; c++) a.vband[c * bn + bi] = v[c][e];
          }
        }
      }
    }
  };
  if constexpr (kZChunk<T, N, PROP> > 1) {
    // the state and accumulator through pointers the compiler may take as
    // unaliased: the batched loads need fewer registers that way
    [&](cx<T>* __restrict__ st, cx<T>* __restrict__ ac) { combine(st, ac); }(a.state, a.acc);
  } else {
    combine(a.state, a.acc);
  }
  if constexpr (mode_writes_state(MODE)) {
    if (a.nonfin) flag_wave(a.nonfin, bad);
  }
  if constexpr (MODE != kModeTend) {
    if (do_p1) z_inverse<T, N, NC>(v, t, b, jy, xt, sub, mx, my, a.kb, w1, lds, twr);
  }
}

// ---------------------------------------------------------------------------
// Plain (undealiased) 3D transforms, used by the FFT entry points, for F
// stacked fields: spec [F][N][N][N/2+1] complex, phys [F][N][N][N] real.  The
// z passes take the field from blockIdx.y; the y and x passes treat the F*N
// z-planes of the stack as rows.
// ---------------------------------------------------------------------------
// inverse z: spec -> Wm(FULL)[F][N][XT][N][16]; grid (N * XT * SUB, F).
// GRAD: spec is a velocity state [3][N][N][N/2+1] and field f = 3i + j of the
// output is the gradient d u_i / d x_j, i k_j u_i on the kept modes (kb = 2 pi / L).
template <typename T, int N, bool GRAD = false>
__global__ void __launch_bounds__((Strided<T, N>::THREADS))
    k3f_z_inv(const cx<T>* __restrict__ spec, cx<T>* __restrict__ w, const cx<T>* __restrict__ tw,
              T kb = T(0)) {
  using G = Geo<N, true>;
  using C = Strided<T, N>;
  constexpr int P = G::P, NH = N / 2 + 1;
  __shared__ cx<T> lds[C::LB * N];
  const int b = threadIdx.x % C::LB, t = threadIdx.x / C::LB;
  const Twiddles<T, N, false> twr(tw, t);
  int blk = blockIdx.x;
  const int sub = blk % C::SUB;
  blk /= C::SUB;
  const int xt = blk % G::XT, iy = blk / G::XT;
  const int mx = xt * kTile + sub * C::LB + b;
  spec += (size_t)(GRAD ? blockIdx.y / 3 : blockIdx.y) * N * N * NH;
  w += (size_t)blockIdx.y * N * G::XT * N * kTile;
  cx<T> v[1][8];
  if constexpr (GRAD) {
    using GK = Geo<N, false>;
    const int j = blockIdx.y % 3, my = iy <= N / 2 ? iy : iy - N;
    const bool col = mx <= GK::K && my <= GK::K && my >= -GK::K;
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int iz = t + e * P, mz = iz <= N / 2 ? iz : iz - N;
      const bool keep = col && mz <= GK::K && mz >= -GK::K;
      const cx<T> u = keep ? spec[((size_t)iz * N + iy) * NH + mx] : cx<T>{0, 0};
      const T kj = kb * (T)(j == 0 ? mx : (j == 1 ? my : mz));
      v[0][e] = mul_i(cscale(u, kj));
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; e++)
      v[0][e] = mx < G::H ? spec[((size_t)(t + e * P) * N + iy) * NH + mx] : cx<T>{0, 0};
  }
  fft_lines<T, N, +1, 1>(v, t, lds, [=](int, int pos) { return pos * C::LB + b; }, twr);
  const size_t zstride = (size_t)G::XT * N * kTile;
  cx<T>* dst = w + ((size_t)xt * N + iy) * kTile + sub * C::LB + b;
#pragma unroll
  for (int e = 0; e < 8; e++) dst[(size_t)(t + e * P) * zstride] = v[0][e];
}

// forward z: Wm(FULL) -> spec; grid (N * XT * SUB, fields)
template <typename T, int N>
__global__ void __launch_bounds__((Strided<T, N>::THREADS))
    k3f_z_fwd(const cx<T>* __restrict__ w, cx<T>* __restrict__ spec, const cx<T>* __restrict__ tw) {
  using G = Geo<N, true>;
  using C = Strided<T, N>;
  constexpr int P = G::P, NH = N / 2 + 1;
  __shared__ cx<T> lds[C::LB * N];
  const int b = threadIdx.x % C::LB, t = threadIdx.x / C::LB;
  const Twiddles<T, N, false> twr(tw, t);
  int blk = blockIdx.x;
  const int sub = blk % C::SUB;
  blk /= C::SUB;
  const int xt = blk % G::XT, iy = blk / G::XT;
  const int mx = xt * kTile + sub * C::LB + b;
  spec += (size_t)blockIdx.y * N * N * NH;
  w += (size_t)blockIdx.y * N * G::XT * N * kTile;
  const size_t zstride = (size_t)G::XT * N * kTile;
  const cx<T>* src = w + ((size_t)xt * N + iy) * kTile + sub * C::LB + b;
  cx<T> v[1][8];
#pragma unroll
  for (int e = 0; e < 8; e++) v[0][e] = src[(size_t)(t + e * P) * zstride];
  fft_lines<T, N, -1, 1>(v, t, lds, [=](int, int pos) { return pos * C::LB + b; }, twr);
  if (mx < G::H) {
#pragma unroll
    for (int e = 0; e < 8; e++) spec[((size_t)(t + e * P) * N + iy) * NH + mx] = v[0][e];
  }
}

// x c2r of rows (y0, y0+1) of nz planes: Wn(FULL)[nz][XT][N][16] -> phys
// [nz][N][N]; grid (N/2/RP, nz)
template <typename T, int N>
__global__ void __launch_bounds__((RowPairs<N>::THREADS))
    kf_x_c2r(const cx<T>* __restrict__ w, T* __restrict__ phys, const cx<T>* __restrict__ tw) {
  using G = Geo<N, true>;
  using R = RowPairs<N>;
  constexpr int P = G::P;
  __shared__ cx<T> lds[R::RP * R::NPAD];
  const int rp = threadIdx.x / P, t = threadIdx.x % P;
  const Twiddles<T, N, false> twr(tw, t);
  const int z = blockIdx.y, y0 = 2 * (blockIdx.x * R::RP + rp);
  const cx<T>* wz = w + (size_t)z * G::XT * N * kTile;
  auto at = [=](int y, int m) { return wz[((size_t)(m >> 4) * N + y) * kTile + (m & 15)]; };
  cx<T> v[1][8];
#pragma unroll
  for (int e = 0; e < 8; e++)
    v[0][e] = c2r_pair_at<T, N, true>(
        t + e * P, [&](int m) { return at(y0, m); }, [&](int m) { return at(y0 + 1, m); });
  fft_lines<T, N, +1, 1>(v, t, lds + rp * R::NPAD,
                         [=](int, int pos) { return R::pad(pos); }, twr);
  T* row = phys + ((size_t)z * N + y0) * N;
#pragma unroll
  for (int e = 0; e < 8; e++) {
    row[t + e * P] = v[0][e].re;
    row[N + t + e * P] = v[0][e].im;
  }
}

// x r2c of rows (y0, y0+1): phys -> Wn(FULL), scaled; grid (N/2/RP, nz)
template <typename T, int N>
__global__ void __launch_bounds__((RowPairs<N>::THREADS))
    kf_x_r2c(const T* __restrict__ phys, cx<T>* __restrict__ w, const cx<T>* __restrict__ tw,
             T scale) {
  using G = Geo<N, true>;
  using R = RowPairs<N>;
  constexpr int P = G::P;
  __shared__ cx<T> lds[R::RP * R::NPAD];
  const int rp = threadIdx.x / P, t = threadIdx.x % P;
  const Twiddles<T, N, false> twr(tw, t);
  const int z = blockIdx.y, y0 = 2 * (blockIdx.x * R::RP + rp);
  const T* row = phys + ((size_t)z * N + y0) * N;
  cx<T> v[1][8];
#pragma unroll
  for (int e = 0; e < 8; e++) v[0][e] = {row[t + e * P] * scale, row[N + t + e * P] * scale};
  cx<T>* my = lds + rp * R::NPAD;
  auto lidx = [=](int, int pos) { return R::pad(pos); };
  fft_lines<T, N, -1, 1>(v, t, my, lidx, twr);
#pragma unroll
  for (int e = 0; e < 8; e++) my[lidx(0, t + e * P)] = v[0][e];
  __syncthreads();
  cx<T>* wz = w + (size_t)z * G::XT * N * kTile;
  for (int m = t; m < G::XT * kTile; m += P) {
    cx<T> A = {0, 0}, B = {0, 0};
    if (m < G::H) r2c_untangle(my[lidx(0, m)], my[lidx(0, (N - m) & (N - 1))], A, B);
    const size_t o = ((size_t)(m >> 4) * N) * kTile + (m & 15);
    wz[o + (size_t)y0 * kTile] = A;
    wz[o + (size_t)(y0 + 1) * kTile] = B;
  }
}

}  // namespace fs
