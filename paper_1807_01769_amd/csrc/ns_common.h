// ns_common.h -- geometry of the dealiased spectral layout and the passes
// shared by the 2D and 3D solvers.
//
// Spectral index conventions (domain [0, L)^d, k = (2 pi / L) m):
//   full axes (ky, kz): FFT index i in [0, N), mode m = i (i <= N/2) or i - N;
//   half axis (kx):     index = mode m in [0, N/2].
// Dealiasing (2/3 rule, cube): a mode is kept iff 3|m_a| < N on every axis,
// i.e. |m_a| <= K = floor((N-1)/3).  Kept full-axis modes are stored
// compactly as j in [0, M), M = 2K+1 (j <= K: m = j; j > K: m = j - M).
// Kept half-axis modes are m in [0, H), H = K+1, grouped in XT tiles of 16.
//
// The "FULL" geometry (K = N/2, M = N) describes undealiased transforms.
//
// Intermediate workspace arrays are tile-blocked so that every strided pass
// reads and writes whole 16-element (128 B for complex64) rows:
//   Wm[f][z][xt][j][16]  (compact index along y; from N = 1024 on the 3D step
//                         uses Wm[f][xt][z][j][16], see Geo::wm_row)
//   Wn[f][z][xt][y][16]  (full index along y)
// In 2D the z extent is 1.
#pragma once
#include "fft_core.h"

namespace fs {

constexpr int kTile = 16;

// Streaming access to intermediates that are written once and read once by
// the next pass (far larger than the caches): non-temporal loads and stores.
template <typename T>
__device__ __forceinline__ void st_nt(cx<T>* p, cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 x;
  x.x = v.re;
  x.y = v.im;
  __builtin_nontemporal_store(x, reinterpret_cast<v2*>(p));
}
template <typename T>
__device__ __forceinline__ cx<T> ld_nt(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 x = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return cx<T>{x.x, x.y};
}

template <int N, bool FULL>
struct Geo {
  static constexpr int K = FULL ? N / 2 : (N - 1) / 3;
  static constexpr int M = FULL ? N : 2 * K + 1;
  static constexpr int H = K + 1;
  static constexpr int XT = (H + kTile - 1) / kTile;
  static constexpr int P = N / 8;
  // compact index -> FFT index, and back (-1 when the mode is not kept)
  __host__ __device__ static constexpr int j2i(int j) { return j <= K ? j : j + (N - M); }
  __host__ __device__ static constexpr int i2j(int i) {
    return i <= K ? i : (i >= N - K ? i - (N - M) : -1);
  }
  // signed mode number of a kept compact index
  __host__ __device__ static constexpr int jmode(int j) { return j <= K ? j : j - M; }
  // First element of row (field f, kx tile xt, z plane z) of the compact-y
  // workspace of a dealiased 3D step, and the distance between the rows of
  // adjacent z planes.  From N = 1024 on the z planes of one kx tile are
  // adjacent, Wm[f][xt][z][j][16]: a z line then steps M rows per plane, not
  // XT * M (1.9 MB at 1024), so the 128 planes that one access of a z-pass
  // block touches lie in a few large pages instead of one page each, which
  // the per-CU address translation cache could not hold.  Below 1024 the
  // planes lie within few pages either way and Wm[f][z][xt][j][16] keeps the
  // y passes' neighbouring blocks on neighbouring rows.
  static constexpr bool kWmTileMajor = N >= 1024;
  __host__ __device__ static constexpr size_t wm_row(int f, int xt, int z) {
    return kWmTileMajor ? (((size_t)f * XT + xt) * N + z) * M * kTile
                        : (((size_t)f * N + z) * XT + xt) * M * kTile;
  }
  static constexpr size_t kWmZ = (size_t)(kWmTileMajor ? 1 : XT) * M * kTile;
};

__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Lines per block of a strided (y or z) pass: at most CAP (<= 16, one tile),
// at most 1024 threads and at most 64 KiB of LDS.
template <typename T, int N, int CAP = kTile>
struct Strided {
  static constexpr int P = N / 8;
  static constexpr int LB =
      cmin(CAP, cmin(65536 / (N * (int)sizeof(cx<T>)), 1024 / P));
  static constexpr int SUB = kTile / LB;
  static constexpr int THREADS = LB * P;
};

// Lines per block of the y passes.
constexpr int kYLines = kTile;

// Row pairs per block of an x pass (a row pair is owned by P lanes; at most
// LANES lanes per block unless one row pair needs more).
template <int N, int LANES = 64>
struct RowPairs {
  static constexpr int P = N / 8;
  static constexpr int RP = cmax(1, cmin(LANES / P, N / 2));
  static constexpr int THREADS = RP * P;
  static constexpr int NPAD = N + N / 8;  // LDS line stride, +1 slot per 8
  __host__ __device__ static constexpr int pad(int pos) { return pos + (pos >> 3); }
};

// Workgroups are dealt to the chip's XCDs round-robin by linear block id,
// and every XCD has its own L2.  Passes whose blocks cover part of a
// 128-byte line (or whose rows are not line aligned) order their blocks so
// that all blocks of one row go to the same XCD, consecutively: linear id B
// runs on XCD B % kXcd as that XCD's (B / kXcd)-th block.  Returns false for
// the padding blocks of the last round.
constexpr int kXcd = 8;
__host__ __device__ constexpr int xcd_grid(int rows, int per_row) {
  return kXcd * ((rows + kXcd - 1) / kXcd) * per_row;
}
__device__ __forceinline__ bool xcd_row_block(int rows, int per_row, int& row, int& rem) {
  const int xcd = blockIdx.x % kXcd, q = blockIdx.x / kXcd;
  row = (q / per_row) * kXcd + xcd;
  rem = q % per_row;
  return row < rows;
}

// Parameters of a fused RK4 stage epilogue.
template <typename T>
struct StageArgs {
  cx<T>* state;        // caller's spectral state (ABI layout)
  cx<T>* acc;          // RK4 accumulator, compact blocked layout
  cx<T>* tend;         // tendency output (ABI layout), tendency mode only
  cx<T>* vband;        // stage input on the forcing-band cube
  const T* alpha;      // forcing coefficient (device scalar)
  const T* e1;         // exp(-nu dt k^2) per FFT index (one axis)
  const T* eh1;        // exp(-nu dt k^2 / 2) per FFT index
  const cx<T>* tw;     // twiddle table of the transform size
  T kb;                // 2 pi / L
  T dt;                // step (used when dtp is null)
  const T* dtp;        // device step of the current step (adaptive steps), or null
  cx<T>* sin;          // 2D Boussinesq: stage input [2][XT][M][16] (else null)
  T n2;                // Boussinesq: squared buoyancy frequency
  T rotf;              // 3D rotating frame: Coriolis parameter f (z axis)
  unsigned* nonfin;    // non-null: flag set when the last stage writes a non-finite value
  int bw;              // half width of the forcing-band cube (modes)
  int m2min, m2max;    // band: m2min <= |m|^2 <= m2max; m2max < 0 => off
};

template <typename T>
__device__ __forceinline__ T stage_dt(const StageArgs<T>& a) {
  return a.dtp ? *a.dtp : a.dt;
}

// kStage1..4: the four stages of Lawson RK4; kRk2a, kRk2b: the two of the
// Lawson midpoint rule (RK2); kModeTend: tendency only.
enum StageMode : int {
  kModeTend = 0,
  kStage1 = 1,
  kStage2 = 2,
  kStage3 = 3,
  kStage4 = 4,
  kRk2a = 5,
  kRk2b = 6
};
// what a stage epilogue touches besides the tendency
__host__ __device__ constexpr bool mode_reads_state(int m) {
  return m != kModeTend && m != kStage4;
}
__host__ __device__ constexpr bool mode_reads_acc(int m) {
  return m == kStage2 || m == kStage3 || m == kStage4;
}
__host__ __device__ constexpr bool mode_writes_acc(int m) {
  return m == kStage1 || m == kStage2 || m == kStage3;
}
__host__ __device__ constexpr bool mode_writes_state(int m) { return m == kStage4 || m == kRk2b; }

// Lawson stage combination at one mode.  `u` is u_n, `a` the RK4
// accumulator, `nl` the tendency of this stage; returns the next stage input
// (last stage: u_{n+1}).  E = exp(-nu k^2 dt), Eh = exp(-nu k^2 dt/2).
//   RK4 stage1: a = E u + dt/6 E k1          next = Eh (u + dt/2 k1)
//       stage2: a += dt/3 Eh k2              next = Eh u + dt/2 k2
//       stage3: a += dt/3 Eh k3              next = E u + dt Eh k3
//       stage4: u_{n+1} = a + dt/6 k4
//   RK2 stage a: next = Eh (u + dt/2 k1);  stage b: u_{n+1} = E u + dt Eh k2
template <int MODE, typename T>
__device__ __forceinline__ cx<T> rk4_combine(cx<T> u, cx<T>& a, cx<T> nl, T E, T Eh, T dt) {
  const T d2 = dt * (T)0.5, d3 = dt / (T)3, d6 = dt / (T)6;
  if constexpr (MODE == kStage1) {
    a = cscale(u, E) + cscale(nl, d6 * E);
    return cscale(u + cscale(nl, d2), Eh);
  } else if constexpr (MODE == kStage2) {
    a = a + cscale(nl, d3 * Eh);
    return cscale(u, Eh) + cscale(nl, d2);
  } else if constexpr (MODE == kStage3) {
    a = a + cscale(nl, d3 * Eh);
    return cscale(u, E) + cscale(nl, dt * Eh);
  } else if constexpr (MODE == kStage4) {
    return a + cscale(nl, d6);
  } else if constexpr (MODE == kRk2a) {
    return cscale(u + cscale(nl, d2), Eh);
  } else {
    return cscale(u, E) + cscale(nl, dt * Eh);
  }
}

// Exact linear propagators of one mode, for the Lawson stage combinations
// below; apply(w, d, half, o) sets o = E(t) w with t = dt (half: dt / 2) and d
// the viscous factor exp(-nu k^2 t).
//
// Frame rotating about z: on solenoidal fields the Coriolis force is
// -sigma khat x w, sigma = f kz / |k|, so
//   E(t) w = exp(-nu k^2 t) (cos(sigma t) w - sin(sigma t) khat x w)
// (c1, s1 / c2, s2: cosine and sine of sigma dt and sigma dt / 2).
template <typename T>
struct RotProp {
  static constexpr int NC = 3;
  T kh[3];
  T c1, s1, c2, s2;
  __device__ __forceinline__ void apply(const cx<T> (&w)[3], T d, bool half, cx<T> (&o)[3]) const {
    const T c = half ? c2 : c1, s = half ? s2 : s1;
    const cx<T> x[3] = {cscale(w[2], kh[1]) - cscale(w[1], kh[2]),
                        cscale(w[0], kh[2]) - cscale(w[2], kh[0]),
                        cscale(w[1], kh[0]) - cscale(w[0], kh[1])};
#pragma unroll
    for (int q = 0; q < 3; q++) o[q] = cscale(cscale(w[q], c) - cscale(x[q], s), d);
  }
};

// Stratified (Boussinesq) flow, w = (u, b): the buoyancy force projects to
// b q with q = z - khat khat_z, and a = uz, b oscillate at
// sigma = N |k_h| / |k| (g2 = |k_h|^2 / |k|^2):
//   E(t) (u, b) = exp(-nu k^2 t) (u + [(c - 1) a / g2 + S b] q,  c b - N^2 S a)
// with c = cos(sigma t), S = sin(sigma t) / sigma (t when sigma = 0); cm1 is
// c - 1, computed as -2 sin^2(sigma t / 2).  ig2 = 1 / g2 (0 when k_h = 0,
// where q = 0).
template <typename T>
struct StratProp {
  static constexpr int NC = 4;
  T q[3];
  T ig2, n2;
  T cm1f, sf, cm1h, sh;  // full step, half step
  __device__ __forceinline__ void set(T kx, T ky, T kz, T N2, T dt) {
    const T kh2 = kx * kx + ky * ky, k2 = kh2 + kz * kz;
    const T ik2 = k2 > (T)0 ? (T)1 / k2 : (T)0;
    const T g2 = kh2 * ik2;
    q[0] = -kx * kz * ik2;
    q[1] = -ky * kz * ik2;
    q[2] = g2;
    ig2 = g2 > (T)0 ? (T)1 / g2 : (T)0;
    n2 = N2;
    const T sg = sqrt(N2 * g2);
    // sines and cosines of sigma dt / 4 give both steps by double angles
    const T s4 = sin(sg * dt * (T)0.25), c4 = cos(sg * dt * (T)0.25);
    const T s2 = (T)2 * s4 * c4, c2 = (T)1 - (T)2 * s4 * s4;  // of sigma dt / 2
    cm1h = (T)-2 * s4 * s4;
    cm1f = (T)-2 * s2 * s2;
    if (sg > (T)0) {
      const T isg = (T)1 / sg;
      sh = s2 * isg;
      sf = (T)2 * s2 * c2 * isg;
    } else {
      sh = dt * (T)0.5;
      sf = dt;
    }
  }
  __device__ __forceinline__ void apply(const cx<T> (&w)[4], T d, bool half, cx<T> (&o)[4]) const {
    const T cm1 = half ? cm1h : cm1f, S = half ? sh : sf;
    const cx<T> coef = cscale(w[2], cm1 * ig2) + cscale(w[3], S);
#pragma unroll
    for (int c = 0; c < 3; c++) o[c] = cscale(w[c] + cscale(coef, q[c]), d);
    o[3] = cscale(cscale(w[3], (T)1 + cm1) - cscale(w[2], n2 * S), d);
  }
};

// Rotating and stratified flow, w = (u, b): on a solenoidal mode write
// u = a1 e1 + a2 e2 with e1 = khat x z / g, e2 = khat x e1 (g = |k_h| / |k|;
// e1 = x when k_h = 0).  Coriolis force, buoyancy force and stratification
// couple (a1, a2, b) as
//   a1' = sf a2,  a2' = -sf a1 - g b,  b' = N^2 g a2,   sf = f khat_z,
// a rotation in (a1, a2, b / N) at rate w, w^2 = sf^2 + N^2 g^2, so
// E(t) = I + s K + c K^2 with s = sin(w t) / w, c = (1 - cos(w t)) / w^2
// (t and t^2 / 2 when w = 0), times exp(-nu k^2 t); the khat component of u
// is carried along unchanged.
template <typename T>
struct StratRotProp {
  static constexpr int NC = 4;
  T kh[3], e1[2], e2[3];
  T g, sf, n2;
  T snf, ccf, snh, cch;  // s and c of the full and the half step
  __device__ __forceinline__ void set(T kx, T ky, T kz, T N2, T f, T dt) {
    const T k2 = kx * kx + ky * ky + kz * kz;
    const T ikn = k2 > (T)0 ? (T)1 / sqrt(k2) : (T)0;
    kh[0] = kx * ikn;
    kh[1] = ky * ikn;
    kh[2] = kz * ikn;
    g = sqrt(kh[0] * kh[0] + kh[1] * kh[1]);
    if (g > (T)0) {
      const T ig = (T)1 / g;
      e1[0] = kh[1] * ig;
      e1[1] = -kh[0] * ig;
      e2[0] = kh[0] * kh[2] * ig;
      e2[1] = kh[1] * kh[2] * ig;
      e2[2] = -g;
    } else {
      e1[0] = (T)1;
      e1[1] = (T)0;
      e2[0] = (T)0;
      e2[1] = kh[2];
      e2[2] = (T)0;
    }
    n2 = N2;
    sf = f * kh[2];
    const T w2 = sf * sf + N2 * g * g, w = sqrt(w2);
    // sines and cosines of w dt / 4 give both steps by double angles
    const T s4 = sin(w * dt * (T)0.25), c4 = cos(w * dt * (T)0.25);
    const T s2 = (T)2 * s4 * c4, c2 = (T)1 - (T)2 * s4 * s4;  // of w dt / 2
    if (w > (T)0) {
      const T iw = (T)1 / w, iw2 = (T)1 / w2;
      snh = s2 * iw;
      snf = (T)2 * s2 * c2 * iw;
      cch = (T)2 * s4 * s4 * iw2;
      ccf = (T)2 * s2 * s2 * iw2;
    } else {
      snh = dt * (T)0.5;
      snf = dt;
      cch = dt * dt * (T)0.125;
      ccf = dt * dt * (T)0.5;
    }
  }
  __device__ __forceinline__ void apply(const cx<T> (&w)[4], T d, bool half, cx<T> (&o)[4]) const {
    const T s = half ? snh : snf, c = half ? cch : ccf;
    const cx<T> a0 = cscale(w[0], kh[0]) + cscale(w[1], kh[1]) + cscale(w[2], kh[2]);
    const cx<T> a1 = cscale(w[0], e1[0]) + cscale(w[1], e1[1]);
    const cx<T> a2 = cscale(w[0], e2[0]) + cscale(w[1], e2[1]) + cscale(w[2], e2[2]);
    const T sg = sf * g, ng2 = n2 * g * g;
    const cx<T> m1 = cscale(a1, (T)1 - c * sf * sf) + cscale(a2, s * sf) - cscale(w[3], c * sg);
    const cx<T> m2 = cscale(a2, (T)1 - c * (sf * sf + ng2)) - cscale(a1, s * sf) - cscale(w[3], s * g);
    const cx<T> mb = cscale(w[3], (T)1 - c * ng2) + cscale(a2, s * g * n2) - cscale(a1, c * sg * n2);
    o[0] = cscale(cscale(a0, kh[0]) + cscale(m1, e1[0]) + cscale(m2, e2[0]), d);
    o[1] = cscale(cscale(a0, kh[1]) + cscale(m1, e1[1]) + cscale(m2, e2[1]), d);
    o[2] = cscale(cscale(a0, kh[2]) + cscale(m2, e2[2]), d);
    o[3] = cscale(mb, d);
  }
};

// The mean mode (k = 0).  A periodic pressure has no mean gradient, so the
// linear terms act on the mean unprojected: with Coriolis acceleration
// -f z x u the horizontal mean turns (dux/dt = f uy, duy/dt = -f ux), and
// with buoyancy the vertical mean and the mean buoyancy oscillate at N
// (duz/dt = b, db/dt = -N^2 uz):
//   ux' = c ux + s uy,  uy' = c uy - s ux         (c, s of f t),
//   uz' = cn uz + sn b, b' = cn b - N^2 sn uz    (cn = cos N t, sn = sin(N t) / N,
//                                                 t when N = 0).
// NC = 3: velocity only (uz is carried unchanged).  Viscosity does not act at
// k = 0 (the factor d passed in is 1 there).
template <typename T, int NC_>
struct MeanProp {
  static constexpr int NC = NC_;
  T cf, sf, ch, sh;      // Coriolis: cos and sin of f dt and of f dt / 2
  T cnf, snf, cnh, snh;  // buoyancy: cos(N t) and sin(N t) / N at dt and dt / 2
  T n2;
  __device__ __forceinline__ void set(T f, T N2, T dt) {
    cf = cos(f * dt);
    sf = sin(f * dt);
    ch = cos(f * dt * (T)0.5);
    sh = sin(f * dt * (T)0.5);
    n2 = N2;
    const T nb = sqrt(N2);
    cnf = cos(nb * dt);
    cnh = cos(nb * dt * (T)0.5);
    if (nb > (T)0) {
      snf = sin(nb * dt) / nb;
      snh = sin(nb * dt * (T)0.5) / nb;
    } else {
      snf = dt;
      snh = dt * (T)0.5;
    }
  }
  __device__ __forceinline__ void apply(const cx<T> (&w)[NC], T d, bool half,
                                        cx<T> (&o)[NC]) const {
    const T c = half ? ch : cf, s = half ? sh : sf;
    o[0] = cscale(cscale(w[0], c) + cscale(w[1], s), d);
    o[1] = cscale(cscale(w[1], c) - cscale(w[0], s), d);
    if constexpr (NC == 4) {
      const T cn = half ? cnh : cnf, sn = half ? snh : snf;
      o[2] = cscale(cscale(w[2], cn) + cscale(w[3], sn), d);
      o[3] = cscale(cscale(w[3], cn) - cscale(w[2], n2 * sn), d);
    } else {
      o[2] = cscale(w[2], d);
    }
  }
};

// The Lawson stage combinations of rk4_combine with a propagator acting on
// the NC components of one mode.
template <int MODE, class Prop, typename T, int NC>
__device__ __forceinline__ void prop_combine(const cx<T> (&u)[NC], cx<T> (&a)[NC],
                                             const cx<T> (&nl)[NC], T E, T Eh, T dt,
                                             const Prop& R, cx<T> (&next)[NC]) {
  static_assert(Prop::NC == NC, "propagator and mode vector differ in size");
  const T d2 = dt * (T)0.5, d3 = dt / (T)3, d6 = dt / (T)6;
  cx<T> w[NC], o[NC];
  if constexpr (MODE == kStage1) {
#pragma unroll
    for (int q = 0; q < NC; q++) w[q] = u[q] + cscale(nl[q], d6);
    R.apply(w, E, false, a);
#pragma unroll
    for (int q = 0; q < NC; q++) w[q] = u[q] + cscale(nl[q], d2);
    R.apply(w, Eh, true, next);
  } else if constexpr (MODE == kStage2) {
    R.apply(nl, Eh, true, o);
#pragma unroll
    for (int q = 0; q < NC; q++) a[q] = a[q] + cscale(o[q], d3);
    R.apply(u, Eh, true, o);
#pragma unroll
    for (int q = 0; q < NC; q++) next[q] = o[q] + cscale(nl[q], d2);
  } else if constexpr (MODE == kStage3) {
    R.apply(nl, Eh, true, o);
#pragma unroll
    for (int q = 0; q < NC; q++) a[q] = a[q] + cscale(o[q], d3);
    R.apply(u, E, false, w);
#pragma unroll
    for (int q = 0; q < NC; q++) next[q] = w[q] + cscale(o[q], dt);
  } else if constexpr (MODE == kStage4) {
#pragma unroll
    for (int q = 0; q < NC; q++) next[q] = a[q] + cscale(nl[q], d6);
  } else if constexpr (MODE == kRk2a) {
#pragma unroll
    for (int q = 0; q < NC; q++) w[q] = u[q] + cscale(nl[q], d2);
    R.apply(w, Eh, true, next);
  } else {
    R.apply(nl, Eh, true, o);
    R.apply(u, E, false, w);
#pragma unroll
    for (int q = 0; q < NC; q++) next[q] = w[q] + cscale(o[q], dt);
  }
}

// Non-finite check of the values a lane wrote: one atomic per wave that saw one.
template <typename T>
__device__ __forceinline__ bool nonfinite(cx<T> v) {
  return !(__builtin_isfinite(v.re) && __builtin_isfinite(v.im));
}
__device__ __forceinline__ void flag_wave(unsigned* flag, bool bad) {
  const unsigned long long m = __ballot(bad);
  if (m != 0 && (threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicOr(flag, 1u);
}

// Largest |value| of a velocity sample into a device maximum (non-negative
// doubles order like their bit patterns): wave maximum, then one atomic.
__device__ __forceinline__ void umax_wave(unsigned long long* umax, double m) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmax(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(umax, (unsigned long long)__double_as_longlong(m));
}

// ---------------------------------------------------------------------------
// Strided passes along y: blocks of [XT][M][16] <-> [XT][N][16].
// rows = fields * z extent; grid xcd_grid(rows, XT * YCfg::SUB).
//
// A block transforms whole 128-byte tile rows (16 lines) where it can.  Up to
// N = 512 that is 16 lanes groups of N/8 threads; at N = 1024 in single
// precision 16 groups would need 2048 threads, so each lane carries two
// adjacent lines (F = 2), read and written as one 16-byte access: eight lanes
// then cover a 128-byte row in one instruction (128 KB of LDS per block).
// The inverse pass of a stage (STEP), whose (ux, uy, wz) unit holds two
// lines per lane at once and so runs at 4 waves per SIMD, pairs lines from
// N = 256 on: at N = 512, 512-thread blocks of 16 lines, two per CU, keep as
// many lines in flight per CU as the 8-wave single-line blocks would.
// Elsewhere the block holds LB < 16 lines (LDS and thread limits).
// ---------------------------------------------------------------------------
template <typename T, int N, bool STEP = false>
struct YCfg {
  static constexpr int P = N / 8;
  static constexpr bool kPair = sizeof(T) == 4 &&
                                (STEP ? N >= 256 : kTile * P > 1024) &&
                                (size_t)kTile * N * sizeof(cx<T>) <= 163840;
  static constexpr int F = kPair ? 2 : 1;                              // lines per lane
  static constexpr int LB = kPair ? kTile / 2 : Strided<T, N, kYLines>::LB;  // lane groups
  static constexpr int LINES = LB * F;                                 // lines per block
  static constexpr int SUB = kTile / LINES;
  static constexpr int THREADS = LB * P;
};

// F lines of lane group b at one position: F = 1 one value, F = 2 the two
// adjacent lines 2b, 2b + 1 as one 16-byte access (non-temporal)
template <typename T, int F>
__device__ __forceinline__ void ld_lines(const cx<T>* p, cx<T> (&v)[F][8], int e) {
  if constexpr (F == 1) {
    v[0][e] = ld_nt(p);
  } else {
    typedef T v4 __attribute__((ext_vector_type(4)));
    const v4 x = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
    v[0][e] = cx<T>{x.x, x.y};
    v[1][e] = cx<T>{x.z, x.w};
  }
}
template <typename T, int F>
__device__ __forceinline__ void st_lines(cx<T>* p, const cx<T> (&v)[F][8], int e) {
  if constexpr (F == 1) {
    st_nt(p, v[0][e]);
  } else {
    typedef T v4 __attribute__((ext_vector_type(4)));
    v4 x;
    x.x = v[0][e].re;
    x.y = v[0][e].im;
    x.z = v[1][e].re;
    x.w = v[1][e].im;
    __builtin_nontemporal_store(x, reinterpret_cast<v4*>(p));
  }
}

template <typename T, int N, bool FULL>
__global__ void __launch_bounds__((YCfg<T, N>::THREADS))
    k_y_inv(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
            const cx<T>* __restrict__ tw, int rows) {
  using G = Geo<N, FULL>;
  using C = YCfg<T, N>;
  constexpr int F = C::F;
  __shared__ cx<T> lds[C::LINES * N];
  const int b = threadIdx.x % C::LB, t = threadIdx.x / C::LB;
  const Twiddles<T, N, false> twr(tw, t);
  int row, rem;
  if (!xcd_row_block(rows, G::XT * C::SUB, row, rem)) return;  // whole block
  const int sub = rem % C::SUB;
  const size_t tile = (size_t)row * G::XT + rem / C::SUB;  // row = field*nz + z
  const cx<T>* src = in + tile * G::M * kTile + sub * C::LINES + F * b;
  cx<T> v[F][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int j = G::i2j(t + e * G::P);
    if (j >= 0) {
      ld_lines<T, F>(&src[j * kTile], v, e);
    } else {
#pragma unroll
      for (int f = 0; f < F; f++) v[f][e] = cx<T>{0, 0};
    }
  }
  fft_lines<T, N, +1, F>(v, t, lds, [=](int f, int pos) { return pos * C::LINES + F * b + f; },
                         twr);
  cx<T>* dst = out + tile * N * kTile + sub * C::LINES + F * b;
#pragma unroll
  for (int e = 0; e < 8; e++) st_lines<T, F>(&dst[(t + e * G::P) * kTile], v, e);
}

// The pointer as a value the compiler cannot see through: loads from it
// stay below this point (loads through a read-only kernel argument may
// otherwise be scheduled anywhere, barriers included).
template <typename P>
__device__ __forceinline__ P* opaque_ptr(P* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// ---------------------------------------------------------------------------
// Inverse y pass of a stage: Wm (fields ux uy uz wx wy [b]) -> Wn (fields ux
// uy uz wz wx wy [b]).  The vertical vorticity wz = i (kx uy - ky ux) needs
// no kz, so it is formed here from the ux, uy lines the pass reads anyway
// rather than transformed and stored by the z pass: one field fewer written
// there and read here.  Each z plane has `units` row units: unit 0 reads ux,
// uy and writes ux, uy, wz; unit u >= 1 carries Wm field u + 1 to Wn field
// u + 2 (uz to field 2).  rows = units * N; grid xcd_grid(rows, XT * SUB).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__((YCfg<T, N, true>::THREADS), 4)
    k_y_inv_step(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                 const cx<T>* __restrict__ tw, T kb, int rows) {
  using G = Geo<N, false>;
  using C = YCfg<T, N, true>;
  constexpr int F = C::F;
  constexpr int P = G::P;
  __shared__ cx<T> lds[C::LINES * N];
  const int b = threadIdx.x % C::LB, t = threadIdx.x / C::LB;
  int row, rem;
  if (!xcd_row_block(rows, G::XT * C::SUB, row, rem)) return;  // whole block
  const int unit = row / N, z = row % N;
  const int xt = rem / C::SUB;
  const int lane = (rem % C::SUB) * C::LINES + F * b;  // first line of the lane in its tile
  auto lidx = [=](int f, int pos) { return pos * C::LINES + F * b + f; };
  const size_t zoff = (size_t)z * G::XT + xt;
  const int fin = unit == 0 ? 0 : unit + 1;
  const int fout = unit == 0 ? 0 : (unit == 1 ? 2 : unit + 2);
  const cx<T>* src = in + G::wm_row(fin, xt, z) + lane;
  cx<T>* dst = out + (zoff + (size_t)fout * N * G::XT) * N * kTile + lane;
  cx<T> v[F][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int j = G::i2j(t + e * P);
    if (j >= 0) {
      ld_lines<T, F>(&src[j * kTile], v, e);
    } else {
#pragma unroll
      for (int f = 0; f < F; f++) v[f][e] = cx<T>{0, 0};
    }
  }
  if (unit != 0) {
    const Twiddles<T, N, false> twr(tw, t);
    fft_lines<T, N, +1, F>(v, t, lds, lidx, twr);
#pragma unroll
    for (int e = 0; e < 8; e++) st_lines<T, F>(&dst[(t + e * P) * kTile], v, e);
    return;
  }
  // unit 0: wz = i (kx uy - ky ux), its ky part from ux first
  cx<T> w[F][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int j = G::i2j(t + e * P);
    const T ky = j >= 0 ? kb * (T)G::jmode(j) : (T)0;
#pragma unroll
    for (int f = 0; f < F; f++) w[f][e] = mul_i(cscale(v[f][e], -ky));
  }
  {
    // twiddles read afresh for every transform: shared by the block's
    // transforms, their values would stay in registers across all of them
    const Twiddles<T, N, false> twr(opaque_ptr(tw), t);
    fft_lines<T, N, +1, F>(v, t, lds, lidx, twr);
  }
#pragma unroll
  for (int e = 0; e < 8; e++) st_lines<T, F>(&dst[(t + e * P) * kTile], v, e);
  // uy is loaded only now: hoisted above the ux transform, its loads would
  // hold a third line of registers through it
  const cx<T>* src1 = opaque_ptr(in) + G::wm_row(1, xt, z) + lane;
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int j = G::i2j(t + e * P);
    if (j >= 0) {
      ld_lines<T, F>(&src1[j * kTile], v, e);
    } else {
#pragma unroll
      for (int f = 0; f < F; f++) v[f][e] = cx<T>{0, 0};
    }
  }
#pragma unroll
  for (int f = 0; f < F; f++) {
    const T kx = kb * (T)(xt * kTile + lane + f);
#pragma unroll
    for (int e = 0; e < 8; e++) w[f][e] = w[f][e] + mul_i(cscale(v[f][e], kx));
  }
  {
    const Twiddles<T, N, false> twr(opaque_ptr(tw), t);
    fft_lines<T, N, +1, F>(v, t, lds, lidx, twr);
  }
  cx<T>* dst1 = dst + (size_t)N * G::XT * N * kTile;
#pragma unroll
  for (int e = 0; e < 8; e++) st_lines<T, F>(&dst1[(t + e * P) * kTile], v, e);
  {
    const Twiddles<T, N, false> twr(opaque_ptr(tw), t);
    fft_lines<T, N, +1, F>(w, t, lds, lidx, twr);
  }
  cx<T>* dst3 = dst + (size_t)3 * N * G::XT * N * kTile;
#pragma unroll
  for (int e = 0; e < 8; e++) st_lines<T, F>(&dst3[(t + e * P) * kTile], w, e);
}

// (the forward pass of a stage, !FULL, pairs lines as the inverse one does)
template <typename T, int N, bool FULL>
__global__ void __launch_bounds__((YCfg<T, N, !FULL>::THREADS))
    k_y_fwd(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
            const cx<T>* __restrict__ tw, int rows) {
  using G = Geo<N, FULL>;
  using C = YCfg<T, N, !FULL>;
  constexpr int F = C::F;
  __shared__ cx<T> lds[C::LINES * N];
  const int b = threadIdx.x % C::LB, t = threadIdx.x / C::LB;
  const Twiddles<T, N, false> twr(tw, t);
  int row, rem;
  if (!xcd_row_block(rows, G::XT * C::SUB, row, rem)) return;  // whole block
  const int sub = rem % C::SUB;
  const size_t tile = (size_t)row * G::XT + rem / C::SUB;  // row = field*nz + z
  const cx<T>* src = in + tile * N * kTile + sub * C::LINES + F * b;
  cx<T> v[F][8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    if constexpr (F == 1) {
      v[0][e] = src[(t + e * G::P) * kTile];
    } else {
      typedef T v4 __attribute__((ext_vector_type(4)));
      const v4 x = *reinterpret_cast<const v4*>(&src[(t + e * G::P) * kTile]);
      v[0][e] = cx<T>{x.x, x.y};
      v[1][e] = cx<T>{x.z, x.w};
    }
  }
  fft_lines<T, N, -1, F>(v, t, lds, [=](int f, int pos) { return pos * C::LINES + F * b + f; },
                         twr);
  const size_t orow = FULL ? tile * G::M * kTile
                           : G::wm_row(row / N, rem / C::SUB, row % N);
  cx<T>* dst = out + orow + sub * C::LINES + F * b;
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int j = G::i2j(t + e * G::P);
    if (j >= 0) st_lines<T, F>(&dst[j * kTile], v, e);
  }
}

// ---------------------------------------------------------------------------
// Real-transform helpers for the x passes.
// Two real lines a(x), b(x) travel as one complex line a + i b:
//   inverse: Z[k] = A[k] + i B[k], with A[N-k] = conj A[k] (k > N/2);
//            the imaginary parts of the self-conjugate A[0], A[N/2] are
//            dropped (the real part of the inverse of the Hermitian
//            completion, as C2R defines);
//   forward: A[k] = (Z[k] + conj Z[N-k]) / 2,  B[k] = (Z[k] - conj Z[N-k]) / 2i.
// ---------------------------------------------------------------------------
template <typename T, int N, bool FULL, class FA, class FB>
__device__ __forceinline__ cx<T> c2r_pair_at(int k, FA fa, FB fb) {
  using G = Geo<N, FULL>;
  if (k <= G::K) {
    cx<T> A = fa(k), B = fb(k);
    if (k == 0 || (FULL && k == N / 2)) {
      A.im = 0;
      B.im = 0;
    }
    return {A.re - B.im, A.im + B.re};
  } else if (k >= N - G::K) {
    const int m = N - k;
    cx<T> A = fa(m), B = fb(m);
    return {A.re + B.im, B.re - A.im};
  }
  return {0, 0};
}

template <typename T>
__device__ __forceinline__ void r2c_untangle(cx<T> zk, cx<T> zn, cx<T>& A, cx<T>& B) {
  const T h = (T)0.5;
  A = {(zk.re + zn.re) * h, (zk.im - zn.im) * h};
  B = {(zk.im + zn.im) * h, (zn.re - zk.re) * h};
}

}  // namespace fs
