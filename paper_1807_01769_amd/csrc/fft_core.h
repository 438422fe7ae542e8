// fft_core.h -- register-resident Stockham FFT for CDNA (wave64).
//
// One transform line of length N (power of two, 16..1024) is owned by
// P = N/8 lanes; lane t holds the 8 values at positions t + e*P (e = 0..7).
// Every stage is a set of radix-8 (or a final radix-4/2) butterflies done
// in registers; between stages the values move through LDS once (write at
// the Stockham output position, barrier, read back at t + e*P, barrier).
// With this ownership the last stage leaves lane t holding X[t + e*P], so
// passes load their input straight from global memory in that pattern and
// store results straight back -- no LDS on the way in or out.
//
// Twiddles come from a per-size table W[m] = exp(-2 pi i m / N) built in FP64
// on the host and rounded once to T (round to nearest even).
#pragma once
#include <hip/hip_runtime.h>

namespace fs {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) {
  return {a.re * s, a.im * s};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> conjg(cx<T> a) {
  return {a.re, -a.im};
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  return {-a.im, a.re};
}
// (S i) * a, S = -1 (forward) or +1 (inverse)
template <int S, typename T>
__host__ __device__ __forceinline__ cx<T> mul_si(cx<T> a) {
  if constexpr (S < 0)
    return {a.im, -a.re};
  else
    return {-a.im, a.re};
}

template <int S, typename T>
__host__ __device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a;
  a = t + b;
  b = t - b;
}

template <int S, typename T>
__host__ __device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_si<S>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

// 8-point DFT in natural order: two 4-point DFTs (even/odd inputs) and the
// eighth-root rotations exp(S i pi k / 4), k = 1..3, on the odd half.
template <int S, typename T>
__host__ __device__ __forceinline__ void dft8(cx<T>& v0, cx<T>& v1, cx<T>& v2, cx<T>& v3,
                                              cx<T>& v4, cx<T>& v5, cx<T>& v6, cx<T>& v7) {
  const T c = (T)0.70710678118654752440084436210485;
  dft4<S>(v0, v2, v4, v6);  // E0..E3 in v0, v2, v4, v6
  dft4<S>(v1, v3, v5, v7);  // O0..O3 in v1, v3, v5, v7
  cx<T> o1 = v3, o2 = v5, o3 = v7;
  // (a + ib)(1 + S i)/sqrt2 and (a + ib)(-1 + S i)/sqrt2
  o1 = {(o1.re - (T)S * o1.im) * c, (o1.im + (T)S * o1.re) * c};
  o2 = mul_si<S>(o2);
  o3 = {(-o3.re - (T)S * o3.im) * c, (-o3.im + (T)S * o3.re) * c};
  cx<T> e0 = v0, e1 = v2, e2 = v4, e3 = v6, o0 = v1;
  v0 = e0 + o0;
  v4 = e0 - o0;
  v1 = e1 + o1;
  v5 = e1 - o1;
  v2 = e2 + o2;
  v6 = e2 - o2;
  v3 = e3 + o3;
  v7 = e3 - o3;
}

// Radix of the stage that starts with sub-transform length NS.
template <int N, int NS>
struct StageRadix {
  static constexpr int value = (N / NS >= 8) ? 8 : N / NS;
};

// Stage bookkeeping: stage s starts with sub-transform length NS(s) = 8^s
// (the last stage may have radix 4 or 2).
template <int N>
struct Stages {
  static constexpr int count() {
    int c = 0;
    for (int ns = 1; ns < N; ns *= (N / ns >= 8 ? 8 : N / ns)) c++;
    return c;
  }
  static constexpr int C = count();
};

// Per-lane twiddles.  With REGS every lane loads the twiddles of all its
// butterflies once (w[s][q*(R-1) + r-1] = W^{r k N/(NS R)}, k = (t + qP) mod
// NS) and keeps them in registers for every transform of the kernel (worth
// it when a kernel runs several transforms); otherwise they are read from
// the table when used.  FP64 always reads the table (register budget).
template <typename T, int N, bool REGS = true>
struct Twiddles {
  static constexpr bool kRegs = REGS && sizeof(T) == 4;
  static constexpr int C = Stages<N>::C;
  cx<T> w[kRegs ? C : 1][7];
  const cx<T>* __restrict__ tab;

  __device__ __forceinline__ Twiddles(const cx<T>* __restrict__ table, int t) : tab(table) {
    if constexpr (kRegs) load_stage<1, 0>(t);
  }
  template <int NS, int S_>
  __device__ __forceinline__ void load_stage(int t) {
    constexpr int P = N / 8;
    constexpr int R = StageRadix<N, NS>::value;
    constexpr int NB = 8 / R;
    if constexpr (NS > 1) {
#pragma unroll
      for (int q = 0; q < NB; q++) {
        const int k = (t + q * P) & (NS - 1);
#pragma unroll
        for (int r = 1; r < R; r++) w[S_][q * (R - 1) + r - 1] = tab[r * k * (N / (NS * R))];
      }
    }
    if constexpr (NS * R < N) load_stage<NS * R, (NS > 1 ? S_ + 1 : S_)>(t);
  }
  // twiddle of register (q, r) of stage S_ (index NS) for lane t
  template <int NS, int S_>
  __device__ __forceinline__ cx<T> get(int t, int q, int r) const {
    if constexpr (kRegs) {
      constexpr int R = StageRadix<N, NS>::value;
      return w[S_][q * (R - 1) + r - 1];
    } else {
      constexpr int P = N / 8;
      constexpr int R = StageRadix<N, NS>::value;
      const int k = (t + q * P) & (NS - 1);
      return tab[r * k * (N / (NS * R))];
    }
  }
};

// Butterflies of one Stockham stage on lane t's 8 registers.  A radix-R
// stage does 8/R butterflies per lane: butterfly q is j = t + q*P and uses
// registers q + (8/R)*r, r = 0..R-1.
template <typename T, int N, int S, int NS, int SI, class TW>
__host__ __device__ __forceinline__ void stage_bfly(cx<T> (&v)[8], int t, const TW& tw) {
  constexpr int R = StageRadix<N, NS>::value;
  constexpr int NB = 8 / R;
#pragma unroll
  for (int q = 0; q < NB; q++) {
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; r++) {
        cx<T> w = tw.template get<NS, SI>(t, q, r);
        if constexpr (S > 0) w.im = -w.im;
        v[q + NB * r] = cmul(v[q + NB * r], w);
      }
    }
    if constexpr (R == 8) {
      dft8<S>(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
    } else if constexpr (R == 4) {
      dft4<S>(v[q], v[q + 2], v[q + 4], v[q + 6]);
    } else {
      dft2<S>(v[q], v[q + 4]);
    }
  }
}

// Stockham output position of register e of lane t after the stage NS.
template <int N, int NS>
__host__ __device__ __forceinline__ int stage_out_pos(int t, int e) {
  constexpr int P = N / 8;
  constexpr int R = StageRadix<N, NS>::value;
  constexpr int NB = 8 / R;
  const int q = e % NB, r = e / NB;
  const int j = t + q * P;
  return (j / NS) * NS * R + (j & (NS - 1)) + r * NS;
}

// F lines per lane, transformed together (they share the barriers).
// `idx(f, pos)` maps (line f of this lane, position) to an LDS element
// offset; the caller owns disjoint LDS for every (lane group, line).
// Every lane of the block must call this (it contains __syncthreads).
template <typename T, int N, int S, int F, int NS = 1, int SI = 0, class Idx, class TW>
__device__ __forceinline__ void fft_lines(cx<T> (&v)[F][8], int t, cx<T>* lds, Idx idx,
                                          const TW& tw) {
  constexpr int P = N / 8;
  constexpr int R = StageRadix<N, NS>::value;
#pragma unroll
  for (int f = 0; f < F; f++) stage_bfly<T, N, S, NS, SI>(v[f], t, tw);
  if constexpr (NS * R < N) {
#pragma unroll
    for (int f = 0; f < F; f++)
#pragma unroll
      for (int e = 0; e < 8; e++) lds[idx(f, stage_out_pos<N, NS>(t, e))] = v[f][e];
    __syncthreads();
#pragma unroll
    for (int f = 0; f < F; f++)
#pragma unroll
      for (int e = 0; e < 8; e++) v[f][e] = lds[idx(f, t + e * P)];
    __syncthreads();
    fft_lines<T, N, S, F, NS * R, (NS > 1 ? SI + 1 : SI)>(v, t, lds, idx, tw);
  }
}

}  // namespace fs
