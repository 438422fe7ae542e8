// ops2d.hip -- launch sequences of the 2D solver for every supported size.
#include <algorithm>
#include <cmath>

#include "fs_internal.h"
#include "ns2d_kernels.h"
#include "ns3d_kernels.h"

namespace fs {
namespace {

template <typename T>
StageArgs<T> stage_args2(Plan* p, void* state, void* tend) {
  StageArgs<T> a{};
  a.state = (cx<T>*)state;
  a.acc = (cx<T>*)p->acc;
  a.tend = (cx<T>*)tend;
  a.vband = nullptr;
  a.alpha = nullptr;
  a.e1 = (const T*)p->e1;
  a.eh1 = (const T*)p->eh1;
  a.tw = (const cx<T>*)p->tw;
  a.kb = (T)(2.0 * M_PI / p->L);
  a.dt = (T)p->dt;
  a.dtp = (const T*)p->dtdev;
  a.sin = (cx<T>*)p->sin;
  a.n2 = (T)p->n2;
  a.bw = 0;
  a.m2min = 0;
  a.m2max = -1;
  a.nonfin = (p->flags & FS_CHECK_FINITE) ? p->nonfin : nullptr;
  return a;
}

template <typename T, int N, int NF>
struct L2 {
  using G = Geo<N, false>;
  using GF = Geo<N, true>;
  using C = Strided<T, N>;
  using R = RowPairs<N>;
  static constexpr int LB = C::LB, RP = R::RP;
  static cx<T>* A(Plan* p) { return (cx<T>*)p->bufA; }
  static cx<T>* B(Plan* p) { return (cx<T>*)p->bufB; }
  static const cx<T>* TW(Plan* p) { return (const cx<T>*)p->tw; }
  static Batch one(int bpr) { return Batch{nullptr, 0, 0, 0, bpr}; }

  static void p1(Plan* p, const void* state) {
    p->begin(KID_P1);
    hipLaunchKernelGGL((k2_p1<T, N, LB, NF>), dim3(G::XT * kTile / LB), dim3(LB * N / 8), 0,
                       p->launch, (const cx<T>*)state, A(p),
                       stage_args2<T>(p, (void*)state, nullptr), one(G::XT * kTile / LB));
    launched(p, "k2_p1");
    p->end(KID_P1);
  }
  static void x(Plan* p, bool umax = false) {
    p->begin(KID_X);
    hipLaunchKernelGGL((k2_x<T, N, RP, NF>), dim3(N / 2 / RP), dim3(RP * N / 8), 0, p->launch,
                       (const cx<T>*)A(p), B(p), TW(p), (T)(1.0 / ((double)N * N)), one(N / 2 / RP),
                       umax ? p->umaxdev : nullptr);
    launched(p, "k2_x");
    p->end(KID_X);
  }
  template <int MODE>
  static void yk(Plan* p, void* state, void* tend, int do_p1) {
    p->begin(KID_Z);
    hipLaunchKernelGGL((k2_y<T, N, LB, MODE, NF>), dim3(G::XT * kTile / LB), dim3(LB * N / 8), 0,
                       p->launch, (const cx<T>*)B(p), A(p), stage_args2<T>(p, state, tend),
                       one(G::XT * kTile / LB), do_p1);
    launched(p, "k2_y");
    p->end(KID_Z);
  }
  static void stage(Plan* p, void* state, int mode, int do_p1) {
    const bool adapt = p->cfl > 0 && (mode == kStage1 || mode == kRk2a);
    x(p, adapt);
    if (adapt) launch_dtstep<T>(p);
    switch (mode) {
      case kStage1: yk<kStage1>(p, state, nullptr, 1); break;
      case kStage2: yk<kStage2>(p, state, nullptr, 1); break;
      case kStage3: yk<kStage3>(p, state, nullptr, 1); break;
      case kRk2a: yk<kRk2a>(p, state, nullptr, 1); break;
      case kRk2b: yk<kRk2b>(p, state, nullptr, do_p1); break;
      default: yk<kStage4>(p, state, nullptr, do_p1); break;
    }
  }
  static void tendency(Plan* p, const void* state, void* out, bool, bool fill) {
    if (fill) launch_fill<T>(p, out, (size_t)NF * N * (N / 2 + 1));
    p1(p, state);
    x(p);
    yk<kModeTend>(p, (void*)state, out, 0);
  }
  static void fft_inv(Plan* p, const void* spec, void* phys) {
    p->begin(KID_FFT);
    hipLaunchKernelGGL((k2f_y_inv<T, N>), dim3(GF::XT * C::SUB), dim3(C::THREADS), 0, p->launch,
                       (const cx<T>*)spec, B(p), TW(p));
    launched(p, "k2f_y_inv");
    p->end(KID_FFT);
    p->begin(KID_FFT);
    hipLaunchKernelGGL((kf_x_c2r<T, N>), dim3(N / 2 / R::RP, 1), dim3(R::THREADS), 0, p->launch,
                       (const cx<T>*)B(p), (T*)phys, TW(p));
    launched(p, "kf_x_c2r");
    p->end(KID_FFT);
  }
  static void fft_fwd(Plan* p, const void* phys, void* spec) {
    p->begin(KID_FFT);
    hipLaunchKernelGGL((kf_x_r2c<T, N>), dim3(N / 2 / R::RP, 1), dim3(R::THREADS), 0, p->launch,
                       (const T*)phys, B(p), TW(p), (T)(1.0 / ((double)N * N)));
    launched(p, "kf_x_r2c");
    p->end(KID_FFT);
    p->begin(KID_FFT);
    hipLaunchKernelGGL((k2f_y_fwd<T, N>), dim3(GF::XT * C::SUB), dim3(C::THREADS), 0, p->launch,
                       (const cx<T>*)B(p), (cx<T>*)spec, TW(p));
    launched(p, "k2f_y_fwd");
    p->end(KID_FFT);
  }
  static Ops ops() {
    Ops o{};
    o.p1 = p1;
    o.stage = stage;
    o.tendency = tendency;
    o.fft_fwd = fft_fwd;
    o.fft_inv = fft_inv;
    o.alpha = nullptr;
    o.diag = launch_diag<T>;
    o.dtstep = launch_dtstep<T>;
    o.transfer = launch_transfer<T>;
    o.spectra1d = launch_spectra1d<T>;
    o.structure = launch_structure<T>;
    const size_t wn3 = (size_t)(2 + NF) * G::XT * N * kTile;  // (u, v, w[, b])
    const size_t wn2 = (size_t)2 * NF * G::XT * N * kTile;    // products
    const size_t wfull = (size_t)GF::XT * N * kTile;
    // diagnostics keep one spectral and one physical field in A
    const size_t two = wfull + (size_t)N * (N / 2 + 1);
    o.elems_a = std::max({wn3, wfull, two});
    o.elems_full = wfull;
    o.elems_b = wn2 > wfull ? wn2 : wfull;
    o.elems_acc = (size_t)NF * G::XT * G::M * kTile;
    o.elems_sin = NF > 1 ? (size_t)NF * G::XT * G::M * kTile : 0;
    return o;
  }
};

}  // namespace

template <typename T, int NF>
Ops ops2_of(int n) {
  switch (n) {
    case 16: return L2<T, 16, NF>::ops();
    case 32: return L2<T, 32, NF>::ops();
    case 64: return L2<T, 64, NF>::ops();
    case 128: return L2<T, 128, NF>::ops();
    case 256: return L2<T, 256, NF>::ops();
    case 512: return L2<T, 512, NF>::ops();
    case 1024: return L2<T, 1024, NF>::ops();
    default: return Ops{};
  }
}

template <typename T>
Ops make_ops2(int n, int nfield) {
  return nfield == 2 ? ops2_of<T, 2>(n) : ops2_of<T, 1>(n);
}

template Ops make_ops2<float>(int, int);
template Ops make_ops2<double>(int, int);

}  // namespace fs
