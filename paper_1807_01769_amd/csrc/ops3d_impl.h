// ops3d_impl.h -- launch sequences of the 3D solver for every supported size.
// Included by one small translation unit per (precision, Boussinesq) pair,
// so that the four sets of kernels compile in parallel.
#pragma once
#include <algorithm>
#include <cmath>

#include "fs_internal.h"
#include "ns3d_kernels.h"

namespace fs {
namespace ops3d_detail {

template <typename T>
StageArgs<T> stage_args(Plan* p, void* state, void* tend) {
  StageArgs<T> a{};
  a.state = (cx<T>*)state;
  a.acc = (cx<T>*)p->acc;
  a.tend = (cx<T>*)tend;
  a.vband = (cx<T>*)p->vband;
  a.alpha = (const T*)p->alpha;
  a.e1 = (const T*)p->e1;
  a.eh1 = (const T*)p->eh1;
  a.tw = (const cx<T>*)p->tw;
  a.kb = (T)(2.0 * M_PI / p->L);
  a.dt = (T)p->dt;
  a.dtp = (const T*)p->dtdev;
  a.sin = nullptr;
  a.n2 = (T)p->n2;
  a.rotf = (T)p->rotf;
  a.bw = p->bw;
  a.m2min = p->m2min;
  a.m2max = p->m2max;
  a.nonfin = (p->flags & FS_CHECK_FINITE) ? p->nonfin : nullptr;
  return a;
}

// STRAT: Boussinesq flow (state u, b; seven inverse and six forward fields)
template <typename T, int N, bool STRAT>
struct L3 {
  static constexpr int NC = STRAT ? 4 : 3;    // state components
  static constexpr int FINV = STRAT ? 7 : 6;  // fields of the x pass's input
  static constexpr int FZ = FINV - 1;         // fields of the z pass's output (no wz)
  static constexpr int FFWD = STRAT ? 6 : 3;  // fields of the forward passes
  using G = Geo<N, false>;
  using GF = Geo<N, true>;
  using C = Strided<T, N>;
  using YC = YCfg<T, N>;
  using ZC = ZCfg<T, N, NC>;
  using R = RowPairs<N>;
  static cx<T>* A(Plan* p) { return (cx<T>*)p->bufA; }
  static cx<T>* B(Plan* p) { return (cx<T>*)p->bufB; }
  static const cx<T>* TW(Plan* p) { return (const cx<T>*)p->tw; }

  static void p1(Plan* p, const void* state) {
    p->begin(KID_P1);
    hipLaunchKernelGGL((k3_p1<T, N, NC>), dim3(xcd_grid(G::M, G::XT * ZC::SUB)), dim3(ZC::THREADS), 0,
                       p->launch, (const cx<T>*)state, A(p),
                       stage_args<T>(p, (void*)state, nullptr));
    launched(p, "k3_p1");
    p->end(KID_P1);
  }
  static void yinv(Plan* p) {
    p->begin(KID_YINV);
    // row units per z plane: (ux, uy -> ux, uy, wz) and one per other field
    constexpr int units = FINV - 2;
    using YS = YCfg<T, N, true>;
    hipLaunchKernelGGL((k_y_inv_step<T, N>), dim3(xcd_grid(units * N, G::XT * YS::SUB)),
                       dim3(YS::THREADS), 0, p->launch, (const cx<T>*)A(p), B(p), TW(p),
                       (T)(2.0 * M_PI / p->L), units * N);
    launched(p, "k_y_inv_step");
    p->end(KID_YINV);
  }
  static void x(Plan* p, bool umax = false) {
    p->begin(KID_X);
    using XR = XRows<T, N, STRAT>;
    hipLaunchKernelGGL((k3_x<T, N, STRAT>), dim3(N / 2 / XR::RP, N), dim3(XR::THREADS), 0, p->launch,
                       (const cx<T>*)B(p), A(p), TW(p), (T)(1.0 / ((double)N * N * N)),
                       umax ? p->umaxdev : nullptr);
    launched(p, "k3_x");
    p->end(KID_X);
  }
  static void yfwd(Plan* p) {
    p->begin(KID_YFWD);
    using YS = YCfg<T, N, true>;
    hipLaunchKernelGGL((k_y_fwd<T, N, false>), dim3(xcd_grid(FFWD * N, G::XT * YS::SUB)),
                       dim3(YS::THREADS), 0, p->launch, (const cx<T>*)A(p), B(p), TW(p), FFWD * N);
    launched(p, "k_y_fwd");
    p->end(KID_YFWD);
  }
  template <int MODE>
  static void zk(Plan* p, void* state, void* tend, int do_p1) {
    p->begin(KID_Z);
    const dim3 grid(xcd_grid(G::M, G::XT * ZC::SUB));
    if constexpr (STRAT) {
      if (MODE != kModeTend && p->rotf != 0.0)
        hipLaunchKernelGGL((k3_z<T, N, MODE, kPropStratRot>), grid, dim3(ZC::THREADS), 0,
                           p->launch, (const cx<T>*)B(p), A(p), stage_args<T>(p, state, tend), do_p1);
      else
        hipLaunchKernelGGL((k3_z<T, N, MODE, kPropStrat>), grid, dim3(ZC::THREADS), 0, p->launch,
                           (const cx<T>*)B(p), A(p), stage_args<T>(p, state, tend), do_p1);
    } else if (MODE != kModeTend && p->rotf != 0.0)
      hipLaunchKernelGGL((k3_z<T, N, MODE, kPropRot>), grid, dim3(ZC::THREADS), 0, p->launch,
                         (const cx<T>*)B(p), A(p), stage_args<T>(p, state, tend), do_p1);
    else
      hipLaunchKernelGGL((k3_z<T, N, MODE>), grid, dim3(ZC::THREADS), 0, p->launch,
                         (const cx<T>*)B(p), A(p), stage_args<T>(p, state, tend), do_p1);
    launched(p, "k3_z");
    p->end(KID_Z);
  }
  static void stage(Plan* p, void* state, int mode, int do_p1) {
    const bool adapt = p->cfl > 0 && (mode == kStage1 || mode == kRk2a);
    yinv(p);
    x(p, adapt);
    if (adapt) launch_dtstep<T>(p);
    yfwd(p);
    switch (mode) {
      case kStage1: zk<kStage1>(p, state, nullptr, 1); break;
      case kStage2: zk<kStage2>(p, state, nullptr, 1); break;
      case kStage3: zk<kStage3>(p, state, nullptr, 1); break;
      case kRk2a: zk<kRk2a>(p, state, nullptr, 1); break;
      case kRk2b: zk<kRk2b>(p, state, nullptr, do_p1); break;
      default: zk<kStage4>(p, state, nullptr, do_p1); break;
    }
  }
  static void tendency(Plan* p, const void* state, void* out, bool fresh_alpha, bool fill) {
    if (fill) launch_fill<T>(p, out, (size_t)NC * N * N * (N / 2 + 1));
    if (p->m2max >= 0 && fresh_alpha) launch_alpha<T>(p, state);
    p1(p, state);
    yinv(p);
    x(p);
    yfwd(p);
    zk<kModeTend>(p, (void*)state, out, 0);
  }
  // nf stacked fields through caller workspaces wa, wb (elems_full each per
  // field); grad: spec is a velocity state and the nf = 9 outputs are its
  // gradients d u_i / d x_j (field 3i + j) on the kept modes
  static void fft_inv_n(Plan* p, const void* spec, void* phys, int nf, void* wa, void* wb,
                        bool grad) {
    p->begin(KID_FFT);
    if (grad)
      hipLaunchKernelGGL((k3f_z_inv<T, N, true>), dim3(N * GF::XT * C::SUB, 9), dim3(C::THREADS),
                         0, p->launch, (const cx<T>*)spec, (cx<T>*)wa, TW(p),
                         (T)(2.0 * M_PI / p->L));
    else
      hipLaunchKernelGGL((k3f_z_inv<T, N>), dim3(N * GF::XT * C::SUB, nf), dim3(C::THREADS), 0,
                         p->launch, (const cx<T>*)spec, (cx<T>*)wa, TW(p), (T)0);
    launched(p, "k3f_z_inv");
    p->end(KID_FFT);
    p->begin(KID_FFT);
    hipLaunchKernelGGL((k_y_inv<T, N, true>), dim3(xcd_grid(nf * N, GF::XT * YC::SUB)),
                       dim3(YC::THREADS), 0, p->launch, (const cx<T>*)wa, (cx<T>*)wb, TW(p),
                       nf * N);
    launched(p, "k_y_inv full");
    p->end(KID_FFT);
    p->begin(KID_FFT);
    hipLaunchKernelGGL((kf_x_c2r<T, N>), dim3(N / 2 / R::RP, nf * N), dim3(R::THREADS), 0,
                       p->launch, (const cx<T>*)wb, (T*)phys, TW(p));
    launched(p, "kf_x_c2r");
    p->end(KID_FFT);
  }
  static void fft_fwd_n(Plan* p, const void* phys, void* spec, int nf, void* wa, void* wb) {
    p->begin(KID_FFT);
    hipLaunchKernelGGL((kf_x_r2c<T, N>), dim3(N / 2 / R::RP, nf * N), dim3(R::THREADS), 0,
                       p->launch, (const T*)phys, (cx<T>*)wb, TW(p),
                       (T)(1.0 / ((double)N * N * N)));
    launched(p, "kf_x_r2c");
    p->end(KID_FFT);
    p->begin(KID_FFT);
    hipLaunchKernelGGL((k_y_fwd<T, N, true>), dim3(xcd_grid(nf * N, GF::XT * YC::SUB)),
                       dim3(YC::THREADS), 0, p->launch, (const cx<T>*)wb, (cx<T>*)wa, TW(p),
                       nf * N);
    launched(p, "k_y_fwd full");
    p->end(KID_FFT);
    p->begin(KID_FFT);
    hipLaunchKernelGGL((k3f_z_fwd<T, N>), dim3(N * GF::XT * C::SUB, nf), dim3(C::THREADS), 0,
                       p->launch, (const cx<T>*)wa, (cx<T>*)spec, TW(p));
    launched(p, "k3f_z_fwd");
    p->end(KID_FFT);
  }
  static void fft_inv(Plan* p, const void* spec, void* phys) {
    fft_inv_n(p, spec, phys, 1, p->bufA, p->bufB, false);
  }
  static void fft_fwd(Plan* p, const void* phys, void* spec) {
    fft_fwd_n(p, phys, spec, 1, p->bufA, p->bufB);
  }
  static Ops ops() {
    Ops o{};
    o.p1 = p1;
    o.stage = stage;
    o.tendency = tendency;
    o.fft_fwd = fft_fwd;
    o.fft_inv = fft_inv;
    o.fft_fwd_n = fft_fwd_n;
    o.fft_inv_n = fft_inv_n;
    o.alpha = launch_alpha<T>;
    o.dtstep = launch_dtstep<T>;
    o.diag = launch_diag<T>;
    o.transfer = launch_transfer<T>;
    o.spectra1d = launch_spectra1d<T>;
    o.structure = launch_structure<T>;
    // A: z-pass output Wm[FZ], later the x-pass output Wn[FFWD];
    // B: y-inverse output Wn[FINV], later the y-forward output Wm[FFWD].
    // Diagnostics also keep one undealiased field plus one physical field
    // (N^3 reals) in A.
    const size_t wm = (size_t)N * G::XT * G::M * kTile, wn = (size_t)N * G::XT * N * kTile;
    const size_t wfull = (size_t)N * GF::XT * N * kTile;
    const size_t phys = ((size_t)N * N * N * sizeof(T) + sizeof(cx<T>) - 1) / sizeof(cx<T>);
    o.elems_a = std::max({FZ * wm, FFWD * wn, wfull + phys});
    o.elems_b = std::max({FINV * wn, FFWD * wm, wfull});
    o.elems_acc = (size_t)NC * G::XT * G::M * G::M * kTile;
    o.elems_full = wfull;
    return o;
  }
};

}  // namespace ops3d_detail

// the ops table of the 3D solver at size n (n a supported power of two)
template <typename T, bool STRAT>
Ops ops3_of(int n) {
  using ops3d_detail::L3;
  switch (n) {
    case 16: return L3<T, 16, STRAT>::ops();
    case 32: return L3<T, 32, STRAT>::ops();
    case 64: return L3<T, 64, STRAT>::ops();
    case 128: return L3<T, 128, STRAT>::ops();
    case 256: return L3<T, 256, STRAT>::ops();
    case 512: return L3<T, 512, STRAT>::ops();
    case 1024: return L3<T, 1024, STRAT>::ops();
    default: return Ops{};
  }
}

}  // namespace fs
