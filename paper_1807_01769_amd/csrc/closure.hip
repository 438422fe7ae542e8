// closure.hip -- the learned subgrid-stress closure on the device:
//  * training samples from a fine (DNS) spectral state: the sharp cube cutoff
//    onto a coarse grid whose dealiased set is exactly the kept cube, the
//    velocity gradients A_ij = d ubar_i / d x_j of the filtered field and the
//    deviatoric subgrid stress tau_ij = cutoff(u_i u_j) - ubar_i ubar_j at
//    the coarse points, their mean squares, and the standardised BF16
//    features / FP32 targets the network trains on;
//  * the LES step: the Lawson integrating-factor RK4 scheme of the solver
//    whose nonlinear term is the coarse tendency plus P[-i k_j tau_ij^], tau
//    given at every stage by the network applied to the standardised
//    gradients of the stage state.
// Stress components are ordered xx, yy, zz, xy, xz, yz; gradients as
// A[3i+j].  Single precision (the network is BF16/FP32).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "bf16.h"
#include "fs.h"
#include "fs_internal.h"
#include "ns_common.h"

namespace fs {
namespace {

using cf = cx<float>;
constexpr int kThr = 256;
__constant__ int kTauI[6] = {0, 1, 2, 0, 0, 1};
__constant__ int kTauJ[6] = {0, 1, 2, 1, 2, 2};

__device__ __forceinline__ int fmode(int i, int n) { return i <= n / 2 ? i : i - n; }
__device__ __forceinline__ int iabs(int a) { return a < 0 ? -a : a; }

struct Six {
  float v[6];
};

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThr - 1) / kThr); }

// coarse(m) = fine(m) on |m_a| <= Kc = floor((nc-1)/3), zero elsewhere; every
// element of `coarse` is written.  blockIdx.y = field.
__global__ void __launch_bounds__(kThr)
    k_cutoff(const cf* __restrict__ fine, int nf, cf* __restrict__ coarse, int nc, int box) {
  const int64_t hf = nf / 2 + 1, hc = nc / 2 + 1;
  const int64_t nsc = (int64_t)nc * nc * hc, nsf = (int64_t)nf * nf * hf;
  const int64_t q = (int64_t)blockIdx.x * kThr + threadIdx.x;
  if (q >= nsc) return;
  const int ix = (int)(q % hc), iy = (int)((q / hc) % nc), iz = (int)(q / (hc * nc));
  const int my = fmode(iy, nc), mz = fmode(iz, nc), Kc = (nc - 1) / 3;
  cf v = {0.f, 0.f};
  if (ix <= Kc && iabs(my) <= Kc && iabs(mz) <= Kc) {
    const int64_t fz = (mz + nf) % nf, fy = (my + nf) % nf;
    v = fine[blockIdx.y * nsf + (fz * nf + fy) * hf + ix];
    if (box) {
      // box filter of width L / (2 Kc): sin(x) / x per axis, x = pi m / (2 Kc)
      const float c = 3.14159265358979f / (2.0f * (float)Kc);
      const int ms[3] = {ix, my, mz};
      float g = 1.0f;
#pragma unroll
      for (int a = 0; a < 3; a++)
        if (ms[a] != 0) g *= sinf(c * (float)ms[a]) / (c * (float)ms[a]);
      v = {v.re * g, v.im * g};
    }
  }
  coarse[blockIdx.y * nsc + q] = v;
}

// out = in on the kept set of an n grid, zero elsewhere (one field)
__global__ void __launch_bounds__(kThr)
    k_mask(const cf* __restrict__ in, cf* __restrict__ out, int n) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  const int64_t q = (int64_t)blockIdx.x * kThr + threadIdx.x;
  if (q >= ns) return;
  const int ix = (int)(q % h), iy = (int)((q / h) % n), iz = (int)(q / (h * n));
  const int K = (n - 1) / 3;
  const bool keep = ix <= K && iabs(fmode(iy, n)) <= K && iabs(fmode(iz, n)) <= K;
  out[q] = keep ? in[q] : cf{0.f, 0.f};
}

// out = a * b, four values per thread (n4 = count / 4)
__global__ void __launch_bounds__(kThr)
    k_mul(const float4* __restrict__ a, const float4* __restrict__ b, float4* __restrict__ out,
          int64_t n4) {
  const int64_t q = (int64_t)blockIdx.x * kThr + threadIdx.x;
  if (q >= n4) return;
  const float4 x = a[q], y = b[q];
  out[q] = make_float4(x.x * y.x, x.y * y.y, x.z * y.z, x.w * y.w);
}

// tau_s -= ubar_i ubar_j, then the trace is removed from the diagonal
__global__ void __launch_bounds__(kThr)
    k_tau_finish(float* __restrict__ tau, const float* __restrict__ ub, int64_t np) {
  const int64_t q = (int64_t)blockIdx.x * kThr + threadIdx.x;
  if (q >= np) return;
  const float u0 = ub[q], u1 = ub[np + q], u2 = ub[2 * np + q];
  const float a = tau[q] - u0 * u0, b = tau[np + q] - u1 * u1, c = tau[2 * np + q] - u2 * u2;
  const float tr = (a + b + c) * (1.0f / 3.0f);
  tau[q] = a - tr;
  tau[np + q] = b - tr;
  tau[2 * np + q] = c - tr;
  tau[3 * np + q] -= u0 * u1;
  tau[4 * np + q] -= u0 * u2;
  tau[5 * np + q] -= u1 * u2;
}

// mean square of every field (FP64, fixed summation order): block f reduces
// field f of `in` ([nfield][np])
__global__ void __launch_bounds__(1024) k_msq(const float* __restrict__ in, int64_t np, double* out) {
  __shared__ double part[1024];
  const float* f = in + blockIdx.x * np;
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < np; q += 1024) {
    const double v = f[q];
    s += v * v;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = part[0] / (double)np;
}

// x[p] = BF16(A[k][p] * inv_a) in slots 0..8, zero in 9..15; with tau,
// t[p][s] = tau[s][p] * inv_tau[s]
__global__ void __launch_bounds__(kThr)
    k_features(const float* __restrict__ A, int64_t np, float inv_a, uint4* __restrict__ x,
               const float* __restrict__ tau, Six inv_tau, float* __restrict__ t) {
  const int64_t q = (int64_t)blockIdx.x * kThr + threadIdx.x;
  if (q >= np) return;
  unsigned short h[16];
#pragma unroll
  for (int k = 0; k < 16; k++) h[k] = k < 9 ? (unsigned short)to_bf16(A[k * np + q] * inv_a) : 0;
  uint4 lo, hi;
  lo.x = h[0] | (unsigned)h[1] << 16;
  lo.y = h[2] | (unsigned)h[3] << 16;
  lo.z = h[4] | (unsigned)h[5] << 16;
  lo.w = h[6] | (unsigned)h[7] << 16;
  hi.x = h[8] | (unsigned)h[9] << 16;
  hi.y = h[10] | (unsigned)h[11] << 16;
  hi.z = h[12] | (unsigned)h[13] << 16;
  hi.w = h[14] | (unsigned)h[15] << 16;
  x[2 * q] = lo;
  x[2 * q + 1] = hi;
  if (tau) {
#pragma unroll
    for (int s = 0; s < 6; s++) t[q * 6 + s] = tau[s * np + q] * inv_tau.v[s];
  }
}

// The subgrid term P[-i k_j tau_ij^] of one mode (k != 0; P v = v - k (k.v)/|k|^2)
// from the six stress spectra th at element q, added to t[3].
__device__ __forceinline__ void sgs_term(const cf* __restrict__ th, int64_t ns, int64_t q,
                                         const float (&k)[3], cf (&t)[3]) {
  float sr[3] = {0.f, 0.f, 0.f}, si[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 6; c++) {
    const int i = kTauI[c], j = kTauJ[c];
    const cf t = th[c * ns + q];
    // -i k_j t = (k_j t.im, -k_j t.re)
    sr[i] += k[j] * t.im;
    si[i] -= k[j] * t.re;
    if (i != j) {
      sr[j] += k[i] * t.im;
      si[j] -= k[i] * t.re;
    }
  }
  const float inv = 1.0f / (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const float pr = (k[0] * sr[0] + k[1] * sr[1] + k[2] * sr[2]) * inv;
  const float pi = (k[0] * si[0] + k[1] * si[1] + k[2] * si[2]) * inv;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    t[c].re += sr[c] - k[c] * pr;
    t[c].im += si[c] - k[c] * pi;
  }
}

// tend += P[-i k_j tau_ij^] on the kept set, k != 0
__global__ void __launch_bounds__(kThr)
    k_sgs(cf* __restrict__ tend, const cf* __restrict__ th, int n, float kb) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  const int64_t q = (int64_t)blockIdx.x * kThr + threadIdx.x;
  if (q >= ns) return;
  const int ix = (int)(q % h), my = fmode((int)((q / h) % n), n), mz = fmode((int)(q / (h * n)), n);
  const int K = (n - 1) / 3;
  if (!(ix <= K && iabs(my) <= K && iabs(mz) <= K) || (ix == 0 && my == 0 && mz == 0)) return;
  const float k[3] = {kb * (float)ix, kb * (float)my, kb * (float)mz};
  cf t[3] = {tend[q], tend[ns + q], tend[2 * ns + q]};
  sgs_term(th, ns, q, k, t);
#pragma unroll
  for (int c = 0; c < 3; c++) tend[c * ns + q] = t[c];
}

// One Lawson stage combination on the kept set only (threads over the
// compact M x M x H cube, all three components of a mode per thread);
// E = exp(-nu |k|^2 dt) as the product of the per-axis factors.  With th
// (the six stress spectra), the subgrid term P[-i k_j tau_ij^] is added to
// the stage tendency nl first.
template <int MODE>
__global__ void __launch_bounds__(kThr)
    k_lawson(cf* __restrict__ u, cf* __restrict__ acc, cf* __restrict__ v,
             const cf* __restrict__ nl, const cf* __restrict__ th, const float* __restrict__ e1,
             const float* __restrict__ eh1, int n, float kb, float dt) {
  const int K = (n - 1) / 3, M = 2 * K + 1, H = K + 1;
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  const int64_t t = (int64_t)blockIdx.x * kThr + threadIdx.x;
  if (t >= (int64_t)M * M * H) return;
  const int ix = (int)(t % H), jy = (int)((t / H) % M), jz = (int)(t / ((int64_t)H * M));
  const int iy = jy <= K ? jy : jy + (n - M), iz = jz <= K ? jz : jz + (n - M);
  const int64_t q = ((int64_t)iz * n + iy) * h + ix;
  const float E = e1[ix] * e1[iy] * e1[iz], Eh = eh1[ix] * eh1[iy] * eh1[iz];
  cf k3[3] = {nl[q], nl[ns + q], nl[2 * ns + q]};
  const int my = jy <= K ? jy : jy - M, mz = jz <= K ? jz : jz - M;
  if (th && (ix != 0 || my != 0 || mz != 0)) {
    const float k[3] = {kb * (float)ix, kb * (float)my, kb * (float)mz};
    sgs_term(th, ns, q, k, k3);
  }
#pragma unroll
  for (int c = 0; c < 3; c++) {
    const int64_t qc = c * ns + q;
    cf a = acc[qc];
    const cf next = rk4_combine<MODE, float>(u[qc], a, k3[c], E, Eh, dt);
    if constexpr (MODE == kStage4) {
      u[qc] = next;
    } else {
      acc[qc] = a;
      v[qc] = next;
    }
  }
}

bool plan_ok(Plan* p, const char* what) { return launched(p, what); }

}  // namespace
}  // namespace fs

using fs::Plan;
using fs::cf;

namespace {

fs_status fail(fs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fs::set_error("%s", buf);
  return s;
}

// 3D single-precision plan of the plain velocity state (no buoyancy field)
bool is_3d_f32(const fs_plan* p) {
  return p->p.ndim == 3 && p->p.prec == FS_F32 && p->p.nfield == 3;
}

int64_t spec_elems(int n) { return (int64_t)n * n * (n / 2 + 1); }
int64_t phys_elems(int n) { return (int64_t)n * n * n; }

// Carves 256-byte aligned pieces out of one allocation.
struct Carver {
  size_t total = 0;
  size_t take(size_t bytes) {
    const size_t off = total;
    total += (bytes + 255) & ~(size_t)255;
    return off;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// Training samples
// ---------------------------------------------------------------------------
struct fs_closure {
  fs_plan* fine = nullptr;
  fs_plan* coarse = nullptr;
  void* base = nullptr;
  cf* fspec = nullptr;      // one fine spectral field
  float* uf = nullptr;      // fine physical velocity [3][nf^3]
  float* prod = nullptr;    // one fine physical product
  cf* cspec = nullptr;      // one coarse spectral field
  float* ub = nullptr;      // coarse physical filtered velocity [3][nc^3]
  void *wa = nullptr, *wb = nullptr;  // coarse transform workspaces for 9 fields
  int box = 0;              // FS_FILTER_BOX: box filter before the cutoff
};

extern "C" {

fs_status fs_closure_create(fs_closure** out, fs_plan* fine, fs_plan* coarse) {
  if (!out || !fine || !coarse) return fail(FS_E_INVALID, "NULL argument");
  *out = nullptr;
  if (!is_3d_f32(fine) || !is_3d_f32(coarse))
    return fail(FS_E_UNSUPPORTED, "closure samples need two 3D single-precision velocity plans");
  const int nf = fine->p.n, nc = coarse->p.n;
  if (nc >= nf) return fail(FS_E_INVALID, "coarse n = %d must be below fine n = %d", nc, nf);
  if (std::fabs(fine->p.L - coarse->p.L) > 1e-12 * fine->p.L)
    return fail(FS_E_INVALID, "fine and coarse plans must share the box size L");
  if (fine->p.device != coarse->p.device)
    return fail(FS_E_INVALID, "fine and coarse plans must be on one device");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != fine->p.device)
    return fail(FS_E_INVALID, "the plans' device must be current");
  Carver cv;
  const size_t o_fspec = cv.take(sizeof(cf) * spec_elems(nf));
  const size_t o_uf = cv.take(sizeof(float) * 3 * phys_elems(nf));
  const size_t o_prod = cv.take(sizeof(float) * phys_elems(nf));
  const size_t o_cspec = cv.take(sizeof(cf) * spec_elems(nc));
  const size_t o_ub = cv.take(sizeof(float) * 3 * phys_elems(nc));
  const size_t wfull = sizeof(cf) * 9 * coarse->p.ops.elems_full;
  const size_t o_wa = cv.take(wfull), o_wb = cv.take(wfull);
  fs_closure* c = new fs_closure;
  if (fs::dev_malloc(&c->base, cv.total) != hipSuccess) {
    hipGetLastError();
    delete c;
    return fail(FS_E_NOMEM, "hipMalloc of %zu bytes failed", cv.total);
  }
  char* b = (char*)c->base;
  c->fine = fine;
  c->coarse = coarse;
  c->fspec = (cf*)(b + o_fspec);
  c->uf = (float*)(b + o_uf);
  c->prod = (float*)(b + o_prod);
  c->cspec = (cf*)(b + o_cspec);
  c->ub = (float*)(b + o_ub);
  c->wa = b + o_wa;
  c->wb = b + o_wb;
  *out = c;
  return FS_OK;
}

fs_status fs_closure_set_filter(fs_closure* c, int filter) {
  if (!c) return fail(FS_E_INVALID, "NULL closure");
  if (filter != FS_FILTER_SHARP && filter != FS_FILTER_BOX)
    return fail(FS_E_INVALID, "filter = %d must be FS_FILTER_SHARP or FS_FILTER_BOX", filter);
  c->box = filter == FS_FILTER_BOX;
  return FS_OK;
}

fs_status fs_closure_destroy(fs_closure* c) {
  if (!c) return FS_OK;
  if (c->base) hipFree(c->base);
  delete c;
  return FS_OK;
}

static fs_status closure_usable(fs_closure* c) {
  if (!c) return fail(FS_E_INVALID, "closure is NULL");
  if (c->fine->p.failed || c->coarse->p.failed)
    return fail(FS_E_DEVICE, "a plan of the closure failed earlier");
  if (c->fine->p.stream != c->coarse->p.stream)
    return fail(FS_E_INVALID, "fine and coarse plans must use one stream");
  return FS_OK;
}

fs_status fs_closure_samples(fs_closure* c, const void* fine_state, void* coarse_state, float* A,
                             float* tau) {
  if (fs_status s = closure_usable(c)) return s;
  if (!fine_state || !coarse_state || !A || !tau) return fail(FS_E_INVALID, "NULL array");
  Plan* pf = &c->fine->p;
  Plan* pc = &c->coarse->p;
  const int nf = pf->n, nc = pc->n;
  const int64_t nsf = spec_elems(nf), npf = phys_elems(nf);
  const int64_t nsc = spec_elems(nc), npc = phys_elems(nc);
  const cf* us = (const cf*)fine_state;
  cf* uc = (cf*)coarse_state;
  hipStream_t s = pf->stream;
  // filtered state, its physical velocity and gradients
  hipLaunchKernelGGL(fs::k_cutoff, dim3(fs::blocks_for(nsc), 3), dim3(fs::kThr), 0, s, us, nf, uc,
                     nc, c->box);
  if (!fs::plan_ok(pc, "k_cutoff")) return FS_E_DEVICE;
  pc->ops.fft_inv_n(pc, uc, c->ub, 3, c->wa, c->wb, false);
  pc->ops.fft_inv_n(pc, uc, A, 9, c->wa, c->wb, true);  // the nine gradients
  // fine physical velocity (kept modes only)
  for (int i = 0; i < 3; i++) {
    hipLaunchKernelGGL(fs::k_mask, dim3(fs::blocks_for(nsf)), dim3(fs::kThr), 0, s, us + i * nsf,
                       c->fspec, nf);
    if (!fs::plan_ok(pf, "k_mask")) return FS_E_DEVICE;
    pf->ops.fft_inv(pf, c->fspec, c->uf + i * npf);
  }
  // cutoff(u_i u_j) at the coarse points
  static const int ti[6] = {0, 1, 2, 0, 0, 1}, tj[6] = {0, 1, 2, 1, 2, 2};
  for (int st = 0; st < 6; st++) {
    hipLaunchKernelGGL(fs::k_mul, dim3(fs::blocks_for(npf / 4)), dim3(fs::kThr), 0, s,
                       (const float4*)(c->uf + ti[st] * npf), (const float4*)(c->uf + tj[st] * npf),
                       (float4*)c->prod, npf / 4);
    if (!fs::plan_ok(pf, "k_mul")) return FS_E_DEVICE;
    pf->ops.fft_fwd(pf, c->prod, c->fspec);
    hipLaunchKernelGGL(fs::k_cutoff, dim3(fs::blocks_for(nsc), 1), dim3(fs::kThr), 0, s,
                       (const cf*)c->fspec, nf, c->cspec, nc, c->box);
    if (!fs::plan_ok(pc, "k_cutoff")) return FS_E_DEVICE;
    pc->ops.fft_inv(pc, c->cspec, tau + st * npc);
  }
  hipLaunchKernelGGL(fs::k_tau_finish, dim3(fs::blocks_for(npc)), dim3(fs::kThr), 0, s, tau,
                     (const float*)c->ub, npc);
  if (!fs::plan_ok(pc, "k_tau_finish")) return FS_E_DEVICE;
  return (pf->failed || pc->failed) ? FS_E_DEVICE : FS_OK;
}

fs_status fs_closure_moments(fs_closure* c, const float* A, const float* tau, double* msq) {
  if (fs_status s = closure_usable(c)) return s;
  if (!A || !tau || !msq) return fail(FS_E_INVALID, "NULL array");
  Plan* pc = &c->coarse->p;
  const int64_t np = phys_elems(pc->n);
  hipLaunchKernelGGL(fs::k_msq, dim3(9), dim3(1024), 0, pc->stream, A, np, msq);
  if (!fs::plan_ok(pc, "k_msq")) return FS_E_DEVICE;
  hipLaunchKernelGGL(fs::k_msq, dim3(6), dim3(1024), 0, pc->stream, tau, np, msq + 9);
  return fs::plan_ok(pc, "k_msq") ? FS_OK : FS_E_DEVICE;
}

fs_status fs_closure_features(fs_closure* c, const float* A, const float* tau, float a_scale,
                              const float* tau_scale, void* x_bf16, float* t) {
  if (fs_status s = closure_usable(c)) return s;
  if (!A || !x_bf16) return fail(FS_E_INVALID, "NULL array");
  if ((tau == nullptr) != (t == nullptr)) return fail(FS_E_INVALID, "tau and t go together");
  if (tau && !tau_scale) return fail(FS_E_INVALID, "tau_scale is NULL");
  if (!(a_scale > 0.f) || !std::isfinite(a_scale)) return fail(FS_E_INVALID, "a_scale must be > 0");
  fs::Six inv{};
  for (int s = 0; s < 6 && tau; s++) {
    if (!(tau_scale[s] > 0.f) || !std::isfinite(tau_scale[s]))
      return fail(FS_E_INVALID, "tau_scale[%d] must be > 0", s);
    inv.v[s] = 1.0f / tau_scale[s];
  }
  Plan* pc = &c->coarse->p;
  const int64_t np = phys_elems(pc->n);
  hipLaunchKernelGGL(fs::k_features, dim3(fs::blocks_for(np)), dim3(fs::kThr), 0, pc->stream, A,
                     np, 1.0f / a_scale, (uint4*)x_bf16, tau, inv, t);
  return fs::plan_ok(pc, "k_features") ? FS_OK : FS_E_DEVICE;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// LES step
// ---------------------------------------------------------------------------
struct fs_les {
  fs_plan* plan = nullptr;
  fs_mlp* net = nullptr;
  float inv_a = 1.f, clip = 0.f;
  fs::Six scale{};
  void* base = nullptr;
  cf *acc = nullptr, *v = nullptr, *k = nullptr, *th = nullptr;
  float *A = nullptr, *tau = nullptr;
  void *wa = nullptr, *wb = nullptr;
  hipGraphExec_t graph = nullptr;
  void* gstate = nullptr;
};

namespace {

// tend = coarse tendency of `state` + P[-i k_j tau_ij^], tau = net(A(state)).
// Inside a step (step = true) only the kept modes of tend are written and the
// subgrid term is left to the combine, which reads the stress spectra.
void les_tendency(fs_les* les, const void* state, cf* tend, bool fresh_alpha, bool step) {
  Plan* p = &les->plan->p;
  p->ops.tendency(p, state, tend, fresh_alpha, !step);
  if (!les->net) return;
  const int n = p->n;
  const int64_t ns = spec_elems(n), np = phys_elems(n);
  const float kb = (float)(2.0 * M_PI / p->L);
  p->ops.fft_inv_n(p, state, les->A, 9, les->wa, les->wb, true);  // the nine gradients
  fs::StressMap sm;
  for (int c = 0; c < 6; c++) sm.scale[c] = les->scale.v[c];
  sm.clip = les->clip;
  fs::mlp_forward_planar_launch(fs::mlp_of(les->net), les->A, np, les->inv_a, les->tau, sm,
                                p->launch);
  fs::plan_ok(p, "k_mlp_forward_planar");
  p->ops.fft_fwd_n(p, les->tau, les->th, 6, les->wa, les->wb);
  if (step) return;
  hipLaunchKernelGGL(fs::k_sgs, dim3(fs::blocks_for(ns)), dim3(fs::kThr), 0, p->launch, tend,
                     (const cf*)les->th, n, kb);
  fs::plan_ok(p, "k_sgs");
}

template <int MODE>
void les_combine(fs_les* les, void* state) {
  Plan* p = &les->plan->p;
  const int n = p->n, K = (n - 1) / 3, M = 2 * K + 1, H = K + 1;
  hipLaunchKernelGGL((fs::k_lawson<MODE>), dim3(fs::blocks_for((int64_t)M * M * H)),
                     dim3(fs::kThr), 0, p->launch, (cf*)state, les->acc, les->v,
                     (const cf*)les->k, les->net ? (const cf*)les->th : nullptr,
                     (const float*)p->e1, (const float*)p->eh1, n,
                     (float)(2.0 * M_PI / p->L), (float)p->dt);
  fs::plan_ok(p, "k_lawson");
}

void les_step(fs_les* les, void* state) {
  Plan* p = &les->plan->p;
  if (p->ops.alpha && p->m2max >= 0) p->ops.alpha(p, state);
  les_tendency(les, state, les->k, false, true);
  les_combine<fs::kStage1>(les, state);
  les_tendency(les, les->v, les->k, false, true);
  les_combine<fs::kStage2>(les, state);
  les_tendency(les, les->v, les->k, false, true);
  les_combine<fs::kStage3>(les, state);
  les_tendency(les, les->v, les->k, false, true);
  les_combine<fs::kStage4>(les, state);
}

bool les_capture(fs_les* les, void* state) {
  Plan* p = &les->plan->p;
  if (les->graph) hipGraphExecDestroy(les->graph);
  les->graph = nullptr;
  les->gstate = nullptr;
  hipGraph_t g = nullptr;
  p->launch = p->cap;
  if (!p->ok(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal), "begin capture")) {
    p->launch = p->stream;
    return false;
  }
  les_step(les, state);
  hipError_t e = hipStreamEndCapture(p->cap, &g);
  p->launch = p->stream;
  if (!p->ok(e, "end capture")) return false;
  if (p->failed) {
    hipGraphDestroy(g);
    return false;
  }
  e = hipGraphInstantiate(&les->graph, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (!p->ok(e, "instantiate")) return false;
  les->gstate = state;
  return true;
}

}  // namespace

extern "C" {

fs_status fs_les_create(fs_les** out, fs_plan* coarse, fs_mlp* model, float a_scale,
                        const float* tau_scale, float clip) {
  if (!out || !coarse) return fail(FS_E_INVALID, "NULL argument");
  *out = nullptr;
  if (!is_3d_f32(coarse)) return fail(FS_E_UNSUPPORTED, "the LES needs a 3D single-precision velocity plan");
  if (coarse->p.failed) return fail(FS_E_DEVICE, "plan failed earlier");
  if (model && (coarse->p.cfl > 0 || coarse->p.scheme != FS_SCHEME_RK4 || coarse->p.rotf != 0))
    return fail(FS_E_UNSUPPORTED, "the closure LES steps with fixed-dt, non-rotating RK4 plans");
  fs_les* les = new fs_les;
  les->plan = coarse;
  les->net = model;
  if (model) {
    if (!(a_scale > 0.f) || !std::isfinite(a_scale)) {
      delete les;
      return fail(FS_E_INVALID, "a_scale must be > 0");
    }
    if (!tau_scale) {
      delete les;
      return fail(FS_E_INVALID, "tau_scale is NULL");
    }
    for (int s = 0; s < 6; s++) {
      if (!std::isfinite(tau_scale[s])) {
        delete les;
        return fail(FS_E_INVALID, "tau_scale[%d] is not finite", s);
      }
      les->scale.v[s] = tau_scale[s];
    }
    if (!(clip >= 0.f) || !std::isfinite(clip)) {
      delete les;
      return fail(FS_E_INVALID, "clip must be >= 0");
    }
    les->inv_a = 1.0f / a_scale;
    les->clip = clip;
    const int n = coarse->p.n;
    const int64_t ns = spec_elems(n), np = phys_elems(n);
    Carver cv;
    const size_t o_acc = cv.take(sizeof(cf) * 3 * ns), o_v = cv.take(sizeof(cf) * 3 * ns),
                 o_k = cv.take(sizeof(cf) * 3 * ns),
                 o_th = cv.take(sizeof(cf) * 6 * ns), o_A = cv.take(sizeof(float) * 9 * np),
                 o_tau = cv.take(sizeof(float) * 6 * np),
                 o_wa = cv.take(sizeof(cf) * 9 * coarse->p.ops.elems_full),
                 o_wb = cv.take(sizeof(cf) * 9 * coarse->p.ops.elems_full);
    if (fs::dev_malloc(&les->base, cv.total) != hipSuccess) {
      hipGetLastError();
      delete les;
      return fail(FS_E_NOMEM, "hipMalloc of %zu bytes failed", cv.total);
    }
    char* b = (char*)les->base;
    les->acc = (cf*)(b + o_acc);
    les->v = (cf*)(b + o_v);
    les->k = (cf*)(b + o_k);
    les->th = (cf*)(b + o_th);
    les->A = (float*)(b + o_A);
    les->tau = (float*)(b + o_tau);
    les->wa = b + o_wa;
    les->wb = b + o_wb;
  }
  *out = les;
  return FS_OK;
}

fs_status fs_les_destroy(fs_les* les) {
  if (!les) return FS_OK;
  if (les->graph) hipGraphExecDestroy(les->graph);
  if (les->base) hipFree(les->base);
  delete les;
  return FS_OK;
}

fs_status fs_les_tendency(fs_les* les, const void* state, void* tend) {
  if (!les) return fail(FS_E_INVALID, "LES is NULL");
  if (!state || !tend) return fail(FS_E_INVALID, "NULL array");
  if (state == tend) return fail(FS_E_INVALID, "state and tend must not overlap");
  if (!les->net) return fs_tendency(les->plan, state, tend);
  Plan* p = &les->plan->p;
  if (p->failed) return fail(FS_E_DEVICE, "plan failed earlier");
  les_tendency(les, state, (cf*)tend, true, false);
  return p->failed ? FS_E_DEVICE : FS_OK;
}

fs_status fs_les_step_rk4(fs_les* les, void* state, int nsteps) {
  if (!les) return fail(FS_E_INVALID, "LES is NULL");
  if (!les->net) return fs_step_rk4(les->plan, state, nsteps);
  if (!state) return fail(FS_E_INVALID, "NULL state");
  if (nsteps < 0) return fail(FS_E_INVALID, "nsteps = %d must be >= 0", nsteps);
  Plan* p = &les->plan->p;
  if (p->failed) return fail(FS_E_DEVICE, "plan failed earlier");
  if (nsteps == 0) return FS_OK;
  const bool graphs = !(p->flags & (FS_NO_GRAPH | FS_PROFILE));
  if (!graphs) {
    for (int s = 0; s < nsteps && !p->failed; s++) les_step(les, state);
    return p->failed ? FS_E_DEVICE : FS_OK;
  }
  if (les->gstate != state || !les->graph) {
    if (!les_capture(les, state)) return FS_E_DEVICE;
  }
  for (int s = 0; s < nsteps; s++)
    if (!p->ok(hipGraphLaunch(les->graph, p->stream), "graph launch")) return FS_E_DEVICE;
  return FS_OK;
}

}  // extern "C"
