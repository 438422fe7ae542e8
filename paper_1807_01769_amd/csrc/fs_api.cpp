// fs_api.cpp -- the C ABI of libfs: argument validation, plan construction
// (FP64 tables rounded once to the working precision, one workspace
// allocation), step graphs and kernel timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fs.h"
#include "fs_internal.h"
#include "ns_common.h"

namespace fs {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

namespace {
std::mutex g_alloc_mu;
std::string g_alloc_hook;  // last value of FS_TEST_FAIL_ALLOC seen
long g_alloc_count = 0;    // allocations since it took that value

bool injected_failure() {
  const char* v = std::getenv("FS_TEST_FAIL_ALLOC");
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  if (!v || !*v) {
    g_alloc_hook.clear();
    return false;
  }
  if (g_alloc_hook != v) {
    g_alloc_hook = v;
    g_alloc_count = 0;
  }
  return ++g_alloc_count == std::atol(v);
}
}  // namespace

hipError_t dev_malloc(void** ptr, size_t bytes) {
  if (injected_failure()) {
    *ptr = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(ptr, bytes);
}

hipError_t pinned_malloc(void** ptr, size_t bytes) {
  if (injected_failure()) {
    *ptr = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipHostMalloc(ptr, bytes, hipHostMallocDefault);
}

bool Plan::ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  set_error("%s: %s", what, hipGetErrorString(e));
  failed = true;
  return false;
}

bool launched(Plan* p, const char* what) { return p->ok(hipGetLastError(), what); }

void Plan::begin(int kid) {
  (void)kid;
  if (!(flags & FS_PROFILE)) return;
  if (pool_used + 2 > pool.size()) {
    for (int i = 0; i < 64; i++) {
      hipEvent_t e;
      if (!ok(hipEventCreate(&e), "hipEventCreate")) return;
      pool.push_back(e);
    }
  }
  Mark m{kid, pool[pool_used], pool[pool_used + 1]};
  pool_used += 2;
  ok(hipEventRecord(m.a, launch), "hipEventRecord");
  marks.push_back(m);
}

void Plan::end(int kid) {
  (void)kid;
  if (!(flags & FS_PROFILE) || marks.empty()) return;
  ok(hipEventRecord(marks.back().b, launch), "hipEventRecord");
}

}  // namespace fs

using fs::Plan;

namespace {

const char* kKernelNames[fs::KID_COUNT] = {"p1",    "y_inverse", "x_c2r_product_r2c",
                                           "y_forward", "z_stage", "forcing_alpha",
                                           "fill",  "fft_only",  "diagnostics"};

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
bool isfin(double x) { return std::isfinite(x); }
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

fs_status fail(fs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fs::g_err = buf;
  return s;
}

fs_status usable(const fs_plan* plan) {
  if (!plan) return fail(FS_E_INVALID, "plan is NULL");
  if (plan->p.failed) return fail(FS_E_DEVICE, "plan failed earlier: %s", fs::g_err.c_str());
  return FS_OK;
}

fs_status device_status(Plan* p) { return p->failed ? FS_E_DEVICE : FS_OK; }

void release(Plan* p) {
  if (p->gmid) hipGraphExecDestroy(p->gmid);
  if (p->glast) hipGraphExecDestroy(p->glast);
  p->gmid = p->glast = nullptr;
  for (auto e : p->pool) hipEventDestroy(e);
  p->pool.clear();
  if (p->cap) hipStreamDestroy(p->cap);
  p->cap = nullptr;
  if (p->base && p->owns_base) hipFree(p->base);
  p->base = nullptr;
  if (p->nonfin_host) hipHostFree(p->nonfin_host);
  p->nonfin_host = nullptr;
  if (p->nonfin_ev) hipEventDestroy(p->nonfin_ev);
  p->nonfin_ev = nullptr;
}

// FS_CHECK_FINITE: the flag copied after the last step call; reports (and
// clears) a non-finite value written by it.
fs_status check_finite(Plan* p) {
  if (!p->nonfin_pending) return FS_OK;
  p->nonfin_pending = false;
  if (!p->ok(hipEventSynchronize(p->nonfin_ev), "flag event")) return FS_E_DEVICE;
  if (*p->nonfin_host == 0) return FS_OK;
  *p->nonfin_host = 0;
  if (!p->ok(hipMemsetAsync(p->nonfin, 0, sizeof(unsigned), p->stream), "clear flag"))
    return FS_E_DEVICE;
  return fail(FS_E_NONFINITE, "the last fs_step_rk4 call wrote non-finite values");
}

// One RK4 step (forcing coefficient, four stages) on p->launch.
void enqueue_step(Plan* p, void* state, int do_p1) {
  if (p->ops.alpha && p->m2max >= 0) p->ops.alpha(p, state);
  if (p->scheme == FS_SCHEME_RK2) {
    p->ops.stage(p, state, fs::kRk2a, 1);
    p->ops.stage(p, state, fs::kRk2b, do_p1);
  } else {
    for (int mode = fs::kStage1; mode <= fs::kStage4; mode++)
      p->ops.stage(p, state, mode, mode == fs::kStage4 ? do_p1 : 1);
  }
}

bool capture(Plan* p, void* state, int do_p1, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  p->launch = p->cap;
  if (!p->ok(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal), "begin capture")) {
    p->launch = p->stream;
    return false;
  }
  enqueue_step(p, state, do_p1);
  hipError_t e = hipStreamEndCapture(p->cap, &g);
  p->launch = p->stream;
  if (!p->ok(e, "end capture") || p->failed) {
    if (g) hipGraphDestroy(g);
    return false;
  }
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return p->ok(e, "hipGraphInstantiate");
}

int K_of(int n) { return (n - 1) / 3; }

}  // namespace

// Validation and the host side of a plan (fields, kernels); no device call.
fs_status configure(Plan* p, int n, double L, double nu, double dt, const fs_plan_opts& o) {
  if (n <= 0) return fail(FS_E_INVALID, "n = %d must be positive", n);
  if (!is_pow2(n) || n < 16 || n > 1024)
    return fail(FS_E_UNSUPPORTED, "n = %d: supported sizes are powers of two 16..1024", n);
  if (!(isfin(L) && L > 0)) return fail(FS_E_INVALID, "L must be finite and > 0");
  if (!(isfin(nu) && nu >= 0)) return fail(FS_E_INVALID, "nu must be finite and >= 0");
  if (!(isfin(dt) && dt > 0)) return fail(FS_E_INVALID, "dt must be finite and > 0");
  if (o.ndim != 2 && o.ndim != 3) return fail(FS_E_INVALID, "ndim = %d must be 2 or 3", o.ndim);
  if (o.precision != FS_F32 && o.precision != FS_F64)
    return fail(FS_E_INVALID, "precision = %d must be FS_F32 or FS_F64", o.precision);
  if (o.flags & ~(FS_NO_GRAPH | FS_PROFILE | FS_NO_AUTOTUNE | FS_BOUSSINESQ | FS_CHECK_FINITE))
    return fail(FS_E_INVALID, "unknown flags");
  if (!(isfin(o.n2) && o.n2 >= 0)) return fail(FS_E_INVALID, "n2 must be finite and >= 0");
  if (!isfin(o.rotation)) return fail(FS_E_INVALID, "rotation must be finite");
  if (o.rotation != 0.0 && o.ndim != 3)
    return fail(FS_E_UNSUPPORTED, "rotation is implemented for ndim = 3");
  if (!(isfin(o.forcing_power) && o.forcing_power >= 0))
    return fail(FS_E_INVALID, "forcing_power must be finite and >= 0");
  if (o.scheme != FS_SCHEME_RK4 && o.scheme != FS_SCHEME_RK2)
    return fail(FS_E_INVALID, "scheme = %d must be FS_SCHEME_RK4 or FS_SCHEME_RK2", o.scheme);
  if (!(isfin(o.cfl) && o.cfl >= 0)) return fail(FS_E_INVALID, "cfl must be finite and >= 0");
  const double kb = 2.0 * M_PI / L;
  const int K = K_of(n);
  int bw = 0, m2min = 0, m2max = -1;
  if (o.forcing_power > 0) {
    if (o.ndim != 3) return fail(FS_E_UNSUPPORTED, "forcing is implemented for ndim = 3 only");
    if (!(isfin(o.forcing_kmin) && isfin(o.forcing_kmax) && o.forcing_kmin >= 0 &&
          o.forcing_kmax >= o.forcing_kmin && o.forcing_kmax > 0))
      return fail(FS_E_INVALID, "forcing band must satisfy 0 <= kmin <= kmax, kmax > 0");
    const double bwd = std::floor(o.forcing_kmax / kb);  // checked before the conversion
    if (!(bwd <= K)) return fail(FS_E_INVALID, "forcing band reaches beyond the dealiased modes");
    bw = (int)bwd;
    // integer |m|^2 range, evaluated as |k| = kb sqrt(m2) in FP64
    m2min = 1 << 30;
    for (int m2 = 1; m2 <= 3 * bw * bw; m2++) {
      const double km = kb * std::sqrt((double)m2);
      if (km >= o.forcing_kmin && km <= o.forcing_kmax) {
        if (m2 < m2min) m2min = m2;
        m2max = m2;
      }
    }
    if (m2max < 0) return fail(FS_E_INVALID, "forcing band contains no mode");
    if (bw < 1) bw = 1;
  }
  if (o.ndim == 3 && o.precision == FS_F64 && n > 512)
    return fail(FS_E_UNSUPPORTED, "3D FP64 plans support n <= 512");
  p->n = n;
  p->ndim = o.ndim;
  p->prec = o.precision;
  p->L = L;
  p->nu = nu;
  p->dt = dt;
  p->fpow = o.forcing_power;
  p->fkmin = o.forcing_kmin;
  p->fkmax = o.forcing_kmax;
  p->bw = bw;
  p->m2min = m2min;
  p->m2max = m2max;
  p->flags = o.flags;
  p->scheme = o.scheme;
  p->cfl = o.cfl;
  p->nfield = (o.ndim == 3 ? 3 : 1) + ((o.flags & FS_BOUSSINESQ) ? 1 : 0);
  p->n2 = o.n2;
  p->rotf = o.rotation;
  p->stream = (hipStream_t)o.stream;
  p->launch = p->stream;
  if (o.ndim == 3)
    p->ops = o.precision == FS_F32 ? fs::make_ops3<float>(n, p->nfield)
                                   : fs::make_ops3<double>(n, p->nfield);
  else
    p->ops = o.precision == FS_F32 ? fs::make_ops2<float>(n, p->nfield)
                                   : fs::make_ops2<double>(n, p->nfield);
  if (!p->ops.stage) return fail(FS_E_UNSUPPORTED, "no kernels for n = %d", n);
  return FS_OK;
}

constexpr int kPieces = 11;

// Byte sizes and offsets of the pieces carved out of the plan's one
// workspace allocation; returns the total.
size_t carve(const Plan* p, size_t off[kPieces], size_t sz[kPieces]) {
  const int n = p->n, bw = p->bw;
  const size_t rs = p->prec == FS_F32 ? 4 : 8, cs = 2 * rs;
  const int band_elems = 3 * (2 * bw + 1) * (2 * bw + 1) * (bw + 1);
  const size_t dpart = (size_t)fs::kDiagMaxBlocks * (fs::kDiagMaxBins + 2) * sizeof(double);
  const size_t v[kPieces] = {cs * n,
                             rs * n,
                             rs * n,
                             cs * p->ops.elems_a,
                             cs * p->ops.elems_b,
                             cs * p->ops.elems_acc,
                             cs * (size_t)(band_elems > 0 ? band_elems : 1),
                             rs * 2,
                             dpart,
                             64,  // step, elapsed time, velocity maximum, non-finite flag
                             cs * (p->ops.elems_sin ? p->ops.elems_sin : 1)};
  size_t total = 0;
  for (int i = 0; i < kPieces; i++) {
    sz[i] = v[i];
    off[i] = total;
    total += align256(v[i]);
  }
  return total;
}

extern "C" {

void fs_plan_opts_default(fs_plan_opts* o) {
  if (!o) return;
  o->ndim = 3;
  o->precision = FS_F32;
  o->stream = nullptr;
  o->forcing_power = 0.0;
  o->forcing_kmin = 2.0;
  o->forcing_kmax = 3.0;
  o->flags = 0;
  o->scheme = FS_SCHEME_RK4;
  o->cfl = 0.0;
  o->n2 = 0.0;
  o->rotation = 0.0;
  o->workspace = nullptr;
  o->workspace_bytes = 0;
}

fs_status fs_plan_workspace_bytes(int n, const fs_plan_opts* opts, size_t* bytes) {
  if (!bytes) return fail(FS_E_INVALID, "bytes is NULL");
  fs_plan_opts o;
  fs_plan_opts_default(&o);
  if (opts) o = *opts;
  Plan p;
  if (fs_status st = configure(&p, n, 2.0 * M_PI, 0.0, 1.0, o)) return st;
  size_t off[kPieces], sz[kPieces];
  *bytes = carve(&p, off, sz);
  return FS_OK;
}

fs_status fs_plan_create(fs_plan** out, int n, double L, double nu, double dt,
                         const fs_plan_opts* opts) {
  if (!out) return fail(FS_E_INVALID, "out is NULL");
  *out = nullptr;
  fs_plan_opts o;
  fs_plan_opts_default(&o);
  if (opts) o = *opts;
  fs_plan* h = new (std::nothrow) fs_plan();
  if (!h) return fail(FS_E_NOMEM, "host allocation failed");
  Plan* p = &h->p;
  if (fs_status st = configure(p, n, L, nu, dt, o)) {
    delete h;
    return st;
  }
  size_t off[kPieces], sz[kPieces];
  const size_t total = carve(p, off, sz);
  if (o.workspace && (o.workspace_bytes < total || ((uintptr_t)o.workspace & 255))) {
    delete h;
    return fail(FS_E_INVALID, "workspace must be 256-byte aligned and hold %zu bytes", total);
  }
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete h;
    return fail(FS_E_DEVICE, "no HIP device");
  }
  const size_t rs = o.precision == FS_F32 ? 4 : 8;
  if (o.workspace) {
    p->base = o.workspace;
    p->owns_base = false;
  } else if (fs::dev_malloc(&p->base, total) != hipSuccess) {
    hipGetLastError();
    delete h;
    return fail(FS_E_NOMEM, "hipMalloc of %zu bytes failed", total);
  }
  p->bytes_total = total;
  char* b = (char*)p->base;
  p->tw = b + off[0];
  p->e1 = b + off[1];
  p->eh1 = b + off[2];
  p->bufA = b + off[3];
  p->bufB = b + off[4];
  p->acc = b + off[5];
  p->vband = b + off[6];
  p->alpha = b + off[7];
  p->dpart = (double*)(b + off[8]);
  p->tdev = (double*)(b + off[9]);
  p->umaxdev = (unsigned long long*)(b + off[9] + 8);
  p->dtdev = b + off[9] + 16;
  p->sin = p->ops.elems_sin ? b + off[10] : nullptr;
  p->nonfin = (unsigned*)(b + off[9] + 24);
  p->dpart_blocks = fs::kDiagMaxBlocks;
  if ((o.flags & FS_CHECK_FINITE) &&
      (!p->ok(fs::pinned_malloc((void**)&p->nonfin_host, sizeof(unsigned)), "pinned flag") ||
       !p->ok(hipEventCreateWithFlags(&p->nonfin_ev, hipEventDisableTiming), "flag event"))) {
    std::string msg = fs::g_err;
    const bool nomem = p->nonfin_host == nullptr;
    hipGetLastError();
    release(p);
    delete h;
    return fail(nomem ? FS_E_NOMEM : FS_E_DEVICE, "%s", msg.c_str());
  }
  if (p->nonfin_host) *p->nonfin_host = 0;

  const float dt32 = (float)dt;
  const double kb = 2.0 * M_PI / L;
  // FP64 tables, rounded once
  std::vector<char> host(sz[0] + sz[1] + sz[2]);
  for (int m = 0; m < n; m++) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    const double c = std::cos(a), s = std::sin(a);
    const int mm = m <= n / 2 ? m : m - n;
    const double k2 = kb * kb * (double)mm * (double)mm;
    const double e = std::exp(-nu * dt * k2), eh = std::exp(-0.5 * nu * dt * k2);
    if (rs == 4) {
      float* t = (float*)host.data();
      t[2 * m] = (float)c;
      t[2 * m + 1] = (float)s;
      ((float*)(host.data() + sz[0]))[m] = (float)e;
      ((float*)(host.data() + sz[0] + sz[1]))[m] = (float)eh;
    } else {
      double* t = (double*)host.data();
      t[2 * m] = c;
      t[2 * m + 1] = s;
      ((double*)(host.data() + sz[0]))[m] = e;
      ((double*)(host.data() + sz[0] + sz[1]))[m] = eh;
    }
  }
  bool ok = p->ok(hipMemcpy(p->tw, host.data(), sz[0], hipMemcpyHostToDevice), "copy tables") &&
            p->ok(hipMemcpy(p->e1, host.data() + sz[0], sz[1], hipMemcpyHostToDevice),
                  "copy tables") &&
            p->ok(hipMemcpy(p->eh1, host.data() + sz[0] + sz[1], sz[2], hipMemcpyHostToDevice),
                  "copy tables") &&
            p->ok(hipMemset(p->vband, 0, sz[6]), "clear band") &&
            p->ok(hipMemset(p->alpha, 0, sz[7]), "clear alpha") &&
            p->ok(hipMemset(b + off[9], 0, sz[9]), "clear step scalars") &&
            (rs == 4 ? p->ok(hipMemcpy(p->dtdev, &dt32, 4, hipMemcpyHostToDevice), "dt")
                     : p->ok(hipMemcpy(p->dtdev, &dt, 8, hipMemcpyHostToDevice), "dt")) &&
            p->ok(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking), "capture stream");
  if (!ok) {
    std::string msg = fs::g_err;
    release(p);
    delete h;
    return fail(FS_E_DEVICE, "%s", msg.c_str());
  }
  *out = h;
  return FS_OK;
}

fs_status fs_plan_destroy(fs_plan* plan) {
  if (!plan) return FS_OK;
  Plan* p = &plan->p;
  if (p->stream) hipStreamSynchronize(p->stream);
  else hipDeviceSynchronize();
  release(p);
  delete plan;
  return FS_OK;
}

fs_status fs_plan_set_stream(fs_plan* plan, void* stream) {
  if (fs_status s = usable(plan)) return s;
  plan->p.stream = (hipStream_t)stream;
  plan->p.launch = plan->p.stream;
  return FS_OK;
}

fs_status fs_state_elems(const fs_plan* plan, size_t* n_complex) {
  if (!plan || !n_complex) return fail(FS_E_INVALID, "NULL argument");
  const size_t n = plan->p.n;
  *n_complex = (size_t)plan->p.nfield * (plan->p.ndim == 3 ? n : 1) * n * (n / 2 + 1);
  return FS_OK;
}

fs_status fs_workspace_bytes(const fs_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(FS_E_INVALID, "NULL argument");
  *bytes = plan->p.bytes_total;
  return FS_OK;
}

fs_status fs_spectrum_bins(const fs_plan* plan, int* nbins) {
  if (!plan || !nbins) return fail(FS_E_INVALID, "NULL argument");
  const int K = K_of(plan->p.n);
  *nbins = (int)std::floor(std::sqrt((double)plan->p.ndim) * K + 0.5) + 1;
  return FS_OK;
}

fs_status fs_fft_forward(fs_plan* plan, const void* phys, void* spec) {
  if (fs_status s = usable(plan)) return s;
  if (!phys || !spec) return fail(FS_E_INVALID, "NULL array");
  plan->p.ops.fft_fwd(&plan->p, phys, spec);
  return device_status(&plan->p);
}

fs_status fs_fft_inverse(fs_plan* plan, const void* spec, void* phys) {
  if (fs_status s = usable(plan)) return s;
  if (!phys || !spec) return fail(FS_E_INVALID, "NULL array");
  plan->p.ops.fft_inv(&plan->p, spec, phys);
  return device_status(&plan->p);
}

fs_status fs_tendency(fs_plan* plan, const void* state, void* tend) {
  if (fs_status s = usable(plan)) return s;
  if (!state || !tend) return fail(FS_E_INVALID, "NULL array");
  if (state == tend) return fail(FS_E_INVALID, "state and tend must not overlap");
  if (fs_status st = check_finite(&plan->p)) return st;
  plan->p.ops.tendency(&plan->p, state, tend, true, true);
  return device_status(&plan->p);
}

fs_status fs_step_rk4(fs_plan* plan, void* state, int nsteps) {
  if (fs_status s = usable(plan)) return s;
  if (!state) return fail(FS_E_INVALID, "NULL state");
  if (nsteps < 0) return fail(FS_E_INVALID, "nsteps = %d must be >= 0", nsteps);
  if (nsteps == 0) return FS_OK;
  Plan* p = &plan->p;
  if (fs_status st = check_finite(p)) return st;
  p->ops.p1(p, state);
  const bool graphs = !(p->flags & (FS_NO_GRAPH | FS_PROFILE));
  if (graphs) {
    if (p->gstate != state || !p->gmid || !p->glast) {
      if (p->gmid) hipGraphExecDestroy(p->gmid);
      if (p->glast) hipGraphExecDestroy(p->glast);
      p->gmid = p->glast = nullptr;
      p->gstate = nullptr;
      if (!capture(p, state, 1, &p->gmid) || !capture(p, state, 0, &p->glast))
        return FS_E_DEVICE;
      p->gstate = state;
    }
    for (int s = 0; s < nsteps; s++)
      if (!p->ok(hipGraphLaunch(s + 1 < nsteps ? p->gmid : p->glast, p->stream), "graph launch"))
        return FS_E_DEVICE;
  } else {
    for (int s = 0; s < nsteps; s++) enqueue_step(p, state, s + 1 < nsteps);
  }
  if (p->cfl <= 0) p->t_fixed += nsteps * p->dt;
  if (p->nonfin_host && !p->failed) {
    p->ok(hipMemcpyAsync(p->nonfin_host, p->nonfin, sizeof(unsigned), hipMemcpyDeviceToHost,
                         p->stream),
          "copy flag");
    p->ok(hipEventRecord(p->nonfin_ev, p->stream), "flag event");
    p->nonfin_pending = !p->failed;
  }
  return device_status(p);
}

fs_status fs_plan_time(fs_plan* plan, double* time, double* last_dt) {
  if (fs_status s = usable(plan)) return s;
  if (fs_status st = check_finite(&plan->p)) return st;
  fs::launch_time(&plan->p, time, last_dt);
  return device_status(&plan->p);
}

fs_status fs_energy_spectrum(fs_plan* plan, const void* state, double* spectrum, int nbins,
                             double* energy, double* enstrophy) {
  if (fs_status s = usable(plan)) return s;
  if (!state || !spectrum) return fail(FS_E_INVALID, "NULL array");
  if (nbins < 1 || nbins > fs::kDiagMaxBins)
    return fail(FS_E_INVALID, "nbins = %d must be in 1..%d", nbins, fs::kDiagMaxBins);
  if (fs_status st = check_finite(&plan->p)) return st;
  plan->p.ops.diag(&plan->p, state, spectrum, nbins, energy, enstrophy);
  return device_status(&plan->p);
}

fs_status fs_energy_spectra_1d(fs_plan* plan, const void* state, double* out) {
  if (fs_status s = usable(plan)) return s;
  if (!state || !out) return fail(FS_E_INVALID, "NULL array");
  plan->p.ops.spectra1d(&plan->p, state, out);
  return device_status(&plan->p);
}

fs_status fs_structure_functions(fs_plan* plan, const void* state, int nr, const int* r, int pmax,
                                 double* out) {
  if (fs_status s = usable(plan)) return s;
  if (!state || !r || !out) return fail(FS_E_INVALID, "NULL array");
  if (nr < 1 || nr > fs::kSfMaxR)
    return fail(FS_E_INVALID, "nr = %d must be in 1..%d", nr, fs::kSfMaxR);
  if (pmax < 1 || pmax > fs::kSfMaxP)
    return fail(FS_E_INVALID, "pmax = %d must be in 1..%d", pmax, fs::kSfMaxP);
  for (int j = 0; j < nr; j++)
    if (r[j] < 1 || r[j] >= plan->p.n)
      return fail(FS_E_INVALID, "r[%d] = %d must be in 1..n-1", j, r[j]);
  plan->p.ops.structure(&plan->p, state, nr, r, pmax, out);
  return device_status(&plan->p);
}

fs_status fs_energy_transfer(fs_plan* plan, const void* state, const void* tend, double* transfer,
                             double* flux, int nbins, double* energy_rate,
                             double* enstrophy_rate) {
  if (fs_status s = usable(plan)) return s;
  if (!state || !tend || !transfer) return fail(FS_E_INVALID, "NULL array");
  if (nbins < 1 || nbins > fs::kDiagMaxBins)
    return fail(FS_E_INVALID, "nbins = %d must be in 1..%d", nbins, fs::kDiagMaxBins);
  plan->p.ops.transfer(&plan->p, state, tend, transfer, flux, nbins, energy_rate,
                       enstrophy_rate);
  return device_status(&plan->p);
}

fs_status fs_profile_read(fs_plan* plan, double* ms, long* counts, const char** names, int nk) {
  if (fs_status s = usable(plan)) return s;
  Plan* p = &plan->p;
  for (auto& m : p->marks) {
    float t = 0.f;
    if (!p->ok(hipEventSynchronize(m.b), "hipEventSynchronize")) return FS_E_DEVICE;
    if (!p->ok(hipEventElapsedTime(&t, m.a, m.b), "hipEventElapsedTime")) return FS_E_DEVICE;
    p->kms[m.kid] += t;
    p->kcount[m.kid] += 1;
  }
  p->marks.clear();
  p->pool_used = 0;
  for (int k = 0; k < nk && k < fs::KID_COUNT; k++) {
    if (ms) ms[k] = p->kms[k];
    if (counts) counts[k] = p->kcount[k];
    if (names) names[k] = kKernelNames[k];
  }
  for (int k = 0; k < fs::KID_COUNT; k++) {
    p->kms[k] = 0;
    p->kcount[k] = 0;
  }
  return FS_OK;
}

const char* fs_status_str(fs_status s) {
  switch (s) {
    case FS_OK: return "FS_OK";
    case FS_E_INVALID: return "FS_E_INVALID";
    case FS_E_UNSUPPORTED: return "FS_E_UNSUPPORTED";
    case FS_E_NOMEM: return "FS_E_NOMEM";
    case FS_E_DEVICE: return "FS_E_DEVICE";
    case FS_E_NONFINITE: return "FS_E_NONFINITE";
  }
  return "FS_E_UNKNOWN";
}

const char* fs_last_error(void) { return fs::g_err.c_str(); }

}  // extern "C"
