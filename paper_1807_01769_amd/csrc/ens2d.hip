// ens2d.hip -- ensembles of 2D runs of uneven sizes advanced together.
//
// Runs are grouped by grid size into classes; every kernel of the 2D step is
// batched over the runs of one class (see ns2d_kernels.h), so one class-stage
// is two launches whatever the number of runs.  The classes are independent
// chains; fs_ensemble_step_rk4 captures each class's chain, for all requested
// steps, as one hipGraph and launches the classes' graphs once each on their
// own streams, which run concurrently.
//
// Classes of at most 128 points a side are advanced block-resident: one block
// per run holds the run's (kx, y) intermediate in LDS through all steps of a
// call (k2_resident), one launch per call, the class-batched result up to
// rounding; FS_NO_RESIDENT runs them class-batched like the larger classes.
//
// Schedules: the y passes can use 16, 8, 4 or 2 kx lines per block and the
// x pass one, two or four times the default row pairs per block.  At creation an
// autotuner times every candidate of every class on the class's own
// workspace (a measured plan choice in the manner of FFTW's MEASURE
// planning) and keeps the fastest; choices are cached per (size, runs,
// device) for the life of the process.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fs.h"
#include "fs_internal.h"
#include "ns2d_kernels.h"

namespace fs {
namespace {

constexpr int kEnsSizes[] = {64, 128, 256, 512};
constexpr int kYCand[] = {16, 8, 4, 2};  // lines per y-pass block
constexpr int kXCand[] = {1, 2, 4};   // multiples of the default row pairs

struct EnsClass {
  int n = 0, nruns = 0;
  int ylines = 16, xmul = 1;           // chosen schedule
  bool resident = false;               // advanced by k2_resident
  double us_y = 0, us_x = 0;           // tuned per-launch times (microseconds)
  std::vector<int> runs;               // global run index of each local run
  long long* state_off = nullptr;      // device, per local run
  void *w1 = nullptr, *w2 = nullptr, *acc = nullptr;
  void *tw = nullptr, *e1 = nullptr, *eh1 = nullptr;
  size_t w1s = 0, w2s = 0, accs = 0;   // per-run strides (complex elements)
  hipStream_t stream = nullptr;        // capture branch
};

struct Ensemble {
  int nruns = 0;
  double L = 0, nu = 0, dt = 0;
  unsigned flags = 0;
  hipStream_t stream = nullptr;
  std::vector<int> n;
  std::vector<long long> offsets;  // nruns + 1
  std::vector<EnsClass> cls;
  void* base = nullptr;
  size_t bytes = 0;
  std::vector<hipGraphExec_t> graphs;  // one per class
  void* gstate = nullptr;
  int gsteps = -1;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  bool failed = false;
};

bool ok(Ensemble* e, hipError_t err, const char* what) {
  if (err == hipSuccess) return true;
  set_error("%s: %s", what, hipGetErrorString(err));
  e->failed = true;
  return false;
}

StageArgs<float> args_of(const Ensemble* e, const EnsClass& c, void* state) {
  StageArgs<float> a{};
  a.state = (cx<float>*)state;
  a.acc = (cx<float>*)c.acc;
  a.tend = nullptr;
  a.vband = nullptr;
  a.alpha = nullptr;
  a.e1 = (const float*)c.e1;
  a.eh1 = (const float*)c.eh1;
  a.tw = (const cx<float>*)c.tw;
  a.kb = (float)(2.0 * M_PI / e->L);
  a.dt = (float)e->dt;
  a.bw = 0;
  a.m2min = 0;
  a.m2max = -1;
  return a;
}

// launchers of one class for a given size and schedule
template <int N, int LB>
void launch_p1(const Ensemble* e, const EnsClass& c, void* state, hipStream_t s) {
  using G = Geo<N, false>;
  const int bpr = G::XT * kTile / LB;
  Batch bt{c.state_off, 0, c.w1s, 0, bpr};
  hipLaunchKernelGGL((k2_p1<float, N, LB>), dim3(bpr * c.nruns), dim3(LB * N / 8), 0, s,
                     (const cx<float>*)state, (cx<float>*)c.w1, args_of(e, c, state), bt);
}

template <int N, int LB>
void launch_y(const Ensemble* e, const EnsClass& c, void* state, int mode, int do_p1,
              hipStream_t s) {
  using G = Geo<N, false>;
  const int bpr = G::XT * kTile / LB;
  Batch bt{c.state_off, c.w2s, c.w1s, c.accs, bpr};
  const dim3 grid(bpr * c.nruns), block(LB * N / 8);
  const auto a = args_of(e, c, state);
  const cx<float>* in = (const cx<float>*)c.w2;
  cx<float>* out = (cx<float>*)c.w1;
  switch (mode) {
    case 1: hipLaunchKernelGGL((k2_y<float, N, LB, kStage1>), grid, block, 0, s, in, out, a, bt, 1); break;
    case 2: hipLaunchKernelGGL((k2_y<float, N, LB, kStage2>), grid, block, 0, s, in, out, a, bt, 1); break;
    case 3: hipLaunchKernelGGL((k2_y<float, N, LB, kStage3>), grid, block, 0, s, in, out, a, bt, 1); break;
    default: hipLaunchKernelGGL((k2_y<float, N, LB, kStage4>), grid, block, 0, s, in, out, a, bt, do_p1); break;
  }
}

template <int N, int RP>
void launch_x(const Ensemble* e, const EnsClass& c, hipStream_t s) {
  (void)e;
  const int bpr = N / 2 / RP;
  Batch bt{nullptr, c.w1s, c.w2s, 0, bpr};
  hipLaunchKernelGGL((k2_x<float, N, RP>), dim3(bpr * c.nruns), dim3(RP * N / 8), 0, s,
                     (const cx<float>*)c.w1, (cx<float>*)c.w2, (const cx<float>*)c.tw,
                     (float)(1.0 / ((double)N * N)), bt, (unsigned long long*)nullptr);
}

template <int N>
void dispatch_p1(const Ensemble* e, const EnsClass& c, void* st, hipStream_t s) {
  switch (c.ylines) {
    case 16: launch_p1<N, 16>(e, c, st, s); break;
    case 8: launch_p1<N, 8>(e, c, st, s); break;
    case 4: launch_p1<N, 4>(e, c, st, s); break;
    default: launch_p1<N, 2>(e, c, st, s); break;
  }
}
template <int N>
void dispatch_y(const Ensemble* e, const EnsClass& c, void* st, int mode, int do_p1, hipStream_t s) {
  switch (c.ylines) {
    case 16: launch_y<N, 16>(e, c, st, mode, do_p1, s); break;
    case 8: launch_y<N, 8>(e, c, st, mode, do_p1, s); break;
    case 4: launch_y<N, 4>(e, c, st, mode, do_p1, s); break;
    default: launch_y<N, 2>(e, c, st, mode, do_p1, s); break;
  }
}
// row pairs per x-pass block: xmul times the default, as long as the block
// stays within the run's row pairs (and so within 64 KiB of LDS)
template <int N>
constexpr int x_rowpairs(int xmul) {
  constexpr int RP0 = RowPairs<N>::RP;
  return (xmul >= 4 && 4 * RP0 <= N / 2) ? 4 * RP0 : (xmul >= 2 && 2 * RP0 <= N / 2) ? 2 * RP0 : RP0;
}
template <int N>
void dispatch_x(const Ensemble* e, const EnsClass& c, hipStream_t s) {
  constexpr int RP0 = RowPairs<N>::RP;
  switch (x_rowpairs<N>(c.xmul) / RP0) {
    case 4:
      if constexpr (4 * RP0 <= N / 2) launch_x<N, 4 * RP0>(e, c, s);
      break;
    case 2:
      if constexpr (2 * RP0 <= N / 2) launch_x<N, 2 * RP0>(e, c, s);
      break;
    default: launch_x<N, RP0>(e, c, s); break;
  }
}

void class_p1(const Ensemble* e, const EnsClass& c, void* st, hipStream_t s) {
  switch (c.n) {
    case 64: dispatch_p1<64>(e, c, st, s); break;
    case 128: dispatch_p1<128>(e, c, st, s); break;
    case 256: dispatch_p1<256>(e, c, st, s); break;
    default: dispatch_p1<512>(e, c, st, s); break;
  }
}
void class_y(const Ensemble* e, const EnsClass& c, void* st, int mode, int do_p1, hipStream_t s) {
  switch (c.n) {
    case 64: dispatch_y<64>(e, c, st, mode, do_p1, s); break;
    case 128: dispatch_y<128>(e, c, st, mode, do_p1, s); break;
    case 256: dispatch_y<256>(e, c, st, mode, do_p1, s); break;
    default: dispatch_y<512>(e, c, st, mode, do_p1, s); break;
  }
}
void class_x(const Ensemble* e, const EnsClass& c, hipStream_t s) {
  switch (c.n) {
    case 64: dispatch_x<64>(e, c, s); break;
    case 128: dispatch_x<128>(e, c, s); break;
    case 256: dispatch_x<256>(e, c, s); break;
    default: dispatch_x<512>(e, c, s); break;
  }
}

template <int N>
void launch_resident(const Ensemble* e, const EnsClass& c, void* state, int nsteps,
                     hipStream_t s) {
  if constexpr (Resident<N>::kFits) {
    Batch bt{c.state_off, 0, 0, c.accs, 1};
    hipLaunchKernelGGL((k2_resident<N>), dim3(c.nruns), dim3(Resident<N>::THREADS), 0, s,
                       args_of(e, c, state), bt, nsteps);
  }
}
bool resident_size(int n) { return n == 64 || n == 128; }

// all steps of one class on stream s
void class_steps(Ensemble* e, EnsClass& c, void* state, int nsteps, hipStream_t s) {
  if (c.resident) {
    if (c.n == 64) launch_resident<64>(e, c, state, nsteps, s);
    else launch_resident<128>(e, c, state, nsteps, s);
    return;
  }
  class_p1(e, c, state, s);
  for (int k = 0; k < nsteps; k++)
    for (int mode = 1; mode <= 4; mode++) {
      class_x(e, c, s);
      class_y(e, c, state, mode, (mode < 4 || k + 1 < nsteps) ? 1 : 0, s);
    }
}

// --- autotuning -------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, std::pair<int, int>> g_tuned;

double time_us(Ensemble* e, hipStream_t s, const std::function<void()>& fn, int reps) {
  hipEvent_t a, b;
  if (!ok(e, hipEventCreate(&a), "hipEventCreate") || !ok(e, hipEventCreate(&b), "hipEventCreate"))
    return 1e30;
  fn();  // warm-up
  ok(e, hipEventRecord(a, s), "hipEventRecord");
  for (int i = 0; i < reps; i++) fn();
  ok(e, hipEventRecord(b, s), "hipEventRecord");
  ok(e, hipEventSynchronize(b), "hipEventSynchronize");
  float ms = 0.f;
  ok(e, hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms * 1e3 / reps;
}

void tune_class(Ensemble* e, EnsClass& c, void* scratch_state, int device) {
  const auto key = std::make_tuple(c.n, c.nruns, device);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      c.ylines = it->second.first;
      c.xmul = it->second.second;
      return;
    }
  }
  hipStream_t s = c.stream;
  double best = 1e30;
  int bestL = 16;
  for (int L : kYCand) {
    c.ylines = L;
    const double us = time_us(e, s, [&] { class_y(e, c, scratch_state, 2, 1, s); }, 5);
    if (us < best) {
      best = us;
      bestL = L;
    }
  }
  c.ylines = bestL;
  c.us_y = best;
  best = 1e30;
  int bestX = 1;
  for (int X : kXCand) {
    c.xmul = X;
    const double us = time_us(e, s, [&] { class_x(e, c, s); }, 5);
    if (us < best) {
      best = us;
      bestX = X;
    }
  }
  c.xmul = bestX;
  c.us_x = best;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = {c.ylines, c.xmul};
}

bool supported_size(int n) {
  for (int s : kEnsSizes)
    if (s == n) return true;
  return false;
}

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

void release(Ensemble* e) {
  for (auto& g : e->graphs)
    if (g) hipGraphExecDestroy(g);
  e->graphs.clear();
  for (auto& c : e->cls)
    if (c.stream) hipStreamDestroy(c.stream);
  for (auto ev : e->joins) hipEventDestroy(ev);
  if (e->fork) hipEventDestroy(e->fork);
  if (e->base) hipFree(e->base);
  e->base = nullptr;
}

}  // namespace
}  // namespace fs

struct fs_ensemble {
  fs::Ensemble e;
};

using fs::Ensemble;
using fs::EnsClass;

extern "C" {

fs_status fs_ensemble_create(fs_ensemble** out, int nruns, const int* n, double L, double nu,
                             double dt, const fs_plan_opts* opts) {
  if (!out || !n) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  *out = nullptr;
  fs_plan_opts o;
  fs_plan_opts_default(&o);
  o.ndim = 2;
  if (opts) o = *opts;
  if (nruns <= 0) {
    fs::set_error("nruns = %d must be positive", nruns);
    return FS_E_INVALID;
  }
  if (!(std::isfinite(L) && L > 0) || !(std::isfinite(nu) && nu >= 0) ||
      !(std::isfinite(dt) && dt > 0)) {
    fs::set_error("L > 0, nu >= 0, dt > 0 must be finite");
    return FS_E_INVALID;
  }
  if (o.ndim != 2) {
    fs::set_error("ensembles are 2D (opts.ndim = 2)");
    return FS_E_INVALID;
  }
  if (o.precision != FS_F32) {
    fs::set_error("ensembles run in FP32");
    return FS_E_UNSUPPORTED;
  }
  if (o.forcing_power != 0.0) {
    fs::set_error("ensembles have no forcing");
    return FS_E_UNSUPPORTED;
  }
  if (o.flags & ~(FS_NO_GRAPH | FS_NO_AUTOTUNE | FS_NO_RESIDENT)) {
    fs::set_error("unsupported flags for an ensemble");
    return FS_E_INVALID;
  }
  if (o.scheme != FS_SCHEME_RK4 || o.cfl != 0.0 || o.n2 != 0.0 || o.rotation != 0.0 ||
      o.workspace) {
    fs::set_error("ensembles step with fixed-dt RK4 and allocate their own workspace");
    return FS_E_UNSUPPORTED;
  }
  for (int r = 0; r < nruns; r++)
    if (!fs::supported_size(n[r])) {
      fs::set_error("run %d: n = %d, ensemble sizes are 64, 128, 256, 512", r, n[r]);
      return FS_E_UNSUPPORTED;
    }

  fs_ensemble* h = new (std::nothrow) fs_ensemble();
  if (!h) return FS_E_NOMEM;
  Ensemble* e = &h->e;
  e->nruns = nruns;
  e->L = L;
  e->nu = nu;
  e->dt = dt;
  e->flags = o.flags;
  e->stream = (hipStream_t)o.stream;
  e->n.assign(n, n + nruns);
  e->offsets.resize(nruns + 1);
  e->offsets[0] = 0;
  for (int r = 0; r < nruns; r++)
    e->offsets[r + 1] = e->offsets[r] + (long long)n[r] * (n[r] / 2 + 1);
  for (int sz : fs::kEnsSizes) {
    EnsClass c;
    c.n = sz;
    for (int r = 0; r < nruns; r++)
      if (n[r] == sz) c.runs.push_back(r);
    if (!c.runs.empty()) {
      c.nruns = (int)c.runs.size();
      c.resident = fs::resident_size(sz) && !(o.flags & FS_NO_RESIDENT);
      e->cls.push_back(c);
    }
  }
  // memory: per class offsets, w1, w2, acc, tables; plus one scratch state for tuning
  size_t total = 0, scratch = 0;
  std::vector<size_t> offs;
  for (auto& c : e->cls) {
    const int N = c.n, K = (N - 1) / 3, M = 2 * K + 1, XT = (K + 1 + 15) / 16;
    c.w1s = (size_t)3 * XT * N * 16;
    c.w2s = (size_t)2 * XT * N * 16;
    c.accs = (size_t)XT * M * 16;
    const size_t sz[7] = {sizeof(long long) * c.nruns, 8 * c.w1s * c.nruns, 8 * c.w2s * c.nruns,
                          8 * c.accs * c.nruns, 8 * (size_t)N, 4 * (size_t)N, 4 * (size_t)N};
    for (size_t b : sz) {
      offs.push_back(total);
      total += fs::a256(b);
    }
    scratch = std::max(scratch, (size_t)8 * c.nruns * N * (N / 2 + 1));
  }
  const size_t scratch_off = total;
  total += fs::a256(scratch);
  if (fs::dev_malloc(&e->base, total) != hipSuccess) {
    hipGetLastError();
    delete h;
    fs::set_error("hipMalloc of %zu bytes failed", total);
    return FS_E_NOMEM;
  }
  e->bytes = total;
  char* b = (char*)e->base;
  bool good = true;
  int device = 0;
  good = fs::ok(e, hipGetDevice(&device), "hipGetDevice");
  size_t k = 0;
  const double kb = 2.0 * M_PI / L;
  for (auto& c : e->cls) {
    c.state_off = (long long*)(b + offs[k++]);
    c.w1 = b + offs[k++];
    c.w2 = b + offs[k++];
    c.acc = b + offs[k++];
    c.tw = b + offs[k++];
    c.e1 = b + offs[k++];
    c.eh1 = b + offs[k++];
    const int N = c.n;
    std::vector<long long> so(c.nruns);
    for (int l = 0; l < c.nruns; l++) so[l] = e->offsets[c.runs[l]];
    std::vector<float> tw(2 * N), e1(N), eh1(N);
    for (int m = 0; m < N; m++) {
      const double a = -2.0 * M_PI * (double)m / (double)N;
      tw[2 * m] = (float)std::cos(a);
      tw[2 * m + 1] = (float)std::sin(a);
      const int mm = m <= N / 2 ? m : m - N;
      const double k2 = kb * kb * (double)mm * (double)mm;
      e1[m] = (float)std::exp(-nu * dt * k2);
      eh1[m] = (float)std::exp(-0.5 * nu * dt * k2);
    }
    good = good &&
           fs::ok(e, hipMemcpy(c.state_off, so.data(), sizeof(long long) * c.nruns, hipMemcpyHostToDevice), "copy") &&
           fs::ok(e, hipMemcpy(c.tw, tw.data(), 8 * N, hipMemcpyHostToDevice), "copy") &&
           fs::ok(e, hipMemcpy(c.e1, e1.data(), 4 * N, hipMemcpyHostToDevice), "copy") &&
           fs::ok(e, hipMemcpy(c.eh1, eh1.data(), 4 * N, hipMemcpyHostToDevice), "copy") &&
           fs::ok(e, hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking), "stream");
  }
  good = good && fs::ok(e, hipEventCreateWithFlags(&e->fork, hipEventDisableTiming), "event");
  e->joins.resize(e->cls.size(), nullptr);
  for (auto& ev : e->joins)
    good = good && fs::ok(e, hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
  if (good) {
    void* scratch_state = b + scratch_off;
    good = fs::ok(e, hipMemset(scratch_state, 0, scratch), "clear scratch");
    // the scratch state stands in for the packed state while tuning: use
    // zero offsets so every run of a class reads the same scratch run
    for (auto& c : e->cls) {
      if (!good) break;
      if (!(o.flags & FS_NO_AUTOTUNE) && !c.resident) {
        std::vector<long long> zero(c.nruns, 0);
        for (int l = 0; l < c.nruns; l++) zero[l] = (long long)l * c.n * (c.n / 2 + 1);
        good = fs::ok(e, hipMemcpy(c.state_off, zero.data(), sizeof(long long) * c.nruns, hipMemcpyHostToDevice), "copy");
        if (good) fs::tune_class(e, c, scratch_state, device);
        std::vector<long long> so(c.nruns);
        for (int l = 0; l < c.nruns; l++) so[l] = e->offsets[c.runs[l]];
        good = good && !e->failed &&
               fs::ok(e, hipMemcpy(c.state_off, so.data(), sizeof(long long) * c.nruns, hipMemcpyHostToDevice), "copy");
      }
    }
    good = good && fs::ok(e, hipDeviceSynchronize(), "tune sync");
  }
  if (!good) {
    std::string msg = fs_last_error();
    fs::release(e);
    delete h;
    fs::set_error("%s", msg.c_str());
    return FS_E_DEVICE;
  }
  *out = h;
  return FS_OK;
}

fs_status fs_ensemble_offsets(const fs_ensemble* ens, int64_t* offsets) {
  if (!ens || !offsets) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  for (int r = 0; r <= ens->e.nruns; r++) offsets[r] = ens->e.offsets[r];
  return FS_OK;
}

fs_status fs_ensemble_schedule(const fs_ensemble* ens, int cls, int* n, int* nruns, int* y_lines,
                               int* x_rowpairs, double* us_y, double* us_x) {
  if (!ens) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  if (cls < 0 || cls >= (int)ens->e.cls.size()) {
    fs::set_error("class %d out of range", cls);
    return FS_E_INVALID;
  }
  const EnsClass& c = ens->e.cls[cls];
  if (n) *n = c.n;
  if (nruns) *nruns = c.nruns;
  if (c.resident) {
    if (y_lines) *y_lines = 0;
    if (x_rowpairs) *x_rowpairs = 0;
    if (us_y) *us_y = 0;
    if (us_x) *us_x = 0;
    return FS_OK;
  }
  if (y_lines) *y_lines = c.ylines;
  int rp = 1;
  switch (c.n) {
    case 64: rp = fs::x_rowpairs<64>(c.xmul); break;
    case 128: rp = fs::x_rowpairs<128>(c.xmul); break;
    case 256: rp = fs::x_rowpairs<256>(c.xmul); break;
    default: rp = fs::x_rowpairs<512>(c.xmul); break;
  }
  if (x_rowpairs) *x_rowpairs = rp;
  if (us_y) *us_y = c.us_y;
  if (us_x) *us_x = c.us_x;
  return FS_OK;
}

fs_status fs_ensemble_step_rk4(fs_ensemble* ens, void* packed_state, int nsteps) {
  if (!ens || !packed_state) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  Ensemble* e = &ens->e;
  if (e->failed) return FS_E_DEVICE;
  if (nsteps < 0) {
    fs::set_error("nsteps = %d must be >= 0", nsteps);
    return FS_E_INVALID;
  }
  if (nsteps == 0) return FS_OK;
  const bool graphs = !(e->flags & FS_NO_GRAPH);
  if (graphs && !e->graphs.empty() && (e->gstate != packed_state || e->gsteps != nsteps)) {
    for (auto& g : e->graphs)
      if (g) hipGraphExecDestroy(g);
    e->graphs.clear();
  }
  if (graphs && e->graphs.empty()) {
    // one graph per class: the class's whole chain of steps, captured on its
    // own stream (a single graph holding the classes as parallel branches
    // ran them 7 % slower than separate streams do)
    e->graphs.assign(e->cls.size(), nullptr);
    bool good = true;
    for (size_t i = 0; good && i < e->cls.size(); i++) {
      auto& c = e->cls[i];
      hipGraph_t g = nullptr;
      good = fs::ok(e, hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal),
                    "begin capture");
      if (!good) break;
      fs::class_steps(e, c, packed_state, nsteps, c.stream);
      good = fs::ok(e, hipGetLastError(), "capture launch");
      const hipError_t err = hipStreamEndCapture(c.stream, &g);
      good = good && fs::ok(e, err, "end capture");
      if (good) good = fs::ok(e, hipGraphInstantiate(&e->graphs[i], g, nullptr, nullptr, 0),
                              "instantiate");
      if (g) hipGraphDestroy(g);
    }
    if (!good) return FS_E_DEVICE;
    e->gstate = packed_state;
    e->gsteps = nsteps;
  }
  // the classes' chains on their own streams (a graph launch each, or their
  // kernels directly), forked from and joined back into the caller's stream
  bool good = fs::ok(e, hipEventRecord(e->fork, e->stream), "fork");
  for (size_t i = 0; good && i < e->cls.size(); i++) {
    auto& c = e->cls[i];
    good = fs::ok(e, hipStreamWaitEvent(c.stream, e->fork, 0), "fork wait");
    if (!good) break;
    if (graphs) {
      good = fs::ok(e, hipGraphLaunch(e->graphs[i], c.stream), "graph launch");
    } else {
      fs::class_steps(e, c, packed_state, nsteps, c.stream);
      good = fs::ok(e, hipGetLastError(), "launch");
    }
    good = good && fs::ok(e, hipEventRecord(e->joins[i], c.stream), "join") &&
           fs::ok(e, hipStreamWaitEvent(e->stream, e->joins[i], 0), "join wait");
  }
  return good ? FS_OK : FS_E_DEVICE;
}

fs_status fs_ensemble_destroy(fs_ensemble* ens) {
  if (!ens) return FS_OK;
  Ensemble* e = &ens->e;
  if (e->stream)
    hipStreamSynchronize(e->stream);
  else
    hipDeviceSynchronize();
  fs::release(e);
  delete ens;
  return FS_OK;
}

}  // extern "C"
