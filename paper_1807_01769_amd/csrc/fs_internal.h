// fs_internal.h -- plan object and kernel-family dispatch shared by the host
// sources of libfs.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "fs.h"

namespace fs {

enum KernelId {
  KID_P1 = 0,
  KID_YINV,
  KID_X,
  KID_YFWD,
  KID_Z,
  KID_ALPHA,
  KID_FILL,
  KID_FFT,
  KID_DIAG,
  KID_COUNT
};

struct Plan;

// Kernel sequences of one (ndim, precision, n) combination.
struct Ops {
  // first inverse pass of a stage from the caller's state (also records the
  // forcing-band stage input)
  void (*p1)(Plan*, const void* state);
  // one RK4 stage (mode 1..4) after its first pass; do_p1 = 0 skips the next
  // stage's inverse transforms at the end of the last step
  void (*stage)(Plan*, void* state, int mode, int do_p1);
  // tendency of `state` into `out` on the kept modes (with fill, zeros on
  // every other element); with fresh_alpha the forcing coefficient is
  // recomputed from `state`, otherwise the one left on the device by the
  // last `alpha` call is used
  void (*tendency)(Plan*, const void* state, void* out, bool fresh_alpha, bool fill);
  void (*fft_fwd)(Plan*, const void* phys, void* spec);
  void (*fft_inv)(Plan*, const void* spec, void* phys);
  // nf stacked fields at once through caller workspaces wa, wb of
  // nf * elems_full complex elements each (3D only; may be null); with grad
  // the input is a velocity state and the nine outputs its gradients
  void (*fft_fwd_n)(Plan*, const void* phys, void* spec, int nf, void* wa, void* wb);
  void (*fft_inv_n)(Plan*, const void* spec, void* phys, int nf, void* wa, void* wb, bool grad);
  // forcing coefficient from the state (3D only; may be null)
  void (*alpha)(Plan*, const void* state);
  // adaptive step: dt from the velocity maximum of the step, decay tables,
  // elapsed time
  void (*dtstep)(Plan*);
  // diagnostics
  void (*diag)(Plan*, const void* state, double* spectrum, int nbins, double* energy,
               double* enstrophy);
  // 1D spectra of the velocity components
  void (*spectra1d)(Plan*, const void* state, double* out);
  // longitudinal structure functions of the velocity (r: host array)
  void (*structure)(Plan*, const void* state, int nr, const int* r, int pmax, double* out);
  // spectral energy transfer of a tendency
  void (*transfer)(Plan*, const void* state, const void* tend, double* transfer, double* flux,
                   int nbins, double* energy_rate, double* enstrophy_rate);
  // workspace element counts (complex elements of the plan's precision)
  size_t elems_a, elems_b, elems_acc;
  size_t elems_full;  // one undealiased field in the transform workspace layout
  size_t elems_sin;   // 2D Boussinesq stage-input buffer (0 otherwise)
};

struct Plan {
  int n = 0, ndim = 3, prec = FS_F32;
  double L = 0, nu = 0, dt = 0;
  double fpow = 0, fkmin = 2, fkmax = 3;
  int bw = 0, m2min = 0, m2max = -1;  // forcing band in integer |m|^2
  unsigned flags = 0;
  int scheme = FS_SCHEME_RK4;
  double cfl = 0;           // > 0: dt_n = min(dt, cfl (L/n) / max|u_c|) every step
  int nfield = 1;           // state fields: 2D 1 (vorticity), 3D 3 (velocity); + 1 buoyancy
  double n2 = 0;            // Boussinesq: squared buoyancy frequency
  double rotf = 0;          // 3D rotating frame: Coriolis parameter
  double t_fixed = 0;       // elapsed time of fixed-dt steps (host)
  int device = 0;
  hipStream_t stream = nullptr;  // caller's stream
  hipStream_t launch = nullptr;  // stream kernels go to right now
  hipStream_t cap = nullptr;     // private stream used for graph capture
  Ops ops{};
  // device memory (one allocation, carved)
  void* base = nullptr;
  bool owns_base = true;  // false when the caller supplied the workspace
  size_t bytes_total = 0;
  void *tw = nullptr, *e1 = nullptr, *eh1 = nullptr;
  void *bufA = nullptr, *bufB = nullptr, *acc = nullptr, *vband = nullptr, *alpha = nullptr;
  double* dpart = nullptr;  // diagnostics partial sums
  void* dtdev = nullptr;    // step of the current step (working precision)
  void* sin = nullptr;      // 2D Boussinesq stage input
  double* tdev = nullptr;   // elapsed time of adaptive steps
  unsigned long long* umaxdev = nullptr;  // velocity maximum of the step (double bits)
  unsigned* nonfin = nullptr;     // FS_CHECK_FINITE: set when a step wrote a non-finite value
  unsigned* nonfin_host = nullptr;  // pinned copy of *nonfin, written after each step call
  hipEvent_t nonfin_ev = nullptr;   // completion of that copy
  bool nonfin_pending = false;
  int dpart_blocks = 0;
  // captured step graphs for one state pointer
  hipGraphExec_t gmid = nullptr, glast = nullptr;
  void* gstate = nullptr;
  // profiling
  struct Mark {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  double kms[KID_COUNT] = {};
  long kcount[KID_COUNT] = {};
  bool failed = false;

  // bracket a kernel launch (records events when profiling)
  void begin(int kid);
  void end(int kid);
  bool ok(hipError_t e, const char* what);
};

void set_error(const char* fmt, ...);

// Every device and pinned-host allocation of the library goes through these.
// Test hook: while the environment variable FS_TEST_FAIL_ALLOC holds "k"
// (optionally followed by a tag, "2#plan"), the k-th allocation counted from
// the moment the variable took its current value fails as if the device were
// out of memory, so that the FS_E_NOMEM paths can be exercised.
hipError_t dev_malloc(void** ptr, size_t bytes);
hipError_t pinned_malloc(void** ptr, size_t bytes);
// check the launch just made; marks the plan failed on error
bool launched(Plan* p, const char* what);

template <typename T>
Ops make_ops3(int n, int nfield);
template <typename T>
Ops make_ops2(int n, int nfield);

// diagnostics launchers (diag.hip)
template <typename T>
void launch_diag(Plan* p, const void* state, double* spectrum, int nbins, double* energy,
                 double* enstrophy);
template <typename T>
void launch_spectra1d(Plan* p, const void* state, double* out);
template <typename T>
void launch_structure(Plan* p, const void* state, int nr, const int* r, int pmax, double* out);
template <typename T>
void launch_transfer(Plan* p, const void* state, const void* tend, double* transfer,
                     double* flux, int nbins, double* energy_rate, double* enstrophy_rate);
template <typename T>
void launch_alpha(Plan* p, const void* state);
template <typename T>
void launch_dtstep(Plan* p);
void launch_time(Plan* p, double* t, double* dt);
template <typename T>
void launch_fill(Plan* p, void* ptr, size_t n_complex);

// closure network (mlp.hip)
struct Mlp;
void mlp_forward_launch(Mlp* net, const void* x, float* y, int64_t P, const float* out_scale,
                        hipStream_t s);
// network output o -> stress: clip(y_o) * scale[o] (clip <= 0: none)
struct StressMap {
  float scale[6];
  float clip;
};
// tau[6][P] = StressMap(net(BF16(A[9][P] * inv_a)))
void mlp_forward_planar_launch(Mlp* net, const float* A, int64_t P, float inv_a, float* tau,
                               StressMap sm, hipStream_t s);
int mlp_nparams();

constexpr int kDiagThreads = 256;
constexpr int kDiagMaxBins = 1024;
constexpr int kSfMaxR = 64;  // separations per structure-function call
constexpr int kSfMaxP = 8;   // highest moment
constexpr int kDiagMaxBlocks = 1024;

}  // namespace fs

struct fs_plan {
  fs::Plan p;
};
struct fs_mlp;
namespace fs {
Mlp* mlp_of(fs_mlp* net);
}
