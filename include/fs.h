/*
 * fs.h -- C ABI of the MI355X pseudo-spectral Navier-Stokes library (libfs.so).
 *
 * The library advances the incompressible Navier-Stokes equations in a
 * periodic box [0, L)^d (d = 2 in vorticity form, d = 3 in velocity form)
 * with a Fourier pseudo-spectral method and the fourth-order Runge-Kutta
 * scheme at constant time step, the viscous term integrated exactly.  This is
 * the numerical method of the FluidSim paper (section "Implementation and
 * architecture": the operators object provides FFT/IFFT, dealiasing, curl and
 * divergence, the time-stepping object advances the state with RK4; section
 * "CFD pseudo-spectral code comparisons": one 3D step is made of FFTs, the
 * RK4 update, curl, vector product and projection, with part of the linear
 * terms treated exactly).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Wavenumbers k = (2 pi / L) m, m integer.  Forward transforms carry the
 * factor 1/N^d; inverse transforms are unscaled.  Dealiasing is the 2/3 rule
 * on a cube: a mode is kept iff 3|m_a| < N on every axis.  Entry points that
 * take a spectral state treat modes outside the kept set as zero and never
 * write them (except fs_tendency, which writes zeros there).
 *
 * Layouts (C order, interleaved complex, contiguous):
 *   3D state / tendency : complex[3][N][N][N/2+1]   (component, kz, ky, kx)
 *                         (FS_BOUSSINESQ: complex[4][...], + buoyancy)
 *   2D state / tendency : complex[N][N/2+1]         (ky, kx), vorticity
 *                         (FS_BOUSSINESQ: complex[2][N][N/2+1], + buoyancy)
 *   3D physical field   : real[N][N][N]             (z, y, x)
 *   2D physical field   : real[N][N]                (y, x)
 * ky and kz are in FFT order (0..N/2-1, -N/2..-1).  "complex" is two floats
 * (FS_F32) or two doubles (FS_F64).
 *
 * Memory and streams: every array argument is device memory owned by the
 * caller (e.g. a torch tensor), 16-byte aligned.  The plan owns its
 * workspace and tables, allocated once by fs_plan_create; no other call
 * allocates device memory.  Every call enqueues work on the plan's stream and
 * returns without synchronising; results are visible to later work on that
 * stream.  Plans are not thread safe; distinct plans are independent.
 *
 * Errors: arguments are validated on the host before anything is enqueued;
 * on error nothing is enqueued, outputs are untouched and the status is
 * negative.  fs_last_error() returns a description of the last failure of
 * the calling thread.  A HIP runtime failure marks the plan failed
 * (FS_E_DEVICE for every later call); destroy it.
 */
#ifndef FS_H_
#define FS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FS_OK = 0,
  FS_E_INVALID = -1,     /* bad argument (null pointer, n, L, nu, dt, ...) */
  FS_E_UNSUPPORTED = -2, /* valid but not implemented (e.g. n not 2^k in 16..1024) */
  FS_E_NOMEM = -3,       /* device allocation failed at plan creation */
  FS_E_DEVICE = -4,      /* HIP runtime error; the plan is unusable */
  FS_E_NONFINITE = -5    /* FS_CHECK_FINITE: the last step wrote non-finite values */
} fs_status;

enum { FS_F32 = 0, FS_F64 = 1 };
/* time schemes (the time-stepping object of the paper advances with RK2 or
 * RK4): Lawson integrating-factor RK4, or the Lawson midpoint rule (RK2)
 *   v = Eh (u + dt/2 N(u)),  u <- E u + dt Eh N(v) */
enum { FS_SCHEME_RK4 = 0, FS_SCHEME_RK2 = 1 };

/* flags */
#define FS_NO_GRAPH 0x1u /* launch kernels one by one instead of a captured graph */
#define FS_PROFILE 0x2u  /* time every kernel with events (see fs_profile_read) */
#define FS_NO_AUTOTUNE 0x4u /* ensembles: keep the default schedules */
#define FS_NO_RESIDENT 0x20u /* ensembles: no block-resident small classes */
/* Boussinesq (stably stratified) flow with a buoyancy field b (Prandtl
 * number 1, squared buoyancy frequency opts.n2), advected in conservative
 * form and dealiased like the velocity.
 * 2D, vertical plane, gravity along -y:
 *   dw/dt + u.grad w = db/dx + nu lap w,  db/dt + u.grad b = -n2 v + nu lap b;
 *   state complex[2][N][N/2+1] (w_hat, b_hat); the coupling terms are part of
 *   the tendency, the diffusion stays exact.
 * 3D, gravity along -z:
 *   du/dt + w x u = -grad p + b z + nu lap u,  db/dt + u.grad b = -n2 uz + nu lap b;
 *   state complex[4][N][N][N/2+1] (ux, uy, uz, b hats).  The linear terms
 *   (buoyancy force, stratification, diffusion) are integrated exactly: with
 *   q = z - khat khat_z, g2 = |k_h|^2/|k|^2, s = sqrt(n2 g2), c = cos(s t),
 *   S = sin(s t)/s (t when s = 0),
 *   E(t)(u, b) = exp(-nu k^2 t) (u + [(c-1) uz/g2 + S b] q,  c b - n2 S uz);
 *   fs_tendency returns the nonlinear terms (-i k.(u b)^ for b).  With a
 *   rotation as well, the Coriolis force joins the exactly integrated terms
 *   (see fs_plan_opts.rotation); forcing acts on u; adaptive steps take their
 *   size from u.
 * The mean mode (k = 0, 3D): a periodic pressure has no mean gradient, so the
 *   linear terms act on the mean unprojected.  Over a time t the mean
 *   velocity U and mean buoyancy B become
 *     Ux' = cos(f t) Ux + sin(f t) Uy,  Uy' = cos(f t) Uy - sin(f t) Ux,
 *     Uz' = cos(N t) Uz + S B,          B'  = cos(N t) B - n2 S Uz,
 *   S = sin(N t)/N (t when N = 0), f = opts.rotation (0 without rotation),
 *   N^2 = opts.n2 (Boussinesq plans; without buoyancy Uz is unchanged); the
 *   nonlinear terms never change the mean (their mean is zero), so without
 *   rotation or buoyancy the mean velocity is carried unchanged.
 * Diagnostics, transfer and 1D spectra describe the velocity (2D: vorticity)
 * part. */
#define FS_BOUSSINESQ 0x8u
/* Check every step for non-finite values: the last stage of each step flags
 * any non-finite value it writes to the state (one device flag, set by the
 * step's own kernels, copied to pinned host memory after each fs_step_rk4
 * call).  The next fs_step_rk4, fs_tendency, fs_energy_spectrum or
 * fs_plan_time call waits for that copy and, if the flag is set, clears it
 * and returns FS_E_NONFINITE without enqueuing anything; the plan stays
 * usable.  Costs one host wait per call on the previous step call. */
#define FS_CHECK_FINITE 0x10u

typedef struct fs_plan fs_plan;

typedef struct {
  int ndim;             /* 2 or 3 (default 3) */
  int precision;        /* FS_F32 (default) or FS_F64 */
  void *stream;         /* hipStream_t the plan enqueues on; NULL = null stream */
  double forcing_power; /* 3D only: constant injected power P; 0 = no forcing */
  double forcing_kmin;  /* forcing band kmin <= |k| <= kmax (default 2, 3) */
  double forcing_kmax;
  unsigned flags;       /* FS_NO_GRAPH | FS_PROFILE | FS_NO_AUTOTUNE | FS_BOUSSINESQ |
                           FS_CHECK_FINITE | FS_NO_RESIDENT */
  int scheme;           /* FS_SCHEME_RK4 (default) or FS_SCHEME_RK2 */
  double cfl;           /* > 0: adaptive steps, dt_n = min(dt, cfl (L/n) / umax_n) with
                           umax_n the largest |u_c| of the physical velocity of u_n
                           (2D: from the vorticity), measured on the GPU during the
                           step's first stage; 0 (default): the fixed step dt */
  double n2;            /* FS_BOUSSINESQ: squared buoyancy frequency N^2 >= 0 */
  double rotation;      /* 3D: Coriolis parameter f of a frame rotating about z
                           (acceleration -f z x u); 0 (default): none.  Folded into
                           the exact linear propagator: for solenoidal fields
                           E(t) u = exp(-nu k^2 t)(cos(s t) u - sin(s t) khat x u),
                           s = f kz / |k|; fs_tendency excludes it.  With
                           FS_BOUSSINESQ, u = a1 e1 + a2 e2 (e1 = khat x z / g,
                           e2 = khat x e1, g = |k_h|/|k|) and (a1, a2, b) obey
                           a1' = sf a2, a2' = -sf a1 - g b, b' = n2 g a2
                           (sf = f khat_z), integrated exactly as the rotation
                           exp(t K) = I + s K + c K^2 in (a1, a2, b/N):
                           w^2 = sf^2 + n2 g^2, s = sin(w t)/w,
                           c = (1 - cos(w t))/w^2 */
  void *workspace;      /* optional caller-owned device workspace (e.g. a torch
                           tensor), 256-byte aligned, of at least
                           fs_plan_workspace_bytes bytes; the plan uses it instead
                           of allocating and never frees it; it must outlive the
                           plan and not be shared with another live plan.
                           NULL (default): the plan allocates its own */
  size_t workspace_bytes; /* size of workspace in bytes */
} fs_plan_opts;

/* Fill *opts with the defaults listed above. */
void fs_plan_opts_default(fs_plan_opts *opts);

/*
 * Create a plan for grid size n (power of two, 16..1024), box length L > 0,
 * kinematic viscosity nu >= 0 and time step dt > 0 (the four physical
 * parameters of one constant-step RK4 run).  Builds the twiddle and
 * integrating-factor tables in FP64 on the host (rounded once to the plan's
 * precision) and allocates the workspace.  opts may be NULL (defaults).
 * The forcing band must lie inside the kept cube.
 * Errors: FS_E_INVALID, FS_E_UNSUPPORTED, FS_E_NOMEM, FS_E_DEVICE.
 */
fs_status fs_plan_create(fs_plan **out, int n, double L, double nu, double dt,
                         const fs_plan_opts *opts);

/* Elapsed simulated time of the plan's steps since creation and the step size
 * of the last step (device doubles, each nullable); enqueued like the steps. */
fs_status fs_plan_time(fs_plan *plan, double *time, double *last_dt);

/* Release a plan and its workspace (waits for its stream).  NULL is a no-op. */
fs_status fs_plan_destroy(fs_plan *plan);

/* Replace the stream the plan enqueues on (NULL = null stream). */
fs_status fs_plan_set_stream(fs_plan *plan, void *stream);

/* Number of complex elements of a state: 3*N*N*(N/2+1) (3D) or N*(N/2+1) (2D),
 * times 4/3 (3D) or 2 (2D) with FS_BOUSSINESQ. */
fs_status fs_state_elems(const fs_plan *plan, size_t *n_complex);

/* Device bytes of the plan's workspace and tables (its own allocation or the
 * part of the caller's workspace it uses). */
fs_status fs_workspace_bytes(const fs_plan *plan, size_t *bytes);

/* Device workspace a plan of size n with these options needs (NULL opts:
 * defaults), before creating it; validates n and opts like fs_plan_create
 * (L, nu and dt do not change the size).  Needs no device. */
fs_status fs_plan_workspace_bytes(int n, const fs_plan_opts *opts, size_t *bytes);

/* Number of spectrum bins that covers every kept mode:
 * floor(sqrt(d) * K + 1/2) + 1 with K = floor((N-1)/3). */
fs_status fs_spectrum_bins(const fs_plan *plan, int *nbins);

/*
 * Forward real-to-complex transform of one scalar field (the paper's
 * fft_as_arg, section "Performance", profiling): spec = N^-d sum_x phys(x)
 * exp(-i k.x) for kx in [0, N/2].  Undealiased; out of place; phys is not
 * modified.  phys: real[N]^d; spec: complex[N]^(d-1)[N/2+1].
 */
fs_status fs_fft_forward(fs_plan *plan, const void *phys, void *spec);

/*
 * Inverse complex-to-real transform (ifft_as_arg): phys(x) = Re sum_k
 * spec_full(k) exp(i k.x), spec_full the Hermitian completion of spec (the
 * imaginary parts of self-conjugate modes do not contribute).  Unscaled;
 * spec is not modified.
 */
fs_status fs_fft_inverse(fs_plan *plan, const void *spec, void *phys);

/*
 * Nonlinear tendency of a spectral state, dealiased (3D: the curl, vector
 * product and projection tasks; 2D: velocity from vorticity and the
 * divergence of the vorticity flux), without the viscous term:
 *   3D: tend = P[(u x w)^] + alpha u_hat on the forcing band, w = curl u,
 *       P v = v - k (k.v)/|k|^2, tend(0) = 0, alpha = power / sum_band
 *       w |u_hat|^2 computed from `state` (0 when forcing is off);
 *   2D: tend = -i kx (u w)^ - i ky (v w)^, u_hat = i ky w_hat/|k|^2,
 *       v_hat = -i kx w_hat/|k|^2, tend(0) = 0.
 * Every element of tend is written (zero outside the kept set).  state and
 * tend must not overlap.
 */
fs_status fs_tendency(fs_plan *plan, const void *state, void *tend);

/*
 * Advance state in place by nsteps >= 0 steps of the Lawson integrating-factor
 * RK4 scheme (RK4 at constant step, section "Performance", 2D and 3D
 * benchmarks; exact viscous factor E = exp(-nu |k|^2 dt)):
 *   k1 = N(u)  k2 = N(Eh (u + dt/2 k1))  k3 = N(Eh u + dt/2 k2)
 *   k4 = N(E u + dt Eh k3)   u' = E u + dt/6 (E k1 + 2 Eh k2 + 2 Eh k3 + k4)
 * with Eh = exp(-nu |k|^2 dt/2) and N the tendency of fs_tendency.  With
 * forcing, alpha is recomputed from u at the start of every step and held
 * for its four stages.  Modes outside the kept set are not written.
 */
fs_status fs_step_rk4(fs_plan *plan, void *state, int nsteps);

/*
 * FP64 diagnostics of a state (sim.output.spatial_means and spectra of the
 * paper, section "Implementation and architecture"), reduced
 * deterministically on the GPU over the kept set with half-spectrum weights
 * w = 1 (kx = 0), 2 (kx > 0):
 *   energy    E = 1/2 sum w |u_hat|^2      (2D: |u_hat|^2 = |w_hat|^2/|k|^2)
 *   enstrophy Z = 1/2 sum w |w_hat|^2      (3D: w_hat = i k x u_hat)
 *   spectrum[s] = 1/2 sum over modes with floor(|m| + 1/2) = s of w |u_hat|^2
 * for s < nbins (1 <= nbins <= 1024); modes in higher shells count in E only.
 * spectrum (nbins doubles), energy and enstrophy (one double each, may be
 * NULL) are device pointers.
 */
fs_status fs_energy_spectrum(fs_plan *plan, const void *state, double *spectrum, int nbins,
                             double *energy, double *enstrophy);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * diagnostics of fs_energy_spectrum without a plan and without any
 * allocation.  The state is described by (ndim, n, precision, L) as a plan
 * with those values would describe it (same layout and supported sizes); the
 * results are bit for bit those of fs_energy_spectrum.  The block partial
 * sums live in a static device array of 8 MiB, one copy per device, held
 * until the process ends: a call needing more, blocks * (nbins + 2) doubles
 * with blocks = min(rows / 4, 1024), rows = M^2 in 3D and M in 2D,
 * M = 2 floor((n-1)/3) + 1 (nbins > 1022 at the largest grids), is rejected
 * with FS_E_INVALID.
 * Enqueued on `stream` (a hipStream_t; NULL = null stream) with no
 * synchronisation; calls that overlap on one device share the array and race.
 * Errors: FS_E_INVALID / FS_E_UNSUPPORTED before anything is enqueued,
 * FS_E_DEVICE if the device or the launch fails.
 */
fs_status fs_energy_spectrum_static(int ndim, int n, int precision, double L, const void *state,
                                    double *spectrum, int nbins, double *energy,
                                    double *enstrophy, void *stream);

/*
 * 1D spectra ("spectra as functions of ... a component of the wavenumber",
 * section "Implementation and architecture"): the energy of each velocity
 * component binned by the modulus of one wavenumber component,
 *   out[a][c][k] = 1/2 sum over kept modes with |m_a| = k of w |u_c_hat|^2,
 * a, c over the d axes / components (2D: velocity from the vorticity), k = 0..K
 * with K = floor((n-1)/3): out holds d*d*(K+1) device doubles.  Each axis
 * sums to the component's energy.  Deterministic; uses the plan's transform
 * workspace as scratch (no other call may run on the plan concurrently).
 */
fs_status fs_energy_spectra_1d(fs_plan *plan, const void *state, double *out);

/*
 * Longitudinal structure functions of the velocity (the statistics of
 * velocity increments the paper's output object provides, section
 * "Implementation and architecture"): with u the physical velocity of the
 * kept modes (2D: from the vorticity) and du_a(x, r) = u_a(x + r e_a) -
 * u_a(x) for r grid spacings along axis a (periodic), averaged over every
 * grid point and the d axes,
 *   out[j * pmax + p - 1]        = < du^p >      (signed moments)
 *   out[(nr + j) * pmax + p - 1] = < |du|^p >    (absolute moments)
 * for p = 1..pmax (1 <= pmax <= 8) and the nr separations r[j] (host array,
 * 1 <= nr <= 64, 1 <= r[j] <= n-1).  out holds 2 * nr * pmax device doubles.
 * Increments are formed in FP64 from the working-precision velocity and
 * summed in FP64, deterministically.  Uses the plan's transform workspace as
 * scratch (no other call may run on the plan concurrently); for
 * FS_BOUSSINESQ states the velocity part is used.
 */
fs_status fs_structure_functions(fs_plan *plan, const void *state, int nr, const int *r, int pmax,
                                 double *out);

/*
 * Spectral energy budget of a tendency (the spectra of energy transfer the
 * paper's output object provides, section "Implementation and
 * architecture"): with tend = d state / dt (e.g. from fs_tendency; viscosity
 * excluded, forcing included when the plan forces),
 *   transfer[s] = sum over modes of shell s of w Re(conj(u_hat) . tend)
 *                 (2D: w Re(conj(w_hat) tend) / |k|^2),
 *   energy_rate = the sum over every kept mode (dE/dt of the tendency),
 *   enstrophy_rate = sum w Re(conj(w_hat) . i k x tend) (2D: sum w
 *                 Re(conj(w_hat) tend)).
 *   flux[s] = -sum_{s' <= s} transfer[s'], the energy flux through shell s
 *                 (nullable; summed in shell order).
 * Same weights, shells, determinism and pointer rules as fs_energy_spectrum;
 * state and tend are not modified.
 */
fs_status fs_energy_transfer(fs_plan *plan, const void *state, const void *tend,
                             double *transfer, double *flux, int nbins, double *energy_rate,
                             double *enstrophy_rate);

/*
 * With FS_PROFILE: accumulate the elapsed time of every kernel launched since
 * the previous call (waits for them) into ms[kid] and launch counts into
 * counts[kid] for kid < nk; names[kid] receives a static kernel name.  Kernel
 * ids: 0 p1 (first inverse pass from the state), 1 y-inverse, 2 x (C2R,
 * product, R2C), 3 y-forward, 4 z/y fused stage pass, 5 forcing coefficient,
 * 6 fill, 7 transform-only passes, 8 diagnostics.  Any pointer may be NULL.
 */
fs_status fs_profile_read(fs_plan *plan, double *ms, long *counts, const char **names, int nk);

/*
 * Ensembles of independent 2D runs of uneven sizes (the 2D benchmark setup
 * of the paper's "Performance" section, many runs at once), FP32.
 *
 * fs_ensemble_create: nruns runs with grid sizes n[r] in {64, 128, 256, 512}
 * sharing L, nu, dt (opts: ndim must be 2, precision FS_F32, no forcing;
 * flags FS_NO_GRAPH, FS_NO_AUTOTUNE, FS_NO_RESIDENT; fixed-dt RK4, no rotation
 * or buoyancy, no caller workspace).  The packed state is the concatenation
 * of the runs' 2D states, run r at complex offset offsets[r] (see
 * fs_ensemble_offsets).  Runs of equal size form a class.  Classes of 64 and
 * 128 points a side are advanced block-resident: one block per run keeps the
 * run's intermediate fields in LDS through all steps of a call and touches
 * HBM only for the state and its accumulator (the class-batched results up
 * to rounding; FS_NO_RESIDENT treats them like the larger classes).  For the other
 * classes the block schedule is chosen at creation by timing candidates on
 * the device (unless FS_NO_AUTOTUNE).  Owns its workspace.
 */
typedef struct fs_ensemble fs_ensemble;
fs_status fs_ensemble_create(fs_ensemble **out, int nruns, const int *n, double L, double nu,
                             double dt, const fs_plan_opts *opts);
/* Host array of nruns + 1 complex offsets; offsets[nruns] is the total size. */
fs_status fs_ensemble_offsets(const fs_ensemble *ens, int64_t *offsets);
/*
 * Advance every run of the packed state (device memory) by nsteps Lawson
 * IF-RK4 steps, exactly as fs_step_rk4 would advance each run alone.  All
 * steps of one size class are captured as one hipGraph (reused while the
 * pointer and nsteps are unchanged); the classes' graphs are launched once
 * each on streams of their own, forked from and joined back into the
 * ensemble's stream, so that the classes run concurrently.  With FS_NO_GRAPH
 * the same chains are launched kernel by kernel on those streams.
 */
fs_status fs_ensemble_step_rk4(fs_ensemble *ens, void *packed_state, int nsteps);
/* Chosen schedule of class cls (classes in increasing size): its size, run
 * count, y-pass lines per block, x-pass row pairs per block and the tuned
 * per-launch times in microseconds (0 when taken from the cache); a
 * block-resident class reports 0 for the last four. */
fs_status fs_ensemble_schedule(const fs_ensemble *ens, int cls, int *n, int *nruns, int *y_lines,
                               int *x_rowpairs, double *us_y, double *us_x);
fs_status fs_ensemble_destroy(fs_ensemble *ens); /* NULL is a no-op */

/*
 * Learned subgrid-stress closure network (a small MLP: 9 filtered velocity
 * gradients -> 6 deviatoric subgrid stresses, two hidden layers of 64 with
 * GELU(x) = x Phi(x)), evaluated and trained with BF16 matrix-core products
 * accumulated in FP32; FP32 master weights and Adam moments.
 *
 * Parameter vector (FP32, fs_mlp_nparams() = 5190 values):
 *   W1[64][9] b1[64] W2[64][64] b2[64] W3[6][64] b3[6]   (W[out][in]).
 * Features: BF16 [npts][16], the 9 inputs in slots 0..8, slots 9..15 zero.
 * Targets and outputs: FP32 [npts][6].  All arrays are device memory.
 * The network owns its parameters, moments and scratch (allocated once).
 * The architecture is fixed: the matrix-core kernels chain the three layers
 * in registers with lane layouts specific to these widths.
 */
typedef struct fs_mlp fs_mlp;
/* Xavier-uniform weights from a counter-based hash of (seed, index), zero
 * biases; work is enqueued on `stream` (hipStream_t, NULL = null stream). */
fs_status fs_mlp_create(fs_mlp **out, uint64_t seed, void *stream);
fs_status fs_mlp_destroy(fs_mlp *net); /* NULL is a no-op */
fs_status fs_mlp_nparams(int *n);
/* Copy the FP32 master parameters from / to device memory (set resets Adam's
 * step count, not its moments). */
fs_status fs_mlp_set_params(fs_mlp *net, const float *params);
fs_status fs_mlp_get_params(const fs_mlp *net, float *params);
/* y = net(x) for npts points. */
fs_status fs_mlp_forward(fs_mlp *net, const void *x_bf16, float *y, int64_t npts);
/* Gradient of the mean squared error over all npts*6 outputs into grad
 * (5190 floats, device) and the loss into *loss (device double, nullable);
 * reduced deterministically. */
fs_status fs_mlp_grad(fs_mlp *net, const void *x_bf16, const float *y_target, int64_t npts,
                      float *grad, double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * gradient of the batch; *loss (nullable) receives the batch loss before
 * the step. */
fs_status fs_mlp_train_step(fs_mlp *net, const void *x_bf16, const float *y_target, int64_t npts,
                            float lr, double *loss);

/*
 * Filtered-DNS training samples for the closure.  The coarse grid nc < nf
 * keeps |m_a| <= Kc = floor((nc-1)/3): the sharp cube cutoff of a fine state
 * IS a coarse state, so filtered DNS and LES share one space.  Both plans are
 * 3D FS_F32 with the same L, on one device and one stream; the object owns
 * fine and coarse scratch (about 4 fine physical fields), allocated once.
 */
typedef struct fs_closure fs_closure;
fs_status fs_closure_create(fs_closure **out, fs_plan *fine, fs_plan *coarse);
fs_status fs_closure_destroy(fs_closure *c); /* NULL is a no-op */
/*
 * Filter of the samples (and of the coarse state they return):
 *   FS_FILTER_SHARP (default): the sharp cube cutoff to the coarse kept set;
 *   FS_FILTER_BOX: the box (top-hat) filter of width L / (2 Kc) along each
 *     axis, i.e. every mode times prod_a sin(x_a) / x_a with x_a = pi m_a /
 *     (2 Kc), then the same cutoff (Kc = floor((nc - 1) / 3)).
 */
#define FS_FILTER_SHARP 0
#define FS_FILTER_BOX 1
fs_status fs_closure_set_filter(fs_closure *c, int filter);
/*
 * From a fine state ([3][nf][nf][nf/2+1], modes outside its kept set
 * ignored):
 *   coarse_state [3][nc][nc][nc/2+1]: the filtered state (every element written);
 *   A   real[9][nc^3]: A[3i+j] = d ubar_i / d x_j at the coarse points;
 *   tau real[6][nc^3]: tau_ij = filter(u_i u_j) - ubar_i ubar_j, with the
 *       fine product formed on the fine grid, trace removed; order xx, yy,
 *       zz, xy, xz, yz.
 */
fs_status fs_closure_samples(fs_closure *c, const void *fine_state, void *coarse_state, float *A,
                             float *tau);
/* msq (device double[15]): mean squares over the coarse grid of the 9 A
 * fields then the 6 tau fields (fixed summation order). */
fs_status fs_closure_moments(fs_closure *c, const float *A, const float *tau, double *msq);
/* Network inputs and targets: x_bf16 [nc^3][16] = BF16(A_k / a_scale) in
 * slots 0..8 (rest zero); with tau (then t too, and host tau_scale[6]),
 * t [nc^3][6] = tau_s / tau_scale[s].  Scales must be > 0. */
fs_status fs_closure_features(fs_closure *c, const float *A, const float *tau, float a_scale,
                              const float *tau_scale, void *x_bf16, float *t);

/*
 * LES on a coarse 3D FS_F32 plan with the learned closure.  The nonlinear
 * term of every RK4 stage becomes N + P[-i k_j tau_ij^] with N the plan's
 * tendency (forcing included, its coefficient frozen per step) and
 *   tau_s = clip(net(A(v) / a_scale)_s) * tau_scale[s]
 * for the stage state v (clip(y) = min(max(y, -clip), clip); clip = 0: none),
 * the features rounded to BF16 as in training.  The viscous term stays exact
 * (Lawson).  model = NULL is the no-model LES: the calls then are exactly
 * fs_tendency / fs_step_rk4 of the plan.  The LES reads the network's
 * parameters when its work runs; it borrows plan and model (both must
 * outlive it) and owns ~40 coarse fields of scratch when a model is given.
 * With a model the plan must use fixed steps, RK4 and no rotation (else
 * FS_E_UNSUPPORTED).
 */
typedef struct fs_les fs_les;
fs_status fs_les_create(fs_les **out, fs_plan *coarse, fs_mlp *model, float a_scale,
                        const float *tau_scale, float clip);
fs_status fs_les_destroy(fs_les *les); /* NULL is a no-op */
/* LES nonlinear term of `state` (forcing coefficient from `state`). */
fs_status fs_les_tendency(fs_les *les, const void *state, void *tend);
/* nsteps >= 0 LES steps in place (one captured graph per state pointer). */
fs_status fs_les_step_rk4(fs_les *les, void *state, int nsteps);

/* Status name and last error message of the calling thread. */
const char *fs_status_str(fs_status s);
const char *fs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FS_H_ */
