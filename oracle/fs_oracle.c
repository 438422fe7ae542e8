/*
 * fs_oracle.c -- plain, slow FP64 CPU reference of the pseudo-spectral
 * Navier-Stokes RK4 step.  TEST INFRASTRUCTURE ONLY: it is loaded by the test
 * suite, by the smoke check and by the benchmark's CPU-baseline leg, never by
 * the product path.  It shares no code with the GPU library.
 *
 * What the paper fixes (FluidSim, section "Implementation and architecture",
 * description of sim.oper / sim.time_stepping; section "CFD pseudo-spectral
 * code comparisons", the 3D task list "FFT, Runge-Kutta 4, curl, vector
 * product and projection"): a Fourier pseudo-spectral solver in a periodic box
 * with FFT/IFFT, dealiasing, curl and divergence operators, advanced by RK4 at
 * constant time step, with part of the linear terms treated exactly.  The
 * paper prints no formulas; everything below is the textbook definition of
 * each of those operations, written out plainly:
 *
 *   transforms   forward  u_hat(k) = N^-d sum_x u(x) exp(-i k.x)  (R2C keeps
 *                kx in [0, N/2]); inverse unscaled; iterative radix-2
 *                Cooley-Tukey with every twiddle taken from libm cos/sin.
 *   dealiasing   keep a mode iff 3|m_a| < N on every axis (2/3 rule, cube);
 *                every entry point treats modes outside that set as zero.
 *   3D tendency  N(u) = P[(u x w)^] with w_hat = i k x u_hat and
 *                P v = v - k (k.v)/|k|^2, N(0) = 0, plus band forcing.
 *   2D tendency  u_hat = i ky w_hat/|k|^2, v_hat = -i kx w_hat/|k|^2,
 *                N(w) = -i kx (u w)^ - i ky (v w)^, N(0) = 0.
 *   time step    Lawson integrating-factor RK4 with E = exp(-nu |k|^2 dt).
 *   diagnostics  E = 1/2 sum w |u_hat|^2, Z = 1/2 sum w |w_hat|^2 with
 *                w = 1 on kx = 0 and 2 elsewhere; shell s = floor(|m| + 1/2).
 *
 * Parity status of every function is listed in the header comment of
 * oracle/__init__.py.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* threads                                                                  */
/* ------------------------------------------------------------------------ */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* 1D FFT: iterative radix-2 decimation in time, in place, unnormalised.     */
/* sign = -1 forward, +1 inverse.  n must be a power of two.                 */
/* ------------------------------------------------------------------------ */
static void fft_line(cplx *x, int n, int sign, const cplx *tw /* n/2 */) {
  /* bit-reversal permutation */
  for (int i = 1, j = 0; i < n; i++) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      cplx t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
  for (int len = 2; len <= n; len <<= 1) {
    int half = len >> 1, step = n / len;
    for (int i = 0; i < n; i += len)
      for (int j = 0; j < half; j++) {
        cplx w = tw[j * step];
        if (sign > 0) w = conj(w);
        cplx a = x[i + j], b = x[i + j + half] * w;
        x[i + j] = a + b;
        x[i + j + half] = a - b;
      }
  }
}

/* twiddles exp(-2 pi i j / n), j < n/2, each from libm */
static cplx *make_twiddles(int n) {
  cplx *tw = malloc(sizeof(cplx) * (size_t)(n / 2 > 0 ? n / 2 : 1));
  for (int j = 0; j < n / 2; j++) {
    double a = -2.0 * M_PI * (double)j / (double)n;
    tw[j] = cos(a) + I * sin(a);
  }
  return tw;
}

static int is_pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }

void or_fft1d(cplx *x, int n, int sign) {
  if (!is_pow2(n)) return;
  cplx *tw = make_twiddles(n);
  fft_line(x, n, sign, tw);
  free(tw);
}

/* Transform a C-order complex array of shape (n0, n1, ..., n_{d-1}) along
 * one axis: gather each line, transform, scatter back. */
static void fft_axis(cplx *a, int ndim, const int *shape, int axis, int sign) {
  int64_t inner = 1, outer = 1;
  for (int d = axis + 1; d < ndim; d++) inner *= shape[d];
  for (int d = 0; d < axis; d++) outer *= shape[d];
  int n = shape[axis];
  cplx *tw = make_twiddles(n);
  int64_t lines = outer * inner;
#pragma omp parallel
  {
    cplx *buf = malloc(sizeof(cplx) * (size_t)n);
#pragma omp for schedule(static)
    for (int64_t l = 0; l < lines; l++) {
      int64_t o = l / inner, in = l % inner;
      cplx *base = a + o * (int64_t)n * inner + in;
      for (int i = 0; i < n; i++) buf[i] = base[(int64_t)i * inner];
      fft_line(buf, n, sign, tw);
      for (int i = 0; i < n; i++) base[(int64_t)i * inner] = buf[i];
    }
    free(buf);
  }
  free(tw);
}

void or_fftn(cplx *a, int ndim, const int *shape, int sign) {
  for (int ax = 0; ax < ndim; ax++) fft_axis(a, ndim, shape, ax, sign);
}

static int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}

/* R2C: complex FFT of the real field over all axes, scaled by 1/N^d, then
 * keep kx in [0, N/2].  phys: N^d reals (C order, x last);
 * spec: N^{d-1} x (N/2+1). */
void or_rfftn(int ndim, int n, const double *phys, cplx *spec) {
  int shape[3] = {n, n, n};
  int64_t tot = ipow(n, ndim), h = n / 2 + 1, rows = tot / n;
  cplx *a = malloc(sizeof(cplx) * (size_t)tot);
  for (int64_t i = 0; i < tot; i++) a[i] = phys[i];
  or_fftn(a, ndim, shape, -1);
  double s = 1.0 / (double)tot;
  for (int64_t r = 0; r < rows; r++)
    for (int64_t kx = 0; kx < h; kx++) spec[r * h + kx] = a[r * n + kx] * s;
  free(a);
}

/* C2R: rebuild the full Hermitian spectrum from the half one
 * (F(-k) = conj F(k) for kx > N/2), inverse complex FFT (unscaled), real
 * part. */
void or_irfftn(int ndim, int n, const cplx *spec, double *phys) {
  int shape[3] = {n, n, n};
  int64_t tot = ipow(n, ndim), h = n / 2 + 1, rows = tot / n;
  cplx *a = malloc(sizeof(cplx) * (size_t)tot);
  for (int64_t r = 0; r < rows; r++) {
    /* row r indexes (kz, ky) or (ky); its mirror indexes (-kz, -ky) */
    int64_t mr;
    if (ndim == 1) {
      mr = 0;
    } else if (ndim == 2) {
      mr = (n - r) % n;
    } else {
      int64_t kz = r / n, ky = r % n;
      mr = ((n - kz) % n) * n + (n - ky) % n;
    }
    for (int64_t kx = 0; kx < n; kx++) {
      if (kx < h)
        a[r * n + kx] = spec[r * h + kx];
      else
        a[r * n + kx] = conj(spec[mr * h + (n - kx)]);
    }
  }
  or_fftn(a, ndim, shape, +1);
  for (int64_t i = 0; i < tot; i++) phys[i] = creal(a[i]);
  free(a);
}

/* One forward coefficient by the direct sum, for checks at sizes where a
 * whole transform is too expensive: N^-3 sum_x u(x) exp(-i k.x), with
 * exp(-i k.x) = exp(-i kx x) exp(-i ky y) exp(-i kz z) and every factor from
 * libm.  phys: real[n][n][n] (z, y, x). */
void or_dft_mode3d(int n, const double *phys, int mx, int my, int mz, double *re, double *im) {
  cplx *ex = malloc(sizeof(cplx) * n), *ey = malloc(sizeof(cplx) * n), *ez = malloc(sizeof(cplx) * n);
  for (int j = 0; j < n; j++) {
    double a = 2.0 * M_PI * (double)j / (double)n;
    ex[j] = cos(a * mx) - I * sin(a * mx);
    ey[j] = cos(a * my) - I * sin(a * my);
    ez[j] = cos(a * mz) - I * sin(a * mz);
  }
  cplx total = 0;
  for (int z = 0; z < n; z++) {
    cplx sy = 0;
    for (int y = 0; y < n; y++) {
      const double *row = phys + ((int64_t)z * n + y) * n;
      cplx sx = 0;
      for (int x = 0; x < n; x++) sx += row[x] * ex[x];
      sy += sx * ey[y];
    }
    total += sy * ez[z];
  }
  total /= (double)n * n * n;
  *re = creal(total);
  *im = cimag(total);
  free(ex);
  free(ey);
  free(ez);
}

/* ------------------------------------------------------------------------ */
/* Wavenumbers and the dealiasing set                                        */
/* ------------------------------------------------------------------------ */
/* integer mode number of FFT index i on a full axis of length n */
static int mode_full(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }
/* 2/3 rule on one axis: keep iff 3|m| < n */
static int keep1(int m, int n) { return 3 * abs(m) < n; }

int or_kept(int m, int n) { return keep1(m, n); }

/* ------------------------------------------------------------------------ */
/* 3D tendency: N(u) = P[(u x curl u)^] on the kept set, plus band forcing.  */
/* uh: [3][n][n][n/2+1]; nh same shape (all modes written).                  */
/* alpha multiplies u_hat on modes with kf_min <= |k| <= kf_max.              */
/* ------------------------------------------------------------------------ */
void or_tendency3d(int n, double L, const cplx *uh, double alpha, double kf_min,
                   double kf_max, cplx *nh) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h, np = (int64_t)n * n * n;
  const double kb = 2.0 * M_PI / L;
  cplx *um = malloc(sizeof(cplx) * 3 * ns); /* masked input */
  cplx *wh = malloc(sizeof(cplx) * 3 * ns); /* vorticity i k x u */
  double *ur = malloc(sizeof(double) * 3 * np), *wr = malloc(sizeof(double) * 3 * np);
  double *pr = malloc(sizeof(double) * 3 * np);
  cplx *ph = malloc(sizeof(cplx) * 3 * ns);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int mz = mode_full(iz, n), my = mode_full(iy, n), mx = ix;
    int keep = keep1(mx, n) && keep1(my, n) && keep1(mz, n);
    double kx = kb * mx, ky = kb * my, kz = kb * mz;
    cplx u0 = keep ? uh[i] : 0, u1 = keep ? uh[ns + i] : 0, u2 = keep ? uh[2 * ns + i] : 0;
    um[i] = u0;
    um[ns + i] = u1;
    um[2 * ns + i] = u2;
    wh[i] = I * (ky * u2 - kz * u1);
    wh[ns + i] = I * (kz * u0 - kx * u2);
    wh[2 * ns + i] = I * (kx * u1 - ky * u0);
  }
  for (int c = 0; c < 3; c++) {
    or_irfftn(3, n, um + c * ns, ur + c * np);
    or_irfftn(3, n, wh + c * ns, wr + c * np);
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < np; i++) {
    double u0 = ur[i], u1 = ur[np + i], u2 = ur[2 * np + i];
    double w0 = wr[i], w1 = wr[np + i], w2 = wr[2 * np + i];
    pr[i] = u1 * w2 - u2 * w1;
    pr[np + i] = u2 * w0 - u0 * w2;
    pr[2 * np + i] = u0 * w1 - u1 * w0;
  }
  for (int c = 0; c < 3; c++) or_rfftn(3, n, pr + c * np, ph + c * ns);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int mz = mode_full(iz, n), my = mode_full(iy, n), mx = ix;
    int keep = keep1(mx, n) && keep1(my, n) && keep1(mz, n);
    double kx = kb * mx, ky = kb * my, kz = kb * mz;
    double k2 = kx * kx + ky * ky + kz * kz;
    cplx r0 = 0, r1 = 0, r2 = 0;
    if (keep && k2 > 0) {
      cplx p0 = ph[i], p1 = ph[ns + i], p2 = ph[2 * ns + i];
      cplx kp = (kx * p0 + ky * p1 + kz * p2) / k2;
      r0 = p0 - kx * kp;
      r1 = p1 - ky * kp;
      r2 = p2 - kz * kp;
      double km = sqrt(k2);
      if (alpha != 0.0 && km >= kf_min && km <= kf_max) {
        r0 += alpha * um[i];
        r1 += alpha * um[ns + i];
        r2 += alpha * um[2 * ns + i];
      }
    }
    nh[i] = r0;
    nh[ns + i] = r1;
    nh[2 * ns + i] = r2;
  }
  free(um);
  free(wh);
  free(ur);
  free(wr);
  free(pr);
  free(ph);
}

/* The 3D tendency (no forcing) at single modes by the direct Galerkin sum of
 * the rotational form: (u x w)^(k) = sum over kept p, q = k - p kept of
 * u_hat(p) x (i q x u_hat(q)), then the projection and the mean-mode rule.
 * u_hat at negative kx is the conjugate of the stored mode.  modes: nm
 * triples (mx >= 0, my, mz); out: nm x 3 complex values. */
static cplx u_at(int n, const cplx *uh, int c, int mx, int my, int mz) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  int conj_ = 0;
  if (mx < 0) {
    mx = -mx;
    my = -my;
    mz = -mz;
    conj_ = 1;
  }
  const int64_t q = ((int64_t)((mz + n) % n) * n + (my + n) % n) * h + mx;
  const cplx v = uh[c * ns + q];
  return conj_ ? conj(v) : v;
}

void or_tendency3d_modes(int n, double L, const cplx *uh, int nm, const int *modes, cplx *out) {
  const int K = (n - 1) / 3;
  const double kb = 2.0 * M_PI / L;
#pragma omp parallel for schedule(dynamic)
  for (int t = 0; t < nm; t++) {
    const int kx = modes[3 * t], ky = modes[3 * t + 1], kz = modes[3 * t + 2];
    cplx acc[3] = {0, 0, 0};
    for (int pz = -K; pz <= K; pz++) {
      const int qz = kz - pz;
      if (qz < -K || qz > K) continue;
      for (int py = -K; py <= K; py++) {
        const int qy = ky - py;
        if (qy < -K || qy > K) continue;
        for (int px = -K; px <= K; px++) {
          const int qx = kx - px;
          if (qx < -K || qx > K) continue;
          cplx up[3], uq[3];
          for (int c = 0; c < 3; c++) {
            up[c] = u_at(n, uh, c, px, py, pz);
            uq[c] = u_at(n, uh, c, qx, qy, qz);
          }
          const double q3[3] = {kb * qx, kb * qy, kb * qz};
          /* w(q) = i q x u(q) */
          const cplx w[3] = {I * (q3[1] * uq[2] - q3[2] * uq[1]), I * (q3[2] * uq[0] - q3[0] * uq[2]),
                             I * (q3[0] * uq[1] - q3[1] * uq[0])};
          acc[0] += up[1] * w[2] - up[2] * w[1];
          acc[1] += up[2] * w[0] - up[0] * w[2];
          acc[2] += up[0] * w[1] - up[1] * w[0];
        }
      }
    }
    const double k3[3] = {kb * kx, kb * ky, kb * kz};
    const double k2 = k3[0] * k3[0] + k3[1] * k3[1] + k3[2] * k3[2];
    const int keep = abs(kx) <= K && abs(ky) <= K && abs(kz) <= K && k2 > 0;
    const cplx kp = keep ? (k3[0] * acc[0] + k3[1] * acc[1] + k3[2] * acc[2]) / k2 : 0;
    for (int c = 0; c < 3; c++) out[3 * t + c] = keep ? acc[c] - k3[c] * kp : 0;
  }
}

/* Constant-power forcing coefficient: alpha = P / sum_band w |u_hat|^2, so
 * that the injected power sum w Re(u_hat* . alpha u_hat) equals P; 0 when
 * the band holds no energy or P == 0. */
double or_forcing_alpha3d(int n, double L, const cplx *uh, double power, double kf_min,
                          double kf_max) {
  if (power == 0.0) return 0.0;
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  const double kb = 2.0 * M_PI / L;
  double s = 0.0;
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int mz = mode_full(iz, n), my = mode_full(iy, n), mx = ix;
    if (!(keep1(mx, n) && keep1(my, n) && keep1(mz, n))) continue;
    double km = kb * sqrt((double)mx * mx + (double)my * my + (double)mz * mz);
    if (km < kf_min || km > kf_max || km == 0.0) continue;
    double w = mx == 0 ? 1.0 : 2.0;
    for (int c = 0; c < 3; c++) {
      cplx u = uh[c * ns + i];
      s += w * (creal(u) * creal(u) + cimag(u) * cimag(u));
    }
  }
  return s > 0.0 ? power / s : 0.0;
}

/* ------------------------------------------------------------------------ */
/* 2D tendency in vorticity form.  wh, nh: [n][n/2+1].                       */
/* ------------------------------------------------------------------------ */
void or_tendency2d(int n, double L, const cplx *wh, cplx *nh) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * h, np = (int64_t)n * n;
  const double kb = 2.0 * M_PI / L;
  cplx *uh = malloc(sizeof(cplx) * 3 * ns);
  double *r = malloc(sizeof(double) * 3 * np), *q = malloc(sizeof(double) * 2 * np);
  cplx *fh = malloc(sizeof(cplx) * 2 * ns);
  for (int64_t i = 0; i < ns; i++) {
    int my = mode_full((int)(i / h), n), mx = (int)(i % h);
    int keep = keep1(mx, n) && keep1(my, n);
    double kx = kb * mx, ky = kb * my, k2 = kx * kx + ky * ky;
    cplx w = keep ? wh[i] : 0;
    uh[i] = k2 > 0 ? I * ky * w / k2 : 0;        /* u =  d psi / dy */
    uh[ns + i] = k2 > 0 ? -I * kx * w / k2 : 0;  /* v = -d psi / dx */
    uh[2 * ns + i] = w;
  }
  for (int c = 0; c < 3; c++) or_irfftn(2, n, uh + c * ns, r + c * np);
  for (int64_t i = 0; i < np; i++) {
    q[i] = r[i] * r[2 * np + i];
    q[np + i] = r[np + i] * r[2 * np + i];
  }
  or_rfftn(2, n, q, fh);
  or_rfftn(2, n, q + np, fh + ns);
  for (int64_t i = 0; i < ns; i++) {
    int my = mode_full((int)(i / h), n), mx = (int)(i % h);
    int keep = keep1(mx, n) && keep1(my, n);
    double kx = kb * mx, ky = kb * my;
    nh[i] = (keep && (mx != 0 || my != 0)) ? -I * kx * fh[i] - I * ky * fh[ns + i] : 0;
  }
  free(uh);
  free(r);
  free(q);
  free(fh);
}

/* ------------------------------------------------------------------------ */
/* 2D Boussinesq (stably stratified) flow in the vertical (x, y) plane,     */
/* gravity along -y, buoyancy b, Brunt-Vaisala frequency N (N2 = N^2):       */
/*   d w / dt + u . grad w = d b / dx            (+ nu lap w)                 */
/*   d b / dt + u . grad b = -N2 v               (+ nu lap b, Prandtl 1)      */
/* with w = dv/dx - du/dy.  State [2][n][n/2+1] (w_hat, b_hat); tendency:    */
/*   N_w = -i kx (u w)^ - i ky (v w)^ + i kx b_hat                           */
/*   N_b = -i kx (u b)^ - i ky (v b)^ - N2 v_hat,  v_hat = -i kx w_hat/|k|^2  */
/* dealiased on the kept set, zero at k = 0.                                  */
/* ------------------------------------------------------------------------ */
void or_tendency2d_strat(int n, double L, double N2, const cplx *s, cplx *out) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * h, np = (int64_t)n * n;
  const double kb = 2.0 * M_PI / L;
  cplx *g = malloc(sizeof(cplx) * 4 * ns);
  double *r = malloc(sizeof(double) * 4 * np), *q = malloc(sizeof(double) * 4 * np);
  cplx *fh = malloc(sizeof(cplx) * 4 * ns);
  for (int64_t i = 0; i < ns; i++) {
    int my = mode_full((int)(i / h), n), mx = (int)(i % h);
    int keep = keep1(mx, n) && keep1(my, n);
    double kx = kb * mx, ky = kb * my, k2 = kx * kx + ky * ky;
    cplx w = keep ? s[i] : 0, b = keep ? s[ns + i] : 0;
    g[i] = k2 > 0 ? I * ky * w / k2 : 0;
    g[ns + i] = k2 > 0 ? -I * kx * w / k2 : 0;
    g[2 * ns + i] = w;
    g[3 * ns + i] = b;
  }
  for (int c = 0; c < 4; c++) or_irfftn(2, n, g + c * ns, r + c * np);
  for (int64_t i = 0; i < np; i++) {
    q[i] = r[i] * r[2 * np + i];               /* u w */
    q[np + i] = r[np + i] * r[2 * np + i];     /* v w */
    q[2 * np + i] = r[i] * r[3 * np + i];      /* u b */
    q[3 * np + i] = r[np + i] * r[3 * np + i]; /* v b */
  }
  for (int c = 0; c < 4; c++) or_rfftn(2, n, q + c * np, fh + c * ns);
  for (int64_t i = 0; i < ns; i++) {
    int my = mode_full((int)(i / h), n), mx = (int)(i % h);
    int keep = keep1(mx, n) && keep1(my, n) && (mx != 0 || my != 0);
    double kx = kb * mx, ky = kb * my;
    out[i] = keep ? -I * kx * fh[i] - I * ky * fh[ns + i] + I * kx * g[3 * ns + i] : 0;
    out[ns + i] = keep ? -I * kx * fh[2 * ns + i] - I * ky * fh[3 * ns + i] - N2 * g[ns + i] : 0;
  }
  free(g);
  free(r);
  free(q);
  free(fh);
}

/* ------------------------------------------------------------------------ */
/* Lawson integrating-factor RK4 (exact viscous factor E = exp(-nu k^2 dt)): */
/*   k1 = N(u)            k2 = N(E_h (u + dt/2 k1))                          */
/*   k3 = N(E_h u + dt/2 k2)            k4 = N(E u + dt E_h k3)              */
/*   u' = E u + dt/6 (E k1 + 2 E_h k2 + 2 E_h k3 + k4),   E_h = E^(1/2)       */
/* Modes outside the kept set are returned as zero.                          */
/* ------------------------------------------------------------------------ */
typedef void (*tend_fn)(const cplx *u, cplx *out, void *ctx);
typedef void (*hook_fn)(const cplx *u, void *ctx);

/* The Lawson combination itself, for nf modes x ncomp components with
 * per-mode factors E = exp(L dt), Eh = exp(L dt / 2).  `pre` (optional) runs
 * on u_n before the first stage of every step. */
static void lawson_rk4(int64_t nf, int ncomp, const double *E, const double *Eh, double dt,
                       cplx *u, int nsteps, tend_fn f, hook_fn pre, void *ctx) {
  const int64_t tot = nf * ncomp;
  cplx *k1 = malloc(sizeof(cplx) * tot), *k2 = malloc(sizeof(cplx) * tot);
  cplx *k3 = malloc(sizeof(cplx) * tot), *k4 = malloc(sizeof(cplx) * tot);
  cplx *v = malloc(sizeof(cplx) * tot);
  for (int s = 0; s < nsteps; s++) {
    if (pre) pre(u, ctx);
    f(u, k1, ctx);
    for (int64_t i = 0; i < tot; i++) v[i] = Eh[i % nf] * (u[i] + 0.5 * dt * k1[i]);
    f(v, k2, ctx);
    for (int64_t i = 0; i < tot; i++) v[i] = Eh[i % nf] * u[i] + 0.5 * dt * k2[i];
    f(v, k3, ctx);
    for (int64_t i = 0; i < tot; i++) v[i] = E[i % nf] * u[i] + dt * Eh[i % nf] * k3[i];
    f(v, k4, ctx);
    for (int64_t i = 0; i < tot; i++) {
      double e = E[i % nf], eh = Eh[i % nf];
      u[i] = e * u[i] + dt / 6.0 * (e * k1[i] + 2.0 * eh * k2[i] + 2.0 * eh * k3[i] + k4[i]);
    }
  }
  free(k1);
  free(k2);
  free(k3);
  free(k4);
  free(v);
}

/* Lawson integrating-factor RK2 (the exponential midpoint rule):
 * v = Eh (u + dt/2 N(u)),  u <- E u + dt Eh N(v). */
static void lawson_rk2(int64_t nf, int ncomp, const double *E, const double *Eh, double dt,
                       cplx *u, int nsteps, tend_fn f, hook_fn pre, void *ctx) {
  const int64_t tot = nf * ncomp;
  cplx *k1 = malloc(sizeof(cplx) * tot), *k2 = malloc(sizeof(cplx) * tot);
  cplx *v = malloc(sizeof(cplx) * tot);
  for (int s = 0; s < nsteps; s++) {
    if (pre) pre(u, ctx);
    f(u, k1, ctx);
    for (int64_t i = 0; i < tot; i++) v[i] = Eh[i % nf] * (u[i] + 0.5 * dt * k1[i]);
    f(v, k2, ctx);
    for (int64_t i = 0; i < tot; i++) u[i] = E[i % nf] * u[i] + dt * Eh[i % nf] * k2[i];
  }
  free(k1);
  free(k2);
  free(v);
}

/* factor exp(-nu |k|^2 t) of element i of one field; 0 outside kept set */
static double decay(int ndim, int n, double L, double nu, double t, int64_t i) {
  const int64_t h = n / 2 + 1;
  const double kb = 2.0 * M_PI / L;
  int mx = (int)(i % h), my, mz = 0;
  if (ndim == 2) {
    my = mode_full((int)(i / h), n);
  } else {
    my = mode_full((int)((i / h) % n), n);
    mz = mode_full((int)(i / (n * h)), n);
  }
  if (!(keep1(mx, n) && keep1(my, n) && keep1(mz, n))) return 0.0;
  double k2 = kb * kb * ((double)mx * mx + (double)my * my + (double)mz * mz);
  return exp(-nu * k2 * t);
}

struct grid_ctx {
  int n;
  double L, alpha, power, kf_min, kf_max;
};

static void tend3(const cplx *u, cplx *out, void *ctx) {
  struct grid_ctx *c = ctx;
  or_tendency3d(c->n, c->L, u, c->alpha, c->kf_min, c->kf_max, out);
}

/* constant-power forcing: alpha from u_n, frozen for the whole step */
static void alpha3(const cplx *u, void *ctx) {
  struct grid_ctx *c = ctx;
  c->alpha = or_forcing_alpha3d(c->n, c->L, u, c->power, c->kf_min, c->kf_max);
}

static void tend2(const cplx *u, cplx *out, void *ctx) {
  struct grid_ctx *c = ctx;
  or_tendency2d(c->n, c->L, u, out);
}

static void grid_steps(int ndim, int n, double L, double nu, double dt, cplx *u, int nsteps,
                       struct grid_ctx *c) {
  const int64_t h = n / 2 + 1, nf = (ndim == 2 ? (int64_t)n * h : (int64_t)n * n * h);
  double *E = malloc(sizeof(double) * nf), *Eh = malloc(sizeof(double) * nf);
  for (int64_t i = 0; i < nf; i++) {
    E[i] = decay(ndim, n, L, nu, dt, i);
    Eh[i] = decay(ndim, n, L, nu, 0.5 * dt, i);
  }
  if (ndim == 3)
    lawson_rk4(nf, 3, E, Eh, dt, u, nsteps, tend3, alpha3, c);
  else
    lawson_rk4(nf, 1, E, Eh, dt, u, nsteps, tend2, NULL, c);
  free(E);
  free(Eh);
}

void or_step3d(int n, double L, double nu, double dt, double power, double kf_min,
               double kf_max, cplx *uh, int nsteps) {
  struct grid_ctx c = {n, L, 0.0, power, kf_min, kf_max};
  grid_steps(3, n, L, nu, dt, uh, nsteps, &c);
}

struct strat_ctx {
  int n;
  double L, N2;
};

static void tend2s(const cplx *u, cplx *out, void *ctx) {
  struct strat_ctx *c = ctx;
  or_tendency2d_strat(c->n, c->L, c->N2, u, out);
}

/* Lawson RK4 of the 2D Boussinesq system (both fields decay with nu). */
void or_step2d_strat(int n, double L, double nu, double dt, double N2, cplx *s, int nsteps) {
  struct strat_ctx c = {n, L, N2};
  const int64_t nf = (int64_t)n * (n / 2 + 1);
  double *E = malloc(sizeof(double) * nf), *Eh = malloc(sizeof(double) * nf);
  for (int64_t i = 0; i < nf; i++) {
    E[i] = decay(2, n, L, nu, dt, i);
    Eh[i] = decay(2, n, L, nu, 0.5 * dt, i);
  }
  lawson_rk4(nf, 2, E, Eh, dt, s, nsteps, tend2s, NULL, &c);
  free(E);
  free(Eh);
}

void or_step2d(int n, double L, double nu, double dt, cplx *wh, int nsteps) {
  struct grid_ctx c = {n, L, 0.0, 0.0, 0.0, 0.0};
  grid_steps(2, n, L, nu, dt, wh, nsteps, &c);
}

/* ------------------------------------------------------------------------ */
/* The mean mode (k = 0) under the linear terms.  A periodic pressure has no */
/* mean gradient, so nothing projects the mean: with Coriolis acceleration   */
/* -f z x u the mean velocity obeys dux/dt = f uy, duy/dt = -f ux (an        */
/* inertial oscillation, uz unchanged), and with buoyancy b z and the        */
/* stratification -N2 uz the vertical mean and the mean buoyancy obey        */
/* duz/dt = b, db/dt = -N2 uz.  Exactly, over a time t:                       */
/*   ux' = cos(f t) ux + sin(f t) uy,   uy' = cos(f t) uy - sin(f t) ux,      */
/*   uz' = cos(N t) uz + S b,           b'  = cos(N t) b - N2 S uz,           */
/* with S = sin(N t) / N (t when N = 0).  Viscosity does not act at k = 0.    */
/* in/out point at the mode of the first component; components ns apart;    */
/* nc = 3 (velocity only) or 4 (velocity, buoyancy).                          */
/* ------------------------------------------------------------------------ */
static void mean_propagate(double f, double N2, double t, const cplx *in, int64_t ns, int nc,
                           cplx *out) {
  const cplx ux = in[0], uy = in[ns], uz = in[2 * ns];
  const double cf = cos(f * t), sf = sin(f * t);
  out[0] = cf * ux + sf * uy;
  out[ns] = cf * uy - sf * ux;
  if (nc == 3) {
    out[2 * ns] = uz;
    return;
  }
  const cplx b = in[3 * ns];
  const double Nb = sqrt(N2), cn = cos(Nb * t), S = Nb > 0 ? sin(Nb * t) / Nb : t;
  out[2 * ns] = cn * uz + S * b;
  out[3 * ns] = cn * b - N2 * S * uz;
}

/* ------------------------------------------------------------------------ */
/* Rotating frame (3D): Coriolis acceleration -f z x u.  On solenoidal fields */
/* its projection is -sigma khat x u with sigma = f kz / |k|, a rotation about */
/* khat, so the linear part (viscosity + rotation) has the exact propagator   */
/*   E(t) u = exp(-nu k^2 t) (cos(sigma t) u - sin(sigma t) khat x u),         */
/* applied mode by mode in the Lawson RK4 scheme in place of exp(-nu k^2 t).  */
/* ------------------------------------------------------------------------ */
static void rot_apply(int n, double L, double nu, double f, double t, const cplx *in, cplx *out) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  const double kb = 2.0 * M_PI / L;
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int m[3] = {ix, mode_full(iy, n), mode_full(iz, n)};
    const int keep = keep1(m[0], n) && keep1(m[1], n) && keep1(m[2], n);
    const double k[3] = {kb * m[0], kb * m[1], kb * m[2]};
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (!keep) {
      for (int c = 0; c < 3; c++) out[c * ns + i] = 0;
      continue;
    }
    if (k2 == 0) {
      mean_propagate(f, 0.0, t, in + i, ns, 3, out + i);
      continue;
    }
    const double kn = sqrt(k2), kh[3] = {k[0] / kn, k[1] / kn, k[2] / kn};
    const double sg = f * k[2] / kn, d = exp(-nu * k2 * t);
    const double co = cos(sg * t), si = sin(sg * t);
    const cplx u[3] = {in[i], in[ns + i], in[2 * ns + i]};
    const cplx x[3] = {kh[1] * u[2] - kh[2] * u[1], kh[2] * u[0] - kh[0] * u[2],
                       kh[0] * u[1] - kh[1] * u[0]};
    for (int c = 0; c < 3; c++) out[c * ns + i] = d * (co * u[c] - si * x[c]);
  }
}

/* Lawson RK4 (scheme 4) or RK2 (scheme 2) with an operator propagator      */
/* prop(t, in, out) = E(t) in over `tot` complex values (E = E(dt),           */
/* Eh = E(dt/2)); hook (if any) runs on u_n before the step's first stage.   */
/* With cfl > 0 each step takes dt_n = min(dt, cfl (L/n) / max|u_c|) from   */
/* the velocity (first three fields) of u_n; the elapsed time is added to   */
/* *t_out (if given).                                                         */
typedef void (*prop_fn)(double t, const cplx *in, cplx *out, void *ctx);
static double umax_state(int ndim, int n, double L, const cplx *s);

static void lawson_prop(int64_t tot, double dt_max, int scheme, cplx *uh, int nsteps,
                        tend_fn tend, hook_fn hook, prop_fn prop, void *ctx, int n, double L,
                        double cfl, double *t_out) {
  cplx *k1 = malloc(sizeof(cplx) * tot), *k2 = malloc(sizeof(cplx) * tot);
  cplx *k3 = malloc(sizeof(cplx) * tot), *k4 = malloc(sizeof(cplx) * tot);
  cplx *v = malloc(sizeof(cplx) * tot), *w = malloc(sizeof(cplx) * tot);
  cplx *acc = malloc(sizeof(cplx) * tot);
  double t_el = 0.0;
  for (int s = 0; s < nsteps; s++) {
    double dt = dt_max;
    if (cfl > 0) {
      const double um = umax_state(3, n, L, uh);
      if (um > 0) dt = fmin(dt_max, cfl * (L / n) / um);
    }
    t_el += dt;
    if (hook) hook(uh, ctx);
    tend(uh, k1, ctx);
    /* v = Eh (u + dt/2 k1) */
    for (int64_t i = 0; i < tot; i++) w[i] = uh[i] + 0.5 * dt * k1[i];
    prop(0.5 * dt, w, v, ctx);
    tend(v, k2, ctx);
    if (scheme == 2) { /* midpoint rule: u' = E u + dt Eh k2 */
      prop(0.5 * dt, k2, w, ctx);
      prop(dt, uh, v, ctx);
      for (int64_t i = 0; i < tot; i++) uh[i] = v[i] + dt * w[i];
      continue;
    }
    /* v = Eh u + dt/2 k2 */
    prop(0.5 * dt, uh, v, ctx);
    for (int64_t i = 0; i < tot; i++) v[i] += 0.5 * dt * k2[i];
    tend(v, k3, ctx);
    /* v = E u + dt Eh k3 */
    prop(0.5 * dt, k3, w, ctx);
    prop(dt, uh, v, ctx);
    for (int64_t i = 0; i < tot; i++) v[i] += dt * w[i];
    tend(v, k4, ctx);
    /* u' = E (u + dt/6 k1) + dt/3 Eh (k2 + k3) + dt/6 k4 */
    for (int64_t i = 0; i < tot; i++) w[i] = uh[i] + dt / 6.0 * k1[i];
    prop(dt, w, acc, ctx);
    for (int64_t i = 0; i < tot; i++) w[i] = k2[i] + k3[i];
    prop(0.5 * dt, w, v, ctx);
    for (int64_t i = 0; i < tot; i++) uh[i] = acc[i] + dt / 3.0 * v[i] + dt / 6.0 * k4[i];
  }
  if (t_out) *t_out += t_el;
  free(k1);
  free(k2);
  free(k3);
  free(k4);
  free(v);
  free(w);
  free(acc);
}

struct rot_ctx {
  struct grid_ctx g;
  double nu, f;
};

static void rot_prop(double t, const cplx *in, cplx *out, void *ctx) {
  struct rot_ctx *c = ctx;
  rot_apply(c->g.n, c->g.L, c->nu, c->f, t, in, out);
}
static void rot_tend(const cplx *u, cplx *out, void *ctx) { tend3(u, out, &((struct rot_ctx *)ctx)->g); }
static void rot_hook(const cplx *u, void *ctx) { alpha3(u, &((struct rot_ctx *)ctx)->g); }

void or_step3d_rot(int n, double L, double nu, double dt, double f, double power, double kf_min,
                   double kf_max, int scheme, double cfl, cplx *uh, int nsteps, double *t_out) {
  struct rot_ctx c = {{n, L, 0.0, power, kf_min, kf_max}, nu, f};
  lawson_prop(3 * (int64_t)n * n * (n / 2 + 1), dt, scheme, uh, nsteps, rot_tend, rot_hook,
              rot_prop, &c, n, L, cfl, t_out);
}

/* ------------------------------------------------------------------------ */
/* 3D Boussinesq (stably stratified) flow, gravity along -z, buoyancy b,     */
/* squared buoyancy frequency N2, Prandtl number 1:                          */
/*   du/dt = u x w - grad(p + |u|^2/2) + b z + nu lap u,   div u = 0         */
/*   db/dt + u . grad b = -N2 uz + nu lap b                                  */
/* State [4][n][n][n/2+1] = (ux, uy, uz, b) hats.  The nonlinear tendency is */
/*   N_u = P[(u x w)^] (+ band forcing),  N_b = -i k . (u b)^               */
/* (dealiased, zero at k = 0).  The linear part L(u, b) = (P[b z], -N2 uz)   */
/* has P[b z] = b q with q = z - khat khat_z; a = uz and b then oscillate    */
/* with sigma = N |k_h| / |k| (g2 = |k_h|^2 / |k|^2 = q_z):                  */
/*   a' = g2 b,  b' = -N2 a,                                                 */
/* so exp(tL)(u, b) = (u + [(c - 1) a / g2 + b S] q,  c b - N2 S a)          */
/* with c = cos(sigma t), S = sin(sigma t) / sigma (S = t at sigma = 0) and  */
/* c - 1 = -2 sin^2(sigma t / 2); with viscosity every component also decays */
/* by exp(-nu k^2 t).  This is the propagator of the Lawson scheme.          */
/* ------------------------------------------------------------------------ */
void or_strat_propagate(int n, double L, double nu, double N2, double t, const cplx *in,
                        cplx *out) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  const double kb = 2.0 * M_PI / L, Nb = sqrt(N2);
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int m[3] = {ix, mode_full(iy, n), mode_full(iz, n)};
    const int keep = keep1(m[0], n) && keep1(m[1], n) && keep1(m[2], n);
    const double k[3] = {kb * m[0], kb * m[1], kb * m[2]};
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (!keep) {
      for (int c = 0; c < 4; c++) out[c * ns + i] = 0;
      continue;
    }
    if (k2 == 0) {
      mean_propagate(0.0, N2, t, in + i, ns, 4, out + i);
      continue;
    }
    const double g2 = (k[0] * k[0] + k[1] * k[1]) / k2;
    const double q[3] = {-k[0] * k[2] / k2, -k[1] * k[2] / k2, g2};
    const double sg = Nb * sqrt(g2);
    const double cm1 = -2.0 * pow(sin(0.5 * sg * t), 2); /* cos(sg t) - 1 */
    const double S = sg > 0 ? sin(sg * t) / sg : t;
    const double d = exp(-nu * k2 * t);
    const cplx u[3] = {in[i], in[ns + i], in[2 * ns + i]}, b = in[3 * ns + i];
    const cplx coef = (g2 > 0 ? cm1 * u[2] / g2 : 0) + S * b;
    for (int c = 0; c < 3; c++) out[c * ns + i] = d * (u[c] + coef * q[c]);
    out[3 * ns + i] = d * ((1.0 + cm1) * b - N2 * S * u[2]);
  }
}

/* Rotating and stratified (frame rotating about z with Coriolis parameter f,
 * buoyancy as above).  On a solenoidal mode write u = a1 e1 + a2 e2 with
 * e1 = khat x z / g, e2 = khat x e1 (g = |k_h| / |k|; for k_h = 0, e1 = x,
 * e2 = khat x x).  Then q = z - khat khat_z = -g e2, u_z = -g a2 and
 *   a1' = sf a2,  a2' = -sf a1 - g b,  b' = N2 g a2,   sf = f khat_z;
 * in (a1, a2, b / N) this is the skew-symmetric K = [[0, sf, 0], [-sf, 0, -sN],
 * [0, sN, 0]], sN = N g, whose exponential is I + s K + c K^2 (Rodrigues),
 * s = sin(w t) / w, c = (1 - cos(w t)) / w^2, w^2 = sf^2 + sN^2.  Back in
 * (a1, a2, b), finite at N2 = 0:
 *   a1' = (1 - c sf^2) a1 + s sf a2 - c sf g b
 *   a2' = -s sf a1 + (1 - c w^2) a2 - s g b
 *   b'  = -c sf g N2 a1 + s g N2 a2 + (1 - c N2 g^2) b,
 * times exp(-nu k^2 t); the khat component of the velocity is left as it is
 * (the propagator acts on solenoidal fields). */
void or_stratrot_propagate(int n, double L, double nu, double N2, double f, double t,
                           const cplx *in, cplx *out) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  const double kb = 2.0 * M_PI / L;
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int m[3] = {ix, mode_full(iy, n), mode_full(iz, n)};
    const int keep = keep1(m[0], n) && keep1(m[1], n) && keep1(m[2], n);
    const double k[3] = {kb * m[0], kb * m[1], kb * m[2]};
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (!keep) {
      for (int c = 0; c < 4; c++) out[c * ns + i] = 0;
      continue;
    }
    if (k2 == 0) {
      mean_propagate(f, N2, t, in + i, ns, 4, out + i);
      continue;
    }
    const double kn = sqrt(k2), kh[3] = {k[0] / kn, k[1] / kn, k[2] / kn};
    const double g = sqrt(kh[0] * kh[0] + kh[1] * kh[1]);
    double e1[3], e2[3];
    if (g > 0) {
      e1[0] = kh[1] / g;
      e1[1] = -kh[0] / g;
      e1[2] = 0;
    } else {
      e1[0] = 1;
      e1[1] = 0;
      e1[2] = 0;
    }
    e2[0] = kh[1] * e1[2] - kh[2] * e1[1];
    e2[1] = kh[2] * e1[0] - kh[0] * e1[2];
    e2[2] = kh[0] * e1[1] - kh[1] * e1[0];
    const double sf = f * kh[2], w2 = sf * sf + N2 * g * g, w = sqrt(w2);
    const double sn = w > 0 ? sin(w * t) / w : t;
    const double cc = w > 0 ? 2.0 * pow(sin(0.5 * w * t), 2) / w2 : 0.5 * t * t;
    const double d = exp(-nu * k2 * t);
    const cplx u[3] = {in[i], in[ns + i], in[2 * ns + i]}, b = in[3 * ns + i];
    const cplx a0 = u[0] * kh[0] + u[1] * kh[1] + u[2] * kh[2];
    const cplx a1 = u[0] * e1[0] + u[1] * e1[1] + u[2] * e1[2];
    const cplx a2 = u[0] * e2[0] + u[1] * e2[1] + u[2] * e2[2];
    const cplx n1 = (1 - cc * sf * sf) * a1 + sn * sf * a2 - cc * sf * g * b;
    const cplx n2 = -sn * sf * a1 + (1 - cc * w2) * a2 - sn * g * b;
    const cplx nb = -cc * sf * g * N2 * a1 + sn * g * N2 * a2 + (1 - cc * N2 * g * g) * b;
    for (int c = 0; c < 3; c++) out[c * ns + i] = d * (a0 * kh[c] + n1 * e1[c] + n2 * e2[c]);
    out[3 * ns + i] = d * nb;
  }
}

void or_tendency3d_strat(int n, double L, const cplx *s, double alpha, double kf_min,
                         double kf_max, cplx *out) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h, np = (int64_t)n * n * n;
  const double kb = 2.0 * M_PI / L;
  /* velocity part: the 3D tendency of the first three fields */
  or_tendency3d(n, L, s, alpha, kf_min, kf_max, out);
  /* buoyancy: -i k . (u b)^ of the masked fields */
  cplx *g = malloc(sizeof(cplx) * 4 * ns), *fh = malloc(sizeof(cplx) * 3 * ns);
  double *r = malloc(sizeof(double) * 4 * np), *f = malloc(sizeof(double) * 3 * np);
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int keep = keep1(ix, n) && keep1(mode_full(iy, n), n) && keep1(mode_full(iz, n), n);
    for (int c = 0; c < 4; c++) g[c * ns + i] = keep ? s[c * ns + i] : 0;
  }
  for (int c = 0; c < 4; c++) or_irfftn(3, n, g + c * ns, r + c * np);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < np; i++)
    for (int c = 0; c < 3; c++) f[c * np + i] = r[c * np + i] * r[3 * np + i];
  for (int c = 0; c < 3; c++) or_rfftn(3, n, f + c * np, fh + c * ns);
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int m[3] = {ix, mode_full(iy, n), mode_full(iz, n)};
    int keep = keep1(m[0], n) && keep1(m[1], n) && keep1(m[2], n) &&
               (m[0] != 0 || m[1] != 0 || m[2] != 0);
    cplx d = 0;
    for (int c = 0; c < 3; c++) d += kb * m[c] * fh[c * ns + i];
    out[3 * ns + i] = keep ? -I * d : 0;
  }
  free(g);
  free(fh);
  free(r);
  free(f);
}

struct strat3_ctx {
  struct grid_ctx g;
  double nu, N2, f;
};

static void strat3_prop(double t, const cplx *in, cplx *out, void *ctx) {
  struct strat3_ctx *c = ctx;
  if (c->f != 0.0)
    or_stratrot_propagate(c->g.n, c->g.L, c->nu, c->N2, c->f, t, in, out);
  else
    or_strat_propagate(c->g.n, c->g.L, c->nu, c->N2, t, in, out);
}
static void strat3_tend(const cplx *u, cplx *out, void *ctx) {
  struct grid_ctx *g = &((struct strat3_ctx *)ctx)->g;
  or_tendency3d_strat(g->n, g->L, u, g->alpha, g->kf_min, g->kf_max, out);
}
static void strat3_hook(const cplx *u, void *ctx) { alpha3(u, &((struct strat3_ctx *)ctx)->g); }

/* Lawson RK4 / RK2 of the 3D Boussinesq system with the exact propagator of
 * viscosity, buoyancy force and stratification (and, with f != 0, rotation);
 * forcing acts on u only. */
void or_step3d_strat(int n, double L, double nu, double dt, double N2, double f, double power,
                     double kf_min, double kf_max, int scheme, double cfl, cplx *s, int nsteps,
                     double *t_out) {
  struct strat3_ctx c = {{n, L, 0.0, power, kf_min, kf_max}, nu, N2, f};
  lawson_prop(4 * (int64_t)n * n * (n / 2 + 1), dt, scheme, s, nsteps, strat3_tend, strat3_hook,
              strat3_prop, &c, n, L, cfl, t_out);
}

/* Largest |u_c| over the grid points and velocity components of a kept-set
 * state (3D velocity; 2D velocity from the vorticity). */
static double umax_state(int ndim, int n, double L, const cplx *s) {
  const int64_t h = n / 2 + 1, ns = ndim == 3 ? (int64_t)n * n * h : (int64_t)n * h;
  const int64_t np = ndim == 3 ? (int64_t)n * n * n : (int64_t)n * n;
  const double kb = 2.0 * M_PI / L;
  cplx *g = malloc(sizeof(cplx) * ns);
  double *phys = malloc(sizeof(double) * np);
  double m = 0.0;
  for (int c = 0; c < ndim; c++) {
    for (int64_t i = 0; i < ns; i++) {
      int mx = (int)(i % h), my, mz = 0;
      if (ndim == 3) {
        my = mode_full((int)((i / h) % n), n);
        mz = mode_full((int)(i / (n * h)), n);
      } else {
        my = mode_full((int)(i / h), n);
      }
      if (!(keep1(mx, n) && keep1(my, n) && keep1(mz, n))) {
        g[i] = 0;
        continue;
      }
      if (ndim == 3) {
        g[i] = s[c * ns + i];
      } else {
        const double kx = kb * mx, ky = kb * my, k2 = kx * kx + ky * ky;
        g[i] = k2 == 0 ? 0 : (c == 0 ? I * ky * s[i] / k2 : -I * kx * s[i] / k2);
      }
    }
    or_irfftn(ndim, n, g, phys);
    for (int64_t q = 0; q < np; q++) m = fmax(m, fabs(phys[q]));
  }
  free(g);
  free(phys);
  return m;
}

/* General stepping: scheme 4 (Lawson RK4) or 2 (Lawson RK2); with cfl > 0 the
 * step of step n is dt_n = min(dt_max, cfl (L/n) / umax(u_n)) (dt_max when
 * the velocity vanishes), else dt_max.  *t_out (nullable) += the steps. */
static void steps_ex(int ndim, int n, double L, double nu, double dt_max, int scheme, double cfl,
                     cplx *u, int nsteps, struct grid_ctx *c, double *t_out) {
  const int64_t h = n / 2 + 1, nf = ndim == 2 ? (int64_t)n * h : (int64_t)n * n * h;
  double *E = malloc(sizeof(double) * nf), *Eh = malloc(sizeof(double) * nf);
  double t = 0.0, last = -1.0;
  for (int s = 0; s < nsteps; s++) {
    double dt = dt_max;
    if (cfl > 0) {
      const double um = umax_state(ndim, n, L, u);
      if (um > 0) dt = fmin(dt_max, cfl * (L / n) / um);
    }
    if (dt != last) {
      for (int64_t i = 0; i < nf; i++) {
        E[i] = decay(ndim, n, L, nu, dt, i);
        Eh[i] = decay(ndim, n, L, nu, 0.5 * dt, i);
      }
      last = dt;
    }
    tend_fn f = ndim == 3 ? tend3 : tend2;
    hook_fn pre = ndim == 3 ? alpha3 : NULL;
    if (scheme == 2)
      lawson_rk2(nf, ndim == 3 ? 3 : 1, E, Eh, dt, u, 1, f, pre, c);
    else
      lawson_rk4(nf, ndim == 3 ? 3 : 1, E, Eh, dt, u, 1, f, pre, c);
    t += dt;
  }
  if (t_out) *t_out += t;
  free(E);
  free(Eh);
}

void or_step3d_ex(int n, double L, double nu, double dt_max, double power, double kf_min,
                  double kf_max, int scheme, double cfl, cplx *uh, int nsteps, double *t_out) {
  struct grid_ctx c = {n, L, 0.0, power, kf_min, kf_max};
  steps_ex(3, n, L, nu, dt_max, scheme, cfl, uh, nsteps, &c, t_out);
}

void or_step2d_ex(int n, double L, double nu, double dt_max, int scheme, double cfl, cplx *wh,
                  int nsteps, double *t_out) {
  struct grid_ctx c = {n, L, 0.0, 0.0, 0.0, 0.0};
  steps_ex(2, n, L, nu, dt_max, scheme, cfl, wh, nsteps, &c, t_out);
}

double or_umax(int ndim, int n, double L, const cplx *s) { return umax_state(ndim, n, L, s); }

/* The same Lawson combination on the scalar ODE y' = -lam y + y^2 (linear
 * part exact, quadratic part by RK4); used only to pin the scheme. */
static void tend_sq(const cplx *u, cplx *out, void *ctx) {
  (void)ctx;
  out[0] = u[0] * u[0];
}

double or_lawson_scalar(double lam, double y0, double dt, int nsteps) {
  double E = exp(-lam * dt), Eh = exp(-0.5 * lam * dt);
  cplx y = y0;
  lawson_rk4(1, 1, &E, &Eh, dt, &y, nsteps, tend_sq, NULL, NULL);
  return creal(y);
}

double or_lawson_scalar2(double lam, double y0, double dt, int nsteps) {
  double E = exp(-lam * dt), Eh = exp(-0.5 * lam * dt);
  cplx y = y0;
  lawson_rk2(1, 1, &E, &Eh, dt, &y, nsteps, tend_sq, NULL, NULL);
  return creal(y);
}

/* ------------------------------------------------------------------------ */
/* Diagnostics over the kept set: E = 1/2 sum w |u_hat|^2,                   */
/* Z = 1/2 sum w |w_hat|^2, shell spectrum E(s), s = floor(|m| + 1/2),       */
/* bins s >= nbins dropped from the spectrum only.                            */
/* ------------------------------------------------------------------------ */
void or_diag3d(int n, double L, const cplx *uh, int nbins, double *spec, double *E,
               double *Z) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  const double kb = 2.0 * M_PI / L;
  double e = 0, z = 0;
  for (int b = 0; b < nbins; b++) spec[b] = 0.0;
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int mz = mode_full(iz, n), my = mode_full(iy, n), mx = ix;
    if (!(keep1(mx, n) && keep1(my, n) && keep1(mz, n))) continue;
    double w = mx == 0 ? 1.0 : 2.0;
    double kx = kb * mx, ky = kb * my, kz = kb * mz;
    cplx u0 = uh[i], u1 = uh[ns + i], u2 = uh[2 * ns + i];
    double eu = 0.5 * w * (creal(u0 * conj(u0)) + creal(u1 * conj(u1)) + creal(u2 * conj(u2)));
    cplx w0 = I * (ky * u2 - kz * u1), w1 = I * (kz * u0 - kx * u2), w2 = I * (kx * u1 - ky * u0);
    double ew = 0.5 * w * (creal(w0 * conj(w0)) + creal(w1 * conj(w1)) + creal(w2 * conj(w2)));
    e += eu;
    z += ew;
    int s = (int)floor(sqrt((double)mx * mx + (double)my * my + (double)mz * mz) + 0.5);
    if (s < nbins) spec[s] += eu;
  }
  *E = e;
  *Z = z;
}

void or_diag2d(int n, double L, const cplx *wh, int nbins, double *spec, double *E, double *Z) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * h;
  const double kb = 2.0 * M_PI / L;
  double e = 0, z = 0;
  for (int b = 0; b < nbins; b++) spec[b] = 0.0;
  for (int64_t i = 0; i < ns; i++) {
    int my = mode_full((int)(i / h), n), mx = (int)(i % h);
    if (!(keep1(mx, n) && keep1(my, n))) continue;
    if (mx == 0 && my == 0) continue;
    double w = mx == 0 ? 1.0 : 2.0;
    double k2 = kb * kb * ((double)mx * mx + (double)my * my);
    double a2 = creal(wh[i] * conj(wh[i]));
    double eu = 0.5 * w * a2 / k2;
    e += eu;
    z += 0.5 * w * a2;
    int s = (int)floor(sqrt((double)mx * mx + (double)my * my) + 0.5);
    if (s < nbins) spec[s] += eu;
  }
  *E = e;
  *Z = z;
}

/* ------------------------------------------------------------------------ */
/* 1D spectra: energy of each velocity component binned by the modulus of   */
/* one wavenumber component, out[a][c][k] = 1/2 sum over kept modes with     */
/* |m_a| = k of w |u_c_hat|^2, k = 0..K (a = x, y, z; 2D: a = x, y and the   */
/* velocity u_hat = i ky w_hat/|k|^2, v_hat = -i kx w_hat/|k|^2).            */
/* ------------------------------------------------------------------------ */
void or_spectra1d3d(int n, const cplx *uh, double *out) {
  const int K = (n - 1) / 3, nb = K + 1;
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  for (int i = 0; i < 9 * nb; i++) out[i] = 0.0;
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int m[3] = {ix, mode_full(iy, n), mode_full(iz, n)};
    if (!(keep1(m[0], n) && keep1(m[1], n) && keep1(m[2], n))) continue;
    double w = ix == 0 ? 1.0 : 2.0;
    for (int c = 0; c < 3; c++) {
      const cplx u = uh[c * ns + i];
      const double e = 0.5 * w * creal(u * conj(u));
      for (int a = 0; a < 3; a++) out[(a * 3 + c) * nb + abs(m[a])] += e;
    }
  }
}

void or_spectra1d2d(int n, double L, const cplx *wh, double *out) {
  const int K = (n - 1) / 3, nb = K + 1;
  const int64_t h = n / 2 + 1, ns = (int64_t)n * h;
  const double kb = 2.0 * M_PI / L;
  for (int i = 0; i < 4 * nb; i++) out[i] = 0.0;
  for (int64_t i = 0; i < ns; i++) {
    int m[2] = {(int)(i % h), mode_full((int)(i / h), n)};
    if (!(keep1(m[0], n) && keep1(m[1], n))) continue;
    if (m[0] == 0 && m[1] == 0) continue;
    double w = m[0] == 0 ? 1.0 : 2.0;
    double kx = kb * m[0], ky = kb * m[1], k2 = kx * kx + ky * ky;
    const cplx vel[2] = {I * ky * wh[i] / k2, -I * kx * wh[i] / k2};
    for (int c = 0; c < 2; c++) {
      const double e = 0.5 * w * creal(vel[c] * conj(vel[c]));
      for (int a = 0; a < 2; a++) out[(a * 2 + c) * nb + abs(m[a])] += e;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Longitudinal structure functions of the physical velocity (the output of  */
/* velocity increments): du_a(x, r) = u_a(x + r e_a) - u_a(x) for a          */
/* separation of r grid spacings along axis a (periodic), with u the         */
/* velocity of the kept modes (2D: from the vorticity).  Averaged over every */
/* grid point and the d axes:                                                */
/*   out[j * pmax + p - 1]              = < du^p >                          */
/*   out[(nr + j) * pmax + p - 1]       = < |du|^p >,   p = 1..pmax.         */
/* ------------------------------------------------------------------------ */
void or_structure(int ndim, int n, double L, const cplx *st, int nr, const int *r, int pmax,
                  double *out) {
  const int64_t h = n / 2 + 1, ns = (ndim == 3 ? (int64_t)n : 1) * n * h;
  const int64_t np = (ndim == 3 ? (int64_t)n : 1) * n * n;
  const double kb = 2.0 * M_PI / L;
  cplx *g = malloc(sizeof(cplx) * ns);
  double *u = malloc(sizeof(double) * np);
  for (int i = 0; i < 2 * nr * pmax; i++) out[i] = 0.0;
  for (int a = 0; a < ndim; a++) {
    /* velocity component a of the kept modes */
    for (int64_t i = 0; i < ns; i++) {
      int mx = (int)(i % h), my = mode_full((int)((i / h) % n), n);
      int mz = ndim == 3 ? mode_full((int)(i / (n * h)), n) : 0;
      int keep = keep1(mx, n) && keep1(my, n) && keep1(mz, n);
      cplx v = 0;
      if (keep && ndim == 3) {
        v = st[a * ns + i];
      } else if (keep && (mx != 0 || my != 0)) {
        double kx = kb * mx, ky = kb * my, k2 = kx * kx + ky * ky;
        v = a == 0 ? I * ky * st[i] / k2 : -I * kx * st[i] / k2;
      }
      g[i] = v;
    }
    or_irfftn(ndim, n, g, u);
    /* axis a has stride n^a in the physical layout (x fastest) */
    const int64_t stride = a == 0 ? 1 : (a == 1 ? n : (int64_t)n * n);
    for (int j = 0; j < nr; j++) {
      double sp[8] = {0}, ap[8] = {0};
      for (int64_t x = 0; x < np; x++) {
        int64_t q = (x / stride) % n, q2 = (q + r[j]) % n;
        double d = u[x + (q2 - q) * stride] - u[x], dp = 1.0;
        for (int p = 0; p < pmax; p++) {
          dp *= d;
          sp[p] += dp;
          ap[p] += fabs(dp);
        }
      }
      for (int p = 0; p < pmax; p++) {
        out[j * pmax + p] += sp[p] / ((double)np * ndim);
        out[(nr + j) * pmax + p] += ap[p] / ((double)np * ndim);
      }
    }
  }
  free(g);
  free(u);
}

/* ------------------------------------------------------------------------ */
/* Spectral energy budget: with E = 1/2 sum w |u_hat|^2 and du_hat/dt = N_hat  */
/* (no viscosity), dE/dt = sum w Re(conj(u_hat) . N_hat); its shell sums are   */
/* the transfer T(s), s = floor(|m| + 1/2) (bins >= nbins dropped from T       */
/* only).  *Et = the total; *Zt = the enstrophy rate sum w Re(conj(w) . (i k x */
/* N)) in 3D.  2D: state and N are the vorticity and its tendency,             */
/* T = w Re(conj(w_hat) N_hat) / |k|^2 and *Zt = sum w Re(conj(w_hat) N_hat).  */
/* ------------------------------------------------------------------------ */
void or_transfer3d(int n, double L, const cplx *uh, const cplx *nh, int nbins, double *T,
                   double *Et, double *Zt) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h;
  const double kb = 2.0 * M_PI / L;
  double e = 0, z = 0;
  for (int b = 0; b < nbins; b++) T[b] = 0.0;
  for (int64_t i = 0; i < ns; i++) {
    int iz = (int)(i / (n * h)), iy = (int)((i / h) % n), ix = (int)(i % h);
    int mz = mode_full(iz, n), my = mode_full(iy, n), mx = ix;
    if (!(keep1(mx, n) && keep1(my, n) && keep1(mz, n))) continue;
    double w = mx == 0 ? 1.0 : 2.0;
    double k[3] = {kb * mx, kb * my, kb * mz};
    const cplx u[3] = {uh[i], uh[ns + i], uh[2 * ns + i]};
    const cplx a[3] = {nh[i], nh[ns + i], nh[2 * ns + i]};
    double te = 0;
    for (int c = 0; c < 3; c++) te += w * creal(conj(u[c]) * a[c]);
    cplx wu[3], wa[3];
    for (int c = 0; c < 3; c++) {
      const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      wu[c] = I * (k[c1] * u[c2] - k[c2] * u[c1]);
      wa[c] = I * (k[c1] * a[c2] - k[c2] * a[c1]);
    }
    double tz = 0;
    for (int c = 0; c < 3; c++) tz += w * creal(conj(wu[c]) * wa[c]);
    e += te;
    z += tz;
    int s = (int)floor(sqrt((double)mx * mx + (double)my * my + (double)mz * mz) + 0.5);
    if (s < nbins) T[s] += te;
  }
  *Et = e;
  *Zt = z;
}

void or_transfer2d(int n, double L, const cplx *wh, const cplx *nh, int nbins, double *T,
                   double *Et, double *Zt) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * h;
  const double kb = 2.0 * M_PI / L;
  double e = 0, z = 0;
  for (int b = 0; b < nbins; b++) T[b] = 0.0;
  for (int64_t i = 0; i < ns; i++) {
    int my = mode_full((int)(i / h), n), mx = (int)(i % h);
    if (!(keep1(mx, n) && keep1(my, n))) continue;
    if (mx == 0 && my == 0) continue;
    double w = mx == 0 ? 1.0 : 2.0;
    double k2 = kb * kb * ((double)mx * mx + (double)my * my);
    double tz = w * creal(conj(wh[i]) * nh[i]);
    e += tz / k2;
    z += tz;
    int s = (int)floor(sqrt((double)mx * mx + (double)my * my) + 0.5);
    if (s < nbins) T[s] += tz / k2;
  }
  *Et = e;
  *Zt = z;
}

/* ======================================================================== */
/* Learned-closure building blocks (filtered DNS -> coarse LES).              */
/* A coarse grid nc keeps |m_a| <= Kc = floor((nc-1)/3): exactly its own      */
/* dealiased set, so the sharp cube cutoff of a fine field is the coarse      */
/* state.  Stress components are ordered xx, yy, zz, xy, xz, yz.              */
/* ======================================================================== */
static const int TAU_I[6] = {0, 1, 2, 0, 0, 1}, TAU_J[6] = {0, 1, 2, 1, 2, 2};

/* sharp cube cutoff: coarse(m) = fine(m) for |m_a| <= Kc, else 0.
 * fine: [nf][nf][nf/2+1] (one field), coarse: [nc][nc][nc/2+1]. */
/* With box != 0 the kept modes are first multiplied by the transfer function
 * of the box (top-hat) filter of width D = L / (2 Kc) along each axis: the
 * average of e^{i k x} over [x - D/2, x + D/2] is e^{i k x} sin(k D/2) / (k D/2),
 * with k D / 2 = pi m / (2 Kc) for integer mode m. */
static double box_gain(int m, int Kc) {
  if (m == 0) return 1.0;
  const double x = M_PI * m / (2.0 * Kc);
  return sin(x) / x;
}

void or_cutoff3d(int nf, const cplx *fine, int nc, int box, cplx *coarse) {
  const int Kc = (nc - 1) / 3;
  const int64_t hf = nf / 2 + 1, hc = nc / 2 + 1;
  for (int iz = 0; iz < nc; iz++)
    for (int iy = 0; iy < nc; iy++)
      for (int ix = 0; ix < hc; ix++) {
        const int mz = mode_full(iz, nc), my = mode_full(iy, nc), mx = ix;
        cplx v = 0;
        if (abs(mz) <= Kc && abs(my) <= Kc && mx <= Kc) {
          const int fz = (mz + nf) % nf, fy = (my + nf) % nf;
          v = fine[((int64_t)fz * nf + fy) * hf + mx];
          if (box) v *= box_gain(mx, Kc) * box_gain(my, Kc) * box_gain(mz, Kc);
        }
        coarse[((int64_t)iz * nc + iy) * hc + ix] = v;
      }
}

/* A[3i+j] = d u_i / d x_j on the n^3 grid, from the spectral velocity u
 * [3][n][n][n/2+1] (modes outside the kept cube ignored): C2R of i k_j u_i. */
void or_grad3d(int n, double L, const cplx *u, double *A) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h, np = (int64_t)n * n * n;
  const double kb = 2.0 * M_PI / L;
  cplx *g = malloc(sizeof(cplx) * ns);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      for (int64_t q = 0; q < ns; q++) {
        int iz = (int)(q / (n * h)), iy = (int)((q / h) % n), ix = (int)(q % h);
        int m[3] = {ix, mode_full(iy, n), mode_full(iz, n)};
        int keep = keep1(m[0], n) && keep1(m[1], n) && keep1(m[2], n);
        g[q] = keep ? I * kb * m[j] * u[i * ns + q] : 0;
      }
      or_irfftn(3, n, g, A + (3 * i + j) * np);
    }
  free(g);
}

/* Subgrid stress on the coarse grid from a fine spectral velocity:
 * tau_ij = cutoff(u_i u_j) - ubar_i ubar_j at the coarse points, with the
 * fine product formed on the fine grid; the trace is then removed.  With box
 * the filter is the box filter followed by the cutoff (ubar included). */
void or_sgs_tau3d(int nf, const cplx *uf, int nc, int box, double *tau) {
  const int64_t hf = nf / 2 + 1, nsf = (int64_t)nf * nf * hf, npf = (int64_t)nf * nf * nf;
  const int64_t hc = nc / 2 + 1, nsc = (int64_t)nc * nc * hc, npc = (int64_t)nc * nc * nc;
  double *uphys = malloc(sizeof(double) * 3 * npf), *prod = malloc(sizeof(double) * npf);
  cplx *pf = malloc(sizeof(cplx) * nsf), *pc = malloc(sizeof(cplx) * nsc);
  double *ub = malloc(sizeof(double) * 3 * npc);
  for (int c = 0; c < 3; c++) {
    /* fine physical velocity (masked to the fine kept set) */
    cplx *tmp = malloc(sizeof(cplx) * nsf);
    for (int64_t q = 0; q < nsf; q++) {
      int iz = (int)(q / (nf * hf)), iy = (int)((q / hf) % nf), ix = (int)(q % hf);
      int keep = keep1(ix, nf) && keep1(mode_full(iy, nf), nf) && keep1(mode_full(iz, nf), nf);
      tmp[q] = keep ? uf[c * nsf + q] : 0;
    }
    or_irfftn(3, nf, tmp, uphys + c * npf);
    or_cutoff3d(nf, tmp, nc, box, pc);
    or_irfftn(3, nc, pc, ub + c * npc);
    free(tmp);
  }
  for (int s = 0; s < 6; s++) {
    const int i = TAU_I[s], j = TAU_J[s];
    for (int64_t q = 0; q < npf; q++) prod[q] = uphys[i * npf + q] * uphys[j * npf + q];
    or_rfftn(3, nf, prod, pf);
    or_cutoff3d(nf, pf, nc, box, pc);
    or_irfftn(3, nc, pc, tau + s * npc);
    for (int64_t q = 0; q < npc; q++) tau[s * npc + q] -= ub[i * npc + q] * ub[j * npc + q];
  }
  for (int64_t q = 0; q < npc; q++) {
    const double tr = (tau[q] + tau[npc + q] + tau[2 * npc + q]) / 3.0;
    for (int s = 0; s < 3; s++) tau[s * npc + q] -= tr;
  }
  free(uphys);
  free(prod);
  free(pf);
  free(pc);
  free(ub);
}

/* ---- MLP 9 -> 64 -> 64 -> 6 with GELU(x) = x Phi(x) (exact, erf) -------- */
/* params: W1[64][9] b1[64] W2[64][64] b2[64] W3[6][64] b3[6] (5190 values)  */
enum { MI = 9, MH = 64, MO = 6 };
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MH * MI)
#define OFF_W2 (OFF_B1 + MH)
#define OFF_B2 (OFF_W2 + MH * MH)
#define OFF_W3 (OFF_B2 + MH)
#define OFF_B3 (OFF_W3 + MO * MH)
#define NPARAM (OFF_B3 + MO)

int or_mlp_nparams(void) { return NPARAM; }

static double gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }
static double gelu_d(double x) {
  return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * exp(-0.5 * x * x) / sqrt(2.0 * M_PI);
}

/* one point: pre-activations z1, z2, activations h1, h2, output y */
static void mlp_point(const double *p, const double *x, double *z1, double *h1, double *z2,
                      double *h2, double *y) {
  for (int o = 0; o < MH; o++) {
    double s = p[OFF_B1 + o];
    for (int k = 0; k < MI; k++) s += p[OFF_W1 + o * MI + k] * x[k];
    z1[o] = s;
    h1[o] = gelu(s);
  }
  for (int o = 0; o < MH; o++) {
    double s = p[OFF_B2 + o];
    for (int k = 0; k < MH; k++) s += p[OFF_W2 + o * MH + k] * h1[k];
    z2[o] = s;
    h2[o] = gelu(s);
  }
  for (int o = 0; o < MO; o++) {
    double s = p[OFF_B3 + o];
    for (int k = 0; k < MH; k++) s += p[OFF_W3 + o * MH + k] * h2[k];
    y[o] = s;
  }
}

void or_mlp_forward(const double *p, const double *x, int64_t P, double *y) {
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < P; q++) {
    double z1[MH], h1[MH], z2[MH], h2[MH];
    mlp_point(p, x + q * MI, z1, h1, z2, h2, y + q * MO);
  }
}

/* mean squared error over all P*6 outputs and its gradient (back propagation) */
double or_mlp_loss_grad(const double *p, const double *x, const double *t, int64_t P,
                        double *grad) {
  for (int i = 0; i < NPARAM; i++) grad[i] = 0.0;
  double loss = 0.0;
  const double scale = 1.0 / ((double)P * MO);
  for (int64_t q = 0; q < P; q++) {
    double z1[MH], h1[MH], z2[MH], h2[MH], y[MO], dy[MO], dz2[MH], dz1[MH];
    mlp_point(p, x + q * MI, z1, h1, z2, h2, y);
    for (int o = 0; o < MO; o++) {
      const double d = y[o] - t[q * MO + o];
      loss += d * d * scale;
      dy[o] = 2.0 * d * scale;
      grad[OFF_B3 + o] += dy[o];
      for (int k = 0; k < MH; k++) grad[OFF_W3 + o * MH + k] += dy[o] * h2[k];
    }
    for (int k = 0; k < MH; k++) {
      double s = 0.0;
      for (int o = 0; o < MO; o++) s += p[OFF_W3 + o * MH + k] * dy[o];
      dz2[k] = s * gelu_d(z2[k]);
      grad[OFF_B2 + k] += dz2[k];
      for (int m = 0; m < MH; m++) grad[OFF_W2 + k * MH + m] += dz2[k] * h1[m];
    }
    for (int k = 0; k < MH; k++) {
      double s = 0.0;
      for (int o = 0; o < MH; o++) s += p[OFF_W2 + o * MH + k] * dz2[o];
      dz1[k] = s * gelu_d(z1[k]);
      grad[OFF_B1 + k] += dz1[k];
      for (int m = 0; m < MI; m++) grad[OFF_W1 + k * MI + m] += dz1[k] * x[q * MI + m];
    }
  }
  return loss;
}

/* Adam (Kingma & Ba): step counts from 1 */
void or_adam(double *w, double *m, double *v, const double *g, int n, int step, double lr,
             double b1, double b2, double eps) {
  const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int i = 0; i < n; i++) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}

/* P[-i k_j tau_ij^] added to nh on the kept set, k != 0 (tau physical,
 * [6][n^3], xx, yy, zz, xy, xz, yz order) */
static void add_sgs(int n, double L, const double *tau, cplx *nh) {
  const int64_t h = n / 2 + 1, ns = (int64_t)n * n * h, np = (int64_t)n * n * n;
  const double kb = 2.0 * M_PI / L;
  cplx *th = malloc(sizeof(cplx) * 6 * ns);
  for (int s = 0; s < 6; s++) or_rfftn(3, n, tau + s * np, th + s * ns);
  for (int64_t q = 0; q < ns; q++) {
    int iz = (int)(q / (n * h)), iy = (int)((q / h) % n), ix = (int)(q % h);
    int m[3] = {ix, mode_full(iy, n), mode_full(iz, n)};
    if (!(keep1(m[0], n) && keep1(m[1], n) && keep1(m[2], n))) continue;
    double k[3] = {kb * m[0], kb * m[1], kb * m[2]};
    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (k2 == 0) continue;
    cplx s[3] = {0, 0, 0};
    for (int c = 0; c < 6; c++) {
      const int i = TAU_I[c], j = TAU_J[c];
      s[i] += -I * k[j] * th[c * ns + q];
      if (i != j) s[j] += -I * k[i] * th[c * ns + q];
    }
    cplx ks = (k[0] * s[0] + k[1] * s[1] + k[2] * s[2]) / k2;
    for (int c = 0; c < 3; c++) nh[c * ns + q] += s[c] - k[c] * ks;
  }
  free(th);
}

/* LES tendency with a given physical stress: N = P[(u x w)^ - i k_j tau_ij^],
 * tau: [6][n^3] in xx, yy, zz, xy, xz, yz order. */
void or_tendency3d_les(int n, double L, const cplx *uh, const double *tau, cplx *nh) {
  or_tendency3d(n, L, uh, 0.0, 0.0, 0.0, nh);
  add_sgs(n, L, tau, nh);
}

/* Round to the nearest BF16 value (8 significant bits), ties to even; the
 * closure stores its features in this format.  Normal range only. */
double or_round_bf16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  const double f = frexp(x, &e); /* x = f 2^e, 0.5 <= |f| < 1 */
  return ldexp(nearbyint(ldexp(f, 8)), e - 8);
}

void or_round_bf16_array(double *x, int64_t n) {
  for (int64_t i = 0; i < n; i++) x[i] = or_round_bf16(x[i]);
}

/* The network's stress for a coarse spectral velocity: features
 * x_k = A_k / a_scale (A = or_grad3d, optionally rounded to BF16), outputs
 * y = MLP(x), tau_s = clip(y_s) tau_scale[s] (clip <= 0: none). */
struct les_net {
  const double *params, *tau_scale;
  double a_scale, clip;
  int round_bf16;
};

static void les_tau(int n, double L, const cplx *uh, const struct les_net *net, double *tau) {
  const int64_t np = (int64_t)n * n * n;
  double *A = malloc(sizeof(double) * 9 * np), *x = malloc(sizeof(double) * MI * np);
  double *y = malloc(sizeof(double) * MO * np);
  or_grad3d(n, L, uh, A);
  for (int64_t q = 0; q < np; q++)
    for (int k = 0; k < MI; k++) {
      const double v = A[k * np + q] / net->a_scale;
      x[q * MI + k] = net->round_bf16 ? or_round_bf16(v) : v;
    }
  or_mlp_forward(net->params, x, np, y);
  for (int64_t q = 0; q < np; q++)
    for (int s = 0; s < MO; s++) {
      double v = y[q * MO + s];
      if (net->clip > 0) v = fmin(fmax(v, -net->clip), net->clip);
      tau[s * np + q] = v * net->tau_scale[s];
    }
  free(A);
  free(x);
  free(y);
}

void or_les_tau3d(int n, double L, const cplx *uh, const double *params, double a_scale,
                  const double *tau_scale, double clip, int round_bf16, double *tau) {
  struct les_net net = {params, tau_scale, a_scale, clip, round_bf16};
  les_tau(n, L, uh, &net, tau);
}

/* LES nonlinear term with the network closure: the resolved tendency
 * (forcing coefficient alpha on the band) plus P[-i k_j tau_ij^]. */
void or_les_tendency3d(int n, double L, const cplx *uh, double alpha, double kf_min,
                       double kf_max, const double *params, double a_scale,
                       const double *tau_scale, double clip, int round_bf16, cplx *nh) {
  const int64_t np = (int64_t)n * n * n;
  struct les_net net = {params, tau_scale, a_scale, clip, round_bf16};
  double *tau = malloc(sizeof(double) * 6 * np);
  les_tau(n, L, uh, &net, tau);
  or_tendency3d(n, L, uh, alpha, kf_min, kf_max, nh);
  add_sgs(n, L, tau, nh);
  free(tau);
}

struct les_ctx {
  struct grid_ctx g;
  struct les_net net;
};

static void tend_les(const cplx *u, cplx *out, void *ctx) {
  struct les_ctx *c = ctx;
  or_les_tendency3d(c->g.n, c->g.L, u, c->g.alpha, c->g.kf_min, c->g.kf_max, c->net.params,
                    c->net.a_scale, c->net.tau_scale, c->net.clip, c->net.round_bf16, out);
}

static void alpha_les(const cplx *u, void *ctx) { alpha3(u, &((struct les_ctx *)ctx)->g); }

/* LES steps: the Lawson RK4 scheme of or_step3d with the closure term. */
void or_step3d_les(int n, double L, double nu, double dt, double power, double kf_min,
                   double kf_max, const double *params, double a_scale, const double *tau_scale,
                   double clip, int round_bf16, cplx *uh, int nsteps) {
  struct les_ctx c = {{n, L, 0.0, power, kf_min, kf_max},
                      {params, tau_scale, a_scale, clip, round_bf16}};
  const int64_t nf = (int64_t)n * n * (n / 2 + 1);
  double *E = malloc(sizeof(double) * nf), *Eh = malloc(sizeof(double) * nf);
  for (int64_t i = 0; i < nf; i++) {
    E[i] = decay(3, n, L, nu, dt, i);
    Eh[i] = decay(3, n, L, nu, 0.5 * dt, i);
  }
  lawson_rk4(nf, 3, E, Eh, dt, uh, nsteps, tend_les, alpha_les, &c);
  free(E);
  free(Eh);
}
