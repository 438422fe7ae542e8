/* Sanitizer driver for the FP64 reference (test infrastructure): calls every
 * entry point of oracle/fs_oracle.c on small inputs, built together with it
 * under AddressSanitizer and UndefinedBehaviorSanitizer.  Values are not
 * checked here (the Python pins do that); any out-of-bounds access, leak or
 * undefined operation aborts the run with a report. */
#include <complex.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

void or_set_threads(int n);
void or_fft1d(cplx *x, int n, int sign);
void or_fftn(cplx *a, int ndim, const int *shape, int sign);
void or_rfftn(int ndim, int n, const double *phys, cplx *spec);
void or_irfftn(int ndim, int n, const cplx *spec, double *phys);
void or_dft_mode3d(int n, const double *phys, int mx, int my, int mz, double *re, double *im);
void or_tendency3d(int n, double L, const cplx *uh, double alpha, double kf_min, double kf_max,
                   cplx *nh);
void or_tendency3d_modes(int n, double L, const cplx *uh, int nm, const int *modes, cplx *out);
double or_forcing_alpha3d(int n, double L, const cplx *uh, double power, double kf_min,
                          double kf_max);
void or_tendency2d(int n, double L, const cplx *wh, cplx *nh);
void or_tendency2d_strat(int n, double L, double N2, const cplx *s, cplx *out);
void or_step3d(int n, double L, double nu, double dt, double power, double kf_min, double kf_max,
               cplx *uh, int nsteps);
void or_step2d_strat(int n, double L, double nu, double dt, double N2, cplx *s, int nsteps);
void or_step2d(int n, double L, double nu, double dt, cplx *wh, int nsteps);
void or_step3d_rot(int n, double L, double nu, double dt, double f, double power, double kf_min,
                   double kf_max, int scheme, double cfl, cplx *uh, int nsteps, double *t_out);
void or_strat_propagate(int n, double L, double nu, double N2, double t, const cplx *in,
                        cplx *out);
void or_stratrot_propagate(int n, double L, double nu, double N2, double f, double t,
                           const cplx *in, cplx *out);
void or_tendency3d_strat(int n, double L, const cplx *s, double alpha, double kf_min,
                         double kf_max, cplx *out);
void or_step3d_strat(int n, double L, double nu, double dt, double N2, double f, double power,
                     double kf_min, double kf_max, int scheme, double cfl, cplx *s, int nsteps,
                     double *t_out);
void or_step3d_ex(int n, double L, double nu, double dt_max, double power, double kf_min,
                  double kf_max, int scheme, double cfl, cplx *uh, int nsteps, double *t_out);
void or_step2d_ex(int n, double L, double nu, double dt_max, int scheme, double cfl, cplx *wh,
                  int nsteps, double *t_out);
double or_umax(int ndim, int n, double L, const cplx *s);
double or_lawson_scalar(double lam, double y0, double dt, int nsteps);
double or_lawson_scalar2(double lam, double y0, double dt, int nsteps);
void or_diag3d(int n, double L, const cplx *uh, int nbins, double *spec, double *E, double *Z);
void or_diag2d(int n, double L, const cplx *wh, int nbins, double *spec, double *E, double *Z);
void or_spectra1d3d(int n, const cplx *uh, double *out);
void or_spectra1d2d(int n, double L, const cplx *wh, double *out);
void or_structure(int ndim, int n, double L, const cplx *st, int nr, const int *r, int pmax,
                  double *out);
void or_transfer3d(int n, double L, const cplx *uh, const cplx *nh, int nbins, double *T,
                   double *Et, double *Zt);
void or_transfer2d(int n, double L, const cplx *wh, const cplx *nh, int nbins, double *T,
                   double *Et, double *Zt);
void or_cutoff3d(int nf, const cplx *fine, int nc, int box, cplx *coarse);
void or_grad3d(int n, double L, const cplx *u, double *A);
void or_sgs_tau3d(int nf, const cplx *uf, int nc, int box, double *tau);
int or_mlp_nparams(void);
void or_mlp_forward(const double *p, const double *x, int64_t P, double *y);
double or_mlp_loss_grad(const double *p, const double *x, const double *t, int64_t P,
                        double *grad);
void or_adam(double *w, double *m, double *v, const double *g, int n, int step, double lr,
             double b1, double b2, double eps);
void or_tendency3d_les(int n, double L, const cplx *uh, const double *tau, cplx *nh);
double or_round_bf16(double x);
void or_round_bf16_array(double *x, int64_t n);
void or_les_tau3d(int n, double L, const cplx *uh, const double *params, double a_scale,
                  const double *tau_scale, double clip, int round_bf16, double *tau);
void or_les_tendency3d(int n, double L, const cplx *uh, double alpha, double kf_min,
                       double kf_max, const double *params, double a_scale,
                       const double *tau_scale, double clip, int round_bf16, cplx *nh);
void or_step3d_les(int n, double L, double nu, double dt, double power, double kf_min,
                   double kf_max, const double *params, double a_scale, const double *tau_scale,
                   double clip, int round_bf16, cplx *uh, int nsteps);

static uint64_t state = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in [-0.5, 0.5) */
  state ^= state << 13;
  state ^= state >> 7;
  state ^= state << 17;
  return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}
static void *alloc(size_t n, size_t sz) {
  void *p = calloc(n, sz);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return p;
}
static cplx *rnd_c(size_t n) {
  cplx *a = alloc(n, sizeof(cplx));
  for (size_t i = 0; i < n; i++) a[i] = 0.1 * urand() + 0.1 * I * urand();
  return a;
}
static double *rnd_d(size_t n, double s) {
  double *a = alloc(n, sizeof(double));
  for (size_t i = 0; i < n; i++) a[i] = s * urand();
  return a;
}

int main(void) {
  const double L = 6.283185307179586;
  or_set_threads(2);
  /* transforms */
  {
    cplx *x = rnd_c(16);
    or_fft1d(x, 16, -1);
    int shape[3] = {4, 4, 8};
    cplx *a = rnd_c(128);
    or_fftn(a, 3, shape, +1);
    double *ph = rnd_d(512, 1.0), re, im;
    cplx *sp = alloc(8 * 8 * 5, sizeof(cplx));
    or_rfftn(3, 8, ph, sp);
    or_irfftn(3, 8, sp, ph);
    or_dft_mode3d(8, ph, 1, -2, 3, &re, &im);
    free(x), free(a), free(ph), free(sp);
  }
  /* 3D solvers at n = 16 */
  const int n = 16, h = n / 2 + 1;
  const size_t ns = (size_t)n * n * h, np = (size_t)n * n * n;
  {
    cplx *u = rnd_c(3 * ns), *nh = alloc(3 * ns, sizeof(cplx));
    double t = 0, spec[32], E, Z, T[32], Et, Zt, sf[2 * 3 * 4];
    int modes[6] = {1, 0, 0, 2, -3, 4}, r[3] = {1, 3, 8};
    or_tendency3d(n, L, u, or_forcing_alpha3d(n, L, u, 0.1, 2.0, 3.0), 2.0, 3.0, nh);
    or_tendency3d_modes(n, L, u, 2, modes, nh);
    or_transfer3d(n, L, u, nh, 32, T, &Et, &Zt);
    or_step3d(n, L, 1e-2, 1e-3, 0.1, 2.0, 3.0, u, 2);
    or_step3d_ex(n, L, 1e-2, 1e-3, 0.1, 2.0, 3.0, 2, 0.5, u, 2, &t);
    or_step3d_rot(n, L, 1e-2, 1e-3, 2.0, 0.1, 2.0, 3.0, 4, 0.5, u, 2, &t);
    or_diag3d(n, L, u, 32, spec, &E, &Z);
    double *s1 = alloc(3 * 3 * (n / 3 + 1), sizeof(double));
    or_spectra1d3d(n, u, s1);
    or_structure(3, n, L, u, 3, r, 4, sf);
    (void)or_umax(3, n, L, u);
    free(s1), free(u), free(nh);
  }
  {
    cplx *s = rnd_c(4 * ns), *out = alloc(4 * ns, sizeof(cplx));
    double t = 0;
    or_strat_propagate(n, L, 1e-2, 4.0, 0.1, s, out);
    or_stratrot_propagate(n, L, 1e-2, 4.0, 2.0, 0.1, s, out);
    or_tendency3d_strat(n, L, s, 0.0, 2.0, 3.0, out);
    or_step3d_strat(n, L, 1e-2, 1e-3, 4.0, 2.0, 0.1, 2.0, 3.0, 4, 0.5, s, 2, &t);
    or_step3d_strat(n, L, 1e-2, 1e-3, 4.0, 0.0, 0.1, 2.0, 3.0, 2, 0.0, s, 1, &t);
    free(s), free(out);
  }
  /* 2D solvers */
  {
    const int m = 32;
    const size_t ms = (size_t)m * (m / 2 + 1);
    cplx *w = rnd_c(2 * ms), *o = alloc(2 * ms, sizeof(cplx));
    double t = 0, spec[32], E, Z, T[32], Et, Zt, sf[2 * 2 * 3];
    int r[2] = {1, 5};
    or_tendency2d(m, L, w, o);
    or_transfer2d(m, L, w, o, 32, T, &Et, &Zt);
    or_step2d(m, L, 1e-3, 1e-3, w, 2);
    or_step2d_ex(m, L, 1e-3, 1e-3, 4, 0.5, w, 2, &t);
    or_diag2d(m, L, w, 32, spec, &E, &Z);
    double *s1 = alloc(2 * 2 * (m / 3 + 1), sizeof(double));
    or_spectra1d2d(m, L, w, s1);
    or_structure(2, m, L, w, 2, r, 3, sf);
    or_tendency2d_strat(m, L, 2.0, w, o);
    or_step2d_strat(m, L, 1e-3, 1e-3, 2.0, w, 2);
    free(s1), free(w), free(o);
  }
  (void)or_lawson_scalar(1.0, 0.5, 0.1, 4);
  (void)or_lawson_scalar2(1.0, 0.5, 0.1, 4);
  /* closure: cutoff 16 -> 8, gradients, stress, network, LES */
  {
    const int nc = 8, hc = nc / 2 + 1;
    const size_t nsc = (size_t)nc * nc * hc, npc = (size_t)nc * nc * nc;
    cplx *uf = rnd_c(3 * ns), *uc = alloc(3 * nsc, sizeof(cplx)), *nh = alloc(3 * nsc, sizeof(cplx));
    double *A = alloc(9 * npc, sizeof(double)), *tau = alloc(6 * npc, sizeof(double));
    or_cutoff3d(n, uf, nc, 0, uc);
    or_cutoff3d(n, uf, nc, 1, uc);
    or_grad3d(nc, L, uc, A);
    or_sgs_tau3d(n, uf, nc, 0, tau);
    or_sgs_tau3d(n, uf, nc, 1, tau);
    or_tendency3d_les(nc, L, uc, tau, nh);
    const int np_ = or_mlp_nparams();
    const int64_t P = 40;
    double *p = rnd_d(np_, 0.3), *g = alloc(np_, sizeof(double)), *m = alloc(np_, sizeof(double));
    double *v = alloc(np_, sizeof(double)), *x = rnd_d(9 * P, 1.0), *y = alloc(6 * P, sizeof(double));
    double *tg = rnd_d(6 * P, 1.0), ts[6] = {1, 1, 1, 1, 1, 1};
    or_mlp_forward(p, x, P, y);
    (void)or_mlp_loss_grad(p, x, tg, P, g);
    or_adam(p, m, v, g, np_, 1, 1e-3, 0.9, 0.999, 1e-8);
    (void)or_round_bf16(0.3);
    or_round_bf16_array(x, 9 * P);
    or_les_tau3d(nc, L, uc, p, 1.0, ts, 6.0, 1, tau);
    or_les_tendency3d(nc, L, uc, 0.0, 2.0, 3.0, p, 1.0, ts, 6.0, 1, nh);
    or_step3d_les(nc, L, 1e-2, 1e-3, 0.1, 2.0, 3.0, p, 1.0, ts, 6.0, 1, uc, 1);
    free(uf), free(uc), free(nh), free(A), free(tau), free(p), free(g), free(m), free(v);
    free(x), free(y), free(tg);
  }
  (void)np;
  printf("oracle sanitizer run: ok\n");
  return 0;
}
