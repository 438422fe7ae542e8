// diag.hip -- FP64 diagnostics (energy, enstrophy, shell spectrum; the
// spectral energy transfer of a tendency; 1D spectra; structure functions),
// the constant-power forcing coefficient and a fill kernel.
//
// All reductions are deterministic: every partial sum is formed in a fixed
// order (per-lane accumulators, fixed shuffle trees, wave-private LDS bins,
// then a second kernel summing block partials in block order), so a rerun on
// the same input gives the same bits.
#include <cmath>
#include <mutex>

#include "fft_core.h"
#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kWaves = kDiagThreads / 64;

__device__ __forceinline__ int dmode(int i, int n) { return i <= n / 2 ? i : i - n; }
__device__ __forceinline__ int j2i_rt(int j, int K, int n) { return j <= K ? j : j + n - (2 * K + 1); }

// Pass 1: one wave per row of kept modes ((kz, ky) in 3D, ky in 2D); lanes
// run along kx, where the shell index is non-decreasing, so the spectrum
// contributions of a 64-mode chunk form contiguous segments that a segmented
// scan sums before one lane per segment adds into the wave's own bins.
// TR (transfer): with tend = dstate/dt the per-mode values become the rates
// w Re(conj(u) . N) (binned) and w Re(conj(w) . curl N) (3D; 2D: the state
// is the vorticity, energy rate w Re(conj(w) N) / |k|^2, enstrophy rate
// w Re(conj(w) N)).
template <typename T, bool TR>
__global__ void __launch_bounds__(kDiagThreads)
    k_diag1(const cx<T>* __restrict__ state, const cx<T>* __restrict__ tend, int ndim, int n,
            int K, double kb, int nbins, double* __restrict__ partial) {
  __shared__ double bins[kWaves][kDiagMaxBins];
  __shared__ double red[2][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int s = threadIdx.x; s < kWaves * kDiagMaxBins; s += kDiagThreads)
    (&bins[0][0])[s] = 0.0;
  __syncthreads();
  const int M = 2 * K + 1, H = K + 1, NH = n / 2 + 1;
  const int rows = ndim == 3 ? M * M : M;
  const int W = gridDim.x * kWaves;
  const size_t cstride = (size_t)n * n * NH;
  double eacc = 0.0, zacc = 0.0;
  for (int r = blockIdx.x * kWaves + wave; r < rows; r += W) {
    int iz = 0, mz = 0, iy, my;
    if (ndim == 3) {
      iz = j2i_rt(r / M, K, n);
      iy = j2i_rt(r % M, K, n);
      mz = dmode(iz, n);
    } else {
      iy = j2i_rt(r, K, n);
    }
    my = dmode(iy, n);
    const size_t rowoff = ((size_t)iz * n + iy) * NH;
    for (int c0 = 0; c0 < H; c0 += 64) {
      const int mx = c0 + lane;
      double eu = 0.0, ez = 0.0;
      int s = 0x7fffffff;
      if (mx < H) {
        const double w = mx == 0 ? 1.0 : 2.0;
        const double kx = kb * mx, ky = kb * my, kz = kb * mz;
        const int m2 = mx * mx + my * my + mz * mz;
        if (ndim == 3) {
          const cx<T> a = state[rowoff + mx], b = state[cstride + rowoff + mx],
                      c = state[2 * cstride + rowoff + mx];
          const double ar = a.re, ai = a.im, br = b.re, bi = b.im, cr = c.re, ci = c.im;
          // k x u, real and imaginary parts separately
          const double x0r = ky * cr - kz * br, x0i = ky * ci - kz * bi;
          const double x1r = kz * ar - kx * cr, x1i = kz * ai - kx * ci;
          const double x2r = kx * br - ky * ar, x2i = kx * bi - ky * ai;
          if constexpr (TR) {
            const cx<T> p = tend[rowoff + mx], q = tend[cstride + rowoff + mx],
                        r = tend[2 * cstride + rowoff + mx];
            const double pr = p.re, pi = p.im, qr = q.re, qi = q.im, rr = r.re, ri = r.im;
            eu = w * (ar * pr + ai * pi + br * qr + bi * qi + cr * rr + ci * ri);
            const double y0r = ky * rr - kz * qr, y0i = ky * ri - kz * qi;
            const double y1r = kz * pr - kx * rr, y1i = kz * pi - kx * ri;
            const double y2r = kx * qr - ky * pr, y2i = kx * qi - ky * pi;
            ez = w * (x0r * y0r + x0i * y0i + x1r * y1r + x1i * y1i + x2r * y2r + x2i * y2i);
          } else {
            eu = 0.5 * w * (ar * ar + ai * ai + br * br + bi * bi + cr * cr + ci * ci);
            ez = 0.5 * w * (x0r * x0r + x0i * x0i + x1r * x1r + x1i * x1i + x2r * x2r + x2i * x2i);
          }
          s = (int)floor(sqrt((double)m2) + 0.5);
        } else if (m2 > 0) {
          const cx<T> a = state[rowoff + mx];
          double a2;
          if constexpr (TR) {
            const cx<T> p = tend[rowoff + mx];
            a2 = 2.0 * ((double)a.re * p.re + (double)a.im * p.im);
          } else {
            a2 = (double)a.re * a.re + (double)a.im * a.im;
          }
          const double k2 = kx * kx + ky * ky;
          eu = 0.5 * w * a2 / k2;
          ez = 0.5 * w * a2;
          s = (int)floor(sqrt((double)m2) + 0.5);
        } else {
          s = 0;
        }
      }
      eacc += eu;
      zacc += ez;
      double val = eu;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_up(val, d, 64);
        const int so = __shfl_up(s, d, 64);
        if (lane >= d && so == s) val += o;
      }
      const int sn = __shfl_down(s, 1, 64);
      const bool last = lane == 63 || sn != s;
      if (last && s < nbins) bins[wave][s] += val;
    }
  }
  // fixed-order wave reduction of the totals
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    eacc += __shfl_down(eacc, d, 64);
    zacc += __shfl_down(zacc, d, 64);
  }
  if (lane == 0) {
    red[0][wave] = eacc;
    red[1][wave] = zacc;
  }
  __syncthreads();
  double* out = partial + (size_t)blockIdx.x * (nbins + 2);
  for (int s = threadIdx.x; s < nbins; s += kDiagThreads) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) v += bins[w][s];
    out[s] = v;
  }
  if (threadIdx.x == 0) {
    double e = 0.0, z = 0.0;
    for (int w = 0; w < kWaves; w++) {
      e += red[0][w];
      z += red[1][w];
    }
    out[nbins] = e;
    out[nbins + 1] = z;
  }
}

// Pass 2: sum block partials in block order.
__global__ void __launch_bounds__(kDiagThreads)
    k_diag2(const double* __restrict__ partial, int nblocks, int nbins, double* spectrum,
            double* energy, double* enstrophy) {
  for (int s = threadIdx.x; s < nbins + 2; s += kDiagThreads) {
    double v = 0.0;
    for (int b = 0; b < nblocks; b++) v += partial[(size_t)b * (nbins + 2) + s];
    if (s < nbins)
      spectrum[s] = v;
    else if (s == nbins && energy)
      *energy = v;
    else if (s == nbins + 1 && enstrophy)
      *enstrophy = v;
  }
}

// 1D spectra, pass 1.  Waves take rows of kept modes ((kz, ky) in 3D, ky in
// 2D) in a fixed order; lanes run along kx.  Per row the wave sums each
// velocity component's energy over kx (fixed shuffle tree) into
// rowsum[row][c]; per lane it accumulates the energy of its kx values over the
// rows it visits into xpart[wave][c][kx].  NC = velocity components (2 or 3).
template <typename T, int NC>
__global__ void __launch_bounds__(kDiagThreads)
    k_spec1d_rows(const cx<T>* __restrict__ state, int n, int K, double kb,
                  double* __restrict__ rowsum, double* __restrict__ xpart) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int W = gridDim.x * kWaves;
  const int M = 2 * K + 1, H = K + 1, NH = n / 2 + 1;
  const int rows = NC == 3 ? M * M : M;
  const size_t cstride = (size_t)n * n * NH;
  constexpr int kMaxChunks = 6;  // H <= 342 (n <= 1024)
  double xacc[kMaxChunks][NC];
#pragma unroll
  for (int q = 0; q < kMaxChunks; q++)
#pragma unroll
    for (int c = 0; c < NC; c++) xacc[q][c] = 0.0;
  for (int r = wave; r < rows; r += W) {
    int iz = 0, iy;
    if (NC == 3) {
      iz = j2i_rt(r / M, K, n);
      iy = j2i_rt(r % M, K, n);
    } else {
      iy = j2i_rt(r, K, n);
    }
    const int my = dmode(iy, n);
    const size_t rowoff = ((size_t)iz * n + iy) * NH;
    double rs[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) rs[c] = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxChunks; q++) {
      const int mx = q * 64 + lane;
      if (q * 64 >= H) break;
      double e[NC];
#pragma unroll
      for (int c = 0; c < NC; c++) e[c] = 0.0;
      if (mx < H) {
        const double w = mx == 0 ? 1.0 : 2.0;
        if constexpr (NC == 3) {
#pragma unroll
          for (int c = 0; c < 3; c++) {
            const cx<T> u = state[c * cstride + rowoff + mx];
            e[c] = 0.5 * w * ((double)u.re * u.re + (double)u.im * u.im);
          }
        } else {
          const int m2 = mx * mx + my * my;
          if (m2 > 0) {
            const cx<T> a = state[rowoff + mx];
            const double kx = kb * mx, ky = kb * my, k2 = kx * kx + ky * ky;
            const double a2 = (double)a.re * a.re + (double)a.im * a.im;
            e[0] = 0.5 * w * a2 * ky * ky / (k2 * k2);
            e[1] = 0.5 * w * a2 * kx * kx / (k2 * k2);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < NC; c++) {
        xacc[q][c] += e[c];
        rs[c] += e[c];
      }
    }
#pragma unroll
    for (int c = 0; c < NC; c++) {
      double v = rs[c];
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
      if (lane == 0) rowsum[(size_t)r * NC + c] = v;
    }
  }
#pragma unroll
  for (int q = 0; q < kMaxChunks; q++) {
    const int mx = q * 64 + lane;
    if (mx < H) {
#pragma unroll
      for (int c = 0; c < NC; c++) xpart[((size_t)wave * NC + c) * H + mx] = xacc[q][c];
    }
  }
}

// 1D spectra, pass 2: out[a][c][k] with one thread per output in a fixed
// summation order (x: waves in order; y, z: rows with |m_a| = k in row order).
template <int NC>
__global__ void __launch_bounds__(kDiagThreads)
    k_spec1d_bins(const double* __restrict__ rowsum, const double* __restrict__ xpart, int W,
                  int n, int K, double* __restrict__ out) {
  const int H = K + 1, M = 2 * K + 1;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= NC * NC * H) return;
  const int k = id % H, c = (id / H) % NC, a = id / (H * NC);
  double s = 0.0;
  if (a == 0) {
    for (int w = 0; w < W; w++) s += xpart[((size_t)w * NC + c) * H + k];
  } else {
    // compact indices j with |mode| = k: j = k and (k > 0) j = M - k
    const int jn = k > 0 ? 2 : 1;
    if (NC == 2) {
      for (int q = 0; q < jn; q++) s += rowsum[(size_t)(q == 0 ? k : M - k) * NC + c];
    } else if (a == 1) {  // ky: rows r = jz * M + jy
      for (int jz = 0; jz < M; jz++)
        for (int q = 0; q < jn; q++)
          s += rowsum[((size_t)jz * M + (q == 0 ? k : M - k)) * NC + c];
    } else {  // kz
      for (int q = 0; q < jn; q++)
        for (int jy = 0; jy < M; jy++)
          s += rowsum[((size_t)(q == 0 ? k : M - k) * M + jy) * NC + c];
    }
  }
  out[id] = s;
}

// flux[s] = -(transfer[0] + ... + transfer[s]), summed in shell order
__global__ void k_flux(const double* __restrict__ transfer, int nbins, double* __restrict__ flux) {
  double c = 0.0;
  for (int s = 0; s < nbins; s++) {
    c += transfer[s];
    flux[s] = -c;
  }
}

// Forcing coefficient alpha = power / sum_band w |u_hat|^2 (0 if the band is
// empty), one block, fixed-order tree.
template <typename T>
__global__ void __launch_bounds__(kDiagThreads)
    k_alpha(const cx<T>* __restrict__ state, int n, int bw, int m2min, int m2max, double power,
            T* __restrict__ alpha) {
  __shared__ double red[kDiagThreads];
  const int NH = n / 2 + 1;
  const size_t cstride = (size_t)n * n * NH;
  const int side = 2 * bw + 1, cnt = side * side * (bw + 1);
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < cnt; idx += kDiagThreads) {
    const int mx = idx % (bw + 1);
    const int my = (idx / (bw + 1)) % side - bw;
    const int mz = idx / ((bw + 1) * side) - bw;
    const int m2 = mx * mx + my * my + mz * mz;
    if (m2 < m2min || m2 > m2max) continue;
    const double w = mx == 0 ? 1.0 : 2.0;
    const int iz = mz < 0 ? mz + n : mz, iy = my < 0 ? my + n : my;
    const size_t o = ((size_t)iz * n + iy) * NH + mx;
    for (int c = 0; c < 3; c++) {
      const cx<T> u = state[c * cstride + o];
      acc += w * ((double)u.re * u.re + (double)u.im * u.im);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int d = kDiagThreads / 2; d >= 1; d >>= 1) {
    if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) alpha[0] = (T)(red[0] > 0.0 ? power / red[0] : 0.0);
}

// Adaptive step of a step: dt = min(dt_max, cfl (L/n) / umax) (dt_max when
// the velocity vanishes), the per-axis decay tables exp(-nu k^2 dt) and
// exp(-nu k^2 dt/2) computed in FP64 and rounded once, the elapsed time; the
// velocity maximum is cleared for the next step.  One block.
template <typename T>
__global__ void __launch_bounds__(kDiagThreads)
    k_dtstep(unsigned long long* __restrict__ umax, int n, double L, double nu, double dt_max,
             double cfl, T* __restrict__ dtdev, double* __restrict__ tdev, T* __restrict__ e1,
             T* __restrict__ eh1) {
  __shared__ double dts;
  if (threadIdx.x == 0) {
    const double um = __longlong_as_double((long long)*umax);
    dts = um > 0.0 ? fmin(dt_max, cfl * (L / n) / um) : dt_max;
  }
  __syncthreads();
  const double dt = dts, kb = 2.0 * M_PI / L;
  for (int m = threadIdx.x; m < n; m += kDiagThreads) {
    const double mm = m <= n / 2 ? m : m - n;
    const double k2 = kb * kb * mm * mm;
    e1[m] = (T)exp(-nu * dt * k2);
    eh1[m] = (T)exp(-0.5 * nu * dt * k2);
  }
  if (threadIdx.x == 0) {
    *dtdev = (T)dt;
    *tdev += dt;
    *umax = 0ull;
  }
}

template <typename T>
__global__ void k_time(const double* __restrict__ tdev, double t_fixed, const T* __restrict__ dtdev,
                       double* t, double* dt) {
  if (t) *t = t_fixed + *tdev;
  if (dt) *dt = (double)*dtdev;
}

template <typename T>
__global__ void k_fill_zero(cx<T>* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = cx<T>{0, 0};
}

// ---------------------------------------------------------------------------
// Longitudinal structure functions.  k_vel_comp writes velocity component c
// of the kept modes of a state (2D: from the vorticity) as one spectral field
// [n..][n/2+1]; after its inverse transform, k_incr forms the increments
// du = u(x + r e_c) - u(x) (differences of the stored values taken in FP64)
// and per-lane FP64 sums of du^p and |du|^p, p = 1..pmax, over a contiguous
// chunk of grid points (blockIdx.x) for separation j (blockIdx.y); a fixed
// shuffle tree and the block's waves in order give one partial per block.
// k_incr_final adds the partials over components and chunks in order.
// ---------------------------------------------------------------------------
constexpr int kSfChunks = 256;
constexpr int kSfThreads = 256;
struct SfSeps {
  int r[kSfMaxR];
};

template <typename T>
__global__ void k_vel_comp(const cx<T>* __restrict__ state, int ndim, int n, int K, T kb, int c,
                           cx<T>* __restrict__ out) {
  const int NH = n / 2 + 1;
  const size_t ns = (size_t)(ndim == 3 ? n : 1) * n * NH;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ns;
       i += (size_t)gridDim.x * blockDim.x) {
    const int mx = (int)(i % NH), my = dmode((int)((i / NH) % n), n);
    const int mz = ndim == 3 ? dmode((int)(i / ((size_t)n * NH)), n) : 0;
    const bool keep = mx <= K && abs(my) <= K && abs(mz) <= K;
    cx<T> v = {0, 0};
    if (keep && ndim == 3) {
      v = state[c * ns + i];
    } else if (keep && (mx != 0 || my != 0)) {
      const T kx = kb * (T)mx, ky = kb * (T)my, k2 = kx * kx + ky * ky;
      const cx<T> w = state[i];
      // u = i ky w / k^2, v = -i kx w / k^2
      v = c == 0 ? cx<T>{-ky * w.im / k2, ky * w.re / k2} : cx<T>{kx * w.im / k2, -kx * w.re / k2};
    }
    out[i] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(kSfThreads)
    k_incr(const T* __restrict__ u, int n, int logn, int ndim, int axis, SfSeps sep, int nr,
           int pmax, double* __restrict__ part) {
  __shared__ double red[kSfThreads / 64][2 * kSfMaxP];
  const long long np = (long long)n * n * (ndim == 3 ? n : 1);
  const int j = blockIdx.y, r = sep.r[j];
  const int ls = axis * logn;  // log2 of the axis stride
  const long long per = (np + gridDim.x - 1) / gridDim.x;
  const long long b0 = (long long)blockIdx.x * per;
  const long long b1 = b0 + per < np ? b0 + per : np;
  double sp[kSfMaxP], ap[kSfMaxP];
#pragma unroll
  for (int p = 0; p < kSfMaxP; p++) sp[p] = ap[p] = 0.0;
  for (long long x = b0 + threadIdx.x; x < b1; x += kSfThreads) {
    const int q = (int)((x >> ls) & (n - 1));
    const int q2 = q + r < n ? q + r : q + r - n;
    const double d = (double)u[x + ((long long)(q2 - q) << ls)] - (double)u[x];
    double dp = 1.0;
#pragma unroll
    for (int p = 0; p < kSfMaxP; p++) {
      if (p < pmax) {
        dp *= d;
        sp[p] += dp;
        ap[p] += fabs(dp);
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < kSfMaxP; p++) {
    for (int o = 32; o >= 1; o >>= 1) {
      sp[p] += __shfl_xor(sp[p], o, 64);
      ap[p] += __shfl_xor(ap[p], o, 64);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int p = 0; p < kSfMaxP; p++) {
      red[wave][p] = sp[p];
      red[wave][kSfMaxP + p] = ap[p];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * kSfMaxP) {
    double t = 0.0;
    for (int w = 0; w < kSfThreads / 64; w++) t += red[w][threadIdx.x];
    part[(((size_t)axis * nr + j) * gridDim.x + blockIdx.x) * 2 * kSfMaxP + threadIdx.x] = t;
  }
}

__global__ void k_incr_final(const double* __restrict__ part, int ndim, int nr, int pmax,
                             int chunks, double inv, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * nr * pmax) return;
  const int which = t / (nr * pmax), j = (t / pmax) % nr, p = t % pmax;
  double s = 0.0;
  for (int a = 0; a < ndim; a++)
    for (int b = 0; b < chunks; b++)
      s += part[(((size_t)a * nr + j) * chunks + b) * 2 * kSfMaxP + which * kSfMaxP + p];
  out[t] = s * inv;
}

}  // namespace

template <typename T>
void launch_diag(Plan* p, const void* state, double* spectrum, int nbins, double* energy,
                 double* enstrophy) {
  const int K = (p->n - 1) / 3, M = 2 * K + 1;
  const int rows = p->ndim == 3 ? M * M : M;
  int blocks = (rows + kWaves - 1) / kWaves;
  if (blocks > p->dpart_blocks) blocks = p->dpart_blocks;
  p->begin(KID_DIAG);
  hipLaunchKernelGGL((k_diag1<T, false>), dim3(blocks), dim3(kDiagThreads), 0, p->launch,
                     (const cx<T>*)state, (const cx<T>*)nullptr, p->ndim, p->n, K,
                     2.0 * M_PI / p->L, nbins, p->dpart);
  launched(p, "k_diag1");
  hipLaunchKernelGGL(k_diag2, dim3(1), dim3(kDiagThreads), 0, p->launch, (const double*)p->dpart,
                     blocks, nbins, spectrum, energy, enstrophy);
  launched(p, "k_diag2");
  p->end(KID_DIAG);
}

template <typename T>
void launch_transfer(Plan* p, const void* state, const void* tend, double* transfer,
                     double* flux, int nbins, double* energy_rate, double* enstrophy_rate) {
  const int K = (p->n - 1) / 3, M = 2 * K + 1;
  const int rows = p->ndim == 3 ? M * M : M;
  int blocks = (rows + kWaves - 1) / kWaves;
  if (blocks > p->dpart_blocks) blocks = p->dpart_blocks;
  p->begin(KID_DIAG);
  hipLaunchKernelGGL((k_diag1<T, true>), dim3(blocks), dim3(kDiagThreads), 0, p->launch,
                     (const cx<T>*)state, (const cx<T>*)tend, p->ndim, p->n, K,
                     2.0 * M_PI / p->L, nbins, p->dpart);
  launched(p, "k_diag1 transfer");
  hipLaunchKernelGGL(k_diag2, dim3(1), dim3(kDiagThreads), 0, p->launch, (const double*)p->dpart,
                     blocks, nbins, transfer, energy_rate, enstrophy_rate);
  launched(p, "k_diag2");
  if (flux) {
    hipLaunchKernelGGL(k_flux, dim3(1), dim3(1), 0, p->launch, (const double*)transfer, nbins,
                       flux);
    launched(p, "k_flux");
  }
  p->end(KID_DIAG);
}

// Uses the plan's first transform workspace as scratch (free between calls).
template <typename T>
void launch_spectra1d(Plan* p, const void* state, double* out) {
  const int K = (p->n - 1) / 3, M = 2 * K + 1, H = K + 1;
  const int nc = p->ndim;
  const int rows = nc == 3 ? M * M : M;
  int blocks = (rows + kWaves - 1) / kWaves;
  if (blocks > 256) blocks = 256;
  const int W = blocks * kWaves;
  double* rowsum = (double*)p->bufA;
  double* xpart = rowsum + (size_t)rows * nc;
  const size_t need = ((size_t)rows * nc + (size_t)W * nc * H) * sizeof(double);
  if (need > p->ops.elems_a * sizeof(cx<T>)) {
    set_error("1D spectra scratch of %zu bytes exceeds the plan workspace", need);
    p->failed = true;
    return;
  }
  const double kb = 2.0 * M_PI / p->L;
  const unsigned ob = (unsigned)((nc * nc * H + kDiagThreads - 1) / kDiagThreads);
  p->begin(KID_DIAG);
  if (nc == 3) {
    hipLaunchKernelGGL((k_spec1d_rows<T, 3>), dim3(blocks), dim3(kDiagThreads), 0, p->launch,
                       (const cx<T>*)state, p->n, K, kb, rowsum, xpart);
    launched(p, "k_spec1d_rows");
    hipLaunchKernelGGL((k_spec1d_bins<3>), dim3(ob), dim3(kDiagThreads), 0, p->launch,
                       (const double*)rowsum, (const double*)xpart, W, p->n, K, out);
  } else {
    hipLaunchKernelGGL((k_spec1d_rows<T, 2>), dim3(blocks), dim3(kDiagThreads), 0, p->launch,
                       (const cx<T>*)state, p->n, K, kb, rowsum, xpart);
    launched(p, "k_spec1d_rows");
    hipLaunchKernelGGL((k_spec1d_bins<2>), dim3(ob), dim3(kDiagThreads), 0, p->launch,
                       (const double*)rowsum, (const double*)xpart, W, p->n, K, out);
  }
  launched(p, "k_spec1d_bins");
  p->end(KID_DIAG);
}

// Structure functions: component c of the velocity is written as a spectral
// field, inverse transformed and its increments reduced, using the plan's
// transform workspace (3D: spectral field at B + F, transform through A and B,
// physical field at A + F; 2D: spectral field at A + F, physical field at A,
// transform through B; F = one undealiased field).
template <typename T>
void launch_structure(Plan* p, const void* state, int nr, const int* r, int pmax, double* out) {
  const int n = p->n, nd = p->ndim, K = (n - 1) / 3;
  const size_t F = p->ops.elems_full;
  const size_t ns = (size_t)(nd == 3 ? n : 1) * n * (n / 2 + 1);
  const size_t nphys = (size_t)(nd == 3 ? n : 1) * n * n;
  const size_t phys_c = (nphys * sizeof(T) + sizeof(cx<T>) - 1) / sizeof(cx<T>);
  const bool fits = nd == 3 ? (F + phys_c <= p->ops.elems_a && F + ns <= p->ops.elems_b)
                            : (F + ns <= p->ops.elems_a && phys_c <= F);
  const size_t part_elems = (size_t)nd * nr * kSfChunks * 2 * kSfMaxP;
  if (!fits || ns > F || part_elems > (size_t)kDiagMaxBlocks * (kDiagMaxBins + 2)) {
    set_error("structure-function scratch exceeds the plan workspace");
    p->failed = true;
    return;
  }
  cx<T>* A = (cx<T>*)p->bufA;
  cx<T>* B = (cx<T>*)p->bufB;
  cx<T>* spec = nd == 3 ? B + F : A + F;
  T* phys = nd == 3 ? (T*)(A + F) : (T*)A;
  SfSeps sep{};
  for (int j = 0; j < nr; j++) sep.r[j] = r[j];
  int logn = 0;
  while ((1 << logn) < n) logn++;
  const int vb = (int)((ns + kDiagThreads - 1) / kDiagThreads);
  for (int c = 0; c < nd; c++) {
    p->begin(KID_DIAG);
    hipLaunchKernelGGL((k_vel_comp<T>), dim3(vb < 4096 ? vb : 4096), dim3(kDiagThreads), 0,
                       p->launch, (const cx<T>*)state, nd, n, K, (T)(2.0 * M_PI / p->L), c, spec);
    launched(p, "k_vel_comp");
    p->end(KID_DIAG);
    if (nd == 3)
      p->ops.fft_inv_n(p, spec, phys, 1, A, B, false);
    else
      p->ops.fft_inv(p, spec, phys);
    p->begin(KID_DIAG);
    hipLaunchKernelGGL((k_incr<T>), dim3(kSfChunks, nr), dim3(kSfThreads), 0, p->launch,
                       (const T*)phys, n, logn, nd, c, sep, nr, pmax, p->dpart);
    launched(p, "k_incr");
    p->end(KID_DIAG);
  }
  p->begin(KID_DIAG);
  hipLaunchKernelGGL(k_incr_final, dim3((2 * nr * pmax + 255) / 256), dim3(256), 0, p->launch,
                     (const double*)p->dpart, nd, nr, pmax, kSfChunks,
                     1.0 / ((double)nphys * nd), out);
  launched(p, "k_incr_final");
  p->end(KID_DIAG);
}

template <typename T>
void launch_alpha(Plan* p, const void* state) {
  p->begin(KID_ALPHA);
  hipLaunchKernelGGL((k_alpha<T>), dim3(1), dim3(kDiagThreads), 0, p->launch, (const cx<T>*)state,
                     p->n, p->bw, p->m2min, p->m2max, p->fpow, (T*)p->alpha);
  launched(p, "k_alpha");
  p->end(KID_ALPHA);
}

template <typename T>
void launch_dtstep(Plan* p) {
  p->begin(KID_ALPHA);
  hipLaunchKernelGGL((k_dtstep<T>), dim3(1), dim3(kDiagThreads), 0, p->launch, p->umaxdev, p->n,
                     p->L, p->nu, p->dt, p->cfl, (T*)p->dtdev, p->tdev, (T*)p->e1, (T*)p->eh1);
  launched(p, "k_dtstep");
  p->end(KID_ALPHA);
}

void launch_time(Plan* p, double* t, double* dt) {
  if (p->prec == FS_F32)
    hipLaunchKernelGGL((k_time<float>), dim3(1), dim3(1), 0, p->launch, (const double*)p->tdev,
                       p->t_fixed, (const float*)p->dtdev, t, dt);
  else
    hipLaunchKernelGGL((k_time<double>), dim3(1), dim3(1), 0, p->launch, (const double*)p->tdev,
                       p->t_fixed, (const double*)p->dtdev, t, dt);
  launched(p, "k_time");
}

template <typename T>
void launch_fill(Plan* p, void* ptr, size_t n_complex) {
  p->begin(KID_FILL);
  size_t blocks = (n_complex + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL((k_fill_zero<T>), dim3((unsigned)blocks), dim3(256), 0, p->launch,
                     (cx<T>*)ptr, n_complex);
  launched(p, "k_fill_zero");
  p->end(KID_FILL);
}

// ---------------------------------------------------------------------------
// Diagnostics without a plan and without allocation.  The block partial sums
// of k_diag1 go to a file-scope device array instead of a plan's workspace;
// every device the library runs on holds its own copy until the process ends.
// Each call writes every partial it later reads (nbins + 2 values per block),
// so nothing needs clearing between calls; calls that overlap on one device
// share the array and race.
// ---------------------------------------------------------------------------
constexpr size_t kStaticDiagDoubles = (size_t)1 << 20;  // 8 MiB
static __device__ __align__(256) double scratch[kStaticDiagDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// the address of this device's copy of `scratch` (the host-side name is only
// a stand-in for it); looked up once per device, with that device current
double* scratch_on(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = (double*)ptr;
  }
  return g_scratch[dev];
}

template <typename T>
void diag_static(int ndim, int n, double L, const void* state, double* spectrum, int nbins,
                 double* energy, double* enstrophy, double* part, int blocks, hipStream_t s) {
  const int K = (n - 1) / 3;
  hipLaunchKernelGGL((k_diag1<T, false>), dim3(blocks), dim3(kDiagThreads), 0, s,
                     (const cx<T>*)state, (const cx<T>*)nullptr, ndim, n, K, 2.0 * M_PI / L, nbins,
                     part);
  hipLaunchKernelGGL(k_diag2, dim3(1), dim3(kDiagThreads), 0, s, (const double*)part, blocks,
                     nbins, spectrum, energy, enstrophy);
}
}  // namespace

template void launch_diag<float>(Plan*, const void*, double*, int, double*, double*);
template void launch_diag<double>(Plan*, const void*, double*, int, double*, double*);
template void launch_transfer<float>(Plan*, const void*, const void*, double*, double*, int,
                                     double*, double*);
template void launch_transfer<double>(Plan*, const void*, const void*, double*, double*, int,
                                      double*, double*);
template void launch_spectra1d<float>(Plan*, const void*, double*);
template void launch_spectra1d<double>(Plan*, const void*, double*);
template void launch_structure<float>(Plan*, const void*, int, const int*, int, double*);
template void launch_structure<double>(Plan*, const void*, int, const int*, int, double*);
template void launch_alpha<float>(Plan*, const void*);
template void launch_alpha<double>(Plan*, const void*);
template void launch_dtstep<float>(Plan*);
template void launch_dtstep<double>(Plan*);
template void launch_fill<float>(Plan*, void*, size_t);
template void launch_fill<double>(Plan*, void*, size_t);

}  // namespace fs

extern "C" fs_status fs_energy_spectrum_static(int ndim, int n, int precision, double L,
                                               const void* state, double* spectrum, int nbins,
                                               double* energy, double* enstrophy, void* stream) {
  using namespace fs;
  if (ndim != 2 && ndim != 3) {
    set_error("ndim = %d must be 2 or 3", ndim);
    return FS_E_INVALID;
  }
  if (precision != FS_F32 && precision != FS_F64) {
    set_error("precision = %d must be FS_F32 or FS_F64", precision);
    return FS_E_INVALID;
  }
  if (n < 16 || n > 1024 || (n & (n - 1)) || (ndim == 3 && precision == FS_F64 && n > 512)) {
    set_error("n = %d: supported sizes are the plans' (powers of two 16..1024, 3D FP64 <= 512)", n);
    return FS_E_UNSUPPORTED;
  }
  if (!(std::isfinite(L) && L > 0)) {
    set_error("L must be finite and > 0");
    return FS_E_INVALID;
  }
  if (!state || !spectrum) {
    set_error("NULL array");
    return FS_E_INVALID;
  }
  if (nbins < 1 || nbins > kDiagMaxBins) {
    set_error("nbins = %d must be in 1..%d", nbins, kDiagMaxBins);
    return FS_E_INVALID;
  }
  // the same partial-sum grid as the plan's reduction, so the results agree bit for bit
  const int K = (n - 1) / 3, M = 2 * K + 1;
  const int rows = ndim == 3 ? M * M : M;
  int blocks = (rows + kWaves - 1) / kWaves;
  if (blocks > kDiagMaxBlocks) blocks = kDiagMaxBlocks;
  const size_t need = (size_t)blocks * (size_t)(nbins + 2);
  if (need > kStaticDiagDoubles) {
    set_error("nbins = %d at n = %d needs %zu bytes of partial sums; the static scratch holds "
              "%zu (fs_energy_spectrum with a plan has no such limit)",
              nbins, n, need * sizeof(double), kStaticDiagDoubles * sizeof(double));
    return FS_E_INVALID;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    hipGetLastError();
    set_error("no usable HIP device");
    return FS_E_DEVICE;
  }
  double* part = scratch_on(dev);
  if (!part) {
    set_error("hipGetSymbolAddress of the static scratch failed");
    return FS_E_DEVICE;
  }
  if (precision == FS_F32)
    diag_static<float>(ndim, n, L, state, spectrum, nbins, energy, enstrophy, part, blocks,
                       (hipStream_t)stream);
  else
    diag_static<double>(ndim, n, L, state, spectrum, nbins, energy, enstrophy, part, blocks,
                        (hipStream_t)stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("diagnostics launch: %s", hipGetErrorString(e));
    return FS_E_DEVICE;
  }
  return FS_OK;
}
