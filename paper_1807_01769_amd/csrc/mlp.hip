// mlp.hip -- the learned subgrid-stress closure network, 9 -> 64 -> 64 -> 6,
// GELU(x) = x Phi(x) (exact, erf), trained and evaluated with BF16 matrix
// cores (v_mfma_f32_16x16x16_bf16, FP32 accumulate).
//
// Layout of one layer on the matrix cores.  Activations travel transposed:
// a tile of 16 points is H[f][p] (feature f, point p) and a layer computes
// D[o][p] = sum_k W[o][k] H[k][p] with the weights as the A operand (16x16
// blocks, lane l holds A[l%16][4(l/16)+j]) and the activations as the B
// operand (lane l holds B[4(l/16)+j][l%16]).  The FP32 result D lands in
// lane l as D[4(l/16)+j][l%16] -- exactly the B-operand layout of the next
// layer, so layers chain in registers.  Weight gradients contract over
// points instead; their operands are 16x16 transposes through a per-wave
// LDS tile.
//
// Parameters (FP32 master, 5190 values): W1[64][9] b1[64] W2[64][64] b2[64]
// W3[6][64] b3[6].  The BF16 copies are repacked into lane order (one
// 16x16 block = 64 lanes x 4 values) after every update.  Features are BF16
// [P][16] (9 used, rest zero); targets and outputs FP32 [P][6].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "bf16.h"
#include "fs.h"
#include "fs_internal.h"

namespace fs {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 9, kHid = 64, kOut = 6;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + kHid * kIn, OFF_W2 = OFF_B1 + kHid,
              OFF_B2 = OFF_W2 + kHid * kHid, OFF_W3 = OFF_B2 + kHid,
              OFF_B3 = OFF_W3 + kOut * kHid, NPARAM = OFF_B3 + kOut;
// lane-ordered BF16 blocks: W1 (4), W2 (4x4), W3 (4), W3^T (4), W2^T (4x4)
constexpr int BLK_W1 = 0, BLK_W2 = 4, BLK_W3 = 20, BLK_W3T = 24, BLK_W2T = 28, NBLK = 44;
constexpr int kThreads = 256, kWaves = kThreads / 64;
// Forward grids stop at one resident round (256 CUs x 3 four-wave blocks at
// the kernels' 3 waves per SIMD): every wave loads the network into
// registers once and runs over several point tiles.
constexpr int kForwardBlocks = 768;

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// element (row, col) of the 16x16 A-operand block `blk`, from the master
__device__ float block_elem(const float* w, int blk, int row, int col) {
  if (blk < BLK_W2) {  // W1: rows 16 ob + row, cols k (< 9)
    const int o = 16 * (blk - BLK_W1) + row;
    return col < kIn ? w[OFF_W1 + o * kIn + col] : 0.f;
  } else if (blk < BLK_W3) {  // W2[16 ob + row][16 kb + col]
    const int ob = (blk - BLK_W2) / 4, kb = (blk - BLK_W2) % 4;
    return w[OFF_W2 + (16 * ob + row) * kHid + 16 * kb + col];
  } else if (blk < BLK_W3T) {  // W3[row (< 6)][16 kb + col]
    const int kb = blk - BLK_W3;
    return row < kOut ? w[OFF_W3 + row * kHid + 16 * kb + col] : 0.f;
  } else if (blk < BLK_W2T) {  // W3^T[16 fb + row][col (< 6)] = W3[col][16 fb + row]
    const int fb = blk - BLK_W3T;
    return col < kOut ? w[OFF_W3 + col * kHid + 16 * fb + row] : 0.f;
  } else {  // W2^T[16 fb + row][16 ob + col] = W2[16 ob + col][16 fb + row]
    const int fb = (blk - BLK_W2T) / 4, ob = (blk - BLK_W2T) % 4;
    return w[OFF_W2 + (16 * ob + col) * kHid + 16 * fb + row];
  }
}

// repack: lane l of block b holds A[l%16][4(l/16)+j], j = 0..3
__global__ void k_mlp_pack(const float* __restrict__ w, s4* __restrict__ packed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NBLK * 64) return;
  const int blk = i / 64, l = i % 64;
  s4 v;
  for (int j = 0; j < 4; j++) v[j] = to_bf16(block_elem(w, blk, l % 16, 4 * (l / 16) + j));
  packed[i] = v;
}

struct Net {
  s4 w1[4], w2[16], w3[4];
  f4 b1[4], b2[4], b3;
};

__device__ __forceinline__ void load_net(Net& n, const s4* __restrict__ pk, const float* __restrict__ w,
                                         int l) {
  for (int b = 0; b < 4; b++) n.w1[b] = pk[(BLK_W1 + b) * 64 + l];
  for (int b = 0; b < 16; b++) n.w2[b] = pk[(BLK_W2 + b) * 64 + l];
  for (int b = 0; b < 4; b++) n.w3[b] = pk[(BLK_W3 + b) * 64 + l];
  const int r0 = 4 * (l / 16);
  for (int ob = 0; ob < 4; ob++)
    for (int j = 0; j < 4; j++) {
      n.b1[ob][j] = w[OFF_B1 + 16 * ob + r0 + j];
      n.b2[ob][j] = w[OFF_B2 + 16 * ob + r0 + j];
    }
  for (int j = 0; j < 4; j++) n.b3[j] = r0 + j < kOut ? w[OFF_B3 + r0 + j] : 0.f;
}

// input tile (B operand): features 4(l/16)+j of point p0 + l%16 (0 past P)
__device__ __forceinline__ s4 load_x(const short* __restrict__ x, int64_t p0, int64_t P, int l) {
  const int64_t p = p0 + (l % 16);
  s4 v = {0, 0, 0, 0};
  if (p < P) v = *reinterpret_cast<const s4*>(x + p * 16 + 4 * (l / 16));
  return v;
}

// forward of one tile; keeps pre-activations and BF16 activations
__device__ __forceinline__ f4 forward_tile(const Net& n, s4 x, f4 (&z1)[4], s4 (&h1)[4],
                                           f4 (&z2)[4], s4 (&h2)[4]) {
#pragma unroll
  for (int ob = 0; ob < 4; ob++) {
    z1[ob] = mfma(n.w1[ob], x, n.b1[ob]);
#pragma unroll
    for (int j = 0; j < 4; j++) h1[ob][j] = to_bf16(gelu(z1[ob][j]));
  }
#pragma unroll
  for (int ob = 0; ob < 4; ob++) {
    f4 acc = n.b2[ob];
#pragma unroll
    for (int kb = 0; kb < 4; kb++) acc = mfma(n.w2[ob * 4 + kb], h1[kb], acc);
    z2[ob] = acc;
#pragma unroll
    for (int j = 0; j < 4; j++) h2[ob][j] = to_bf16(gelu(acc[j]));
  }
  f4 y = n.b3;
#pragma unroll
  for (int kb = 0; kb < 4; kb++) y = mfma(n.w3[kb], h2[kb], y);
  return y;
}

// y[p][o] = out_scale[o] * net(x)[o]  (out_scale may be null: 1)
__global__ void __launch_bounds__(kThreads)
    k_mlp_forward(const short* __restrict__ x, float* __restrict__ y, int64_t P,
                  const s4* __restrict__ pk, const float* __restrict__ w,
                  const float* __restrict__ out_scale) {
  const int l = threadIdx.x % 64;
  const int64_t wave = (int64_t)blockIdx.x * kWaves + threadIdx.x / 64;
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  Net n;
  load_net(n, pk, w, l);
  const int r0 = 4 * (l / 16);
  float sc[4];
  for (int j = 0; j < 4; j++) sc[j] = (out_scale && r0 + j < kOut) ? out_scale[r0 + j] : 1.f;
  const int64_t ntiles = (P + 15) / 16;
  for (int64_t tile = wave; tile < ntiles; tile += nw) {
    f4 z1[4], z2[4];
    s4 h1[4], h2[4];
    const f4 out = forward_tile(n, load_x(x, tile * 16, P, l), z1, h1, z2, h2);
    const int64_t p = tile * 16 + (l % 16);
    if (p < P) {
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (r0 + j < kOut) y[p * kOut + r0 + j] = out[j] * sc[j];
    }
  }
}

// 16x16 transpose through a per-wave LDS tile: lane l gives v[j] for
// element (row 4(l/16)+j, col l%16); returns element (row l%16, col 4(l/16)+j).
__device__ __forceinline__ s4 transpose16(short* tile, s4 v, int l) {
  const int r0 = 4 * (l / 16), c = l % 16;
#pragma unroll
  for (int j = 0; j < 4; j++) tile[(r0 + j) * 17 + c] = v[j];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  s4 out;
#pragma unroll
  for (int j = 0; j < 4; j++) out[j] = tile[c * 17 + r0 + j];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return out;
}

// Forward + backward of the mean squared error over all P*6 outputs.  Every
// wave accumulates the gradient of its tiles; partial[wave][NPARAM + 1]
// receives it in parameter order (last slot: the wave's loss share).
__global__ void __launch_bounds__(kThreads)
    k_mlp_grad(const short* __restrict__ x, const float* __restrict__ t, int64_t P,
               const s4* __restrict__ pk, const float* __restrict__ w,
               float* __restrict__ partial) {
  __shared__ short tiles[kWaves][16 * 17];
  const int l = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int64_t wave = (int64_t)blockIdx.x * kWaves + wv;
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  short* tile = tiles[wv];
  Net n;
  load_net(n, pk, w, l);
  s4 w3t[4], w2t[16];
  for (int b = 0; b < 4; b++) w3t[b] = pk[(BLK_W3T + b) * 64 + l];
  for (int b = 0; b < 16; b++) w2t[b] = pk[(BLK_W2T + b) * 64 + l];
  const int r0 = 4 * (l / 16);
  const float gscale = 2.0f / ((float)P * kOut);
  f4 gw1[4], gw2[16], gw3[4], gb1[4], gb2[4], gb3;
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < 4; i++) gw1[i] = gw3[i] = gb1[i] = gb2[i] = zero;
  for (int i = 0; i < 16; i++) gw2[i] = zero;
  gb3 = zero;
  float loss = 0.f;
  const int64_t ntiles = (P + 15) / 16;
  for (int64_t tix = wave; tix < ntiles; tix += nw) {
    const int64_t p = tix * 16 + (l % 16);
    const s4 xin = load_x(x, tix * 16, P, l);
    f4 z1[4], z2[4];
    s4 h1[4], h2[4];
    const f4 y = forward_tile(n, xin, z1, h1, z2, h2);
    // dY[o][p] = 2 (y - t) / (P 6), zero for padding outputs and points
    f4 dy = zero;
#pragma unroll
    for (int j = 0; j < 4; j++)
      if (r0 + j < kOut && p < P) {
        const float d = y[j] - t[p * kOut + r0 + j];
        loss += d * d;
        dy[j] = d * gscale;
      }
    s4 dyb;
#pragma unroll
    for (int j = 0; j < 4; j++) dyb[j] = to_bf16(dy[j]);
    gb3 += dy;
    // dH2 = W3^T dY, dZ2 = dH2 * gelu'(z2)
    f4 dz2[4];
    s4 dz2b[4];
#pragma unroll
    for (int fb = 0; fb < 4; fb++) {
      const f4 d = mfma(w3t[fb], dyb, zero);
#pragma unroll
      for (int j = 0; j < 4; j++) dz2[fb][j] = d[j] * gelu_d(z2[fb][j]);
#pragma unroll
      for (int j = 0; j < 4; j++) dz2b[fb][j] = to_bf16(dz2[fb][j]);
      gb2[fb] += dz2[fb];
    }
    // dH1 = W2^T dZ2, dZ1 = dH1 * gelu'(z1)
    s4 dz1b[4];
#pragma unroll
    for (int fb = 0; fb < 4; fb++) {
      f4 d = zero;
#pragma unroll
      for (int ob = 0; ob < 4; ob++) d = mfma(w2t[fb * 4 + ob], dz2b[ob], d);
      f4 dz1;
#pragma unroll
      for (int j = 0; j < 4; j++) dz1[j] = d[j] * gelu_d(z1[fb][j]);
#pragma unroll
      for (int j = 0; j < 4; j++) dz1b[fb][j] = to_bf16(dz1[j]);
      gb1[fb] += dz1;
    }
    // weight gradients: dW[o][f] += sum_p dZ[o][p] H[f][p]; both operands are
    // the transposes of the tiles held (contraction over points)
    const s4 dyT = transpose16(tile, dyb, l);
    s4 h2T[4];
#pragma unroll
    for (int fb = 0; fb < 4; fb++) h2T[fb] = transpose16(tile, h2[fb], l);
#pragma unroll
    for (int fb = 0; fb < 4; fb++) gw3[fb] = mfma(dyT, h2T[fb], gw3[fb]);
    s4 h1T[4];
#pragma unroll
    for (int fb = 0; fb < 4; fb++) h1T[fb] = transpose16(tile, h1[fb], l);
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
      const s4 dT = transpose16(tile, dz2b[ob], l);
#pragma unroll
      for (int fb = 0; fb < 4; fb++) gw2[ob * 4 + fb] = mfma(dT, h1T[fb], gw2[ob * 4 + fb]);
    }
    const s4 xT = transpose16(tile, xin, l);
#pragma unroll
    for (int ob = 0; ob < 4; ob++) gw1[ob] = mfma(transpose16(tile, dz1b[ob], l), xT, gw1[ob]);
  }
  // write the wave's partial gradient in parameter order.  gw*: lane l holds
  // element (row 4(l/16)+j, col l%16) of each 16x16 block.
  float* out = partial + wave * (NPARAM + 1);
  const int c = l % 16;
#pragma unroll
  for (int ob = 0; ob < 4; ob++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int o = 16 * ob + r0 + j;
      if (c < kIn) out[OFF_W1 + o * kIn + c] = gw1[ob][j];
#pragma unroll
      for (int fb = 0; fb < 4; fb++) out[OFF_W2 + o * kHid + 16 * fb + c] = gw2[ob * 4 + fb][j];
    }
#pragma unroll
  for (int fb = 0; fb < 4; fb++)
#pragma unroll
    for (int j = 0; j < 4; j++)
      if (r0 + j < kOut) out[OFF_W3 + (r0 + j) * kHid + 16 * fb + c] = gw3[fb][j];
  // biases: sum the 16 point lanes of each row group (fixed butterfly order)
#pragma unroll
  for (int ob = 0; ob < 4; ob++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      float s1 = gb1[ob][j], s2 = gb2[ob][j];
#pragma unroll
      for (int d = 1; d < 16; d <<= 1) {
        s1 += __shfl_xor(s1, d, 64);
        s2 += __shfl_xor(s2, d, 64);
      }
      if (c == 0) {
        out[OFF_B1 + 16 * ob + r0 + j] = s1;
        out[OFF_B2 + 16 * ob + r0 + j] = s2;
      }
    }
#pragma unroll
  for (int j = 0; j < 4; j++) {
    float s3 = gb3[j];
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) s3 += __shfl_xor(s3, d, 64);
    if (c == 0 && r0 + j < kOut) out[OFF_B3 + r0 + j] = s3;
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) loss += __shfl_xor(loss, d, 64);
  if (l == 0) out[NPARAM] = loss / ((float)P * kOut);
}

// Deterministic two-level sum of the wave partials: group g of kGroup waves
// (wave order) -> part2[g][i] in FP64, then the groups in order -> grad[i]
// (and the loss, slot NPARAM).  Grid of the first level: (params, groups).
constexpr int kGroup = 32, kMaxGroups = 1024 / kGroup;
__global__ void k_mlp_reduce1(const float* __restrict__ partial, int nw,
                              double* __restrict__ part2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > NPARAM) return;
  const int w0 = blockIdx.y * kGroup, w1 = w0 + kGroup < nw ? w0 + kGroup : nw;
  double s = 0.0;
  for (int w = w0; w < w1; w++) s += partial[(size_t)w * (NPARAM + 1) + i];
  part2[(size_t)blockIdx.y * (NPARAM + 1) + i] = s;
}
__global__ void k_mlp_reduce2(const double* __restrict__ part2, int ng, float* __restrict__ grad,
                              double* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > NPARAM) return;
  double s = 0.0;
  for (int g = 0; g < ng; g++) s += part2[(size_t)g * (NPARAM + 1) + i];
  if (i < NPARAM) {
    if (grad) grad[i] = (float)s;
  } else if (loss) {
    *loss = s;
  }
}

// Adam on the FP32 master weights; c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ void k_mlp_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_copy_f32(const float* __restrict__ a, float* __restrict__ b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace

struct Mlp {
  hipStream_t stream = nullptr;
  void* base = nullptr;
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *partial = nullptr;
  double* part2 = nullptr;
  s4* packed = nullptr;
  int nwaves = 0, step = 0;
  bool failed = false;
  bool ok(hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    set_error("%s: %s", what, hipGetErrorString(e));
    failed = true;
    return false;
  }
  bool launched(const char* what) { return ok(hipGetLastError(), what); }
  bool pack() {
    hipLaunchKernelGGL(k_mlp_pack, dim3((NBLK * 64 + 255) / 256), dim3(256), 0, stream, w, packed);
    return launched("k_mlp_pack");
  }
};

// used by the closure/LES code
// The LES form: features read planar from the gradients A[9][P] and
// standardised and rounded exactly as k_features stores them; outputs
// clipped, scaled and written planar as the stress tau[6][P].
__global__ void __launch_bounds__(kThreads)
    k_mlp_forward_planar(const float* __restrict__ A, int64_t P, float inv_a,
                         float* __restrict__ tau, StressMap sm, const s4* __restrict__ pk,
                         const float* __restrict__ w) {
  const int l = threadIdx.x % 64;
  const int64_t wave = (int64_t)blockIdx.x * kWaves + threadIdx.x / 64;
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  Net n;
  load_net(n, pk, w, l);
  const int r0 = 4 * (l / 16);
  const int64_t ntiles = (P + 15) / 16;
  for (int64_t tile = wave; tile < ntiles; tile += nw) {
    const int64_t p = tile * 16 + (l % 16);
    s4 xin = {0, 0, 0, 0};
    if (p < P) {
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (r0 + j < kIn) xin[j] = to_bf16(A[(r0 + j) * P + p] * inv_a);
    }
    f4 z1[4], z2[4];
    s4 h1[4], h2[4];
    const f4 out = forward_tile(n, xin, z1, h1, z2, h2);
    if (p < P) {
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (r0 + j < kOut) {
          float v = out[j];
          if (sm.clip > 0.f) v = fminf(fmaxf(v, -sm.clip), sm.clip);
          tau[(r0 + j) * P + p] = v * sm.scale[r0 + j];
        }
    }
  }
}

void mlp_forward_planar_launch(Mlp* net, const float* A, int64_t P, float inv_a, float* tau,
                               StressMap sm, hipStream_t s) {
  const int64_t tiles = (P + 15) / 16;
  int64_t blocks = (tiles + kWaves - 1) / kWaves;
  if (blocks > kForwardBlocks) blocks = kForwardBlocks;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_mlp_forward_planar, dim3((unsigned)blocks), dim3(kThreads), 0, s, A, P,
                     inv_a, tau, sm, net->packed, net->w);
}

void mlp_forward_launch(Mlp* net, const void* x, float* y, int64_t P, const float* out_scale,
                        hipStream_t s) {
  const int64_t tiles = (P + 15) / 16;
  int64_t blocks = (tiles + kWaves - 1) / kWaves;
  if (blocks > kForwardBlocks) blocks = kForwardBlocks;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(kThreads), 0, s, (const short*)x,
                     y, P, net->packed, net->w, out_scale);
}

int mlp_nparams() { return NPARAM; }

}  // namespace fs

struct fs_mlp {
  fs::Mlp m;
};

namespace fs {
Mlp* mlp_of(fs_mlp* net) { return net ? &net->m : nullptr; }
}  // namespace fs

extern "C" {

fs_status fs_mlp_create(fs_mlp** out, uint64_t seed, void* stream) {
  if (!out) {
    fs::set_error("out is NULL");
    return FS_E_INVALID;
  }
  *out = nullptr;
  fs_mlp* h = new (std::nothrow) fs_mlp();
  if (!h) return FS_E_NOMEM;
  fs::Mlp* n = &h->m;
  n->stream = (hipStream_t)stream;
  n->nwaves = 1024;
  const size_t np = fs::NPARAM;
  const size_t bytes = 4 * (4 * np + 64) + sizeof(fs::s4) * fs::NBLK * 64 +
                       4 * (size_t)n->nwaves * (np + 1) + 8 * (size_t)fs::kMaxGroups * (np + 1) +
                       2048;
  if (fs::dev_malloc(&n->base, bytes) != hipSuccess) {
    hipGetLastError();
    delete h;
    fs::set_error("hipMalloc failed");
    return FS_E_NOMEM;
  }
  char* b = (char*)n->base;
  auto take = [&](size_t sz) {
    char* p = b;
    b += (sz + 255) & ~(size_t)255;
    return p;
  };
  n->w = (float*)take(4 * np);
  n->m = (float*)take(4 * np);
  n->v = (float*)take(4 * np);
  n->g = (float*)take(4 * np);
  n->packed = (fs::s4*)take(sizeof(fs::s4) * fs::NBLK * 64);
  n->partial = (float*)take(4 * (size_t)n->nwaves * (np + 1));
  n->part2 = (double*)take(8 * (size_t)fs::kMaxGroups * (np + 1));
  // Xavier-uniform initial weights from a counter-based hash of (seed, index);
  // biases zero
  std::vector<float> hw(np, 0.f);
  auto uni = [&](uint64_t i) {
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + i + 1;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  };
  auto fill = [&](int off, int fan_out, int fan_in) {
    const double a = std::sqrt(6.0 / (fan_in + fan_out));
    for (int i = 0; i < fan_out * fan_in; i++) hw[off + i] = (float)(a * uni(off + i));
  };
  fill(fs::OFF_W1, fs::kHid, fs::kIn);
  fill(fs::OFF_W2, fs::kHid, fs::kHid);
  fill(fs::OFF_W3, fs::kOut, fs::kHid);
  bool good = n->ok(hipMemcpy(n->w, hw.data(), 4 * np, hipMemcpyHostToDevice), "copy") &&
              n->ok(hipMemset(n->m, 0, 4 * np), "clear") && n->ok(hipMemset(n->v, 0, 4 * np), "clear") &&
              n->pack() && n->ok(hipStreamSynchronize(n->stream), "sync");
  if (!good) {
    hipFree(n->base);
    delete h;
    return FS_E_DEVICE;
  }
  *out = h;
  return FS_OK;
}

fs_status fs_mlp_destroy(fs_mlp* net) {
  if (!net) return FS_OK;
  if (net->m.stream) hipStreamSynchronize(net->m.stream);
  else hipDeviceSynchronize();
  hipFree(net->m.base);
  delete net;
  return FS_OK;
}

fs_status fs_mlp_nparams(int* n) {
  if (!n) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  *n = fs::NPARAM;
  return FS_OK;
}

fs_status fs_mlp_set_params(fs_mlp* net, const float* params) {
  if (!net || !params) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  fs::Mlp* n = &net->m;
  if (n->failed) return FS_E_DEVICE;
  hipLaunchKernelGGL(fs::k_copy_f32, dim3((fs::NPARAM + 255) / 256), dim3(256), 0, n->stream,
                     params, n->w, fs::NPARAM);
  if (!n->launched("copy params") || !n->pack()) return FS_E_DEVICE;
  n->step = 0;
  return FS_OK;
}

fs_status fs_mlp_get_params(const fs_mlp* net, float* params) {
  if (!net || !params) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  const fs::Mlp* n = &net->m;
  if (n->failed) return FS_E_DEVICE;
  hipLaunchKernelGGL(fs::k_copy_f32, dim3((fs::NPARAM + 255) / 256), dim3(256), 0, n->stream,
                     (const float*)n->w, params, fs::NPARAM);
  return hipGetLastError() == hipSuccess ? FS_OK : FS_E_DEVICE;
}

fs_status fs_mlp_forward(fs_mlp* net, const void* x_bf16, float* y, int64_t npts) {
  if (!net || !x_bf16 || !y) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  if (npts < 0) {
    fs::set_error("npts must be >= 0");
    return FS_E_INVALID;
  }
  fs::Mlp* n = &net->m;
  if (n->failed) return FS_E_DEVICE;
  if (npts == 0) return FS_OK;
  fs::mlp_forward_launch(n, x_bf16, y, npts, nullptr, n->stream);
  return n->launched("k_mlp_forward") ? FS_OK : FS_E_DEVICE;
}

// The gradient kernel runs one wave per 16-point tile up to n->nwaves waves
// (then waves loop over tiles); the partials are summed in two fixed-order
// levels, so the result is deterministic for a given npts.
static fs_status mlp_grad_impl(fs::Mlp* n, const void* x, const float* t, int64_t P, float* grad,
                               double* loss) {
  const int64_t tiles = (P + 15) / 16;
  int nw = (int)(tiles < n->nwaves ? tiles : n->nwaves);
  nw = (nw + fs::kWaves - 1) / fs::kWaves * fs::kWaves;
  hipLaunchKernelGGL(fs::k_mlp_grad, dim3(nw / fs::kWaves), dim3(fs::kThreads), 0, n->stream,
                     (const short*)x, t, P, n->packed, (const float*)n->w, n->partial);
  if (!n->launched("k_mlp_grad")) return FS_E_DEVICE;
  const int ng = (nw + fs::kGroup - 1) / fs::kGroup;
  const unsigned pb = (fs::NPARAM + 1 + 255) / 256;
  hipLaunchKernelGGL(fs::k_mlp_reduce1, dim3(pb, ng), dim3(256), 0, n->stream,
                     (const float*)n->partial, nw, n->part2);
  if (!n->launched("k_mlp_reduce1")) return FS_E_DEVICE;
  hipLaunchKernelGGL(fs::k_mlp_reduce2, dim3(pb), dim3(256), 0, n->stream,
                     (const double*)n->part2, ng, grad, loss);
  return n->launched("k_mlp_reduce2") ? FS_OK : FS_E_DEVICE;
}

fs_status fs_mlp_grad(fs_mlp* net, const void* x_bf16, const float* y_target, int64_t npts,
                      float* grad, double* loss) {
  if (!net || !x_bf16 || !y_target || !grad) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  if (npts <= 0) {
    fs::set_error("npts must be > 0");
    return FS_E_INVALID;
  }
  fs::Mlp* n = &net->m;
  if (n->failed) return FS_E_DEVICE;
  return mlp_grad_impl(n, x_bf16, y_target, npts, grad, loss);
}

fs_status fs_mlp_train_step(fs_mlp* net, const void* x_bf16, const float* y_target, int64_t npts,
                            float lr, double* loss) {
  if (!net || !x_bf16 || !y_target) {
    fs::set_error("NULL argument");
    return FS_E_INVALID;
  }
  if (npts <= 0 || !(lr > 0.f) || !std::isfinite(lr)) {
    fs::set_error("npts must be > 0 and lr a positive finite number");
    return FS_E_INVALID;
  }
  fs::Mlp* n = &net->m;
  if (n->failed) return FS_E_DEVICE;
  if (fs_status s = mlp_grad_impl(n, x_bf16, y_target, npts, n->g, loss)) return s;
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, n->step)), c2 = (float)(1.0 - std::pow(0.999, n->step));
  hipLaunchKernelGGL(fs::k_mlp_adam, dim3((fs::NPARAM + 255) / 256), dim3(256), 0, n->stream, n->w,
                     n->m, n->v, (const float*)n->g, lr, b1, b2, 1e-8f, c1, c2);
  if (!n->launched("k_mlp_adam")) return FS_E_DEVICE;
  return n->pack() ? FS_OK : FS_E_DEVICE;
}

}  // extern "C"
