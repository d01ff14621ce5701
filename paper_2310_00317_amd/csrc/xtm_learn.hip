// xtm_learn.hip -- gfx950 kernels of the learned early-stop path: early-turn
// features, the 16-128-128-1 loss predictor (BF16 MFMA operands, FP32
// accumulation) with its training step, and particle retirement.
//
// Rounding points of the network (shared with the reference): every GEMM
// operand (standardised inputs, activations, weights, back-propagated
// signals) is rounded FP32 -> BF16 to nearest even; products accumulate in
// FP32; bias, ReLU, sigmoid and loss are FP32.
//
// Matrix-core tiles: v_mfma_f32_16x16x16_bf16 with the operand layout
//   A (16 x 16, rows m, cols k): lane l holds A[l % 16][4 (l / 16) + j], j = 0..3
//   B (16 x 16, rows k, cols n): lane l holds B[4 (l / 16) + j][l % 16]
//   D (16 x 16):                 lane l holds D[4 (l / 16) + j][l % 16]
#include <mutex>

#include "xtm_internal.h"
#include "xtm_maps.h"

namespace xtm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// parameter vector layout (FP32): W1[16][128], b1[128], W2[128][128], b2[128], w3[128], b3
constexpr int kIn = 16, kH = 128;
constexpr int oW1 = 0, oB1 = oW1 + kIn * kH, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH, kParams = oB3 + 1;
static_assert(kParams == 18817, "parameter count");
constexpr int kSamplesPerBlock = 64;  // 4 waves x 16 samples

__device__ __forceinline__ unsigned short to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) {
  return __uint_as_float((unsigned int)h << 16);
}
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// The network lives in LDS for the whole block: W1 and W2 rounded to BF16
// once (36 KB), the bias vectors and w3 in FP32.
struct NetLds {
  unsigned short w1[kIn * kH];   // bf16 W1[k][n]
  unsigned short w2[kH * kH];    // bf16 W2[k][n]
  float b1[kH], b2[kH], w3[kH];  // w3 already rounded to bf16 values
  float b3;
};

__device__ void load_net(NetLds& s, const float* __restrict__ th) {
  for (int i = threadIdx.x; i < kIn * kH; i += blockDim.x) s.w1[i] = to_bf16(th[oW1 + i]);
  for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) s.w2[i] = to_bf16(th[oW2 + i]);
  for (int i = threadIdx.x; i < kH; i += blockDim.x) {
    s.b1[i] = th[oB1 + i];
    s.b2[i] = th[oB2 + i];
    s.w3[i] = from_bf16(to_bf16(th[oW3 + i]));
  }
  if (threadIdx.x == 0) s.b3 = th[oB3];
}

// Forward pass of one wave's 16 samples (rows s0 .. s0+15 of X).  Writes
// bf16 X, H1, H2 and the ReLU masks (z > 0) for rows r0 .. r0+15 of the
// block-local arrays, and returns z3 for lane l < 16 (sample s0 + l).
// The ReLU masks are read back from the activations: bf16(relu(z)) != 0 iff
// z > 0 (only z below half the smallest bf16 subnormal would differ).
__device__ float wave_forward(const NetLds& net, const float* __restrict__ X,
                              const float* __restrict__ norm,
                              int64_t B, int64_t s0, int r0, unsigned short (*sx)[kIn],
                              unsigned short (*h1)[kH], unsigned short (*h2)[kH]) {
  const int l = threadIdx.x & 63;
  const int row = l & 15, quad = l >> 4;
  // layer 1 operand: standardised inputs
  bf16x4 a;
  for (int j = 0; j < 4; ++j) {
    const int f = 4 * quad + j;
    const int64_t s = s0 + row;
    const float x = (s < B) ? X[s * kIn + f] : 0.0f;
    const unsigned short v = to_bf16((x - norm[f]) * norm[kIn + f]);
    a[j] = (short)v;
    sx[r0 + row][f] = v;
  }
  for (int nt = 0; nt < kH / 16; ++nt) {
    bf16x4 b;
    for (int j = 0; j < 4; ++j) b[j] = (short)net.w1[(4 * quad + j) * kH + nt * 16 + row];
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = mfma16(a, b, c);
    for (int j = 0; j < 4; ++j) {
      const int n = nt * 16 + row;
      const float z = c[j] + net.b1[n];
      h1[r0 + 4 * quad + j][n] = to_bf16(z > 0.f ? z : 0.f);
    }
  }
  __syncthreads();
  for (int nt = 0; nt < kH / 16; ++nt) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < kH / 16; ++kt) {
      bf16x4 aa, b;
      for (int j = 0; j < 4; ++j) {
        aa[j] = (short)h1[r0 + row][kt * 16 + 4 * quad + j];
        b[j] = (short)net.w2[(kt * 16 + 4 * quad + j) * kH + nt * 16 + row];
      }
      c = mfma16(aa, b, c);
    }
    for (int j = 0; j < 4; ++j) {
      const int n = nt * 16 + row;
      const float z = c[j] + net.b2[n];
      h2[r0 + 4 * quad + j][n] = to_bf16(z > 0.f ? z : 0.f);
    }
  }
  __syncthreads();
  float z3 = 0.f;
  if (l < 16) {
    float acc = 0.f;
    for (int k = 0; k < kH; ++k) acc += from_bf16(h2[r0 + l][k]) * net.w3[k];
    z3 = acc + net.b3;
  }
  return z3;
}

struct FwdLds {
  NetLds net;
  unsigned short x[kSamplesPerBlock][kIn];
  unsigned short h1[kSamplesPerBlock][kH];
  unsigned short h2[kSamplesPerBlock][kH];
};

// Each block loads the network once and then runs 64-sample tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... (the loop bound is uniform over
// the block, so every wave meets the same barriers).
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ theta,
                                                     const float* __restrict__ norm,
                                                     const float* __restrict__ X, int64_t B,
                                                     float* __restrict__ logit) {
  __shared__ FwdLds s;
  load_net(s.net, theta);
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t n_tiles = (B + kSamplesPerBlock - 1) / kSamplesPerBlock;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t s0 = t * kSamplesPerBlock + 16 * w;
    const float z = wave_forward(s.net, X, norm, B, s0, 16 * w, s.x, s.h1, s.h2);
    if (l < 16 && s0 + l < B) logit[s0 + l] = z;
    __syncthreads();
  }
}

struct GradLds {
  NetLds net;
  unsigned short x[kSamplesPerBlock][kIn];
  unsigned short h1[kSamplesPerBlock][kH];
  unsigned short h2[kSamplesPerBlock][kH];   // H2, then reused for bf16 dZ1
  unsigned short dz2[kSamplesPerBlock][kH];  // bf16 dZ2
  float gb1[4][kH];                          // per-wave partial sums of unrounded dZ1
  float dz3[kSamplesPerBlock];               // unrounded dL/dz3
  float lossv[kSamplesPerBlock];
};

// Per-block partial gradient (mean over the whole batch B) into part[blockIdx][kParams]
// and the block's summed loss into loss_part[blockIdx].
__global__ void __launch_bounds__(256) k_mlp_grad(const float* __restrict__ theta,
                                                  const float* __restrict__ norm,
                                                  const float* __restrict__ X,
                                                  const float* __restrict__ Y, int64_t B,
                                                  float pos_weight, float* __restrict__ part,
                                                  float* __restrict__ loss_part) {
  __shared__ GradLds s;
  load_net(s.net, theta);
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row = l & 15, quad = l >> 4;
  const int64_t base = (int64_t)blockIdx.x * kSamplesPerBlock;
  const int64_t s0 = base + 16 * w;
  const float z = wave_forward(s.net, X, norm, B, s0, 16 * w, s.x, s.h1, s.h2);
  if (l < 16) {
    const int64_t si = s0 + l;
    float d = 0.f, lv = 0.f;
    if (si < B) {
      const float y = Y[si];
      const float sg = 1.0f / (1.0f + expf(-z));
      d = (sg * (pos_weight * y + (1.0f - y)) - pos_weight * y) / (float)B;
      const float lz = log1pf(expf(-fabsf(z)));
      const float sp_neg = fmaxf(-z, 0.f) + lz, sp_pos = fmaxf(z, 0.f) + lz;
      lv = pos_weight * y * sp_neg + (1.0f - y) * sp_pos;
    }
    s.dz3[16 * w + l] = d;
    s.lossv[16 * w + l] = lv;
  }
  __syncthreads();
  float* g = part + (size_t)blockIdx.x * kParams;
  // dZ2 = bf16(dz3) bf16(w3) masked; b2, w3, b3 partial sums (fixed order)
  for (int n = threadIdx.x; n < kH; n += blockDim.x) {
    float gb2 = 0.f, gw3 = 0.f;
    for (int r = 0; r < kSamplesPerBlock; ++r) {
      const float dq = from_bf16(to_bf16(s.dz3[r]));
      const float d2 = s.h2[r][n] ? dq * s.net.w3[n] : 0.f;
      s.dz2[r][n] = to_bf16(d2);
      gb2 += d2;
      gw3 += from_bf16(s.h2[r][n]) * dq;
    }
    g[oB2 + n] = gb2;
    g[oW3 + n] = gw3;
  }
  if (threadIdx.x == 0) {
    float gb3 = 0.f, ls = 0.f;
    for (int r = 0; r < kSamplesPerBlock; ++r) {
      gb3 += s.dz3[r];
      ls += s.lossv[r];
    }
    g[oB3] = gb3;
    loss_part[blockIdx.x] = ls;
  }
  __syncthreads();
  // dH1 = bf16(dZ2) bf16(W2)^T per wave; dZ1 = dH1 masked (mask from H1),
  // stored as bf16 in the H2 slot; unrounded column sums give the b1 partial
  for (int nt = 0; nt < kH / 16; ++nt) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < kH / 16; ++kt) {
      bf16x4 a, b;
      for (int j = 0; j < 4; ++j) {
        a[j] = (short)s.dz2[16 * w + row][kt * 16 + 4 * quad + j];
        b[j] = (short)s.net.w2[(nt * 16 + row) * kH + kt * 16 + 4 * quad + j];
      }
      c = mfma16(a, b, c);
    }
    float colsum = 0.f;
    for (int j = 0; j < 4; ++j) {
      const int r = 16 * w + 4 * quad + j, n = nt * 16 + row;
      const float d1 = s.h1[r][n] ? c[j] : 0.f;
      s.h2[r][n] = to_bf16(d1);
      colsum += d1;
    }
    // lanes l, l^16, l^32, l^48 hold the same column: fixed-order combine
    colsum += __shfl_xor(colsum, 16, 64);
    colsum += __shfl_xor(colsum, 32, 64);
    if (quad == 0) s.gb1[w][nt * 16 + row] = colsum;
  }
  __syncthreads();
  for (int n = threadIdx.x; n < kH; n += blockDim.x)
    g[oB1 + n] = ((s.gb1[0][n] + s.gb1[1][n]) + s.gb1[2][n]) + s.gb1[3][n];
  // weight gradients with K = samples of the block (4 k-steps of 16)
  // W2[j1][n2] = sum_s H1[s][j1] dZ2[s][n2]: 64 output tiles, 16 per wave
  for (int t = w; t < 64; t += 4) {
    const int mt = t >> 3, nt = t & 7;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < kSamplesPerBlock / 16; ++kt) {
      bf16x4 a, b;
      for (int j = 0; j < 4; ++j) {
        a[j] = (short)s.h1[kt * 16 + 4 * quad + j][mt * 16 + row];
        b[j] = (short)s.dz2[kt * 16 + 4 * quad + j][nt * 16 + row];
      }
      c = mfma16(a, b, c);
    }
    for (int j = 0; j < 4; ++j) g[oW2 + (mt * 16 + 4 * quad + j) * kH + nt * 16 + row] = c[j];
  }
  // W1[f][j1] = sum_s X[s][f] dZ1[s][j1]: 8 output tiles, 2 per wave
  for (int nt = w; nt < 8; nt += 4) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < kSamplesPerBlock / 16; ++kt) {
      bf16x4 a, b;
      for (int j = 0; j < 4; ++j) {
        a[j] = (short)s.x[kt * 16 + 4 * quad + j][row];
        b[j] = (short)s.h2[kt * 16 + 4 * quad + j][nt * 16 + row];   // bf16 dZ1
      }
      c = mfma16(a, b, c);
    }
    for (int j = 0; j < 4; ++j) g[oW1 + (4 * quad + j) * kH + nt * 16 + row] = c[j];
  }
}

// grad[i] = sum over blocks b = 0..nb-1 (in order) of part[b][i]; loss likewise.
__global__ void __launch_bounds__(256) k_mlp_reduce(const float* __restrict__ part, int nb,
                                                    const float* __restrict__ loss_part,
                                                    float* __restrict__ grad,
                                                    float* __restrict__ loss, int64_t B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kParams) {
    float acc = 0.f;
    for (int b = 0; b < nb; ++b) acc += part[(size_t)b * kParams + i];
    grad[i] = acc;
  }
  if (i == 0 && loss) {
    float acc = 0.f;
    for (int b = 0; b < nb; ++b) acc += loss_part[b];
    *loss = acc / (float)B;
  }
}

// Adam (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// theta <- theta - lr mhat / (sqrt(vhat) + eps), bias-corrected with step t >= 1.
// The update is evaluated in FP64 from the FP32 masters and moments (b1 = 0.9,
// b2 = 0.999 exactly, not their FP32 roundings) and stored back in FP32.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ theta, float* __restrict__ m,
                                              float* __restrict__ v,
                                              const float* __restrict__ grad, int step, float lr,
                                              double b1, double b2, double eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  const double g = grad[i];
  const double mi = b1 * (double)m[i] + (1.0 - b1) * g;
  const double vi = b2 * (double)v[i] + (1.0 - b2) * g * g;
  m[i] = (float)mi;
  v[i] = (float)vi;
  const double mh = mi / (1.0 - pow(b1, (double)step));
  const double vh = vi / (1.0 - pow(b2, (double)step));
  theta[i] = (float)((double)theta[i] - (double)lr * mh / (sqrt(vh) + eps));
}

// He-normal initialisation: weights std sqrt(2/fan_in) times the Philox
// deviate of (seed, index j, 0, 0, 0); biases zero.
__global__ void __launch_bounds__(256) k_mlp_init(float* __restrict__ theta,
                                                  unsigned long long seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  double std = 0.0;
  if (i < oB1) std = sqrt(2.0 / kIn);
  else if (i >= oW2 && i < oB2) std = sqrt(2.0 / kH);
  else if (i >= oW3 && i < oB3) std = sqrt(2.0 / kH);
  theta[i] = std == 0.0 ? 0.0f : (float)(std * xtmm::gauss_at(seed, i, 0, 0, 0));
}

// ------------------------------------------------------------- features
constexpr int kWin = 512, kRecTurns = 1024;

__device__ __forceinline__ int rev9(int v) { return (int)(__brev((unsigned)v) >> 23); }

struct FeatLds {
  float2 z[4][kWin];  // x first half, y first half, x second half, y second half
  double jx[kRecTurns], jy[kRecTurns];
  double red[256];
  float fred[256];
  int ired[256];
};

__device__ double block_sum(double v, double* buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) buf[threadIdx.x] += buf[threadIdx.x + s];
    __syncthreads();
  }
  const double r = buf[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) buf[threadIdx.x] = fmax(buf[threadIdx.x], buf[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = buf[0];
  __syncthreads();
  return r;
}

// Argmax of |z[a][k]| over k (first index on ties), then the Hann three-point
// interpolation; returns ((k + d) / 512) mod 1.
__device__ float tune_of(FeatLds& s, int a) {
  float best = -1.f;
  int bi = 0;
  for (int k = threadIdx.x; k < kWin; k += blockDim.x) {
    const float2 v = s.z[a][k];
    const float m = sqrtf(v.x * v.x + v.y * v.y);
    if (m > best) {
      best = m;
      bi = k;
    }
  }
  s.fred[threadIdx.x] = best;
  s.ired[threadIdx.x] = bi;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      const float o = s.fred[threadIdx.x + st];
      const int oi = s.ired[threadIdx.x + st];
      if (o > s.fred[threadIdx.x] || (o == s.fred[threadIdx.x] && oi < s.ired[threadIdx.x])) {
        s.fred[threadIdx.x] = o;
        s.ired[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int k = s.ired[0];
  __syncthreads();
  auto mag = [&](int kk) {
    const float2 v = s.z[a][(kk + kWin) % kWin];
    return sqrtf(v.x * v.x + v.y * v.y);
  };
  const float am = mag(k - 1), b = mag(k), c = mag(k + 1);
  const float d = 2.0f * (c - am) / (am + 2.0f * b + c);
  float q = ((float)k + d) / (float)kWin;
  q = q - floorf(q);
  return q;
}

// One workgroup of 256 per particle: record [1024][4][n] (x, px, y, py at
// element 0 at the start of each turn) -> 16 features (definitions in
// include/xtm.h).  The action statistics are taken in FP64 from the FP32
// record (two passes for the spread); the spectra are FP32 FFTs.
// tw[k] = (cos, sin)(2 pi k / 512) for k < 256, win[n] = sin^2(pi n / 512).
__global__ void __launch_bounds__(256) k_features(const float* __restrict__ rec, int64_t n,
                                                  double bx, double ax, double by, double ay,
                                                  double emit, double r_ap,
                                                  const float2* __restrict__ tw,
                                                  const float* __restrict__ win,
                                                  float* __restrict__ out) {
  __shared__ FeatLds s;
  const int64_t p = blockIdx.x;
  if (p >= n) return;
  const double sbx = sqrt(bx), sby = sqrt(by);
  double rmax = 0.0, amax = 0.0;
  for (int t = threadIdx.x; t < kRecTurns; t += blockDim.x) {
    const double x = rec[((size_t)t * 4 + 0) * n + p], px = rec[((size_t)t * 4 + 1) * n + p];
    const double y = rec[((size_t)t * 4 + 2) * n + p], py = rec[((size_t)t * 4 + 3) * n + p];
    const double ux = x / sbx, pux = (ax * x + bx * px) / sbx;
    const double uy = y / sby, puy = (ay * y + by * py) / sby;
    const double jx = 0.5 * (ux * ux + pux * pux), jy = 0.5 * (uy * uy + puy * puy);
    s.jx[t] = jx;
    s.jy[t] = jy;
    rmax = fmax(rmax, sqrt(x * x + y * y));
    amax = fmax(amax, 2.0 * (jx + jy) / emit);
    const int h = t >= kWin, tt = t - h * kWin;
    const float wv = win[tt];
    s.z[2 * h + 0][rev9(tt)] = make_float2(wv * (float)ux, -wv * (float)pux);
    s.z[2 * h + 1][rev9(tt)] = make_float2(wv * (float)uy, -wv * (float)puy);
  }
  __syncthreads();
  // radix-2 decimation-in-time FFT, 4 transforms x 256 butterflies per stage
  for (int half = 1; half < kWin; half <<= 1) {
    for (int task = threadIdx.x; task < 4 * (kWin / 2); task += blockDim.x) {
      const int a = task / (kWin / 2), bfly = task % (kWin / 2);
      const int grp = bfly / half, pos = bfly % half;
      const int i0 = grp * 2 * half + pos, i1 = i0 + half;
      const float2 wt = tw[pos * (kWin / 2 / half)];   // exp(-i 2 pi k / 512) = (cos, -sin)
      const float2 v1 = s.z[a][i1], v0 = s.z[a][i0];
      const float tr = wt.x * v1.x + wt.y * v1.y;
      const float ti = wt.x * v1.y - wt.y * v1.x;
      s.z[a][i1] = make_float2(v0.x - tr, v0.y - ti);
      s.z[a][i0] = make_float2(v0.x + tr, v0.y + ti);
    }
    __syncthreads();
  }
  const float qx1 = tune_of(s, 0), qy1 = tune_of(s, 1), qx2 = tune_of(s, 2), qy2 = tune_of(s, 3);
  // action statistics: sums, first and last quarters, then the spread
  constexpr int kQ = kRecTurns / 4;
  double sx = 0.0, sy = 0.0, fx0 = 0.0, fx1 = 0.0, fy0 = 0.0, fy1 = 0.0;
  for (int t = threadIdx.x; t < kRecTurns; t += blockDim.x) {
    sx += s.jx[t];
    sy += s.jy[t];
    if (t < kQ) { fx0 += s.jx[t]; fy0 += s.jy[t]; }
    if (t >= kRecTurns - kQ) { fx1 += s.jx[t]; fy1 += s.jy[t]; }
  }
  sx = block_sum(sx, s.red);
  sy = block_sum(sy, s.red);
  fx0 = block_sum(fx0, s.red);
  fx1 = block_sum(fx1, s.red);
  fy0 = block_sum(fy0, s.red);
  fy1 = block_sum(fy1, s.red);
  const double mx = sx / kRecTurns, my = sy / kRecTurns;
  double vx = 0.0, vy = 0.0;
  for (int t = threadIdx.x; t < kRecTurns; t += blockDim.x) {
    vx += (s.jx[t] - mx) * (s.jx[t] - mx);
    vy += (s.jy[t] - my) * (s.jy[t] - my);
  }
  vx = block_sum(vx, s.red);
  vy = block_sum(vy, s.red);
  rmax = block_max(rmax, s.red);
  amax = block_max(amax, s.red);
  if (threadIdx.x == 0) {
    const double e = 1e-6 * emit;
    auto cdiff = [](double a, double b) {
      double d = fabs(a - b);
      d = d - floor(d);
      return fmin(d, 1.0 - d);
    };
    const double a0x = sqrt(2.0 * s.jx[0] / emit), a0y = sqrt(2.0 * s.jy[0] / emit);
    const double r0 = sqrt(a0x * a0x + a0y * a0y);
    float* o = out + (size_t)p * 16;
    o[0] = (float)a0x;
    o[1] = (float)a0y;
    o[2] = (float)r0;
    o[3] = (float)atan2(a0y, a0x);
    o[4] = qx1;
    o[5] = qy1;
    o[6] = qx2;
    o[7] = qy2;
    o[8] = (float)log10(cdiff(qx2, qx1) + 1e-12);
    o[9] = (float)log10(cdiff(qy2, qy1) + 1e-12);
    o[10] = (float)((fx1 / kQ + e) / (fx0 / kQ + e) - 1.0);
    o[11] = (float)((fy1 / kQ + e) / (fy0 / kQ + e) - 1.0);
    o[12] = (float)(sqrt(vx / kRecTurns) / (mx + e));
    o[13] = (float)(sqrt(vy / kRecTurns) / (my + e));
    o[14] = (float)(rmax / r_ap);
    o[15] = (float)(amax / (r0 * r0 + 1e-6));
  }
}

// Column mean and 1/std of features over rows with mask != 0 (one
// workgroup, fixed reduction order): thread t accumulates rows t, t + 256,
// ... (each row's 16 values from one 64-byte stretch), then the
// 33 sums are reduced pairwise across the workgroup; norm = [mean[16],
// inv_std[16]].
__global__ void __launch_bounds__(256) k_feature_stats(const float* __restrict__ f,
                                                       const int32_t* __restrict__ mask,
                                                       int64_t n, float* __restrict__ norm) {
  __shared__ double acc[33][256];
  double s1[16], s2[16], cnt = 0.0;
  for (int c = 0; c < 16; ++c) s1[c] = s2[c] = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    if (mask && !mask[i]) continue;
    const float* row = f + i * 16;
    for (int c = 0; c < 16; ++c) {
      const double v = row[c];
      s1[c] += v;
      s2[c] += v * v;
    }
    cnt += 1.0;
  }
  for (int c = 0; c < 16; ++c) {
    acc[c][threadIdx.x] = s1[c];
    acc[16 + c][threadIdx.x] = s2[c];
  }
  acc[32][threadIdx.x] = cnt;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 33; ++k) acc[k][threadIdx.x] += acc[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 16) {
    const int c = threadIdx.x;
    const double nn = acc[32][0];
    const double m = nn > 0 ? acc[c][0] / nn : 0.0;
    const double var = nn > 0 ? acc[16 + c][0] / nn - m * m : 1.0;
    norm[c] = (float)m;
    norm[16 + c] = (float)(1.0 / sqrt(var > 1e-30 ? var : 1.0));
  }
}

// Retire alive particles whose logit >= threshold unless audited: audited iff
// the first Philox word of (key audit_seed, counter (pid_lo, pid_hi,
// 0xFFFFFFFF, 0)) is below audit_threshold.  Retired particles get state 2.
// counts[0] += retired, counts[1] += audited (alive, eligible by logit);
// audit_flags[p] = 1 for each audited particle when the array is given.
__global__ void __launch_bounds__(256) k_retire(SoA P, const int32_t* __restrict__ idx,
                                                const int32_t* __restrict__ ctrl,
                                                const float* __restrict__ logit,
                                                float threshold, unsigned long long audit_seed,
                                                unsigned int audit_threshold,
                                                unsigned int* __restrict__ counts,
                                                int32_t* __restrict__ audit_flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ctrl[0]) return;
  const int32_t p = idx[i];
  if (P.state[p] != 1) return;
  if (!(logit[p] >= threshold)) return;
  const unsigned long long pid = (unsigned long long)P.pid[p];
  xtmm::U4 c{(unsigned int)pid, (unsigned int)(pid >> 32), 0xFFFFFFFFu, 0u};
  const xtmm::U4 w = xtmm::philox4x32_10(c, (unsigned int)audit_seed,
                                         (unsigned int)(audit_seed >> 32));
  if (w.a < audit_threshold) {
    atomicAdd(&counts[1], 1u);
    if (audit_flags) audit_flags[p] = 1;
    return;
  }
  P.state[p] = 2;
  atomicAdd(&counts[0], 1u);
}

// Score of the retire rule without the network: -max(f8, f9), the larger of
// the two tune-diffusion features negated (a NaN feature gives a NaN score,
// which no threshold retires).
__global__ void __launch_bounds__(256) k_rule_score(const float* __restrict__ f, int64_t n,
                                                    float* __restrict__ score) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float a = f[i * kIn + 8], b = f[i * kIn + 9];
  score[i] = (a != a || b != b) ? __builtin_nanf("") : -(a > b ? a : b);
}

// Rows perm[start .. start+B-1] of (X, Y) into the contiguous batch (Xb, Yb).
__global__ void __launch_bounds__(256) k_gather_rows(const float* __restrict__ X,
                                                     const float* __restrict__ Y,
                                                     const int32_t* __restrict__ perm,
                                                     int64_t B, float* __restrict__ Xb,
                                                     float* __restrict__ Yb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * kIn) return;
  const int64_t r = i / kIn, f = i - r * kIn;
  const int64_t src = perm[r];
  Xb[i] = X[src * kIn + f];
  if (f == 0) Yb[r] = Y[src];
}

// ------------------------------------------------------------- launchers
hipError_t launch_gather_rows(const float* X, const float* Y, const int32_t* perm, int64_t B,
                              float* Xb, float* Yb, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((B * kIn + 255) / 256)), dim3(256), 0, s, X, Y,
                     perm, B, Xb, Yb);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* theta, const float* norm, const float* X, int64_t B,
                              float* logit, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  // at most two blocks per compute unit: each loads the network once
  const int64_t tiles = (B + kSamplesPerBlock - 1) / kSamplesPerBlock;
  const unsigned nb = (unsigned)(tiles < 512 ? tiles : 512);
  hipLaunchKernelGGL(k_mlp_forward, dim3(nb), dim3(256), 0, s, theta, norm, X, B, logit);
  return hipGetLastError();
}

int64_t mlp_workspace_floats(int64_t B) {
  const int64_t nb = (B + kSamplesPerBlock - 1) / kSamplesPerBlock;
  return nb * (kParams + 1);
}

// Workspace of the allocation-free gradient entry point (batches of at most
// kMlpNoAllocMaxBatch rows).  Every launch of k_mlp_grad writes all the
// partials the reduction then reads, so the array never needs clearing.  In
// host code `scratch` names a host-side stand-in: kernels receive the device
// address looked up below, never the symbol itself.
constexpr int64_t kNoAllocFloats =
    ((kMlpNoAllocMaxBatch + kSamplesPerBlock - 1) / kSamplesPerBlock) * (kParams + 1);
static __device__ __align__(256) float scratch[kNoAllocFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t mlp_noalloc_workspace(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

hipError_t launch_mlp_grad(const float* theta, const float* norm, const float* X, const float* Y,
                           int64_t B, float pos_weight, float* grad, float* loss, float* work,
                           hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const int nb = (int)((B + kSamplesPerBlock - 1) / kSamplesPerBlock);
  float* part = work;
  float* lpart = work + (size_t)nb * kParams;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, theta, norm, X, Y, B, pos_weight,
                     part, lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, s, part, nb, lpart,
                     grad, loss, B);
  return hipGetLastError();
}

hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, theta, m, v, grad, step,
                     lr, 0.9, 0.999, 1e-8);
  return hipGetLastError();
}

hipError_t launch_mlp_init(float* theta, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_init, dim3((kParams + 255) / 256), dim3(256), 0, s, theta, seed);
  return hipGetLastError();
}

hipError_t launch_features(const float* rec, int64_t n, const double twiss4[4], double emit,
                           double r_ap, const float2* tw, const float* win, float* out,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)n), dim3(256), 0, s, rec, n, twiss4[0], twiss4[1],
                     twiss4[2], twiss4[3], emit, r_ap, tw, win, out);
  return hipGetLastError();
}

hipError_t launch_feature_stats(const float* f, const int32_t* mask, int64_t n, float* norm,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_feature_stats, dim3(1), dim3(256), 0, s, f, mask, n, norm);
  return hipGetLastError();
}

hipError_t launch_retire(SoA P, const int32_t* idx, const int32_t* ctrl, int64_t grid_upper,
                         const float* logit, float threshold, unsigned long long audit_seed,
                         unsigned int audit_threshold, unsigned int* counts, int32_t* audit_flags,
                         hipStream_t s) {
  if (grid_upper <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_retire, dim3((unsigned)((grid_upper + 255) / 256)), dim3(256), 0, s, P, idx,
                     ctrl, logit, threshold, audit_seed, audit_threshold, counts, audit_flags);
  return hipGetLastError();
}

hipError_t launch_rule_score(const float* f, int64_t n, float* score, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rule_score, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f, n, score);
  return hipGetLastError();
}

}  // namespace xtm
