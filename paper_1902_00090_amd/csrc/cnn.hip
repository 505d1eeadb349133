// Convolutional subspace predictor (Sec. 3 CNN paragraph; Methods): forward,
// backward and Adam on gfx950, bf16 activations with FP32 accumulation on the
// matrix cores.
//
// The paper's architecture figure is not available; the layer list (the
// reading used throughout) is an encoder-decoder of eight 3x3 convolutions,
// zero padding 1, ReLU after all but the last:
//   1->32, 32->64 (stride 2), 64->128 (stride 2), 128->128,
//   x2 nearest upsample + 128->64, x2 nearest upsample + 64->32, 32->32,
//   32->2k (linear).
// The input is (eps - 2.085) / (12.25 - 2.085); output channels (2j, 2j+1)
// are the real and imaginary parts of v_j (complex inputs/outputs as images
// of depth 2, Methods).
//
// Layouts: activations NHWC bf16 with the channel count padded to a multiple
// of 16 (padded channels hold zeros); the normalised input is FP32 [B][H][W];
// the last layer's output is FP32 NHWC with 2k channels.  Master weights,
// gradients and Adam moments are FP32 in [cout][cin][3][3] + [cout] per
// layer; the GEMM copies are bf16, forward Wf[tap][coutp][cinp] and
// backward-data Wb[tap][cinp][coutp].
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 with the GEMM
// rows = output channels and columns = pixels: lane l holds A[l%16][8(l/16)+i],
// B[8(l/16)+i][l%16] (i < 8) and receives C[4(l/16)+i][l%16] (i < 4), so one
// lane's results are 4 consecutive channels of one pixel (an 8-byte store).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "common.h"
#include "op.h"
#include "resloss.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

#define NL 8
#define CNN_EPS_LO 2.085f
#define CNN_EPS_HI 12.25f

enum { MAP_S1 = 0, MAP_S2 = 1, MAP_UP = 2 };

struct CnnLayer {
  int cin, cout, stride, up, relu;
  int cinp, coutp;           // padded channel counts (multiples of 16; cin 1 stays 1)
  int Hin, Win, Hout, Wout;  // per-image grid sizes
  size_t woff, boff;         // offsets of weights / bias in the parameter vector
  int mode;                  // MAP_S1, MAP_S2 or MAP_UP
};

struct dd_cnn {
  int nx, ny, maxB, k;
  int cin0;                  // input planes: 1 (permittivity) or 3 (+ effective-index field)
  CnnLayer L[NL];
  size_t nparams = 0;
  float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
  int adam_t = 0;
  bf16* wf[NL] = {};
  bf16* wb[NL] = {};
  float* x0 = nullptr;       // normalised input planes [B][cin0][H][W]
  double* iscale = nullptr;  // [maxB] effective-index field scale sqrt(D) / ||F||
  // residual-loss scratch (allocated on first use): V = output fields, W = A V,
  // r = b - W c, s = A^H r
  float2 *rl_V = nullptr, *rl_W = nullptr, *rl_r = nullptr, *rl_s = nullptr;
  bf16* act[NL] = {};        // act[l] = output of layer l (l < NL-1), NHWC bf16
  float* out = nullptr;      // last layer output [B][H][W][2k]
  bf16* dz[NL] = {};         // gradient w.r.t. the pre-activation of layer l
  float* wpart = nullptr;    // split partial weight gradients
  size_t wpart_elems = 0;
  float* lpart = nullptr;    // loss partial sums
  float* biaspad = nullptr;  // [NL][256] zero-padded FP32 biases for the GEMM epilogue
  std::vector<void*> allocs;
};

// ------------------------------------------------------------ helpers ----
__device__ __forceinline__ bf16x8 load8(const bf16* p) {
  return __builtin_bit_cast(bf16x8, *(const u32x4*)p);
}
__device__ __forceinline__ bf16x8 zero8() {
  return __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u});
}
__device__ __forceinline__ float bf2f(bf16 v) { return (float)v; }

// Source pixel (in the layer-input grid) that output pixel (y, x) reads at
// tap (dy, dx); false when it falls in the zero padding.
__device__ __forceinline__ bool fwd_src(int mode, int y, int x, int dy, int dx, int Hin, int Win,
                                        int Hout, int Wout, int& ys, int& xs) {
  if (mode == MAP_S1) {
    ys = y + dy - 1; xs = x + dx - 1;
    return ys >= 0 && ys < Hin && xs >= 0 && xs < Win;
  } else if (mode == MAP_S2) {
    ys = 2 * y + dy - 1; xs = 2 * x + dx - 1;
    return ys >= 0 && ys < Hin && xs >= 0 && xs < Win;
  } else {  // upsampled grid has the output's size
    const int uy = y + dy - 1, ux = x + dx - 1;
    ys = uy >> 1; xs = ux >> 1;
    return uy >= 0 && uy < Hout && ux >= 0 && ux < Wout;
  }
}

// Backward-data gather: for layer-input pixel (y, x) and entry e, the layer-
// output pixel whose gradient reaches it through tap e % 9 (for upsampled
// layers e / 9 picks one of the four upsampled positions of (y, x)).
__device__ __forceinline__ bool bwd_src(int mode, int e, int y, int x, int Hout, int Wout,
                                        int& py, int& px, int& tap) {
  tap = e % 9;
  const int dy = tap / 3, dx = tap % 3;
  if (mode == MAP_S1) {
    py = y - dy + 1; px = x - dx + 1;
    return py >= 0 && py < Hout && px >= 0 && px < Wout;
  } else if (mode == MAP_S2) {
    const int ty = y - dy + 1, tx = x - dx + 1;
    if (ty < 0 || tx < 0 || (ty & 1) || (tx & 1)) return false;
    py = ty >> 1; px = tx >> 1;
    return py < Hout && px < Wout;
  } else {
    const int s = e / 9;
    const int uy = 2 * y + (s >> 1), ux = 2 * x + (s & 1);
    py = uy - dy + 1; px = ux - dx + 1;
    return py >= 0 && py < Hout && px >= 0 && px < Wout;
  }
}

// ------------------------------------------------- implicit GEMM (MFMA) ----
// Forward (BWD = false): out[p][r] = act(bias[r] + sum_{tap,c} Wf[tap][r][c] *
//   src[map(p, tap)][c]), p over output pixels, r < M = coutp.
// Backward data (BWD = true): dzprev[q][r] = mask(q, r) * sum_{e,c} Wb[tap][r][c]
//   * dz[gather(q, e)][c], q over layer-input pixels, r < M = cinp, mask = the
//   ReLU mask of the previous layer's output (the layer input).
// MT = M / 16 row tiles per wave, NT pixel tiles of 16 per wave, 4 waves.
struct GemmArgs {
  const bf16* src;       // forward: layer input; backward: dz of this layer
  const bf16* W;         // Wf or Wb
  const float* bias;     // forward only
  const bf16* mask;      // backward: layer input activations (ReLU mask)
  bf16* out;             // bf16 result (NHWC, M channels)
  float* outf;           // final layer: FP32 result with nreal channels
  int nreal;             // channels of outf
  int B, Hq, Wq;         // grid of the result pixels
  int Hs, Ws;            // grid of the source pixels
  int Hout, Wout;        // layer output grid (for the map functions)
  int Ksrc;              // channels of the source (multiple of 32)
  int M;                 // result channels (= 16 MT)
  int mode, entries, relu;
};

template <int MT, int NT, bool BWD>
__global__ __launch_bounds__(256) void k_conv_gemm(GemmArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int npix = a.B * a.Hq * a.Wq;
  const int pbase = (blockIdx.x * 4 + wave) * NT * 16;
  f32x4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  int pb[NT], py[NT], px[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int p = pbase + j * 16 + (lane & 15);
    const int pc = min(p, npix - 1);
    pb[j] = pc / (a.Hq * a.Wq);
    const int rem = pc - pb[j] * a.Hq * a.Wq;
    py[j] = rem / a.Wq;
    px[j] = rem - py[j] * a.Wq;
    if (p >= npix) pb[j] = -1;
  }
  const int kq = 8 * (lane >> 4);
  for (int e = 0; e < a.entries; ++e) {
    const bf16* srcp[NT];
    int tap = e;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      srcp[j] = nullptr;
      if (pb[j] < 0) continue;
      int sy, sx;
      bool ok;
      if (!BWD) {
        ok = fwd_src(a.mode, py[j], px[j], e / 3, e % 3, a.Hs, a.Ws, a.Hout, a.Wout, sy, sx);
      } else {
        ok = bwd_src(a.mode, e, py[j], px[j], a.Hout, a.Wout, sy, sx, tap);
      }
      if (ok) srcp[j] = a.src + ((size_t)(pb[j] * a.Hs + sy) * a.Ws + sx) * a.Ksrc;
    }
    if (BWD) tap = e % 9;
    const bf16* wt = a.W + (size_t)tap * a.M * a.Ksrc;
    for (int c0 = 0; c0 < a.Ksrc; c0 += 32) {
      bf16x8 bv[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j) bv[j] = srcp[j] ? load8(srcp[j] + c0 + kq) : zero8();
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const bf16x8 av = load8(wt + (size_t)(i * 16 + (lane & 15)) * a.Ksrc + c0 + kq);
#pragma unroll
        for (int j = 0; j < NT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  // epilogue: lane holds channels r0..r0+3 of pixel column (lane & 15)
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int p = pbase + j * 16 + (lane & 15);
    if (p >= npix) continue;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const int r0 = i * 16 + 4 * (lane >> 4);
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[q] = acc[i][j][q];
        if (!BWD) {
          v[q] += a.bias[r0 + q];
          if (a.relu) v[q] = fmaxf(v[q], 0.f);
        }
      }
      if (BWD) {
        const bf16* mk = a.mask + (size_t)p * a.M + r0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (!(bf2f(mk[q]) > 0.f)) v[q] = 0.f;
      }
      if (a.outf) {
        float* o = a.outf + (size_t)p * a.nreal + r0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (r0 + q < a.nreal) o[q] = v[q];
      } else {
        bf16 h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = (bf16)v[q];
        *(u32x2*)(a.out + (size_t)p * a.M + r0) = __builtin_bit_cast(u32x2, h);
      }
    }
  }
}

// ---------------------------------------- LDS-tiled forward convolution ----
// Forward pass of the stride-1 layers, plain (MAP_S1) or after a x2 nearest
// upsample (MAP_UP), and (BWD) the backward-data pass of the plain stride-1
// layers: the gradient at a layer-input pixel gathers dz through the kernel
// rotated by 180 degrees (tap t reads weight tap 8 - t of the transposed
// copy), masked by the ReLU of the layer input.  A workgroup computes a 4 x 64 tile of output pixels of
// one image for all M = 16 MT output channels.  For every 32 input channels
// the 6 x 66 input patch (halo included; zero padding and the upsampling are
// resolved while staging) is written once to LDS and read there by all nine
// taps, so each source value is fetched from memory once instead of nine
// times.  Wave w owns output row w of the tile (four pixel tiles of 16).  The
// weights come from the L2-resident packed copy.  Operand layouts are those of
// k_conv_gemm.
#define CT_TH 4
#define CT_TW 64
#define CT_PH (CT_TH + 2)
#define CT_PW (CT_TW + 2)
#define CT_PS 40   // bf16 per staged pixel: 32 channels + 8 of padding (80-byte stride)
template <int MT, bool BWD = false>
__global__ __launch_bounds__(256) void k_conv_tile(GemmArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 patch[CT_PH * CT_PW * CT_PS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x0 = blockIdx.x * CT_TW, y0 = blockIdx.y * CT_TH, b = blockIdx.z;
  const int Hq = a.Hq, Wq = a.Wq;
  const bool up = (a.mode == MAP_UP);
  f32x4 acc[MT][4];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = 8 * (lane >> 4);
  for (int c0 = 0; c0 < a.Ksrc; c0 += 32) {
    for (int u = threadIdx.x; u < CT_PH * CT_PW * 4; u += 256) {
      const int pix = u >> 2, q = u & 3;
      const int py = pix / CT_PW, px = pix - py * CT_PW;
      const int uy = y0 + py - 1, ux = x0 + px - 1;   // conv-input grid (= output grid)
      u32x4 v = u32x4{0u, 0u, 0u, 0u};
      if (uy >= 0 && uy < Hq && ux >= 0 && ux < Wq) {
        const int sy = up ? (uy >> 1) : uy, sx = up ? (ux >> 1) : ux;
        v = *(const u32x4*)(a.src + ((size_t)(b * a.Hs + sy) * a.Ws + sx) * a.Ksrc + c0 + 8 * q);
      }
      *(u32x4*)(patch + pix * CT_PS + 8 * q) = v;
    }
    __syncthreads();
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3, dx = t - 3 * (t / 3);
      bf16x8 bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bv[j] = *(const bf16x8*)(patch + ((wave + dy) * CT_PW + 16 * j + (lane & 15) + dx) * CT_PS + kq);
      const bf16* wt = a.W + (size_t)(BWD ? 8 - t : t) * a.M * a.Ksrc + c0 + kq;
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const bf16x8 av = load8(wt + (size_t)(i * 16 + (lane & 15)) * a.Ksrc);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int y = y0 + wave;
  if (y >= Hq) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int x = x0 + 16 * j + (lane & 15);
    if (x >= Wq) continue;
    const size_t p = ((size_t)b * Hq + y) * Wq + x;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const int r0 = i * 16 + 4 * (lane >> 4);
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (BWD) {
          v[q] = (bf2f(a.mask[p * a.M + r0 + q]) > 0.f) ? acc[i][j][q] : 0.f;
        } else {
          v[q] = acc[i][j][q] + a.bias[r0 + q];
          if (a.relu) v[q] = fmaxf(v[q], 0.f);
        }
      }
      if (!BWD && a.outf) {
        float* o = a.outf + p * a.nreal + r0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (r0 + q < a.nreal) o[q] = v[q];
      } else {
        bf16 h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = (bf16)v[q];
        *(u32x2*)(a.out + p * a.M + r0) = __builtin_bit_cast(u32x2, h);
      }
    }
  }
}

// ------------------------------------------------------------- layer 1 ----
// Cin = 1 or 3 input planes: direct FP32 arithmetic (9 taps per plane), 32
// output channels per pixel.  x0 is planar [B][C][H][W].
__global__ __launch_bounds__(256) void k_conv1_fwd(const float* __restrict__ x0,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ bias, int B, int C,
                                                   int H, int W, int coutp,
                                                   bf16* __restrict__ out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= B * H * W) return;
  const int b = p / (H * W), rem = p - b * H * W, y = rem / W, x = rem - (rem / W) * W;
  float xin[3][9];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int ys = y + t / 3 - 1, xs = x + t % 3 - 1;
      xin[c][t] = (c < C && ys >= 0 && ys < H && xs >= 0 && xs < W)
                      ? x0[(((size_t)b * C + c) * H + ys) * W + xs] : 0.f;
    }
  for (int co = 0; co < coutp; co += 4) {
    bf16 h[4];
    for (int q = 0; q < 4; ++q) {
      float s = bias[co + q];
      const float* wr = w + (size_t)(co + q) * C * 9;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (c < C)
#pragma unroll
          for (int t = 0; t < 9; ++t) s += wr[c * 9 + t] * xin[c][t];
      h[q] = (bf16)fmaxf(s, 0.f);
    }
    *(u32x2*)(out + (size_t)p * coutp + co) = __builtin_bit_cast(u32x2, h);
  }
}

// Layer-1 weight gradient partials: thread (co, j) with j = 9 ci + tap (j = 9C
// is the bias) sums over the rows [r0, r1) of the batch (row = one image row),
// walking x without divisions.  Block size: cout (9C + 1) rounded up to 64.
__global__ __launch_bounds__(1024) void k_conv1_wgrad(const float* __restrict__ x0,
                                                      const bf16* __restrict__ dz, int B, int C,
                                                      int H, int W, int cout, int coutp,
                                                      int rows_per, float* __restrict__ part) {
  const int t = threadIdx.x, J = 9 * C + 1;
  const int r0 = blockIdx.x * rows_per, r1 = min(B * H, r0 + rows_per);
  if (t >= cout * J) return;
  const int co = t / J, j = t % J;
  const bool isb = (j == 9 * C);
  const int ci = isb ? 0 : j / 9, tap = isb ? 0 : j % 9;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  float s = 0.f;
  for (int row = r0; row < r1; ++row) {
    const int b = row / H, y = row - b * H;
    const int ys = y + dy;
    const bool rowok = isb || (ys >= 0 && ys < H);
    if (!rowok) continue;
    const float* xr = x0 + (((size_t)b * C + ci) * H + (isb ? 0 : ys)) * W;
    const bf16* g = dz + (size_t)row * W * coutp + co;
    for (int x = 0; x < W; ++x) {
      float xv = 1.f;
      if (!isb) {
        const int xs = x + dx;
        xv = (xs >= 0 && xs < W) ? xr[xs] : 0.f;
      }
      s += bf2f(g[(size_t)x * coutp]) * xv;
    }
  }
  part[(size_t)blockIdx.x * cout * J + t] = s;
}

// --------------------------------------------------- weight gradients ----
// dW[tap][r][c] = sum_p dz[p][r] * x[map(p, tap)][c] for one tap (grid.y) and
// a slice of output pixels (grid.x); dz and x tiles of 32 pixels are staged
// transposed in LDS so that MFMA operands are 16-byte reads.  r < Mr (coutp),
// c < Nc (cinp); C tiles (Mr/16 x Nc/16) are split over the 4 waves.
#define WG_MAXC 128
__global__ __launch_bounds__(256) void k_conv_wgrad(const bf16* __restrict__ dz,
                                                    const bf16* __restrict__ x, int B,
                                                    int Hout, int Wout, int Hin, int Win,
                                                    int Mr, int Nc, int mode, int per,
                                                    float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) bf16 As[WG_MAXC][40];  // [r][pixel], padded rows
  __shared__ __attribute__((aligned(16))) bf16 Bs[WG_MAXC][40];  // [c][pixel]
  const int tap = blockIdx.y, dy = tap / 3, dx = tap % 3;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int npix = B * Hout * Wout;
  const int p0 = blockIdx.x * per, p1 = min(npix, p0 + per);
  const int tr = Mr / 16, tc = Nc / 16, ntiles = tr * tc;
  constexpr int MAXT = (WG_MAXC / 16) * (WG_MAXC / 16) / 4;
  f32x4 acc[MAXT];
  for (int i = 0; i < MAXT; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int pc = p0; pc < p1; pc += 32) {
    __syncthreads();
    // stage 32 pixels: dz rows (Mr channels) and x at the tap's source pixel
    for (int idx = threadIdx.x; idx < 32 * (Mr / 8); idx += 256) {
      const int pp = idx / (Mr / 8), cg = (idx % (Mr / 8)) * 8;
      const int p = pc + pp;
      bf16x8 v = zero8();
      if (p < p1) v = load8(dz + (size_t)p * Mr + cg);
#pragma unroll
      for (int q = 0; q < 8; ++q) As[cg + q][pp] = v[q];
    }
    for (int idx = threadIdx.x; idx < 32 * (Nc / 8); idx += 256) {
      const int pp = idx / (Nc / 8), cg = (idx % (Nc / 8)) * 8;
      const int p = pc + pp;
      bf16x8 v = zero8();
      if (p < p1) {
        const int b = p / (Hout * Wout), rem = p - b * Hout * Wout;
        const int y = rem / Wout, xx = rem - (rem / Wout) * Wout;
        int ys, xs;
        if (fwd_src(mode, y, xx, dy, dx, Hin, Win, Hout, Wout, ys, xs))
          v = load8(x + ((size_t)(b * Hin + ys) * Win + xs) * Nc + cg);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) Bs[cg + q][pp] = v[q];
    }
    __syncthreads();
    const int kq = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < MAXT; ++i) {
      const int t = wave + 4 * i;
      if (t < ntiles) {
        const int ti = t / tc, tj = t % tc;
        const bf16x8 av = *(const bf16x8*)&As[ti * 16 + (lane & 15)][kq];
        const bf16x8 bv = *(const bf16x8*)&Bs[tj * 16 + (lane & 15)][kq];
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i], 0, 0, 0);
      }
    }
  }
  // partial layout [slice][tap][r][c]
  float* out = part + (((size_t)blockIdx.x * 9 + tap) * Mr) * Nc;
#pragma unroll
  for (int i = 0; i < MAXT; ++i) {
    const int t = wave + 4 * i;
    if (t < ntiles) {
      const int ti = t / tc, tj = t % tc;
      const int c = tj * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) out[(size_t)(ti * 16 + 4 * (lane >> 4) + q) * Nc + c] = acc[i][q];
    }
  }
}

// Weight gradients of the stride-1 and upsampling layers whose output rows are
// whole multiples of 32 pixels, all nine taps per workgroup.  A workgroup walks
// row segments of 32 output pixels.  Per segment it stages, transposed in LDS:
//  * dz of the segment once, [r][pixel];
//  * the three source rows of the conv input, each in three copies shifted by
//    one column, so that every tap reads its x operand at the same 16-byte
//    aligned offsets.
// It then issues the 9 (Mr/16)(Nc/16) MFMA tiles of the segment, spread over
// the four waves.  Compared with one workgroup per tap, dz is staged once
// instead of nine times, a source row is fetched once for three taps, and there
// are nine times as many products per barrier.  Partials use k_conv_wgrad's
// [slice][tap][r][c] layout.
#define WR_MR 32
#define WR_NC 64
template <int MT, int NT>
__global__ __launch_bounds__(256) void k_conv_wgrad_rows(const bf16* __restrict__ dz,
                                                         const bf16* __restrict__ x, int B,
                                                         int Hout, int Wout, int Hin, int Win,
                                                         int mode, int segs_per,
                                                         float* __restrict__ part) {
  constexpr int Mr = 16 * MT, Nc = 16 * NT, NTILE = 9 * MT * NT, PER_WAVE = (NTILE + 3) / 4;
  __shared__ __attribute__((aligned(16))) bf16 As[WR_MR][40];
  __shared__ __attribute__((aligned(16))) bf16 Xs[9][WR_NC][40];   // [3 dy * 3 dx][c][pixel]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int W32 = Wout / 32;
  const int nseg = B * Hout * W32;
  const int s0 = blockIdx.x * segs_per, s1 = min(nseg, s0 + segs_per);
  const bool up = (mode == MAP_UP);
  f32x4 acc[PER_WAVE];
#pragma unroll
  for (int i = 0; i < PER_WAVE; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = 8 * (lane >> 4);
  for (int sg = s0; sg < s1; ++sg) {
    const int b = sg / (Hout * W32), rem = sg - b * Hout * W32;
    const int y = rem / W32, x0 = (rem - y * W32) * 32;
    __syncthreads();
    for (int idx = threadIdx.x; idx < 32 * (Mr / 8); idx += 256) {
      const int pp = idx / (Mr / 8), cg = (idx % (Mr / 8)) * 8;
      const bf16x8 v = load8(dz + (((size_t)b * Hout + y) * Wout + x0 + pp) * Mr + cg);
#pragma unroll
      for (int q = 0; q < 8; ++q) As[cg + q][pp] = v[q];
    }
    for (int idx = threadIdx.x; idx < 3 * 34 * (Nc / 8); idx += 256) {
      const int dy = idx / (34 * (Nc / 8)), r2 = idx - dy * 34 * (Nc / 8);
      const int j = r2 / (Nc / 8), cg = (r2 % (Nc / 8)) * 8;
      const int uy = y + dy - 1, ux = x0 + j - 1;   // conv-input grid (= output grid)
      bf16x8 v = zero8();
      if (uy >= 0 && uy < Hout && ux >= 0 && ux < Wout) {
        const int sy = up ? (uy >> 1) : uy, sx = up ? (ux >> 1) : ux;
        v = load8(x + (((size_t)b * Hin + sy) * Win + sx) * Nc + cg);
      }
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int k = j - dx;   // this value is pixel k of tap (dy, dx)
        if (k >= 0 && k < 32) {
#pragma unroll
          for (int q = 0; q < 8; ++q) Xs[dy * 3 + dx][cg + q][k] = v[q];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER_WAVE; ++i) {
      const int t = wave + 4 * i;
      if (t < NTILE) {
        const int tap = t / (MT * NT), rr = t - tap * MT * NT, ti = rr / NT, tj = rr - ti * NT;
        const bf16x8 av = *(const bf16x8*)&As[ti * 16 + (lane & 15)][kq];
        const bf16x8 bv = *(const bf16x8*)&Xs[tap][tj * 16 + (lane & 15)][kq];
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < PER_WAVE; ++i) {
    const int t = wave + 4 * i;
    if (t < NTILE) {
      const int tap = t / (MT * NT), rr = t - tap * MT * NT, ti = rr / NT, tj = rr - ti * NT;
      float* out = part + (((size_t)blockIdx.x * 9 + tap) * Mr) * Nc;
      const int c = tj * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) out[(size_t)(ti * 16 + 4 * (lane >> 4) + q) * Nc + c] = acc[i][q];
    }
  }
}

// Layer-1 weight and bias gradients as one GEMM over row segments of 32
// pixels: dW[co][j] = sum_p dz[p][co] u[p][j], where u[p] is the pixel's
// 9 C input values (plane-major, tap-minor, the [cout][cin][3][3] order of
// the weights), then 1 for the bias, then zeros up to 32 columns.  dz and u
// are staged transposed in LDS (u rounded to bf16), one MFMA tile per wave and
// segment, FP32 accumulation.  Needs W % 32 == 0, coutp == 32 and 9 C + 1 <= 32.
// Partials [slice][32][32].
__global__ __launch_bounds__(256) void k_conv1_wgrad_rows(const float* __restrict__ x0,
                                                          const bf16* __restrict__ dz, int B,
                                                          int C, int H, int W, int segs_per,
                                                          float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) bf16 As[32][40];
  __shared__ __attribute__((aligned(16))) bf16 Us[32][40];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int W32 = W / 32, nseg = B * H * W32;
  const int s0 = blockIdx.x * segs_per, s1 = min(nseg, s0 + segs_per);
  const int ti = wave >> 1, tj = wave & 1;   // the four 16 x 16 tiles of the 32 x 32 result
  const int J = 9 * C;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = 8 * (lane >> 4);
  for (int sg = s0; sg < s1; ++sg) {
    const int b = sg / (H * W32), rem = sg - b * H * W32;
    const int y = rem / W32, xb = (rem - y * W32) * 32;
    __syncthreads();
    for (int idx = threadIdx.x; idx < 32 * 4; idx += 256) {
      const int pp = idx >> 2, cg = (idx & 3) * 8;
      const bf16x8 v = load8(dz + (((size_t)b * H + y) * W + xb + pp) * 32 + cg);
#pragma unroll
      for (int q = 0; q < 8; ++q) As[cg + q][pp] = v[q];
    }
    for (int idx = threadIdx.x; idx < 32 * 32; idx += 256) {
      const int j = idx >> 5, k = idx & 31;   // consecutive threads: consecutive pixels
      float v = 0.f;
      if (j < J) {
        const int ci = j / 9, t = j - 9 * ci;
        const int ys = y + t / 3 - 1, xs = xb + k + t % 3 - 1;
        if (ys >= 0 && ys < H && xs >= 0 && xs < W) v = x0[(((size_t)b * C + ci) * H + ys) * W + xs];
      } else if (j == J) {
        v = 1.f;
      }
      Us[j][k] = (bf16)v;
    }
    __syncthreads();
    const bf16x8 av = *(const bf16x8*)&As[ti * 16 + (lane & 15)][kq];
    const bf16x8 bv = *(const bf16x8*)&Us[tj * 16 + (lane & 15)][kq];
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
  float* out = part + (size_t)blockIdx.x * 32 * 32;
#pragma unroll
  for (int q = 0; q < 4; ++q) out[(ti * 16 + 4 * (lane >> 4) + q) * 32 + tj * 16 + (lane & 15)] = acc[q];
}

// Sum the [slice][32][32] partials of k_conv1_wgrad_rows in slice order.
__global__ void k_conv1_rows_reduce(const float* __restrict__ part, int nslices, int cout, int C,
                                    float* __restrict__ gw, float* __restrict__ gb) {
  const int J = 9 * C;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= cout * (J + 1)) return;
  const int co = t / (J + 1), j = t % (J + 1);
  float s = 0.f;
  for (int sl = 0; sl < nslices; ++sl) s += part[((size_t)sl * 32 + co) * 32 + j];
  if (j < J) gw[(size_t)co * J + j] = s;
  else gb[co] = s;
}

// Bias-gradient partials: column sums of dz over a pixel slice.  Thread t
// handles channel t % Mr of pixels p0 + t / Mr + j * (256 / Mr), so a wave's
// loads cover whole pixel rows (coalesced); the 256 / Mr lanes of a channel
// are then added in a fixed order.
__global__ __launch_bounds__(256) void k_bias_grad(const bf16* __restrict__ dz, int npix, int Mr,
                                                   int per, float* __restrict__ part) {
  // thread = (pixel lane g, group of 8 channels cg): 16-byte loads, G pixels
  // per round; Mr is a multiple of 16
  __shared__ float red[256 * 8];
  const int p0 = blockIdx.x * per, p1 = min(npix, p0 + per);
  const int CG = Mr / 8, G = 256 / CG, cg = threadIdx.x % CG, g = threadIdx.x / CG;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (g < G)
    for (int p = p0 + g; p < p1; p += G) {
      const bf16x8 v = load8(dz + (size_t)p * Mr + 8 * cg);
#pragma unroll
      for (int q = 0; q < 8; ++q) s[q] += (float)v[q];
    }
#pragma unroll
  for (int q = 0; q < 8; ++q) red[threadIdx.x * 8 + q] = s[q];
  __syncthreads();
  if (threadIdx.x < Mr) {
    const int c = threadIdx.x, cgc = c / 8, q = c % 8;
    float t = 0.f;
    for (int gg = 0; gg < G; ++gg) t += red[(gg * CG + cgc) * 8 + q];
    part[(size_t)blockIdx.x * Mr + c] = t;
  }
}

// Sum the slices (fixed order) into the FP32 gradient in [cout][cin][3][3] order.
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nslices, int Mr, int Nc,
                               int cout, int cin, float* __restrict__ g) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= cout * cin * 9) return;
  const int co = idx / (cin * 9), rem = idx % (cin * 9), ci = rem / 9, tap = rem % 9;
  float s = 0.f;
  for (int sl = 0; sl < nslices; ++sl) s += part[(((size_t)sl * 9 + tap) * Mr + co) * Nc + ci];
  g[idx] = s;
}
__global__ void k_bgrad_reduce(const float* __restrict__ part, int nslices, int Mr, int cout,
                               float* __restrict__ g) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= cout) return;
  float s = 0.f;
  for (int sl = 0; sl < nslices; ++sl) s += part[(size_t)sl * Mr + r];
  g[r] = s;
}
__global__ void k_conv1_reduce(const float* __restrict__ part, int nslices, int cout, int C,
                               float* __restrict__ gw, float* __restrict__ gb) {
  const int J = 9 * C + 1;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= cout * J) return;
  float s = 0.f;
  for (int sl = 0; sl < nslices; ++sl) s += part[(size_t)sl * cout * J + t];
  const int co = t / J, j = t % J;
  if (j < 9 * C) gw[(size_t)co * 9 * C + j] = s;   // [cout][cin][3][3]
  else gb[co] = s;
}

// ------------------------------------------------ input, loss, output ----
// Input planes [B][C][H][W]: plane 0 = (eps - 2.085) / (12.25 - 2.085); for
// C = 3, planes 1 and 2 = real and imaginary part of the effective-index field
// scaled to unit RMS per pixel (iscale[b] = sqrt(D) / ||F_b||).
__global__ void k_inputs(const float* __restrict__ eps, const float2* __restrict__ eim,
                         const double* __restrict__ iscale, int B, int D, int C,
                         float* __restrict__ x0) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= B * D) return;
  const int b = i / D, e = i - b * D;
  x0[(size_t)b * C * D + e] = (eps[i] - CNN_EPS_LO) / (CNN_EPS_HI - CNN_EPS_LO);
  if (C == 3) {
    const float s = (float)iscale[b];
    const float2 f = eim[i];
    x0[((size_t)b * C + 1) * D + e] = f.x * s;
    x0[((size_t)b * C + 2) * D + e] = f.y * s;
  }
}

// iscale[b] = sqrt(D / sum |F_b|^2) (0 for an all-zero field); one block per problem
__global__ __launch_bounds__(256) void k_eim_scale(const float2* __restrict__ eim, int D,
                                                   double* __restrict__ iscale) {
  const float2* f = eim + (size_t)blockIdx.x * D;
  double s = 0.0;
  for (int e = threadIdx.x; e < D; e += 256) s += (double)f[e].x * f[e].x + (double)f[e].y * f[e].y;
  __shared__ double lds[8];
  s = block_sum1<double>(s, lds);
  if (threadIdx.x == 0) iscale[blockIdx.x] = (s > 0.0) ? sqrt((double)D / s) : 0.0;
}

// loss partials and dz of the last (linear) layer: out [p][2k] FP32, target
// [B][k][D] complex64; dz = 2 (out - t) / count in bf16 with coutp channels.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out,
                                             const float2* __restrict__ target, int B, int D,
                                             int k, int coutp, float scale,
                                             bf16* __restrict__ dz, float* __restrict__ lpart) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  float s = 0.f;
  if (p < B * D) {
    const int b = p / D, e = p - b * D;
    const float* o = out + (size_t)p * 2 * k;
    // coutp is a multiple of 16: the row of dz is written 8 channels (16 B) at a time
    for (int c0 = 0; c0 < coutp; c0 += 8) {
      bf16x8 h;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = c0 + q;
        float g = 0.f;
        if (c < 2 * k) {
          const float2 t = target[((size_t)b * k + c / 2) * D + e];
          const float d = o[c] - ((c & 1) ? t.y : t.x);
          s += d * d;
          g = scale * d;
        }
        h[q] = (bf16)g;
      }
      *(u32x4*)(dz + (size_t)p * coutp + c0) = __builtin_bit_cast(u32x4, h);
    }
  }
  __shared__ float lds[8];
  s = block_sum1<float>(s, lds);
  if (threadIdx.x == 0) lpart[blockIdx.x] = s;
}

__global__ void k_to_fields(const float* __restrict__ out, int B, int D, int k,
                            float2* __restrict__ U) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= B * D) return;
  const int b = p / D, e = p - b * D;
  for (int j = 0; j < k; ++j)
    U[((size_t)b * k + j) * D + e] = make_float2(out[(size_t)p * 2 * k + 2 * j],
                                                  out[(size_t)p * 2 * k + 2 * j + 1]);
}

// ------------------------------------------------------- parameters ----
// bf16 GEMM copies of one layer's FP32 weights [cout][cin][3][3].
__global__ void k_pack_weights(const float* __restrict__ w, int cout, int cin, int coutp,
                               int cinp, bf16* __restrict__ wf, bf16* __restrict__ wb) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= 9 * coutp * cinp) return;
  const int tap = idx / (coutp * cinp), rem = idx % (coutp * cinp);
  const int co = rem / cinp, ci = rem % cinp;
  const float v = (co < cout && ci < cin) ? w[((size_t)co * cin + ci) * 9 + tap] : 0.f;
  wf[idx] = (bf16)v;
  if (wb) wb[((size_t)tap * cinp + ci) * coutp + co] = (bf16)v;
}

// Adam (Kingma & Ba) on the FP32 master parameters.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float c1,
                       float c2, float eps) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bias for layers whose coutp > cout: a zero-padded FP32 copy
__global__ void k_pad_bias(const float* __restrict__ b, int cout, int coutp, float* __restrict__ bp) {
  const int i = threadIdx.x;
  if (i < coutp) bp[i] = (i < cout) ? b[i] : 0.f;
}

// ============================================================ host side ====
static int rup16(int c) { return (c + 15) / 16 * 16; }

// pixels per weight-gradient slice: about 256 slices, multiples of 32
static int wgrad_per(int npix) { return std::max(2048, ((npix + 255) / 256 + 31) / 32 * 32); }

template <typename X>
static hipError_t cnn_alloc(dd_cnn* n, X** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count * sizeof(X), 256));
  if (e == hipSuccess) {
    n->allocs.push_back((void*)*p);
    e = hipMemset(*p, 0, std::max<size_t>(count * sizeof(X), 256));
  }
  return e;
}

extern "C" void dd_cnn_destroy(dd_cnn* net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  for (void* p : net->allocs) (void)hipFree(p);
  delete net;
}

static dd_status pack_all(dd_cnn* n, hipStream_t st) {
  for (int l = 0; l < NL; ++l) {
    const CnnLayer& L = n->L[l];
    if (l == 0) continue;  // layer 1 reads the FP32 master weights directly
    const int tot = 9 * L.coutp * L.cinp;
    k_pack_weights<<<(tot + 255) / 256, 256, 0, st>>>(n->params + L.woff, L.cout, L.cin, L.coutp,
                                                      L.cinp, n->wf[l], n->wb[l]);
  }
  DD_HIP_CHECK(hipGetLastError());
  return DD_OK;
}

extern "C" dd_status dd_cnn_create(int nx, int ny, int max_batch, int k, int in_channels,
                                   unsigned long long seed, dd_cnn** out) {
  if (!out) { dd_set_error("dd_cnn_create: out is NULL"); return DD_EINVAL; }
  *out = nullptr;
  if (nx < 4 || ny < 4 || nx % 4 || ny % 4 || max_batch < 1 || k < 1 || 2 * k > 64 ||
      (in_channels != 1 && in_channels != 3)) {
    dd_set_error("dd_cnn_create: need nx, ny multiples of 4, max_batch >= 1, 1 <= k <= 32 "
                 "and 1 or 3 input channels");
    return DD_EINVAL;
  }
  dd_cnn* n = new dd_cnn();
  n->nx = nx; n->ny = ny; n->maxB = max_batch; n->k = k; n->cin0 = in_channels;
  const int spec[NL][5] = {{in_channels, 32, 1, 0, 1}, {32, 64, 2, 0, 1}, {64, 128, 2, 0, 1},
                           {128, 128, 1, 0, 1}, {128, 64, 1, 1, 1}, {64, 32, 1, 1, 1},
                           {32, 32, 1, 0, 1}, {32, 2 * k, 1, 0, 0}};
  int H = ny, W = nx;
  size_t off = 0;
  for (int l = 0; l < NL; ++l) {
    CnnLayer& L = n->L[l];
    L.cin = spec[l][0]; L.cout = spec[l][1]; L.stride = spec[l][2]; L.up = spec[l][3];
    L.relu = spec[l][4];
    L.cinp = (l == 0) ? L.cin : rup16(L.cin);
    L.coutp = std::max(32, rup16(L.cout));
    L.Hin = H; L.Win = W;
    if (L.up) { L.Hout = 2 * H; L.Wout = 2 * W; }
    else if (L.stride == 2) { L.Hout = H / 2; L.Wout = W / 2; }
    else { L.Hout = H; L.Wout = W; }
    L.mode = L.up ? MAP_UP : (L.stride == 2 ? MAP_S2 : MAP_S1);
    L.woff = off; off += (size_t)L.cout * L.cin * 9;
    L.boff = off; off += L.cout;
    H = L.Hout; W = L.Wout;
  }
  n->nparams = off;
  // He-uniform initialisation (host mt19937_64), zero biases
  std::vector<float> hp(off, 0.f);
  std::mt19937_64 rng(seed);
  for (int l = 0; l < NL; ++l) {
    const CnnLayer& L = n->L[l];
    const float bound = std::sqrt(6.0f / (L.cin * 9));
    std::uniform_real_distribution<float> ud(-bound, bound);
    for (size_t i = 0; i < (size_t)L.cout * L.cin * 9; ++i) hp[L.woff + i] = ud(rng);
  }
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  chk(cnn_alloc(n, &n->params, off + 64));
  chk(cnn_alloc(n, &n->grads, off + 64));
  chk(cnn_alloc(n, &n->am, off + 64));
  chk(cnn_alloc(n, &n->av, off + 64));
  const size_t D = (size_t)nx * ny;
  chk(cnn_alloc(n, &n->x0, (size_t)max_batch * D * in_channels));
  chk(cnn_alloc(n, &n->iscale, (size_t)max_batch));
  size_t wp = 0;
  for (int l = 0; l < NL && e == hipSuccess; ++l) {
    const CnnLayer& L = n->L[l];
    const size_t pix = (size_t)max_batch * L.Hout * L.Wout;
    if (l > 0) {
      chk(cnn_alloc(n, &n->wf[l], (size_t)9 * L.coutp * L.cinp));
      chk(cnn_alloc(n, &n->wb[l], (size_t)9 * L.coutp * L.cinp));
    }
    if (l < NL - 1) chk(cnn_alloc(n, &n->act[l], pix * L.coutp));
    chk(cnn_alloc(n, &n->dz[l], pix * L.coutp));
    // weight-gradient partials (slices as in backward())
    // any batch B <= max_batch gives at most ~257 slices (wgrad_per)
    const size_t per = (size_t)wgrad_per((int)pix);
    const size_t slices = std::max<size_t>((pix + per - 1) / per, 260);
    if (l > 0) wp = std::max(wp, slices * 9 * L.coutp * L.cinp);
    wp = std::max(wp, slices * (size_t)L.coutp);
    wp = std::max(wp, (size_t)512 * L.cout * (9 * L.cin + 1));
  }
  n->wpart_elems = wp;
  chk(cnn_alloc(n, &n->wpart, wp));
  chk(cnn_alloc(n, &n->out, (size_t)max_batch * D * 2 * k));
  chk(cnn_alloc(n, &n->lpart, (size_t)max_batch * D / 256 + 256));
  chk(cnn_alloc(n, &n->biaspad, (size_t)256 * NL));
  if (e == hipSuccess) chk(hipMemcpy(n->params, hp.data(), sizeof(float) * off, hipMemcpyHostToDevice));
  if (e != hipSuccess) {
    dd_set_error("dd_cnn_create: %s", hipGetErrorString(e));
    dd_cnn_destroy(n);
    return e == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP;
  }
  dd_status rc = pack_all(n, 0);
  if (rc != DD_OK) { dd_cnn_destroy(n); return rc; }
  DD_HIP_CHECK(hipDeviceSynchronize());
  *out = n;
  return DD_OK;
}

extern "C" int dd_cnn_layer_info(const dd_cnn* n, int l, int* cin, int* cout, int* stride,
                                 int* up, int* relu) {
  if (!n) return -1;
  if (l < 0 || l >= NL) return NL;
  const CnnLayer& L = n->L[l];
  if (cin) *cin = L.cin;
  if (cout) *cout = L.cout;
  if (stride) *stride = L.stride;
  if (up) *up = L.up;
  if (relu) *relu = L.relu;
  return NL;
}

extern "C" size_t dd_cnn_num_params(const dd_cnn* n) { return n ? n->nparams : 0; }

extern "C" dd_status dd_cnn_get_params(const dd_cnn* n, float* host, size_t count) {
  if (!n || !host || count != n->nparams) {
    dd_set_error("dd_cnn_get_params: bad argument (count must be %zu)", n ? n->nparams : (size_t)0);
    return DD_EINVAL;
  }
  DD_HIP_CHECK(hipDeviceSynchronize());
  DD_HIP_CHECK(hipMemcpy(host, n->params, sizeof(float) * count, hipMemcpyDeviceToHost));
  return DD_OK;
}

extern "C" dd_status dd_cnn_set_params(dd_cnn* n, const float* host, size_t count) {
  if (!n || !host || count != n->nparams) {
    dd_set_error("dd_cnn_set_params: bad argument (count must be %zu)", n ? n->nparams : (size_t)0);
    return DD_EINVAL;
  }
  DD_HIP_CHECK(hipDeviceSynchronize());
  DD_HIP_CHECK(hipMemcpy(n->params, host, sizeof(float) * count, hipMemcpyHostToDevice));
  DD_HIP_CHECK(hipMemset(n->am, 0, sizeof(float) * count));
  DD_HIP_CHECK(hipMemset(n->av, 0, sizeof(float) * count));
  n->adam_t = 0;
  dd_status rc = pack_all(n, 0);
  if (rc != DD_OK) return rc;
  DD_HIP_CHECK(hipDeviceSynchronize());
  return DD_OK;
}

template <int MT, int NT, bool BWD>
static void launch_gemm(const GemmArgs& a, int npix, hipStream_t st) {
  const int per_block = 4 * NT * 16;
  k_conv_gemm<MT, NT, BWD><<<(npix + per_block - 1) / per_block, 256, 0, st>>>(a);
}

static void gemm_dispatch(const GemmArgs& a, int npix, bool bwd, hipStream_t st) {
  const int MT = a.M / 16;
  if (!bwd && (a.mode == MAP_S1 || a.mode == MAP_UP) && a.Ksrc % 32 == 0) {
    const dim3 grid((a.Wq + CT_TW - 1) / CT_TW, (a.Hq + CT_TH - 1) / CT_TH, a.B);
    switch (MT) {
      case 2: k_conv_tile<2><<<grid, 256, 0, st>>>(a); break;
      case 4: k_conv_tile<4><<<grid, 256, 0, st>>>(a); break;
      default: k_conv_tile<8><<<grid, 256, 0, st>>>(a); break;
    }
    return;
  }
  if (bwd && a.mode == MAP_S1 && a.Ksrc % 32 == 0) {
    const dim3 grid((a.Wq + CT_TW - 1) / CT_TW, (a.Hq + CT_TH - 1) / CT_TH, a.B);
    switch (MT) {
      case 2: k_conv_tile<2, true><<<grid, 256, 0, st>>>(a); break;
      case 4: k_conv_tile<4, true><<<grid, 256, 0, st>>>(a); break;
      default: k_conv_tile<8, true><<<grid, 256, 0, st>>>(a); break;
    }
    return;
  }
  if (!bwd) {
    switch (MT) {
      case 2: launch_gemm<2, 8, false>(a, npix, st); break;
      case 4: launch_gemm<4, 4, false>(a, npix, st); break;
      default: launch_gemm<8, 2, false>(a, npix, st); break;
    }
  } else {
    switch (MT) {
      case 2: launch_gemm<2, 8, true>(a, npix, st); break;
      case 4: launch_gemm<4, 4, true>(a, npix, st); break;
      default: launch_gemm<8, 2, true>(a, npix, st); break;
    }
  }
}

static dd_status forward(dd_cnn* n, const float* eps, const void* eim, int B, hipStream_t st,
                         float* biaspad) {
  const int D = n->nx * n->ny;
  if (n->cin0 == 3) k_eim_scale<<<B, 256, 0, st>>>((const float2*)eim, D, n->iscale);
  k_inputs<<<(B * D + 255) / 256, 256, 0, st>>>(eps, (const float2*)eim, n->iscale, B, D, n->cin0,
                                                 n->x0);
  {
    const CnnLayer& L = n->L[0];
    k_conv1_fwd<<<(B * D + 255) / 256, 256, 0, st>>>(n->x0, n->params + L.woff,
                                                      n->params + L.boff, B, n->cin0, n->ny,
                                                      n->nx, L.coutp, n->act[0]);
  }
  for (int l = 1; l < NL; ++l) {
    const CnnLayer& L = n->L[l];
    k_pad_bias<<<1, 256, 0, st>>>(n->params + L.boff, L.cout, L.coutp, biaspad + 256 * l);
    GemmArgs a{};
    a.src = n->act[l - 1];
    a.W = n->wf[l];
    a.bias = biaspad + 256 * l;
    a.B = B; a.Hq = L.Hout; a.Wq = L.Wout;
    a.Hs = L.Hin; a.Ws = L.Win; a.Hout = L.Hout; a.Wout = L.Wout;
    a.Ksrc = L.cinp; a.M = L.coutp; a.mode = L.mode; a.entries = 9; a.relu = L.relu;
    if (l == NL - 1) { a.outf = n->out; a.nreal = L.cout; }
    else a.out = n->act[l];
    gemm_dispatch(a, B * L.Hout * L.Wout, false, st);
  }
  DD_HIP_CHECK(hipGetLastError());
  return DD_OK;
}

// Backward pass from the gradient of the last layer's pre-activation in
// dz[NL-1]; parameter gradients land in n->grads.
static dd_status backward_from_dz(dd_cnn* n, int B, hipStream_t st) {
  for (int l = NL - 1; l >= 1; --l) {
    const CnnLayer& L = n->L[l];
    const int npo = B * L.Hout * L.Wout;
    // weight and bias gradients of layer l: about 256 pixel slices
    const int per = wgrad_per(npo);
    const int slices = (npo + per - 1) / per;
    const bool rows = (L.mode == MAP_S1 || L.mode == MAP_UP) && L.Wout % 32 == 0 &&
                      L.coutp == 32 && (L.cinp == 32 || L.cinp == 64);
    int wslices = slices;
    if (rows) {
      // row segments of 32 output pixels, at most `slices` workgroups
      const int nseg = B * L.Hout * (L.Wout / 32);
      const int sp = (nseg + slices - 1) / slices;
      wslices = (nseg + sp - 1) / sp;
      if (L.cinp == 32)
        k_conv_wgrad_rows<2, 2><<<wslices, 256, 0, st>>>(n->dz[l], n->act[l - 1], B, L.Hout,
                                                         L.Wout, L.Hin, L.Win, L.mode, sp,
                                                         n->wpart);
      else
        k_conv_wgrad_rows<2, 4><<<wslices, 256, 0, st>>>(n->dz[l], n->act[l - 1], B, L.Hout,
                                                         L.Wout, L.Hin, L.Win, L.mode, sp,
                                                         n->wpart);
    } else {
      k_conv_wgrad<<<dim3(slices, 9), 256, 0, st>>>(n->dz[l], n->act[l - 1], B, L.Hout, L.Wout,
                                                     L.Hin, L.Win, L.coutp, L.cinp, L.mode, per,
                                                     n->wpart);
    }
    const int tot = L.cout * L.cin * 9;
    k_wgrad_reduce<<<(tot + 255) / 256, 256, 0, st>>>(n->wpart, wslices, L.coutp, L.cinp, L.cout,
                                                      L.cin, n->grads + L.woff);
    k_bias_grad<<<slices, 256, 0, st>>>(n->dz[l], npo, L.coutp, per, n->wpart);
    k_bgrad_reduce<<<1, 256, 0, st>>>(n->wpart, slices, L.coutp, L.cout, n->grads + L.boff);
    // data gradient into the previous layer (masked by its ReLU)
    GemmArgs a{};
    a.src = n->dz[l];
    a.W = n->wb[l];
    a.mask = n->act[l - 1];
    a.out = n->dz[l - 1];
    a.B = B; a.Hq = L.Hin; a.Wq = L.Win;
    a.Hs = L.Hout; a.Ws = L.Wout; a.Hout = L.Hout; a.Wout = L.Wout;
    a.Ksrc = L.coutp; a.M = L.cinp; a.mode = L.mode; a.entries = L.up ? 36 : 9;
    gemm_dispatch(a, B * L.Hin * L.Win, true, st);
  }
  {
    const CnnLayer& L = n->L[0];
    const int nt = L.cout * (9 * n->cin0 + 1);
    if (n->nx % 32 == 0 && L.coutp == 32 && 9 * n->cin0 + 1 <= 32) {
      const int nseg = B * n->ny * (n->nx / 32);
      const int sp = (nseg + 255) / 256, slices = (nseg + sp - 1) / sp;
      k_conv1_wgrad_rows<<<slices, 256, 0, st>>>(n->x0, n->dz[0], B, n->cin0, n->ny, n->nx, sp,
                                                 n->wpart);
      k_conv1_rows_reduce<<<(nt + 255) / 256, 256, 0, st>>>(n->wpart, slices, L.cout, n->cin0,
                                                            n->grads + L.woff, n->grads + L.boff);
    } else {
      const int rows = B * n->ny, rows_per = std::max(1, (rows + 511) / 512);
      const int slices = (rows + rows_per - 1) / rows_per;
      k_conv1_wgrad<<<slices, (nt + 63) / 64 * 64, 0, st>>>(n->x0, n->dz[0], B, n->cin0, n->ny,
                                                            n->nx, L.cout, L.coutp, rows_per,
                                                            n->wpart);
      k_conv1_reduce<<<(nt + 255) / 256, 256, 0, st>>>(n->wpart, slices, L.cout, n->cin0,
                                                       n->grads + L.woff, n->grads + L.boff);
    }
  }
  DD_HIP_CHECK(hipGetLastError());
  return DD_OK;
}

// loss + backward; grads land in n->grads.  *loss receives the batch MSE.
static dd_status backward(dd_cnn* n, const void* target, int B, float* loss, hipStream_t st) {
  const int D = n->nx * n->ny;
  const int k = n->k;
  const CnnLayer& LL = n->L[NL - 1];
  const float scale = 2.0f / ((float)B * D * 2 * k);
  const int nlb = (B * D + 255) / 256;
  k_mse<<<nlb, 256, 0, st>>>(n->out, (const float2*)target, B, D, k, LL.coutp, scale,
                             n->dz[NL - 1], n->lpart);
  dd_status rc = backward_from_dz(n, B, st);
  if (rc != DD_OK) return rc;
  DD_HIP_CHECK(hipGetLastError());
  if (loss) {
    std::vector<float> lp(nlb);
    DD_HIP_CHECK(hipMemcpyAsync(lp.data(), n->lpart, sizeof(float) * nlb, hipMemcpyDeviceToHost, st));
    DD_HIP_CHECK(hipStreamSynchronize(st));
    double s = 0.0;
    for (float v : lp) s += v;
    *loss = (float)(s / ((double)B * D * 2 * k));
  }
  return DD_OK;
}

static dd_status check_batch(const dd_cnn* n, const void* eps, const void* eim, int B,
                             const char* who) {
  if (!n || !eps || B < 1 || B > n->maxB) {
    dd_set_error("%s: need a network, eps and 1 <= B <= max_batch (%d)", who, n ? n->maxB : 0);
    return DD_EINVAL;
  }
  if ((n->cin0 == 3) != (eim != nullptr)) {
    dd_set_error("%s: this network takes %s", who,
                 n->cin0 == 3 ? "the effective-index field (eim must not be NULL)"
                              : "the permittivity only (eim must be NULL)");
    return DD_EINVAL;
  }
  return DD_OK;
}

static dd_status predict(dd_cnn* n, const float* eps, const void* eim, int B, void* U,
                         hipStream_t st, const char* who) {
  dd_status rc = check_batch(n, eps, eim, B, who);
  if (rc != DD_OK) return rc;
  if (!U) { dd_set_error("%s: U is NULL", who); return DD_EINVAL; }
  rc = forward(n, eps, eim, B, st, n->biaspad);
  if (rc != DD_OK) return rc;
  const int D = n->nx * n->ny;
  k_to_fields<<<(B * D + 255) / 256, 256, 0, st>>>(n->out, B, D, n->k, (float2*)U);
  DD_HIP_CHECK(hipGetLastError());
  DD_HIP_CHECK(hipStreamSynchronize(st));
  return DD_OK;
}

extern "C" dd_status predict_subspace(dd_cnn* n, const float* eps, int B, void* U,
                                      hipStream_t st) {
  return predict(n, eps, nullptr, B, U, st, "predict_subspace");
}

extern "C" dd_status predict_subspace_eim(dd_cnn* n, const float* eps, const void* eim, int B,
                                          void* U, hipStream_t st) {
  if (!eim) { dd_set_error("predict_subspace_eim: eim is NULL"); return DD_EINVAL; }
  return predict(n, eps, eim, B, U, st, "predict_subspace_eim");
}

extern "C" dd_status dd_cnn_grad(dd_cnn* n, const float* eps, const void* eim, const void* target,
                                 int B, float* loss, float* host_grad, size_t count,
                                 hipStream_t st) {
  dd_status rc = check_batch(n, eps, eim, B, "dd_cnn_grad");
  if (rc != DD_OK) return rc;
  if (!target || (host_grad && count != n->nparams)) {
    dd_set_error("dd_cnn_grad: bad target or gradient size");
    return DD_EINVAL;
  }
  rc = forward(n, eps, eim, B, st, n->biaspad);
  if (rc != DD_OK) return rc;
  rc = backward(n, target, B, loss, st);
  if (rc != DD_OK) return rc;
  if (host_grad) {
    DD_HIP_CHECK(hipMemcpyAsync(host_grad, n->grads, sizeof(float) * count, hipMemcpyDeviceToHost, st));
  }
  DD_HIP_CHECK(hipStreamSynchronize(st));
  return DD_OK;
}

extern "C" dd_status dd_cnn_train_step(dd_cnn* n, const float* eps, const void* eim,
                                       const void* target, int B, float lr, float b1, float b2,
                                       float* loss, hipStream_t st) {
  dd_status rc = check_batch(n, eps, eim, B, "dd_cnn_train_step");
  if (rc != DD_OK) return rc;
  if (!target || !(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f)) {
    dd_set_error("dd_cnn_train_step: bad target or Adam parameters");
    return DD_EINVAL;
  }
  rc = forward(n, eps, eim, B, st, n->biaspad);
  if (rc != DD_OK) return rc;
  rc = backward(n, target, B, loss, st);
  if (rc != DD_OK) return rc;
  n->adam_t += 1;
  const float c1 = 1.f - std::pow(b1, (float)n->adam_t);
  const float c2 = 1.f - std::pow(b2, (float)n->adam_t);
  k_adam<<<(unsigned)((n->nparams + 255) / 256), 256, 0, st>>>(n->params, n->grads, n->am, n->av,
                                                                n->nparams, lr, b1, b2, c1, c2, 1e-8f);
  rc = pack_all(n, st);
  if (rc != DD_OK) return rc;
  DD_HIP_CHECK(hipStreamSynchronize(st));
  return DD_OK;
}

// Residual-loss step (Sec. 3, eq:res_loss): forward, the loss of every image's
// predicted fields against its own operator and right-hand side, the
// gradient through A^H into the last layer, backward.  *loss = batch mean.
static dd_status res_step(dd_cnn* n, const float* eps, const void* eim,
                          const fdfd_op* const* ops, const void* const* b, int B, float* loss,
                          hipStream_t st, const char* who) {
  dd_status rc = check_batch(n, eps, eim, B, who);
  if (rc != DD_OK) return rc;
  if (!ops || !b) { dd_set_error("%s: need ops and b", who); return DD_EINVAL; }
  for (int p = 0; p < B; ++p)
    if (!ops[p] || !b[p] || ops[p]->nx != n->nx || ops[p]->ny != n->ny) {
      dd_set_error("%s: problem %d needs an operator of %d x %d and b", who, p, n->nx, n->ny);
      return DD_EINVAL;
    }
  const size_t D = (size_t)n->nx * n->ny;
  if (!n->rl_V) {
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
    chk(cnn_alloc(n, &n->rl_V, (size_t)n->maxB * n->k * D));
    chk(cnn_alloc(n, &n->rl_W, (size_t)n->maxB * n->k * D));
    chk(cnn_alloc(n, &n->rl_r, (size_t)n->maxB * D));
    chk(cnn_alloc(n, &n->rl_s, (size_t)n->maxB * D));
    if (e != hipSuccess) {
      dd_set_error("%s: %s", who, hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP;
    }
  }
  rc = forward(n, eps, eim, B, st, n->biaspad);
  if (rc != DD_OK) return rc;
  k_to_fields<<<(unsigned)((B * D + 255) / 256), 256, 0, st>>>(n->out, B, (int)D, n->k, n->rl_V);
  DD_HIP_CHECK(hipGetLastError());
  std::vector<const void*> Vp(B);
  for (int p = 0; p < B; ++p) Vp[p] = n->rl_V + (size_t)p * n->k * D;
  std::vector<double> lv(B);
  rc = res_loss_core(ops, b, Vp.data(), B, n->k, n->rl_W, n->rl_r, n->rl_s, lv.data(),
                     n->dz[NL - 1], n->L[NL - 1].coutp, 1.0 / B, st);
  if (rc != DD_OK) return rc;
  rc = backward_from_dz(n, B, st);
  if (rc != DD_OK) return rc;
  if (loss) {
    double s = 0.0;
    for (double v : lv) s += v;
    *loss = (float)(s / B);
  }
  return DD_OK;
}

extern "C" dd_status dd_cnn_grad_res(dd_cnn* n, const float* eps, const void* eim,
                                     const fdfd_op* const* ops, const void* const* b, int B,
                                     float* loss, float* host_grad, size_t count,
                                     hipStream_t st) {
  if (n && host_grad && count != n->nparams) {
    dd_set_error("dd_cnn_grad_res: gradient size must be %zu", n->nparams);
    return DD_EINVAL;
  }
  dd_status rc = res_step(n, eps, eim, ops, b, B, loss, st, "dd_cnn_grad_res");
  if (rc != DD_OK) return rc;
  if (host_grad) {
    DD_HIP_CHECK(hipMemcpyAsync(host_grad, n->grads, sizeof(float) * count, hipMemcpyDeviceToHost, st));
  }
  DD_HIP_CHECK(hipStreamSynchronize(st));
  return DD_OK;
}

extern "C" dd_status dd_cnn_train_step_res(dd_cnn* n, const float* eps, const void* eim,
                                           const fdfd_op* const* ops, const void* const* b, int B,
                                           float lr, float b1, float b2, float* loss,
                                           hipStream_t st) {
  if (!(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f)) {
    dd_set_error("dd_cnn_train_step_res: bad Adam parameters");
    return DD_EINVAL;
  }
  dd_status rc = res_step(n, eps, eim, ops, b, B, loss, st, "dd_cnn_train_step_res");
  if (rc != DD_OK) return rc;
  n->adam_t += 1;
  const float c1 = 1.f - std::pow(b1, (float)n->adam_t);
  const float c2 = 1.f - std::pow(b2, (float)n->adam_t);
  k_adam<<<(unsigned)((n->nparams + 255) / 256), 256, 0, st>>>(n->params, n->grads, n->am, n->av,
                                                                n->nparams, lr, b1, b2, c1, c2, 1e-8f);
  rc = pack_all(n, st);
  if (rc != DD_OK) return rc;
  DD_HIP_CHECK(hipStreamSynchronize(st));
  return DD_OK;
}

extern "C" dd_status dd_cnn_debug_activation(const dd_cnn* n, int layer, int B, float* host,
                                             size_t count) {
  if (!n || !host || layer < -1 || layer >= NL || B < 1 || B > n->maxB) {
    dd_set_error("dd_cnn_debug_activation: bad argument");
    return DD_EINVAL;
  }
  DD_HIP_CHECK(hipDeviceSynchronize());
  const size_t D = (size_t)n->nx * n->ny;
  if (layer == -1) {
    const size_t cnt = B * D * n->cin0;
    if (count != cnt) { dd_set_error("dd_cnn_debug_activation: count must be %zu", cnt); return DD_EINVAL; }
    DD_HIP_CHECK(hipMemcpy(host, n->x0, sizeof(float) * count, hipMemcpyDeviceToHost));
    return DD_OK;
  }
  const CnnLayer& L = n->L[layer];
  const size_t pix = (size_t)B * L.Hout * L.Wout;
  if (layer == NL - 1) {
    if (count != pix * L.cout) { dd_set_error("dd_cnn_debug_activation: count must be %zu", pix * L.cout); return DD_EINVAL; }
    DD_HIP_CHECK(hipMemcpy(host, n->out, sizeof(float) * count, hipMemcpyDeviceToHost));
    return DD_OK;
  }
  if (count != pix * L.cout) { dd_set_error("dd_cnn_debug_activation: count must be %zu", pix * L.cout); return DD_EINVAL; }
  std::vector<bf16> tmp(pix * L.coutp);
  DD_HIP_CHECK(hipMemcpy(tmp.data(), n->act[layer], sizeof(bf16) * tmp.size(), hipMemcpyDeviceToHost));
  for (size_t p = 0; p < pix; ++p)
    for (int c = 0; c < L.cout; ++c) host[p * L.cout + c] = (float)tmp[p * L.coutp + c];
  return DD_OK;
}
