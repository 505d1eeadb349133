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
#include "predfile.h"
#include "resloss.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

#define NL 8
#define CNN_EPS_LO 2.085f
#define CNN_EPS_HI 12.25f

enum { MAP_S1 = 0, MAP_S2 = 1, MAP_UP = 2 };

struct CnnLayer {
  int cin, cout, stride, up, relu;
  int cinp, coutp;           // padded channel counts (32, 64 or 128; layer 1's cin stays 1 or 3)
  int Hin, Win, Hout, Wout;  // per-image grid sizes
  size_t woff, boff;         // offsets of weights / bias in the parameter vector
  int mode;                  // MAP_S1, MAP_S2 or MAP_UP
};

struct dd_cnn {
  int nx, ny, maxB, k;
  int cin0;                  // input planes: 1 (permittivity) or 3 (+ effective-index field)
  int ncu = 1;               // compute units of the device the network was created on
  CnnLayer L[NL];
  size_t nparams = 0;
  float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
  int adam_t = 0;
  bf16* wf[NL] = {};
  bf16* wb[NL] = {};
  bf16* wu[NL] = {};         // upsampled layers: effective backward-data weights [16][cinp][coutp]
  float* x0 = nullptr;       // normalised input planes [B][cin0][H][W]
  double* iscale = nullptr;  // [maxB] effective-index field scale sqrt(D) / ||F||
  double* espart = nullptr;  // [maxB][ES_SLICES] partial sums of |F|^2
  // residual-loss scratch (allocated on first use): V = output fields, W = A V,
  // r = b - W c, s = A^H r
  float2 *rl_W = nullptr, *rl_r = nullptr, *rl_s = nullptr;
  void* rl_scratch = nullptr;      // residual-loss descriptors, coefficients, Gram partials
  size_t rl_scratch_bytes = 0;
  bf16* act[NL] = {};        // act[l] = output of layer l (l < NL-1), NHWC bf16
  float* out = nullptr;      // last layer output: complex fields [B][k][D] (FP32 pairs)
  const float* last_fields = nullptr;   // where the last forward pass wrote its fields
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

// ------------------------------------------ convolutions as MFMA GEMMs ----
// Forward: out[p][r] = act(bias[r] + sum_{tap,c} Wf[tap][r][c] *
//   src[map(p, tap)][c]), p over output pixels, r < M = coutp.
// Backward data: dzprev[q][r] = mask(q, r) * sum_{tap,c} Wb[tap][r][c] *
//   dz[gather(q, tap)][c], q over layer-input pixels, r < M = cinp, mask = the
//   ReLU mask of the previous layer's output (the layer input).
// Operands of v_mfma_f32_16x16x32_bf16: A = 16 rows (result channels) x 32
// source channels of one tap's weights, B = 32 source channels x 16 pixels;
// lane l holds row / pixel l % 16 and channels 8 (l / 16) .. 8 (l / 16) + 7
// (16-byte reads of NHWC data); the accumulator holds rows 4 (l / 16) .. + 3
// of pixel l % 16.  MT = M / 16 row tiles.
struct GemmArgs {
  const bf16* src;       // forward: layer input; backward: dz of this layer
  const bf16* W;         // Wf or Wb
  const float* bias;     // forward only
  const bf16* mask;      // backward: layer input activations (ReLU mask)
  bf16* out;             // bf16 result (NHWC, M channels)
  float* outf;           // final layer: complex fields [B][nreal / 2][Hq Wq] (FP32 pairs)
  int nreal;             // real channels of the final layer (2 k)
  int B, Hq, Wq;         // grid of the result pixels
  int Hs, Ws;            // grid of the source pixels
  int Ksrc;              // channels of the source (multiple of 32)
  int M;                 // result channels (= 16 MT)
  int mode, relu;
};

// Final-layer epilogue: channels r0..r0+3 of pixel e of image b are (Re, Im)
// of fields r0 / 2 and r0 / 2 + 1; they go to the complex field layout
// [B][kf][D] (16 lanes with consecutive pixels write 128 contiguous bytes).
__device__ __forceinline__ void store_fields(float* outf, int kf, int D, int b, int e, int r0,
                                             const float* v) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = r0 / 2 + h;
    if (j < kf)
      *(float2*)(outf + (((size_t)b * kf + j) * D + e) * 2) = make_float2(v[2 * h], v[2 * h + 1]);
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
// weights come from the L2-resident packed copy.  Operand layouts are those
// described at GemmArgs.
#define CT_TH 4
#define CT_TW 64
#define CT_PH (CT_TH + 2)
#define CT_PW (CT_TW + 2)
#define CT_PS 40   // bf16 per staged pixel: 32 channels + 8 of padding (80-byte stride)
template <int MT, bool BWD = false, bool WL = false>
__global__ __launch_bounds__(256) void k_conv_tile(GemmArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 patch[CT_PH * CT_PW * CT_PS];
  // WL: the chunk's weights of all nine taps are staged in LDS with the patch
  // ([tap][row][40], 80-byte rows), so the tap loop waits on no global load
  __shared__ __attribute__((aligned(16))) bf16 wl[WL ? 9 * 16 * MT * CT_PS : 8];
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
  // weight operand of tap t of the chunk at c0 (rows i * 16 + lane % 16)
  auto wload = [&](int t, int c0, bf16x8 (&av)[MT]) {
    const bf16* wt = a.W + (size_t)(BWD ? 8 - t : t) * a.M * a.Ksrc + c0 + kq;
#pragma unroll
    for (int i = 0; i < MT; ++i) av[i] = load8(wt + (size_t)(i * 16 + (lane & 15)) * a.Ksrc);
  };
  constexpr int NSTG = (CT_PH * CT_PW * 4 + 255) / 256;   // staging loads per thread
  constexpr int NWI = 9 * 16 * MT * 4, NWS = WL ? (NWI + 255) / 256 : 1;   // weight items
  for (int c0 = 0; c0 < a.Ksrc; c0 += 32) {
    // all of this thread's patch loads are issued before the first LDS store,
    // and tap 0's weights are in flight meanwhile
    bf16x8 wcur[MT], wnext[MT];
    u32x4 wv[NWS];
    if (WL) {
#pragma unroll
      for (int it = 0; it < NWS; ++it) {
        const int u = threadIdx.x + 256 * it;   // (tap, row, quarter)
        const int tq = u / (16 * MT * 4), rem = u - tq * 16 * MT * 4;
        wv[it] = u32x4{0u, 0u, 0u, 0u};
        if (u < NWI)
          wv[it] = *(const u32x4*)(a.W + ((size_t)(BWD ? 8 - tq : tq) * a.M + (rem >> 2)) * a.Ksrc +
                                   c0 + 8 * (rem & 3));
      }
    } else {
      wload(0, c0, wcur);
    }
    u32x4 sv[NSTG];
#pragma unroll
    for (int it = 0; it < NSTG; ++it) {
      const int u = threadIdx.x + 256 * it;
      const int pix = u >> 2, q = u & 3;
      const int py = pix / CT_PW, px = pix - py * CT_PW;
      const int uy = y0 + py - 1, ux = x0 + px - 1;   // conv-input grid (= output grid)
      sv[it] = u32x4{0u, 0u, 0u, 0u};
      if (u < CT_PH * CT_PW * 4 && uy >= 0 && uy < Hq && ux >= 0 && ux < Wq) {
        const int sy = up ? (uy >> 1) : uy, sx = up ? (ux >> 1) : ux;
        sv[it] = *(const u32x4*)(a.src + ((size_t)(b * a.Hs + sy) * a.Ws + sx) * a.Ksrc + c0 + 8 * q);
      }
    }
#pragma unroll
    for (int it = 0; it < NSTG; ++it) {
      const int u = threadIdx.x + 256 * it;
      if (u < CT_PH * CT_PW * 4) *(u32x4*)(patch + (u >> 2) * CT_PS + 8 * (u & 3)) = sv[it];
    }
    if (WL) {
#pragma unroll
      for (int it = 0; it < NWS; ++it) {
        const int u = threadIdx.x + 256 * it;
        if (u < NWI) *(u32x4*)(wl + (u >> 2) * CT_PS + 8 * (u & 3)) = wv[it];
      }
    }
    __syncthreads();
    // taps: the next tap's weights are loaded while this tap's MFMAs run
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {
      if (WL) {
#pragma unroll
        for (int i = 0; i < MT; ++i)
          wcur[i] = *(const bf16x8*)(wl + ((t * 16 * MT) + i * 16 + (lane & 15)) * CT_PS + kq);
      } else if (t + 1 < 9) {
        wload(t + 1, c0, wnext);
      }
      const int dy = t / 3, dx = t - 3 * (t / 3);
      bf16x8 bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bv[j] = *(const bf16x8*)(patch + ((wave + dy) * CT_PW + 16 * j + (lane & 15) + dx) * CT_PS + kq);
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wcur[i], bv[j], acc[i][j], 0, 0, 0);
      if (!WL && t + 1 < 9) {
#pragma unroll
        for (int i = 0; i < MT; ++i) wcur[i] = wnext[i];
      }
    }
    __syncthreads();
  }
  const int y = y0 + wave;
  if (y >= Hq) return;
  // epilogue operands (bias, or the ReLU mask of the layer input) are all
  // loaded before any result is stored
  float4 bias4[MT];
  u32x2 mk[MT][4];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const int r0 = i * 16 + 4 * (lane >> 4);
    if (!BWD) bias4[i] = *(const float4*)(a.bias + r0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = x0 + 16 * j + (lane & 15);
      mk[i][j] = u32x2{0u, 0u};
      if (BWD && x < Wq)
        mk[i][j] = *(const u32x2*)(a.mask + (((size_t)b * Hq + y) * Wq + x) * a.M + r0);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int x = x0 + 16 * j + (lane & 15);
    if (x >= Wq) continue;
    const size_t p = ((size_t)b * Hq + y) * Wq + x;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const int r0 = i * 16 + 4 * (lane >> 4);
      float v[4];
      if (BWD) {
        const bf16x4 m4 = __builtin_bit_cast(bf16x4, mk[i][j]);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = ((float)m4[q] > 0.f) ? acc[i][j][q] : 0.f;
      } else {
        const float bq[4] = {bias4[i].x, bias4[i].y, bias4[i].z, bias4[i].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          v[q] = acc[i][j][q] + bq[q];
          if (a.relu) v[q] = fmaxf(v[q], 0.f);
        }
      }
      if (!BWD && a.outf) {
        store_fields(a.outf, a.nreal / 2, Hq * Wq, b, y * Wq + x, r0, v);
      } else {
        bf16 h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = (bf16)v[q];
        *(u32x2*)(a.out + p * a.M + r0) = __builtin_bit_cast(u32x2, h);
      }
    }
  }
}

// Stride-2 reads from LDS, for two passes of the same form: output pixel
// (y, x) of a 4 x 32 tile sums taps (ty, tx) over a KS x KS window of the
// source at (2 y - 1 + ty, 2 x - 1 + tx), weight tap KS ty + tx:
//  * KS = 3, forward of the stride-2 layers: source = layer input, weights Wf,
//    bias and ReLU epilogue;
//  * KS = 4, backward data of the upsampling layers (BWD): source = dz on the
//    upsampled grid, the 16 effective weights of k_pack_up_weights, ReLU-mask
//    epilogue.
// A workgroup stages the (2 CS_TH + KS - 2) x (2 CS_TW + KS - 2) source patch of
// its tile in LDS per 32 source channels (zero padding resolved while staging)
// and applies the taps from there; wave w owns output row y0 + w (two pixel
// tiles of 16).  Loads are issued as in k_conv_tile, and WL stages the
// weights in LDS as there; operand layouts are those described at GemmArgs.
#define CS_TH 4
#define CS_TW 32
template <int MT, int KS, bool BWD, bool WL = false>
__global__ __launch_bounds__(256) void k_conv_tile_s2(GemmArgs a) {
  constexpr int PH = 2 * CS_TH + KS - 2, PW = 2 * CS_TW + KS - 2, NTAP = KS * KS;
  __shared__ __attribute__((aligned(16))) bf16 patch[PH * PW * CT_PS];
  // WL: the chunk's weights, staged with the patch ([tap][row][40]) in groups
  // of NTW taps (all nine for KS = 3; two groups of eight for the 16 taps of
  // KS = 4, whose weights would not fit LDS at once)
  constexpr int NTW = WL ? (NTAP > 9 ? NTAP / 2 : NTAP) : 1;
  __shared__ __attribute__((aligned(16))) bf16 wl[WL ? NTW * 16 * MT * CT_PS : 8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x0 = blockIdx.x * CS_TW, y0 = blockIdx.y * CS_TH, b = blockIdx.z;
  const int Hq = a.Hq, Wq = a.Wq;
  f32x4 acc[MT][2];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = 8 * (lane >> 4);
  auto wload = [&](int t, int c0, bf16x8 (&av)[MT]) {
    const bf16* wt = a.W + (size_t)t * a.M * a.Ksrc + c0 + kq;
#pragma unroll
    for (int i = 0; i < MT; ++i) av[i] = load8(wt + (size_t)(i * 16 + (lane & 15)) * a.Ksrc);
  };
  constexpr int NSTG = (PH * PW * 4 + 255) / 256;
  constexpr int NWI = WL ? NTW * 16 * MT * 4 : 0, NWS = (NWI + 255) / 256;
  u32x4 wv[NWS > 0 ? NWS : 1];
  // weights of taps g0 .. g0 + NTW - 1 of chunk c0 into registers, then LDS
  auto wfetch = [&](int g0, int c0) {
#pragma unroll
    for (int it = 0; it < NWS; ++it) {
      const int u = threadIdx.x + 256 * it;   // (tap, row, quarter)
      const int tq = u / (16 * MT * 4), rem = u - tq * 16 * MT * 4;
      wv[it] = u32x4{0u, 0u, 0u, 0u};
      if (u < NWI)
        wv[it] = *(const u32x4*)(a.W + ((size_t)(g0 + tq) * a.M + (rem >> 2)) * a.Ksrc + c0 +
                                 8 * (rem & 3));
    }
  };
  auto wstore = [&]() {
#pragma unroll
    for (int it = 0; it < NWS; ++it) {
      const int u = threadIdx.x + 256 * it;
      if (u < NWI) *(u32x4*)(wl + (u >> 2) * CT_PS + 8 * (u & 3)) = wv[it];
    }
  };
  // without WL the 9-tap kernels keep the weights of the next PD taps in
  // flight in a register ring (a tap's MFMAs are too few to cover an L2 load
  // one tap ahead); the 16-tap kernels load one tap ahead (a ring cost them
  // occupancy)
  constexpr int PD = (WL || KS == 4) ? 1 : (NTAP < 16 / MT ? NTAP : 16 / MT);
  for (int c0 = 0; c0 < a.Ksrc; c0 += 32) {
    bf16x8 wcur[MT], wr[PD][MT];
    if (WL) {
      wfetch(0, c0);
    } else {
#pragma unroll
      for (int d = 0; d < PD; ++d) wload(d, c0, wr[d]);
    }
    u32x4 sv[NSTG];
#pragma unroll
    for (int it = 0; it < NSTG; ++it) {
      const int u = threadIdx.x + 256 * it;
      const int pix = u >> 2, q = u & 3;
      const int py = pix / PW, px = pix - py * PW;
      const int sy = 2 * y0 + py - 1, sx = 2 * x0 + px - 1;   // source grid
      sv[it] = u32x4{0u, 0u, 0u, 0u};
      if (u < PH * PW * 4 && sy >= 0 && sy < a.Hs && sx >= 0 && sx < a.Ws)
        sv[it] = *(const u32x4*)(a.src + ((size_t)(b * a.Hs + sy) * a.Ws + sx) * a.Ksrc + c0 + 8 * q);
    }
#pragma unroll
    for (int it = 0; it < NSTG; ++it) {
      const int u = threadIdx.x + 256 * it;
      if (u < PH * PW * 4) *(u32x4*)(patch + (u >> 2) * CT_PS + 8 * (u & 3)) = sv[it];
    }
    if (WL) wstore();
    __syncthreads();
    // MFMAs of tap t with weights w
    auto tap = [&](int t, const bf16x8 (&w)[MT]) {
      const int ty = t / KS, tx = t - KS * (t / KS);
      bf16x8 bv[2];
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bv[j] = *(const bf16x8*)(patch + ((2 * wave + ty) * PW + 2 * (16 * j + (lane & 15)) + tx) *
                                             CT_PS + kq);
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[i], bv[j], acc[i][j], 0, 0, 0);
    };
    if constexpr (WL) {
#pragma unroll 1
      for (int t = 0; t < NTAP; ++t) {
        if (t > 0 && t % NTW == 0) {   // next tap group (only for NTW < NTAP)
          __syncthreads();
          wfetch(t, c0);
          wstore();
          __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < MT; ++i)
          wcur[i] = *(const bf16x8*)(wl + ((t % NTW) * 16 * MT + i * 16 + (lane & 15)) * CT_PS + kq);
        tap(t, wcur);
      }
    } else if constexpr (PD == 1) {
#pragma unroll 1
      for (int t = 0; t < NTAP; ++t) {
        bf16x8 wnext[MT];
        if (t + 1 < NTAP) wload(t + 1, c0, wnext);
        tap(t, wr[0]);
        if (t + 1 < NTAP) {
#pragma unroll
          for (int i = 0; i < MT; ++i) wr[0][i] = wnext[i];
        }
      }
    } else {
#pragma unroll 1
      for (int tg = 0; tg < NTAP; tg += PD) {
#pragma unroll
        for (int d = 0; d < PD; ++d) {
          const int t = tg + d;
          if (t < NTAP) tap(t, wr[d]);
          if (t + PD < NTAP) wload(t + PD, c0, wr[d]);
        }
      }
    }
    __syncthreads();
  }
  const int y = y0 + wave;
  if (y >= Hq) return;
  float4 bias4[MT];
  u32x2 mk[MT][2];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const int r0 = i * 16 + 4 * (lane >> 4);
    if (!BWD) bias4[i] = *(const float4*)(a.bias + r0);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int x = x0 + 16 * j + (lane & 15);
      mk[i][j] = u32x2{0u, 0u};
      if (BWD && x < Wq)
        mk[i][j] = *(const u32x2*)(a.mask + (((size_t)b * Hq + y) * Wq + x) * a.M + r0);
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int x = x0 + 16 * j + (lane & 15);
    if (x >= Wq) continue;
    const size_t p = ((size_t)b * Hq + y) * Wq + x;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const int r0 = i * 16 + 4 * (lane >> 4);
      bf16 h[4];
      if (BWD) {
        const bf16x4 m4 = __builtin_bit_cast(bf16x4, mk[i][j]);
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = (bf16)(((float)m4[q] > 0.f) ? acc[i][j][q] : 0.f);
      } else {
        const float bq[4] = {bias4[i].x, bias4[i].y, bias4[i].z, bias4[i].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float v = acc[i][j][q] + bq[q];
          if (a.relu) v = fmaxf(v, 0.f);
          h[q] = (bf16)v;
        }
      }
      *(u32x2*)(a.out + p * a.M + r0) = __builtin_bit_cast(u32x2, h);
    }
  }
}

// Backward data of the stride-2 layers, LDS-tiled: a workgroup computes an
// 8 x 64 tile of layer-input pixels (all M = 16 MT channels, y0 a multiple of
// 8) from the 5 x 33 dz pixels it reads (rows y0/2 .. y0/2 + 4, columns
// x0/2 .. x0/2 + 32), staged in LDS per 32 dz channels with the weights of
// all nine taps (backward-data copy [tap][cinp][coutp]).  Tap (dy, dx)
// reaches input row y only when y + 1 - dy is even (dy = 1 at even y, 0 and 2
// at odd y) and column x only when x + 1 - dx is even (dx = 1 at even x, 0
// and 2 at odd x).  Wave w owns the even row y0 + 2w and the odd row
// y0 + 2w + 1, four pixel tiles of 16 each: even columns x0 + 2i (tiles 0,
// 1) and odd columns x0 + 2i + 1 (tiles 2, 3), so every wave applies each of
// the nine taps to two tiles.  Per dz row a wave reads two B operands per
// tile pair (dz column c for dx = 1 at even x and dx = 2 at odd x, column c + 1
// for dx = 0 at odd x); dz row w serves dy = 1 of the even row and dy = 2 of
// the odd row.  The next chunk's patch and weights are loaded while the
// current chunk's MFMAs run.  The epilogue masks by the ReLU of the layer
// input.
#define BS_TH 8
#define BS_TW 64
#define BS_PR 5
#define BS_PC 34
template <int MT>
__global__ __launch_bounds__(256) void k_bwd_s2_tile(GemmArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 patch[BS_PR * BS_PC * CT_PS];
  __shared__ __attribute__((aligned(16))) bf16 wl[9 * 16 * MT * CT_PS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x0 = blockIdx.x * BS_TW, y0 = blockIdx.y * BS_TH, b = blockIdx.z;
  const int Hq = a.Hq, Wq = a.Wq, py0 = y0 / 2, px0 = x0 / 2;
  f32x4 acc[2][4][MT];   // [row: even, odd][tile][row tile]
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < MT; ++i) acc[h][j][i] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = 8 * (lane >> 4);
  constexpr int NPI = BS_PR * BS_PC * 4, NSTG = (NPI + 255) / 256;   // patch items
  constexpr int NWI = 9 * 16 * MT * 4, NWS = (NWI + 255) / 256;      // weight items
  u32x4 sv[NSTG], wv[NWS];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int it = 0; it < NWS; ++it) {
      const int u = threadIdx.x + 256 * it;   // (tap, row, quarter)
      const int tq = u / (16 * MT * 4), rem = u - tq * 16 * MT * 4;
      wv[it] = u32x4{0u, 0u, 0u, 0u};
      if (u < NWI)
        wv[it] = *(const u32x4*)(a.W + ((size_t)tq * a.M + (rem >> 2)) * a.Ksrc + c0 + 8 * (rem & 3));
    }
#pragma unroll
    for (int it = 0; it < NSTG; ++it) {
      const int u = threadIdx.x + 256 * it;
      const int pix = u >> 2, q = u & 3;
      const int pr = pix / BS_PC, pc = pix - pr * BS_PC;
      const int sy = py0 + pr, sx = px0 + pc;   // dz grid
      sv[it] = u32x4{0u, 0u, 0u, 0u};
      if (u < NPI && sy < a.Hs && sx < a.Ws)
        sv[it] = *(const u32x4*)(a.src + ((size_t)(b * a.Hs + sy) * a.Ws + sx) * a.Ksrc + c0 + 8 * q);
    }
  };
  fetch(0);
  for (int c0 = 0; c0 < a.Ksrc; c0 += 32) {
    __syncthreads();   // the previous chunk's readers are done
#pragma unroll
    for (int it = 0; it < NSTG; ++it) {
      const int u = threadIdx.x + 256 * it;
      if (u < NPI) *(u32x4*)(patch + (u >> 2) * CT_PS + 8 * (u & 3)) = sv[it];
    }
#pragma unroll
    for (int it = 0; it < NWS; ++it) {
      const int u = threadIdx.x + 256 * it;
      if (u < NWI) *(u32x4*)(wl + (u >> 2) * CT_PS + 8 * (u & 3)) = wv[it];
    }
    __syncthreads();
    if (c0 + 32 < a.Ksrc) fetch(c0 + 32);
    // dz rows w (r = 0) and w + 1 (r = 1) of the patch
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      bf16x8 bc[2], bn[2];   // dz columns c and c + 1 of the two tile pairs
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const bf16* pp = patch + ((wave + r) * BS_PC + 16 * jj + (lane & 15)) * CT_PS + kq;
        bc[jj] = *(const bf16x8*)pp;
        bn[jj] = *(const bf16x8*)(pp + CT_PS);
      }
      // (input row h, dy): r = 0 serves (even, 1) and (odd, 2); r = 1 serves (odd, 0)
#pragma unroll
      for (int s2 = 0; s2 < 2 - r; ++s2) {
        const int h = (r == 0 && s2 == 0) ? 0 : 1;
        const int dy = (r == 1) ? 0 : (s2 == 0 ? 1 : 2);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          bf16x8 wcur[MT];
#pragma unroll
          for (int i = 0; i < MT; ++i)
            wcur[i] = *(const bf16x8*)(wl + ((3 * dy + dx) * 16 * MT + i * 16 + (lane & 15)) *
                                                CT_PS + kq);
          // dx = 1: even tiles 0, 1 from column c; dx = 2: odd tiles from
          // column c; dx = 0: odd tiles from column c + 1
          const int j0 = (dx == 1) ? 0 : 2;
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            const bf16x8 bv = (dx == 0) ? bn[jj] : bc[jj];
#pragma unroll
            for (int i = 0; i < MT; ++i)
              acc[h][j0 + jj][i] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(wcur[i], bv, acc[h][j0 + jj][i], 0, 0, 0);
          }
        }
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int y = y0 + 2 * wave + h;
    if (y >= Hq) break;
    u32x2 mk[4][MT];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = x0 + 2 * (16 * (j & 1) + (lane & 15)) + (j >> 1);
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        mk[j][i] = u32x2{0u, 0u};
        if (x < Wq)
          mk[j][i] = *(const u32x2*)(a.mask + (((size_t)b * Hq + y) * Wq + x) * a.M + i * 16 +
                                     4 * (lane >> 4));
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = x0 + 2 * (16 * (j & 1) + (lane & 15)) + (j >> 1);
      if (x >= Wq) continue;
      const size_t p = ((size_t)b * Hq + y) * Wq + x;
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const bf16x4 m4 = __builtin_bit_cast(bf16x4, mk[j][i]);
        bf16 hv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) hv[q] = (bf16)(((float)m4[q] > 0.f) ? acc[h][j][i][q] : 0.f);
        *(u32x2*)(a.out + p * a.M + i * 16 + 4 * (lane >> 4)) = __builtin_bit_cast(u32x2, hv);
      }
    }
  }
}

// ------------------------------------------------------------- layer 1 ----
// Cin = 1 or 3 input planes, 32 output channels, FP32 throughout on the
// matrix cores: per 16 output pixels the product W[32][9C] . X[9C][16] runs as
// FP32 16x16x4 MFMAs over K = 9C padded to a multiple of 4 (k = 9 c + tap,
// padded rows zero).  Lane l supplies weight row l % 16 / k-slot l / 16 and
// the input of pixel l % 16 at k-slot l / 16; its accumulators hold output
// channels 4 (l / 16) + q of pixel l % 16.  A wave takes C1_NT tiles of 16
// consecutive pixels (row-major over [B][H][W]) and issues every input load
// before its first MFMA; 8-byte bf16 stores of 4 channels.  x0 is planar
// [B][C][H][W], w is [32][C][9].
#define C1_NT 8
template <int C>
__global__ __launch_bounds__(256) void k_conv1_fwd(const float* __restrict__ x0,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ bias, int B, int H,
                                                   int W, bf16* __restrict__ out) {
  constexpr int KS = (9 * C + 3) / 4;   // k-steps of 4
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ks = lane >> 4, col = lane & 15;
  const int total = B * H * W;
  float av[2][KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = 4 * s + ks;
#pragma unroll
    for (int i = 0; i < 2; ++i) av[i][s] = (k < 9 * C) ? w[(16 * i + col) * 9 * C + k] : 0.f;
  }
  // per k-slot: plane offset and tap shift, the same for every pixel tile
  const int HW = H * W;
  int koff[KS], kdy[KS], kdx[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = 4 * s + ks, c = k / 9, t = k - 9 * c;
    kdy[s] = (k < 9 * C) ? t / 3 - 1 : -H;   // padded k-slots fall outside every row
    kdx[s] = t % 3 - 1;
    koff[s] = c * HW + kdy[s] * W + kdx[s];
  }
  const int base = (blockIdx.x * 4 + wave) * 16 * C1_NT;
  float bv[C1_NT][KS];
  // (b, y, x) of this lane's pixel, advanced by 16 pixels per tile
  int b = (unsigned)(base + col) / (unsigned)HW, x = base + col - b * HW;
  int y = (unsigned)x / (unsigned)W;
  x -= y * W;
#pragma unroll
  for (int j = 0; j < C1_NT; ++j) {
    const int p = base + 16 * j + col;
    if (j > 0) {
      x += 16;
      while (x >= W) {
        x -= W;
        if (++y == H) { y = 0; ++b; }
      }
    }
    const int pb = p + b * (C - 1) * HW;   // element (b, 0, y, x) of the planar input
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      // out-of-range taps read element 0 and are zeroed after the load, so
      // every load is issued unconditionally
      const bool ok = (p < total) & ((unsigned)(y + kdy[s]) < (unsigned)H) &
                      ((unsigned)(x + kdx[s]) < (unsigned)W);
      const float v = x0[ok ? (unsigned)(pb + koff[s]) : 0u];
      bv[j][s] = ok ? v : 0.f;
    }
  }
  float bq[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) bq[i][q] = bias[16 * i + 4 * ks + q];
#pragma unroll
  for (int j = 0; j < C1_NT; ++j) {
    f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][s], bv[j][s], acc[i], 0, 0, 0);
    const int p = base + 16 * j + col;
    if (p >= total) continue;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      bf16 h[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) h[q] = (bf16)fmaxf(acc[i][q] + bq[i][q], 0.f);
      *(u32x2*)(out + (size_t)p * 32 + 16 * i + 4 * ks) = __builtin_bit_cast(u32x2, h);
    }
  }
}

// --------------------------------------------------- weight gradients ----
// Weight gradients of a 3x3 layer (stride 1, stride 2 or upsampling) as GEMMs
// dW[tap][r][c] = sum_p dz[p][r] in[src(p, tap)][c] over stages of PX = 32 S
// pixels of one output row (the last chunk of a row is ragged).  Work items:
// (pixel slice, channel block of NB = 16 NT input channels, dy), dy fastest,
// or with ND = 3 (slice, channel block) taking all three dy.  Per stage the
// workgroup stages in LDS, transposed to [channel][pixel]:
//  * dz of the stage, all Mr = 16 MT output channels;
//  * per dy, the input row the stage reads, NB channels from channel n0,
//    once for the three dx taps:
//    - stride 1 (MK = MAP_S1): input columns x0 - 8 .. x0 + PX + 7 at columns
//      0 .. PX + 15; dx reads at shifts -1, 0, +1;
//    - upsampling (MAP_UP): the same, the source row expanded x2 while
//      staging;
//    - stride 2 (MAP_S2): output pixel p reads input columns 2p - 1, 2p and
//      2p + 1, so the row is split by parity: odd columns 2j + 1 (j = x0 - 1 ..
//      x0 + PX - 1) at columns j - x0 + 8, even columns 2j (j = x0 ..
//      x0 + PX - 1) at columns PX + 8 + j - x0.  dx = 2 and dx = 1 read the
//      odd and even halves aligned, dx = 0 the odd half shifted by one.  The
//      one odd column left of the chunk (2 x0 - 1) is loaded by a thread of
//      its own rather than as a block of 8.
// A staging block is 8 pixels x 8 channels: loaded with 16-byte reads,
// transposed in registers, stored with 16-byte writes; the next stage's
// blocks are loaded while the current stage's MFMAs run.  Shifted operands
// are built from aligned 16-byte LDS reads by funnel shifts.  Per stage that
// moves PX + 16 (stride 1), PX / 2 + 8 (upsampling) or 2 PX + 1 (stride 2)
// input pixels per dy instead of 3 PX.  A wave owns (row tile, column tile)
// units and applies all three dx to each.  The slice's (dy 0, first channel
// block) item also sums dz over its pixels (the bias gradient) as dz^T times
// a column of ones.  Partials: weights [slice][tap][r][c], bias [slice][r].
// (The network's upsampling layers use k_conv_wgrad_up and its 32-channel
// stride-1 layers k_conv_wgrad_ring; the upsampling map here serves other
// channel counts.)
template <int MT, int NT, int S, int MK, int ND = 1>
__global__ __launch_bounds__(256) void k_conv_wgrad_row(const bf16* __restrict__ dz,
                                                        const bf16* __restrict__ x, int B,
                                                        int Hout, int Wout, int Hin, int Win,
                                                        int Nc, int stages_per, int nwork,
                                                        float* __restrict__ part,
                                                        float* __restrict__ bpart) {
  constexpr bool UP = MK == MAP_UP, S2 = MK == MAP_S2;
  constexpr int Mr = 16 * MT, NB = 16 * NT, PX = 32 * S, LD = PX + 8;
  // staged columns per channel and row pitch (a pitch of an odd number of
  // 16-byte units)
  constexpr int XC = S2 ? 2 * PX + 8 : PX + 16, LDX = S2 ? XC : XC + 8;
  constexpr int ABLK = (PX / 8) * (Mr / 8);
  // source groups of 8 pixels (stride 2: odd groups, then even groups)
  constexpr int XG = UP ? (PX / 16 + 1) : S2 ? 2 * (PX / 8) : (PX / 8 + 2);
  constexpr int XBLK = XG * (NB / 8);
  constexpr int NBLK = ABLK + ND * XBLK, BPT = (NBLK + 255) / 256;
  constexpr int NU = MT * NT, PER_WAVE = (NU + 3) / 4;
  static_assert(!S2 || ND * (NB / 8) <= 256, "stride-2 halo loads: one per thread");
  __shared__ __attribute__((aligned(16))) bf16 As[Mr][LD];
  __shared__ __attribute__((aligned(16))) bf16 Xs[ND][NB][LDX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // 1D grid, a multiple of 8 long: consecutive work items (the dy and the
  // channel blocks of one pixel slice) go to the same XCD, whose L2 then
  // serves their shared dz and input rows
  const int w = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  if (w >= nwork) return;
  const int nblk = Nc / NB;
  // ND = 3: one item takes all three dy (first dy0 = 0) and stages dz once
  const int dy0 = (ND == 3) ? 0 : w % 3;
  const int n0 = ((ND == 3) ? w % nblk : (w / 3) % nblk) * NB;
  const int slice = (ND == 3) ? w / nblk : w / (3 * nblk);
  const int nch = (Wout + PX - 1) / PX, nst = B * Hout * nch;
  const int s0 = slice * stages_per, s1 = min(nst, s0 + stages_per);
  bf16x8 reg[BPT][8];
  bf16x8 hreg = zero8();
  unsigned okm[BPT];   // stride 2: bit i, element i of the block is in range
  bool hok = false;
  auto load = [&](int sg) {
    const int b = sg / (Hout * nch), rem = sg - b * Hout * nch, y = rem / nch;
    const int x0 = (rem - y * nch) * PX;
    if constexpr (S2) {
      // Every load is issued unconditionally (reads out of range go to
      // element 0 of their array) and out-of-range values are zeroed when
      // the block is stored to LDS: with conditional loads, or zeroing right
      // after the load, the waves waited for the prefetch before the current
      // stage's MFMAs.  First the odd column 2 x0 - 1 of row rd.
      const bool hv = threadIdx.x < ND * (NB / 8);
      const int rd = hv ? threadIdx.x / (NB / 8) : 0, cg = (threadIdx.x % (NB / 8)) * 8;
      const int ys = 2 * y + dy0 + rd - 1, c = 2 * x0 - 1;
      hok = hv && ys >= 0 && ys < Hin && c >= 0 && c < Win;
      hreg = load8(x + (hok ? (((size_t)b * Hin + ys) * Win + c) * Nc + n0 + cg : 0));
#pragma unroll
      for (int bi = 0; bi < BPT; ++bi) {
        const int blk = threadIdx.x + 256 * bi;
        // element i is input column c0 + 2 i of source row ys (dz: pixel
        // x0 + 8 pg + i), in range for 0 <= column < climit
        const bf16* src = dz;
        long off0 = 0;
        int c0 = 0, cstep = 1, climit = 0, ostep = 0;
        if (blk < ABLK) {
          const int pg = blk / (Mr / 8), cg = (blk % (Mr / 8)) * 8;
          c0 = x0 + pg * 8; climit = Wout; ostep = Mr;
          off0 = (((long)b * Hout + y) * Wout + c0) * Mr + cg;
        } else if (blk < NBLK) {
          const int rd = (blk - ABLK) / XBLK, r = blk - ABLK - rd * XBLK;   // dy row, item
          const int ys = 2 * y + dy0 + rd - 1;
          const int m = r / (NB / 8), cg = (r % (NB / 8)) * 8;
          c0 = 2 * (x0 + 8 * (m % (PX / 8))) + (m < PX / 8 ? 1 : 0);   // odd, then even groups
          cstep = 2;
          climit = (ys >= 0 && ys < Hin) ? Win : 0;
          src = x; ostep = 2 * Nc;
          off0 = (((long)b * Hin + ys) * Win + c0) * Nc + n0 + cg;
        }
        okm[bi] = 0;
        if (blk < NBLK) {   // false only in the last round, for its spare threads
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int c = c0 + cstep * i;
            const bool ok = c >= 0 && c < climit;
            reg[bi][i] = load8(src + (ok ? off0 + (long)i * ostep : 0));
            okm[bi] |= (unsigned)ok << i;
          }
        }
      }
    } else {
#pragma unroll
      for (int bi = 0; bi < BPT; ++bi) {
        const int blk = threadIdx.x + 256 * bi;
#pragma unroll
        for (int i = 0; i < 8; ++i) reg[bi][i] = zero8();
        if (blk < ABLK) {
          const int pg = blk / (Mr / 8), cg = (blk % (Mr / 8)) * 8;
          const bf16* src = dz + (((size_t)b * Hout + y) * Wout + x0) * Mr + cg;
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (x0 + pg * 8 + i < Wout) reg[bi][i] = load8(src + (size_t)(pg * 8 + i) * Mr);
        } else if (blk < NBLK) {
          const int rd = (blk - ABLK) / XBLK, r = blk - ABLK - rd * XBLK;   // dy row, item
          const int uy = y + dy0 + rd - 1;   // row of the stride-1 or upsampled grid
          if (uy >= 0 && uy < Hout) {
            const int ys = UP ? (uy >> 1) : uy;
            const int m = r / (NB / 8), cg = (r % (NB / 8)) * 8;
            const int c0 = UP ? (x0 / 2 - 4 + 8 * m) : (x0 - 8 + 8 * m);   // first source column
            const bf16* src = x + ((size_t)b * Hin + ys) * Win * Nc + n0 + cg;
#pragma unroll
            for (int i = 0; i < 8; ++i)
              if (c0 + i >= 0 && c0 + i < Win) reg[bi][i] = load8(src + (size_t)(c0 + i) * Nc);
          }
        }
      }
    }
  };
  f32x4 acc[PER_WAVE][3 * ND];   // [unit][row (dy - dy0) * 3 + dx]
#pragma unroll
  for (int i = 0; i < PER_WAVE; ++i)
#pragma unroll
    for (int d = 0; d < 3 * ND; ++d) acc[i][d] = f32x4{0.f, 0.f, 0.f, 0.f};
  constexpr int BT = (MT + 3) / 4;
  const bool bias = (dy0 == 0 && n0 == 0);
  f32x4 accb[BT];
#pragma unroll
  for (int i = 0; i < BT; ++i) accb[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ones;
#pragma unroll
  for (int q = 0; q < 8; ++q) ones[q] = (bf16)1.f;
  const int kq = 8 * (lane >> 4);
  if (s0 < s1) load(s0);
  for (int sg = s0; sg < s1; ++sg) {
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < BPT; ++bi) {
      if constexpr (S2) {
#pragma unroll
        for (int i = 0; i < 8; ++i) reg[bi][i] = ((okm[bi] >> i) & 1) ? reg[bi][i] : zero8();
      }
      const int blk = threadIdx.x + 256 * bi;
      if (blk < ABLK) {
        bf16* dst = &As[(blk % (Mr / 8)) * 8][(blk / (Mr / 8)) * 8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          bf16x8 t;
#pragma unroll
          for (int i = 0; i < 8; ++i) t[i] = reg[bi][i][q];
          *(bf16x8*)(dst + q * LD) = t;
        }
      } else if (blk < NBLK) {
        const int rd = (blk - ABLK) / XBLK, r = blk - ABLK - rd * XBLK;
        const int m = r / (NB / 8), cg = (r % (NB / 8)) * 8;
        bf16 (*Xr)[LDX] = Xs[rd];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (UP) {   // source pixel i fills columns 16 m + 2 i and 16 m + 2 i + 1
            bf16x8 lo, hi;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              lo[2 * i] = lo[2 * i + 1] = reg[bi][i][q];
              hi[2 * i] = hi[2 * i + 1] = reg[bi][i + 4][q];
            }
            *(bf16x8*)&Xr[cg + q][16 * m] = lo;
            *(bf16x8*)&Xr[cg + q][16 * m + 8] = hi;
          } else {   // stride 2: odd and even groups both land at column 8 m + 8
            bf16x8 t;
#pragma unroll
            for (int i = 0; i < 8; ++i) t[i] = reg[bi][i][q];
            *(bf16x8*)&Xr[cg + q][S2 ? 8 * m + 8 : 8 * m] = t;
          }
        }
      }
    }
    if (S2 && threadIdx.x < ND * (NB / 8)) {
      const int rd = threadIdx.x / (NB / 8), cg = (threadIdx.x % (NB / 8)) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) Xs[rd][cg + q][7] = hok ? hreg[q] : (bf16)0.f;
    }
    __syncthreads();
    if (sg + 1 < s1) load(sg + 1);
#pragma unroll
    for (int kk = 0; kk < S; ++kk) {
#pragma unroll
      for (int i = 0; i < PER_WAVE; ++i) {
        const int u = wave + 4 * i;
        if (u < NU) {
          const int ti = u / NT, tj = u - ti * NT;
          const bf16x8 av = *(const bf16x8*)&As[ti * 16 + (lane & 15)][kk * 32 + kq];
#pragma unroll
          for (int rd = 0; rd < ND; ++rd) {
            // stride 1 / upsampling: the column of dx = 1; stride 2: the
            // odd column of dx = 2
            const bf16* xr = &Xs[rd][tj * 16 + (lane & 15)][kk * 32 + kq + 8];
            const u32x4 a4 = __builtin_bit_cast(u32x4, *(const bf16x8*)(xr - 8));
            const u32x4 b4 = __builtin_bit_cast(u32x4, *(const bf16x8*)xr);
            // stride 1: the next 8 columns; stride 2: the even columns (dx = 1)
            const u32x4 c4 = __builtin_bit_cast(u32x4, *(const bf16x8*)(xr + (S2 ? PX : 8)));
            // columns shifted by one bf16: word j = high half of word j-1, low half of word j
            const unsigned s0w = (a4[3] >> 16) | (b4[0] << 16), s1w = (b4[0] >> 16) | (b4[1] << 16);
            const unsigned s2w = (b4[1] >> 16) | (b4[2] << 16), s3w = (b4[2] >> 16) | (b4[3] << 16);
            const unsigned s4w = (b4[3] >> 16) | (c4[0] << 16);
            const bf16x8 bl = __builtin_bit_cast(bf16x8, u32x4{s0w, s1w, s2w, s3w});   // dx = 0
            const bf16x8 bm = __builtin_bit_cast(bf16x8, S2 ? c4 : b4);                // dx = 1
            const bf16x8 br = __builtin_bit_cast(bf16x8, S2 ? b4 : u32x4{s1w, s2w, s3w, s4w});   // dx = 2
            acc[i][3 * rd] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl, acc[i][3 * rd], 0, 0, 0);
            acc[i][3 * rd + 1] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bm, acc[i][3 * rd + 1], 0, 0, 0);
            acc[i][3 * rd + 2] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, br, acc[i][3 * rd + 2], 0, 0, 0);
          }
        }
      }
      if (bias) {
#pragma unroll
        for (int i = 0; i < BT; ++i) {
          const int ti = wave + 4 * i;
          if (ti < MT) {
            const bf16x8 av = *(const bf16x8*)&As[ti * 16 + (lane & 15)][kk * 32 + kq];
            accb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, ones, accb[i], 0, 0, 0);
          }
        }
      }
    }
  }
  if (bias) {
#pragma unroll
    for (int i = 0; i < BT; ++i) {
      const int ti = wave + 4 * i;
      if (ti < MT && (lane & 15) == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) bpart[(size_t)slice * Mr + ti * 16 + 4 * (lane >> 4) + q] = accb[i][q];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < PER_WAVE; ++i) {
    const int u = wave + 4 * i;
    if (u < NU) {
      const int ti = u / NT, tj = u - ti * NT;
      const int c = tj * 16 + (lane & 15);
#pragma unroll
      for (int d = 0; d < 3 * ND; ++d) {   // tap (dy0 + d / 3) * 3 + d % 3 = 3 dy0 + d
        float* out = part + (((size_t)slice * 9 + dy0 * 3 + d) * Mr) * Nc + n0;
#pragma unroll
        for (int q = 0; q < 4; ++q) out[(size_t)(ti * 16 + 4 * (lane >> 4) + q) * Nc + c] = acc[i][d][q];
      }
    }
  }
}

// Weight gradients of a stride-1 layer, all three dy per work item, with the
// input rows kept in a ring: a slice's stages walk down one column chunk
// (stage order image, chunk, row), so stage y needs input rows y - 1, y and
// y + 1 and the next stage only row y + 2, which replaces row y - 1 in the
// ring of three staged rows.  A stage therefore loads its dz row and one
// input row (k_conv_wgrad_row with all three dy loads three input rows).  At
// the first stage of a slice, and where the walk enters a new chunk or image,
// rows y - 1 and y are loaded as well.  Staging blocks, the column shifts of
// the three dx taps and the partials are those of k_conv_wgrad_row (dsplit 1).
template <int MT, int NT, int S>
__global__ __launch_bounds__(256) void k_conv_wgrad_ring(const bf16* __restrict__ dz,
                                                         const bf16* __restrict__ x, int B,
                                                         int H, int W, int Nc, int stages_per,
                                                         int nwork, float* __restrict__ part,
                                                         float* __restrict__ bpart) {
  constexpr int Mr = 16 * MT, NB = 16 * NT, PX = 32 * S, LD = PX + 8;
  constexpr int XC = PX + 16, LDX = XC + 8;          // staged columns x0 - 8 .. x0 + PX + 7
  constexpr int ABLK = (PX / 8) * (Mr / 8);
  constexpr int XBLK = (PX / 8 + 2) * (NB / 8);      // one input row
  constexpr int NBLK = ABLK + XBLK, BPT = (NBLK + 255) / 256;
  constexpr int NU = MT * NT, PER_WAVE = (NU + 3) / 4;
  __shared__ __attribute__((aligned(16))) bf16 As[Mr][LD];
  __shared__ __attribute__((aligned(16))) bf16 Xs[3][NB][LDX];   // ring: row r in slot r mod 3
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int w = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  if (w >= nwork) return;
  const int nblk = Nc / NB;
  const int n0 = (w % nblk) * NB, slice = w / nblk;
  const int nch = (W + PX - 1) / PX, nst = B * nch * H;
  const int s0 = slice * stages_per, s1 = min(nst, s0 + stages_per);
  auto slot = [](int r) { return (r + 3) % 3; };   // r >= -1
  bf16x8 reg[BPT][8];
  // input row ry (zeros outside the image) of chunk x0 into the X blocks'
  // registers; with dzrow, dz row y of the chunk into the A blocks' too
  auto load = [&](int b, int x0, int y, int ry, bool dzrow) {
#pragma unroll
    for (int bi = 0; bi < BPT; ++bi) {
      const int blk = threadIdx.x + 256 * bi;
#pragma unroll
      for (int i = 0; i < 8; ++i) reg[bi][i] = zero8();
      if (blk < ABLK) {
        if (dzrow) {
          const int pg = blk / (Mr / 8), cg = (blk % (Mr / 8)) * 8;
          const bf16* src = dz + (((size_t)b * H + y) * W + x0) * Mr + cg;
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (x0 + pg * 8 + i < W) reg[bi][i] = load8(src + (size_t)(pg * 8 + i) * Mr);
        }
      } else if (blk < NBLK && ry >= 0 && ry < H) {
        const int r = blk - ABLK, m = r / (NB / 8), cg = (r % (NB / 8)) * 8;
        const int c0 = x0 - 8 + 8 * m;   // first source column
        const bf16* src = x + ((size_t)b * H + ry) * W * Nc + n0 + cg;
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (c0 + i >= 0 && c0 + i < W) reg[bi][i] = load8(src + (size_t)(c0 + i) * Nc);
      }
    }
  };
  auto store = [&](int xslot, bool dzrow) {
#pragma unroll
    for (int bi = 0; bi < BPT; ++bi) {
      const int blk = threadIdx.x + 256 * bi;
      if (blk < ABLK) {
        if (dzrow) {
          bf16* dst = &As[(blk % (Mr / 8)) * 8][(blk / (Mr / 8)) * 8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            bf16x8 t;
#pragma unroll
            for (int i = 0; i < 8; ++i) t[i] = reg[bi][i][q];
            *(bf16x8*)(dst + q * LD) = t;
          }
        }
      } else if (blk < NBLK) {
        const int r = blk - ABLK, m = r / (NB / 8), cg = (r % (NB / 8)) * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          bf16x8 t;
#pragma unroll
          for (int i = 0; i < 8; ++i) t[i] = reg[bi][i][q];
          *(bf16x8*)&Xs[xslot][cg + q][8 * m] = t;
        }
      }
    }
  };
  auto decode = [&](int sg, int& b, int& x0, int& y) {
    b = sg / (nch * H);
    const int rem = sg - b * nch * H, ch = rem / H;
    y = rem - ch * H;
    x0 = ch * PX;
  };
  f32x4 acc[PER_WAVE][9];   // [unit][dy * 3 + dx]
#pragma unroll
  for (int i = 0; i < PER_WAVE; ++i)
#pragma unroll
    for (int d = 0; d < 9; ++d) acc[i][d] = f32x4{0.f, 0.f, 0.f, 0.f};
  constexpr int BT = (MT + 3) / 4;
  const bool bias = (n0 == 0);
  f32x4 accb[BT];
#pragma unroll
  for (int i = 0; i < BT; ++i) accb[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ones;
#pragma unroll
  for (int q = 0; q < 8; ++q) ones[q] = (bf16)1.f;
  const int kq = 8 * (lane >> 4);
  if (s0 < s1) {
    int b, x0, y;
    decode(s0, b, x0, y);
    load(b, x0, y, y + 1, true);
  }
  for (int sg = s0; sg < s1; ++sg) {
    int b, x0, y;
    decode(sg, b, x0, y);
    __syncthreads();   // the previous stage's readers of As and of row y - 2's slot are done
    store(slot(y + 1), true);
    if (sg == s0 || y == 0) {   // a new walk: rows y - 1 and y as well
      for (int r = y - 1; r <= y; ++r) {
        load(b, x0, y, r, false);
        store(slot(r), false);
      }
    }
    __syncthreads();
    if (sg + 1 < s1) {
      int bn, xn, yn;
      decode(sg + 1, bn, xn, yn);
      load(bn, xn, yn, yn + 1, true);
    }
    const int sl[3] = {slot(y - 1), slot(y), slot(y + 1)};
#pragma unroll
    for (int kk = 0; kk < S; ++kk) {
#pragma unroll
      for (int i = 0; i < PER_WAVE; ++i) {
        const int u = wave + 4 * i;
        if (u < NU) {
          const int ti = u / NT, tj = u - ti * NT;
          const bf16x8 av = *(const bf16x8*)&As[ti * 16 + (lane & 15)][kk * 32 + kq];
#pragma unroll
          for (int dy = 0; dy < 3; ++dy) {
            const bf16* xr = &Xs[sl[dy]][tj * 16 + (lane & 15)][kk * 32 + kq + 8];   // dx = 1
            const u32x4 a4 = __builtin_bit_cast(u32x4, *(const bf16x8*)(xr - 8));
            const u32x4 b4 = __builtin_bit_cast(u32x4, *(const bf16x8*)xr);
            const u32x4 c4 = __builtin_bit_cast(u32x4, *(const bf16x8*)(xr + 8));
            const unsigned s0w = (a4[3] >> 16) | (b4[0] << 16), s1w = (b4[0] >> 16) | (b4[1] << 16);
            const unsigned s2w = (b4[1] >> 16) | (b4[2] << 16), s3w = (b4[2] >> 16) | (b4[3] << 16);
            const unsigned s4w = (b4[3] >> 16) | (c4[0] << 16);
            const bf16x8 bl = __builtin_bit_cast(bf16x8, u32x4{s0w, s1w, s2w, s3w});   // dx = 0
            const bf16x8 bm = __builtin_bit_cast(bf16x8, b4);                          // dx = 1
            const bf16x8 br = __builtin_bit_cast(bf16x8, u32x4{s1w, s2w, s3w, s4w});   // dx = 2
            acc[i][3 * dy] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl, acc[i][3 * dy], 0, 0, 0);
            acc[i][3 * dy + 1] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bm, acc[i][3 * dy + 1], 0, 0, 0);
            acc[i][3 * dy + 2] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, br, acc[i][3 * dy + 2], 0, 0, 0);
          }
        }
      }
      if (bias) {
#pragma unroll
        for (int i = 0; i < BT; ++i) {
          const int ti = wave + 4 * i;
          if (ti < MT) {
            const bf16x8 av = *(const bf16x8*)&As[ti * 16 + (lane & 15)][kk * 32 + kq];
            accb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, ones, accb[i], 0, 0, 0);
          }
        }
      }
    }
  }
  if (bias) {
#pragma unroll
    for (int i = 0; i < BT; ++i) {
      const int ti = wave + 4 * i;
      if (ti < MT && (lane & 15) == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) bpart[(size_t)slice * Mr + ti * 16 + 4 * (lane >> 4) + q] = accb[i][q];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < PER_WAVE; ++i) {
    const int u = wave + 4 * i;
    if (u < NU) {
      const int ti = u / NT, tj = u - ti * NT;
      const int c = tj * 16 + (lane & 15);
#pragma unroll
      for (int d = 0; d < 9; ++d) {
        float* out = part + (((size_t)slice * 9 + d) * Mr) * Nc + n0;
#pragma unroll
        for (int q = 0; q < 4; ++q) out[(size_t)(ti * 16 + 4 * (lane >> 4) + q) * Nc + c] = acc[i][d][q];
      }
    }
  }
}

// Weight gradients of the upsampling layers at the source resolution.  The
// layer input u is the source x repeated over 2 x 2 blocks, so for output
// pixel (2i + a, 2j + b) tap t reads x at (i + dy, j + dx) with
// d = (parity + t - 1) >> 1: per parity only two row and two column shifts
// occur, d = parity + s - 1 for s = 0, 1.  The sixteen products
//   G[a][b][sy][sx][r][c] = sum_{i,j} dz[2i + a][2j + b][r] x[i + a + sy - 1][j + b + sx - 1][c]
// give every tap as a sum of four, dW[ty][tx] = sum_{a,b} G[a][b][sy(a, ty)][sx(b, tx)]
// with sy(a, t) = ((a + t - 1) >> 1) - a + 1 (k_up_tapmap): 16 products per
// source pixel instead of the 36 of the upsampled grid.  Work items: (pixel
// slice, channel block of NB = 16 NT input channels, output-row parity a),
// a fastest.  A stage is PX = 32 S source pixels of source row i; the
// workgroup stages in LDS, transposed to [channel][pixel]:
//  * dz of output row 2i + a, columns 2j and 2j + 1 (b = 0, 1) in two halves;
//  * source rows i + a - 1 and i + a (sy = 0, 1), columns j0 - 8 ..
//    j0 + PX + 7, read by the column shifts -1, 0, +1 as in k_conv_wgrad_row.
// Loads, staging blocks and funnel shifts are those of k_conv_wgrad_row.
// Partials: [slice][16][r][c] (index ((a 2 + b) 2 + sy) 2 + sx), bias
// [slice][a][r] (every channel-block-0 item sums its dz row).
template <int MT, int NT, int S>
__global__ __launch_bounds__(256) void k_conv_wgrad_up(const bf16* __restrict__ dz,
                                                       const bf16* __restrict__ x, int B,
                                                       int Hout, int Wout, int Hin, int Win,
                                                       int Nc, int stages_per, int nwork,
                                                       float* __restrict__ part,
                                                       float* __restrict__ bpart) {
  constexpr int Mr = 16 * MT, NB = 16 * NT, PX = 32 * S, LD = PX + 8;
  constexpr int XC = PX + 16, LDX = XC + 8;
  constexpr int AHALF = (PX / 8) * (Mr / 8), ABLK = 2 * AHALF;   // dz: b = 0, then b = 1
  constexpr int XBLK = (PX / 8 + 2) * (NB / 8);                  // per source row
  constexpr int NBLK = ABLK + 2 * XBLK, BPT = (NBLK + 255) / 256;
  constexpr int NU = MT * NT, PER_WAVE = (NU + 3) / 4;
  __shared__ __attribute__((aligned(16))) bf16 As[2][Mr][LD];
  __shared__ __attribute__((aligned(16))) bf16 Xs[2][NB][LDX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int w = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  if (w >= nwork) return;
  const int nblk = Nc / NB;
  const int a = w & 1, n0 = ((w >> 1) % nblk) * NB, slice = w / (2 * nblk);
  const int nch = (Win + PX - 1) / PX, nst = B * Hin * nch;
  const int s0 = slice * stages_per, s1 = min(nst, s0 + stages_per);
  bf16x8 reg[BPT][8];
  auto load = [&](int sg) {
    const int b = sg / (Hin * nch), rem = sg - b * Hin * nch, i = rem / nch;
    const int j0 = (rem - i * nch) * PX;
#pragma unroll
    for (int bi = 0; bi < BPT; ++bi) {
      const int blk = threadIdx.x + 256 * bi;
#pragma unroll
      for (int e = 0; e < 8; ++e) reg[bi][e] = zero8();
      if (blk < ABLK) {
        const int par = blk / AHALF, r = blk - par * AHALF;
        const int pg = r / (Mr / 8), cg = (r % (Mr / 8)) * 8;
        const int Y = 2 * i + a;
        const bf16* src = dz + ((size_t)b * Hout + Y) * Wout * Mr + cg;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int X = 2 * (j0 + 8 * pg + e) + par;
          if (Y < Hout && X < Wout) reg[bi][e] = load8(src + (size_t)X * Mr);
        }
      } else if (blk < NBLK) {
        const int sy = (blk - ABLK) / XBLK, r = blk - ABLK - sy * XBLK;
        const int ys = i + a + sy - 1;
        if (ys >= 0 && ys < Hin) {
          const int m = r / (NB / 8), cg = (r % (NB / 8)) * 8;
          const int c0 = j0 - 8 + 8 * m;
          const bf16* src = x + ((size_t)b * Hin + ys) * Win * Nc + n0 + cg;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (c0 + e >= 0 && c0 + e < Win) reg[bi][e] = load8(src + (size_t)(c0 + e) * Nc);
        }
      }
    }
  };
  f32x4 acc[PER_WAVE][8];   // [unit][(b 2 + sy) 2 + sx]
#pragma unroll
  for (int u = 0; u < PER_WAVE; ++u)
#pragma unroll
    for (int d = 0; d < 8; ++d) acc[u][d] = f32x4{0.f, 0.f, 0.f, 0.f};
  constexpr int BT = (MT + 3) / 4;
  const bool bias = (n0 == 0);
  f32x4 accb[BT];
#pragma unroll
  for (int u = 0; u < BT; ++u) accb[u] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ones;
#pragma unroll
  for (int q = 0; q < 8; ++q) ones[q] = (bf16)1.f;
  const int kq = 8 * (lane >> 4);
  if (s0 < s1) load(s0);
  for (int sg = s0; sg < s1; ++sg) {
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < BPT; ++bi) {
      const int blk = threadIdx.x + 256 * bi;
      bf16* dst = nullptr;
      if (blk < ABLK) {
        const int par = blk / AHALF, r = blk - par * AHALF;
        dst = &As[par][(r % (Mr / 8)) * 8][(r / (Mr / 8)) * 8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          bf16x8 t;
#pragma unroll
          for (int e = 0; e < 8; ++e) t[e] = reg[bi][e][q];
          *(bf16x8*)(dst + q * LD) = t;
        }
      } else if (blk < NBLK) {
        const int sy = (blk - ABLK) / XBLK, r = blk - ABLK - sy * XBLK;
        const int m = r / (NB / 8), cg = (r % (NB / 8)) * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          bf16x8 t;
#pragma unroll
          for (int e = 0; e < 8; ++e) t[e] = reg[bi][e][q];
          *(bf16x8*)&Xs[sy][cg + q][8 * m] = t;
        }
      }
    }
    __syncthreads();
    if (sg + 1 < s1) load(sg + 1);
#pragma unroll
    for (int kk = 0; kk < S; ++kk) {
#pragma unroll
      for (int u = 0; u < PER_WAVE; ++u) {
        const int uu = wave + 4 * u;
        if (uu < NU) {
          const int ti = uu / NT, tj = uu - ti * NT;
          const bf16x8 av0 = *(const bf16x8*)&As[0][ti * 16 + (lane & 15)][kk * 32 + kq];
          const bf16x8 av1 = *(const bf16x8*)&As[1][ti * 16 + (lane & 15)][kk * 32 + kq];
#pragma unroll
          for (int sy = 0; sy < 2; ++sy) {
            const bf16* xr = &Xs[sy][tj * 16 + (lane & 15)][kk * 32 + kq + 8];   // shift 0
            const u32x4 a4 = __builtin_bit_cast(u32x4, *(const bf16x8*)(xr - 8));
            const u32x4 b4 = __builtin_bit_cast(u32x4, *(const bf16x8*)xr);
            const u32x4 c4 = __builtin_bit_cast(u32x4, *(const bf16x8*)(xr + 8));
            const unsigned s0w = (a4[3] >> 16) | (b4[0] << 16), s1w = (b4[0] >> 16) | (b4[1] << 16);
            const unsigned s2w = (b4[1] >> 16) | (b4[2] << 16), s3w = (b4[2] >> 16) | (b4[3] << 16);
            const unsigned s4w = (b4[3] >> 16) | (c4[0] << 16);
            const bf16x8 bl = __builtin_bit_cast(bf16x8, u32x4{s0w, s1w, s2w, s3w});   // -1
            const bf16x8 bm = __builtin_bit_cast(bf16x8, b4);                          // 0
            const bf16x8 br = __builtin_bit_cast(bf16x8, u32x4{s1w, s2w, s3w, s4w});   // +1
            // b = 0: column shifts -1 (sx 0), 0 (sx 1); b = 1: 0 (sx 0), +1 (sx 1)
            acc[u][2 * sy] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av0, bl, acc[u][2 * sy], 0, 0, 0);
            acc[u][2 * sy + 1] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av0, bm, acc[u][2 * sy + 1], 0, 0, 0);
            acc[u][4 + 2 * sy] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av1, bm, acc[u][4 + 2 * sy], 0, 0, 0);
            acc[u][5 + 2 * sy] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av1, br, acc[u][5 + 2 * sy], 0, 0, 0);
          }
        }
      }
      if (bias) {
#pragma unroll
        for (int u = 0; u < BT; ++u) {
          const int ti = wave + 4 * u;
          if (ti < MT) {
#pragma unroll
            for (int par = 0; par < 2; ++par) {
              const bf16x8 av = *(const bf16x8*)&As[par][ti * 16 + (lane & 15)][kk * 32 + kq];
              accb[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, ones, accb[u], 0, 0, 0);
            }
          }
        }
      }
    }
  }
  if (bias) {
#pragma unroll
    for (int u = 0; u < BT; ++u) {
      const int ti = wave + 4 * u;
      if (ti < MT && (lane & 15) == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          bpart[((size_t)slice * 2 + a) * Mr + ti * 16 + 4 * (lane >> 4) + q] = accb[u][q];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PER_WAVE; ++u) {
    const int uu = wave + 4 * u;
    if (uu < NU) {
      const int ti = uu / NT, tj = uu - ti * NT;
      const int c = tj * 16 + (lane & 15);
#pragma unroll
      for (int d = 0; d < 8; ++d) {   // product index (a 2 + b) 2 + sy) 2 + sx = 8 a + d
        float* out = part + (((size_t)slice * 16 + 8 * a + d) * Mr) * Nc + n0;
#pragma unroll
        for (int q = 0; q < 4; ++q) out[(size_t)(ti * 16 + 4 * (lane >> 4) + q) * Nc + c] = acc[u][d][q];
      }
    }
  }
}

// The nine tap gradients of an upsampling layer from the sixteen products
// summed over slices (S [16][Mr][Nc], see k_conv_wgrad_up), in a fixed order.
__global__ void k_up_tapmap(const float* __restrict__ S, int Mr, int Nc, int cout, int cin,
                            float* __restrict__ g) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;   // (co, ci, tap)
  if (id >= cout * cin * 9) return;
  const int tap = id % 9, ci = (id / 9) % cin, co = id / (9 * cin);
  const int ty = tap / 3, tx = tap % 3;
  float v = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int sy = ((a + ty - 1) >> 1) - a + 1, sx = ((b + tx - 1) >> 1) - b + 1;
      v += S[((size_t)(((a * 2 + b) * 2 + sy) * 2 + sx) * Mr + co) * Nc + ci];
    }
  g[id] = v;
}

// Layer-1 weight and bias gradients on FP32 matrix cores: dW[co][j] =
// sum_p dz[p][co] u[p][j], where u[p] is the pixel's 9 C input values
// (plane-major, tap-minor: the [cout][cin][3][3] order of the weights), then 1
// for the bias, then zeros.  Per 4 pixels, 16x16x4 FP32 MFMAs take
// A[r][px] = dz[px][2 r + i] (row r of tile i is channel 2 r + i, so a lane's
// two channels are one 4-byte load) and B[px][jj] = u[px][16 jt + jj].  A
// workgroup owns the contiguous pixel range [p0, p0 + pix_per); per
// iteration it takes 16 pixels, pixel p0 + 16 it + 4 w + px for wave w, and
// C1W_U iterations' loads are issued before their MFMAs.  The four waves are
// summed in LDS; partials [slice][32][32] (column 9 C = bias).
#define C1W_U 4
template <int C>
__global__ __launch_bounds__(256) void k_conv1_wgrad(const float* __restrict__ x0,
                                                     const bf16* __restrict__ dz, int B, int H,
                                                     int W, int pix_per,
                                                     float* __restrict__ part) {
  constexpr int J = 9 * C, NJT = (J + 16) / 16;   // column tiles holding J + 1 columns
  __shared__ float red[4][32 * 32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, col = lane & 15;
  const int HW = H * W, total = B * HW;
  const int p0 = blockIdx.x * pix_per, p1 = min(total, p0 + pix_per);
  int koff[NJT], kdy[NJT], kdx[NJT];
  bool kone[NJT];
#pragma unroll
  for (int jt = 0; jt < NJT; ++jt) {
    const int j = 16 * jt + col, c = j / 9, t = j - 9 * c;
    kone[jt] = (j == J);
    kdy[jt] = (j < J) ? t / 3 - 1 : -H;   // bias and padding columns read no input
    kdx[jt] = t % 3 - 1;
    koff[jt] = c * HW + kdy[jt] * W + kdx[jt];
  }
  // (b, y, x) of this lane's pixel, advanced by 16 pixels per iteration
  int p = p0 + 4 * wave + g;
  int b = (unsigned)p / (unsigned)HW, x = p - b * HW;
  int y = (unsigned)x / (unsigned)W;
  x -= y * W;
  f32x4 acc[2][NJT];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jt = 0; jt < NJT; ++jt) acc[i][jt] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int it0 = 0; p0 + 16 * it0 < p1; it0 += C1W_U) {
    uint32_t dv[C1W_U];
    float uv[C1W_U][NJT];
#pragma unroll
    for (int u = 0; u < C1W_U; ++u) {
      const bool pv = p < p1;
      // out-of-range reads go to element 0 / pixel p0 and are zeroed after
      const uint32_t d = *(const uint32_t*)(dz + (size_t)(pv ? p : p0) * 32 + 2 * col);
      dv[u] = pv ? d : 0u;
      const int pb = p + b * (C - 1) * HW;   // element (b, 0, y, x) of the planar input
#pragma unroll
      for (int jt = 0; jt < NJT; ++jt) {
        const bool ok = pv & ((unsigned)(y + kdy[jt]) < (unsigned)H) &
                        ((unsigned)(x + kdx[jt]) < (unsigned)W);
        const float v = x0[ok ? (unsigned)(pb + koff[jt]) : 0u];
        uv[u][jt] = ok ? v : ((pv & kone[jt]) ? 1.f : 0.f);
      }
      p += 16;
      x += 16;
      while (x >= W) {
        x -= W;
        if (++y == H) { y = 0; ++b; }
      }
    }
#pragma unroll
    for (int u = 0; u < C1W_U; ++u) {
      const float a0 = __uint_as_float(dv[u] << 16), a1 = __uint_as_float(dv[u] & 0xffff0000u);
#pragma unroll
      for (int jt = 0; jt < NJT; ++jt) {
        acc[0][jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, uv[u][jt], acc[0][jt], 0, 0, 0);
        acc[1][jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, uv[u][jt], acc[1][jt], 0, 0, 0);
      }
    }
  }
  // lane holds rows 4 g + q (channel 2 (4 g + q) + i) of column 16 jt + col
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float* r = &red[wave][(2 * (4 * g + q) + i) * 32 + col];
#pragma unroll
      for (int jt = 0; jt < NJT; ++jt) r[16 * jt] = acc[i][jt][q];
      if (NJT == 1) r[16] = 0.f;
    }
  __syncthreads();
  float* out = part + (size_t)blockIdx.x * 32 * 32;
  for (int e = threadIdx.x; e < 32 * 32; e += 256)
    out[e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// Sum over slices of [slice][nent] partials for 16 consecutive entries per
// workgroup: 16 slice groups (slices g, g + 16, ...) added in group order.
__device__ __forceinline__ float slice_sum16(const float* __restrict__ part, int nslices, int nent,
                                             int ent, float (*red)[16]) {
  const int j = threadIdx.x & 15, grp = threadIdx.x >> 4;
  float s = 0.f;
  if (ent < nent) {
    // slices grp, grp + 16, ... added in order; eight loads in flight at a time
    int sl = grp;
    for (; sl + 112 < nslices; sl += 128) {
      float a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = part[(size_t)(sl + 16 * q) * nent + ent];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += a[q];
    }
    for (; sl < nslices; sl += 16) s += part[(size_t)sl * nent + ent];
  }
  red[grp][j] = s;
  __syncthreads();
  float t = 0.f;
  if (grp == 0)
    for (int g = 0; g < 16; ++g) t += red[g][j];
  return t;
}

// Sum the [slice][32][32] partials of k_conv1_wgrad (16 entries per block).
__global__ __launch_bounds__(256) void k_conv1_rows_reduce(const float* __restrict__ part,
                                                           int nslices, int cout, int C,
                                                           float* __restrict__ gw,
                                                           float* __restrict__ gb) {
  __shared__ float red[16][16];
  const int J = 9 * C;
  const int ent = blockIdx.x * 16 + (threadIdx.x & 15);
  const float s = slice_sum16(part, nslices, 32 * 32, ent, red);
  const int co = ent / 32, j = ent % 32;
  if ((threadIdx.x >> 4) == 0 && co < cout && j <= J) {
    if (j < J) gw[(size_t)co * J + j] = s;
    else gb[co] = s;
  }
}

// Sum the slices (fixed order) into the FP32 gradient in [cout][cin][3][3]
// order.  A workgroup takes 64 consecutive partial entries ([tap][r][c]
// order, coalesced reads) and four slice groups (slices g, g + 4, ...), which
// are then added in group order.
// NE = 9: the tap gradients, written to g ([cout][cin][9]); NE = 16: the
// products of an upsampling layer, written to S ([16][Mr][Nc]) for k_up_tapmap.
template <int NE>
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int nslices,
                                                      int Mr, int Nc, int cout, int cin,
                                                      float* __restrict__ g) {
  __shared__ float red[4][64];
  const int j = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int ent = blockIdx.x * 64 + j, nent = NE * Mr * Nc;
  float s = 0.f;
  if (ent < nent) {
    // slices grp, grp + 4, ... added in order; eight loads in flight at a time
    int sl = grp;
    for (; sl + 28 < nslices; sl += 32) {
      float a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = part[(size_t)(sl + 4 * q) * nent + ent];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += a[q];
    }
    for (; sl < nslices; sl += 4) s += part[(size_t)sl * nent + ent];
  }
  red[grp][j] = s;
  __syncthreads();
  if (grp == 0 && ent < nent) {
    const float v = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
    if (NE == 16) {
      g[ent] = v;
    } else {
      const int tap = ent / (Mr * Nc), rem = ent - tap * Mr * Nc, co = rem / Nc, ci = rem - co * Nc;
      if (co < cout && ci < cin) g[((size_t)co * cin + ci) * 9 + tap] = v;
    }
  }
}
__global__ __launch_bounds__(256) void k_bgrad_reduce(const float* __restrict__ part, int nslices,
                                                      int Mr, int cout, float* __restrict__ g) {
  __shared__ float red[16][16];
  const int r = blockIdx.x * 16 + (threadIdx.x & 15);
  const float s = slice_sum16(part, nslices, Mr, r, red);
  if ((threadIdx.x >> 4) == 0 && r < cout) g[r] = s;
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

// iscale[b] = sqrt(D / sum |F_b|^2) (0 for an all-zero field), in two steps:
// ES_SLICES partial sums per problem (grid (ES_SLICES, B)), then their sum in
// slice order.
#define ES_SLICES 64
__global__ __launch_bounds__(256) void k_eim_scale_part(const float2* __restrict__ eim, int D,
                                                        double* __restrict__ part) {
  const float2* f = eim + (size_t)blockIdx.y * D;
  const int per = (D + ES_SLICES - 1) / ES_SLICES, e0 = blockIdx.x * per, e1 = min(D, e0 + per);
  double s = 0.0;
  for (int e = e0 + threadIdx.x; e < e1; e += 256) {
    const float2 v = f[e];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  __shared__ double lds[8];
  s = block_sum1<double>(s, lds);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * ES_SLICES + blockIdx.x] = s;
}
__global__ void k_eim_scale(const double* __restrict__ part, int B, int D,
                            double* __restrict__ iscale) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int i = 0; i < ES_SLICES; ++i) s += part[(size_t)b * ES_SLICES + i];
  iscale[b] = (s > 0.0) ? sqrt((double)D / s) : 0.0;
}

// loss partials and dz of the last (linear) layer: out and target are complex
// fields [B][k][D]; dz = 2 (out - t) / count in bf16 with coutp channels.
// One thread per (pixel, group of 8 channels) (coutp is a multiple of 32), so
// that a pixel's dz row is written by consecutive threads 16 B at a time.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out,
                                             const float2* __restrict__ target, int B, int D,
                                             int k, int coutp, float scale,
                                             bf16* __restrict__ dz, float* __restrict__ lpart) {
  const int CG = coutp / 8;
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  float s = 0.f;
  if (t < (long)B * D * CG) {
    const int p = (int)(t / CG), c0 = (int)(t - (long)p * CG) * 8;
    const int b = p / D, e = p - b * D;
    const float2* o = (const float2*)out + (size_t)b * k * D + e;   // field j at o[j D]
    bf16x8 h;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = c0 / 2 + q;
      float gx = 0.f, gy = 0.f;
      if (j < k) {
        const float2 v = o[(size_t)j * D], tv = target[((size_t)b * k + j) * D + e];
        const float dx = v.x - tv.x, dy = v.y - tv.y;
        s += dx * dx + dy * dy;
        gx = scale * dx; gy = scale * dy;
      }
      h[2 * q] = (bf16)gx;
      h[2 * q + 1] = (bf16)gy;
    }
    *(u32x4*)(dz + (size_t)p * coutp + c0) = __builtin_bit_cast(u32x4, h);
  }
  __shared__ float lds[8];
  s = block_sum1<float>(s, lds);
  if (threadIdx.x == 0) lpart[blockIdx.x] = s;
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

// Effective backward-data weights of an upsampled layer (k_conv_tile_s2):
// wu[e][ci][co] = sum of w[co][ci][dy][dx] over the taps whose dz offset is
// (oy, ox) = (e / 4 - 1, e % 4 - 1), i.e. sy = oy + dy - 1 and sx = ox + dx - 1
// in {0, 1}; FP32 sums rounded once to bf16.
__global__ void k_pack_up_weights(const float* __restrict__ w, int cout, int cin, int coutp,
                                  int cinp, bf16* __restrict__ wu) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= 16 * cinp * coutp) return;
  const int e = idx / (cinp * coutp), rem = idx % (cinp * coutp);
  const int ci = rem / coutp, co = rem % coutp;
  const int oy = e / 4 - 1, ox = e % 4 - 1;
  float v = 0.f;
  if (co < cout && ci < cin)
    for (int dy = 0; dy < 3; ++dy) {
      const int sy = oy + dy - 1;
      if (sy < 0 || sy > 1) continue;
      for (int dx = 0; dx < 3; ++dx) {
        const int sx = ox + dx - 1;
        if (sx < 0 || sx > 1) continue;
        v += w[((size_t)co * cin + ci) * 9 + dy * 3 + dx];
      }
    }
  wu[idx] = (bf16)v;
}

// bias for layers whose coutp > cout: a zero-padded FP32 copy
__global__ void k_pad_bias(const float* __restrict__ b, int cout, int coutp, float* __restrict__ bp) {
  const int i = threadIdx.x;
  if (i < coutp) bp[i] = (i < cout) ? b[i] : 0.f;
}

// ============================================================ host side ====
// MFMA kernels take 32, 64 or 128 channels (the K loop steps 32 channels)
static int rup32(int c) { return (c + 31) / 32 * 32; }

// pixels per weight-gradient slice: about 256 slices, multiples of 32

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
    if (L.up)
      k_pack_up_weights<<<(16 * L.cinp * L.coutp + 255) / 256, 256, 0, st>>>(
          n->params + L.woff, L.cout, L.cin, L.coutp, L.cinp, n->wu[l]);
    k_pad_bias<<<1, 256, 0, st>>>(n->params + L.boff, L.cout, L.coutp, n->biaspad + 256 * l);
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
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        ncu > 0)
      n->ncu = ncu;
  }
  const int spec[NL][5] = {{in_channels, 32, 1, 0, 1}, {32, 64, 2, 0, 1}, {64, 128, 2, 0, 1},
                           {128, 128, 1, 0, 1}, {128, 64, 1, 1, 1}, {64, 32, 1, 1, 1},
                           {32, 32, 1, 0, 1}, {32, 2 * k, 1, 0, 0}};
  int H = ny, W = nx;
  size_t off = 0;
  for (int l = 0; l < NL; ++l) {
    CnnLayer& L = n->L[l];
    L.cin = spec[l][0]; L.cout = spec[l][1]; L.stride = spec[l][2]; L.up = spec[l][3];
    L.relu = spec[l][4];
    L.cinp = (l == 0) ? L.cin : rup32(L.cin);
    L.coutp = rup32(L.cout);
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
  chk(cnn_alloc(n, &n->espart, (size_t)max_batch * ES_SLICES));
  size_t wp = 0;
  for (int l = 0; l < NL && e == hipSuccess; ++l) {
    const CnnLayer& L = n->L[l];
    const size_t pix = (size_t)max_batch * L.Hout * L.Wout;
    if (l > 0) {
      chk(cnn_alloc(n, &n->wf[l], (size_t)9 * L.coutp * L.cinp));
      chk(cnn_alloc(n, &n->wb[l], (size_t)9 * L.coutp * L.cinp));
      if (L.up) chk(cnn_alloc(n, &n->wu[l], (size_t)16 * L.coutp * L.cinp));
    }
    if (l < NL - 1) chk(cnn_alloc(n, &n->act[l], pix * L.coutp));
    chk(cnn_alloc(n, &n->dz[l], pix * L.coutp));
    // gradient partials: room for 8 workgroups per CU (256 threads each)
    // over 3 dy and the 64-channel blocks (k_conv_wgrad_row takes fewer
    // slices when its occupancy asks for more than fit); layer 1 uses
    // [slice][32][32] (at most 8 slices per CU)
    if (l > 0) {
      const size_t nblk = (size_t)std::max(1, L.cinp / 64);
      const size_t sl = std::max<size_t>(1, (size_t)8 * n->ncu / (3 * nblk));
      const size_t wl = (size_t)L.coutp * L.cinp;
      wp = std::max(wp, sl * (9 * wl + L.coutp));
      // upsampling (k_conv_wgrad_up, up to 4 workgroups per CU over the two
      // parities): 16 products and two bias rows per slice, then their sums
      if (L.up) wp = std::max(wp, (size_t)2 * n->ncu / nblk * (16 * wl + 2 * L.coutp) + 16 * wl);
    } else {
      wp = std::max(wp, (size_t)8 * n->ncu * 32 * 32);
    }
  }
  n->wpart_elems = wp;
  chk(cnn_alloc(n, &n->wpart, wp));
  chk(cnn_alloc(n, &n->out, (size_t)max_batch * D * 2 * k));
  chk(cnn_alloc(n, &n->lpart, (size_t)max_batch * D * 8 / 256 + 256));   // k_mse: coutp / 8 <= 8
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

static dd_status gemm_dispatch(const GemmArgs& a, bool bwd, hipStream_t st) {
  const int MT = a.M / 16;
  if ((MT != 2 && MT != 4 && MT != 8) || a.M % 16 || a.Ksrc % 32) {
    dd_set_error("dd_cnn: no convolution kernel for %d result / %d source channels", a.M, a.Ksrc);
    return DD_EINVAL;
  }
  // several 32-channel chunks: weights staged in LDS (fewer resident
  // workgroups, no global loads in the tap loop); one chunk: weights from L2
  const bool wl = a.Ksrc > 32;
  if (!bwd && (a.mode == MAP_S1 || a.mode == MAP_UP)) {
    const dim3 grid((a.Wq + CT_TW - 1) / CT_TW, (a.Hq + CT_TH - 1) / CT_TH, a.B);
    switch (MT) {
      case 2:
        if (wl) k_conv_tile<2, false, true><<<grid, 256, 0, st>>>(a);
        else k_conv_tile<2><<<grid, 256, 0, st>>>(a);
        break;
      case 4:
        if (wl) k_conv_tile<4, false, true><<<grid, 256, 0, st>>>(a);
        else k_conv_tile<4><<<grid, 256, 0, st>>>(a);
        break;
      case 8:
        if (wl) k_conv_tile<8, false, true><<<grid, 256, 0, st>>>(a);
        else k_conv_tile<8><<<grid, 256, 0, st>>>(a);
        break;
    }
    return DD_OK;
  }
  if (bwd && a.mode == MAP_S1) {
    const dim3 grid((a.Wq + CT_TW - 1) / CT_TW, (a.Hq + CT_TH - 1) / CT_TH, a.B);
    switch (MT) {
      case 2:
        if (wl) k_conv_tile<2, true, true><<<grid, 256, 0, st>>>(a);
        else k_conv_tile<2, true><<<grid, 256, 0, st>>>(a);
        break;
      case 4:
        if (wl) k_conv_tile<4, true, true><<<grid, 256, 0, st>>>(a);
        else k_conv_tile<4, true><<<grid, 256, 0, st>>>(a);
        break;
      case 8:
        if (wl) k_conv_tile<8, true, true><<<grid, 256, 0, st>>>(a);
        else k_conv_tile<8, true><<<grid, 256, 0, st>>>(a);
        break;
    }
    return DD_OK;
  }
  if ((!bwd && a.mode == MAP_S2 && !a.outf) || (bwd && a.mode == MAP_UP)) {
    const dim3 grid((a.Wq + CS_TW - 1) / CS_TW, (a.Hq + CS_TH - 1) / CS_TH, a.B);
    if (!bwd) {
      switch (MT) {
        case 2: k_conv_tile_s2<2, 3, false><<<grid, 256, 0, st>>>(a); break;
        case 4: k_conv_tile_s2<4, 3, false><<<grid, 256, 0, st>>>(a); break;
        case 8:
          if (a.Ksrc > 32) k_conv_tile_s2<8, 3, false, true><<<grid, 256, 0, st>>>(a);
          else k_conv_tile_s2<8, 3, false><<<grid, 256, 0, st>>>(a);
          break;
      }
    } else {
      switch (MT) {
        case 2: k_conv_tile_s2<2, 4, true><<<grid, 256, 0, st>>>(a); break;
        case 4: k_conv_tile_s2<4, 4, true><<<grid, 256, 0, st>>>(a); break;
        case 8:
          if (a.Ksrc > 32) k_conv_tile_s2<8, 4, true, true><<<grid, 256, 0, st>>>(a);
          else k_conv_tile_s2<8, 4, true><<<grid, 256, 0, st>>>(a);
          break;
      }
    }
    return DD_OK;
  }
  if (bwd && a.mode == MAP_S2) {
    const dim3 grid((a.Wq + BS_TW - 1) / BS_TW, (a.Hq + BS_TH - 1) / BS_TH, a.B);
    // the stride-2 layers have 32- and 64-channel inputs
    switch (MT) {
      case 2: k_bwd_s2_tile<2><<<grid, 256, 0, st>>>(a); return DD_OK;
      case 4: k_bwd_s2_tile<4><<<grid, 256, 0, st>>>(a); return DD_OK;
    }
    dd_set_error("dd_cnn: no stride-2 backward-data kernel for %d channels", a.M);
    return DD_EINVAL;
  }
  dd_set_error("dd_cnn: no convolution kernel for this layer map");
  return DD_EINVAL;
}

// fields: destination of the complex output fields [B][k][D] (n->out if NULL)
static dd_status forward(dd_cnn* n, const float* eps, const void* eim, int B, hipStream_t st,
                         void* fields = nullptr) {
  const int D = n->nx * n->ny;
  if (n->cin0 == 3) {
    k_eim_scale_part<<<dim3(ES_SLICES, B), 256, 0, st>>>((const float2*)eim, D, n->espart);
    k_eim_scale<<<(B + 255) / 256, 256, 0, st>>>(n->espart, B, D, n->iscale);
  }
  k_inputs<<<(B * D + 255) / 256, 256, 0, st>>>(eps, (const float2*)eim, n->iscale, B, D, n->cin0,
                                                 n->x0);
  {
    const CnnLayer& L = n->L[0];
    const dim3 grid((B * D + 64 * C1_NT - 1) / (64 * C1_NT));
    if (n->cin0 == 3)
      k_conv1_fwd<3><<<grid, 256, 0, st>>>(n->x0, n->params + L.woff, n->params + L.boff, B,
                                           n->ny, n->nx, n->act[0]);
    else
      k_conv1_fwd<1><<<grid, 256, 0, st>>>(n->x0, n->params + L.woff, n->params + L.boff, B,
                                           n->ny, n->nx, n->act[0]);
  }
  for (int l = 1; l < NL; ++l) {
    const CnnLayer& L = n->L[l];
    GemmArgs a{};
    a.src = n->act[l - 1];
    a.W = n->wf[l];
    a.bias = n->biaspad + 256 * l;
    a.B = B; a.Hq = L.Hout; a.Wq = L.Wout;
    a.Hs = L.Hin; a.Ws = L.Win;
    a.Ksrc = L.cinp; a.M = L.coutp; a.mode = L.mode; a.relu = L.relu;
    if (l == NL - 1) {
      a.outf = fields ? (float*)fields : n->out;
      a.nreal = L.cout;
      n->last_fields = a.outf;
    }
    else a.out = n->act[l];
    const dd_status rc = gemm_dispatch(a, false, st);
    if (rc != DD_OK) return rc;
  }
  DD_HIP_CHECK(hipGetLastError());
  return DD_OK;
}

// Work split of the weight-gradient kernel k_conv_wgrad_row
// over nst stages: one round of resident workgroups (cap per CU), within the
// partial buffer (weights, then bias).
struct WgradSplit {
  int slices, stages_per, nwork, grid;
};
// dsplit: work items per (slice, channel block), 3 (one per dy), 2 (one per
// output-row parity, upsampling) or 1.  ne: weight partials per slice (9
// taps, or the 16 products of an upsampling layer, which also keep their
// 16 Mr Nc sums after the partials); nbias: bias partials per slice.
static WgradSplit wgrad_split(const dd_cnn* n, int cap, int Mr, int Nc, int NB, int nst,
                              int dsplit = 3, int ne = 9, int nbias = 1) {
  const int nblk = Nc / NB;
  const size_t per = (size_t)ne * Mr * Nc + (size_t)nbias * Mr;
  const size_t reserve = ne == 9 ? 0 : (size_t)ne * Mr * Nc;
  int slices = std::max(1, cap * n->ncu / (dsplit * nblk));
  slices = (int)std::min<size_t>((size_t)slices, (n->wpart_elems - reserve) / per);
  slices = std::max(1, std::min(slices, nst));
  const int sp = (nst + slices - 1) / slices;
  slices = (nst + sp - 1) / sp;
  const int nwork = slices * dsplit * nblk;
  return {slices, sp, nwork, (nwork + 7) / 8 * 8};
}

// resident workgroups per CU of a kernel (at least 1)
template <typename K>
static int occupancy(K kern) {
  int c = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, kern, 256, 0) != hipSuccess || c < 1) c = 1;
  return c;
}

template <int MT, int NT, int S, int MK, int ND = 1>
static int launch_wgrad_row(dd_cnn* n, int l, int B, hipStream_t st) {
  static const int cap = occupancy(k_conv_wgrad_row<MT, NT, S, MK, ND>);
  const CnnLayer& L = n->L[l];
  const int Mr = 16 * MT, Nc = L.cinp;
  const int nst = B * L.Hout * ((L.Wout + 32 * S - 1) / (32 * S));
  const WgradSplit w = wgrad_split(n, cap, Mr, Nc, 16 * NT, nst, ND == 3 ? 1 : 3);
  k_conv_wgrad_row<MT, NT, S, MK, ND><<<w.grid, 256, 0, st>>>(
      n->dz[l], n->act[l - 1], B, L.Hout, L.Wout, L.Hin, L.Win, Nc, w.stages_per, w.nwork,
      n->wpart, n->wpart + (size_t)w.slices * 9 * Mr * Nc);
  return w.slices;
}

template <int MT, int NT, int S>
static int launch_wgrad_ring(dd_cnn* n, int l, int B, hipStream_t st) {
  static const int cap = occupancy(k_conv_wgrad_ring<MT, NT, S>);
  const CnnLayer& L = n->L[l];
  const int Mr = 16 * MT, Nc = L.cinp;
  const int nst = B * L.Hout * ((L.Wout + 32 * S - 1) / (32 * S));
  const WgradSplit w = wgrad_split(n, cap, Mr, Nc, 16 * NT, nst, 1);
  k_conv_wgrad_ring<MT, NT, S><<<w.grid, 256, 0, st>>>(
      n->dz[l], n->act[l - 1], B, L.Hout, L.Wout, Nc, w.stages_per, w.nwork, n->wpart,
      n->wpart + (size_t)w.slices * 9 * Mr * Nc);
  return w.slices;
}

// whether an upsampling layer's weight gradient runs on k_conv_wgrad_up
static bool wgrad_up_kernel(const CnnLayer& L) {
  return (L.coutp == 64 && L.cinp % 32 == 0) || (L.coutp == 32 && L.cinp % 64 == 0);
}

template <int MT, int NT, int S>
static int launch_wgrad_up(dd_cnn* n, int l, int B, hipStream_t st) {
  static const int cap = occupancy(k_conv_wgrad_up<MT, NT, S>);
  const CnnLayer& L = n->L[l];
  const int Mr = 16 * MT, Nc = L.cinp;
  const int nst = B * L.Hin * ((L.Win + 32 * S - 1) / (32 * S));
  const WgradSplit w = wgrad_split(n, cap, Mr, Nc, 16 * NT, nst, 2, 16, 2);
  k_conv_wgrad_up<MT, NT, S><<<w.grid, 256, 0, st>>>(
      n->dz[l], n->act[l - 1], B, L.Hout, L.Wout, L.Hin, L.Win, Nc, w.stages_per, w.nwork,
      n->wpart, n->wpart + (size_t)w.slices * 16 * Mr * Nc);
  return w.slices;
}

// Weight- and bias-gradient partials of layer l >= 1 (row chunks, every
// map).  Returns the number of pixel slices written to n->wpart (weights
// [slice][9][coutp][cinp], then bias [slice][coutp]), 0 (nothing launched)
// for channel counts without an instance.
static int wgrad_partials(dd_cnn* n, int l, int B, hipStream_t st) {
  const CnnLayer& L = n->L[l];
  const int Mr = L.coutp, Nc = L.cinp, NB = std::min(Nc, 64);
  if (Nc % NB) return 0;
  // S (stage width 32 S pixels, 1, 2 or 4): the largest whose 8 x 8 staging
  // blocks (dz, then the input pixels of one dy row) fit one per thread.
  // The kernels with 32 output channels take all three dy per work item
  // (ND = 3: dz staged once for the three input rows).
  auto blocks = [&](int S) {
    const int xg = (L.mode == MAP_S1) ? 4 * S + 2 : (L.mode == MAP_UP) ? 2 * S + 1 : 8 * S;
    return 4 * S * (Mr / 8) + xg * (NB / 8);
  };
  const int S = blocks(4) <= 256 ? 4 : (blocks(2) <= 256 ? 2 : 1);
#define WG_CASES(F, F3)                                                    \
  if (Mr == 32 && NB == 32) return S == 4 ? F3(2, 2, 4) : 0;           \
  if (Mr == 32 && NB == 64) return S == 4 ? F3(2, 4, 4) : F(2, 4, 2);  \
  if (Mr == 64 && NB == 32) return S == 4 ? F(4, 2, 4) : F(4, 2, 2);   \
  if (Mr == 64 && NB == 64) return S == 4 ? F(4, 4, 4) : F(4, 4, 2);   \
  if (Mr == 128 && NB == 32) return S == 2 ? F(8, 2, 2) : 0;           \
  if (Mr == 128 && NB == 64) return S == 2 ? F(8, 4, 2) : F(8, 4, 1);
#define WG_ROW1(a, b, c) launch_wgrad_row<a, b, c, MAP_S1>(n, l, B, st)
#define WG_ROWU(a, b, c) launch_wgrad_row<a, b, c, MAP_UP>(n, l, B, st)
#define WG_ROW2(a, b, c) launch_wgrad_row<a, b, c, MAP_S2>(n, l, B, st)
#define WG_ROW13(a, b, c) launch_wgrad_row<a, b, c, MAP_S1, 3>(n, l, B, st)
#define WG_ROWU3(a, b, c) launch_wgrad_row<a, b, c, MAP_UP, 3>(n, l, B, st)
#define WG_ROW23(a, b, c) launch_wgrad_row<a, b, c, MAP_S2, 3>(n, l, B, st)
  if (L.mode == MAP_S1) {
    // 32 output and 32 input channels (layers 7, 8): input rows in a ring
    if (Mr == 32 && NB == 32) return launch_wgrad_ring<2, 2, 4>(n, l, B, st);
    WG_CASES(WG_ROW1, WG_ROW13)
  }
  else if (L.mode == MAP_UP) {
    // the two upsampling layers (128 -> 64 and 64 -> 32 channels) at the
    // source resolution, sixteen products per pixel
    if (wgrad_up_kernel(L)) {
      return Mr == 64 ? launch_wgrad_up<4, 2, 2>(n, l, B, st) : launch_wgrad_up<2, 4, 2>(n, l, B, st);
    }
    WG_CASES(WG_ROWU, WG_ROWU3)
  }
  else {
    // 64 output and 32 input channels: three dy per item at half the stage
    // width (the 18 accumulators per unit fit; 130 -> 101 us at batch 32)
    if (Mr == 64 && NB == 32) return WG_ROW23(4, 2, 2);
    WG_CASES(WG_ROW2, WG_ROW23)
  }
#undef WG_CASES
#undef WG_ROW1
#undef WG_ROWU
#undef WG_ROW2
#undef WG_ROW13
#undef WG_ROWU3
#undef WG_ROW23
  return 0;
}

// Backward pass from the gradient of the last layer's pre-activation in
// dz[NL-1]; parameter gradients land in n->grads.
static dd_status backward_from_dz(dd_cnn* n, int B, hipStream_t st) {
  for (int l = NL - 1; l >= 1; --l) {
    const CnnLayer& L = n->L[l];
    // weight and bias gradients of layer l
    const int wslices = wgrad_partials(n, l, B, st);
    if (wslices <= 0) {
      dd_set_error("dd_cnn: no weight-gradient kernel for %d x %d channels", L.coutp, L.cinp);
      return DD_EINVAL;
    }
    if (L.mode == MAP_UP && wgrad_up_kernel(L)) {
      // sixteen products per slice, then bias [slice][parity][r]; their sums
      // over slices after both, then mapped onto the nine taps
      const int nent = 16 * L.coutp * L.cinp;
      float* S = n->wpart + (size_t)wslices * (nent + 2 * L.coutp);
      k_wgrad_reduce<16><<<(nent + 63) / 64, 256, 0, st>>>(n->wpart, wslices, L.coutp, L.cinp,
                                                           L.cout, L.cin, S);
      const int nmap = 9 * L.cout * L.cin;
      k_up_tapmap<<<(nmap + 255) / 256, 256, 0, st>>>(S, L.coutp, L.cinp, L.cout, L.cin,
                                                      n->grads + L.woff);
      k_bgrad_reduce<<<(L.coutp + 15) / 16, 256, 0, st>>>(n->wpart + (size_t)wslices * nent,
                                                           2 * wslices, L.coutp, L.cout,
                                                           n->grads + L.boff);
    } else {
      const int nent = 9 * L.coutp * L.cinp;
      k_wgrad_reduce<9><<<(nent + 63) / 64, 256, 0, st>>>(n->wpart, wslices, L.coutp, L.cinp,
                                                          L.cout, L.cin, n->grads + L.woff);
      k_bgrad_reduce<<<(L.coutp + 15) / 16, 256, 0, st>>>(n->wpart + (size_t)wslices * nent,
                                                           wslices, L.coutp, L.cout,
                                                           n->grads + L.boff);
    }
    // data gradient into the previous layer (masked by its ReLU)
    GemmArgs a{};
    a.src = n->dz[l];
    a.W = L.up ? n->wu[l] : n->wb[l];
    a.mask = n->act[l - 1];
    a.out = n->dz[l - 1];
    a.B = B; a.Hq = L.Hin; a.Wq = L.Win;
    a.Hs = L.Hout; a.Ws = L.Wout;
    a.Ksrc = L.coutp; a.M = L.cinp; a.mode = L.mode;
    const dd_status rc = gemm_dispatch(a, true, st);
    if (rc != DD_OK) return rc;
  }
  {
    const CnnLayer& L = n->L[0];
    // about four workgroups per CU (fewer partials to sum), within the
    // partial buffer; each takes a multiple of 16 C1W_U pixels
    const int total = B * n->nx * n->ny;
    const int want = (int)std::min<size_t>((size_t)4 * n->ncu, n->wpart_elems / (32 * 32));
    const int step = 16 * C1W_U;
    const int pp = (total + want - 1) / want, pix_per = (pp + step - 1) / step * step;
    const int slices = (total + pix_per - 1) / pix_per;
    if (n->cin0 == 3)
      k_conv1_wgrad<3><<<slices, 256, 0, st>>>(n->x0, n->dz[0], B, n->ny, n->nx, pix_per,
                                               n->wpart);
    else
      k_conv1_wgrad<1><<<slices, 256, 0, st>>>(n->x0, n->dz[0], B, n->ny, n->nx, pix_per,
                                               n->wpart);
    k_conv1_rows_reduce<<<64, 256, 0, st>>>(n->wpart, slices, L.cout, n->cin0,
                                            n->grads + L.woff, n->grads + L.boff);
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
  const int nlb = (int)(((long)B * D * (LL.coutp / 8) + 255) / 256);
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
  rc = forward(n, eps, eim, B, st, U);
  if (rc != DD_OK) return rc;
  DD_HIP_CHECK(hipGetLastError());
  DD_HIP_CHECK(hipStreamSynchronize(st));
  return DD_OK;
}

extern "C" dd_status dd_cnn_predict(dd_cnn* n, const float* eps, int B, void* U,
                                    hipStream_t st) {
  return predict(n, eps, nullptr, B, U, st, "dd_cnn_predict");
}

extern "C" dd_status dd_cnn_predict_eim(dd_cnn* n, const float* eps, const void* eim, int B,
                                        void* U, hipStream_t st) {
  if (!eim) { dd_set_error("dd_cnn_predict_eim: eim is NULL"); return DD_EINVAL; }
  return predict(n, eps, eim, B, U, st, "dd_cnn_predict_eim");
}

extern "C" dd_status dd_cnn_dims(const dd_cnn* n, int* nx, int* ny, int* k, int* in_channels,
                                 int* max_batch) {
  if (!n) { dd_set_error("dd_cnn_dims: NULL network"); return DD_EINVAL; }
  if (nx) *nx = n->nx;
  if (ny) *ny = n->ny;
  if (k) *k = n->k;
  if (in_channels) *in_channels = n->cin0;
  if (max_batch) *max_batch = n->maxB;
  return DD_OK;
}

extern "C" dd_status dd_cnn_save(const dd_cnn* n, const char* path) {
  if (!n || !path) { dd_set_error("dd_cnn_save: NULL argument"); return DD_EINVAL; }
  const size_t np = n->nparams;
  std::vector<float> buf(3 * np);
  DD_HIP_CHECK(hipDeviceSynchronize());
  DD_HIP_CHECK(hipMemcpy(buf.data(), n->params, sizeof(float) * np, hipMemcpyDeviceToHost));
  DD_HIP_CHECK(hipMemcpy(buf.data() + np, n->am, sizeof(float) * np, hipMemcpyDeviceToHost));
  DD_HIP_CHECK(hipMemcpy(buf.data() + 2 * np, n->av, sizeof(float) * np, hipMemcpyDeviceToHost));
  PredFileHeader h{};
  std::memcpy(h.magic, DD_PRED_MAGIC, 8);
  h.kind = DD_PRED_CNN;
  h.nx = n->nx; h.ny = n->ny; h.k = n->k; h.in_channels = n->cin0;
  h.count = (int64_t)np;
  h.adam_t = n->adam_t;
  FILE* f = std::fopen(path, "wb");
  if (!f) { dd_set_error("dd_cnn_save: cannot open '%s' for writing", path); return DD_EINVAL; }
  const bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
                  std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  if (std::fclose(f) != 0 || !ok) {
    dd_set_error("dd_cnn_save: writing '%s' failed", path);
    return DD_EINVAL;
  }
  return DD_OK;
}

extern "C" dd_status dd_cnn_load(const char* path, int max_batch, dd_cnn** out) {
  if (!out) { dd_set_error("dd_cnn_load: out is NULL"); return DD_EINVAL; }
  *out = nullptr;
  PredFileHeader h{};
  char msg[512];
  FILE* f = pred_open(path, h, msg, sizeof(msg));
  if (!f) { dd_set_error("dd_cnn_load: %s", msg); return DD_EINVAL; }
  if (h.kind != DD_PRED_CNN) {
    std::fclose(f);
    dd_set_error("dd_cnn_load: '%s' holds a PCA basis, not a network", path);
    return DD_EINVAL;
  }
  std::vector<float> buf(3 * (size_t)h.count);
  const bool ok = std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  std::fclose(f);
  if (!ok) { dd_set_error("dd_cnn_load: reading '%s' failed", path); return DD_EINVAL; }
  dd_cnn* n = nullptr;
  dd_status rc = dd_cnn_create(h.nx, h.ny, max_batch, h.k, h.in_channels, 0, &n);
  if (rc != DD_OK) return rc;
  if ((int64_t)n->nparams != h.count) {
    dd_cnn_destroy(n);
    dd_set_error("dd_cnn_load: '%s' holds %lld parameters, the network has %zu", path,
                 (long long)h.count, n->nparams);
    return DD_EINVAL;
  }
  const size_t np = n->nparams;
  hipError_t e = hipMemcpy(n->params, buf.data(), sizeof(float) * np, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->am, buf.data() + np, sizeof(float) * np, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(n->av, buf.data() + 2 * np, sizeof(float) * np, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dd_cnn_destroy(n);
    dd_set_error("dd_cnn_load: %s", hipGetErrorString(e));
    return DD_EHIP;
  }
  n->adam_t = (int)h.adam_t;
  rc = pack_all(n, 0);
  if (rc == DD_OK && hipDeviceSynchronize() != hipSuccess) rc = DD_EHIP;
  if (rc != DD_OK) { dd_cnn_destroy(n); return rc; }
  *out = n;
  return DD_OK;
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
  rc = forward(n, eps, eim, B, st);
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
  rc = forward(n, eps, eim, B, st);
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
  if (!n->rl_W) {
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
    chk(cnn_alloc(n, &n->rl_W, (size_t)n->maxB * n->k * D));
    chk(cnn_alloc(n, &n->rl_r, (size_t)n->maxB * D));
    chk(cnn_alloc(n, &n->rl_s, (size_t)n->maxB * D));
    n->rl_scratch_bytes = res_loss_scratch_bytes(n->maxB, n->k);
    chk(cnn_alloc(n, (float2**)&n->rl_scratch, (n->rl_scratch_bytes + 7) / 8));
    if (e != hipSuccess) {
      dd_set_error("%s: %s", who, hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP;
    }
  }
  rc = forward(n, eps, eim, B, st);   // fields V in n->out
  if (rc != DD_OK) return rc;
  DD_HIP_CHECK(hipGetLastError());
  std::vector<const void*> Vp(B);
  for (int p = 0; p < B; ++p) Vp[p] = (const float2*)n->out + (size_t)p * n->k * D;
  std::vector<double> lv(B);
  rc = res_loss_core(ops, b, Vp.data(), B, n->k, n->rl_W, n->rl_r, n->rl_s, lv.data(),
                     n->dz[NL - 1], n->L[NL - 1].coutp, 1.0 / B, st, nullptr, n->rl_scratch,
                     n->rl_scratch_bytes);
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
  if (layer == NL - 1) {   // n->out holds complex fields [B][k][D]: back to [pixel][2k]
    if (count != pix * L.cout) { dd_set_error("dd_cnn_debug_activation: count must be %zu", pix * L.cout); return DD_EINVAL; }
    std::vector<float> f(count);
    if (!n->last_fields) { dd_set_error("dd_cnn_debug_activation: no forward pass yet"); return DD_EINVAL; }
    DD_HIP_CHECK(hipMemcpy(f.data(), n->last_fields, sizeof(float) * count, hipMemcpyDeviceToHost));
    const int kf = n->k;
    for (size_t p = 0; p < pix; ++p) {
      const size_t b = p / D, e = p % D;
      for (int j = 0; j < kf; ++j)
        for (int c = 0; c < 2; ++c) host[p * 2 * kf + 2 * j + c] = f[((b * kf + j) * D + e) * 2 + c];
    }
    return DD_OK;
  }
  if (count != pix * L.cout) { dd_set_error("dd_cnn_debug_activation: count must be %zu", pix * L.cout); return DD_EINVAL; }
  std::vector<bf16> tmp(pix * L.coutp);
  DD_HIP_CHECK(hipMemcpy(tmp.data(), n->act[layer], sizeof(bf16) * tmp.size(), hipMemcpyDeviceToHost));
  for (size_t p = 0; p < pix; ++p)
    for (int c = 0; c < L.cout; ++c) host[p * L.cout + c] = (float)tmp[p * L.coutp + c];
  return DD_OK;
}
