// Residual loss of a predicted subspace and its gradient (Sec. 3, eq:res_loss).
//
// Definition, per problem:
//     l = min_c ||A V c - b||^2 / ||b||^2 = 1 - b^H P b / ||b||^2,
// with W = A V and P the orthogonal projector on span(W).
//
// Gradient.  Let c = W^+ b be the minimiser and r = b - W c the residual.
// Then d(b^H P b) = 2 Re(r^H dW c), so the conjugate (Wirtinger) gradient is
//     dl / d conj(W) = -r c^H / ||b||^2.
// Through W = A V it becomes
//     dl / d conj(V) = -(A^H r) c^H / ||b||^2.
// This needs one adjoint matvec per problem.  The gradient with respect to the
// real and imaginary parts of V is twice its real and imaginary part.
//
// Kernels:
//   * k_rl_apply: W = A V for all k vectors (the operator's stencil).
//   * k_rl_gram / k_rl_gram_reduce: the (k+1)^2 FP64 Gram matrix of [W b]
//     of every problem; c is solved from it on the host.
//   * k_rl_resid: r = b - W c.
//   * k_rl_adjoint: s = A^H r, the transposed stencil, conjugated.
//   * k_rl_dz: writes the CNN's last-layer gradient (bf16, NHWC).
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "common.h"
#include "devbuf.h"
#include "gram.h"   // chol_inv
#include "op.h"
#include "resloss.h"

using cd = std::complex<double>;

namespace {

struct RlDesc {
  int nx, ny, D;
  float omega2;
  const float2* cf;     // stencil coefficients (FP32 copy)
  const float* eps;     // [D]
  const float2* V;      // [k][D]
  float2* W;            // [k][D]
  const double2* b;     // [D]
  float2* r;            // [D]
  float2* s;            // [D]
  const double2* c;     // [k] minimiser
  float2* G;            // [k][D] field gradient (NULL unless requested)
};

// W_j = A V_j for all k vectors: a thread takes one cell of every vector, so
// the neighbour indices, the stencil coefficients and omega^2 eps are formed
// once per cell (the arithmetic is the operator's stencil, term for term).
__global__ __launch_bounds__(256) void k_rl_apply(const RlDesc* __restrict__ desc, int k) {
  const RlDesc d = desc[blockIdx.y];
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= d.D) return;
  const int nx = d.nx, ny = d.ny;
  const int iy = e / nx, ix = e - iy * nx;
  const int ew = (ix == 0) ? e + nx - 1 : e - 1;
  const int ee = (ix == nx - 1) ? e - nx + 1 : e + 1;
  const int es = (iy == 0) ? e + (ny - 1) * nx : e - nx;
  const int en = (iy == ny - 1) ? e - (ny - 1) * nx : e + nx;
  const float2 cxm = d.cf[ix], cxp = d.cf[nx + ix], cym = d.cf[2 * nx + iy],
               cyp = d.cf[2 * nx + ny + iy];
  const float de = d.omega2 * d.eps[e];
#pragma unroll 2
  for (int j = 0; j < k; ++j) {
    const float2* x = d.V + (size_t)j * d.D;
    const float2 c = x[e], w = x[ew], ea = x[ee], s = x[es], n = x[en];
    float2 r = cmul(cxm, csub(c, w));
    r = csub(r, cmul(cxp, csub(ea, c)));
    r = cadd(r, cmul(cym, csub(c, s)));
    r = csub(r, cmul(cyp, csub(n, c)));
    r.x -= de * c.x;
    r.y -= de * c.y;
    d.W[(size_t)j * d.D + e] = r;
  }
}

__global__ __launch_bounds__(256) void k_rl_resid(const RlDesc* __restrict__ desc, int k) {
  const RlDesc d = desc[blockIdx.y];
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= d.D) return;
  double2 v = d.b[e];
  for (int j = 0; j < k; ++j) {
    const float2 w = d.W[(size_t)j * d.D + e];
    const double2 c = d.c[j];
    v.x -= c.x * w.x - c.y * w.y;
    v.y -= c.x * w.y + c.y * w.x;
  }
  d.r[e] = make_float2((float)v.x, (float)v.y);
}

// (A^H y)_c = conj(A_cc) y_c - conj(cxm_e) y_e - conj(cxp_w) y_w - conj(cym_n) y_n
//             - conj(cyp_s) y_s, with A_cc = cxm_c + cxp_c + cym_c + cyp_c - omega^2 eps_c
// and e, w, n, s the periodic neighbours of c (row e holds -cxm_e at column c, ...).
__global__ __launch_bounds__(256) void k_rl_adjoint(const RlDesc* __restrict__ desc) {
  const RlDesc d = desc[blockIdx.y];
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= d.D) return;
  const int nx = d.nx, ny = d.ny;
  const int iy = c / nx, ix = c - iy * nx;
  const int ixe = (ix == nx - 1) ? 0 : ix + 1, ixw = (ix == 0) ? nx - 1 : ix - 1;
  const int iyn = (iy == ny - 1) ? 0 : iy + 1, iys = (iy == 0) ? ny - 1 : iy - 1;
  const float2* cf = d.cf;
  const float2 cxm = cf[ix], cxp = cf[nx + ix], cym = cf[2 * nx + iy], cyp = cf[2 * nx + ny + iy];
  float2 acc = make_float2(cxm.x + cxp.x + cym.x + cyp.x - d.omega2 * d.eps[c],
                           cxm.y + cxp.y + cym.y + cyp.y);
  const float2* y = d.r;
  float2 out = cmul(cconj(acc), y[c]);
  out = csub(out, cmul(cconj(cf[ixe]), y[iy * nx + ixe]));
  out = csub(out, cmul(cconj(cf[nx + ixw]), y[iy * nx + ixw]));
  out = csub(out, cmul(cconj(cf[2 * nx + iyn]), y[iyn * nx + ix]));
  out = csub(out, cmul(cconj(cf[2 * nx + ny + iys]), y[iys * nx + ix]));
  d.s[c] = out;
}

// dz[p][2j] = Re(s_e a_j), dz[p][2j+1] = Im(s_e a_j), p = problem * D + e, where
// a_j = -2 scale conj(c_j) / ||b||^2 (coef holds a); channels >= 2k are zero.
// coutp is a multiple of 8: a pixel's channels are written 16 B at a time.
typedef __bf16 rl_bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int rl_u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_rl_dz(const RlDesc* __restrict__ desc, int k, int coutp,
                                               const double2* __restrict__ coef,
                                               __bf16* __restrict__ dz) {
  const int pb = blockIdx.y;
  const RlDesc d = desc[pb];
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= d.D) return;
  const float2 s = d.s[e];
  __bf16* o = dz + ((size_t)pb * d.D + e) * coutp;
  for (int c0 = 0; c0 < coutp; c0 += 8) {
    rl_bf16x8 h;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ch = c0 + q;
      float g = 0.f;
      if (ch < 2 * k) {
        const double2 a = coef[(size_t)pb * k + ch / 2];
        g = (ch & 1) ? (float)(s.x * a.y + s.y * a.x) : (float)(s.x * a.x - s.y * a.y);
      }
      h[q] = (__bf16)g;
    }
    *(rl_u32x4*)(o + c0) = __builtin_bit_cast(rl_u32x4, h);
  }
}

// G[j][e] = s_e a_j with a_j = -conj(c_j) / ||b||^2 (coef holds a): the
// conjugate gradient dl / d conj(V) = -(A^H r) c^H / ||b||^2 in complex64,
// the field layout of V.
__global__ __launch_bounds__(256) void k_rl_grad(const RlDesc* __restrict__ desc, int k,
                                                 const double2* __restrict__ coef) {
  const int pb = blockIdx.y;
  const RlDesc d = desc[pb];
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= d.D) return;
  const float2 s = d.s[e];
  for (int j = 0; j < k; ++j) {
    const double2 a = coef[(size_t)pb * k + j];
    d.G[(size_t)j * d.D + e] =
        make_float2((float)(s.x * a.x - s.y * a.y), (float)(s.x * a.y + s.y * a.x));
  }
}

// Gram matrix G_ab = x_a^H x_b of [W b] (x_a = W_a for a < k, x_k = b) for
// every problem at once, FP64 sums.  One workgroup per (element slice,
// problem) stages chunks of GE elements of all k+1 vectors in LDS (element
// major, so lanes holding consecutive b read consecutive words) and each
// thread accumulates up to RL_MAXP of the (k+1)(k+2)/2 pairs a <= b in
// registers: every vector is read from HBM once.  part: [problem][slice][pair].
constexpr int RL_GE = 32;
constexpr int RL_LD = 65;                       // k + 1 <= 65, odd stride
constexpr int RL_MAXP = (65 * 66 / 2 + 255) / 256;

__device__ __forceinline__ void rl_pair(int q, int K1, int& a, int& b) {
  a = 0;
  while (q >= K1 - a) { q -= K1 - a; ++a; }
  b = a + q;
}

template <int NI>   // staging values per thread: ceil((k + 1) RL_GE / 256) <= NI
__global__ __launch_bounds__(256) void k_rl_gram(const RlDesc* __restrict__ desc, int k, int nslices,
                                                 double2* __restrict__ part) {
  __shared__ double2 xs[RL_GE * RL_LD];
  const int K1 = k + 1, np = K1 * (K1 + 1) / 2, t = threadIdx.x;
  const int slice = blockIdx.x, p = blockIdx.y;
  const RlDesc d = desc[p];
  const int per = ((d.D + nslices - 1) / nslices + RL_GE - 1) / RL_GE * RL_GE;
  const int e0 = slice * per, e1 = min(d.D, e0 + per);
  // with few pairs (np <= 128) tpp threads share a pair, each taking every
  // tpp-th element of a chunk; otherwise a thread owns pairs t, t + 256, ...
  const int tpp = (np <= 128) ? min(8, 256 / np) : 1;
  const int sub = t % tpp, t0 = t / tpp, npt = (tpp > 1) ? np : 256;   // pairs t0 + q npt
  int pa[RL_MAXP], pb[RL_MAXP];
  double sx[RL_MAXP], sy[RL_MAXP];
#pragma unroll
  for (int q = 0; q < RL_MAXP; ++q) {
    pa[q] = pb[q] = 0;
    if (q * npt + t0 < np && (tpp == 1 || q == 0)) rl_pair(q * npt + t0, K1, pa[q], pb[q]);
    sx[q] = sy[q] = 0.0;
  }
  const int nq = (tpp > 1) ? 1 : RL_MAXP;
  // this thread's staging values of the chunk at c0 (items t, t + 256, ...),
  // loaded one chunk ahead of their use
  double2 xv[NI];
  auto load = [&](int c0) {
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int i = t + 256 * j;
      const int v = i / RL_GE, el = i - v * RL_GE, e = c0 + el;
      xv[j] = make_double2(0.0, 0.0);
      if (i < K1 * RL_GE && e < e1) {
        if (v < k) {
          const float2 w = d.W[(size_t)v * d.D + e];
          xv[j] = make_double2(w.x, w.y);
        } else {
          xv[j] = d.b[e];
        }
      }
    }
  };
  if (e0 < e1) load(e0);
  for (int c0 = e0; c0 < e1; c0 += RL_GE) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int i = t + 256 * j;
      if (i < K1 * RL_GE) xs[(i % RL_GE) * RL_LD + i / RL_GE] = xv[j];
    }
    __syncthreads();
    if (c0 + RL_GE < e1) load(c0 + RL_GE);
#pragma unroll
    for (int q = 0; q < RL_MAXP; ++q) {
      if (q < nq && q * npt + t0 < np) {
        double ax = 0.0, ay = 0.0;
        for (int el = sub; el < RL_GE; el += tpp) {
          const double2 xa = xs[el * RL_LD + pa[q]], xb = xs[el * RL_LD + pb[q]];
          ax += xa.x * xb.x + xa.y * xb.y;
          ay += xa.x * xb.y - xa.y * xb.x;
        }
        sx[q] += ax;
        sy[q] += ay;
      }
    }
  }
  if (tpp > 1) {   // add the tpp partial sums of a pair in sub order
    __syncthreads();
    xs[t] = make_double2(sx[0], sy[0]);
    __syncthreads();
    if (sub == 0 && t0 < np) {
      double tx = 0.0, ty = 0.0;
      for (int j = 0; j < tpp; ++j) {
        tx += xs[t + j].x;
        ty += xs[t + j].y;
      }
      part[((size_t)p * nslices + slice) * np + t0] = make_double2(tx, ty);
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < RL_MAXP; ++q)
    if (q * 256 + t < np)
      part[((size_t)p * nslices + slice) * np + q * 256 + t] = make_double2(sx[q], sy[q]);
}

// Sum of the slice partials in slice order: out[problem][pair].
__global__ __launch_bounds__(256) void k_rl_gram_reduce(const double2* __restrict__ part, int np,
                                                        int nslices, double2* __restrict__ out) {
  const int q = blockIdx.x * 256 + threadIdx.x, p = blockIdx.y;
  if (q >= np) return;
  double sx = 0.0, sy = 0.0;
  for (int sl = 0; sl < nslices; ++sl) {
    const double2 v = part[((size_t)p * nslices + sl) * np + q];
    sx += v.x;
    sy += v.y;
  }
  out[(size_t)p * np + q] = make_double2(sx, sy);
}

// Minimiser c and loss of one problem from the Gram matrix of [W b].
bool solve_small(const std::vector<cd>& G, int k, std::vector<cd>& c, double& loss, double& bb) {
  const int K1 = k + 1;
  bb = G[(size_t)k * K1 + k].real();
  std::vector<cd> L, T, Gr = G;
  bool ok = chol_inv(Gr, K1, k, L, T);
  double shift = 0.0, dmax = 0.0;
  for (int j = 0; j < k; ++j) dmax = std::max(dmax, G[(size_t)j * K1 + j].real());
  for (int tries = 0; !ok && tries < 4; ++tries) {   // rank-deficient W: tiny ridge
    shift = (shift == 0.0) ? 1e-13 * std::max(dmax, 1e-300) : shift * 1e3;
    Gr = G;
    for (int j = 0; j < k; ++j) Gr[(size_t)j * K1 + j] += shift;
    ok = chol_inv(Gr, K1, k, L, T);
  }
  c.assign(k, cd(0.0));
  if (!ok || !(bb > 0.0)) { loss = (bb > 0.0) ? 1.0 : 0.0; return ok; }
  // c = T T^H g with g = W^H b (column k of G)
  std::vector<cd> t(k, cd(0.0));
  for (int o = 0; o < k; ++o)
    for (int a = 0; a <= o; ++a) t[o] += std::conj(T[(size_t)a * k + o]) * G[(size_t)a * K1 + k];
  double q = 0.0;
  for (int o = 0; o < k; ++o) q += std::norm(t[o]);
  for (int a = 0; a < k; ++a)
    for (int o = a; o < k; ++o) c[a] += T[(size_t)a * k + o] * t[o];
  loss = std::min(1.0, std::max(0.0, 1.0 - q / bb));
  return true;
}

}  // namespace

static size_t rl_align(size_t v) { return (v + 255) & ~(size_t)255; }

// Gram partial slices per problem: enough workgroups to fill the chip, at
// most 256, each slice at least 8 staging groups long.
static int rl_slices(int nb, int minD) {
  return std::max(1, std::min({256, (2048 + nb - 1) / nb, minD / (8 * RL_GE)}));
}

size_t res_loss_scratch_bytes(int nb, int k) {
  const size_t K1 = k + 1, np = K1 * (K1 + 1) / 2;
  return rl_align(sizeof(RlDesc) * nb) + rl_align(sizeof(double2) * 2 * (size_t)nb * k) +
         rl_align(sizeof(double2) * ((size_t)nb * 256 * np + (size_t)nb * np));
}

dd_status res_loss_core(const fdfd_op* const* ops, const void* const* b, const void* const* V,
                        int nb, int k, float2* Wbuf, float2* rbuf, float2* sbuf, double* loss,
                        __bf16* dz, int coutp, double scale, hipStream_t st,
                        void* const* Gout, void* scratch, size_t scratch_bytes) {
  std::vector<RlDesc> hd(nb);
  int maxD = 0;
  size_t offW = 0, offR = 0;
  for (int p = 0; p < nb; ++p) {
    const fdfd_op* op = ops[p];
    RlDesc& d = hd[p];
    d.nx = op->nx; d.ny = op->ny; d.D = op->D;
    d.omega2 = (float)(op->omega * op->omega);
    d.cf = op->cf32; d.eps = op->eps32;
    d.V = (const float2*)V[p]; d.W = Wbuf + offW;
    d.b = (const double2*)b[p];
    d.r = rbuf ? rbuf + offR : nullptr;
    d.s = sbuf ? sbuf + offR : nullptr;
    d.G = Gout ? (float2*)Gout[p] : nullptr;
    offW += (size_t)k * op->D;
    offR += (size_t)op->D;
    maxD = std::max(maxD, op->D);
  }
  DevBuf own;
  const size_t need = res_loss_scratch_bytes(nb, k);
  if (scratch && scratch_bytes < need) {
    dd_set_error("res_loss: scratch of %zu bytes, %zu needed", scratch_bytes, need);
    return DD_EINVAL;
  }
  if (!scratch) {
    DD_HIP_CHECK(hipMalloc(&own.p, need));
    scratch = own.p;
  }
  char* sp = (char*)scratch;
  RlDesc* dd = (RlDesc*)sp;
  double2* dc = (double2*)(sp + rl_align(sizeof(RlDesc) * nb));
  double2* gp = (double2*)(sp + rl_align(sizeof(RlDesc) * nb) +
                           rl_align(sizeof(double2) * 2 * (size_t)nb * k));
  for (int p = 0; p < nb; ++p) hd[p].c = dc + (size_t)p * k;
  DD_HIP_CHECK(hipMemcpyAsync(dd, hd.data(), sizeof(RlDesc) * nb, hipMemcpyHostToDevice, st));
  k_rl_apply<<<dim3((maxD + 255) / 256, nb), 256, 0, st>>>(dd, k);
  DD_HIP_CHECK(hipGetLastError());
  std::vector<double2> hc((size_t)2 * nb * k, make_double2(0.0, 0.0));
  // Gram matrices of [W b], all problems in one launch
  const int K1 = k + 1, np = K1 * (K1 + 1) / 2;
  int minD = maxD;
  for (const auto& d : hd) minD = std::min(minD, d.D);
  const int nslices = rl_slices(nb, minD);
  const size_t ngp = (size_t)nb * nslices * np;
  double2* gsum = gp + ngp;
  if (K1 * RL_GE <= 2 * 256)
    k_rl_gram<2><<<dim3(nslices, nb), 256, 0, st>>>(dd, k, nslices, gp);
  else
    k_rl_gram<(RL_LD * RL_GE + 255) / 256><<<dim3(nslices, nb), 256, 0, st>>>(dd, k, nslices, gp);
  k_rl_gram_reduce<<<dim3((np + 255) / 256, nb), 256, 0, st>>>(gp, np, nslices, gsum);
  DD_HIP_CHECK(hipGetLastError());
  std::vector<double2> hg((size_t)nb * np);
  DD_HIP_CHECK(hipMemcpyAsync(hg.data(), gsum, sizeof(double2) * hg.size(), hipMemcpyDeviceToHost, st));
  DD_HIP_CHECK(hipStreamSynchronize(st));
  for (int p = 0; p < nb; ++p) {
    std::vector<cd> G((size_t)K1 * K1, cd(0.0)), c;
    for (int a = 0, q = 0; a < K1; ++a)
      for (int b = a; b < K1; ++b, ++q) {
        const double2 v = hg[(size_t)p * np + q];
        G[(size_t)a * K1 + b] = cd(v.x, v.y);
        G[(size_t)b * K1 + a] = cd(v.x, -v.y);
      }
    double l = 1.0, bb = 0.0;
    solve_small(G, k, c, l, bb);
    loss[p] = l;
    for (int j = 0; j < k; ++j) {
      hc[(size_t)p * k + j] = make_double2(c[j].real(), c[j].imag());
      // d(scale l)/d Re V = 2 scale Re(dl/d conj V), likewise for Im
      const cd a = (bb > 0.0) ? -2.0 * scale * std::conj(c[j]) / bb : cd(0.0);
      hc[(size_t)(nb + p) * k + j] = make_double2(a.real(), a.imag());
    }
  }
  if (dz || Gout) {
    DD_HIP_CHECK(hipMemcpyAsync(dc, hc.data(), sizeof(double2) * hc.size(), hipMemcpyHostToDevice, st));
    k_rl_resid<<<dim3((maxD + 255) / 256, nb), 256, 0, st>>>(dd, k);
    k_rl_adjoint<<<dim3((maxD + 255) / 256, nb), 256, 0, st>>>(dd);
    if (dz)
      k_rl_dz<<<dim3((maxD + 255) / 256, nb), 256, 0, st>>>(dd, k, coutp, dc + (size_t)nb * k, dz);
    if (Gout)
      k_rl_grad<<<dim3((maxD + 255) / 256, nb), 256, 0, st>>>(dd, k, dc + (size_t)nb * k);
    DD_HIP_CHECK(hipGetLastError());
  }
  DD_HIP_CHECK(hipStreamSynchronize(st));
  return DD_OK;
}

extern "C" dd_status res_loss_batched(const fdfd_op* const* ops, const void* const* b,
                                      const void* const* V, int nb, int k, double* out,
                                      hipStream_t stream) {
  if (!ops || !b || !V || !out || nb < 1 || k < 1 || k > 64) {
    dd_set_error("res_loss_batched: need ops, b, V, out, nb >= 1 and 1 <= k <= 64");
    return DD_EINVAL;
  }
  size_t tot = 0;
  for (int p = 0; p < nb; ++p) {
    if (!ops[p] || !b[p] || !V[p]) {
      dd_set_error("res_loss_batched: problem %d has a NULL operator, b or V", p);
      return DD_EINVAL;
    }
    tot += (size_t)ops[p]->D;
  }
  DevBuf wb;
  DD_HIP_CHECK(hipMalloc(&wb.p, sizeof(float2) * tot * k));
  return res_loss_core(ops, b, V, nb, k, (float2*)wb.p, nullptr, nullptr, out, nullptr, 0, 0.0,
                       stream, nullptr);
}

extern "C" dd_status res_loss_grad_batched(const fdfd_op* const* ops, const void* const* b,
                                           const void* const* V, int nb, int k, double* out,
                                           void* const* G, hipStream_t stream) {
  if (!ops || !b || !V || !out || !G || nb < 1 || k < 1 || k > 64) {
    dd_set_error("res_loss_grad_batched: need ops, b, V, out, G, nb >= 1 and 1 <= k <= 64");
    return DD_EINVAL;
  }
  size_t tot = 0;
  for (int p = 0; p < nb; ++p) {
    if (!ops[p] || !b[p] || !V[p] || !G[p]) {
      dd_set_error("res_loss_grad_batched: problem %d has a NULL operator, b, V or G", p);
      return DD_EINVAL;
    }
    tot += (size_t)ops[p]->D;
  }
  DevBuf wb, rb, sb;
  DD_HIP_CHECK(hipMalloc(&wb.p, sizeof(float2) * tot * k));
  DD_HIP_CHECK(hipMalloc(&rb.p, sizeof(float2) * tot));
  DD_HIP_CHECK(hipMalloc(&sb.p, sizeof(float2) * tot));
  // scale 1/2: the coefficient -2 scale conj(c) / ||b||^2 becomes -conj(c) / ||b||^2
  return res_loss_core(ops, b, V, nb, k, (float2*)wb.p, (float2*)rb.p, (float2*)sb.p, out,
                       nullptr, 0, 0.5, stream, G);
}
