// Device kernels of the batched data-driven GMRES solver.
//
// All field sweeps use the same decomposition: a problem's Dp padded elements
// are cut into chunks of DD_BLOCK*R elements, one workgroup per chunk; thread t
// of a chunk owns elements base + r*DD_BLOCK + t (r < R), so every vector access
// is a coalesced 64-lane load and a thread always touches the same elements
// of every basis vector (in-place updates need no synchronisation).
// Cross-workgroup sums go through a partial-sum row per chunk, reduced in a
// fixed order in FP64 by a small one-workgroup-per-problem kernel launched
// after the sweep, so results are deterministic run to run and no sweep ever
// communicates across workgroups (on this chip a device-scope fence inside a
// kernel is a write-back of the XCD's L2).
#pragma once

#include "solver.h"

template <typename T> struct OpP;
template <> struct OpP<float> {
  static __device__ __forceinline__ const float2* cf(const ProbDesc& d) { return d.cf32; }
  static __device__ __forceinline__ const float* eps(const ProbDesc& d) { return d.eps32; }
};
template <> struct OpP<double> {
  static __device__ __forceinline__ const double2* cf(const ProbDesc& d) { return d.cf64; }
  static __device__ __forceinline__ const double* eps(const ProbDesc& d) { return d.eps64; }
};

template <typename T> __device__ __forceinline__ c2<T> to_c(double2 a) {
  return cmk<c2<T>>((T)a.x, (T)a.y);
}
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 dmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 ddiv(double2 a, double2 b) {
  const double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

// ---------------------------------------------------------------------------
// conj(B_v) . w for v < n over this workgroup's elements, 16 vectors at a
// time.  Each wave folds its 16 partial dots with the transposed butterfly
// into LDS (no workgroup barrier between groups, so the next group's loads
// issue while the previous reduction finishes); one barrier at the end adds
// the four waves' rows into prow[0 .. 2*round_up(n,16)).
#define DD_LDSN (2 * (((DD_MAX_K + DD_MAX_M + 1) + 15) / 16) * 16 + 32)
// An extra per-thread scalar (e.g. a squared norm) is summed alongside into
// prow[2*round_up(n,16)].
// With nvs > 1 the groups of 16 vectors are split over nvs workgroups of the
// same chunk: this one (vs) takes groups vs, vs + nvs, ... and writes only
// their entries; the extra scalar is written by vs = 0.
template <typename T, int R>
__device__ __forceinline__ void block_dots(const c2<T>* __restrict__ B, size_t Dp, int n,
                                           const c2<T> (&w)[R], int base,
                                           T* __restrict__ prow, T* lds, T extra = T(0),
                                           int vs = 0, int nvs = 1) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v0 = 16 * vs; v0 < n; v0 += 16 * nvs) {
    T acc[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] = T(0);
#pragma unroll
    for (int vv = 0; vv < 16; ++vv) {
      if (v0 + vv < n) {
        const c2<T>* bp = B + (size_t)(v0 + vv) * Dp + base + threadIdx.x;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const c2<T> b = ld_stream(bp + r * DD_BLOCK);
          acc[2 * vv] += b.x * w[r].x + b.y * w[r].y;
          acc[2 * vv + 1] += b.x * w[r].y - b.y * w[r].x;
        }
      }
    }
    butterfly_step<T, 32>(acc, lane);
    const T sum = acc[0] + __shfl_xor(acc[0], 1, DD_WAVE);
    if ((lane & 1) == 0) lds[wave * DD_LDSN + 2 * v0 + (lane >> 1)] = sum;
  }
  const int nv = 2 * ((n + 15) / 16) * 16;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) extra += __shfl_xor(extra, o, DD_WAVE);
  if (lane == 0) lds[wave * DD_LDSN + nv] = extra;
  __syncthreads();
  for (int i = threadIdx.x; i <= nv; i += DD_BLOCK)
    if (i == nv ? vs == 0 : (i / 32) % nvs == vs)
      prow[i] = lds[i] + lds[DD_LDSN + i] + lds[2 * DD_LDSN + i] + lds[3 * DD_LDSN + i];
}

// FP64 sums over all of problem p's partial rows, added in chunk order (the
// same order every run, so results are deterministic).  Called by a
// one-workgroup-per-problem kernel after the sweep that wrote the rows has
// finished: the kernel boundary makes the rows visible on every XCD, so no
// device-scope fence (an L2 write-back on this chip) is ever issued inside
// a sweep.
// With few values (the norms, a handful of dots) G = 256 / nvals threads
// (at most 64) share one value: thread group g sums the chunk range
// [g per, (g+1) per) and the G group sums are added in group order, so the
// result is the same every run and the serial chain of dependent loads is G
// times shorter (one problem of 480 x 240 in 512-element chunks has 225 rows).
// voff: the first value summed (values voff .. voff + nvals - 1 land in
// red[0 .. nvals - 1]); last >= 0: the last of the nvals values is value
// `last` instead (a value outside the range, summed in the same pass);
// gfix > 0: that many thread groups (gfix nvals <= DD_BLOCK), so that a value
// summed by several workgroups with different nvals is added in the same
// order in all of them.
template <typename PT>
__device__ void reduce_rows(const PlanDev& P, int blk0, int nblk, int nvals, double* red,
                            int voff = 0, int last = -1, int gfix = 0) {
  const PT* part = (const PT*)P.partial + (size_t)blk0 * P.NV + voff;
  __shared__ double grp[DD_BLOCK];
  const int G = (gfix > 0) ? gfix : (nvals >= DD_BLOCK) ? 1 : min(64, DD_BLOCK / nvals);
  const int per = (nblk + G - 1) / G;
  for (int tv = threadIdx.x; tv < ((G == 1) ? nvals : G * nvals); tv += DD_BLOCK) {
    const int v = (G == 1) ? tv : tv % nvals, g = (G == 1) ? 0 : tv / nvals;
    const int vc = (last >= 0 && v == nvals - 1) ? last - voff : v;   // column read
    const int c0 = g * per, c1 = min(nblk, c0 + per);
    double s = 0.0;
    int c = c0;
    for (; c + 16 <= c1; c += 16) {
      double a[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = (double)part[(size_t)(c + q) * P.NV + vc];
#pragma unroll
      for (int q = 0; q < 16; ++q) s += a[q];
    }
    for (; c < c1; ++c) s += (double)part[(size_t)c * P.NV + vc];
    if (G == 1) red[v] = s;
    else grp[tv] = s;
  }
  if (G > 1) {
    __syncthreads();
    for (int v = threadIdx.x; v < nvals; v += DD_BLOCK) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += grp[g * nvals + v];
      red[v] = s;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Cycle end (supplement, eq:final_lsq and the decoupling it admits): with
// q_1 = r~/||r~|| and Q orthogonal to C, the block least-squares problem
// splits into the ordinary GMRES problem min ||beta e1 - H y|| (solved by the
// Givens-rotated triangle) and x_aug = C^H r - B y; the update is
// delta = V R^{-1} x_aug + Q y.  Writes the combine coefficients [z; y].
__device__ void finish_cycle(const PlanDev& P, int p, int k, int n) {
  __shared__ double2 yv[DD_MAX_M];
  __shared__ double2 gl[DD_MAX_M + 1];
  __shared__ double2 xa[DD_MAX_K];
  const int t = threadIdx.x;
  const int m = P.m;
  const double2* H = P.H + (size_t)p * m * (m + 1);
  for (int i = t; i < n; i += DD_BLOCK) gl[i] = P.g[(size_t)p * (m + 1) + i];
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    if (t == 0) yv[i] = ddiv(gl[i], H[(size_t)i * (m + 1) + i]);
    __syncthreads();
    const double2 yi = yv[i];
    for (int l = t; l < i; l += DD_BLOCK) gl[l] = dsub(gl[l], dmul(H[(size_t)i * (m + 1) + l], yi));
    __syncthreads();
  }
  if (t < k) {
    double2 s = P.c0[(size_t)p * P.kmax + t];
    const double2* Bc = P.Bc + (size_t)p * m * P.kmax;
    for (int i = 0; i < n; ++i) s = dsub(s, dmul(Bc[(size_t)i * P.kmax + t], yv[i]));
    xa[t] = s;
  }
  __syncthreads();
  double2* comb = P.comb + (size_t)p * (P.kmax + m);
  if (t < k) {
    const double2* Ri = P.Rinv + (size_t)p * P.kmax * P.kmax;
    double2 z = make_double2(0.0, 0.0);
    for (int b = 0; b < k; ++b) z = dadd(z, dmul(Ri[(size_t)t * P.kmax + b], xa[b]));
    comb[t] = z;
  }
  // fused steps store the Krylov vectors unnormalised: q_i = hscale[i] q~_i
  for (int i = t; i < n; i += DD_BLOCK)
    comb[k + i] = P.fused ? make_double2(yv[i].x * P.hscale[(size_t)p * (m + 1) + i],
                                         yv[i].y * P.hscale[(size_t)p * (m + 1) + i])
                          : yv[i];
  if (t == 0) {
    int* st = P.stI + p * ST_NI;
    st[ST_NCOMB] = n;
    st[ST_PENDING] = 1;
    st[ST_ACTIVE] = 0;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
__global__ void k_fill_const(double2* __restrict__ v, int n, double re) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) v[i] = make_double2(re, 0.0);
}

__global__ void k_init_state(PlanDev P) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P.nb) return;
  for (int i = 0; i < ST_NI; ++i) P.stI[p * ST_NI + i] = 0;
  for (int i = 0; i < SD_ND; ++i) P.stD[p * SD_ND + i] = 0.0;
}

// r = b - A x in FP64; partial rows hold ||r||^2, ||b||^2 and, with a left
// preconditioner, ||P_L r||^2 and ||P_L b||^2.
template <int R>
__global__ __launch_bounds__(DD_BLOCK) void k_residual(PlanDev P) {
  const int chunk = blockIdx.x;
  const int p = P.blk2prob[chunk];
  if (P.stI[p * ST_NI + ST_DONE] != DONE_RUNNING) return;
  const ProbDesc d = P.desc[p];
  const int base = (chunk - d.blk0) * DD_BLOCK * R;
  double sr = 0.0, sb = 0.0, spr = 0.0, spb = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = base + r * DD_BLOCK + threadIdx.x;
    double2 rr = make_double2(0.0, 0.0);
    if (e < d.D) {
      const double2 y = stencil_point<double, double>(d.x, e, d.nx, d.ny, d.cf64, d.eps64, d.omega2);
      const double2 bb = d.b[e];
      rr = dsub(bb, y);
      sb += bb.x * bb.x + bb.y * bb.y;
      if (d.pl64) {
        const double2 l = d.pl64[e];
        const double2 lr = dmul(l, rr), lb = dmul(l, bb);
        spr += lr.x * lr.x + lr.y * lr.y;
        spb += lb.x * lb.x + lb.y * lb.y;
      }
    }
    d.r[e] = rr;
    sr += rr.x * rr.x + rr.y * rr.y;
  }
  __shared__ double lds[8];
  const double tr = block_sum1<double>(sr, lds);
  const double tb = block_sum1<double>(sb, lds);
  const double tpr = block_sum1<double>(spr, lds);
  const double tpb = block_sum1<double>(spb, lds);
  double* prow = (double*)P.partial + (size_t)chunk * P.NV;
  if (threadIdx.x == 0) { prow[0] = tr; prow[1] = tb; prow[2] = tpr; prow[3] = tpb; }
}

// One workgroup per problem: ||r||, ||b||; decides whether the problem has
// converged (||r|| <= tol ||b||), spent its budget, or starts a new cycle.
__global__ __launch_bounds__(DD_BLOCK) void k_post_residual(PlanDev P, int first) {
  const int p = blockIdx.x;
  int* st = P.stI + p * ST_NI;
  if (st[ST_DONE] != DONE_RUNNING) return;
  const ProbDesc d = P.desc[p];
  __shared__ double red[4];
  reduce_rows<double>(P, d.blk0, d.nblk, 4, red);
  if (threadIdx.x != 0) return;
  double* sd = P.stD + p * SD_ND;
  const double rho = sqrt(red[0]);
  if (first) {
    sd[SD_BNORM] = sqrt(red[1]);
    sd[SD_PBNORM] = d.pl64 ? sqrt(red[3]) : sd[SD_BNORM];
  }
  const double bn = sd[SD_BNORM];
  sd[SD_RHO] = rho;
  sd[SD_PRHO] = d.pl64 ? sqrt(red[2]) : rho;
  st[ST_PENDING] = 0;
  st[ST_ACTIVE] = 0;
  if (!isfinite(bn) || !isfinite(rho)) {
    st[ST_DONE] = DONE_NONFINITE;
    sd[SD_TRUE] = rho / bn;
  } else if (bn == 0.0) {
    st[ST_DONE] = DONE_CONVERGED;
    st[ST_FLAGS] |= FLAG_ZERO_B;
    sd[SD_TRUE] = 0.0;
  } else {
    sd[SD_TRUE] = rho / bn;
    if (rho <= P.ctl[0] * bn) {
      st[ST_DONE] = DONE_CONVERGED;
    } else if (st[ST_ITERS] >= (int)P.ctl[1]) {
      st[ST_DONE] = DONE_BUDGET;
    } else {
      st[ST_ACTIVE] = 1;
      st[ST_CYCLES] += 1;
      st[ST_J] = 0;
    }
  }
}

// Projected start, first pass: Q_0 = r / rho in the inner precision and the
// partial dots C^H Q_0 (supplement: q_1 = b~/||b~||, b~ = P b, applied to the
// cycle's residual).
template <typename T, int R>
__global__ __launch_bounds__(DD_BLOCK) void k_start_dot(PlanDev P) {
  const int chunk = blockIdx.x;
  const int p = P.blk2prob[chunk];
  if (P.stI[p * ST_NI + ST_ACTIVE] == 0) return;
  const ProbDesc d = P.desc[p];
  const int base = (chunk - d.blk0) * DD_BLOCK * R;
  const size_t Dp = d.Dp;
  c2<T>* B = (c2<T>*)d.basis + (size_t)(P.kmax - d.k) * Dp;
  const int n = d.k;
  c2<T>* q0 = B + (size_t)n * Dp;
  const double inv = 1.0 / P.stD[p * SD_ND + SD_PRHO];
  c2<T> wv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = base + r * DD_BLOCK + threadIdx.x;
    const double2 rr = d.pl64 ? dmul(d.pl64[e], d.r[e]) : d.r[e];
    wv[r] = cmk<c2<T>>((T)(rr.x * inv), (T)(rr.y * inv));
    q0[e] = wv[r];
  }
  if (n == 0) return;
  __shared__ T lds[4 * DD_LDSN];
  T* prow = (T*)P.partial + (size_t)chunk * P.NV;
  block_dots<T, R>(B, Dp, n, wv, base, prow, lds);
}

// Arnoldi step j, first sweep: w = A q_j (q_j stored unnormalised, scaled on
// the fly by hscale[j]) written to slot Q_{j+1}; partial dots [C Q_0..Q_j]^H w
// and ||w||^2.
// PC: the problem carries a diagonal preconditioner, w = P_L A P_R q_j.
// grid.y > 1 splits the dot products of a chunk over grid.y workgroups (for
// launches with few chunks); each recomputes the chunk's w, blockIdx.y = 0
// stores it.
template <typename T, int R, bool PC = false>
__global__ __launch_bounds__(DD_BLOCK) void k_matvec_dot(PlanDev P, int j) {
  const int chunk = blockIdx.x;
  const int p = P.blk2prob[chunk];
  if (P.stI[p * ST_NI + ST_ACTIVE] == 0) return;
  const ProbDesc d = P.desc[p];
  const int base = (chunk - d.blk0) * DD_BLOCK * R;
  const size_t Dp = d.Dp;
  c2<T>* B = (c2<T>*)d.basis + (size_t)(P.kmax - d.k) * Dp;
  const int n = d.k + j + 1;
  const c2<T>* q = B + (size_t)(n - 1) * Dp;
  // fused steps keep z = A q~ unscaled, in the problem's own buffer
  c2<T>* w = P.fused ? (c2<T>*)d.Z : B + (size_t)n * Dp;
  const double hs = P.fused ? 1.0 : P.hscale[(size_t)p * (P.m + 1) + j];
  c2<T> wv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = base + r * DD_BLOCK + threadIdx.x;
    c2<T> y = cmk<c2<T>>(T(0), T(0));
    if (e < d.D) {
      if (PC) {
        const c2<T>* pr = (const c2<T>*)d.pr;
        const c2<T>* pl = (const c2<T>*)d.pl;
        y = pr ? stencil_point_scaled<T>(q, pr, e, d.nx, d.ny, OpP<T>::cf(d), OpP<T>::eps(d),
                                         (T)d.omega2)
               : stencil_point<T>(q, e, d.nx, d.ny, OpP<T>::cf(d), OpP<T>::eps(d), (T)d.omega2);
        if (pl) y = cmul(pl[e], y);
        y = cscale(y, (T)hs);
      } else {
        y = cscale(stencil_point<T>(q, e, d.nx, d.ny, OpP<T>::cf(d), OpP<T>::eps(d), (T)d.omega2),
                   (T)hs);
      }
    }
    wv[r] = y;
    if (blockIdx.y == 0) w[e] = y;
  }
  T w2 = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) w2 += wv[r].x * wv[r].x + wv[r].y * wv[r].y;
  __shared__ T lds[4 * DD_LDSN];
  T* prow = (T*)P.partial + (size_t)chunk * P.NV;
  block_dots<T, R>(B, Dp, n, wv, base, prow, lds, w2, blockIdx.y, gridDim.y);
}

// One workgroup per problem: the dot products of the sweep before, as FP64
// coefficients (dst 0 -> coefA, 1 -> coefB).  After the first sweep of an
// Arnoldi step it also rescales the dot with the deferred-normalisation
// vector q_j and decides whether this step takes the second pass.
// grid.y > 1 (only without the adaptive second-pass test, which needs all
// coefficients at once): workgroup y sums its own slice of the 2n values,
// so a problem's rows are summed by several workgroups (one problem alone
// otherwise leaves the reduction to a single workgroup).
template <typename PT>
__global__ __launch_bounds__(DD_BLOCK) void k_post_dots(PlanDev P, int j, int mode, int dst) {
  const int p = blockIdx.x;
  int* st = P.stI + p * ST_NI;
  if (st[ST_ACTIVE] == 0) return;
  if (dst == 1 && mode == MODE_ARNOLDI && st[ST_REORTH] == 0) return;
  const ProbDesc d = P.desc[p];
  const int n = (mode == MODE_START) ? d.k : d.k + j + 1;
  if (n == 0) return;
  const int nvr = 2 * ((n + 15) / 16) * 16;
  const bool first_arnoldi = (mode == MODE_ARNOLDI && dst == 0);
  __shared__ double red[DD_NV_MAX];
  __shared__ double cc_l[8];
  if (gridDim.y > 1) {
    // complex values [c0, c1) of this slice
    const int per = (n + gridDim.y - 1) / gridDim.y;
    const int c0 = blockIdx.y * per, c1 = min(n, c0 + per);
    // one pass, or two in every step: the second-pass flag is the mode itself
    if (first_arnoldi && blockIdx.y == 0 && threadIdx.x == 0) st[ST_REORTH] = P.reorth_mode;
    if (c0 >= c1) return;
    reduce_rows<PT>(P, d.blk0, d.nblk, 2 * (c1 - c0), red, 2 * c0);
    const double hs = first_arnoldi ? P.hscale[(size_t)p * (P.m + 1) + j] : 1.0;
    double2* out = (dst == 0 ? P.coefA : P.coefB) + (size_t)p * P.NC;
    for (int v = c0 + threadIdx.x; v < c1; v += DD_BLOCK) {
      const double sc = (first_arnoldi && v == n - 1) ? hs : 1.0;
      out[v] = make_double2(red[2 * (v - c0)] * sc, red[2 * (v - c0) + 1] * sc);
    }
    return;
  }
  reduce_rows<PT>(P, d.blk0, d.nblk, first_arnoldi ? nvr + 1 : 2 * n, red);
  const double hs = first_arnoldi ? P.hscale[(size_t)p * (P.m + 1) + j] : 1.0;
  double2* out = (dst == 0 ? P.coefA : P.coefB) + (size_t)p * P.NC;
  double cc = 0.0;
  for (int v = threadIdx.x; v < n; v += DD_BLOCK) {
    const double s = (first_arnoldi && v == n - 1) ? hs : 1.0;
    const double2 c = make_double2(red[2 * v] * s, red[2 * v + 1] * s);
    out[v] = c;
    cc += c.x * c.x + c.y * c.y;
  }
  if (!first_arnoldi) return;
  cc = block_sum1<double>(cc, cc_l);
  if (threadIdx.x == 0) {
    // Second Gram-Schmidt pass: never, always, or when the first pass removed
    // more than half of ||w||^2 (||w - B c||^2 = ||w||^2 - ||c||^2 for an
    // orthonormal B; "twice is enough" test of Kahan and Parlett).
    int re = P.reorth_mode;
    if (re == 2) re = (red[nvr] - cc < 0.5 * red[nvr]) ? 1 : 0;
    st[ST_REORTH] = re;
  }
}

// w -= [C Q] coef over this thread's elements.  Slot nv (the deferred-
// normalisation vector q_j) is scaled by hs on the way and written back
// normalised.
template <typename T, int R>
__device__ __forceinline__ void block_update(c2<T>* __restrict__ B, size_t Dp, int n,
                                             const c2<T>* coef, c2<T> (&wv)[R], int base,
                                             int nv, T hs) {
  int v = 0;
  // four vectors per round so that 4*R loads are in flight per thread
  for (; v + 4 <= n; v += 4) {
    c2<T> b[4][R];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const c2<T>* bp = B + (size_t)(v + u) * Dp + base + threadIdx.x;
#pragma unroll
      for (int r = 0; r < R; ++r) b[u][r] = ld_stream(bp + r * DD_BLOCK);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (v + u == nv) {
        c2<T>* bp = B + (size_t)(v + u) * Dp + base + threadIdx.x;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          b[u][r] = cscale(b[u][r], hs);
          bp[r * DD_BLOCK] = b[u][r];
        }
      }
      const c2<T> cv = coef[v + u];
#pragma unroll
      for (int r = 0; r < R; ++r) wv[r] = cfnms(wv[r], cv, b[u][r]);
    }
  }
  for (; v < n; ++v) {
    c2<T>* bp = B + (size_t)v * Dp + base + threadIdx.x;
    const c2<T> cv = coef[v];
    c2<T> b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) b[r] = ld_stream(bp + r * DD_BLOCK);
    if (v == nv) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        b[r] = cscale(b[r], hs);
        bp[r * DD_BLOCK] = b[r];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) wv[r] = cfnms(wv[r], cv, b[r]);
  }
}

// CGS2 middle sweep: first update with coefA, then the second-pass dots.
template <typename T, int R>
__global__ __launch_bounds__(DD_BLOCK) void k_update_dot(PlanDev P, int j, int mode) {
  const int chunk = blockIdx.x;
  const int p = P.blk2prob[chunk];
  if (P.stI[p * ST_NI + ST_ACTIVE] == 0) return;
  if (mode == MODE_ARNOLDI && P.stI[p * ST_NI + ST_REORTH] == 0) return;
  const ProbDesc d = P.desc[p];
  const int n = (mode == MODE_START) ? d.k : d.k + j + 1;
  if (n == 0) return;
  const int base = (chunk - d.blk0) * DD_BLOCK * R;
  const size_t Dp = d.Dp;
  c2<T>* B = (c2<T>*)d.basis + (size_t)(P.kmax - d.k) * Dp;
  c2<T>* w = B + (size_t)n * Dp;
  const int nv = (mode == MODE_ARNOLDI) ? n - 1 : -1;
  const T hs = (mode == MODE_ARNOLDI) ? (T)P.hscale[(size_t)p * (P.m + 1) + j] : T(1);
  __shared__ c2<T> coef[DD_MAX_K + DD_MAX_M + 1];
  const double2* cA = P.coefA + (size_t)p * P.NC;
  for (int v = threadIdx.x; v < n; v += DD_BLOCK) coef[v] = to_c<T>(cA[v]);
  __syncthreads();
  c2<T> wv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) wv[r] = w[base + r * DD_BLOCK + threadIdx.x];
  block_update<T, R>(B, Dp, n, coef, wv, base, nv, hs);
#pragma unroll
  for (int r = 0; r < R; ++r) w[base + r * DD_BLOCK + threadIdx.x] = wv[r];
  __shared__ T lds[4 * DD_LDSN];
  T* prow = (T*)P.partial + (size_t)chunk * P.NV;
  block_dots<T, R>(B, Dp, n, wv, base, prow, lds);
}

// Final update sweep of a Gram-Schmidt step; partial rows hold ||w||^2.
template <typename T, int R>
__global__ __launch_bounds__(DD_BLOCK) void k_update_norm(PlanDev P, int j, int mode,
                                                          int start_reorth) {
  const int chunk = blockIdx.x;
  const int p = P.blk2prob[chunk];
  const int* st = P.stI + p * ST_NI;
  if (st[ST_ACTIVE] == 0) return;
  // second pass done in this step (start: per launch; Arnoldi: per problem)
  const int cgs2 = (mode == MODE_START) ? start_reorth : st[ST_REORTH];
  const ProbDesc d = P.desc[p];
  const int k = d.k;
  const int n = (mode == MODE_START) ? k : k + j + 1;
  const int base = (chunk - d.blk0) * DD_BLOCK * R;
  const size_t Dp = d.Dp;
  c2<T>* B = (c2<T>*)d.basis + (size_t)(P.kmax - k) * Dp;
  c2<T>* w = B + (size_t)n * Dp;
  const int nv = (!cgs2 && mode == MODE_ARNOLDI) ? n - 1 : -1;
  const T hs = (nv >= 0) ? (T)P.hscale[(size_t)p * (P.m + 1) + j] : T(1);
  __shared__ c2<T> coef[DD_MAX_K + DD_MAX_M + 1];
  const double2* cS = (cgs2 ? P.coefB : P.coefA) + (size_t)p * P.NC;
  for (int v = threadIdx.x; v < n; v += DD_BLOCK) coef[v] = to_c<T>(cS[v]);
  __syncthreads();
  c2<T> wv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) wv[r] = w[base + r * DD_BLOCK + threadIdx.x];
  block_update<T, R>(B, Dp, n, coef, wv, base, nv, hs);
  T s2 = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    w[base + r * DD_BLOCK + threadIdx.x] = wv[r];
    s2 += wv[r].x * wv[r].x + wv[r].y * wv[r].y;
  }
  __shared__ T lds[8];
  const T tot = block_sum1<T>(s2, lds);
  T* prow = (T*)P.partial + (size_t)chunk * P.NV;
  if (threadIdx.x == 0) prow[0] = tot;
}

// Column j of the Arnoldi relation, given the FP64 coefficients col (the k
// entries of B = C^H A q_j, then the j + 1 entries of H) and the norm of the
// new vector nrm = h_{j+1,j}: stores B and the raw column, applies the
// previous Givens rotations and a new one, updates the residual estimate
// g_{j+1} and the step counters, sets hscale[j + 1] = hs_next, and decides
// whether the cycle ends here (fin, nfin).  Called by all threads of the
// problem's workgroup, with thread t < j holding the previous rotation t
// (cs_t, sn_t: loaded by the caller before its reductions, so that their
// latency overlaps them).
static_assert(DD_MAX_M <= DD_BLOCK, "one previous rotation per thread");
static_assert(DD_MAX_K + DD_MAX_M + 1 <= 2 * DD_BLOCK, "two coefficients per thread");
__device__ void arnoldi_column(const PlanDev& P, int p, int j, int k, double2* col, double nrm,
                               double hs_next, int cgs2, double2 gj, int it0, int nre0,
                               double nsum0, double nsum20, double bn, double ctl_tol,
                               double ctl_maxit, double cs_t, double2 sn_t, int& fin, int& nfin) {
  const int m = P.m, t = threadIdx.x;
  const int n = k + j + 1;
  int* st = P.stI + p * ST_NI;
  double* sd = P.stD + p * SD_ND;
  double2* Hraw = P.Hraw + ((size_t)p * m + j) * (m + 1);
  double2* Hc = P.H + ((size_t)p * m + j) * (m + 1);
  double2* Bc = P.Bc + ((size_t)p * m + j) * P.kmax;
  double2* hcol = col + k;
  for (int v = t; v < k; v += DD_BLOCK) Bc[v] = col[v];
  for (int i = t; i <= j; i += DD_BLOCK) Hraw[i] = col[k + i];
  // Rotations 0..j-1 applied to the new column (entries b_i = hcol[i]):
  // with cur_0 = b_0 and cur_{i+1} = c_i b_{i+1} - conj(s_i) cur_i, entry i
  // becomes c_i cur_i + s_i b_{i+1} and cur_j meets the new rotation.  The
  // recurrence is affine, cur_{i+1} = f_i(cur_i) with f_i(x) = beta_i x +
  // alpha_i, so thread i forms F_i = f_i o ... o f_0 by a scan over the
  // workgroup (six shuffle rounds per wave, then the earlier waves' totals)
  // and has cur_{i+1} = F_i(cur_0) at once, instead of one lane stepping
  // through j rotations one FP64 operation at a time.
  const int lane = t & 63, wv = t >> 6;
  double2 b1 = make_double2(0.0, 0.0);                                       // b_{t+1}
  double2 MB = make_double2(1.0, 0.0), MA = make_double2(0.0, 0.0);          // identity past j
  if (t < j) {
    b1 = hcol[t + 1];
    MB = make_double2(-sn_t.x, sn_t.y);                                      // -conj(s_t)
    MA = make_double2(cs_t * b1.x, cs_t * b1.y);                             // c_t b_{t+1}
  }
  const double2 cur0 = hcol[0];
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {   // inclusive scan: (B, A) o (pB, pA)
    const double2 pB = make_double2(__shfl_up(MB.x, off, 64), __shfl_up(MB.y, off, 64));
    const double2 pA = make_double2(__shfl_up(MA.x, off, 64), __shfl_up(MA.y, off, 64));
    if (lane >= off) {
      MA = dadd(dmul(MB, pA), MA);
      MB = dmul(MB, pB);
    }
  }
  __shared__ double2 tB[DD_BLOCK / 64], tA[DD_BLOCK / 64];
  __shared__ double2 curs[DD_MAX_M + 1];
  if (lane == 63) {
    tB[wv] = MB;
    tA[wv] = MA;
  }
  __syncthreads();   // wave totals visible; every read of hcol above is done
  double2 PB = make_double2(1.0, 0.0), PA = make_double2(0.0, 0.0);   // earlier waves, in order
  for (int w = 0; w < wv; ++w) {
    PA = dadd(dmul(tB[w], PA), tA[w]);
    PB = dmul(tB[w], PB);
  }
  if (t < j) curs[t + 1] = dadd(dmul(dmul(MB, PB), cur0), dadd(dmul(MB, PA), MA));
  if (t == 0) curs[0] = cur0;
  __syncthreads();
  if (t < j) hcol[t] = dadd(make_double2(cs_t * curs[t].x, cs_t * curs[t].y), dmul(sn_t, b1));
  if (t == 0) {
    Hraw[j + 1] = make_double2(nrm, 0.0);
    const double2 cur = curs[j];
    // new rotation zeroing the subdiagonal entry nrm
    const double2 a = cur;
    const double aa = sqrt(a.x * a.x + a.y * a.y);
    double c;
    double2 s, rr;
    if (aa == 0.0) {
      c = 0.0; s = make_double2(1.0, 0.0); rr = make_double2(nrm, 0.0);
    } else {
      const double nu = sqrt(aa * aa + nrm * nrm);
      const double2 al = make_double2(a.x / aa, a.y / aa);
      c = aa / nu;
      s = make_double2(al.x * nrm / nu, al.y * nrm / nu);
      rr = make_double2(al.x * nu, al.y * nu);
    }
    hcol[j] = rr;
    P.cs[(size_t)p * m + j] = c;
    P.sn[(size_t)p * m + j] = s;
    Hc[j + 1] = make_double2(0.0, 0.0);
    double2* g = P.g + (size_t)p * (m + 1);
    const double2 gn = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    g[j + 1] = gn;
    g[j] = make_double2(c * gj.x, c * gj.y);
    P.hscale[(size_t)p * (m + 1) + j + 1] = hs_next;
    const int it = it0 + 1;
    st[ST_ITERS] = it;
    if (cgs2) {
      st[ST_NREORTH] = nre0 + 1;
      sd[SD_NSUM2] = nsum20 + (double)n;
    }
    sd[SD_NSUM] = nsum0 + (double)n;
    st[ST_J] = j + 1;
    const double est = sqrt(gn.x * gn.x + gn.y * gn.y);
    sd[SD_EST] = est / bn;
    if (it <= P.hist_cap) P.hist[(size_t)p * P.hist_cap + it - 1] = est / bn;
    if (est <= ctl_tol * bn || it >= (int)ctl_maxit || !(nrm > 0.0) || !isfinite(nrm) ||
        j + 1 == m) {
      fin = 1;
      nfin = j + 1;
    }
  }
  __syncthreads();
  for (int i = t; i <= j; i += DD_BLOCK) Hc[i] = hcol[i];   // the rotated column
}

// One workgroup per problem: the FP64 bookkeeping after the final update
// sweep.  Start phase: beta, c0 = C^H r.  Arnoldi step: the new Hessenberg
// column, B column, Givens rotation and residual estimate, and at the
// cycle's end the least-squares solve.
template <typename PT>
__global__ __launch_bounds__(DD_BLOCK) void k_post_norm(PlanDev P, int j, int mode,
                                                        int start_reorth) {
  const int p = blockIdx.x;
  int* st = P.stI + p * ST_NI;
  if (st[ST_ACTIVE] == 0) return;
  const int cgs2 = (mode == MODE_START) ? start_reorth : st[ST_REORTH];
  const ProbDesc d = P.desc[p];
  const int k = d.k;
  const int n = (mode == MODE_START) ? k : k + j + 1;
  const int m = P.m;
  const int t = threadIdx.x;
  double* sd = P.stD + p * SD_ND;
  // thread 0's scalar state for an Arnoldi step, loaded before the reduction
  // so that its latency overlaps it (only thread 0 writes these below)
  double2 gj = make_double2(0.0, 0.0);
  int it0 = 0, nre0 = 0;
  double nsum0 = 0.0, nsum20 = 0.0, bn = 0.0, ctl_tol = 0.0, ctl_maxit = 0.0;
  if (t == 0 && mode != MODE_START) {
    gj = P.g[(size_t)p * (m + 1) + j];
    it0 = st[ST_ITERS];
    nre0 = st[ST_NREORTH];
    nsum0 = sd[SD_NSUM];
    nsum20 = sd[SD_NSUM2];
    bn = sd[SD_PBNORM];
    ctl_tol = P.ctl[0];
    ctl_maxit = P.ctl[1];
  }
  // the coefficients and the previous rotations are loaded before the
  // reduction, so that their latency overlaps it (at most two per thread:
  // n <= DD_MAX_K + DD_MAX_M, j < DD_MAX_M = DD_BLOCK)
  const double2* cA = P.coefA + (size_t)p * P.NC;
  const double2* cB = P.coefB + (size_t)p * P.NC;
  double2 cv[2], cw[2];   // first- and second-pass coefficients
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int v = t + q * DD_BLOCK;
    cv[q] = cw[q] = make_double2(0.0, 0.0);
    if (v < n) {
      cv[q] = cA[v];
      cw[q] = cB[v];
    }
  }
  double cs_t = 0.0;
  double2 sn_t = make_double2(0.0, 0.0);
  if (mode != MODE_START && t < j) {
    cs_t = P.cs[(size_t)p * m + t];
    sn_t = P.sn[(size_t)p * m + t];
  }
  __shared__ double red[1];
  reduce_rows<PT>(P, d.blk0, d.nblk, 1, red);
  __shared__ double2 col[DD_MAX_K + DD_MAX_M + 2];
  __shared__ int fin, nfin;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int v = t + q * DD_BLOCK;
    if (v < n) col[v] = cgs2 ? dadd(cv[q], cw[q]) : cv[q];
  }
  if (t == 0) fin = 0;
  __syncthreads();
  const double nrm = sqrt(red[0]);
  if (mode == MODE_START) {
    const double rho = sd[SD_PRHO];
    for (int v = t; v < k; v += DD_BLOCK)
      P.c0[(size_t)p * P.kmax + v] = make_double2(rho * col[v].x, rho * col[v].y);
    if (t == 0) {
      const double beta = nrm * rho;
      sd[SD_BETA] = beta;
      P.g[(size_t)p * (m + 1)] = make_double2(beta, 0.0);
      P.hscale[(size_t)p * (m + 1)] = (nrm > 0.0) ? 1.0 / nrm : 0.0;
      st[ST_J] = 0;
      if (!(nrm > 0.0) || !isfinite(nrm)) { fin = 1; nfin = 0; }
    }
  } else {
    arnoldi_column(P, p, j, k, col, nrm, (nrm > 0.0) ? 1.0 / nrm : 0.0, cgs2, gj, it0, nre0, nsum0,
                   nsum20, bn, ctl_tol, ctl_maxit, cs_t, sn_t, fin, nfin);
  }
  __syncthreads();
  if (fin) finish_cycle(P, p, k, nfin);
}

// x += V z + Q y in FP64 for every problem whose cycle just ended.
template <typename T, int R>
__global__ __launch_bounds__(DD_BLOCK) void k_combine(PlanDev P) {
  const int chunk = blockIdx.x;
  const int p = P.blk2prob[chunk];
  const int* st = P.stI + p * ST_NI;
  if (st[ST_PENDING] == 0) return;
  const ProbDesc d = P.desc[p];
  const int n = st[ST_NCOMB];
  const int k = d.k;
  const int base = (chunk - d.blk0) * DD_BLOCK * R;
  const size_t Dp = d.Dp;
  __shared__ double2 cf[DD_MAX_K + DD_MAX_M];
  const double2* comb = P.comb + (size_t)p * (P.kmax + P.m);
  for (int v = threadIdx.x; v < k + n; v += DD_BLOCK) cf[v] = comb[v];
  __syncthreads();
  const c2<T>* V = (const c2<T>*)d.V;
  const c2<T>* Q = (const c2<T>*)d.basis + (size_t)P.kmax * Dp;
  double2 acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = make_double2(0.0, 0.0);
  for (int v = 0; v < k; ++v) {
    const double2 c = cf[v];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const c2<T> b = ld_stream(V + (size_t)v * Dp + base + r * DD_BLOCK + threadIdx.x);
      acc[r] = dadd(acc[r], dmul(c, make_double2((double)b.x, (double)b.y)));
    }
  }
  if (!d.pr64) {
    for (int i = 0; i < n; ++i) {
      const double2 c = cf[k + i];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const c2<T> b = ld_stream(Q + (size_t)i * Dp + base + r * DD_BLOCK + threadIdx.x);
        acc[r] = dadd(acc[r], dmul(c, make_double2((double)b.x, (double)b.y)));
      }
    }
  } else {
    // right preconditioner: the Krylov part lives in the scaled variable
    double2 aq[R];
#pragma unroll
    for (int r = 0; r < R; ++r) aq[r] = make_double2(0.0, 0.0);
    for (int i = 0; i < n; ++i) {
      const double2 c = cf[k + i];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const c2<T> b = ld_stream(Q + (size_t)i * Dp + base + r * DD_BLOCK + threadIdx.x);
        aq[r] = dadd(aq[r], dmul(c, make_double2((double)b.x, (double)b.y)));
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      acc[r] = dadd(acc[r], dmul(d.pr64[base + r * DD_BLOCK + threadIdx.x], aq[r]));
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = base + r * DD_BLOCK + threadIdx.x;
    if (e < d.D) d.x[e] = dadd(d.x[e], acc[r]);
  }
}

// ============================ fused Arnoldi sweep ============================
// One sweep per Arnoldi step (cgs_passes = 1, k + m + 1 <= 128, nx <= 512).
// The Krylov vectors are normalised one step late, q_i = s_i q~_i with FP64
// scales s_i = hscale[i] (C columns: s = 1), and z_j = A q~_j is kept
// unscaled in a separate double buffer.  With d_v = b_v^H z_j the raw dots of
// z_j against the basis b = [C, q~_0 .. q~_j], the next vector is the
// classical Gram-Schmidt remainder of A q_j = s_j z_j,
//     q~_{j+1} = s_j z_j - sum_v g_v b_v,   g_v = s_j s_v^2 d_v,
// with h_{v,j} = s_v s_j d_v, h_{j+1,j} = ||q~_{j+1}|| and s_{j+1} =
// 1 / ||q~_{j+1}|| (so the stored vectors stay of the size of the entries of
// H).  The sweep of step j forms q~_{j+1}, then z_{j+1} =
// A q~_{j+1} and its raw dots against [C, q~_0 .. q~_{j+1}] plus ||q~_{j+1}||^2,
// so every basis value is fetched from memory once per step where the two
// classical passes (dots, then update) fetch it twice.
//
// The stencil needs q~_{j+1} at the rows above and below, which other tiles
// form in the same launch.  A workgroup therefore walks a strip of
// DD_FUSED_SW columns down a band of rows.  At walk step t it updates row
// y0 - 1 + t over the strip and one halo column on each side (the halo
// columns and the halo rows above and below the band are recomputed rather
// than read), applies the stencil to the row behind it from a ring of three
// updated rows in LDS, and takes that row's dots against the basis values it
// fetched at the step before, still in registers: every basis value is read
// from memory once.  Thread (vl, c) of the 512 handles column c of the strip
// (with its halos, 32 lanes) and the basis vectors v = vl, vl + 16, ...;
// its dots accumulate in registers over the whole band and are folded over
// the columns once at the end.  One partial row per tile, reduced in tile
// order by k_post_fused.
#define DD_FUSED_THREADS 512
#define DD_FUSED_MAXN 128                // basis vectors of one step: n + 1 <= 128
#ifndef DD_FUSED_LANES
#define DD_FUSED_LANES 32                // column lanes of a strip (owned columns + 2 halos)
#endif
#define DD_FUSED_SW (DD_FUSED_LANES - 2)
#define DD_FUSED_VL (DD_FUSED_THREADS / DD_FUSED_LANES)
#define DD_FUSED_PER (DD_FUSED_MAXN / DD_FUSED_VL)

template <typename T>
__device__ __forceinline__ c2<T> stencil_vals(c2<T> c, c2<T> w, c2<T> ea, c2<T> s, c2<T> n,
                                              c2<T> cxm, c2<T> cxp, c2<T> cym, c2<T> cyp, T de) {
  // the arithmetic of stencil_point, on values already at hand
  c2<T> r = cmul(cxm, csub(c, w));
  r = csub(r, cmul(cxp, csub(ea, c)));
  r = cadd(r, cmul(cym, csub(c, s)));
  r = csub(r, cmul(cyp, csub(n, c)));
  r.x -= de * c.x;
  r.y -= de * c.y;
  return r;
}

template <typename V> __device__ __forceinline__ V cfma(V acc, V a, V b) {   // acc + a*b
  return cmk<V>(acc.x + (a.x * b.x - a.y * b.y), acc.y + (a.x * b.y + a.y * b.x));
}
template <typename V> __device__ __forceinline__ V cfmac(V acc, V a, V b) {  // acc + conj(a)*b
  return cmk<V>(acc.x + (a.x * b.x + a.y * b.y), acc.y + (a.x * b.y - a.y * b.x));
}

template <typename T, bool PC>
__global__ __launch_bounds__(DD_FUSED_THREADS, 4) void k_fused_sweep(PlanDev P, int j) {
  using V = c2<T>;
  constexpr int NVL = DD_FUSED_VL, PER = DD_FUSED_PER, L = DD_FUSED_LANES;
  const FusedTile tl = P.tiles[blockIdx.x];
  const int p = tl.p;
  if (p < 0 || P.stI[p * ST_NI + ST_ACTIVE] == 0) return;
  const ProbDesc d = P.desc[p];
  const int nx = d.nx, ny = d.ny;
  const size_t Dp = d.Dp;
  const int k = d.k;
  const int n = k + j + 1;                                   // basis [C, q~_0 .. q~_j]
  const V* B = (const V*)d.basis + (size_t)(P.kmax - k) * Dp;
  V* qn = (V*)d.basis + (size_t)(P.kmax + j + 1) * Dp;       // q~_{j+1}
  const V* zin = (const V*)d.Z + (size_t)(j & 1) * Dp;       // z_j
  V* zout = (V*)d.Z + (size_t)((j + 1) & 1) * Dp;            // z_{j+1}
  const int vl = threadIdx.x / L, cl = threadIdx.x % L;
  const int w = min(DD_FUSED_SW, nx - tl.x0);                // owned columns of the strip
  const bool lane_ok = cl <= w + 1;                          // owned or halo column
  const bool owned = cl >= 1 && cl <= w;
  int c = tl.x0 - 1 + cl;                                    // this lane's column (wrapped)
  c = (c < 0) ? c + nx : ((c >= nx) ? c - nx : c);
  if (!lane_ok) c = 0;                                       // a valid address, value unused
  const int y0 = tl.y0, nrows = tl.y1 - tl.y0;
  const T sj = (T)P.hscale[(size_t)p * (P.m + 1) + j];      // s_j
  __shared__ V coef[DD_FUSED_MAXN];
  __shared__ V part[NVL][L];
  __shared__ V ring[3][L];                                   // q~_{j+1} on the last 3 rows
  __shared__ V ringp[3][L];                                  // P_R q~_{j+1} (stencil input)
  __shared__ V zrow[L];
  const double2* cB = P.coefB + (size_t)p * P.NC;
  for (int v = threadIdx.x; v < n; v += DD_FUSED_THREADS) coef[v] = to_c<T>(cB[v]);
  const V* cf = OpP<T>::cf(d);
  const auto* epsp = OpP<T>::eps(d);
  const T om2 = (T)d.omega2;
  const V* pl = PC ? (const V*)d.pl : nullptr;
  const V* pr = PC ? (const V*)d.pr : nullptr;
  const V zero = cmk<V>(T(0), T(0));
  V cxm = zero, cxp = zero;
  if (vl == 0) {
    cxm = cf[c];
    cxp = cf[nx + c];
  }
  V bprev[PER], bcur[PER], bnext[PER], acc[PER];
  auto wrapy = [&](int y) { return (y < 0) ? y + ny : ((y >= ny) ? y - ny : y); };
  // unconditional loads from valid addresses (vector index clamped, invalid
  // lanes at column 0), zeroed where they are used: a branch per load would
  // make the compiler wait for each before issuing the next
  auto load_row = [&](V (&dst)[PER], int t) {
    const size_t r = (size_t)wrapy(y0 - 1 + t) * nx + c;
#pragma unroll
    for (int i = 0; i < PER; ++i) dst[i] = B[(size_t)min(vl + NVL * i, n - 1) * Dp + r];
  };
#pragma unroll
  for (int i = 0; i < PER; ++i) { bprev[i] = zero; acc[i] = zero; }
  V accn = zero;                 // dots of the new vector (vl = 0 lanes)
  T un2 = T(0);                  // ||q~_{j+1}||^2 over the tile's owned cells
  load_row(bcur, 0);
  __syncthreads();
  for (int t = 0; t <= nrows + 1; ++t) {
    const int yu = wrapy(y0 - 1 + t);
    const size_t ru = (size_t)yu * nx + c;
    // the next row's values are in flight during this step
    if (t <= nrows) load_row(bnext, t + 1);
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (!(vl + NVL * i < n && lane_ok)) bcur[i] = zero;
    // (a) the update of row yu: this thread's share of sum_v g_v b_v
    V pu = zero;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int v = vl + NVL * i;
      pu = cfma(pu, coef[min(v, n - 1)], bcur[i]);
    }
    part[vl][cl] = pu;
    V zj = zero, prv = zero;
    if (vl == 0 && lane_ok) {
      zj = zin[ru];
      if (PC && pr) prv = pr[ru];
    }
    __syncthreads();
    if (vl == 0) {
      V sum = zero;
#pragma unroll
      for (int q = 0; q < NVL; ++q) sum = cadd(sum, part[q][cl]);
      const V u = csub(cscale(zj, sj), sum);
      ring[t % 3][cl] = u;
      ringp[t % 3][cl] = (PC && pr) ? cmul(u, prv) : u;
      if (owned && t >= 1 && t <= nrows) {
        qn[ru] = u;
        un2 += u.x * u.x + u.y * u.y;
      }
    }
    // (b) z_{j+1} = A q~_{j+1} on row ys = yu - 1, then its dots against the
    // basis row fetched at the step before.  The ring is written and read
    // only by the vl = 0 lanes, which are one wave (lanes 0-31 of wave 0), so
    // it needs no barrier of its own.
    if (t >= 2) {
      const int ys = y0 + t - 2;
      if (vl == 0) {
        V z = zero;
        if (owned) {
          const size_t rs = (size_t)ys * nx + c;
          const V* rc = ringp[(t - 1) % 3];
          z = stencil_vals<T>(rc[cl], rc[cl - 1], rc[cl + 1], ringp[(t - 2) % 3][cl],
                              ringp[t % 3][cl], cxm, cxp, cf[2 * nx + ys], cf[2 * nx + ny + ys],
                              om2 * (T)epsp[rs]);
          if (PC && pl) z = cmul(pl[rs], z);
          zout[rs] = z;
          accn = cfmac(accn, ring[(t - 1) % 3][cl], z);
        }
        zrow[cl] = z;
      }
      __syncthreads();
      const V zc = zrow[cl];
#pragma unroll
      for (int i = 0; i < PER; ++i) acc[i] = cfmac(acc[i], bprev[i], zc);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      bprev[i] = bcur[i];
      bcur[i] = bnext[i];
    }
  }
  // ---- partial row: dots d_v (v <= n), then ||q~_{j+1}||^2, folded over the
  // column lanes of each vector lane in a fixed order
#pragma unroll
  for (int o = L / 2; o >= 1; o >>= 1) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      acc[i].x += __shfl_xor(acc[i].x, o, DD_WAVE);
      acc[i].y += __shfl_xor(acc[i].y, o, DD_WAVE);
    }
    accn.x += __shfl_xor(accn.x, o, DD_WAVE);
    accn.y += __shfl_xor(accn.y, o, DD_WAVE);
    un2 += __shfl_xor(un2, o, DD_WAVE);
  }
  T* prow = (T*)P.partial + (size_t)tl.row * P.NV;
  if (cl == 0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int v = vl + NVL * i;
      if (v < n) {
        prow[2 * v] = acc[i].x;
        prow[2 * v + 1] = acc[i].y;
      }
    }
    if (vl == 0) {
      prow[2 * n] = accn.x;
      prow[2 * n + 1] = accn.y;
      prow[2 * (n + 1)] = un2;
    }
  }
}

// After a fused sweep (init = 1: after the first matvec of a cycle,
// k_matvec_dot writing z_0 = A q~_0 unscaled).  Reduces the tile rows: raw
// dots d' of z_{j+1} (z_0) and ||q~_{j+1}||^2.  For a step: completes column
// j of the Arnoldi relation from the previous dots and h_{j+1,j} =
// ||q~_{j+1}||, sets s_{j+1}, runs the Givens update (arnoldi_column) and ends
// the cycle if due.  Then stores the new raw dots and the next update
// coefficients g_v = s_{j+1} s_v^2 d'_v (coefB; s_0 for init).  The raw dots
// alternate between coefA (written by init and odd j... read back by even
// steps) and coefA2, so that a step reads the previous dots while the new ones
// are written: grid.y workgroups per problem each reduce a slice of the new
// dots (every slice sums the norm in the same order, so s_{j+1} is the same
// in all), and slice 0 alone does the Givens update.
template <typename PT>
__global__ __launch_bounds__(DD_BLOCK) void k_post_fused(PlanDev P, int j, int init) {
  const int p = blockIdx.x;
  int* st = P.stI + p * ST_NI;
  if (st[ST_ACTIVE] == 0) return;
  const ProbDesc d = P.desc[p];
  const int k = d.k, m = P.m, t = threadIdx.x;
  const int nn = init ? k + 1 : k + j + 2;      // vectors of the new dots
  const double* hs = P.hscale + (size_t)p * (m + 1);
  double* sd = P.stD + p * SD_ND;
  const bool lead = blockIdx.y == 0;
  // dots written by the call before (init, or step j - 1), and the new ones
  double2* cOld = ((j & 1) ? P.coefA2 : P.coefA) + (size_t)p * P.NC;
  double2* cNew = ((init || (j & 1)) ? P.coefA : P.coefA2) + (size_t)p * P.NC;
  double2* cB = P.coefB + (size_t)p * P.NC;
  double2 gj = make_double2(0.0, 0.0);
  int it0 = 0;
  double nsum0 = 0.0, bn = 0.0, ctl_tol = 0.0, ctl_maxit = 0.0;
  if (lead && t == 0 && !init) {
    gj = P.g[(size_t)p * (m + 1) + j];
    it0 = st[ST_ITERS];
    nsum0 = sd[SD_NSUM];
    bn = sd[SD_PBNORM];
    ctl_tol = P.ctl[0];
    ctl_maxit = P.ctl[1];
  }
  __shared__ double red[DD_NV_MAX];
  __shared__ double nrm2[1];
  __shared__ double2 col[DD_MAX_K + DD_MAX_M + 2];
  __shared__ int fin, nfin;
  // the lead slice's column of the previous dots and the previous rotations,
  // loaded before the reductions so that their latency overlaps them (at
  // most two per thread)
  double2 cv[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  double cs_t = 0.0;
  double2 sn_t = make_double2(0.0, 0.0);
  if (lead && !init) {
    const double sj = hs[j];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int v = t + q * DD_BLOCK;
      if (v < k + j + 1) {
        const double2 dv = cOld[v];
        const double sv = (v < k) ? 1.0 : hs[v - k];
        cv[q] = make_double2(sv * sj * dv.x, sv * sj * dv.y);
      }
    }
    if (t < j) {
      cs_t = P.cs[(size_t)p * m + t];
      sn_t = P.sn[(size_t)p * m + t];
    }
  }
  // complex values [c0, c1) of this slice
  const int per = (nn + gridDim.y - 1) / gridDim.y;
  const int c0 = blockIdx.y * per, c1 = min(nn, c0 + per);
  double snew;
  if (init) {
    // k_matvec_dot's rows: dots [C, q~_0]^H z_0 in 16-vector groups
    if (c0 < c1) reduce_rows<PT>(P, d.blk0, d.nblk, 2 * (c1 - c0), red, 2 * c0);
    snew = hs[0];
  } else {
    // the slice's values and ||q~_{j+1}||^2 (value 2 nn) in one pass, with
    // the thread groups of the largest slice in every slice (the same sum
    // order for the norm, so every slice has the same s_{j+1})
    const int nv = (c0 < c1) ? 2 * (c1 - c0) : 0;
    const int gfix = max(1, min(64, DD_BLOCK / (2 * per + 1)));
    reduce_rows<PT>(P, d.t0, d.nt, nv + 1, red, (c0 < c1) ? 2 * c0 : 2 * nn, 2 * nn, gfix);
    if (t == 0) nrm2[0] = red[nv];
    __syncthreads();
    const double nrm = sqrt(nrm2[0]);
    snew = (nrm > 0.0) ? 1.0 / nrm : 0.0;
    if (lead) {
      if (t == 0) fin = 0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int v = t + q * DD_BLOCK;
        if (v < k + j + 1) col[v] = cv[q];
      }
      __syncthreads();
      arnoldi_column(P, p, j, k, col, nrm, snew, 0, gj, it0, 0, nsum0, 0.0, bn, ctl_tol,
                     ctl_maxit, cs_t, sn_t, fin, nfin);
      __syncthreads();
    }
  }
  // the new raw dots and update coefficients (s_v for v <= k + j are those
  // of earlier steps; s_{j+1} = snew)
  for (int v = c0 + t; v < c1; v += DD_BLOCK) {
    const double2 dv = make_double2(red[2 * (v - c0)], red[2 * (v - c0) + 1]);
    const double sv = (v < k) ? 1.0 : (v - k == (init ? 0 : j + 1) ? snew : hs[v - k]);
    const double gs = snew * sv * sv;
    cNew[v] = dv;
    cB[v] = make_double2(gs * dv.x, gs * dv.y);
  }
  if (lead && !init) {
    __syncthreads();
    if (fin) finish_cycle(P, p, k, nfin);
  }
}

// Diagonal preconditioner of problem p, [Dp] elements, zero in the padding.
// Jacobi (left): P_L = diag(A)^{-1} with diag(A)_c = cxm + cxp + cym + cyp -
// omega^2 eps_c.  PML scaling: P_L = S^{1/2}, P_R = S^{-1/2} with
// S = diag(s_x(i) s_y(j)) (integer-node stretch factors s64), the diagonal
// that makes S A complex symmetric; P_L A P_R is then complex symmetric with
// the spectrum of A.  Principal square roots (Re s > 0).
__global__ void k_precond_init(PlanDev P, int p, int type, const double2* __restrict__ s64,
                               double2* pl64, double2* pr64, float2* pl32, float2* pr32) {
  const ProbDesc d = P.desc[p];
  for (int e = blockIdx.x * DD_BLOCK + threadIdx.x; e < d.Dp; e += gridDim.x * DD_BLOCK) {
    double2 l = make_double2(0.0, 0.0), rr = make_double2(0.0, 0.0);
    if (e < d.D) {
      const int iy = e / d.nx, ix = e - iy * d.nx;
      if (type == DD_PRECOND_JACOBI) {
        const double2* cf = d.cf64;
        const double2 dg = make_double2(
            cf[ix].x + cf[d.nx + ix].x + cf[2 * d.nx + iy].x + cf[2 * d.nx + d.ny + iy].x -
                d.omega2 * d.eps64[e],
            cf[ix].y + cf[d.nx + ix].y + cf[2 * d.nx + iy].y + cf[2 * d.nx + d.ny + iy].y);
        l = ddiv(make_double2(1.0, 0.0), dg);
      } else {
        const double2 sv = dmul(s64[ix], s64[d.nx + iy]);
        const double a = sqrt(sv.x * sv.x + sv.y * sv.y);
        const double re = sqrt(0.5 * (a + sv.x));
        const double im = copysign(sqrt(fmax(0.0, 0.5 * (a - sv.x))), sv.y);
        l = make_double2(re, im);
        rr = ddiv(make_double2(1.0, 0.0), l);
      }
    }
    pl64[e] = l;
    pr64[e] = rr;
    pl32[e] = make_float2((float)l.x, (float)l.y);
    pr32[e] = make_float2((float)rr.x, (float)rr.y);
  }
}

// ============================ augmentation setup ============================
// Copy the caller's vectors into the padded V slots; non-finite entries are
// replaced by zero and mark their column as unusable.
template <typename T>
__global__ void k_copy_pad(PlanDev P, const void* const* U) {
  const int p = blockIdx.z, v = blockIdx.y;
  const ProbDesc d = P.desc[p];
  if (v >= d.k) return;
  const c2<T>* u = (const c2<T>*)U[p] + (size_t)v * d.D;
  c2<T>* V = (c2<T>*)d.V + (size_t)v * d.Dp;
  bool bad = false;
  for (int e = blockIdx.x * DD_BLOCK + threadIdx.x; e < d.Dp; e += gridDim.x * DD_BLOCK) {
    c2<T> a = cmk<c2<T>>(T(0), T(0));
    if (e < d.D) {
      a = u[e];
      if (!isfinite(a.x) || !isfinite(a.y)) { bad = true; a = cmk<c2<T>>(T(0), T(0)); }
    }
    V[e] = a;
  }
  if (bad) atomicOr(&P.bad[p], 1ull << v);
}

// W_v = A V_v written into the C slots (right-aligned), all columns at once.
template <typename T>
__global__ void k_stencil_multi(PlanDev P) {
  const int p = blockIdx.z, v = blockIdx.y;
  const ProbDesc d = P.desc[p];
  if (v >= d.k) return;
  const c2<T>* x = (const c2<T>*)d.V + (size_t)v * d.Dp;
  c2<T>* y = (c2<T>*)d.basis + (size_t)(P.kmax - d.k + v) * d.Dp;
  for (int e = blockIdx.x * DD_BLOCK + threadIdx.x; e < d.Dp; e += gridDim.x * DD_BLOCK) {
    c2<T> a = cmk<c2<T>>(T(0), T(0));
    if (e < d.D) {
      a = stencil_point<T>(x, e, d.nx, d.ny, OpP<T>::cf(d), OpP<T>::eps(d), (T)d.omega2);
      if (d.pl) a = cmul(((const c2<T>*)d.pl)[e], a);   // W = P_L A U (U given in x-space)
    }
    y[e] = a;
  }
}

__host__ __device__ inline int gram_tiles(int k) {
  const int t = (k + 3) / 4;
  return t * (t + 1) / 2;
}

// Partial Gram matrices G = W^H W of the C slots, 4x4 complex tiles of the
// upper triangle, FP64 accumulation; one row of partials per workgroup.
template <typename T>
__global__ __launch_bounds__(DD_BLOCK) void k_gram(PlanDev P) {
  const int p = blockIdx.y;
  const ProbDesc d = P.desc[p];
  const int k = d.k;
  if (k == 0) return;
  const c2<T>* W = (const c2<T>*)d.basis + (size_t)(P.kmax - k) * d.Dp;
  const int nt = (k + 3) / 4;
  const int ntiles_max = gram_tiles(P.kmax);
  __shared__ double lds[128];
  int ti = 0;
  for (int ta = 0; ta < nt; ++ta)
    for (int tb = ta; tb < nt; ++tb, ++ti) {
      double acc[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) acc[i] = 0.0;
      for (int e = blockIdx.x * DD_BLOCK + threadIdx.x; e < d.D; e += gridDim.x * DD_BLOCK) {
        double2 a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int va = ta * 4 + q, vb = tb * 4 + q;
          const c2<T> xa = (va < k) ? W[(size_t)va * d.Dp + e] : cmk<c2<T>>(T(0), T(0));
          const c2<T> xb = (vb < k) ? W[(size_t)vb * d.Dp + e] : cmk<c2<T>>(T(0), T(0));
          a[q] = make_double2((double)xa.x, (double)xa.y);
          b[q] = make_double2((double)xb.x, (double)xb.y);
        }
#pragma unroll
        for (int qa = 0; qa < 4; ++qa)
#pragma unroll
          for (int qb = 0; qb < 4; ++qb) {
            acc[2 * (qa * 4 + qb)] += a[qa].x * b[qb].x + a[qa].y * b[qb].y;
            acc[2 * (qa * 4 + qb) + 1] += a[qa].x * b[qb].y - a[qa].y * b[qb].x;
          }
      }
      block_sum32<double>(acc, lds,
                          P.gpart + (((size_t)p * P.GB + blockIdx.x) * ntiles_max + ti) * 32);
    }
}

// One workgroup per problem: reduce the Gram partials, Cholesky factor with
// column dropping (pivot below 1e-6 of the largest column norm, or a column
// already marked unusable), T = L^{-H} on the kept columns, R^{-1} <- R^{-1} T.
__global__ __launch_bounds__(DD_BLOCK) void k_chol(PlanDev P, int pass) {
  const int p = blockIdx.x;
  const ProbDesc d = P.desc[p];
  const int k = d.k;
  const int t = threadIdx.x;
  const int K = P.kmax;
  if (k == 0) {
    if (t == 0) P.keep[p] = 0ull;
    return;
  }
  double2* G = P.Gm + (size_t)p * K * K;    // G, then L in its lower triangle
  double2* Tm = P.Tm + (size_t)p * K * K;
  double2* Ri = P.Rinv + (size_t)p * K * K;
  const int nt = (k + 3) / 4;
  const int ntiles_max = gram_tiles(K);
  // reduce partials (fixed order over workgroups)
  for (int idx = t; idx < gram_tiles(k) * 16; idx += DD_BLOCK) {
    const int ti = idx >> 4, el = idx & 15;
    int ta = 0, tb = 0, c = 0;
    for (int a = 0; a < nt; ++a)
      for (int b = a; b < nt; ++b, ++c)
        if (c == ti) { ta = a; tb = b; }
    const int qa = el >> 2, qb = el & 3;
    const int ra = ta * 4 + qa, rb = tb * 4 + qb;
    double sx = 0.0, sy = 0.0;
    for (int g = 0; g < P.GB; ++g) {
      const double* row = P.gpart + (((size_t)p * P.GB + g) * ntiles_max + ti) * 32;
      sx += row[2 * el];
      sy += row[2 * el + 1];
    }
    if (ra < k && rb < k) {
      G[(size_t)ra * K + rb] = make_double2(sx, sy);
      G[(size_t)rb * K + ra] = make_double2(sx, -sy);
    }
  }
  __shared__ unsigned long long mask_s;
  __shared__ double maxd_s;
  __shared__ double2 Ljj;
  __shared__ int drop_s;
  if (t == 0) {
    unsigned long long mask = (pass == 0) ? ~P.bad[p] : P.keep[p];
    if (k < 64) mask &= (1ull << k) - 1ull;
    double mx = 0.0;
    for (int i = 0; i < k; ++i)
      if ((mask >> i) & 1ull) {
        const double gi = G[(size_t)i * K + i].x;
        if (isfinite(gi) && gi > mx) mx = gi;
        if (!isfinite(gi)) mask &= ~(1ull << i);
      }
    mask_s = mask;
    maxd_s = sqrt(mx);
  }
  __syncthreads();
  const double thr = 1e-6 * maxd_s;
  for (int jj = 0; jj < k; ++jj) {
    if (t == 0) {
      drop_s = 0;
      if (!((mask_s >> jj) & 1ull)) {
        drop_s = 1;
      } else {
        double s = G[(size_t)jj * K + jj].x;
        for (int l = 0; l < jj; ++l) {
          const double2 v = G[(size_t)jj * K + l];
          s -= v.x * v.x + v.y * v.y;
        }
        if (!(s > thr * thr) || !isfinite(s)) {
          drop_s = 1;
          mask_s &= ~(1ull << jj);
        } else {
          Ljj = make_double2(sqrt(s), 0.0);
        }
      }
    }
    __syncthreads();
    if (drop_s) {
      for (int i = t; i < k; i += DD_BLOCK) {
        if (i >= jj) G[(size_t)i * K + jj] = make_double2(0.0, 0.0);   // column
        if (i < jj) G[(size_t)jj * K + i] = make_double2(0.0, 0.0);    // row left of diag
      }
    } else {
      const double ljj = Ljj.x;
      for (int i = jj + 1 + t; i < k; i += DD_BLOCK) {
        if (!((mask_s >> i) & 1ull)) continue;
        double2 s = G[(size_t)i * K + jj];
        for (int l = 0; l < jj; ++l) {
          const double2 a = G[(size_t)i * K + l], b = G[(size_t)jj * K + l];
          s = dsub(s, make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y));  // a conj(b)
        }
        G[(size_t)i * K + jj] = make_double2(s.x / ljj, s.y / ljj);
      }
      if (t == 0) G[(size_t)jj * K + jj] = Ljj;
    }
    __syncthreads();
  }
  // rows of dropped columns that were filled before the drop decision
  for (int idx = t; idx < k * k; idx += DD_BLOCK) {
    const int i = idx / k, l = idx % k;
    if (l < i && !((mask_s >> i) & 1ull)) G[(size_t)i * K + l] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  const unsigned long long mask = mask_s;
  // T = L^{-H}: solve L^H T = I column by column (one thread per column o)
  for (int o = t; o < k; o += DD_BLOCK) {
    for (int a = k - 1; a >= 0; --a) {
      double2 v = make_double2(0.0, 0.0);
      if (((mask >> o) & 1ull) && ((mask >> a) & 1ull) && a <= o) {
        v = make_double2(a == o ? 1.0 : 0.0, 0.0);
        for (int l = a + 1; l <= o; ++l) {
          if (!((mask >> l) & 1ull)) continue;
          v = dsub(v, dmulc(G[(size_t)l * K + a], Tm[(size_t)l * K + o]));
        }
        const double laa = G[(size_t)a * K + a].x;
        v = make_double2(v.x / laa, v.y / laa);
      }
      Tm[(size_t)a * K + o] = v;
    }
  }
  __syncthreads();
  if (pass == 0) {
    for (int idx = t; idx < k * k; idx += DD_BLOCK) {
      const int a = idx / k, o = idx % k;
      Ri[(size_t)a * K + o] = Tm[(size_t)a * K + o];
    }
  } else {
    // Ri <- Ri * Tm, row by row (each thread owns whole rows)
    for (int a = t; a < k; a += DD_BLOCK) {
      double2 rowv[DD_MAX_K];
      for (int o = 0; o < k; ++o) {
        double2 s = make_double2(0.0, 0.0);
        for (int l = 0; l < k; ++l) s = dadd(s, dmul(Ri[(size_t)a * K + l], Tm[(size_t)l * K + o]));
        rowv[o] = s;
      }
      for (int o = 0; o < k; ++o) Ri[(size_t)a * K + o] = rowv[o];
    }
  }
  if (t == 0) P.keep[p] = mask;
}

// C_o = sum_{i <= o} T[i][o] W_i in place over the C slots: output groups of
// 16 are formed from the highest down, so a group only overwrites inputs
// that no lower group needs.
template <typename T>
__global__ __launch_bounds__(DD_BLOCK) void k_combine_multi(PlanDev P) {
  const int p = blockIdx.y;
  const ProbDesc d = P.desc[p];
  const int k = d.k;
  if (k == 0) return;
  const int K = P.kmax;
  const unsigned long long mask = P.keep[p];
  c2<T>* W = (c2<T>*)d.basis + (size_t)(K - k) * d.Dp;
  const double2* Tm = P.Tm + (size_t)p * K * K;
  __shared__ c2<T> Tg[DD_MAX_K * 16];
  const int ngroups = (k + 15) / 16;
  for (int g = ngroups - 1; g >= 0; --g) {
    const int o0 = g * 16;
    const int imax = min(k, o0 + 16);
    __syncthreads();
    for (int idx = threadIdx.x; idx < imax * 16; idx += DD_BLOCK) {
      const int i = idx / 16, oo = idx % 16;
      Tg[idx] = (o0 + oo < k) ? to_c<T>(Tm[(size_t)i * K + o0 + oo]) : cmk<c2<T>>(T(0), T(0));
    }
    __syncthreads();
    for (int e = blockIdx.x * DD_BLOCK + threadIdx.x; e < d.Dp; e += gridDim.x * DD_BLOCK) {
      c2<T> acc[16];
#pragma unroll
      for (int oo = 0; oo < 16; ++oo) acc[oo] = cmk<c2<T>>(T(0), T(0));
      for (int i = 0; i < imax; ++i) {
        if (!((mask >> i) & 1ull)) continue;
        const c2<T> x = W[(size_t)i * d.Dp + e];
#pragma unroll
        for (int oo = 0; oo < 16; ++oo) {
          const c2<T> c = Tg[i * 16 + oo];
          acc[oo].x += c.x * x.x - c.y * x.y;
          acc[oo].y += c.x * x.y + c.y * x.x;
        }
      }
#pragma unroll
      for (int oo = 0; oo < 16; ++oo)
        if (o0 + oo < k) W[(size_t)(o0 + oo) * d.Dp + e] = acc[oo];
    }
  }
}
