// Subspace recycling along a sequence of related systems (Sec. 1: Krylov
// information carried from earlier solves of related systems into the next;
// supplement Sec. 1: GCROT keeps a few correction directions from one cycle
// to the next).  After a solve, the search space of each problem's last
// cycle, S = [U, Q_n] with U = V R^{-1} (A U = C), is compressed to its
// harmonic Ritz vectors of smallest magnitude, which then augment the next
// system of the sequence.
//
// With W = [C, Q_{n+1}] (orthonormal), A S = W G where
// G = [[I, B], [0, H]] is the matrix of eq:final_lsq, and a harmonic Ritz
// pair (theta, S u) solves G^H G u = theta G^H (W^H S) u.  The device forms
// the dots W^H V over the field (the only part that touches the vectors);
// the host solves the small eigenproblem (dense_small.h) per problem; the
// device forms Y = S Z = V (R^{-1} Z_U) + Q_n Z_Q.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "dense_small.h"
#include "solver_state.h"

// X[p][a][i] = W_a^H V_i in FP64, a < k + nq[p], i < k, in 4 x 4 tiles
// (one workgroup per tile pair and problem, over the whole field).  W_a is
// the C slot a for a < k and the Krylov vector q_{a-k} otherwise, scaled here
// by hscale where it is stored unnormalised.
template <typename T>
__global__ __launch_bounds__(DD_BLOCK) void k_recycle_dots(PlanDev P, const int* __restrict__ nq,
                                                           double2* __restrict__ X, int rows) {
  const int p = blockIdx.y;
  const ProbDesc d = P.desc[p];
  const int k = d.k, nw = k + nq[p];
  if (k == 0 || nw == 0) return;
  const int nvt = (k + 3) / 4, nwt = (nw + 3) / 4;
  if ((int)blockIdx.x >= nvt * nwt) return;
  const int tw = blockIdx.x / nvt, tv = blockIdx.x % nvt;
  const c2<T>* basis = (const c2<T>*)d.basis;
  const c2<T>* Vb = (const c2<T>*)d.V;
  const c2<T>* wp[4];
  double ws[4];
  const c2<T>* vp[4];
  for (int q = 0; q < 4; ++q) {
    const int a = 4 * tw + q, i = 4 * tv + q;
    wp[q] = nullptr;
    ws[q] = 1.0;
    if (a < k) {
      wp[q] = basis + (size_t)(P.kmax - k + a) * d.Dp;
    } else if (a < nw) {
      wp[q] = basis + (size_t)(P.kmax + a - k) * d.Dp;
      // stored unnormalised: the last vector always, every vector on the
      // one-sweep path (q_i = s_i q~_i)
      if (a - k == nq[p] - 1 || P.fused) ws[q] = P.hscale[(size_t)p * (P.m + 1) + (a - k)];
    }
    vp[q] = (i < k) ? Vb + (size_t)i * d.Dp : nullptr;
  }
  double acc[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) acc[i] = 0.0;
  for (int e = threadIdx.x; e < d.D; e += DD_BLOCK) {
    double2 a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const c2<T> x = wp[q] ? wp[q][e] : cmk<c2<T>>(T(0), T(0));
      const c2<T> y = vp[q] ? vp[q][e] : cmk<c2<T>>(T(0), T(0));
      a[q] = make_double2((double)x.x * ws[q], (double)x.y * ws[q]);
      b[q] = make_double2((double)y.x, (double)y.y);
    }
#pragma unroll
    for (int qa = 0; qa < 4; ++qa)
#pragma unroll
      for (int qb = 0; qb < 4; ++qb) {
        acc[2 * (qa * 4 + qb)] += a[qa].x * b[qb].x + a[qa].y * b[qb].y;
        acc[2 * (qa * 4 + qb) + 1] += a[qa].x * b[qb].y - a[qa].y * b[qb].x;
      }
  }
  __shared__ double lds[128];
  __shared__ double out[32];
  block_sum32<double>(acc, lds, out);
  if (threadIdx.x < 16) {
    const int qa = threadIdx.x >> 2, qb = threadIdx.x & 3;
    const int a = 4 * tw + qa, i = 4 * tv + qb;
    if (a < nw && i < k)
      X[((size_t)p * rows + a) * P.kmax + i] = make_double2(out[2 * threadIdx.x], out[2 * threadIdx.x + 1]);
  }
}

// Y[p][o] = sum_i V_i cf[p][o][i] + sum_j q_j cf[p][o][k + j] for o < kout[p]
// (16 outputs per workgroup row of the grid; coefficients in FP64, read
// uniformly by all threads).
template <typename T>
__global__ __launch_bounds__(DD_BLOCK) void k_recycle_combine(PlanDev P, const int* __restrict__ kout,
                                                              const int* __restrict__ nqc,
                                                              const double2* __restrict__ cf, int ldc,
                                                              int kr, void* const* Y) {
  const int p = blockIdx.z, o0 = 16 * blockIdx.y;
  const int ko = kout[p];
  if (o0 >= ko) return;
  const ProbDesc d = P.desc[p];
  const int k = d.k, n = nqc[p];
  const c2<T>* basis = (const c2<T>*)d.basis;
  const c2<T>* Vb = (const c2<T>*)d.V;
  c2<T>* y = (c2<T>*)Y[p];
  const double2* c = cf + (size_t)p * kr * ldc;
  const int no = min(16, ko - o0);
  for (int e = blockIdx.x * DD_BLOCK + threadIdx.x; e < d.D; e += gridDim.x * DD_BLOCK) {
    double2 acc[16];
#pragma unroll
    for (int oo = 0; oo < 16; ++oo) acc[oo] = make_double2(0.0, 0.0);
    for (int v = 0; v < k + n; ++v) {
      const c2<T> x = (v < k) ? Vb[(size_t)v * d.Dp + e] : basis[(size_t)(P.kmax + v - k) * d.Dp + e];
      const double xr = (double)x.x, xi = (double)x.y;
#pragma unroll
      for (int oo = 0; oo < 16; ++oo) {
        if (oo < no) {
          const double2 cc = c[(size_t)(o0 + oo) * ldc + v];
          acc[oo].x += cc.x * xr - cc.y * xi;
          acc[oo].y += cc.x * xi + cc.y * xr;
        }
      }
    }
#pragma unroll
    for (int oo = 0; oo < 16; ++oo)
      if (oo < no) y[(size_t)(o0 + oo) * d.D + e] = cmk<c2<T>>((T)acc[oo].x, (T)acc[oo].y);
  }
}

namespace {

using dd_small::cd;

struct ProbIn {
  int k = 0, n = 0;                 // augmenting columns, Krylov steps of the last cycle
  std::vector<int> kept;            // kept augmenting columns
};

// The small problem of one problem p; fills cf ([kr][ldc] complex, first k
// entries over the V slots, then n over q_0..q_{n-1}), theta and kout.
bool small_problem(const ProbIn& in, int K, int m, int rows, int kr, const double2* X,
                   const double2* Hraw, const double2* Bc, const double2* Ri, const double* hs,
                   bool fused, int ldc, double2* cf, double* theta, int& kout) {
  const int kk = (int)in.kept.size(), n = in.n, k = in.k;
  const int ns = kk + n, nw = kk + (n > 0 ? n + 1 : 0);
  kout = std::min(kr, ns);
  if (kout == 0) return true;
  // G = [[I, B], [0, H]] on the kept columns
  std::vector<cd> G((size_t)nw * ns, cd(0.0, 0.0)), M((size_t)nw * ns, cd(0.0, 0.0));
  for (int r = 0; r < kk; ++r) G[(size_t)r * ns + r] = 1.0;
  for (int j = 0; j < n; ++j) {
    for (int r = 0; r < kk; ++r) {
      const double2 b = Bc[(size_t)j * K + in.kept[r]];
      G[(size_t)r * ns + kk + j] = cd(b.x, b.y);
    }
    for (int i = 0; i <= j + 1; ++i) {
      const double2 h = Hraw[(size_t)j * (m + 1) + i];
      G[(size_t)(kk + i) * ns + kk + j] = cd(h.x, h.y);
    }
  }
  // M = W^H S: W^H U = (W^H V) R^{-1} on the kept columns; C^H Q = 0; Q^H Q = I
  auto xrow = [&](int r) { return (r < kk) ? in.kept[r] : k + (r - kk); };
  for (int r = 0; r < nw; ++r) {
    const double2* xr = X + (size_t)xrow(r) * K;
    for (int c = 0; c < kk; ++c) {
      cd s = 0.0;
      for (int i = 0; i < k; ++i) {
        const double2 ri = Ri[(size_t)i * K + in.kept[c]];
        s += cd(xr[i].x, xr[i].y) * cd(ri.x, ri.y);
      }
      M[(size_t)r * ns + c] = s;
    }
    if (r >= kk && r - kk < n) M[(size_t)r * ns + r] = 1.0;
  }
  std::vector<cd> Z, th;
  if (!dd_small::harmonic_ritz(ns, nw, G, M, kout, Z, th)) return false;
  for (int o = 0; o < kout; ++o) {
    double2* co = cf + (size_t)o * ldc;
    for (int i = 0; i < k; ++i) {
      cd s = 0.0;
      for (int c = 0; c < kk; ++c) {
        const double2 ri = Ri[(size_t)i * K + in.kept[c]];
        s += cd(ri.x, ri.y) * Z[(size_t)c * kout + o];
      }
      co[i] = make_double2(s.real(), s.imag());
    }
    for (int j = 0; j < n; ++j) {
      // the combination reads the stored vectors: q~_j = q_j / s_j on the
      // one-sweep path
      const cd z = Z[(size_t)(kk + j) * kout + o] * (fused ? hs[j] : 1.0);
      co[k + j] = make_double2(z.real(), z.imag());
    }
    theta[2 * o] = th[o].real();
    theta[2 * o + 1] = th[o].imag();
  }
  (void)rows;
  return true;
}

template <typename T>
void launch_recycle_dots(dd_solver* s, const int* nq, double2* X, int rows, int grid_x,
                         hipStream_t st) {
  k_recycle_dots<T><<<dim3(grid_x, s->nb), DD_BLOCK, 0, st>>>(s->P, nq, X, rows);
}

template <typename T>
void launch_recycle_combine(dd_solver* s, const int* kout, const int* nqc, const double2* cf,
                            int ldc, int kr, void* const* Y, hipStream_t st) {
  int maxD = 0;
  for (auto& d : s->hdesc) maxD = std::max(maxD, d.D);
  const int gx = std::min(256, (maxD + DD_BLOCK - 1) / DD_BLOCK);
  k_recycle_combine<T><<<dim3(gx, (kr + 15) / 16, s->nb), DD_BLOCK, 0, st>>>(s->P, kout, nqc, cf,
                                                                               ldc, kr, Y);
}

}  // namespace

extern "C" dd_status dd_solver_recycle(dd_solver* s, int kr, void* const* Y, int* kout,
                                       double* theta, hipStream_t stream) {
  if (!s || !Y || !kout) { dd_set_error("dd_solver_recycle: NULL argument"); return DD_EINVAL; }
  if (kr < 1 || kr > DD_MAX_K) {
    dd_set_error("dd_solver_recycle: kr = %d outside 1..%d", kr, DD_MAX_K);
    return DD_EINVAL;
  }
  if (s->o.precond != DD_PRECOND_NONE) {
    dd_set_error("dd_solver_recycle: not available with a preconditioner");
    return DD_EINVAL;
  }
  if (!s->cycle_valid) {
    dd_set_error("dd_solver_recycle: no solve since the last set_subspace or autotune");
    return DD_EINVAL;
  }
  const int nb = s->nb, K = s->o.kmax, m = s->o.restart;
  for (int p = 0; p < nb; ++p)
    if (!Y[p]) { dd_set_error("dd_solver_recycle: Y[%d] is NULL", p); return DD_EINVAL; }
  // small matrices of the last cycle
  std::vector<int> stI((size_t)nb * ST_NI);
  std::vector<unsigned long long> keep(nb);
  std::vector<double> hs((size_t)nb * (m + 1));
  std::vector<double2> Hraw((size_t)nb * m * (m + 1)), Bc((size_t)nb * m * K), Ri((size_t)nb * K * K);
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  DD_HIP_CHECK(hipMemcpy(stI.data(), s->P.stI, sizeof(int) * stI.size(), hipMemcpyDeviceToHost));
  DD_HIP_CHECK(hipMemcpy(keep.data(), s->P.keep, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost));
  DD_HIP_CHECK(hipMemcpy(hs.data(), s->P.hscale, sizeof(double) * hs.size(), hipMemcpyDeviceToHost));
  DD_HIP_CHECK(hipMemcpy(Hraw.data(), s->P.Hraw, sizeof(double2) * Hraw.size(), hipMemcpyDeviceToHost));
  if (K > 0) {
    DD_HIP_CHECK(hipMemcpy(Bc.data(), s->P.Bc, sizeof(double2) * Bc.size(), hipMemcpyDeviceToHost));
    DD_HIP_CHECK(hipMemcpy(Ri.data(), s->P.Rinv, sizeof(double2) * Ri.size(), hipMemcpyDeviceToHost));
  }
  std::vector<ProbIn> in(nb);
  std::vector<int> nq(nb, 0), nqc(nb, 0);
  int maxtiles = 0;
  const int rows = K + m + 1;
  for (int p = 0; p < nb; ++p) {
    ProbIn& q = in[p];
    q.k = s->hdesc[p].k;
    q.n = std::max(0, std::min(m, stI[(size_t)p * ST_NI + ST_NCOMB]));
    for (int i = 0; i < q.k; ++i)
      if ((keep[p] >> i) & 1ull) q.kept.push_back(i);
    nq[p] = q.n > 0 ? q.n + 1 : 0;
    nqc[p] = q.n;
    maxtiles = std::max(maxtiles, ((q.k + 3) / 4) * ((q.k + nq[p] + 3) / 4));
  }
  // device scratch: X [nb][rows][K], cf [nb][kr][ldc], nq, nqc, kout
  const int ldc = K + m;
  const size_t xbytes = sizeof(double2) * (size_t)nb * rows * std::max(K, 1);
  const size_t cbytes = sizeof(double2) * (size_t)nb * kr * ldc;
  const size_t ibytes = sizeof(int) * (size_t)nb;
  char* scratch = nullptr;
  DD_HIP_CHECK(hipMalloc(&scratch, xbytes + cbytes + 3 * ibytes + 3 * 256));
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  double2* dX = (double2*)scratch;
  double2* dcf = (double2*)(scratch + align(xbytes));
  int* dnq = (int*)(scratch + align(xbytes) + align(cbytes));
  int* dnqc = dnq + nb;
  int* dkout = dnqc + nb;
  auto fail = [&](dd_status rc) { (void)hipFree(scratch); return rc; };
  std::vector<double2> X(xbytes / sizeof(double2));
  if (hipMemcpyAsync(dnq, nq.data(), ibytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(dnqc, nqc.data(), ibytes, hipMemcpyHostToDevice, stream) != hipSuccess) {
    dd_set_error("dd_solver_recycle: copy failed");
    return fail(DD_EHIP);
  }
  if (maxtiles > 0) {
    if (s->o.inner == DD_C64) launch_recycle_dots<float>(s, dnq, dX, rows, maxtiles, stream);
    else launch_recycle_dots<double>(s, dnq, dX, rows, maxtiles, stream);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(X.data(), dX, xbytes, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      dd_set_error("dd_solver_recycle: dot kernel failed");
      return fail(DD_EHIP);
    }
  }
  // the small problems, spread over host threads
  std::vector<double2> cf((size_t)nb * kr * ldc, make_double2(0.0, 0.0));
  std::vector<double> th((size_t)nb * kr * 2, 0.0);
  std::vector<int> ko(nb, 0);
  std::vector<char> ok(nb, 1);
  const int nthr = std::max(1, std::min<int>(nb, (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
  auto work = [&](int t0) {
    for (int p = t0; p < nb; p += nthr)
      ok[p] = small_problem(in[p], K, m, rows, kr, X.data() + (size_t)p * rows * std::max(K, 1),
                            Hraw.data() + (size_t)p * m * (m + 1), Bc.data() + (size_t)p * m * K,
                            Ri.data() + (size_t)p * K * K, hs.data() + (size_t)p * (m + 1),
                            s->fused, ldc, cf.data() + (size_t)p * kr * ldc,
                            th.data() + (size_t)p * kr * 2, ko[p]);
  };
  if (nthr == 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < nthr; ++t) pool.emplace_back(work, t);
    for (auto& t : pool) t.join();
  }
  for (int p = 0; p < nb; ++p)
    if (!ok[p]) {
      dd_set_error("dd_solver_recycle: the small eigenproblem of problem %d failed", p);
      return fail(DD_ENONFINITE);
    }
  if (hipMemcpyAsync(dcf, cf.data(), cbytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(dkout, ko.data(), ibytes, hipMemcpyHostToDevice, stream) != hipSuccess) {
    dd_set_error("dd_solver_recycle: copy failed");
    return fail(DD_EHIP);
  }
  void** dY = nullptr;
  if (hipMalloc(&dY, sizeof(void*) * nb) != hipSuccess) {
    dd_set_error("dd_solver_recycle: allocation failed");
    return fail(DD_ENOMEM);
  }
  bool good = hipMemcpyAsync(dY, Y, sizeof(void*) * nb, hipMemcpyHostToDevice, stream) == hipSuccess;
  if (good) {
    if (s->o.inner == DD_C64) launch_recycle_combine<float>(s, dkout, dnqc, dcf, ldc, kr, dY, stream);
    else launch_recycle_combine<double>(s, dkout, dnqc, dcf, ldc, kr, dY, stream);
    good = hipGetLastError() == hipSuccess && hipStreamSynchronize(stream) == hipSuccess;
  }
  (void)hipFree(dY);
  if (!good) {
    dd_set_error("dd_solver_recycle: combine kernel failed");
    return fail(DD_EHIP);
  }
  (void)hipFree(scratch);
  for (int p = 0; p < nb; ++p) {
    kout[p] = ko[p];
    if (theta)
      for (int o = 0; o < kr; ++o) {
        theta[((size_t)p * kr + o) * 2] = (o < ko[p]) ? th[((size_t)p * kr + o) * 2] : 0.0;
        theta[((size_t)p * kr + o) * 2 + 1] = (o < ko[p]) ? th[((size_t)p * kr + o) * 2 + 1] : 0.0;
      }
  }
  return DD_OK;
}

extern "C" dd_status dd_harmonic_ritz_host(int ns, int nw, const double* G, const double* M, int kr,
                                           double* Z, double* theta) {
  if (ns < 1 || nw < ns || kr < 1 || kr > ns || !G || !M || !Z || !theta) {
    dd_set_error("dd_harmonic_ritz_host: need 1 <= kr <= ns <= nw and non-NULL arrays");
    return DD_EINVAL;
  }
  std::vector<cd> Gv((size_t)nw * ns), Mv((size_t)nw * ns), Zv, th;
  for (size_t i = 0; i < Gv.size(); ++i) {
    Gv[i] = cd(G[2 * i], G[2 * i + 1]);
    Mv[i] = cd(M[2 * i], M[2 * i + 1]);
  }
  if (!dd_small::harmonic_ritz(ns, nw, Gv, Mv, kr, Zv, th)) {
    dd_set_error("dd_harmonic_ritz_host: rank-deficient G or no Schur convergence");
    return DD_ENONFINITE;
  }
  for (size_t i = 0; i < Zv.size(); ++i) { Z[2 * i] = Zv[i].real(); Z[2 * i + 1] = Zv[i].imag(); }
  for (int o = 0; o < kr; ++o) { theta[2 * o] = th[o].real(); theta[2 * o + 1] = th[o].imag(); }
  return DD_OK;
}
