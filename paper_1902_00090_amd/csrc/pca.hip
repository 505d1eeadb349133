// Principal-component basis of solution snapshots (Sec. 3, PCA paragraph) and
// the batched projection loss (Sec. 3, eq:proj_loss).
//
// The basis is the leading left singular vectors of the snapshot matrix
// X = [s_1 .. s_M] whose columns are field vectors (uncentred).  With the
// snapshots stored as M rows of D elements, G = X^H X (G_ab = <s_a, s_b>) is
// formed on the device with FP64 accumulation; its leading eigenpairs
// (sigma_i^2, w_i) come from a Lanczos iteration with full
// reorthogonalisation on the host (FP64); u_i = X w_i / sigma_i is formed on
// the device and the basis is re-orthonormalised by one Cholesky QR pass.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <random>
#include <vector>

#include "common.h"
#include "devbuf.h"
#include "gram.h"

#define DD_MAX_KPCA 64

using cd = std::complex<double>;

// ------------------------------------------------------------ device Gram ----
// G_ab = sum_e conj(S[a][e]) S[b][e] for a 32 x 32 output tile (only tiles with
// b-block >= a-block), over one slice of the element range (split over
// gridDim.z so that small M still fills the chip).  Elements are staged through
// LDS in steps of 64; each thread owns a 2 x 2 block of the tile, FP64 sums.
#define PT 32
#define PE 64
__global__ __launch_bounds__(256) void k_pca_gram(const float2* __restrict__ S, int M, int D,
                                                  int nslices, double2* __restrict__ part) {
  const int ta = blockIdx.x, tb = blockIdx.y;
  if (tb < ta) return;
  const int slice = blockIdx.z;
  const int per = (D + nslices - 1) / nslices;
  const int e0 = slice * per, e1 = min(D, e0 + per);
  __shared__ float2 sa[PT][PE + 1], sb[PT][PE + 1];
  const int t = threadIdx.x;
  const int ra = (t / 16) * 2, rb = (t % 16) * 2;   // this thread's 2x2 block
  double2 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = make_double2(0.0, 0.0);
  for (int eb = e0; eb < e1; eb += PE) {
    for (int idx = t; idx < PT * PE; idx += 256) {
      const int r = idx / PE, c = idx % PE;
      const int e = eb + c;
      const int a = ta * PT + r, b = tb * PT + r;
      sa[r][c] = (a < M && e < e1) ? S[(size_t)a * D + e] : make_float2(0.f, 0.f);
      sb[r][c] = (b < M && e < e1) ? S[(size_t)b * D + e] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < PE; ++c) {
      float2 xa[2], xb[2];
      xa[0] = sa[ra][c]; xa[1] = sa[ra + 1][c];
      xb[0] = sb[rb][c]; xb[1] = sb[rb + 1][c];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double axr = xa[i].x, axi = xa[i].y, bxr = xb[j].x, bxi = xb[j].y;
          acc[i][j].x += axr * bxr + axi * bxi;
          acc[i][j].y += axr * bxi - axi * bxr;
        }
    }
    __syncthreads();
  }
  const int nta = gridDim.x;
  double2* out = part + ((size_t)slice * nta * nta + (size_t)ta * nta + tb) * PT * PT;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) out[(ra + i) * PT + rb + j] = acc[i][j];
}

// G (M x M, row-major, full Hermitian) from the slice partials, fixed order.
__global__ void k_pca_gram_reduce(const double2* __restrict__ part, int M, int nta, int nslices,
                                  double2* __restrict__ G) {
  const int a = blockIdx.y;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= M || b >= M) return;
  const int lo = min(a, b), hi = max(a, b);
  const int ta = lo / PT, tb = hi / PT;
  // tile (ta, tb) holds G[lo-range][hi-range]; within it row = lo, col = hi
  double sx = 0.0, sy = 0.0;
  for (int s = 0; s < nslices; ++s) {
    const double2 v = part[((size_t)s * nta * nta + (size_t)ta * nta + tb) * PT * PT +
                           (lo % PT) * PT + (hi % PT)];
    sx += v.x;
    sy += v.y;
  }
  // stored value is G[lo][hi]; G[a][b] = that or its conjugate
  G[(size_t)a * M + b] = (a <= b) ? make_double2(sx, sy) : make_double2(sx, -sy);
}

// U[i][e] = sum_m coef[m][i] * S[m][e] for i < k (coef FP64, M x k row-major),
// one thread per element, 16 outputs per pass (grid.y = output group).
__global__ __launch_bounds__(256) void k_pca_combine(const float2* __restrict__ S, int M, int D,
                                                     const double2* __restrict__ coef, int k,
                                                     float2* __restrict__ U) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int o0 = blockIdx.y * 16;
  __shared__ double2 cf[64][16];
  double2 acc[16];
#pragma unroll
  for (int o = 0; o < 16; ++o) acc[o] = make_double2(0.0, 0.0);
  for (int m0 = 0; m0 < M; m0 += 64) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * 16; idx += 256) {
      const int mm = idx / 16, o = idx % 16;
      cf[mm][o] = (m0 + mm < M && o0 + o < k) ? coef[(size_t)(m0 + mm) * k + o0 + o]
                                              : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (e < D) {
      const int mend = min(64, M - m0);
      for (int mm = 0; mm < mend; ++mm) {
        const float2 s = S[(size_t)(m0 + mm) * D + e];
#pragma unroll
        for (int o = 0; o < 16; ++o) {
          const double2 c = cf[mm][o];
          acc[o].x += c.x * s.x - c.y * s.y;
          acc[o].y += c.x * s.y + c.y * s.x;
        }
      }
    }
  }
  if (e < D)
#pragma unroll
    for (int o = 0; o < 16; ++o)
      if (o0 + o < k) U[(size_t)(o0 + o) * D + e] = make_float2((float)acc[o].x, (float)acc[o].y);
}

// ------------------------------------------------------------- host math ----
// Eigen-decomposition of a real symmetric n x n matrix by cyclic Jacobi
// rotations (FP64).  A is overwritten; eigenvalues in w, eigenvectors in the
// columns of V (row-major n x n).
static void jacobi_eigh(std::vector<double>& A, int n, std::vector<double>& w,
                        std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double x = A[(size_t)i * n + j] * A[(size_t)i * n + j];
        tot += x;
        if (i != j) off += x;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {  // A <- A J (columns p, q)
          const double arp = A[(size_t)r * n + p], arq = A[(size_t)r * n + q];
          A[(size_t)r * n + p] = c * arp - s * arq;
          A[(size_t)r * n + q] = s * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {  // A <- J^T A (rows p, q)
          const double apr = A[(size_t)p * n + r], aqr = A[(size_t)q * n + r];
          A[(size_t)p * n + r] = c * apr - s * aqr;
          A[(size_t)q * n + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < n; ++r) {  // V <- V J
          const double vrp = V[(size_t)r * n + p], vrq = V[(size_t)r * n + q];
          V[(size_t)r * n + p] = c * vrp - s * vrq;
          V[(size_t)r * n + q] = s * vrp + c * vrq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

// Leading k eigenpairs of the Hermitian M x M matrix G (row-major) by Lanczos
// with full reorthogonalisation (twice per step), restarted never: the Krylov
// dimension grows until the k leading Ritz pairs have residual
// beta_L |s_L,i| <= 1e-12 theta_max, or L = M.  Returns eigenvalues
// (descending) and eigenvectors (M x k, row-major).
static void lanczos_top(const std::vector<cd>& G, int M, int k, std::vector<double>& theta,
                        std::vector<cd>& W) {
  auto matvec = [&](const std::vector<cd>& x, std::vector<cd>& y) {
    for (int a = 0; a < M; ++a) {
      cd s = 0.0;
      const cd* row = &G[(size_t)a * M];
      for (int b = 0; b < M; ++b) s += row[b] * x[b];
      y[a] = s;
    }
  };
  std::mt19937_64 rng(12345);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<std::vector<cd>> Q;
  std::vector<double> alpha, beta;
  std::vector<cd> q(M), w(M);
  double nq = 0.0;
  for (int i = 0; i < M; ++i) { q[i] = cd(nd(rng), nd(rng)); nq += std::norm(q[i]); }
  nq = std::sqrt(nq);
  for (auto& v : q) v /= nq;
  Q.push_back(q);
  std::vector<double> evals, evecs;
  const int Lmax = M;
  for (int L = 1; L <= Lmax; ++L) {
    matvec(Q[L - 1], w);
    double a = 0.0;
    for (int i = 0; i < M; ++i) a += (std::conj(Q[L - 1][i]) * w[i]).real();
    alpha.push_back(a);
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < L; ++j) {
        cd c = 0.0;
        for (int i = 0; i < M; ++i) c += std::conj(Q[j][i]) * w[i];
        for (int i = 0; i < M; ++i) w[i] -= c * Q[j][i];
      }
    double b = 0.0;
    for (int i = 0; i < M; ++i) b += std::norm(w[i]);
    b = std::sqrt(b);
    const bool full = (L == Lmax);
    const bool check = full || (L >= 2 * k + 10 && (L % 10 == 0)) || b == 0.0;
    if (check) {
      std::vector<double> T((size_t)L * L, 0.0);
      for (int i = 0; i < L; ++i) {
        T[(size_t)i * L + i] = alpha[i];
        if (i + 1 < L) T[(size_t)i * L + i + 1] = T[(size_t)(i + 1) * L + i] = beta[i];
      }
      jacobi_eigh(T, L, evals, evecs);
      std::vector<int> order(L);
      for (int i = 0; i < L; ++i) order[i] = i;
      std::sort(order.begin(), order.end(), [&](int x, int y) { return evals[x] > evals[y]; });
      bool conv = full || b == 0.0;
      if (!conv && L >= k) {
        conv = true;
        const double tmax = std::fabs(evals[order[0]]);
        for (int i = 0; i < k; ++i)
          if (b * std::fabs(evecs[(size_t)(L - 1) * L + order[i]]) > 1e-12 * tmax) conv = false;
      }
      if (conv) {
        const int kk = std::min(k, L);
        theta.assign(k, 0.0);
        W.assign((size_t)M * k, cd(0.0));
        for (int i = 0; i < kk; ++i) {
          theta[i] = evals[order[i]];
          for (int j = 0; j < L; ++j) {
            const double s = evecs[(size_t)j * L + order[i]];
            for (int r = 0; r < M; ++r) W[(size_t)r * k + i] += s * Q[j][r];
          }
        }
        return;
      }
    }
    beta.push_back(b);
    for (int i = 0; i < M; ++i) q[i] = w[i] / b;
    Q.push_back(q);
  }
}

// ------------------------------------------------------------------ API ----
// Small Gram of k device vectors (FP64), host side: used for the final Cholesky
// QR pass and for the projection loss.
__global__ __launch_bounds__(256) void k_small_gram(const float2* __restrict__ V, int k, int D,
                                                    const double2* __restrict__ f, int with_f,
                                                    int nslices, double2* __restrict__ part) {
  // part[slice][(k+1) x (k+1)]: Gram of [V; f] restricted to this slice
  const int a = blockIdx.x, slice = blockIdx.y;
  const int per = (D + nslices - 1) / nslices;
  const int e0 = slice * per, e1 = min(D, e0 + per);
  const int K1 = k + 1;
  __shared__ double lds[8];
  for (int b = a; b < K1; ++b) {
    if (!with_f && (a == k || b == k)) continue;
    double sx = 0.0, sy = 0.0;
    for (int e = e0 + threadIdx.x; e < e1; e += 256) {
      double ax, ay, bx, by;
      if (a < k) { const float2 v = V[(size_t)a * D + e]; ax = v.x; ay = v.y; }
      else { const double2 v = f[e]; ax = v.x; ay = v.y; }
      if (b < k) { const float2 v = V[(size_t)b * D + e]; bx = v.x; by = v.y; }
      else { const double2 v = f[e]; bx = v.x; by = v.y; }
      sx += ax * bx + ay * by;
      sy += ax * by - ay * bx;
    }
    sx = block_sum1<double>(sx, lds);
    sy = block_sum1<double>(sy, lds);
    if (threadIdx.x == 0) part[((size_t)slice * K1 + a) * K1 + b] = make_double2(sx, sy);
  }
}

// C = V T (T upper triangular k x k, FP64), in place, one thread per element.
__global__ __launch_bounds__(256) void k_small_combine(float2* __restrict__ V, int k, int D,
                                                       const double2* __restrict__ T) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= D) return;
  float2 x[DD_MAX_KPCA];
  for (int i = 0; i < k; ++i) x[i] = V[(size_t)i * D + e];
  for (int o = 0; o < k; ++o) {
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i <= o; ++i) {
      const double2 c = T[(size_t)i * k + o];
      sx += c.x * x[i].x - c.y * x[i].y;
      sy += c.x * x[i].y + c.y * x[i].x;
    }
    V[(size_t)o * D + e] = make_float2((float)sx, (float)sy);
  }
}

dd_status gram_host(const float2* V, int k, int D, const double2* f, std::vector<cd>& G,
                    hipStream_t stream) {
  const int K1 = k + 1;
  const int nslices = std::max(1, std::min(256, D / 4096));
  DevBuf bpart;
  DD_HIP_CHECK(hipMalloc(&bpart.p, sizeof(double2) * nslices * K1 * K1));
  double2* part = bpart.as<double2>();
  DD_HIP_CHECK(hipMemsetAsync(part, 0, sizeof(double2) * nslices * K1 * K1, stream));
  k_small_gram<<<dim3(f ? K1 : k, nslices), 256, 0, stream>>>(V, k, D, f, f ? 1 : 0, nslices, part);
  std::vector<double2> hp((size_t)nslices * K1 * K1);
  DD_HIP_CHECK(hipMemcpyAsync(hp.data(), part, sizeof(double2) * hp.size(), hipMemcpyDeviceToHost,
                              stream));
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  G.assign((size_t)K1 * K1, cd(0.0));
  for (int s = 0; s < nslices; ++s)
    for (int a = 0; a < K1; ++a)
      for (int b = a; b < K1; ++b) {
        const double2 v = hp[((size_t)s * K1 + a) * K1 + b];
        G[(size_t)a * K1 + b] += cd(v.x, v.y);
      }
  for (int a = 0; a < K1; ++a)
    for (int b = 0; b < a; ++b) G[(size_t)a * K1 + b] = std::conj(G[(size_t)b * K1 + a]);
  return DD_OK;
}

// G_ab = <F_a, F_b> (S x S, FP64) of S device rows of D complex64 values,
// through the tiled Gram kernel.
static dd_status gram_rows(const float2* F, int S, int D, std::vector<cd>& G, hipStream_t stream) {
  const int nta = (S + PT - 1) / PT;
  const int ntiles = nta * (nta + 1) / 2;
  int nslices = std::max(1, std::min(256, 4096 / std::max(1, ntiles)));
  nslices = std::min(nslices, std::max(1, D / PE));
  DevBuf bpart, bG;
  DD_HIP_CHECK(hipMalloc(&bpart.p, sizeof(double2) * nslices * nta * nta * PT * PT));
  DD_HIP_CHECK(hipMalloc(&bG.p, sizeof(double2) * S * S));
  double2 *part = bpart.as<double2>(), *dG = bG.as<double2>();
  k_pca_gram<<<dim3(nta, nta, nslices), 256, 0, stream>>>(F, S, D, nslices, part);
  k_pca_gram_reduce<<<dim3((S + 255) / 256, S), 256, 0, stream>>>(part, S, nta, nslices, dG);
  DD_HIP_CHECK(hipGetLastError());
  std::vector<double2> h((size_t)S * S);
  DD_HIP_CHECK(hipMemcpyAsync(h.data(), dG, sizeof(double2) * S * S, hipMemcpyDeviceToHost, stream));
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  G.resize((size_t)S * S);
  for (size_t i = 0; i < G.size(); ++i) G[i] = cd(h[i].x, h[i].y);
  return DD_OK;
}

// Cholesky G = L L^H of the leading k x k block (stride ld); returns false if
// not positive definite.  T = L^{-H} (upper triangular, row-major k x k).
bool chol_inv(const std::vector<cd>& G, int ld, int k, std::vector<cd>& L,
              std::vector<cd>& T) {
  L.assign((size_t)k * k, cd(0.0));
  for (int j = 0; j < k; ++j) {
    double d = G[(size_t)j * ld + j].real();
    for (int l = 0; l < j; ++l) d -= std::norm(L[(size_t)j * k + l]);
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    L[(size_t)j * k + j] = ljj;
    for (int i = j + 1; i < k; ++i) {
      cd s = G[(size_t)i * ld + j];
      for (int l = 0; l < j; ++l) s -= L[(size_t)i * k + l] * std::conj(L[(size_t)j * k + l]);
      L[(size_t)i * k + j] = s / ljj;
    }
  }
  T.assign((size_t)k * k, cd(0.0));
  for (int o = 0; o < k; ++o)
    for (int a = o; a >= 0; --a) {
      cd v = (a == o) ? cd(1.0) : cd(0.0);
      for (int l = a + 1; l <= o; ++l) v -= std::conj(L[(size_t)l * k + a]) * T[(size_t)l * k + o];
      T[(size_t)a * k + o] = v / L[(size_t)a * k + a].real();
    }
  return true;
}

extern "C" dd_status pca_build(const void* Sv, int M, int D, int k, void* Uv, double* sigma,
                               hipStream_t stream) {
  if (!Sv || !Uv || M < 1 || D < 1 || k < 1 || k > M || k > DD_MAX_KPCA) {
    dd_set_error("pca_build: need S, U, 1 <= k <= min(M, %d), D >= 1", DD_MAX_KPCA);
    return DD_EINVAL;
  }
  const float2* S = (const float2*)Sv;
  float2* U = (float2*)Uv;
  const int nta = (M + PT - 1) / PT;
  const int ntiles = nta * (nta + 1) / 2;
  int nslices = std::max(1, std::min(256, 4096 / std::max(1, ntiles)));
  nslices = std::min(nslices, std::max(1, D / PE));
  DevBuf bpart, bG, bcoef, bT;
  DD_HIP_CHECK(hipMalloc(&bpart.p, sizeof(double2) * nslices * nta * nta * PT * PT));
  DD_HIP_CHECK(hipMalloc(&bG.p, sizeof(double2) * M * M));
  double2 *part = bpart.as<double2>(), *G = bG.as<double2>();
  k_pca_gram<<<dim3(nta, nta, nslices), 256, 0, stream>>>(S, M, D, nslices, part);
  k_pca_gram_reduce<<<dim3((M + 255) / 256, M), 256, 0, stream>>>(part, M, nta, nslices, G);
  DD_HIP_CHECK(hipGetLastError());
  std::vector<cd> hG((size_t)M * M);
  DD_HIP_CHECK(hipMemcpyAsync(hG.data(), G, sizeof(double2) * M * M, hipMemcpyDeviceToHost, stream));
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  for (const cd& v : hG)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) {
      dd_set_error("pca_build: snapshots contain non-finite values");
      return DD_ENONFINITE;
    }
  // G_ab = <s_a, s_b>; with X = [s_1 .. s_M] (D x M), G = X^H X and the left
  // singular vectors are u_i = X w_i / sigma_i for X^H X w_i = sigma_i^2 w_i.
  std::vector<double> theta;
  std::vector<cd> W;
  lanczos_top(hG, M, k, theta, W);
  std::vector<double2> hc((size_t)M * k);
  for (int i = 0; i < k; ++i) {
    const double s = std::sqrt(std::max(theta[i], 0.0));
    if (!(s > 0.0)) {
      dd_set_error("pca_build: snapshot matrix has rank < k");
      return DD_EINVAL;
    }
    if (sigma) sigma[i] = s;
    for (int mrow = 0; mrow < M; ++mrow) {
      const cd c = W[(size_t)mrow * k + i] / s;
      hc[(size_t)mrow * k + i] = make_double2(c.real(), c.imag());
    }
  }
  DD_HIP_CHECK(hipMalloc(&bcoef.p, sizeof(double2) * M * k));
  double2* coef = bcoef.as<double2>();
  DD_HIP_CHECK(hipMemcpyAsync(coef, hc.data(), sizeof(double2) * M * k, hipMemcpyHostToDevice, stream));
  k_pca_combine<<<dim3((D + 255) / 256, (k + 15) / 16), 256, 0, stream>>>(S, M, D, coef, k, U);
  DD_HIP_CHECK(hipGetLastError());
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  // one Cholesky QR pass restores orthonormality lost to FP32 storage
  std::vector<cd> Gu, L, T;
  dd_status rc = gram_host(U, k, D, nullptr, Gu, stream);
  if (rc != DD_OK) return rc;
  if (!chol_inv(Gu, k + 1, k, L, T)) {
    dd_set_error("pca_build: basis Gram matrix not positive definite");
    return DD_EINVAL;
  }
  std::vector<double2> hT((size_t)k * k);
  for (size_t i = 0; i < hT.size(); ++i) hT[i] = make_double2(T[i].real(), T[i].imag());
  DD_HIP_CHECK(hipMalloc(&bT.p, sizeof(double2) * k * k));
  double2* dT = bT.as<double2>();
  DD_HIP_CHECK(hipMemcpyAsync(dT, hT.data(), sizeof(double2) * k * k, hipMemcpyHostToDevice, stream));
  k_small_combine<<<(D + 255) / 256, 256, 0, stream>>>(U, k, D, dT);
  DD_HIP_CHECK(hipGetLastError());
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  return DD_OK;
}

// T[s][j] = sum_m coef[s][m][j] F[m] for the S steps of one trajectory:
// coef is [S][S][k] (FP64, zero outside each step's window), one thread per
// element, grid.y = (step, group of 16 outputs).
__global__ __launch_bounds__(256) void k_local_combine(const float2* __restrict__ F, int S, int D,
                                                       const double2* __restrict__ coef, int k,
                                                       float2* __restrict__ T) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y / ((k + 15) / 16), o0 = (blockIdx.y % ((k + 15) / 16)) * 16;
  if (e >= D) return;
  double2 acc[16];
#pragma unroll
  for (int o = 0; o < 16; ++o) acc[o] = make_double2(0.0, 0.0);
  for (int m = 0; m < S; ++m) {
    const float2 f = F[(size_t)m * D + e];
#pragma unroll
    for (int o = 0; o < 16; ++o) {
      if (o0 + o < k) {
        const double2 c = coef[((size_t)s * S + m) * k + o0 + o];
        acc[o].x += c.x * f.x - c.y * f.y;
        acc[o].y += c.x * f.y + c.y * f.x;
      }
    }
  }
  for (int o = 0; o < 16 && o0 + o < k; ++o)
    T[((size_t)s * k + o0 + o) * D + e] = make_float2((float)acc[o].x, (float)acc[o].y);
}

// Training targets of the convolutional predictor from one trajectory's
// solution fields: for step s, U_loc = the leading k left singular vectors
// of the (unit-normalised) fields of steps s-window..s+window, and target j
// = u_j (u_j^H f_s).  With the window's Gram matrix G (from the trajectory
// Gram matrix) = W diag(sigma^2) W^H, u_j = sum_m W_mj f_m / sigma_j and
// u_j^H f_s = sum_m conj(W_mj) G_ms / sigma_j, so every target is a combination
// of the trajectory's fields with coefficients from a small host problem.
extern "C" dd_status local_pca_targets(const void* Fv, int S, int D, int window, int k,
                                       void* Tv, hipStream_t stream) {
  if (!Fv || !Tv || S < 1 || D < 1 || k < 1 || window < 0 || k > DD_MAX_KPCA) {
    dd_set_error("local_pca_targets: bad argument");
    return DD_EINVAL;
  }
  const float2* F = (const float2*)Fv;
  // trajectory Gram matrix of the normalised fields (normalisation applied here)
  std::vector<cd> G0;
  dd_status rc = gram_rows(F, S, D, G0, stream);
  if (rc != DD_OK) return rc;
  std::vector<double> nrm(S);
  for (int a = 0; a < S; ++a) nrm[a] = std::sqrt(std::max(G0[(size_t)a * S + a].real(), 1e-300));
  std::vector<double2> hc((size_t)S * S * k, make_double2(0.0, 0.0));
  for (int s = 0; s < S; ++s) {
    const int lo = std::max(0, s - window), hi = std::min(S, s + window + 1), M = hi - lo;
    std::vector<cd> G((size_t)M * M);
    for (int a = 0; a < M; ++a)
      for (int b = 0; b < M; ++b)
        G[(size_t)a * M + b] = G0[(size_t)(lo + a) * S + lo + b] / (nrm[lo + a] * nrm[lo + b]);
    const int kk = std::min(k, M);
    std::vector<double> theta;
    std::vector<cd> W;
    lanczos_top(G, M, kk, theta, W);
    for (int j = 0; j < kk; ++j) {
      if (!(theta[j] > 1e-24 * std::max(theta[0], 1e-300))) continue;
      const double sg = std::sqrt(theta[j]);
      cd c = 0.0;  // u_j^H f_s (f_s normalised)
      for (int m = 0; m < M; ++m) c += std::conj(W[(size_t)m * kk + j]) * G[(size_t)m * M + (s - lo)];
      c /= sg;
      for (int m = 0; m < M; ++m) {
        // target_j = sum_m (W_mj / sigma_j) c f_m / ||f_m||  (fields normalised)
        const cd v = W[(size_t)m * kk + j] / sg * c / nrm[lo + m];
        hc[((size_t)s * S + lo + m) * k + j] = make_double2(v.real(), v.imag());
      }
    }
  }
  DevBuf bcoef;
  DD_HIP_CHECK(hipMalloc(&bcoef.p, sizeof(double2) * hc.size()));
  double2* coef = bcoef.as<double2>();
  DD_HIP_CHECK(hipMemcpyAsync(coef, hc.data(), sizeof(double2) * hc.size(), hipMemcpyHostToDevice, stream));
  k_local_combine<<<dim3((D + 255) / 256, S * ((k + 15) / 16)), 256, 0, stream>>>(F, S, D, coef, k,
                                                                                  (float2*)Tv);
  DD_HIP_CHECK(hipGetLastError());
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  return DD_OK;
}

extern "C" dd_status proj_loss_batched(const void* Vv, const void* fv, int nb, int k, int D,
                                       double* out, hipStream_t stream) {
  if (!Vv || !fv || !out || nb < 1 || k < 1 || k > DD_MAX_KPCA || D < 1) {
    dd_set_error("proj_loss_batched: bad argument");
    return DD_EINVAL;
  }
  for (int p = 0; p < nb; ++p) {
    const float2* V = (const float2*)Vv + (size_t)p * k * D;
    const double2* f = (const double2*)fv + (size_t)p * D;
    std::vector<cd> G, L, T;
    dd_status rc = gram_host(V, k, D, f, G, stream);
    if (rc != DD_OK) return rc;
    const int K1 = k + 1;
    const double ff = G[(size_t)k * K1 + k].real();
    // l = 1 - c^H G_VV^{-1} c / ||f||^2 with c = V^H f; G_VV^{-1} = T T^H
    if (!(ff > 0.0)) { out[p] = 0.0; continue; }
    if (!chol_inv(G, K1, k, L, T)) {
      dd_set_error("proj_loss_batched: V of problem %d is rank deficient", p);
      return DD_EINVAL;
    }
    double q = 0.0;
    for (int o = 0; o < k; ++o) {
      cd s = 0.0;  // (T^H c)_o = sum_a conj(T[a][o]) c_a
      for (int a = 0; a <= o; ++a) s += std::conj(T[(size_t)a * k + o]) * G[(size_t)a * K1 + k];
      q += std::norm(s);
    }
    // the loss lies in [0, 1] by definition; rounding can step outside by ~1e-16
    out[p] = std::min(1.0, std::max(0.0, 1.0 - q / ff));
  }
  return DD_OK;
}
