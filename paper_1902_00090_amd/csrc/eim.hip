// Effective-index approximation of the field: the CNN's second input.
//
// The paper feeds its CNN an effective-index simulation of the field next to
// the permittivity (Sec. 3, data-set and CNN paragraphs).  It describes this
// only as a cheap 1D solve of Maxwell's equations.  The separable reading
// used here has three steps.
//
//  1. Every column ix is a 1D slab.  Its fundamental mode phi_ix is the
//     eigenvector of the lowest eigenvalue mu_ix of
//         T = -(second difference in y)/dx^2 - omega^2 eps(ix, .),
//     with zero field outside the column.  phi_ix has unit norm and is
//     positive.
//  2. The amplitude a along x solves the 1D FDFD equation.  It uses the 2D
//     operator's stretched x-differences (periodic wrap) with mu in place of
//     -omega^2 eps:
//         cxm_i (a_i - a_{i-1}) - cxp_i (a_{i+1} - a_i) + mu_i a_i = j_i,
//     where j_i = phi_i^T b[:, i].
//  3. F[iy, ix] = a_ix phi_ix(iy).
//
// The kernels, all in FP64:
//  * k_eim_modes: one thread per column.  Sturm-count bisection for the
//    lowest eigenvalue, then inverse iteration from just below it.  The
//    shifted matrix is then symmetric positive definite with non-positive
//    off-diagonals, so its LDL^T sweep needs no pivoting and keeps the
//    iterate positive.
//  * k_eim_line: one thread per problem.  The cyclic complex tridiagonal
//    system is solved by Sherman-Morrison over a tridiagonal elimination with
//    partial pivoting.  The matrix is indefinite, so pivoting is needed.
//  * k_eim_assemble: writes F in complex64.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"
#include "eim.h"
#include "op.h"

#define DD_EIM_MAX_DEVICES 64

namespace {

struct EimDesc {
  int nx, ny;
  double omega, dx;
  const double* eps;   // [ny][nx]
  const double2* cf;   // cxm [0, nx), cxp [nx, 2nx)
  const double2* b;    // [D] right-hand side
  float2* F;           // [D] output
  size_t off2;         // offset in the D-sized scratch arrays
  size_t off1;         // offset in the nx-sized scratch arrays
};

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double zabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  const double s = 1.0 / zabs2(b);
  return make_double2((a.x * b.x + a.y * b.y) * s, (a.y * b.x - a.x * b.y) * s);
}

// ------------------------------------------------ column modes (step 1) ----
__global__ __launch_bounds__(64) void k_eim_modes(const EimDesc* __restrict__ desc,
                                                  double* __restrict__ phi,
                                                  double* __restrict__ piv,
                                                  double* __restrict__ mu,
                                                  double2* __restrict__ jp) {
  const EimDesc d = desc[blockIdx.y];
  const int ix = blockIdx.x * 64 + threadIdx.x;
  if (ix >= d.nx) return;
  const int nx = d.nx, ny = d.ny;
  const double h2 = 1.0 / (d.dx * d.dx), w2 = d.omega * d.omega, e2 = h2 * h2;
  const double* eps = d.eps + ix;
  double* ph = phi + d.off2 + ix;
  double* pv = piv + d.off2 + ix;
  auto diag = [&](int i) { return 2.0 * h2 - w2 * eps[(size_t)i * nx]; };

  // Gershgorin: the lowest eigenvalue lies in [min diag - 2 h2, min diag]
  double dmin = diag(0), amax = fabs(dmin);
  for (int i = 1; i < ny; ++i) {
    const double t = diag(i);
    dmin = fmin(dmin, t);
    amax = fmax(amax, fabs(t));
  }
  const double pivmin = 1e-290 * fmax(1.0, e2);
  double lo = dmin - 2.0 * h2, hi = dmin;
  for (int it = 0; it < 52; ++it) {
    const double x = 0.5 * (lo + hi);
    // Sturm count: eigenvalues of T below x = negative pivots of T - x I
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < ny; ++i) {
      q = diag(i) - x - (i > 0 ? e2 / q : 0.0);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += (q < 0.0);
    }
    if (cnt >= 1) hi = x; else lo = x;
  }

  // inverse iteration with the shift just below the eigenvalue
  const double sigma = lo - 1e-10 * (amax + 2.0 * h2);
  for (int i = 0; i < ny; ++i) ph[(size_t)i * nx] = 1.0;
  for (int it = 0; it < 4; ++it) {
    double p = diag(0) - sigma, z = ph[0];
    pv[0] = p;
    for (int i = 1; i < ny; ++i) {
      const double l = -h2 / p;              // L factor: off-diagonal / previous pivot
      p = diag(i) - sigma + h2 * l;           // a_i - sigma - e * l
      z = ph[(size_t)i * nx] - l * z;
      pv[(size_t)i * nx] = p;
      ph[(size_t)i * nx] = z;
    }
    double x = ph[(size_t)(ny - 1) * nx] / pv[(size_t)(ny - 1) * nx];
    ph[(size_t)(ny - 1) * nx] = x;
    double ss = x * x;
    for (int i = ny - 2; i >= 0; --i) {
      x = (ph[(size_t)i * nx] + h2 * x) / pv[(size_t)i * nx];
      ph[(size_t)i * nx] = x;
      ss += x * x;
    }
    const double inv = 1.0 / sqrt(ss);
    for (int i = 0; i < ny; ++i) ph[(size_t)i * nx] *= inv;
  }
  // sign (positive), Rayleigh quotient and projection of the source column
  double sum = 0.0;
  for (int i = 0; i < ny; ++i) sum += ph[(size_t)i * nx];
  const double sg = (sum < 0.0) ? -1.0 : 1.0;
  double rq = 0.0, prev = 0.0;
  double2 jj = make_double2(0.0, 0.0);
  const double2* bc = d.b + ix;
  for (int i = 0; i < ny; ++i) {
    const double v = sg * ph[(size_t)i * nx];
    const double next = (i + 1 < ny) ? sg * ph[(size_t)(i + 1) * nx] : 0.0;
    rq += v * (diag(i) * v - h2 * (prev + next));
    const double2 bv = bc[(size_t)i * nx];
    jj.x += v * bv.x;
    jj.y += v * bv.y;
    ph[(size_t)i * nx] = v;
    prev = v;
  }
  mu[d.off1 + ix] = rq;
  jp[d.off1 + ix] = jj;
}

// ----------------------------------------- 1D solve along x (step 2) ------
// Row i of the cyclic system: lower -cxm_i (column i-1), diagonal
// cxm_i + cxp_i + mu_i, upper -cxp_i (column i+1); row 0's lower coefficient
// beta sits in column n-1 and row n-1's upper coefficient alpha in column 0.
// With gamma = -diag_0, M = T + u v^T where T is M without the corners and
// with diag_0 - gamma, diag_{n-1} - alpha beta / gamma, u = (gamma, 0.., alpha)
// and v = (1, 0.., beta / gamma).  Then a = y - (v.y / (1 + v.z)) z with
// T y = j and T z = u.
__global__ __launch_bounds__(64) void k_eim_line(const EimDesc* __restrict__ desc, int nb,
                                                 const double* __restrict__ mu,
                                                 const double2* __restrict__ jp,
                                                 double2* __restrict__ dg, double2* __restrict__ du,
                                                 double2* __restrict__ du2,
                                                 double2* __restrict__ r1,
                                                 double2* __restrict__ r2,
                                                 double2* __restrict__ amp) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p >= nb) return;
  const EimDesc d = desc[p];
  const int n = d.nx;
  const size_t o = d.off1;
  const double2* cxm = d.cf;
  const double2* cxp = d.cf + n;
  auto neg = [](double2 a) { return make_double2(-a.x, -a.y); };
  const double2 beta = neg(cxm[0]), alpha = neg(cxp[n - 1]);
  const double2 diag0 = make_double2(cxm[0].x + cxp[0].x + mu[o], cxm[0].y + cxp[0].y);
  const double2 gamma = neg(diag0);
  const double2 bg = zdiv(beta, gamma);
  for (int i = 0; i < n; ++i) {
    double2 t = make_double2(cxm[i].x + cxp[i].x + mu[o + i], cxm[i].y + cxp[i].y);
    if (i == 0) t = zsub(t, gamma);
    if (i == n - 1) t = zsub(t, zmul(alpha, bg));
    dg[o + i] = t;
    du[o + i] = (i < n - 1) ? neg(cxp[i]) : make_double2(0.0, 0.0);
    du2[o + i] = make_double2(0.0, 0.0);
    r1[o + i] = jp[o + i];
    r2[o + i] = make_double2(0.0, 0.0);
  }
  r2[o] = gamma;
  r2[o + n - 1] = alpha;
  // elimination with partial pivoting (row i+1's sub-diagonal entry is the
  // untouched -cxm_{i+1})
  for (int i = 0; i < n - 1; ++i) {
    const double2 sub = neg(cxm[i + 1]);
    const double2 di = dg[o + i];
    if (zabs2(di) >= zabs2(sub)) {
      const double2 m = zdiv(sub, di);
      dg[o + i + 1] = zsub(dg[o + i + 1], zmul(m, du[o + i]));
      r1[o + i + 1] = zsub(r1[o + i + 1], zmul(m, r1[o + i]));
      r2[o + i + 1] = zsub(r2[o + i + 1], zmul(m, r2[o + i]));
    } else {
      const double2 m = zdiv(di, sub);
      const double2 d1 = dg[o + i + 1], u0 = du[o + i];
      const double2 u1 = (i + 1 < n - 1) ? du[o + i + 1] : make_double2(0.0, 0.0);
      dg[o + i] = sub;
      du[o + i] = d1;
      du2[o + i] = u1;
      dg[o + i + 1] = zsub(u0, zmul(m, d1));
      if (i + 1 < n - 1) du[o + i + 1] = neg(zmul(m, u1));
      const double2 a1 = r1[o + i], b1 = r1[o + i + 1];
      r1[o + i] = b1;
      r1[o + i + 1] = zsub(a1, zmul(m, b1));
      const double2 a2 = r2[o + i], b2 = r2[o + i + 1];
      r2[o + i] = b2;
      r2[o + i + 1] = zsub(a2, zmul(m, b2));
    }
  }
  // back substitution, both right-hand sides, in place
  double2 y1 = zdiv(r1[o + n - 1], dg[o + n - 1]), z1 = zdiv(r2[o + n - 1], dg[o + n - 1]);
  double2 y2 = make_double2(0.0, 0.0), z2 = y2;   // x_{i+2}
  r1[o + n - 1] = y1;
  r2[o + n - 1] = z1;
  for (int i = n - 2; i >= 0; --i) {
    const double2 u = du[o + i], w = du2[o + i], di = dg[o + i];
    const double2 yi = zdiv(zsub(zsub(r1[o + i], zmul(u, y1)), zmul(w, y2)), di);
    const double2 zi = zdiv(zsub(zsub(r2[o + i], zmul(u, z1)), zmul(w, z2)), di);
    r1[o + i] = yi;
    r2[o + i] = zi;
    y2 = y1; z2 = z1;
    y1 = yi; z1 = zi;
  }
  const double2 vy = zadd(r1[o], zmul(bg, r1[o + n - 1]));
  const double2 vz = zadd(make_double2(1.0 + r2[o].x, r2[o].y), zmul(bg, r2[o + n - 1]));
  const double2 f = zdiv(vy, vz);
  for (int i = 0; i < n; ++i) amp[o + i] = zsub(r1[o + i], zmul(f, r2[o + i]));
}

// ------------------------------------------------------ field (step 3) ----
__global__ __launch_bounds__(256) void k_eim_assemble(const EimDesc* __restrict__ desc,
                                                      const double* __restrict__ phi,
                                                      const double2* __restrict__ amp) {
  const EimDesc d = desc[blockIdx.y];
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= d.nx * d.ny) return;
  const int ix = e % d.nx;
  const double2 a = amp[d.off1 + ix];
  const double v = phi[d.off2 + e];
  d.F[e] = make_float2((float)(a.x * v), (float)(a.y * v));
}

}  // namespace

// Scratch layout of one call: phi and pivots (D doubles each); mu (nx
// doubles); j, diagonal, two super-diagonals, two right-hand sides, amplitude
// (nx complex each); then the descriptor table.  Every word is written by the
// kernels before it is read, so nothing needs clearing between calls.
static size_t eim_scratch_bytes(size_t s2, size_t s1, int nb) {
  const size_t s1p = (s1 + 1) & ~(size_t)1;   // keeps the complex arrays 16-byte aligned
  return sizeof(double) * (2 * s2 + s1p) + sizeof(double2) * 7 * s1 + sizeof(EimDesc) * nb;
}

// Validates the arguments and fills the descriptor table; returns the
// scratch bytes the call needs (0 on an invalid argument, message set).
static size_t eim_prepare(const char* who, const fdfd_op* const* ops, int nb,
                          const void* const* b, void* const* F, std::vector<EimDesc>& hd,
                          size_t& s1, int& maxnx, int& maxD) {
  if (!ops || !b || !F || nb < 1) {
    dd_set_error("%s: need nb >= 1 and the ops, b and F arrays", who);
    return 0;
  }
  hd.resize(nb);
  size_t s2 = 0;
  s1 = 0;
  maxnx = 0;
  maxD = 0;
  for (int p = 0; p < nb; ++p) {
    if (!ops[p] || !b[p] || !F[p]) {
      dd_set_error("%s: problem %d has a NULL operator, b or F", who, p);
      return 0;
    }
    const fdfd_op* op = ops[p];
    EimDesc& d = hd[p];
    d.nx = op->nx; d.ny = op->ny; d.omega = op->omega; d.dx = op->dx;
    d.eps = op->eps64; d.cf = op->cf64;
    d.b = (const double2*)b[p]; d.F = (float2*)F[p];
    d.off2 = s2; d.off1 = s1;
    s2 += (size_t)op->D;
    s1 += (size_t)op->nx;
    maxnx = std::max(maxnx, op->nx);
    maxD = std::max(maxD, op->D);
  }
  return eim_scratch_bytes(s2, s1, nb);
}

// Enqueues the three kernels on scratch ws (eim_scratch_bytes long) and waits
// for them.
static hipError_t eim_run(const std::vector<EimDesc>& hd, size_t s1, int maxnx, int maxD,
                          char* ws, hipStream_t stream) {
  const int nb = (int)hd.size();
  size_t s2 = 0;
  for (const auto& d : hd) s2 += (size_t)d.nx * d.ny;
  const size_t s1p = (s1 + 1) & ~(size_t)1;
  double* phi = (double*)ws;
  double* piv = phi + s2;
  double* mu = piv + s2;
  double2* z = (double2*)(mu + s1p);
  double2 *jp = z, *dg = z + s1, *du = z + 2 * s1, *du2 = z + 3 * s1, *r1 = z + 4 * s1,
          *r2 = z + 5 * s1, *amp = z + 6 * s1;
  EimDesc* dd = (EimDesc*)(z + 7 * s1);
  hipError_t e = hipMemcpyAsync(dd, hd.data(), sizeof(EimDesc) * nb, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) {
    k_eim_modes<<<dim3((maxnx + 63) / 64, nb), 64, 0, stream>>>(dd, phi, piv, mu, jp);
    k_eim_line<<<(nb + 63) / 64, 64, 0, stream>>>(dd, nb, mu, jp, dg, du, du2, r1, r2, amp);
    k_eim_assemble<<<dim3((maxD + 255) / 256, nb), 256, 0, stream>>>(dd, phi, amp);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e;
}

extern "C" dd_status eim_field(const fdfd_op* const* ops, int nb, const void* const* b,
                               void* const* F, hipStream_t stream) {
  std::vector<EimDesc> hd;
  size_t s1 = 0;
  int maxnx = 0, maxD = 0;
  const size_t bytes = eim_prepare("eim_field", ops, nb, b, F, hd, s1, maxnx, maxD);
  if (bytes == 0) return DD_EINVAL;
  char* ws = nullptr;
  DD_HIP_CHECK(hipMalloc((void**)&ws, bytes));
  hipError_t e = eim_run(hd, s1, maxnx, maxD, ws, stream);
  (void)hipFree(ws);
  if (e != hipSuccess) {
    dd_set_error("eim_field: %s", hipGetErrorString(e));
    return DD_EHIP;
  }
  return DD_OK;
}

// eim_field on a workspace the caller owns (ws_bytes >= eim_ws_bytes of the
// batch): used by the predictor, which holds one for its largest batch.
size_t eim_ws_bytes(int nx, int ny, int nb) {
  return eim_scratch_bytes((size_t)nx * ny * nb, (size_t)nx * nb, nb);
}

dd_status eim_field_ws(const fdfd_op* const* ops, int nb, const void* const* b, void* const* F,
                       void* ws, size_t ws_bytes, hipStream_t stream) {
  std::vector<EimDesc> hd;
  size_t s1 = 0;
  int maxnx = 0, maxD = 0;
  const size_t bytes = eim_prepare("eim_field", ops, nb, b, F, hd, s1, maxnx, maxD);
  if (bytes == 0) return DD_EINVAL;
  if (!ws || bytes > ws_bytes) {
    dd_set_error("eim_field: the batch needs %zu bytes of workspace, %zu given", bytes, ws_bytes);
    return DD_EINVAL;
  }
  const hipError_t e = eim_run(hd, s1, maxnx, maxD, (char*)ws, stream);
  if (e != hipSuccess) {
    dd_set_error("eim_field: %s", hipGetErrorString(e));
    return DD_EHIP;
  }
  return DD_OK;
}

// ------------------------------------------- allocation-free variant ----
// The scratch of eim_field_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never uses its name as an
// address: eim_scratch_ptr() resolves the current device's copy once with
// hipGetSymbolAddress and every kernel argument and copy goes through that
// pointer.
static __device__ __align__(256) char eim_scratch[DD_EIM_NOALLOC_BYTES];

static std::mutex g_eim_scratch_mu;
static void* g_eim_scratch_ptr[DD_EIM_MAX_DEVICES];

static dd_status eim_scratch_ptr(char** out) {
  int dev = 0;
  DD_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= DD_EIM_MAX_DEVICES) {
    dd_set_error("eim_field_noalloc: device %d beyond the %d supported", dev, DD_EIM_MAX_DEVICES);
    return DD_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_eim_scratch_mu);
  if (!g_eim_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(eim_scratch));
    if (e != hipSuccess || !ptr) {
      dd_set_error("eim_field_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
      return DD_EHIP;
    }
    g_eim_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_eim_scratch_ptr[dev];
  return DD_OK;
}

extern "C" dd_status eim_field_noalloc(const fdfd_op* const* ops, int nb, const void* const* b,
                                       void* const* F, hipStream_t stream) {
  std::vector<EimDesc> hd;
  size_t s1 = 0;
  int maxnx = 0, maxD = 0;
  const size_t bytes = eim_prepare("eim_field_noalloc", ops, nb, b, F, hd, s1, maxnx, maxD);
  if (bytes == 0) return DD_EINVAL;
  if (bytes > (size_t)DD_EIM_NOALLOC_BYTES) {
    dd_set_error("eim_field_noalloc: the batch needs %zu bytes of scratch, more than the %zu "
                 "the library holds (split the batch, or call eim_field)",
                 bytes, (size_t)DD_EIM_NOALLOC_BYTES);
    return DD_EINVAL;
  }
  char* ws = nullptr;
  dd_status rc = eim_scratch_ptr(&ws);
  if (rc != DD_OK) return rc;
  const hipError_t e = eim_run(hd, s1, maxnx, maxD, ws, stream);
  if (e != hipSuccess) {
    dd_set_error("eim_field_noalloc: %s", hipGetErrorString(e));
    return DD_EHIP;
  }
  return DD_OK;
}
