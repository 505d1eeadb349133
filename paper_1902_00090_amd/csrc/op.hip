// FDFD operator: creation (stretched-coordinate PML factors), y = A x.
//
// Sec. 2, Eq. 1 for the E_z polarisation: curl curl E_z z = -laplacian E_z z,
// discretised with E_z on integer Yee nodes, forward differences on half
// nodes and backward differences back onto integer nodes; each difference is
// divided by the local stretch factor s = 1 - i sigma / omega (exp(+i omega t)
// convention, fixed by the sign of the source term -i omega mu0 J).  The
// outer boundary is periodic (the PML sits in front of it); the periodic
// link between the last and first node lies at full PML depth.
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "op.h"

// ------------------------------------------------------------ error state ---
static thread_local char g_err[1024] = "";

void dd_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

extern "C" const char* dd_last_error(void) { return g_err; }

// ------------------------------------------------------------ PML factors ---
// Stretch factor at position p (integer node i or half node i + 1/2) of an
// axis with n nodes and an npml-cell layer at both ends.
static std::complex<double> stretch_at(double p, int n, int npml, double dx, double omega,
                                       int grade, double lnR) {
  if (npml <= 0) return {1.0, 0.0};
  double depth = std::max(0.0, std::max(npml - p, p - (n - 1 - npml)));
  depth = std::min(depth, (double)npml);
  const double L = npml * dx;
  const double sigma_max = -(grade + 1) * lnR / (2.0 * L);
  const double sigma = sigma_max * std::pow(depth / npml, grade);
  return {1.0, -sigma / omega};
}

// cm[i] = 1/(dx^2 s(i) s(i-1/2)), cp[i] = 1/(dx^2 s(i) s(i+1/2)); s(-1/2) is
// the half node of the periodic link n-1 -> 0, i.e. s(n - 1/2).
static void axis_coeffs(int n, int npml, double dx, double omega, int grade, double lnR,
                        std::vector<std::complex<double>>& cm,
                        std::vector<std::complex<double>>& cp) {
  cm.resize(n);
  cp.resize(n);
  std::vector<std::complex<double>> si(n), sh(n);
  for (int i = 0; i < n; ++i) {
    si[i] = stretch_at(i, n, npml, dx, omega, grade, lnR);
    sh[i] = stretch_at(i + 0.5, n, npml, dx, omega, grade, lnR);
  }
  for (int i = 0; i < n; ++i) {
    const std::complex<double> s_minus = sh[(i + n - 1) % n];
    cm[i] = 1.0 / (dx * dx * si[i] * s_minus);
    cp[i] = 1.0 / (dx * dx * si[i] * sh[i]);
  }
}

extern "C" dd_status fdfd_op_create(const float* eps, int nx, int ny, double omega, double dx,
                                    const dd_pml* pml, hipStream_t stream, fdfd_op** out) {
  if (!out) { dd_set_error("fdfd_op_create: out is NULL"); return DD_EINVAL; }
  *out = nullptr;
  dd_pml P = pml ? *pml : dd_pml{0, 0, 3, -16.0};
  if (P.grade_m <= 0) P.grade_m = 3;
  if (P.ln_R == 0.0) P.ln_R = -16.0;
  if (!eps || nx < 3 || ny < 3) {
    dd_set_error("fdfd_op_create: need eps != NULL and nx, ny >= 3 (got %d x %d)", nx, ny);
    return DD_EINVAL;
  }
  if (!(omega > 0.0) || !(dx > 0.0) || !std::isfinite(omega) || !std::isfinite(dx)) {
    dd_set_error("fdfd_op_create: omega and dx must be finite and > 0");
    return DD_EINVAL;
  }
  if (P.npml_x < 0 || P.npml_y < 0 || 2 * P.npml_x >= nx || 2 * P.npml_y >= ny ||
      !(P.ln_R < 0.0)) {
    dd_set_error("fdfd_op_create: invalid PML (npml %d,%d for %d x %d, ln_R %g)", P.npml_x,
                 P.npml_y, nx, ny, P.ln_R);
    return DD_EINVAL;
  }
  if ((long long)nx * ny > (1LL << 30)) {
    dd_set_error("fdfd_op_create: grid too large");
    return DD_EINVAL;
  }
  const int D = nx * ny;
  for (int e = 0; e < D; ++e)
    if (!std::isfinite(eps[e])) {
      dd_set_error("fdfd_op_create: eps[%d] is not finite", e);
      return DD_ENONFINITE;
    }
  std::vector<std::complex<double>> cxm, cxp, cym, cyp;
  axis_coeffs(nx, P.npml_x, dx, omega, P.grade_m, P.ln_R, cxm, cxp);
  axis_coeffs(ny, P.npml_y, dx, omega, P.grade_m, P.ln_R, cym, cyp);
  std::vector<double2> s64(nx + ny);
  for (int i = 0; i < nx; ++i) {
    const std::complex<double> v = stretch_at(i, nx, P.npml_x, dx, omega, P.grade_m, P.ln_R);
    s64[i] = make_double2(v.real(), v.imag());
  }
  for (int j = 0; j < ny; ++j) {
    const std::complex<double> v = stretch_at(j, ny, P.npml_y, dx, omega, P.grade_m, P.ln_R);
    s64[nx + j] = make_double2(v.real(), v.imag());
  }
  const int NC = 2 * nx + 2 * ny;
  std::vector<double2> c64(NC);
  std::vector<float2> c32(NC);
  auto put = [&](int off, const std::vector<std::complex<double>>& v) {
    for (size_t i = 0; i < v.size(); ++i) {
      c64[off + i] = make_double2(v[i].real(), v[i].imag());
      c32[off + i] = make_float2((float)v[i].real(), (float)v[i].imag());
    }
  };
  put(0, cxm);
  put(nx, cxp);
  put(2 * nx, cym);
  put(2 * nx + ny, cyp);
  std::vector<double> e64(eps, eps + D);

  fdfd_op* op = new fdfd_op();
  op->nx = nx; op->ny = ny; op->D = D; op->omega = omega; op->dx = dx; op->pml = P;
  op->eps32 = nullptr; op->eps64 = nullptr; op->cf32 = nullptr; op->cf64 = nullptr;
  op->s64 = nullptr;
  hipError_t e5 = hipMalloc(&op->s64, sizeof(double2) * (nx + ny));
  hipError_t e1 = hipMalloc(&op->eps32, sizeof(float) * D);
  hipError_t e2 = hipMalloc(&op->eps64, sizeof(double) * D);
  hipError_t e3 = hipMalloc(&op->cf32, sizeof(float2) * NC);
  hipError_t e4 = hipMalloc(&op->cf64, sizeof(double2) * NC);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess ||
      e5 != hipSuccess) {
    dd_set_error("fdfd_op_create: hipMalloc failed");
    fdfd_op_destroy(op);
    return DD_ENOMEM;
  }
  // the host arrays are pageable and some are locals: the copies are
  // enqueued on the caller's stream and finished before returning
  hipError_t c = hipMemcpyAsync(op->eps32, eps, sizeof(float) * D, hipMemcpyHostToDevice, stream);
  if (c == hipSuccess)
    c = hipMemcpyAsync(op->eps64, e64.data(), sizeof(double) * D, hipMemcpyHostToDevice, stream);
  if (c == hipSuccess)
    c = hipMemcpyAsync(op->cf32, c32.data(), sizeof(float2) * NC, hipMemcpyHostToDevice, stream);
  if (c == hipSuccess)
    c = hipMemcpyAsync(op->cf64, c64.data(), sizeof(double2) * NC, hipMemcpyHostToDevice, stream);
  if (c == hipSuccess)
    c = hipMemcpyAsync(op->s64, s64.data(), sizeof(double2) * (nx + ny), hipMemcpyHostToDevice,
                       stream);
  if (c == hipSuccess) c = hipStreamSynchronize(stream);
  if (c != hipSuccess) {
    dd_set_error("fdfd_op_create: copy to the device failed: %s", hipGetErrorString(c));
    fdfd_op_destroy(op);
    return DD_EHIP;
  }
  *out = op;
  return DD_OK;
}

extern "C" void fdfd_op_destroy(fdfd_op* op) {
  if (!op) return;
  if (op->eps32) (void)hipFree(op->eps32);
  if (op->eps64) (void)hipFree(op->eps64);
  if (op->cf32) (void)hipFree(op->cf32);
  if (op->cf64) (void)hipFree(op->cf64);
  if (op->s64) (void)hipFree(op->s64);
  delete op;
}

extern "C" int fdfd_op_dims(const fdfd_op* op, int* nx, int* ny) {
  if (!op) return -1;
  if (nx) *nx = op->nx;
  if (ny) *ny = op->ny;
  return op->D;
}

// One output element per thread; neighbours come through L1/L2.
template <typename T, typename EPS>
__global__ __launch_bounds__(DD_BLOCK) void k_apply(const c2<T>* __restrict__ x,
                                                    c2<T>* __restrict__ y, int nx, int ny,
                                                    const c2<T>* __restrict__ cf,
                                                    const EPS* __restrict__ eps, T omega2) {
  const int e = blockIdx.x * DD_BLOCK + threadIdx.x;
  if (e >= nx * ny) return;
  y[e] = stencil_point<T, EPS>(x, e, nx, ny, cf, eps, omega2);
}

extern "C" dd_status fdfd_op_apply(const fdfd_op* op, const void* x, void* y, dd_prec p,
                                   hipStream_t stream) {
  if (!op || !x || !y) { dd_set_error("fdfd_op_apply: NULL argument"); return DD_EINVAL; }
  if (x == y) { dd_set_error("fdfd_op_apply: x and y must not alias"); return DD_EINVAL; }
  const int grid = (op->D + DD_BLOCK - 1) / DD_BLOCK;
  if (p == DD_C64) {
    k_apply<float, float><<<grid, DD_BLOCK, 0, stream>>>(
        (const float2*)x, (float2*)y, op->nx, op->ny, op->cf32, op->eps32,
        (float)(op->omega * op->omega));
  } else if (p == DD_C128) {
    k_apply<double, double><<<grid, DD_BLOCK, 0, stream>>>(
        (const double2*)x, (double2*)y, op->nx, op->ny, op->cf64, op->eps64,
        op->omega * op->omega);
  } else {
    dd_set_error("fdfd_op_apply: unknown precision %d", (int)p);
    return DD_EINVAL;
  }
  DD_HIP_CHECK(hipGetLastError());
  return DD_OK;
}
