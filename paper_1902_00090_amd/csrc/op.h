// FDFD operator object and the 5-point stencil device function (Sec. 2, Eq. 1).
#pragma once

#include "common.h"

// Per-axis stencil coefficients, complex, laid out as
//   [0, nx)        cxm[i] = 1 / (dx^2 s_x(i) s_x(i - 1/2))
//   [nx, 2nx)      cxp[i] = 1 / (dx^2 s_x(i) s_x(i + 1/2))
//   [2nx, 2nx+ny)  cym[j]
//   [2nx+ny, ...)  cyp[j]
// so that (A y)_c = cxm (y_c - y_w) - cxp (y_e - y_c) + cym (y_c - y_s)
//                 - cyp (y_n - y_c) - omega^2 eps_c y_c, with periodic wrap.
struct fdfd_op {
  int nx, ny, D;
  double omega, dx;
  dd_pml pml;
  float* eps32;      // [D]
  double* eps64;     // [D]
  float2* cf32;      // [2nx + 2ny]
  double2* cf64;     // [2nx + 2ny]
  double2* s64;      // [nx + ny] stretch factors at the integer nodes, s_x(i) then s_y(j)
};

// Differences are formed before the complex products: for smooth fields the
// neighbour differences are exact in floating point and only the products round.
template <typename T, typename EPS>
__device__ __forceinline__ c2<T> stencil_point(const c2<T>* __restrict__ x, int e, int nx,
                                               int ny, const c2<T>* __restrict__ cf,
                                               const EPS* __restrict__ eps, T omega2) {
  using V = c2<T>;
  const int iy = e / nx;
  const int ix = e - iy * nx;
  const int ew = (ix == 0) ? e + nx - 1 : e - 1;
  const int ee = (ix == nx - 1) ? e - nx + 1 : e + 1;
  const int es = (iy == 0) ? e + (ny - 1) * nx : e - nx;
  const int en = (iy == ny - 1) ? e - (ny - 1) * nx : e + nx;
  const V c = x[e], w = x[ew], ea = x[ee], s = x[es], n = x[en];
  const V cxm = cf[ix], cxp = cf[nx + ix], cym = cf[2 * nx + iy], cyp = cf[2 * nx + ny + iy];
  V r = cmul(cxm, csub(c, w));
  r = csub(r, cmul(cxp, csub(ea, c)));
  r = cadd(r, cmul(cym, csub(c, s)));
  r = csub(r, cmul(cyp, csub(n, c)));
  const T d = omega2 * (T)eps[e];
  r.x -= d * c.x;
  r.y -= d * c.y;
  return r;
}

// (A (pr .* x))_c: the same stencil applied to the neighbours scaled by the
// per-element factors pr (a right diagonal preconditioner fused into the sweep).
template <typename T, typename EPS>
__device__ __forceinline__ c2<T> stencil_point_scaled(const c2<T>* __restrict__ x,
                                                      const c2<T>* __restrict__ pr, int e, int nx,
                                                      int ny, const c2<T>* __restrict__ cf,
                                                      const EPS* __restrict__ eps, T omega2) {
  using V = c2<T>;
  const int iy = e / nx;
  const int ix = e - iy * nx;
  const int ew = (ix == 0) ? e + nx - 1 : e - 1;
  const int ee = (ix == nx - 1) ? e - nx + 1 : e + 1;
  const int es = (iy == 0) ? e + (ny - 1) * nx : e - nx;
  const int en = (iy == ny - 1) ? e - (ny - 1) * nx : e + nx;
  const V c = cmul(x[e], pr[e]), w = cmul(x[ew], pr[ew]), ea = cmul(x[ee], pr[ee]);
  const V s = cmul(x[es], pr[es]), n = cmul(x[en], pr[en]);
  const V cxm = cf[ix], cxp = cf[nx + ix], cym = cf[2 * nx + iy], cyp = cf[2 * nx + ny + iy];
  V r = cmul(cxm, csub(c, w));
  r = csub(r, cmul(cxp, csub(ea, c)));
  r = cadd(r, cmul(cym, csub(c, s)));
  r = csub(r, cmul(cyp, csub(n, c)));
  const T d = omega2 * (T)eps[e];
  r.x -= d * c.x;
  r.y -= d * c.y;
  return r;
}
