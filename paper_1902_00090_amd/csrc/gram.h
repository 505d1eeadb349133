// Small FP64 Gram matrices of complex64 vector sets and their Cholesky
// inverse factors (implemented in pca.hip, shared by the residual loss).
#pragma once

#include <complex>
#include <vector>

#include "common.h"

// G = [V; f]^H [V; f] ((k+1) x (k+1) with f, else k x k; row-major, stride
// k+1), FP64 sums on the device, result on the host.  V: [k][D] complex64,
// f: [D] complex128 or NULL (device).  Synchronises the stream.
dd_status gram_host(const float2* V, int k, int D, const double2* f,
                    std::vector<std::complex<double>>& G, hipStream_t stream);

// Cholesky G = L L^H of the leading k x k block of G (row stride ld); false if
// it is not positive definite.  T = L^{-H} (upper triangular, row-major k x k),
// so that G^{-1} = T T^H.
bool chol_inv(const std::vector<std::complex<double>>& G, int ld, int k,
              std::vector<std::complex<double>>& L, std::vector<std::complex<double>>& T);
