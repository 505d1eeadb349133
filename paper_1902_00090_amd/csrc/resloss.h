// Residual loss of predicted subspaces (Sec. 3, eq:res_loss): the shared core
// used by res_loss_batched and the CNN's residual-loss training.
#pragma once

#include "common.h"
#include "op.h"

// For nb problems (operator ops[p], right-hand side b[p] [D] complex128,
// subspace V[p] [k][D] complex64, all on the device):
//   loss[p] (host) = min_c ||A V c - b||^2 / ||b||^2;
// when dz != NULL also dz[(p D + e) coutp + ch] (bf16) = derivative of
// scale * loss[p] with respect to the real (ch = 2j) and imaginary (ch = 2j+1)
// part of V[p][j][e], channels >= 2k zero.
// when Gout != NULL (host array of nb device pointers) also
// Gout[p][j][e] (complex64) = 2 scale dl / d conj(V[p][j][e]).
// Wbuf holds k * sum D complex64 values; rbuf and sbuf sum D each (only used
// when dz or Gout is given).  scratch (res_loss_scratch_bytes(nb, k) bytes,
// device) holds the descriptors, coefficients and Gram partials; NULL
// allocates them for the call.  Synchronises the stream.
dd_status res_loss_core(const fdfd_op* const* ops, const void* const* b, const void* const* V,
                        int nb, int k, float2* Wbuf, float2* rbuf, float2* sbuf, double* loss,
                        __bf16* dz, int coutp, double scale, hipStream_t st,
                        void* const* Gout = nullptr, void* scratch = nullptr,
                        size_t scratch_bytes = 0);

// Device scratch res_loss_core needs for nb problems with k vectors.
size_t res_loss_scratch_bytes(int nb, int k);
