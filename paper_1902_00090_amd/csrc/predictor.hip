// Subspace predictors behind one interface (Sec. 3: the model maps a
// permittivity to vectors v_1..v_N that augment GMRES).  Two kinds:
//   * PCA: one fixed basis for every permittivity (Sec. 3, PCA paragraph);
//   * CNN: the convolutional network, with one input plane (permittivity) or
//     three (plus the effective-index field, which this layer computes from
//     the problem's operator and right-hand side).
// A predictor is loaded from a file (predfile.h) written by
// predictor_save_pca or dd_cnn_save.
#include <cstring>
#include <vector>

#include "common.h"
#include "eim.h"
#include "op.h"
#include "predfile.h"

struct dd_predictor {
  int kind = 0;
  int nx = 0, ny = 0, k = 0, in_channels = 0, max_batch = 0;
  float2* U = nullptr;     // PCA basis [k][D]
  dd_cnn* net = nullptr;   // CNN
  float2* eim = nullptr;   // [max_batch][D] effective-index fields (three-plane CNN)
  void* eim_ws = nullptr;  // their workspace, sized for max_batch problems
  size_t eim_ws_bytes = 0;
};

extern "C" void predictor_destroy(dd_predictor* p) {
  if (!p) return;
  if (p->U) (void)hipFree(p->U);
  if (p->eim) (void)hipFree(p->eim);
  if (p->eim_ws) (void)hipFree(p->eim_ws);
  if (p->net) dd_cnn_destroy(p->net);
  delete p;
}

extern "C" dd_status predictor_save_pca(const char* path, const void* U, int k, int nx, int ny,
                                        hipStream_t stream) {
  if (!path || !U || k < 1 || nx < 1 || ny < 1) {
    dd_set_error("predictor_save_pca: need a path, U and k, nx, ny >= 1");
    return DD_EINVAL;
  }
  const size_t n = (size_t)k * nx * ny;
  std::vector<float2> h(n);
  DD_HIP_CHECK(hipMemcpyAsync(h.data(), U, sizeof(float2) * n, hipMemcpyDeviceToHost, stream));
  DD_HIP_CHECK(hipStreamSynchronize(stream));
  PredFileHeader hd{};
  std::memcpy(hd.magic, DD_PRED_MAGIC, 8);
  hd.kind = DD_PRED_PCA;
  hd.nx = nx; hd.ny = ny; hd.k = k; hd.in_channels = 0;
  hd.count = (int64_t)n;
  FILE* f = std::fopen(path, "wb");
  if (!f) { dd_set_error("predictor_save_pca: cannot open '%s' for writing", path); return DD_EINVAL; }
  const bool ok = std::fwrite(&hd, sizeof(hd), 1, f) == 1 &&
                  std::fwrite(h.data(), sizeof(float2), n, f) == n;
  if (std::fclose(f) != 0 || !ok) {
    dd_set_error("predictor_save_pca: writing '%s' failed", path);
    return DD_EINVAL;
  }
  return DD_OK;
}

extern "C" dd_status predictor_load(const char* path, int max_batch, dd_predictor** out) {
  if (!out) { dd_set_error("predictor_load: out is NULL"); return DD_EINVAL; }
  *out = nullptr;
  if (max_batch < 1) { dd_set_error("predictor_load: max_batch must be >= 1"); return DD_EINVAL; }
  PredFileHeader h{};
  char msg[512];
  FILE* f = pred_open(path, h, msg, sizeof(msg));
  if (!f) { dd_set_error("predictor_load: %s", msg); return DD_EINVAL; }
  const size_t D = (size_t)h.nx * h.ny;
  if (h.kind == DD_PRED_PCA && (uint64_t)h.count != (uint64_t)h.k * D) {
    std::fclose(f);
    dd_set_error("predictor_load: '%s': %lld values for k = %d of %d x %d", path,
                 (long long)h.count, h.k, h.nx, h.ny);
    return DD_EINVAL;
  }
  dd_predictor* p = new dd_predictor();
  p->kind = h.kind;
  p->nx = h.nx; p->ny = h.ny; p->k = h.k; p->in_channels = h.in_channels;
  p->max_batch = max_batch;
  if (h.kind == DD_PRED_PCA) {
    std::vector<float2> buf(h.count);
    const bool ok = std::fread(buf.data(), sizeof(float2), buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) { delete p; dd_set_error("predictor_load: reading '%s' failed", path); return DD_EINVAL; }
    hipError_t e = hipMalloc((void**)&p->U, sizeof(float2) * buf.size());
    if (e == hipSuccess)
      e = hipMemcpy(p->U, buf.data(), sizeof(float2) * buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      predictor_destroy(p);
      dd_set_error("predictor_load: %s", hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP;
    }
  } else {
    std::fclose(f);
    dd_status rc = dd_cnn_load(path, max_batch, &p->net);
    if (rc != DD_OK) { delete p; return rc; }
    if (p->in_channels == 3) {
      p->eim_ws_bytes = eim_ws_bytes(p->nx, p->ny, max_batch);
      hipError_t e = hipMalloc((void**)&p->eim, sizeof(float2) * D * max_batch);
      if (e == hipSuccess) e = hipMalloc(&p->eim_ws, p->eim_ws_bytes);
      if (e != hipSuccess) {
        predictor_destroy(p);
        dd_set_error("predictor_load: %s", hipGetErrorString(e));
        return DD_ENOMEM;
      }
    }
  }
  *out = p;
  return DD_OK;
}

extern "C" dd_status predictor_info(const dd_predictor* p, int* kind, int* nx, int* ny, int* k,
                                    int* in_channels) {
  if (!p) { dd_set_error("predictor_info: NULL predictor"); return DD_EINVAL; }
  if (kind) *kind = p->kind;
  if (nx) *nx = p->nx;
  if (ny) *ny = p->ny;
  if (k) *k = p->k;
  if (in_channels) *in_channels = p->in_channels;
  return DD_OK;
}

extern "C" dd_status predict_subspace(dd_predictor* p, const fdfd_op* const* ops,
                                      const void* const* b, const float* eps, int B, void* U,
                                      hipStream_t stream) {
  if (!p || !U || B < 1) {
    dd_set_error("predict_subspace: need a predictor, U and B >= 1");
    return DD_EINVAL;
  }
  const size_t D = (size_t)p->nx * p->ny;
  if (ops)
    for (int i = 0; i < B; ++i)
      if (!ops[i] || ops[i]->nx != p->nx || ops[i]->ny != p->ny) {
        dd_set_error("predict_subspace: problem %d is not on the predictor's %d x %d grid", i,
                     p->nx, p->ny);
        return DD_EINVAL;
      }
  if (p->kind == DD_PRED_PCA) {
    // the same basis for every permittivity
    for (int i = 0; i < B; ++i)
      DD_HIP_CHECK(hipMemcpyAsync((float2*)U + (size_t)i * p->k * D, p->U,
                                  sizeof(float2) * p->k * D, hipMemcpyDeviceToDevice, stream));
    DD_HIP_CHECK(hipStreamSynchronize(stream));
    return DD_OK;
  }
  if (!eps) { dd_set_error("predict_subspace: the CNN needs eps"); return DD_EINVAL; }
  if (B > p->max_batch) {
    dd_set_error("predict_subspace: B = %d above the max_batch %d the predictor was loaded with",
                 B, p->max_batch);
    return DD_EINVAL;
  }
  if (p->in_channels == 1) return dd_cnn_predict(p->net, eps, B, U, stream);
  if (!ops || !b) {
    dd_set_error("predict_subspace: the three-plane CNN needs ops and b (its effective-index "
                 "field input)");
    return DD_EINVAL;
  }
  std::vector<void*> F(B);
  for (int i = 0; i < B; ++i) F[i] = p->eim + (size_t)i * D;
  dd_status rc = eim_field_ws(ops, B, b, F.data(), p->eim_ws, p->eim_ws_bytes, stream);
  if (rc != DD_OK) return rc;
  return dd_cnn_predict_eim(p->net, eps, p->eim, B, U, stream);
}
