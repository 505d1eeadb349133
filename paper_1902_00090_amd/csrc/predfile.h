// File layout of a saved subspace predictor (a PCA basis or a CNN with its
// Adam state), shared by the CNN's save/load and the generic predictor.
//
//   PredFileHeader (48 bytes, little-endian), then
//   PCA: float32 [k][D][2] basis vectors (complex64, the layout of U);
//   CNN: float32 params[count], Adam first moments[count], second
//        moments[count] (the dd_cnn_get_params layout), with adam_t the
//        number of Adam steps taken.
#pragma once

#include <cstdint>
#include <cstdio>
#include <cstring>

#define DD_PRED_MAGIC "DDPRED01"
enum { DD_PRED_PCA = 1, DD_PRED_CNN = 2 };

struct PredFileHeader {
  char magic[8];
  int32_t kind;
  int32_t nx, ny, k, in_channels;
  int32_t reserved;
  int64_t count;      // PCA: k * D complex values; CNN: parameter count
  int64_t adam_t;     // CNN: Adam steps taken; PCA: 0
};
static_assert(sizeof(PredFileHeader) == 48, "predictor file header must be 48 bytes");

// Payload bytes implied by a header (0 for an unknown kind).
inline uint64_t pred_payload_bytes(const PredFileHeader& h) {
  if (h.kind == DD_PRED_PCA) return (uint64_t)h.count * 8;
  if (h.kind == DD_PRED_CNN) return (uint64_t)h.count * 12;
  return 0;
}

// Opens path and reads and checks its header against the file size.
// Returns the open file positioned at the payload, or NULL with msg set.
inline FILE* pred_open(const char* path, PredFileHeader& h, char* msg, size_t msglen) {
  FILE* f = path ? std::fopen(path, "rb") : nullptr;
  if (!f) {
    std::snprintf(msg, msglen, "cannot open '%s'", path ? path : "(null)");
    return nullptr;
  }
  if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, DD_PRED_MAGIC, 8) != 0) {
    std::snprintf(msg, msglen, "'%s' is not a predictor file", path);
    std::fclose(f);
    return nullptr;
  }
  const uint64_t want = pred_payload_bytes(h);
  std::fseek(f, 0, SEEK_END);
  const long long size = std::ftell(f);
  std::fseek(f, (long)sizeof(h), SEEK_SET);
  if (want == 0 || h.nx < 1 || h.ny < 1 || h.k < 1 || h.count < 1 ||
      (uint64_t)size != sizeof(h) + want) {
    std::snprintf(msg, msglen, "'%s': bad header or size (kind %d, %lld bytes, %llu expected)",
                  path, h.kind, size, (unsigned long long)(sizeof(h) + want));
    std::fclose(f);
    return nullptr;
  }
  return f;
}
