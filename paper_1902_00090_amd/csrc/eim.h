// Internal: the effective-index field on a caller-owned workspace.
#pragma once

#include <stddef.h>

#include "common.h"

// Bytes of workspace eim_field_ws needs for nb problems of an nx x ny grid.
size_t eim_ws_bytes(int nx, int ny, int nb);

// eim_field (include/ddgmres.h) on the workspace ws of ws_bytes bytes;
// DD_EINVAL when it is too small for the batch.  Synchronises the stream.
dd_status eim_field_ws(const fdfd_op* const* ops, int nb, const void* const* b, void* const* F,
                       void* ws, size_t ws_bytes, hipStream_t stream);
