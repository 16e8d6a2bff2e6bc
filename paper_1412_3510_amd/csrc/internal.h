// Library-internal entry points shared between the host source files.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/rpca.h"

namespace rpca {

// the HIP device a context was created on
int ctx_device(rpca_ctx ctx);
// record ``msg`` as the context's last error and return ``s``
rpca_status ctx_fail(rpca_ctx ctx, rpca_status s, const char* msg);
// rpca_svd on caller-provided device memory: the working buffers in ``ws``
// (``ws_bytes``, 256-byte aligned) and the LU arrival counters in
// ``counters`` (``counters_n`` entries, cleared here on the stream).  Returns
// RPCA_ERR_NO_MEMORY, before launching anything, when the problem needs more;
// allocates nothing.
rpca_status svd_on_workspace(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its,
                             uint64_t seed, unsigned flags, float* U, int64_t ldu, double* S,
                             float* V, int64_t ldv, char* ws, size_t ws_bytes,
                             unsigned* counters, size_t counters_n);

}  // namespace rpca
