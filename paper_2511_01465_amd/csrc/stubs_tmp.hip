#include "internal.h"
namespace pint {
size_t scan_ws_bytes(int, int64_t, int64_t, int, int) { return 0; }
int affine_scan(int, int64_t, int64_t, int, const void*, const void*, const void*, void*, int, void*, size_t, hipStream_t) { return ST_UNSUPPORTED; }
size_t adjoint_ws_bytes(int, int, int64_t, int64_t, int64_t, int) { return 0; }
int adjoint(const SolveArgs&, const void*, void*, void*, int64_t) { return ST_UNSUPPORTED; }
}
