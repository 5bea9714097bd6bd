#include "internal.h"
namespace pint {
size_t adjoint_ws_bytes(int, int, int64_t, int64_t, int64_t, int) { return 0; }
int adjoint(const SolveArgs&, const void*, void*, void*, int64_t) { return ST_UNSUPPORTED; }
}
