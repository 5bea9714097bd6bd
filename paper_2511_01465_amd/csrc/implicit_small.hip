// The small-d kernels instantiated for the implicit step rules of Sec. 3.4
// (backward Euler and the trapezoidal rule); a translation unit of its own
// so the two rule sets compile in parallel.
#include "newton_small.h"

namespace pint {

int small_launch_implicit(int method, const SmallKArgs& k, const SmallLaunch& l) {
  switch (method) {
    case METHOD_BEULER: return small_launch<METHOD_BEULER>(k, l);
    case METHOD_TRAP: return small_launch<METHOD_TRAP>(k, l);
  }
  return ST_UNSUPPORTED;
}

}  // namespace pint
