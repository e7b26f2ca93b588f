// Trace kernels compiled for degrees (p, q) = (3, 3) and filter size nu = 5.
#include "trace.hpp"

namespace ffrt {
const KernelSet* kernel_set_p3q3nu5() { return KernelsFor<3, 3, 5>::get(); }
}  // namespace ffrt
