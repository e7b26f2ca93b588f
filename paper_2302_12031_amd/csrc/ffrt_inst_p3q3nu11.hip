// Trace kernels compiled for degrees (p, q) = (3, 3) and filter size nu = 11.
#include "trace.hpp"

namespace ffrt {
const KernelSet* kernel_set_p3q3nu11() { return KernelsFor<3, 3, 11>::get(); }
}  // namespace ffrt
