// Trace kernels compiled for degrees (p, q) = (2, 2) and filter size nu = 3.
#include "trace.hpp"

namespace ffrt {
const KernelSet* kernel_set_p2q2nu3() { return KernelsFor<2, 2, 3>::get(); }
}  // namespace ffrt
