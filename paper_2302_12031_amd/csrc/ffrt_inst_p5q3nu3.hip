// Trace kernels compiled for degrees (p, q) = (5, 3) and filter size nu = 3.
#include "trace.hpp"

namespace ffrt {
const KernelSet* kernel_set_p5q3nu3() { return KernelsFor<5, 3, 3>::get(); }
}  // namespace ffrt
