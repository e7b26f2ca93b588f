// Adam update of one design's control points (Kingma & Ba, bias-corrected), shared by the standalone Adam
// kernel and the adjoint's last-workgroup epilogue.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ffrt_internal.h"

namespace ffrt {

// Threads of one workgroup update control points [off, off + n) with gradient g(i) (i relative to off);
// the step counter t is read before and written after a barrier, so every thread must call this.
// P -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
template <class GradAt>
__device__ inline void adam_update(float* Pz, float* m, float* v, int32_t* t, int64_t off, int n,
                                   const ffrt_adam_hparams& hp, GradAt g) {
    const int tn = t[0] + 1;
    const float bc1 = 1.0f - powf(hp.beta1, (float)tn);
    const float bc2 = 1.0f - powf(hp.beta2, (float)tn);
    const float step = hp.lr / bc1, rb2 = 1.0f / sqrtf(bc2);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t k = off + i;
        const float gi = g(i);
        const float mi = hp.beta1 * m[k] + (1.0f - hp.beta1) * gi;
        const float vi = hp.beta2 * v[k] + (1.0f - hp.beta2) * gi * gi;
        m[k] = mi;
        v[k] = vi;
        Pz[k] -= step * mi / (sqrtf(vi) * rb2 + hp.eps);
    }
    __syncthreads();
    if (threadIdx.x == 0) t[0] = tn;
}

}  // namespace ffrt
