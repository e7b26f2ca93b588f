// Adam update of one design's control points (Kingma & Ba, bias-corrected), shared by the standalone Adam
// kernel and the step's finish.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ffrt_internal.h"
#include "loss.hpp"

namespace ffrt {

// Threads of one workgroup update control points [off, off + n) with gradient g(i) (i relative to off);
// the step counter t is read before and written after a barrier, so every thread must call this.
// P -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
template <class GradAt>
__device__ inline void adam_update(float* Pz, float* m, float* v, int32_t* t, int64_t off, int n,
                                   const ffrt_adam_hparams& hp, GradAt g) {
    // The thread's first point is loaded before the step counter, so that its loads overlap the counter's
    // and the bias corrections instead of waiting for them.
    const int i0 = threadIdx.x;
    const bool first = i0 < n;
    float g0 = 0.0f, m0 = 0.0f, v0 = 0.0f, p0 = 0.0f;
    if (first) {
        g0 = g(i0);
        m0 = m[off + i0];
        v0 = v[off + i0];
        p0 = Pz[off + i0];
    }
    const int tn = t[0] + 1;
    const float bc1 = 1.0f - powf(hp.beta1, (float)tn);
    const float bc2 = 1.0f - powf(hp.beta2, (float)tn);
    const float step = hp.lr / bc1, rb2 = 1.0f / sqrtf(bc2);
    auto update = [&](int64_t k, float gi, float mk, float vk, float pk) {
        const float mi = hp.beta1 * mk + (1.0f - hp.beta1) * gi;
        const float vi = hp.beta2 * vk + (1.0f - hp.beta2) * gi * gi;
        m[k] = mi;
        v[k] = vi;
        Pz[k] = pk - step * mi / (sqrtf(vi) * rb2 + hp.eps);
    };
    if (first) update(off + i0, g0, m0, v0, p0);
    for (int i = i0 + (int)blockDim.x; i < n; i += blockDim.x) {
        const int64_t k = off + i;
        const float gi = g(i);
        update(k, gi, m[k], v[k], Pz[k]);
    }
    __syncthreads();
    if (threadIdx.x == 0) t[0] = tn;
}

// dL/dP of design d from its 64-bit fixed-point accumulator (unit from the cotangent bound gmax[d]), which is
// cleared with gmax[d]; then Adam on P, or on theta of the range reparametrisation (sec. 2.4.1) followed by
// P = lo + (tanh(theta) + 1) span / 2, when adam.Pz is set and the design's step is valid.  One workgroup
// per design; every thread must call it (it contains barriers).
__device__ inline void finish_design(const DesignDev& D, int d, unsigned long long* gacc, uint32_t* gmax,
                                     float* dLdP, const int32_t* valid, const AdamArgs& adam) {
    unsigned long long* acc = gacc + D.cp_off;
    float* out = dLdP + D.cp_off;
    const double unit = ldexp(1.0, fixed_point_exponent(gmax[d], D.w0));
    __syncthreads();
    if (threadIdx.x == 0) gmax[d] = 0u;
    auto take = [acc, out, unit](int i) {
        const float g = (float)((double)(long long)acc[i] * unit);
        acc[i] = 0ull;
        out[i] = g;
        return g;
    };
    const int ncp = D.ncp;
    const bool step = adam.Pz && (!valid || valid[d]);
    if (step && adam.theta) {
        float* th = adam.theta + D.cp_off;
        const float* lo = adam.lo + D.cp_off;
        const float* sp = adam.span + D.cp_off;
        auto take_theta = [take, th, sp](int i) {
            const float y = tanhf(th[i]);
            return take(i) * (0.5f * (1.0f - y * y) * sp[i]);
        };
        adam_update(adam.theta, adam.m, adam.v, adam.t + d, D.cp_off, ncp, adam.hp, take_theta);
        float* P = adam.Pz + D.cp_off;
        for (int i = threadIdx.x; i < ncp; i += blockDim.x) P[i] = lo[i] + 0.5f * (tanhf(th[i]) + 1.0f) * sp[i];
    } else if (step) {
        adam_update(adam.Pz, adam.m, adam.v, adam.t + d, D.cp_off, ncp, adam.hp, take);
    } else {
        for (int i = threadIdx.x; i < ncp; i += blockDim.x) take(i);
    }
    __syncthreads();
}

}  // namespace ffrt
