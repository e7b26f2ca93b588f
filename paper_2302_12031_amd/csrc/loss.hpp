// Loss of sec. 2.5 from per-slice sums, added up by one wave in every workgroup of the dL/dI kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ffrt_internal.h"

namespace ffrt {

constexpr int LOSS_Q = 5;  // per slice: sum I, sum T, sum I^2, sum I T, sum T^2 (double)

struct LossOut {
    LossScalars L;  // dL/dI = ((I is - T isT) - dot) coef
    float loss;     // NaN without flux
    int valid;      // 0 without flux (the design's Adam update is skipped)
};

// Exponent e of the adjoint's fixed-point unit 2^e for a design with cotangent bound gmax = max |dL/dI| (its
// float bits, as the kernels keep it) and ray weight w0: 32 bits below the leading bit of S = gmax w0, the
// size of a single ray's weighted cotangent (0 when S is zero or not finite, where every contribution is
// zero).
__device__ inline int fixed_point_exponent(uint32_t gmax_bits, float w0) {
    const double S = (double)__builtin_bit_cast(float, gmax_bits) * (double)w0;
    if (!(S > 0.0) || !(S < 1e300)) return 0;
    int e = 0;
    (void)frexp(S, &e);  // S = m 2^e, m in [0.5, 1): floor(log2 S) = e - 1
    return e - 1 - 32;
}

// Loss and dL/dI scalars from the whole-image sums q = (sum I, sum T, sum I^2, sum I T, sum T^2).
__device__ inline LossOut loss_from_sums(const double* q, const DesignDev& D) {
    LossOut r;
    r.L = {0.0f, 0.0f, 0.0f, 0.0f};
    const double s = q[0], sT = q[1];
    if (!(s > 0.0) || !(sT > 0.0)) {
        r.loss = NAN;
        r.valid = 0;
        return r;
    }
    const double a2 = q[2] / (s * s), ab = q[3] / (s * sT), b2 = q[4] / (sT * sT);
    const double d2 = fmax(a2 - 2.0 * ab + b2, 0.0);
    const double nrm = sqrt(d2), rn = sqrt((double)D.nx * (double)D.ny);
    r.L.is = (float)(1.0 / s);
    r.L.isT = (float)(1.0 / sT);
    r.L.dot = (float)(a2 - ab);
    if (D.loss_kind == 1) {
        // sum of squares L = ||D||^2: dL/dI = 2 (D - sum(D I_hat)) / s
        r.L.coef = (float)(2.0 / s);
        r.loss = (float)d2;
    } else {
        r.L.coef = nrm > 0.0 ? (float)(1.0 / (s * rn * nrm)) : 0.0f;
        r.loss = (float)(nrm / rn);
    }
    r.valid = 1;
    return r;
}

// I_hat = I / s, T_hat = T / s_T, D = I_hat - T_hat, L = ||D||_F / sqrt(n_x n_y),
// dL/dI = (D - sum(D I_hat)) / (s sqrt(n_x n_y) ||D||) (0 where ||D|| = 0) (or, for the sum of squares
// L = ||D||^2, dL/dI = 2 (D - sum(D I_hat)) / s), with
// ||D||^2 = A / s^2 - 2 B / (s s_T) + C / s_T^2 and sum(D I_hat) = A / s^2 - B / (s s_T) from the slice sums
// (A = sum I^2, B = sum I T, C = sum T^2), which in double precision lose nothing that matters to the float
// results.  The LB <= 64 slices are added by a butterfly over the wave, so every lane of every wave that
// calls this gets the same bits (no workgroup has to wait for another).  Call with a full wave.
__device__ inline LossOut loss_from_partials(const double* partial, int d, int LB, const DesignDev& D) {
    const int lane = threadIdx.x & 63;
    double q[LOSS_Q];
#pragma unroll
    for (int k = 0; k < LOSS_Q; ++k) q[k] = lane < LB ? partial[((size_t)d * LB + lane) * LOSS_Q + k] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < LOSS_Q; ++k) q[k] += __shfl_xor(q[k], o);
    return loss_from_sums(q, D);
}

}  // namespace ffrt
