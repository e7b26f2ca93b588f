// Kernels of libffrt that do not depend on the B-spline degrees: clearing, convex-hull bounds and lens
// checks, the loss of sec. 2.5 with dL/dI, Adam, and the ray-sampling generator.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "ffrt_internal.h"

namespace ffrt {

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Compensated (Neumaier) running sum: s + c carries the rounding error of the additions.
struct CSum {
    float s = 0.0f, c = 0.0f;
    __device__ void add(float x) {
        float t = s + x;
        c += (fabsf(s) >= fabsf(x)) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    __device__ float value() const { return s + c; }
};

// Block-wide sum over blockDim.x threads (a multiple of 64, at most 1024).
__device__ inline float block_sum(float v, float* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    float s = 0.0f;
    for (int w = 0; w < nw; ++w) s += sh[w];
    return s;
}

__device__ inline float block_max(float v, float* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    float s = -INFINITY;
    for (int w = 0; w < nw; ++w) s = fmaxf(s, sh[w]);
    return s;
}

// Per design (blocks 0 .. n_designs-1): global bounds of P^z (sec. 2.2.2), slope bounds from the derivative
// control points p (P_{i+1,j} - P_{i,j}) / (u_{i+p+1} - u_{i+1}) (textbook derivative of a B-spline), and the
// lens checks of sec. 2.1.2 (P^z >= z_in + delta) and finiteness.  Every block also clears its share of the
// arrays z0, z1, z2.
__global__ __launch_bounds__(256) void k_prepare(const DesignDev* designs, int n_designs, const float* __restrict__ Pz,
                                                 int p, int q, BoundsDev* bounds, float* z0, int64_t n0, float* z1,
                                                 int64_t n1, float* z2, int64_t n2) {
    {
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (z0) for (int64_t k = i0; k < n0; k += stride) z0[k] = 0.0f;
        if (z1) for (int64_t k = i0; k < n1; k += stride) z1[k] = 0.0f;
        if (z2) for (int64_t k = i0; k < n2; k += stride) z2[k] = 0.0f;
    }
    if (!Pz || (int)blockIdx.x >= n_designs) return;
    __shared__ float sh[16];
    const DesignDev& D = designs[blockIdx.x];
    const float* P = Pz + D.cp_off;
    const int n = D.n_u * D.n_v;
    float lo = INFINITY, hi = -INFINITY, gu = 0.0f, gv = 0.0f;
    float nbad = 0.0f, nnan = 0.0f;
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
        int i = idx / D.n_v, j = idx - (idx / D.n_v) * D.n_v;
        float z = P[idx];
        if (!isfinite(z)) nnan += 1.0f;
        if (!(z >= D.zmin_allowed)) nbad += 1.0f;
        lo = fminf(lo, z);
        hi = fmaxf(hi, z);
        if (i + 1 < D.n_u) {
            int dk = min(i + 1, D.nsu) - max(i + 1 - p, 0);
            gu = fmaxf(gu, fabsf((float)p * (P[idx + D.n_v] - z) / (float)dk));
        }
        if (j + 1 < D.n_v) {
            int dk = min(j + 1, D.nsv) - max(j + 1 - q, 0);
            gv = fmaxf(gv, fabsf((float)q * (P[idx + 1] - z) / (float)dk));
        }
    }
    lo = -block_max(-lo, sh);
    hi = block_max(hi, sh);
    gu = block_max(gu, sh);
    gv = block_max(gv, sh);
    nbad = block_sum(nbad, sh);
    nnan = block_sum(nnan, sh);
    if (threadIdx.x == 0) {
        BoundsDev B;
        B.zmin = lo;
        B.zmax = hi;
        B.zref = 0.5f * (lo + hi);
        // d(ubar)/dx = sxu; a small relative margin keeps the bound conservative under rounding
        B.gx = gu * D.sxu * 1.0001f;
        B.gy = gv * D.syv * 1.0001f;
        B.n_bad = (uint32_t)nbad;
        B.n_nan = (uint32_t)nnan;
        B.pad_ = 0.0f;
        bounds[blockIdx.x] = B;
    }
}

// Sum the NSLOT partial slots of design d into stats[d] (threads of one block).
__device__ void reduce_slots(int d, const BoundsDev* bounds, const ffrt_stats* slots, ffrt_stats* stats) {
    constexpr int NF = sizeof(ffrt_stats) / 4;
    const ffrt_stats* sl = slots + (size_t)d * NSLOT;
    for (int f = threadIdx.x; f < NF; f += blockDim.x) {
        if (f == 0) {
            float acc = 0.0f;
            for (int k = 0; k < NSLOT; ++k) acc += sl[k].flux_on_screen;
            stats[d].flux_on_screen = acc;
        } else {
            uint32_t acc = 0;
            for (int k = 0; k < NSLOT; ++k) acc += reinterpret_cast<const uint32_t*>(sl + k)[f];
            reinterpret_cast<uint32_t*>(stats + d)[f] = acc;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        stats[d].n_constraint_viol = bounds[d].n_bad;
        stats[d].n_nan = bounds[d].n_nan;
    }
}

__global__ void k_stats(const BoundsDev* bounds, const ffrt_stats* slots, ffrt_stats* stats) {
    reduce_slots(blockIdx.x, bounds, slots, stats);
}

// Loss of sec. 2.5 per design: I_hat = I / sum I, I_ref_hat = T / sum T, D = I_hat - I_ref_hat,
// L = ||D||_F / sqrt(n_x n_y), dL/dI = (D - sum(D I_hat)) / (sum(I) sqrt(n_x n_y) ||D||) (0 where ||D|| = 0).
// A design without flux gets L = NaN, dL/dI = 0 and valid = 0 (its Adam update is skipped).
__global__ __launch_bounds__(1024) void k_loss(const DesignDev* designs, const float* __restrict__ irr,
                                               const float* __restrict__ target, float* loss, float* dLdI,
                                               int32_t* valid, const BoundsDev* bounds, const ffrt_stats* slots,
                                               ffrt_stats* stats) {
    __shared__ float sh[16];
    if (stats) reduce_slots(blockIdx.x, bounds, slots, stats);
    const DesignDev& D = designs[blockIdx.x];
    const int64_t n = (int64_t)D.nx * D.ny;
    const float* I = irr + D.img_off;
    const float* T = target + D.img_off;
    float* G = dLdI + D.img_off;
    // compensated per-thread sums: the loss is differenced by finite-difference checks, so its rounding
    // has to stay near one ulp
    CSum a, b;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        a.add(I[i]);
        b.add(T[i]);
    }
    float s = block_sum(a.value(), sh);
    float sT = block_sum(b.value(), sh);
    if (!(s > 0.0f) || !(sT > 0.0f)) {
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) G[i] = 0.0f;
        if (threadIdx.x == 0) {
            loss[blockIdx.x] = NAN;
            valid[blockIdx.x] = 0;
        }
        return;
    }
    const float is = 1.0f / s, isT = 1.0f / sT;
    CSum cd2, cdot;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        float ih = I[i] * is;
        float Dv = ih - T[i] * isT;
        cd2.add(Dv * Dv);
        cdot.add(Dv * ih);
    }
    float d2 = block_sum(cd2.value(), sh);
    float dot = block_sum(cdot.value(), sh);
    const float nrm = sqrtf(d2), rn = sqrtf((float)n);
    const float coef = nrm > 0.0f ? 1.0f / (s * rn * nrm) : 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        float Dv = I[i] * is - T[i] * isT;
        G[i] = (Dv - dot) * coef;
    }
    if (threadIdx.x == 0) {
        loss[blockIdx.x] = nrm / rn;
        valid[blockIdx.x] = 1;
    }
}

__device__ inline double block_sum_f64(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w];
    return s;
}

// The loss value of sec. 2.5 with double-precision reductions (finite-difference checks only).
__global__ __launch_bounds__(1024) void k_loss_f64(const DesignDev* designs, const float* __restrict__ irr,
                                                   const float* __restrict__ target, double* loss) {
    __shared__ double sh[16];
    const DesignDev& D = designs[blockIdx.x];
    const int64_t n = (int64_t)D.nx * D.ny;
    const float* I = irr + D.img_off;
    const float* T = target + D.img_off;
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        a += (double)I[i];
        b += (double)T[i];
    }
    double s = block_sum_f64(a, sh), sT = block_sum_f64(b, sh);
    if (!(s > 0.0) || !(sT > 0.0)) {
        if (threadIdx.x == 0) loss[blockIdx.x] = NAN;
        return;
    }
    double d2 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double Dv = (double)I[i] / s - (double)T[i] / sT;
        d2 += Dv * Dv;
    }
    d2 = block_sum_f64(d2, sh);
    if (threadIdx.x == 0) loss[blockIdx.x] = sqrt(d2 / (double)n);
}

// Adam (Kingma & Ba) per design; the step counter lives on the device so the update can be replayed from
// a graph.  P -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ __launch_bounds__(256) void k_adam(const DesignDev* designs, float* Pz, const float* __restrict__ g,
                                              float* m, float* v, int32_t* t, const int32_t* valid,
                                              ffrt_adam_hparams hp) {
    const int d = blockIdx.x;
    if (valid && !valid[d]) return;
    const DesignDev& D = designs[d];
    const int n = D.n_u * D.n_v;
    const int tn = t[d] + 1;
    const float bc1 = 1.0f - powf(hp.beta1, (float)tn);
    const float bc2 = 1.0f - powf(hp.beta2, (float)tn);
    const float step = hp.lr / bc1, rb2 = 1.0f / sqrtf(bc2);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int64_t k = D.cp_off + i;
        float gi = g[k];
        float mi = hp.beta1 * m[k] + (1.0f - hp.beta1) * gi;
        float vi = hp.beta2 * v[k] + (1.0f - hp.beta2) * gi * gi;
        m[k] = mi;
        v[k] = vi;
        Pz[k] -= step * mi / (sqrtf(vi) * rb2 + hp.eps);
    }
    __syncthreads();
    if (threadIdx.x == 0) t[d] = tn;
}

__global__ void k_rng(uint64_t state0, uint64_t first, int64_t n, uint64_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = mix64(state0 + (first + (uint64_t)i + 1) * GAMMA);
}

}  // namespace

uint64_t splitmix_state0(uint64_t seed, uint64_t stream_id) { return mix64(seed + stream_id * GAMMA); }

hipError_t launch_prepare(const DesignDev* designs, int n_designs, const float* Pz, int p, int q,
                          BoundsDev* bounds, float* z0, int64_t n0, float* z1, int64_t n1, float* z2, int64_t n2,
                          hipStream_t s) {
    int64_t work = std::max<int64_t>(std::max<int64_t>(z0 ? n0 : 0, z1 ? n1 : 0), z2 ? n2 : 0);
    int64_t extra = (work + 255) / 256;
    if (extra > 2048) extra = 2048;
    int grid = (int)std::max<int64_t>(Pz ? n_designs : 0, extra);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_prepare, dim3(grid), dim3(256), 0, s, designs, n_designs, Pz, p, q, bounds, z0, n0, z1, n1,
                       z2, n2);
    return hipGetLastError();
}

hipError_t launch_stats(int n_designs, const BoundsDev* bounds, const ffrt_stats* slots, ffrt_stats* stats,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_stats, dim3(n_designs), dim3(64), 0, s, bounds, slots, stats);
    return hipGetLastError();
}

hipError_t launch_loss(const DesignDev* designs, int n_designs, const float* irr, const float* target,
                       float* loss, float* dLdI, int32_t* valid, const BoundsDev* bounds, const ffrt_stats* slots,
                       ffrt_stats* stats, hipStream_t s) {
    hipLaunchKernelGGL(k_loss, dim3(n_designs), dim3(1024), 0, s, designs, irr, target, loss, dLdI, valid, bounds,
                       slots, stats);
    return hipGetLastError();
}

hipError_t launch_loss_f64(const DesignDev* designs, int n_designs, const float* irr, const float* target,
                           double* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_loss_f64, dim3(n_designs), dim3(1024), 0, s, designs, irr, target, loss);
    return hipGetLastError();
}

hipError_t launch_adam(const DesignDev* designs, int n_designs, float* Pz, const float* g, float* m,
                       float* v, int32_t* t, const int32_t* valid, ffrt_adam_hparams hp, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(n_designs), dim3(256), 0, s, designs, Pz, g, m, v, t, valid, hp);
    return hipGetLastError();
}

hipError_t launch_rng(uint64_t seed, uint64_t stream_id, uint64_t first, int64_t n, uint64_t* out,
                      hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int grid = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_rng, dim3(grid), dim3(256), 0, s, splitmix_state0(seed, stream_id), first, n, out);
    return hipGetLastError();
}

}  // namespace ffrt
