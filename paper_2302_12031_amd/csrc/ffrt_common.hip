// Kernels of libffrt that do not depend on the B-spline degrees: clearing, convex-hull bounds and lens
// checks, the loss of sec. 2.5 with dL/dI, Adam, and the ray-sampling generator.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ffrt_internal.h"

namespace ffrt {

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

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

__global__ void k_zero(float* __restrict__ a, int64_t n, ffrt_stats* stats, int n_stats) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n; k += stride) a[k] = 0.0f;
    if (stats) {
        uint32_t* s = reinterpret_cast<uint32_t*>(stats);
        int64_t ns = (int64_t)n_stats * (sizeof(ffrt_stats) / 4);
        for (int64_t k = i; k < ns; k += stride) s[k] = 0u;
    }
}

// Per design: global bounds of P^z (sec. 2.2.2), slope bounds from the derivative control points
// p (P_{i+1,j} - P_{i,j}) / (u_{i+p+1} - u_{i+1}) (textbook derivative of a B-spline), and the lens checks
// of sec. 2.1.2 (P^z >= z_in + delta) and finiteness, counted into the stats.
__global__ __launch_bounds__(256) void k_bounds(const DesignDev* designs, const float* __restrict__ Pz, int p,
                                                int q, BoundsDev* bounds, ffrt_stats* stats) {
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
        B.pad_[0] = B.pad_[1] = B.pad_[2] = 0.0f;
        // d(ubar)/dx = sxu; a small relative margin keeps the bound conservative under rounding
        B.gx = gu * D.sxu * 1.0001f;
        B.gy = gv * D.syv * 1.0001f;
        bounds[blockIdx.x] = B;
        if (stats) {
            stats[blockIdx.x].n_constraint_viol = (uint32_t)nbad;
            stats[blockIdx.x].n_nan = (uint32_t)nnan;
        }
    }
}

// Loss of sec. 2.5 per design: I_hat = I / sum I, I_ref_hat = T / sum T, D = I_hat - I_ref_hat,
// L = ||D||_F / sqrt(n_x n_y), dL/dI = (D - sum(D I_hat)) / (sum(I) sqrt(n_x n_y) ||D||) (0 where ||D|| = 0).
// A design without flux gets L = NaN, dL/dI = 0 and valid = 0 (its Adam update is skipped).
__global__ __launch_bounds__(1024) void k_loss(const DesignDev* designs, const float* __restrict__ irr,
                                               const float* __restrict__ target, float* loss, float* dLdI,
                                               int32_t* valid) {
    __shared__ float sh[16];
    const DesignDev& D = designs[blockIdx.x];
    const int64_t n = (int64_t)D.nx * D.ny;
    const float* I = irr + D.img_off;
    const float* T = target + D.img_off;
    float* G = dLdI + D.img_off;
    float a = 0.0f, b = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        a += I[i];
        b += T[i];
    }
    float s = block_sum(a, sh);
    float sT = block_sum(b, sh);
    if (!(s > 0.0f) || !(sT > 0.0f)) {
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) G[i] = 0.0f;
        if (threadIdx.x == 0) {
            loss[blockIdx.x] = NAN;
            valid[blockIdx.x] = 0;
        }
        return;
    }
    const float is = 1.0f / s, isT = 1.0f / sT;
    float d2 = 0.0f, dot = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        float ih = I[i] * is;
        float Dv = ih - T[i] * isT;
        d2 += Dv * Dv;
        dot += Dv * ih;
    }
    d2 = block_sum(d2, sh);
    dot = block_sum(dot, sh);
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

hipError_t launch_zero(float* a, int64_t n, ffrt_stats* stats, int n_stats, hipStream_t s) {
    int64_t work = n > (int64_t)n_stats * 16 ? n : (int64_t)n_stats * 16;
    int grid = (int)((work + 255) / 256);
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, a, n, stats, n_stats);
    return hipGetLastError();
}

hipError_t launch_bounds(const DesignDev* designs, int n_designs, const float* Pz, int p, int q,
                         BoundsDev* bounds, ffrt_stats* stats, hipStream_t s) {
    hipLaunchKernelGGL(k_bounds, dim3(n_designs), dim3(256), 0, s, designs, Pz, p, q, bounds, stats);
    return hipGetLastError();
}

hipError_t launch_loss(const DesignDev* designs, int n_designs, const float* irr, const float* target,
                       float* loss, float* dLdI, int32_t* valid, hipStream_t s) {
    hipLaunchKernelGGL(k_loss, dim3(n_designs), dim3(1024), 0, s, designs, irr, target, loss, dLdI, valid);
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
