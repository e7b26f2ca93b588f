// Kernels of libffrt that do not depend on the B-spline degrees: resolving the fixed-point irradiance and
// the ray statistics, the loss of sec. 2.5 with dL/dI, Adam, and the ray-sampling generator.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <mutex>

#include "ffrt_internal.h"
#include "loss.hpp"
#include "optim.hpp"
#include "wave.hpp"

namespace ffrt {

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Sum the NSLOT partial-statistics slots of design d into stats[d] and clear them (waves 0..3 of the
// workgroup: wave w sums fields w, w + 4, w + 8 across the 64 slots, one slot per lane), and count the lens
// checks of sec. 2.1.2 (P^z >= z_in + delta_min, finite) over the design's control points.  For workgroups
// of 256 to 1024 threads; contains a barrier.
__device__ void reduce_slots(int d, const DesignDev& D, const float* Pz, ffrt_stats* slots, ffrt_stats* stats) {
    constexpr int NF = sizeof(ffrt_stats) / 4;
    static_assert(NSLOT == 64 && NF == 13, "one slot per lane, at most three fields per wave");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t* slot = reinterpret_cast<uint32_t*>(slots + (size_t)d * NSLOT + lane);
    uint32_t* out = reinterpret_cast<uint32_t*>(stats + d);
    for (int f = wave; wave < 4 && f < NF - 2; f += 4) {  // the last two fields are the lens checks
        const uint32_t x = slot[f];
        slot[f] = 0u;
        if (f == 0) {  // flux_on_screen (float)
            const float sum = wave_sum(__builtin_bit_cast(float, x));
            if (lane == 0) out[f] = __builtin_bit_cast(uint32_t, sum);
        } else {
            const uint32_t sum = wave_sum(x);
            if (lane == 0) out[f] = sum;
        }
    }
    __shared__ uint32_t s_chk[16][2];
    uint32_t nbad = 0, nnan = 0;
    const float* P = Pz + D.cp_off;
    const int K = D.n_u * D.n_v;
    for (int i = threadIdx.x; i < D.ncp; i += blockDim.x) {
        const float z = P[i];
        nnan += isfinite(z) ? 0u : 1u;
        // sec. 2.1.2: above the flat entry face by delta_min; with a freeform entry face, at least delta_min
        // between the two nets at every control point (then everywhere, by the convex hull property)
        if (i < K) nbad += (D.entry_ff ? z - P[K + i] >= D.delta_min : z >= D.zmin_allowed) ? 0u : 1u;
    }
    nbad = wave_sum(nbad);
    nnan = wave_sum(nnan);
    if (lane == 0) {
        s_chk[wave][0] = nbad;
        s_chk[wave][1] = nnan;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0, n = 0;
        for (int w = 0; w < nw; ++w) {
            b += s_chk[w][0];
            n += s_chk[w][1];
        }
        stats[d].n_constraint_viol = b;
        stats[d].n_nan = n;
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

// Bounds of sec. 2.2.2 for design blockIdx.x: the global convex-hull box [min P^z, max P^z], zref at its
// middle, and slope bounds from the derivative control points p (P_{i+1,j} - P_{i,j}) / (u_{i+p+1} - u_{i+1})
// (the textbook derivative of a B-spline; knot units, so d(ubar)/dx = sxu converts them to mm).
__device__ void face_bounds(const DesignDev& D, const float* P, int p, int q, float* s_b, float& zmin, float& zmax,
                            float& gx, float& gy) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float lo = INFINITY, hi = -INFINITY, gu = 0.0f, gv = 0.0f;
    for (int i = wave; i < D.n_u; i += 4) {  // row i by wave, columns by lane
        const float fu = (float)p / (float)(min(i + 1, D.nsu) - max(i + 1 - p, 0));
        for (int j = lane; j < D.n_v; j += 64) {
            const int idx = i * D.n_v + j;
            const float z = P[idx];
            lo = fminf(lo, z);
            hi = fmaxf(hi, z);
            if (i + 1 < D.n_u) gu = fmaxf(gu, fabsf(fu * (P[idx + D.n_v] - z)));
            if (j + 1 < D.n_v) {
                const float fv = (float)q / (float)(min(j + 1, D.nsv) - max(j + 1 - q, 0));
                gv = fmaxf(gv, fabsf(fv * (P[idx + 1] - z)));
            }
        }
    }
    auto fmin_ = [](float a, float b) { return fminf(a, b); };
    auto fmax_ = [](float a, float b) { return fmaxf(a, b); };
    lo = wave_reduce(lo, fmin_);
    hi = wave_reduce(hi, fmax_);
    gu = wave_reduce(gu, fmax_);
    gv = wave_reduce(gv, fmax_);
    __syncthreads();
    if (lane == 0) {
        s_b[wave * 4 + 0] = lo;
        s_b[wave * 4 + 1] = hi;
        s_b[wave * 4 + 2] = gu;
        s_b[wave * 4 + 3] = gv;
    }
    __syncthreads();
    zmin = fminf(fminf(s_b[0], s_b[4]), fminf(s_b[8], s_b[12]));
    zmax = fmaxf(fmaxf(s_b[1], s_b[5]), fmaxf(s_b[9], s_b[13]));
    // a small relative margin keeps the slope bounds conservative under rounding
    gx = fmaxf(fmaxf(s_b[2], s_b[6]), fmaxf(s_b[10], s_b[14])) * D.sxu * 1.0001f;
    gy = fmaxf(fmaxf(s_b[3], s_b[7]), fmaxf(s_b[11], s_b[15])) * D.syv * 1.0001f;
}

__global__ __launch_bounds__(256) void k_bounds(const DesignDev* designs, const float* __restrict__ Pz, int p, int q,
                                                BoundsDev* bounds, SpanBounds* span_bounds) {
    __shared__ float s_b[16];
    __shared__ float s_net[MAX_CP];  // one face's control net: every bound below reads it from LDS
    const int d = blockIdx.x;
    const DesignDev D = designs[d];  // one load: stores below may alias designs[]
    const int ncp = D.n_u * D.n_v;
    for (int i = threadIdx.x; i < ncp; i += blockDim.x) s_net[i] = Pz[D.cp_off + i];
    __syncthreads();
    const float* P = s_net;
    // per span product (su, sv): control points su..su+p x sv..sv+q; derivative control points along u are
    // i = su..su+p-1 (times the factor of their knot interval), along v likewise
    // (the span products are split over the gridDim.y workgroups of the design; workgroup 0 also forms the
    // global bounds below)
    SpanBounds* sb = span_bounds + D.sb_off;
    for (int s = blockIdx.y * blockDim.x + threadIdx.x; s < D.nsu * D.nsv; s += gridDim.y * blockDim.x) {
        const int su = s / D.nsv, sv = s - (s / D.nsv) * D.nsv;
        float fv[MAX_DEG];  // the factors of the span's derivative control points along v
        for (int b = 0; b < q; ++b) {
            const int j = sv + b;
            fv[b] = (float)q / (float)(min(j + 1, D.nsv) - max(j + 1 - q, 0));
        }
        float lo = INFINITY, hi = -INFINITY, gu = 0.0f, gv = 0.0f;
        for (int a = 0; a <= p; ++a) {
            const int i = su + a;
            const float fu = a < p ? (float)p / (float)(min(i + 1, D.nsu) - max(i + 1 - p, 0)) : 0.0f;
            for (int b = 0; b <= q; ++b) {
                const int j = sv + b;
                const float z = P[i * D.n_v + j];
                lo = fminf(lo, z);
                hi = fmaxf(hi, z);
                if (a < p) gu = fmaxf(gu, fabsf(fu * (P[(i + 1) * D.n_v + j] - z)));
                if (b < q) gv = fmaxf(gv, fabsf(fv[b] * (P[i * D.n_v + j + 1] - z)));
            }
        }
        SpanBounds r;
        r.zmin = lo;
        r.zmax = hi;
        r.gx = gu * D.sxu * 1.0001f;
        r.gy = gv * D.syv * 1.0001f;
        sb[s] = r;
    }
    if (blockIdx.y != 0) return;
    BoundsDev B;
    face_bounds(D, P, p, q, s_b, B.zmin, B.zmax, B.gx, B.gy);
    B.zref = 0.5f * (B.zmin + B.zmax);
    B.zmin_in = B.zmax_in = B.gx_in = B.gy_in = B.zref_in = 0.0f;
    if (D.entry_ff) {  // the entry net follows the exit net
        __syncthreads();
        for (int i = threadIdx.x; i < ncp; i += blockDim.x) s_net[i] = Pz[D.cp_off + ncp + i];
        __syncthreads();
        face_bounds(D, P, p, q, s_b, B.zmin_in, B.zmax_in, B.gx_in, B.gy_in);
        B.zref_in = 0.5f * (B.zmin_in + B.zmax_in);
    }
    if (threadIdx.x == 0) bounds[d] = B;
}

// Slice [lo, hi) of the image of design D handled by workgroup b of LB.
__device__ inline void image_slice(const DesignDev& D, int LB, int b, int64_t& lo, int64_t& hi) {
    const int64_t n = (int64_t)D.nx * D.ny;
    const int64_t chunk = (n + LB - 1) / LB;
    lo = min<int64_t>(n, (int64_t)b * chunk);
    hi = min<int64_t>(n, lo + chunk);
}

// Fixed-point irradiance -> float (the forward accumulates rint(v fx_scale) per pixel), clearing img64 for
// the next forward.  Workgroup 0 of each design also reduces the statistics.
__global__ __launch_bounds__(256) void k_resolve(const DesignDev* designs, int LB, unsigned long long* img64,
                                                 float* irr, const float* Pz, ffrt_stats* slots, ffrt_stats* stats) {
    const int d = blockIdx.x / LB, b = blockIdx.x - d * LB;
    const DesignDev D = designs[d];  // one load: stores below may alias designs[]
    int64_t lo, hi;
    image_slice(D, LB, b, lo, hi);
    for (int64_t i = D.img_off + lo + threadIdx.x; i < D.img_off + hi; i += blockDim.x) {
        irr[i] = (float)(long long)img64[i] * D.fx_unscale;
        img64[i] = 0ull;
    }
    if (stats && b == 0) reduce_slots(d, D, Pz, slots, stats);
}

// Slice sums of the loss of sec. 2.5 (sum I, sum T, sum I^2, sum I T, sum T^2 in double precision) of
// slice b of design d, resolving the fixed-point irradiance first when img64 is given.  No workgroup waits
// for another: the consumers (k_loss_grad, the adjoint) each add up the LB slices themselves.  With stats,
// n_designs more workgroups after the slices reduce each design's statistics, beside the slices rather than
// after one of them.
__global__ __launch_bounds__(256) void k_loss_sums(const DesignDev* designs, int n_designs, int LB,
                                                   unsigned long long* img64, float* irr,
                                                   const float* __restrict__ target, const float* Pz,
                                                   ffrt_stats* slots, ffrt_stats* stats, double* partial) {
    __shared__ double sh[4][LOSS_Q];
    if ((int)blockIdx.x >= n_designs * LB) {
        const int d = blockIdx.x - n_designs * LB;
        reduce_slots(d, designs[d], Pz, slots, stats);
        return;
    }
    const int d = blockIdx.x / LB, b = blockIdx.x - d * LB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const DesignDev D = designs[d];  // one load: stores below may alias designs[]
    int64_t lo, hi;
    image_slice(D, LB, b, lo, hi);
    double q[LOSS_Q] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = D.img_off + lo + threadIdx.x; i < D.img_off + hi; i += blockDim.x) {
        float xf;
        if (img64) {
            xf = (float)(long long)img64[i] * D.fx_unscale;
            irr[i] = xf;
            img64[i] = 0ull;
        } else {
            xf = irr[i];
        }
        const double x = (double)xf, y = (double)target[i];
        q[0] += x;
        q[1] += y;
        q[2] += x * x;
        q[3] += x * y;
        q[4] += y * y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < LOSS_Q; ++k) q[k] += __shfl_xor(q[k], o);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < LOSS_Q; ++k) sh[wave][k] = q[k];
    __syncthreads();
    if (threadIdx.x < LOSS_Q) {
        const int k = threadIdx.x;
        partial[((size_t)d * LB + b) * LOSS_Q + k] = ((sh[0][k] + sh[1][k]) + sh[2][k]) + sh[3][k];
    }
}

// dL/dI of slice b of design d; workgroup 0 also stores the loss value and the validity flag.
__global__ __launch_bounds__(256) void k_loss_grad(const DesignDev* designs, int LB, const float* __restrict__ irr,
                                                   const float* __restrict__ target, const double* partial,
                                                   float* loss, int32_t* valid, float* dLdI, uint32_t* gmax) {
    const int d = blockIdx.x / LB, b = blockIdx.x - d * LB;
    const DesignDev D = designs[d];  // one load: stores below may alias designs[]
    int64_t lo, hi;
    image_slice(D, LB, b, lo, hi);
    // the slice's first pixels (all of them up to 1024 per slice) are loaded before the slice sums are
    // added up, so that both sets of loads overlap
    constexpr int PF = 4;
    const int64_t base = D.img_off + lo + threadIdx.x, end = D.img_off + hi;
    float I[PF], T[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int64_t i = base + (int64_t)k * blockDim.x;
        I[k] = i < end ? irr[i] : 0.0f;
        T[k] = i < end ? target[i] : 0.0f;
    }
    const LossOut R = loss_from_partials(partial, d, LB, D);
    if (b == 0 && threadIdx.x == 0) {
        loss[d] = R.loss;
        valid[d] = R.valid;
    }
    float gm = 0.0f;  // max |dL/dI| over the thread's pixels
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int64_t i = base + (int64_t)k * blockDim.x;
        if (i < end) {
            const float g = ((I[k] * R.L.is - T[k] * R.L.isT) - R.L.dot) * R.L.coef;
            dLdI[i] = g;
            gm = fmaxf(gm, fabsf(g));
        }
    }
    for (int64_t i = base + (int64_t)PF * blockDim.x; i < end; i += blockDim.x) {
        const float Dv = irr[i] * R.L.is - target[i] * R.L.isT;
        const float g = (Dv - R.L.dot) * R.L.coef;
        dLdI[i] = g;
        gm = fmaxf(gm, fabsf(g));
    }
    if (gmax) {
        // the cotangent bound of the adjoint's fixed-point unit: the largest |dL/dI| of the design, as float
        // bits (ordered like the values, being non-negative); kept at zero between steps by the finishing kernel
        gm = wave_reduce(gm, [](float a, float b) { return fmaxf(a, b); });
        if ((threadIdx.x & 63) == 0 && gm > 0.0f) atomicMax(gmax + d, __builtin_bit_cast(uint32_t, gm));
    }
}

// The adjoint's cotangent bound of design blockIdx.x from the dL/dI it is given: max |dL/dI| (float bits).
__global__ __launch_bounds__(256) void k_gscale(const DesignDev* designs, const float* __restrict__ dLdI,
                                                uint32_t* gmax) {
    __shared__ float sh[4];
    const DesignDev D = designs[blockIdx.x];
    const int64_t n = (int64_t)D.nx * D.ny;
    const float* G = dLdI + D.img_off;
    float m = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, fabsf(G[i]));
    m = wave_reduce(m, [](float a, float b) { return fmaxf(a, b); });
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) gmax[blockIdx.x] = __builtin_bit_cast(uint32_t, fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3])));
}

// One workgroup per design after the adjoint: dL/dP from the fixed-point accumulator (which is cleared for
// the next adjoint, as is the cotangent bound) and, when asked, Adam for the designs whose loss found flux.
__global__ __launch_bounds__(256) void k_finish(const DesignDev* designs, unsigned long long* gacc, uint32_t* gmax,
                                                float* dLdP, const int32_t* valid, AdamArgs adam) {
    const int d = blockIdx.x;
    const DesignDev D = designs[d];
    finish_design(D, d, gacc, gmax, dLdP, valid, adam);
}

// Range reparametrisation of sec. 2.4.1 (eq. of the output correction, with or without the offset
// function folded into lo): P = lo + (tanh(theta) + 1) span / 2, and its chain rule.
__global__ void k_reparam(int mode, int64_t n, const float* __restrict__ theta, const float* __restrict__ lo,
                          const float* __restrict__ span, float* P, const float* __restrict__ dLdP,
                          float* dLdtheta) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float y = tanhf(theta[k]);
    if (mode == 0) P[k] = lo[k] + 0.5f * (y + 1.0f) * span[k];
    else dLdtheta[k] = dLdP[k] * (0.5f * (1.0f - y * y) * span[k]);
}

// The loss value of sec. 2.5 (or its sum of squares) with double-precision reductions (finite-difference
// checks only).
__global__ __launch_bounds__(1024) void k_loss_f64(const DesignDev* designs, const float* __restrict__ irr,
                                                   const float* __restrict__ target, double* loss) {
    __shared__ double sh[16];
    const DesignDev D = designs[blockIdx.x];
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
    if (threadIdx.x == 0) loss[blockIdx.x] = D.loss_kind == 1 ? d2 : sqrt(d2 / (double)n);
}

// Adam per design; the step counter lives on the device so the update can be replayed from a graph.
__global__ __launch_bounds__(256) void k_adam(const DesignDev* designs, float* Pz, const float* __restrict__ g,
                                              float* m, float* v, int32_t* t, const int32_t* valid,
                                              ffrt_adam_hparams hp) {
    const int d = blockIdx.x;
    if (valid && !valid[d]) return;
    const DesignDev D = designs[d];  // one load: stores below may alias designs[]
    const float* gd = g + D.cp_off;
    adam_update(Pz, m, v, t + d, D.cp_off, D.ncp, hp, [gd](int i) { return gd[i]; });
}

__global__ void k_rng(uint64_t state0, uint64_t first, int64_t n, uint64_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = mix64(state0 + (first + (uint64_t)i + 1) * GAMMA);
}

// LDS-atomic throughput: every thread adds `iters` rounds of 9 values to a per-workgroup tile of TILE_CAP words
// with ds_add_u32.  Pattern 0: lane l of wave w adds to word 64 w + l + 256 k for tap k (distinct banks, no
// shared addresses: the unit's peak).  Pattern 1: the forward's splat: the lanes of a wave are an 8 x 8 grid
// of rays landing two pixels apart (a hash of lane and round moves each by a pixel) in a tile 40 pixels wide,
// and each adds the 3 x 3 filter window around its landing pixel, one tap per instruction.  The tile's sum
// goes to out[blockIdx.x] so that nothing is left out.
__global__ __launch_bounds__(256) void k_lds_atomics(int pattern, int iters, uint32_t* out) {
    __shared__ uint32_t tile[TILE_CAP];
    for (int i = threadIdx.x; i < TILE_CAP; i += 256) tile[i] = 0u;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int TW = 40;
    for (int it = 0; it < iters; ++it) {
        const uint32_t h = (uint32_t)(lane * 0x9E3779B1u) ^ (uint32_t)(it * 0x85EBCA77u);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            int a;
            if (pattern == 0) {
                a = wave * 64 + lane + 256 * k;
            } else {
                const int px = 2 * (lane & 7) + ((h >> 3) & 1) + (wave & 1) * 16 + k % 3;
                const int py = 2 * (lane >> 3) + ((h >> 7) & 1) + (wave >> 1) * 16 + k / 3;
                a = py * TW + px;
            }
            __hip_atomic_fetch_add(&tile[a], 1u + (h & 1u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    uint32_t s = 0;
    for (int i = threadIdx.x; i < TILE_CAP; i += 256) s += tile[i];
    s = wave_sum(s);
    __shared__ uint32_t part[4];
    if (lane == 0) part[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Fill n 32-bit words with v (a kernel, not a memset node, so that graph captures of its callers replay it
// like any other kernel).
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Device memory owned by the library for the entry points that take no caller workspace: one copy per GPU,
// resident from module load until the process ends.  Host code never uses this name as an address (on the
// host it is only a stand-in for the symbol): static_scratch() resolves each device's own address once.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

}  // namespace

hipError_t static_scratch(void** ptr, int* num_cu) {
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static void* addr[MAX_DEV] = {};
    static int ncu[MAX_DEV] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        int n = 0;
        e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        addr[dev] = p;
        ncu[dev] = n > 0 ? n : 256;
    }
    *ptr = addr[dev];
    *num_cu = ncu[dev];
    return hipSuccess;
}

hipError_t launch_fill_u32(void* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, s, static_cast<uint32_t*>(p), n, v);
    return hipGetLastError();
}

uint64_t splitmix_state0(uint64_t seed, uint64_t stream_id) { return mix64(seed + stream_id * GAMMA); }

hipError_t launch_bounds(const DesignDev* designs, int n_designs, const float* Pz, int p, int q, BoundsDev* bounds,
                         SpanBounds* span_bounds, hipStream_t s) {
    hipLaunchKernelGGL(k_bounds, dim3(n_designs, 4), dim3(256), 0, s, designs, Pz, p, q, bounds, span_bounds);
    return hipGetLastError();
}

int loss_blocks_per_design(int64_t max_pixels) {
    return (int)std::min<int64_t>(64, std::max<int64_t>(1, (max_pixels + 1023) / 1024));
}

hipError_t launch_resolve(const DesignDev* designs, int n_designs, int LB, unsigned long long* img64, float* irr,
                          const float* Pz, ffrt_stats* slots, ffrt_stats* stats, hipStream_t s) {
    hipLaunchKernelGGL(k_resolve, dim3(n_designs * LB), dim3(256), 0, s, designs, LB, img64, irr, Pz, slots, stats);
    return hipGetLastError();
}

hipError_t launch_loss(const DesignDev* designs, int n_designs, int LB, unsigned long long* img64, float* irr,
                       const float* target, const float* Pz, ffrt_stats* slots, ffrt_stats* stats, double* partial,
                       float* loss, float* dLdI, int32_t* valid, uint32_t* gmax, hipStream_t s) {
    hipLaunchKernelGGL(k_loss_sums, dim3(n_designs * LB + (stats ? n_designs : 0)), dim3(256), 0, s, designs,
                       n_designs, LB, img64, irr, target, Pz, slots, stats, partial);
    hipLaunchKernelGGL(k_loss_grad, dim3(n_designs * LB), dim3(256), 0, s, designs, LB, irr, target, partial, loss,
                       valid, dLdI, gmax);
    return hipGetLastError();
}

hipError_t launch_gscale(const DesignDev* designs, int n_designs, const float* dLdI, uint32_t* gmax, hipStream_t s) {
    hipLaunchKernelGGL(k_gscale, dim3(n_designs), dim3(256), 0, s, designs, dLdI, gmax);
    return hipGetLastError();
}

hipError_t launch_finish(const DesignDev* designs, int n_designs, unsigned long long* gacc, uint32_t* gmax,
                         float* dLdP, const int32_t* valid, const AdamArgs& adam, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(n_designs), dim3(256), 0, s, designs, gacc, gmax, dLdP, valid, adam);
    return hipGetLastError();
}

hipError_t launch_reparam(int mode, int64_t n, const float* theta, const float* lo, const float* span, float* P,
                          const float* dLdP, float* dLdtheta, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reparam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mode, n, theta, lo, span, P,
                       dLdP, dLdtheta);
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

hipError_t launch_lds_atomics(int pattern, int iters, int grid, uint32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_lds_atomics, dim3(grid), dim3(256), 0, s, pattern, iters, out);
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
