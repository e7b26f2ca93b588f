// The control-point generators of sec. 2.4: multi-layer perceptrons with the trivial input 1 and three tanh
// layers of the size K = n_u n_v of the control net, followed by the output correction of sec. 2.4.1 (eq. of
// the output correction; the offset function folded into lo):
//   h1 = tanh(w1 + b1),  h2 = tanh(W2 h1 + b2),  y = tanh(W3 h2 + b3),  P = lo + (y + 1) span / 2.
// Activations of a design, packed at 3 cp_off: h1, h2, y (K each).  K counts all of a design's heights (both
// nets of a lens with a freeform entry face) for the dense architecture.
//
// Dense architecture: W2, W3 fully connected.  Parameters of a design, packed: w1 (K), b1 (K), W2 (K x K, row
// i = inputs of neuron i), b2 (K), W3 (K x K), b3 (K).  The two K x K layers are matrix-vector products,
// bound by HBM bandwidth (2 K^2 floats per pass), not by matrix cores.  The back-propagation forms
// dz3 = dL/dP (1 - y^2) span / 2, dh2 = W3^T dz3, dz2 = dh2 (1 - h2^2), dh1 = W2^T dz2, dz1 = dh1 (1 - h1^2);
// the weight gradients dz h^T are never stored: the Adam kernel forms each one from the two vectors as it
// updates the weight.
//
// Sparse architecture: W2, W3 locally connected with the footprint of a (2p+1) x (2q+1) convolution, a weight
// per connection and a bias per neuron.  Neuron k = (i, j) (k = i n_v + j) takes the input at
// (i + a - p, j + b - q), a in [0, 2p], b in [0, 2q]: the control points whose basis functions share a knot
// span with its own.  Packed: w1 (K), b1 (K), W2 (C x K, W2[c][k] with c = a (2q + 1) + b), b2 (K), W3 (C x K),
// b3 (K), C = (2p+1)(2q+1).  A connection that would leave the net does not exist: its stored weight is inert
// (zero gradient).  A design's sparse forward and back-propagation are a few times 10^5 flops: one workgroup
// runs each, with the vectors in LDS and the (2p+1)(2q+1) taps unrolled into independent loads; the
// gradient and Adam pass over the 2 C K + 4 K parameters is spread over many workgroups.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "ffrt_internal.h"
#include "wave.hpp"

namespace ffrt {

namespace {

// Bias-corrected Adam on one parameter q (Kingma & Ba); step = lr / (1 - b1^t), rb2 = 1 / sqrt(1 - b2^t).
__device__ __forceinline__ void adam_one(float* par, float* m, float* v, int64_t q, float g, float step, float rb2,
                                         const ffrt_adam_hparams& hp) {
    const float mi = hp.beta1 * m[q] + (1.0f - hp.beta1) * g;
    const float vi = hp.beta2 * v[q] + (1.0f - hp.beta2) * g * g;
    m[q] = mi;
    v[q] = vi;
    par[q] -= step * mi / (sqrtf(vi) * rb2 + hp.eps);
}

__device__ inline void adam_scales(const int32_t* t, int d, const ffrt_adam_hparams& hp, float& step, float& rb2) {
    const int tn = t[d] + 1;
    step = hp.lr / (1.0f - powf(hp.beta1, (float)tn));
    rb2 = 1.0f / sqrtf(1.0f - powf(hp.beta2, (float)tn));
}

// The gradient + Adam pass streams the parameters and both Adam moments once, reading and writing each: their
// 16-byte loads and stores are non-temporal (measured on a 33.6 M-parameter generator: 182 -> 159 us; the
// weight-only passes gained nothing from it).
typedef float stream4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_stream(const float* p) {
    const stream4 a = __builtin_nontemporal_load(reinterpret_cast<const stream4*>(p));
    return make_float4(a.x, a.y, a.z, a.w);
}
__device__ __forceinline__ void store_stream(float* p, float4 a) {
    __builtin_nontemporal_store(stream4{a.x, a.y, a.z, a.w}, reinterpret_cast<stream4*>(p));
}

// Adam on four consecutive parameters (16-byte aligned) with gradients g.
__device__ __forceinline__ void adam_four(float* __restrict__ par, float* __restrict__ grad, float* __restrict__ m,
                                          float* __restrict__ v, int64_t q, float4 g, bool upd, float step,
                                          float rb2, const ffrt_adam_hparams& hp) {
    if (grad) store_stream(grad + q, g);
    if (!upd) return;
    float4 mm = load_stream(m + q);
    float4 vv = load_stream(v + q);
    float4 pp = load_stream(par + q);
    const float b1 = hp.beta1, b2 = hp.beta2, c1 = 1.0f - hp.beta1, c2 = 1.0f - hp.beta2;
    mm.x = b1 * mm.x + c1 * g.x;
    mm.y = b1 * mm.y + c1 * g.y;
    mm.z = b1 * mm.z + c1 * g.z;
    mm.w = b1 * mm.w + c1 * g.w;
    vv.x = b2 * vv.x + c2 * g.x * g.x;
    vv.y = b2 * vv.y + c2 * g.y * g.y;
    vv.z = b2 * vv.z + c2 * g.z * g.z;
    vv.w = b2 * vv.w + c2 * g.w * g.w;
    pp.x -= step * mm.x / (sqrtf(vv.x) * rb2 + hp.eps);
    pp.y -= step * mm.y / (sqrtf(vv.y) * rb2 + hp.eps);
    pp.z -= step * mm.z / (sqrtf(vv.z) * rb2 + hp.eps);
    pp.w -= step * mm.w / (sqrtf(vv.w) * rb2 + hp.eps);
    store_stream(m + q, mm);
    store_stream(v + q, vv);
    store_stream(par + q, pp);
}

// Gradient g of parameter q: written to grad when given, and Adam applied when upd.
__device__ __forceinline__ void emit(float* par, float* grad, float* m, float* v, int64_t q, float g, bool upd,
                                     float step, float rb2, const ffrt_adam_hparams& hp) {
    if (grad) grad[q] = g;
    if (upd) adam_one(par, m, v, q, g, step, rb2, hp);
}

// Layer 1 (input 1): h1 = tanh(w1 + b1).  With t set, workgroup 0 of a design whose last loss was valid also
// advances its Adam step counter (the Adam pass before it used t + 1).
__global__ __launch_bounds__(256) void k_mlp_layer1(const DesignDev* designs, const int64_t* poff,
                                                    const float* __restrict__ par, float* acts, int32_t* t,
                                                    const int32_t* valid) {
    const int d = blockIdx.y;
    const DesignDev& D = designs[d];
    const int K = D.ncp;
    const float* w1 = par + poff[d];
    const float* b1 = w1 + K;
    float* h1 = acts + 3 * D.cp_off;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) h1[k] = tanhf(w1[k] + b1[k]);
    if (t && blockIdx.x == 0 && threadIdx.x == 0 && (!valid || valid[d])) t[d] += 1;
}

// z_i = sum_j W_ij x_j + b_i, out_i = tanh(z_i); one wave per row, x staged in LDS, four independent partial
// sums per lane.  With lo set (last layer) also P_i = lo_i + (out_i + 1) span_i / 2.  layer: 2 (W2, h1 -> h2)
// or 3 (W3, h2 -> y).
__global__ __launch_bounds__(256) void k_mlp_gemv(const DesignDev* designs, const int64_t* poff, int layer,
                                                  const float* __restrict__ par, float* acts, const float* lo,
                                                  const float* span, float* Pz) {
    extern __shared__ float sx[];
    const int d = blockIdx.y;
    const DesignDev& D = designs[d];
    const int K = D.ncp;
    if ((int)blockIdx.x * 4 >= K) return;
    const float* base = par + poff[d];
    const float* W = base + 2 * K + (layer == 3 ? (int64_t)K * K + K : 0);
    const float* b = W + (int64_t)K * K;
    const float* x = acts + 3 * D.cp_off + (layer == 3 ? K : 0);
    float* out = acts + 3 * D.cp_off + (layer == 3 ? 2 * K : K);
    for (int j = threadIdx.x; j < K; j += blockDim.x) sx[j] = x[j];
    __syncthreads();
    const int lane = threadIdx.x & 63, i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= K) return;
    const float* row = W + (int64_t)i * K;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    if ((K & 3) == 0 && (reinterpret_cast<uintptr_t>(row) & 15) == 0) {
        // 16-byte loads: a wave reads 1 KiB of the row per instruction
        const float4* r4 = reinterpret_cast<const float4*>(row);
        const float4* x4 = reinterpret_cast<const float4*>(sx);
        for (int j4 = lane; j4 < (K >> 2); j4 += 64) {
            const float4 w = r4[j4], x = x4[j4];
            a0 += w.x * x.x;
            a1 += w.y * x.y;
            a2 += w.z * x.z;
            a3 += w.w * x.w;
        }
    } else {
        int j = lane;
        for (; j + 192 < K; j += 256) {
            a0 += row[j] * sx[j];
            a1 += row[j + 64] * sx[j + 64];
            a2 += row[j + 128] * sx[j + 128];
            a3 += row[j + 192] * sx[j + 192];
        }
        for (; j < K; j += 64) a0 += row[j] * sx[j];
    }
    const float acc = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) {
        const float y = tanhf(acc + b[i]);
        out[i] = y;
        if (lo) Pz[D.cp_off + i] = lo[D.cp_off + i] + 0.5f * (y + 1.0f) * span[D.cp_off + i];
    }
}

// dh_j += sum_{i in rows} W_ij dz_i over a chunk of rows.  Layer 3: dz = g (= dz3); layer 2: dz_i =
// g_i (1 - h2_i^2) (g = dh2), formed as it is staged.  Columns by thread, rows by chunk; partial sums are
// added atomically.
constexpr int GT_ROWS = 32;
__global__ __launch_bounds__(256) void k_mlp_gemv_t(const DesignDev* designs, const int64_t* poff, int layer,
                                                    const float* __restrict__ par, const float* acts,
                                                    const float* g, float* dh) {
    __shared__ float sdz[GT_ROWS];
    const int d = blockIdx.z;
    const DesignDev& D = designs[d];
    const int K = D.ncp;
    const int r0 = blockIdx.y * GT_ROWS;
    if (r0 >= K) return;
    const float* W = par + poff[d] + 2 * K + (layer == 3 ? (int64_t)K * K + K : 0);
    const float* h2 = acts + 3 * D.cp_off + K;
    const float* gd = g + D.cp_off;
    if (threadIdx.x < GT_ROWS) {
        const int i = r0 + threadIdx.x;
        float z = 0.0f;
        if (i < K) z = layer == 3 ? gd[i] : gd[i] * (1.0f - h2[i] * h2[i]);
        sdz[threadIdx.x] = z;
    }
    __syncthreads();
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const int r1 = min(K, r0 + GT_ROWS);
    float acc = 0.0f;
#pragma unroll 8
    for (int i = r0; i < r1; ++i) acc += W[(int64_t)i * K + j] * sdz[i - r0];
    if (acc != 0.0f) atomicAdd(&dh[D.cp_off + j], acc);
}

// Gradient of every parameter (written to grad when given) and, with adam set, the Adam update, for the
// designs whose last loss found flux.  Bias corrections use the step count t + 1 (layer 1 advances t).
//   w1, b1: dz1_k = dh1_k (1 - h1_k^2);  W2_ij: dz2_i h1_j;  b2: dz2_i;  W3_ij: dz3_i h2_j;  b3: dz3_i
// with dz2_i = dh2_i (1 - h2_i^2) and dz3 given.  Workgroup x < rows handles weight rows x * MR .. + MR - 1
// of both matrices (columns by thread, coalesced); the workgroup after them the four bias-like vectors.
constexpr int MR = 4;
__global__ __launch_bounds__(256) void k_mlp_grad_adam(const DesignDev* designs, const int64_t* poff,
                                                       float* __restrict__ par, const float* __restrict__ acts,
                                                       const float* __restrict__ dz3, const float* __restrict__ dh2,
                                                       const float* __restrict__ dh1, float* __restrict__ grad,
                                                       float* __restrict__ m, float* __restrict__ v,
                                                       const int32_t* t, const int32_t* valid, int adam,
                                                       ffrt_adam_hparams hp) {
    const int d = blockIdx.y;
    const DesignDev& D = designs[d];
    const int K = D.ncp;
    const int nrb = (K + MR - 1) / MR;
    if ((int)blockIdx.x > nrb) return;
    const bool upd = adam && (!valid || valid[d]);
    float step = 0.0f, rb2 = 0.0f;
    if (upd) adam_scales(t, d, hp, step, rb2);
    const float* h1 = acts + 3 * D.cp_off;
    const float* h2 = h1 + K;
    const int64_t c = D.cp_off, p0 = poff[d];
    const int64_t KK = (int64_t)K * K;
    if ((int)blockIdx.x == nrb) {
        // w1, b1 (dz1), b2 (dz2), b3 (dz3)
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            const float g1 = dh1[c + k] * (1.0f - h1[k] * h1[k]);
            const float g2 = dh2[c + k] * (1.0f - h2[k] * h2[k]);
            const float g3 = dz3[c + k];
            emit(par, grad, m, v, p0 + k, g1, upd, step, rb2, hp);
            emit(par, grad, m, v, p0 + K + k, g1, upd, step, rb2, hp);
            emit(par, grad, m, v, p0 + 2 * K + KK + k, g2, upd, step, rb2, hp);
            emit(par, grad, m, v, p0 + 3 * K + 2 * KK + k, g3, upd, step, rb2, hp);
        }
        return;
    }
    const int i0 = blockIdx.x * MR, i1 = min(K, i0 + MR);
    // 16-byte accesses when every row starts 16-byte aligned in all four buffers
    auto al = [p0](const float* b) { return !b || (reinterpret_cast<uintptr_t>(b + p0) & 15) == 0; };
    const bool vec = (K & 3) == 0 && al(par) && al(grad) && (!upd || (al(m) && al(v)));
    for (int i = i0; i < i1; ++i) {
        const float z2 = dh2[c + i] * (1.0f - h2[i] * h2[i]);
        const float z3 = dz3[c + i];
        const int64_t q2 = p0 + 2 * K + (int64_t)i * K, q3 = p0 + 3 * K + KK + (int64_t)i * K;
        if (vec) {
            for (int j = 4 * threadIdx.x; j < K; j += 4 * blockDim.x) {
                adam_four(par, grad, m, v, q2 + j,
                          make_float4(z2 * h1[j], z2 * h1[j + 1], z2 * h1[j + 2], z2 * h1[j + 3]), upd, step, rb2, hp);
                adam_four(par, grad, m, v, q3 + j,
                          make_float4(z3 * h2[j], z3 * h2[j + 1], z3 * h2[j + 2], z3 * h2[j + 3]), upd, step, rb2, hp);
            }
        } else {
#pragma unroll 4
            for (int j = threadIdx.x; j < K; j += blockDim.x) {
                emit(par, grad, m, v, q2 + j, z2 * h1[j], upd, step, rb2, hp);
                emit(par, grad, m, v, q3 + j, z3 * h2[j], upd, step, rb2, hp);
            }
        }
    }
}

// dz3 = dL/dP (1 - y^2) span / 2 for the packed control points, and the accumulators of W^T products
// cleared for the back-propagation that follows.
__global__ void k_mlp_seed(const DesignDev* designs, const float* dLdP, const float* acts, const float* span,
                           float* dz3, float* dh2, float* dh1) {
    const int d = blockIdx.y;
    const DesignDev& D = designs[d];
    const int K = D.ncp;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int64_t c = D.cp_off + k;
    const float y = acts[3 * D.cp_off + 2 * K + k];
    dz3[c] = dLdP[c] * (0.5f * (1.0f - y * y) * span[c]);
    dh2[c] = 0.0f;
    dh1[c] = 0.0f;
}

// ---- sparse (locally connected) architecture ------------------------------------------------------------
// Neuron k = (i, j) of a net with n_v columns takes the input at (i + a - P, j + b - Q), a in [0, 2P],
// b in [0, 2Q], weight W[c][k], c = a (2Q + 1) + b.  Taps off the net are read at a clamped index and
// multiplied by zero, so every tap is an independent load.

// z_k = sum_c W[c][k] x[src(k, c)]
template <int P, int Q>
__device__ __forceinline__ float sparse_in(const float* W, const float* x, int K, int nu, int nv, int k) {
    const int i0 = k / nv, j0 = k - (k / nv) * nv;
    float acc[2 * P + 1];
#pragma unroll
    for (int a = 0; a <= 2 * P; ++a) {
        const int i = i0 + a - P;
        const bool iv = i >= 0 && i < nu;
        const int ic = min(max(i, 0), nu - 1);
        float s = 0.0f;
#pragma unroll
        for (int b = 0; b <= 2 * Q; ++b) {
            const int j = j0 + b - Q;
            const bool ok = iv && j >= 0 && j < nv;
            const float w = W[(int64_t)(a * (2 * Q + 1) + b) * K + k];
            s += ok ? w * x[ic * nv + min(max(j, 0), nv - 1)] : 0.0f;
        }
        acc[a] = s;
    }
    float z = 0.0f;
#pragma unroll
    for (int a = 0; a <= 2 * P; ++a) z += acc[a];
    return z;
}

// dx_s = sum over the (c, k) with src(k, c) = s of W[c][k] dz_k: k = s - (a - P, b - Q)
template <int P, int Q>
__device__ __forceinline__ float sparse_back(const float* W, const float* dz, int K, int nu, int nv, int s) {
    const int i0 = s / nv, j0 = s - (s / nv) * nv;
    float acc[2 * P + 1];
#pragma unroll
    for (int a = 0; a <= 2 * P; ++a) {
        const int i = i0 - a + P;
        const bool iv = i >= 0 && i < nu;
        const int ic = min(max(i, 0), nu - 1);
        float sum = 0.0f;
#pragma unroll
        for (int b = 0; b <= 2 * Q; ++b) {
            const int j = j0 - b + Q;
            const bool ok = iv && j >= 0 && j < nv;
            const int k = ic * nv + min(max(j, 0), nv - 1);
            const float w = W[(int64_t)(a * (2 * Q + 1) + b) * K + k];
            sum += ok ? w * dz[k] : 0.0f;
        }
        acc[a] = sum;
    }
    float z = 0.0f;
#pragma unroll
    for (int a = 0; a <= 2 * P; ++a) z += acc[a];
    return z;
}

// One workgroup per design: the three layers with h1, h2 in LDS; writes acts and (with lo) Pz; with t set,
// advances the step counter of a design whose last loss was valid.
template <int P, int Q>
__global__ __launch_bounds__(1024) void k_smlp_forward(const DesignDev* designs, const int64_t* poff,
                                                       const float* __restrict__ par, float* acts, const float* lo,
                                                       const float* span, float* Pz, int32_t* t,
                                                       const int32_t* valid) {
    extern __shared__ float sm[];
    constexpr int C = (2 * P + 1) * (2 * Q + 1);
    const int d = blockIdx.x;
    const DesignDev& D = designs[d];
    const int K = D.n_u * D.n_v;
    const float* w1 = par + poff[d];
    const float* b1 = w1 + K;
    const float* W2 = b1 + K;
    const float* b2 = W2 + (int64_t)C * K;
    const float* W3 = b2 + K;
    const float* b3 = W3 + (int64_t)C * K;
    float* h1 = sm;
    float* h2 = sm + K;
    float* a = acts + 3 * D.cp_off;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float x = tanhf(w1[k] + b1[k]);
        h1[k] = x;
        a[k] = x;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float x = tanhf(sparse_in<P, Q>(W2, h1, K, D.n_u, D.n_v, k) + b2[k]);
        h2[k] = x;
        a[K + k] = x;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float y = tanhf(sparse_in<P, Q>(W3, h2, K, D.n_u, D.n_v, k) + b3[k]);
        a[2 * K + k] = y;
        if (lo) Pz[D.cp_off + k] = lo[D.cp_off + k] + 0.5f * (y + 1.0f) * span[D.cp_off + k];
    }
    if (t && threadIdx.x == 0 && (!valid || valid[d])) t[d] += 1;
}

// One workgroup per design: the back-propagated vectors dz1, dz2, dz3 (packed like Pz, written to the
// workspace) with h1, h2 and them in LDS.
template <int P, int Q>
__global__ __launch_bounds__(1024) void k_smlp_backprop(const DesignDev* designs, const int64_t* poff,
                                                        const float* __restrict__ par, const float* acts,
                                                        const float* span, const float* dLdP, float* dz1o,
                                                        float* dz2o, float* dz3o) {
    extern __shared__ float sm[];
    constexpr int C = (2 * P + 1) * (2 * Q + 1);
    const int d = blockIdx.x;
    const DesignDev& D = designs[d];
    const int K = D.n_u * D.n_v;
    const int64_t CK = (int64_t)C * K;
    const float* W2 = par + poff[d] + 2 * K;
    const float* W3 = W2 + CK + K;
    float* dz2 = sm;
    float* dz3 = sm + K;
    const float* a = acts + 3 * D.cp_off;
    const int64_t c = D.cp_off;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float y = a[2 * K + k];
        const float z = dLdP[c + k] * (0.5f * (1.0f - y * y) * span[c + k]);
        dz3[k] = z;
        dz3o[c + k] = z;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float h = a[K + k];
        const float z = sparse_back<P, Q>(W3, dz3, K, D.n_u, D.n_v, k) * (1.0f - h * h);
        dz2[k] = z;
        dz2o[c + k] = z;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float h = a[k];
        dz1o[c + k] = sparse_back<P, Q>(W2, dz2, K, D.n_u, D.n_v, k) * (1.0f - h * h);
    }
}

// Every parameter's gradient (to grad when given) and, with adam set, the Adam update of a valid design
// (step count t + 1).  Workgroup x < C handles connection x of both layers for all neurons; workgroup C the
// four bias-like vectors.
template <int P, int Q>
__global__ __launch_bounds__(256) void k_smlp_update(const DesignDev* designs, const int64_t* poff, float* par,
                                                     const float* acts, const float* dz1, const float* dz2,
                                                     const float* dz3, float* grad, float* m, float* v,
                                                     const int32_t* t, const int32_t* valid, int adam,
                                                     ffrt_adam_hparams hp) {
    constexpr int C = (2 * P + 1) * (2 * Q + 1);
    const int d = blockIdx.y;
    const DesignDev& D = designs[d];
    const int K = D.n_u * D.n_v, nu = D.n_u, nv = D.n_v;
    const int64_t CK = (int64_t)C * K, c = D.cp_off, p0 = poff[d];
    const bool upd = adam && (!valid || valid[d]);
    float step = 0.0f, rb2 = 0.0f;
    if (upd) adam_scales(t, d, hp, step, rb2);
    const float* h1 = acts + 3 * c;
    const float* h2 = h1 + K;
    const int cc = blockIdx.x;
    if (cc == C) {
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            emit(par, grad, m, v, p0 + k, dz1[c + k], upd, step, rb2, hp);
            emit(par, grad, m, v, p0 + K + k, dz1[c + k], upd, step, rb2, hp);
            emit(par, grad, m, v, p0 + 2 * K + CK + k, dz2[c + k], upd, step, rb2, hp);
            emit(par, grad, m, v, p0 + 3 * K + 2 * CK + k, dz3[c + k], upd, step, rb2, hp);
        }
        return;
    }
    const int a = cc / (2 * Q + 1), b = cc - a * (2 * Q + 1);
    const int64_t q2 = p0 + 2 * K + (int64_t)cc * K, q3 = p0 + 3 * K + CK + (int64_t)cc * K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const int i = k / nv + a - P, j = k - (k / nv) * nv + b - Q;
        const bool ok = i >= 0 && i < nu && j >= 0 && j < nv;
        const int s = ok ? i * nv + j : 0;
        emit(par, grad, m, v, q2 + k, ok ? dz2[c + k] * h1[s] : 0.0f, upd, step, rb2, hp);
        emit(par, grad, m, v, q3 + k, ok ? dz3[c + k] * h2[s] : 0.0f, upd, step, rb2, hp);
    }
}

template <int P, int Q>
hipError_t sparse_forward(const DesignDev* designs, int nd, int Kmax, const int64_t* poff, const float* par,
                          float* acts, const float* lo, const float* span, float* Pz, int32_t* t,
                          const int32_t* valid, hipStream_t s) {
    hipLaunchKernelGGL((k_smlp_forward<P, Q>), dim3(nd), dim3(1024), 2 * sizeof(float) * (size_t)Kmax, s, designs,
                       poff, par, acts, lo, span, Pz, t, valid);
    return hipGetLastError();
}

template <int P, int Q>
hipError_t sparse_backward(int part, const DesignDev* designs, int nd, int Kmax, const int64_t* poff, float* par,
                           const float* acts, const float* span, const float* dLdP, float* dz1, float* dz2,
                           float* dz3, float* grad, float* m, float* v, const int32_t* t, const int32_t* valid,
                           const ffrt_adam_hparams* hp, hipStream_t s) {
    if (part != MLP_UPDATE)
        hipLaunchKernelGGL((k_smlp_backprop<P, Q>), dim3(nd), dim3(1024), 2 * sizeof(float) * (size_t)Kmax, s,
                           designs, poff, par, acts, span, dLdP, dz1, dz2, dz3);
    if (part != MLP_BACKPROP) {
        constexpr int C = (2 * P + 1) * (2 * Q + 1);
        ffrt_adam_hparams h = hp ? *hp : ffrt_adam_hparams{0.0f, 0.0f, 0.0f, 0.0f};
        hipLaunchKernelGGL((k_smlp_update<P, Q>), dim3(C + 1, nd), dim3(256), 0, s, designs, poff, par, acts, dz1,
                           dz2, dz3, grad, m, v, t, valid, hp ? 1 : 0, h);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mlp_forward(int arch, int P, int Q, const DesignDev* designs, int nd, int Kmax,
                              const int64_t* poff, const float* par, float* acts, const float* lo, const float* span,
                              float* Pz, int32_t* t, const int32_t* valid, hipStream_t s) {
    if (arch == FFRT_MLP_SPARSE) {
        if (P == 3 && Q == 3)
            return sparse_forward<3, 3>(designs, nd, Kmax, poff, par, acts, lo, span, Pz, t, valid, s);
        if (P == 5 && Q == 3)
            return sparse_forward<5, 3>(designs, nd, Kmax, poff, par, acts, lo, span, Pz, t, valid, s);
        if (P == 2 && Q == 2)
            return sparse_forward<2, 2>(designs, nd, Kmax, poff, par, acts, lo, span, Pz, t, valid, s);
        return hipErrorInvalidValue;
    }
    const unsigned gx = (unsigned)((Kmax + 255) / 256);
    hipLaunchKernelGGL(k_mlp_layer1, dim3(gx, nd), dim3(256), 0, s, designs, poff, par, acts, t, valid);
    const unsigned rows = (unsigned)((Kmax + 3) / 4);
    const size_t lds = sizeof(float) * (size_t)Kmax;
    hipLaunchKernelGGL(k_mlp_gemv, dim3(rows, nd), dim3(256), lds, s, designs, poff, 2, par, acts, nullptr, nullptr,
                       nullptr);
    hipLaunchKernelGGL(k_mlp_gemv, dim3(rows, nd), dim3(256), lds, s, designs, poff, 3, par, acts, lo, span, Pz);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(int arch, int part, int P, int Q, const DesignDev* designs, int nd, int Kmax,
                               const int64_t* poff, float* par, const float* acts, const float* span,
                               const float* dLdP, float* dz3, float* dh2, float* dh1, float* grad, float* m, float* v,
                               const int32_t* t, const int32_t* valid, const ffrt_adam_hparams* hp, hipStream_t s) {
    if (arch == FFRT_MLP_SPARSE) {
        // the three workspace vectors hold dz1, dz2, dz3 here
        if (P == 3 && Q == 3)
            return sparse_backward<3, 3>(part, designs, nd, Kmax, poff, par, acts, span, dLdP, dh1, dh2, dz3, grad, m,
                                         v, t, valid, hp, s);
        if (P == 5 && Q == 3)
            return sparse_backward<5, 3>(part, designs, nd, Kmax, poff, par, acts, span, dLdP, dh1, dh2, dz3, grad, m,
                                         v, t, valid, hp, s);
        if (P == 2 && Q == 2)
            return sparse_backward<2, 2>(part, designs, nd, Kmax, poff, par, acts, span, dLdP, dh1, dh2, dz3, grad, m,
                                         v, t, valid, hp, s);
        return hipErrorInvalidValue;
    }
    const unsigned gx = (unsigned)((Kmax + 255) / 256);
    if (part != MLP_UPDATE) {
        hipLaunchKernelGGL(k_mlp_seed, dim3(gx, nd), dim3(256), 0, s, designs, dLdP, acts, span, dz3, dh2, dh1);
        const unsigned chunks = (unsigned)((Kmax + GT_ROWS - 1) / GT_ROWS);
        hipLaunchKernelGGL(k_mlp_gemv_t, dim3(gx, chunks, nd), dim3(256), 0, s, designs, poff, 3, par, acts, dz3,
                           dh2);
        hipLaunchKernelGGL(k_mlp_gemv_t, dim3(gx, chunks, nd), dim3(256), 0, s, designs, poff, 2, par, acts, dh2,
                           dh1);
        if (part == MLP_BACKPROP) return hipGetLastError();
    }
    ffrt_adam_hparams h = hp ? *hp : ffrt_adam_hparams{0.0f, 0.0f, 0.0f, 0.0f};
    const unsigned nrb = (unsigned)((Kmax + MR - 1) / MR) + 1;
    hipLaunchKernelGGL(k_mlp_grad_adam, dim3(nrb, nd), dim3(256), 0, s, designs, poff, par, acts, dz3, dh2, dh1,
                       grad, m, v, t, valid, hp ? 1 : 0, h);
    return hipGetLastError();
}

}  // namespace ffrt
