// The control-point generators of sec. 2.4: multi-layer perceptrons with the trivial input 1 and three tanh
// layers of the size K = n_u n_v of the control net, followed by the output correction of sec. 2.4.1 (eq. of
// the output correction; the offset function folded into lo):
//   h1 = tanh(w1 + b1),  h2 = tanh(W2 h1 + b2),  y = tanh(W3 h2 + b3),  P = lo + (y + 1) span / 2.
// Activations of a design, packed at 3 cp_off: h1, h2, y (K each).
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
// (zero gradient).  A design's whole sparse generator is a few times 10^5 flops, so one workgroup runs it, with
// the vectors in LDS.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "ffrt_internal.h"
#include "wave.hpp"

namespace ffrt {

namespace {

__device__ inline int64_t mlp_count(int K) { return 2 * (int64_t)K * K + 4 * (int64_t)K; }

// Bias-corrected Adam on one parameter q (Kingma & Ba); step = lr / (1 - b1^t), rb2 = 1 / sqrt(1 - b2^t).
__device__ inline void adam_one(float* par, float* m, float* v, int64_t q, float g, float step, float rb2,
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

// Layer 1 (input 1): h1 = tanh(w1 + b1).  With bump, workgroup 0 of a design whose last loss was valid
// also advances its Adam step counter (the Adam kernel before it used t + 1).
__global__ __launch_bounds__(256) void k_mlp_layer1(const DesignDev* designs, const int64_t* poff,
                                                    const float* __restrict__ par, float* acts, int32_t* t,
                                                    const int32_t* valid) {
    const int d = blockIdx.y;
    const DesignDev& D = designs[d];
    const int K = D.n_u * D.n_v;
    const float* w1 = par + poff[d];
    const float* b1 = w1 + K;
    float* h1 = acts + 3 * D.cp_off;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) h1[k] = tanhf(w1[k] + b1[k]);
    if (t && blockIdx.x == 0 && threadIdx.x == 0 && (!valid || valid[d])) t[d] += 1;
}

// z_i = sum_j W_ij x_j + b_i, out_i = tanh(z_i); one wave per row, x staged in LDS.  With lo set (last
// layer) also P_i = lo_i + (out_i + 1) span_i / 2.  layer: 2 (W2, h1 -> h2) or 3 (W3, h2 -> y).
__global__ __launch_bounds__(256) void k_mlp_gemv(const DesignDev* designs, const int64_t* poff, int layer,
                                                  const float* __restrict__ par, float* acts, const float* lo,
                                                  const float* span, float* Pz) {
    extern __shared__ float sx[];
    const int d = blockIdx.y;
    const DesignDev& D = designs[d];
    const int K = D.n_u * D.n_v;
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
    float acc = 0.0f;
    for (int j = lane; j < K; j += 64) acc += row[j] * sx[j];
    acc = wave_sum(acc);
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
    const int K = D.n_u * D.n_v;
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
    for (int i = r0; i < r1; ++i) acc += W[(int64_t)i * K + j] * sdz[i - r0];
    if (acc != 0.0f) atomicAdd(&dh[D.cp_off + j], acc);
}

// Gradient of every parameter (written to grad when given) and, with Adam set, the Adam update, for the
// designs whose last loss found flux.  Bias corrections use the step count t + 1 (layer 1 advances t).
//   w1, b1: dz1_k = dh1_k (1 - h1_k^2);  W2_ij: dz2_i h1_j;  b2: dz2_i;  W3_ij: dz3_i h2_j;  b3: dz3_i
// with dz2_i = dh2_i (1 - h2_i^2) and dz3 given.
__global__ __launch_bounds__(256) void k_mlp_grad_adam(const DesignDev* designs, const int64_t* poff, float* par,
                                                       const float* acts, const float* dz3, const float* dh2,
                                                       const float* dh1, float* grad, float* m, float* v,
                                                       const int32_t* t, const int32_t* valid, int adam,
                                                       ffrt_adam_hparams hp) {
    const int d = blockIdx.y;
    const DesignDev& D = designs[d];
    const int K = D.n_u * D.n_v;
    const int64_t n = mlp_count(K);
    const bool upd = adam && (!valid || valid[d]);
    float step = 0.0f, rb2 = 0.0f;
    if (upd) adam_scales(t, d, hp, step, rb2);
    const float* h1 = acts + 3 * D.cp_off;
    const float* h2 = h1 + K;
    const int64_t c = D.cp_off;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        float gv;
        if (e < 2 * K) {
            const int k = (int)(e < K ? e : e - K);
            gv = dh1[c + k] * (1.0f - h1[k] * h1[k]);
        } else if (e < 2 * K + (int64_t)K * K) {
            const int64_t r = e - 2 * K;
            const int i = (int)(r / K), j = (int)(r - (int64_t)i * K);
            gv = dh2[c + i] * (1.0f - h2[i] * h2[i]) * h1[j];
        } else if (e < 3 * K + (int64_t)K * K) {
            const int i = (int)(e - 2 * K - (int64_t)K * K);
            gv = dh2[c + i] * (1.0f - h2[i] * h2[i]);
        } else if (e < 3 * K + 2 * (int64_t)K * K) {
            const int64_t r = e - 3 * K - (int64_t)K * K;
            const int i = (int)(r / K), j = (int)(r - (int64_t)i * K);
            gv = dz3[c + i] * h2[j];
        } else {
            const int i = (int)(e - 3 * K - 2 * (int64_t)K * K);
            gv = dz3[c + i];
        }
        const int64_t q = poff[d] + e;
        if (grad) grad[q] = gv;
        if (upd) adam_one(par, m, v, q, gv, step, rb2, hp);
    }
}

// dz3 = dL/dP (1 - y^2) span / 2 for the packed control points, and the accumulators of W^T products
// cleared for the back-propagation that follows.
__global__ void k_mlp_seed(const DesignDev* designs, const float* dLdP, const float* acts, const float* span,
                           float* dz3, float* dh2, float* dh1) {
    const int d = blockIdx.y;
    const DesignDev& D = designs[d];
    const int K = D.n_u * D.n_v;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int64_t c = D.cp_off + k;
    const float y = acts[3 * D.cp_off + 2 * K + k];
    dz3[c] = dLdP[c] * (0.5f * (1.0f - y * y) * span[c]);
    dh2[c] = 0.0f;
    dh1[c] = 0.0f;
}

// ---- sparse (locally connected) architecture ------------------------------------------------------------

struct SparseGeom {
    int K, nu, nv, p, q, cb, C;
    __device__ SparseGeom(const DesignDev& D)
        : K(D.n_u * D.n_v), nu(D.n_u), nv(D.n_v), p(D.n_u - D.nsu), q(D.n_v - D.nsv), cb(2 * q + 1),
          C((2 * p + 1) * (2 * q + 1)) {}
    // input index of connection c of neuron k, or -1 where it leaves the net
    __device__ int src(int k, int c) const {
        const int a = c / cb, b = c - a * cb;
        const int i = k / nv + a - p, j = k % nv + b - q;
        return (i < 0 || i >= nu || j < 0 || j >= nv) ? -1 : i * nv + j;
    }
};

// z_k = sum_c W[c][k] x[src(k, c)]
__device__ inline float sparse_in(const SparseGeom& g, const float* W, const float* x, int k) {
    const int i0 = k / g.nv, j0 = k % g.nv;
    float acc = 0.0f;
    for (int a = 0; a <= 2 * g.p; ++a) {
        const int i = i0 + a - g.p;
        if (i < 0 || i >= g.nu) continue;
        for (int b = 0; b <= 2 * g.q; ++b) {
            const int j = j0 + b - g.q;
            if (j < 0 || j >= g.nv) continue;
            acc += W[(int64_t)(a * g.cb + b) * g.K + k] * x[i * g.nv + j];
        }
    }
    return acc;
}

// dx_s = sum over the (c, k) with src(k, c) = s of W[c][k] dz_k: k = s - (a - p, b - q)
__device__ inline float sparse_back(const SparseGeom& g, const float* W, const float* dz, int s) {
    const int i0 = s / g.nv, j0 = s % g.nv;
    float acc = 0.0f;
    for (int a = 0; a <= 2 * g.p; ++a) {
        const int i = i0 - a + g.p;
        if (i < 0 || i >= g.nu) continue;
        for (int b = 0; b <= 2 * g.q; ++b) {
            const int j = j0 - b + g.q;
            if (j < 0 || j >= g.nv) continue;
            const int k = i * g.nv + j;
            acc += W[(int64_t)(a * g.cb + b) * g.K + k] * dz[k];
        }
    }
    return acc;
}

// One workgroup per design: the three layers with h1, h2 in LDS; writes acts and (with lo) Pz; with t set,
// advances the step counter of a design whose last loss was valid.
__global__ __launch_bounds__(1024) void k_smlp_forward(const DesignDev* designs, const int64_t* poff,
                                                       const float* __restrict__ par, float* acts, const float* lo,
                                                       const float* span, float* Pz, int32_t* t,
                                                       const int32_t* valid) {
    extern __shared__ float sm[];
    const int d = blockIdx.x;
    const DesignDev& D = designs[d];
    const SparseGeom g(D);
    const int K = g.K;
    const float* w1 = par + poff[d];
    const float* b1 = w1 + K;
    const float* W2 = b1 + K;
    const float* b2 = W2 + (int64_t)g.C * K;
    const float* W3 = b2 + K;
    const float* b3 = W3 + (int64_t)g.C * K;
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
        const float x = tanhf(sparse_in(g, W2, h1, k) + b2[k]);
        h2[k] = x;
        a[K + k] = x;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float y = tanhf(sparse_in(g, W3, h2, k) + b3[k]);
        a[2 * K + k] = y;
        if (lo) Pz[D.cp_off + k] = lo[D.cp_off + k] + 0.5f * (y + 1.0f) * span[D.cp_off + k];
    }
    if (t && threadIdx.x == 0 && (!valid || valid[d])) t[d] += 1;
}

// One workgroup per design: back-propagation with h1, h2, dz1, dz2, dz3 in LDS, then every parameter's
// gradient (to grad when given) and, with adam set, the Adam update of a valid design (step count t + 1).
__global__ __launch_bounds__(1024) void k_smlp_backward(const DesignDev* designs, const int64_t* poff, float* par,
                                                        const float* acts, const float* span, const float* dLdP,
                                                        float* grad, float* m, float* v, const int32_t* t,
                                                        const int32_t* valid, int adam, ffrt_adam_hparams hp) {
    extern __shared__ float sm[];
    const int d = blockIdx.x;
    const DesignDev& D = designs[d];
    const SparseGeom g(D);
    const int K = g.K;
    const int64_t CK = (int64_t)g.C * K;
    const float* W2 = par + poff[d] + 2 * K;
    const float* W3 = W2 + CK + K;
    float* h1 = sm;
    float* h2 = sm + K;
    float* dz1 = sm + 2 * K;
    float* dz2 = sm + 3 * K;
    float* dz3 = sm + 4 * K;
    const float* a = acts + 3 * D.cp_off;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        h1[k] = a[k];
        h2[k] = a[K + k];
        const float y = a[2 * K + k];
        dz3[k] = dLdP[D.cp_off + k] * (0.5f * (1.0f - y * y) * span[D.cp_off + k]);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) dz2[k] = sparse_back(g, W3, dz3, k) * (1.0f - h2[k] * h2[k]);
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) dz1[k] = sparse_back(g, W2, dz2, k) * (1.0f - h1[k] * h1[k]);
    __syncthreads();
    const bool upd = adam && (!valid || valid[d]);
    float step = 0.0f, rb2 = 0.0f;
    if (upd) adam_scales(t, d, hp, step, rb2);
    const int64_t n = 2 * CK + 4 * (int64_t)K;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
        float gv;
        if (e < 2 * K) {
            gv = dz1[e < K ? e : e - K];
        } else if (e < 2 * K + CK) {
            const int64_t r = e - 2 * K;
            const int c = (int)(r / K), k = (int)(r - (int64_t)c * K);
            const int s = g.src(k, c);
            gv = s < 0 ? 0.0f : dz2[k] * h1[s];
        } else if (e < 3 * K + CK) {
            gv = dz2[e - 2 * K - CK];
        } else if (e < 3 * K + 2 * CK) {
            const int64_t r = e - 3 * K - CK;
            const int c = (int)(r / K), k = (int)(r - (int64_t)c * K);
            const int s = g.src(k, c);
            gv = s < 0 ? 0.0f : dz3[k] * h2[s];
        } else {
            gv = dz3[e - 3 * K - 2 * CK];
        }
        const int64_t q = poff[d] + e;
        if (grad) grad[q] = gv;
        if (upd) adam_one(par, m, v, q, gv, step, rb2, hp);
    }
}

}  // namespace

hipError_t launch_mlp_forward(int arch, const DesignDev* designs, int nd, int Kmax, const int64_t* poff,
                              const float* par, float* acts, const float* lo, const float* span, float* Pz, int32_t* t,
                              const int32_t* valid, hipStream_t s) {
    if (arch == FFRT_MLP_SPARSE) {
        hipLaunchKernelGGL(k_smlp_forward, dim3(nd), dim3(1024), 2 * sizeof(float) * (size_t)Kmax, s, designs, poff,
                           par, acts, lo, span, Pz, t, valid);
        return hipGetLastError();
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

hipError_t launch_mlp_backward(int arch, int part, const DesignDev* designs, int nd, int Kmax, const int64_t* poff,
                               float* par, const float* acts, const float* span, const float* dLdP, float* dz3,
                               float* dh2, float* dh1, float* grad, float* m, float* v, const int32_t* t,
                               const int32_t* valid, const ffrt_adam_hparams* hp, hipStream_t s) {
    if (arch == FFRT_MLP_SPARSE) {
        if (part == MLP_UPDATE) return hipSuccess;  // fused into the back-propagation kernel
        ffrt_adam_hparams h = hp ? *hp : ffrt_adam_hparams{0.0f, 0.0f, 0.0f, 0.0f};
        hipLaunchKernelGGL(k_smlp_backward, dim3(nd), dim3(1024), 5 * sizeof(float) * (size_t)Kmax, s, designs,
                           poff, par, acts, span, dLdP, grad, m, v, t, valid, hp ? 1 : 0, h);
        return hipGetLastError();
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
    int64_t nmax = 2 * (int64_t)Kmax * Kmax + 4 * (int64_t)Kmax;
    unsigned blocks = (unsigned)std::min<int64_t>((nmax + 255) / 256, 4096);
    hipLaunchKernelGGL(k_mlp_grad_adam, dim3(blocks, nd), dim3(256), 0, s, designs, poff, par, acts, dz3, dh2, dh1,
                       grad, m, v, t, valid, hp ? 1 : 0, h);
    return hipGetLastError();
}

}  // namespace ffrt
