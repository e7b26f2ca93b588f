// gfx950 device code of the tracer: ray sampling, B-spline evaluation from LDS, freeform intersection,
// refraction, splatting (forward) and the hand-written reverse sweep (adjoint).  Templated on the degrees
// P, Q and the filter size NU; included by one translation unit per compiled combination.
//
// Layout of one workgroup (256 threads = 4 wave64s) working on a block of rays:
//   - the block is a BU x BV patch of the source's sample grid (collimated: (u, v); point: (theta, a)),
//     split in 8x8 sub-patches, one per wave and round, so the 64 lanes of a wave trace neighbouring rays;
//   - the design's control heights and both knot tables are staged in LDS once per design;
//   - forward: rays are traced into registers, the workgroup reduces the pixel footprint of the block and,
//     when it fits, splats into a privatised LDS tile that is merged into HBM with one global atomic per
//     touched pixel;
//   - adjoint: every ray is re-traced (inside a step, point-source rays start from the exit root the forward
//     stored), dL/dI is gathered over its filter window, the reverse sweep gives
//     dL/dP for the (P+1)(Q+1) control points of the hit span, reduced across the wave when all its lanes
//     share the span, and accumulated in a privatised LDS copy of the control net.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ffrt_internal.h"
#include "loss.hpp"
#include "wave.hpp"

namespace ffrt {

// ------------------------------------------------------------------------------------------------
// Scalar helpers
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpd(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp_any(float x) { return rcpf(x); }
__device__ __forceinline__ double rcp_any(double x) { return rcpd(x); }
// Square root by the hardware instruction alone (within one ulp for the normal, non-negative arguments it gets
// here: direction cosines and their squares), without the correction steps that round sqrtf correctly; those
// cost a dozen instructions per call, three calls per ray.
__device__ __forceinline__ float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }

// sin(pi r) and cos(pi r) for |r| <= 0.29 by their Taylor series about 0, through r^9 and r^10: the first
// omitted terms, (pi r)^11 / 11! and (pi r)^12 / 12!, stay below 1e-8, a sixth of an ulp of the results.
// Horner in r^2, a third of the instructions of the general sincospif with its own range reduction.
constexpr double PI_D = 3.14159265358979323846;
__device__ __forceinline__ void sincospi_reduced(float r, float& s, float& c) {
    constexpr double p2 = PI_D * PI_D;
    constexpr float s1 = (float)PI_D, s3 = (float)(-PI_D * p2 / 6.0), s5 = (float)(PI_D * p2 * p2 / 120.0),
                    s7 = (float)(-PI_D * p2 * p2 * p2 / 5040.0), s9 = (float)(PI_D * p2 * p2 * p2 * p2 / 362880.0);
    constexpr float c2 = (float)(-p2 / 2.0), c4 = (float)(p2 * p2 / 24.0), c6 = (float)(-p2 * p2 * p2 / 720.0),
                    c8 = (float)(p2 * p2 * p2 * p2 / 40320.0), c10 = (float)(-p2 * p2 * p2 * p2 * p2 / 3628800.0);
    const float r2 = r * r;
    s = r * fmaf(fmaf(fmaf(fmaf(s9, r2, s7), r2, s5), r2, s3), r2, s1);
    c = fmaf(fmaf(fmaf(fmaf(fmaf(c10, r2, c8), r2, c6), r2, c4), r2, c2), r2, 1.0f);
}

// SplitMix64 (Steele, Lea & Flood 2014) in counter form: output `index` of the sequence whose state starts
// at state0 = mix(seed + stream * gamma).
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr uint64_t SPLITMIX_GAMMA = 0x9E3779B97F4A7C15ull;
__device__ __forceinline__ uint64_t splitmix_at(uint64_t state0, uint64_t index) {
    return splitmix_mix(state0 + (index + 1) * SPLITMIX_GAMMA);
}
// The counter of ray `id`, splitmix_at(state0, id) = splitmix_mix(rng_counter(state0, id)): ray id + k has the
// counter + k gamma, so a thread's further rays take a 64-bit addition instead of a multiplication.
__device__ __forceinline__ uint64_t rng_counter(uint64_t state0, int64_t id) {
    return state0 + ((uint64_t)id + 1) * SPLITMIX_GAMMA;
}
// Two 24-bit uniforms in [0, 1), exact in float.
__device__ __forceinline__ void two_uniforms(uint64_t h, float& a, float& b) {
    a = (float)(uint32_t)(h >> 40) * (1.0f / 16777216.0f);
    b = (float)(uint32_t)((h >> 16) & 0xFFFFFFull) * (1.0f / 16777216.0f);
}

// Loads of per-design data through the constant address space: with a wave-uniform index they become
// scalar loads into SGPRs instead of one vector load per lane (the data is read-only during a launch).
#define FFRT_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ T load_uniform(const T* p, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const FFRT_CONST T*)(p))[i];
#else
    return p[i];  // host pass of the single-source compile: never executed
#endif
}

// ------------------------------------------------------------------------------------------------
// B-spline basis from the LDS knot table of one span (sec. 2.1).
// Knot units: ubar = u (n - p), so the clamped knots are the integers clamp(i - p, 0, n - p).  The table
// of span k holds the local knots kap(o) = clamp(o, -k, nspan - k), o = 1-P..P, followed by the
// reciprocals rec(deg, j) = 1 / (kap(j) - kap(j - deg)) (0 for a zero-length interval), deg = 1..P,
// j = 1..deg.  The Cox-de Boor recursion then reads
//   N_{m,deg}(t) = (t - kap(m-deg)) rec(deg,m) N_{m-1,deg-1} + (kap(m+1) - t) rec(deg,m+1) N_{m,deg-1}
// for the nonzero functions m = 0..deg of the span, t = ubar - k in [0, 1].
// Derivatives (d/d ubar): N'_{m,P} = P (rec(P,m) N_{m-1,P-1} - rec(P,m+1) N_{m,P-1}); second derivatives
// apply the same rule to the degree P-1 derivatives.
// ------------------------------------------------------------------------------------------------
// INTERIOR: the span's 2P knots are unclamped, so kap(o) = o and rec(deg, j) = 1/deg are constants and
// the recursion folds into the uniform (cardinal) B-spline without reading the table.
template <int P, bool D2, bool INTERIOR, class T>
__device__ __forceinline__ void span_basis(const float* __restrict__ kt, T t, T* N, T* dN, T* d2N) {
    if constexpr (INTERIOR && P == 3) {
        // The uniform cubic on a unit-spaced span in closed form: the same polynomials as the recurrence
        // below, in Horner form (27 operations for N and N', mostly FMAs, against ~42 for the recurrence).
        const T s = (T)1 - t, t2 = t * t, s2 = s * s;
        N[0] = s2 * s * (T)(1.0 / 6.0);
        N[1] = t2 * (t * (T)0.5 - (T)1) + (T)(2.0 / 3.0);
        N[2] = ((t * (T)-0.5 + (T)0.5) * t + (T)0.5) * t + (T)(1.0 / 6.0);
        N[3] = t2 * t * (T)(1.0 / 6.0);
        dN[0] = s2 * (T)-0.5;
        dN[1] = t * (t * (T)1.5 - (T)2);
        dN[2] = (t * (T)-1.5 + (T)1) * t + (T)0.5;
        dN[3] = t2 * (T)0.5;
        if constexpr (D2) {
            d2N[0] = s;
            d2N[1] = t * (T)3 - (T)2;
            d2N[2] = (T)1 - t * (T)3;
            d2N[3] = t;
        }
        return;
    }
    constexpr int NREC = P * (P + 1) / 2;
    T kap[2 * P];
    T rec[NREC];
    if constexpr (INTERIOR) {
#pragma unroll
        for (int i = 0; i < 2 * P; ++i) kap[i] = (T)(i + 1 - P);
#pragma unroll
        for (int deg = 1; deg <= P; ++deg)
#pragma unroll
            for (int j = 1; j <= deg; ++j) rec[(deg - 1) * deg / 2 + j - 1] = (T)1 / (T)deg;
    } else {
#pragma unroll
        for (int i = 0; i < 2 * P; ++i) kap[i] = (T)kt[i];
#pragma unroll
        for (int i = 0; i < NREC; ++i) rec[i] = (T)kt[2 * P + i];
    }
#define KAP(o) kap[(o) + P - 1]
#define REC(deg, j) rec[((deg) - 1) * (deg) / 2 + (j) - 1]
    T tb[P + 1][P + 1];
    tb[0][0] = (T)1;
#pragma unroll
    for (int deg = 1; deg <= P; ++deg) {
#pragma unroll
        for (int m = 0; m <= deg; ++m) {
            T acc = (T)0;
            if (m >= 1) acc += (t - KAP(m - deg)) * REC(deg, m) * tb[deg - 1][m - 1];
            if (m <= deg - 1) acc += (KAP(m + 1) - t) * REC(deg, m + 1) * tb[deg - 1][m];
            tb[deg][m] = acc;
        }
    }
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        N[m] = tb[P][m];
        T a = (m >= 1) ? REC(P, m) * tb[P - 1][m - 1] : (T)0;
        T b = (m <= P - 1) ? REC(P, m + 1) * tb[P - 1][m] : (T)0;
        dN[m] = (T)P * (a - b);
    }
    if constexpr (D2) {
        if constexpr (P >= 2) {
            T d1[P];
#pragma unroll
            for (int m = 0; m <= P - 1; ++m) {
                T a = (m >= 1) ? REC(P - 1, m) * tb[P - 2][m - 1] : (T)0;
                T b = (m <= P - 2) ? REC(P - 1, m + 1) * tb[P - 2][m] : (T)0;
                d1[m] = (T)(P - 1) * (a - b);
            }
#pragma unroll
            for (int m = 0; m <= P; ++m) {
                T a = (m >= 1) ? REC(P, m) * d1[m - 1] : (T)0;
                T b = (m <= P - 1) ? REC(P, m + 1) * d1[m] : (T)0;
                d2N[m] = (T)P * (a - b);
            }
        } else {
#pragma unroll
            for (int m = 0; m <= P; ++m) d2N[m] = (T)0;
        }
    }
#undef KAP
#undef REC
}

// Surface h(x, y) = Z(X^-1(x), Y^-1(y)) and derivatives (sec. 2.1, 2.1.1) from LDS.  The LDS copy holds
// P^z - zref (partition of unity: h = zref + sum N M (P - zref)), so h below is relative to zref and the
// slopes do not lose digits to the mean lens height.
template <int P, int Q, class T>
struct SurfEval {
    int ku, kv;
    T Nu[P + 1], dNu[P + 1], d2Nu[P + 1];
    T Nv[Q + 1], dNv[Q + 1], d2Nv[Q + 1];
    T h, hx, hy, hxx, hxy, hyy;
};

// The offset x sxu + ubar0 - k of a point from the start of knot span k, in knot units.  The scale is held as
// two floats (sxu + sxu_lo equals the exact (n_u - p) / (2 r_x) to ~1e-15) and the offset is formed by two
// fused multiply-adds whose one visible rounding is that of the result (below 1): rounding x sxu + ubar0
// first would cost up to half an ulp of nspan, ~1e-6 of a span for 30 spans, which moves the normal by
// h_xx times as much and the landing by ~1e-3 pixel on curved, strongly refracting surfaces.
__device__ __forceinline__ float span_offset(float x, float s, float s_lo, float c0) {
    return fmaf(x, s_lo, fmaf(x, s, c0));
}
__device__ __forceinline__ double span_offset(double x, float s, float s_lo, float c0) {
    return fma(x, (double)s + (double)s_lo, (double)c0);
}

// On the given span product (ku, kv) at the local offsets (tu, tv) (knot units from the spans' starts).
template <int P, int Q, bool D2, class T>
__device__ __forceinline__ void eval_surface_local(const DesignDev& D, const float* __restrict__ sP,
                                                   const float* __restrict__ sKu, const float* __restrict__ sKv,
                                                   int ku, int kv, T tu, T tv, SurfEval<P, Q, T>& S) {
    S.ku = ku;
    S.kv = kv;
    // spans k with P-1 <= k <= nspan-P see only unclamped knots
    if (ku >= P - 1 && ku <= D.nsu - P)
        span_basis<P, D2, true, T>(nullptr, tu, S.Nu, S.dNu, S.d2Nu);
    else
        span_basis<P, D2, false, T>(sKu + ku * kt_stride(P), tu, S.Nu, S.dNu, S.d2Nu);
    if (kv >= Q - 1 && kv <= D.nsv - Q)
        span_basis<Q, D2, true, T>(nullptr, tv, S.Nv, S.dNv, S.d2Nv);
    else
        span_basis<Q, D2, false, T>(sKv + kv * kt_stride(Q), tv, S.Nv, S.dNv, S.d2Nv);
    const float* row = sP + ku * D.n_v + kv;  // control point (ku + a, kv + b) of span product (ku, kv)
    T h = 0, hu = 0, hv = 0, huu = 0, huv = 0, hvv = 0;
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        T r0 = 0, r1 = 0, r2 = 0;
#pragma unroll
        for (int b = 0; b <= Q; ++b) {
            T pz = (T)row[a * D.n_v + b];
            r0 += S.Nv[b] * pz;
            r1 += S.dNv[b] * pz;
            if constexpr (D2) r2 += S.d2Nv[b] * pz;
        }
        h += S.Nu[a] * r0;
        hu += S.dNu[a] * r0;
        hv += S.Nu[a] * r1;
        if constexpr (D2) {
            huu += S.d2Nu[a] * r0;
            huv += S.dNu[a] * r1;
            hvv += S.Nu[a] * r2;
        }
    }
    T sx = (T)D.sxu, sy = (T)D.syv;
    S.h = h;
    S.hx = hu * sx;
    S.hy = hv * sy;
    if constexpr (D2) {
        S.hxx = huu * sx * sx;
        S.hxy = huv * sx * sy;
        S.hyy = hvv * sy * sy;
    }
}

// On the given span product (ku, kv) at the point (x, y); eval_surface below picks the one containing it.
// FAST rounds x sxu + ubar0 before taking the span's start off (two operations fewer per axis): good enough
// inside a root search, whose result the offset's rounding moves by ~1e-7 of a span at most, but not for the
// normal that refracts the ray.
template <int P, int Q, bool D2, class T, bool FAST = false>
__device__ __forceinline__ void eval_surface_on(const DesignDev& D, const float* __restrict__ sP,
                                                const float* __restrict__ sKu, const float* __restrict__ sKv, T x,
                                                T y, int ku, int kv, SurfEval<P, Q, T>& S) {
    T tu, tv;
    if constexpr (FAST) {
        tu = (x * (T)D.sxu + (T)D.ubar0) - (T)ku;
        tv = (y * (T)D.syv + (T)D.vbar0) - (T)kv;
    } else {
        tu = span_offset(x, D.sxu, D.sxu_lo, D.ubar0 - (float)ku);
        tv = span_offset(y, D.syv, D.syv_lo, D.vbar0 - (float)kv);
    }
    eval_surface_local<P, Q, D2, T>(D, sP, sKu, sKv, ku, kv, tu, tv, S);
}

template <int P, int Q, bool D2, class T, bool FAST = false>
__device__ __forceinline__ void eval_surface(const DesignDev& D, const float* __restrict__ sP,
                                             const float* __restrict__ sKu, const float* __restrict__ sKv, T x,
                                             T y, SurfEval<P, Q, T>& S) {
    int ku = (int)floor(x * (T)D.sxu + (T)D.ubar0), kv = (int)floor(y * (T)D.syv + (T)D.vbar0);
    eval_surface_on<P, Q, D2, T, FAST>(D, sP, sKu, sKv, x, y, min(max(ku, 0), D.nsu - 1), min(max(kv, 0), D.nsv - 1),
                                 S);
}

// ------------------------------------------------------------------------------------------------
// Sources (sec. 2.2.1) and the flat entry face (point sources).
// ------------------------------------------------------------------------------------------------
struct RayIn {
    int status;
    float ox, oy, oz;   // point on the entry plane (collimated: below the sample, on z = z_in)
    float dx, dy, dz;   // unit direction in the glass
    float w;            // weight after the entry face
    int su, sv;         // collimated: the knot spans of the sample and its offsets in them (knot units)
    float tu, tv;
};

// Azimuth of stratum k of S with jitter xi: theta = 2 pi (k + xi) / S, split into whole quarter turns n and a
// remainder r = (4k - nS) / (2S) + 2 xi / S (|r| <= 1/4 + 2/S) so that the argument of sincospi is rounded once
// at the magnitude of r (exactly, for S a power of two, but for that last rounding) instead of at that of
// theta / pi < 2; the quarter turns are then exact swaps and sign changes.
__device__ __forceinline__ void sample_azimuth(int k, float xi, int S, float inv_S, float& s, float& c) {
    const int n = (int)rintf(4.0f * (float)k * inv_S);
    const float r = fmaf(2.0f * xi, inv_S, (float)(4 * k - n * S) * (0.5f * inv_S));
    float sr, cr;
    if (S >= 64) sincospi_reduced(r, sr, cr);  // |r| < 1/4 + 2/S
    else sincospif(r, &sr, &cr);
    const bool odd = (n & 1) != 0;
    const float a = odd ? cr : sr, b = odd ? sr : cr;
    s = (n & 2) ? -a : a;
    c = ((n + 1) & 2) ? -b : b;
}

// Knot span and offset in it (knot units) of the sample (k + xi) / G of a collimated grid, from the integers:
// (k + xi) nspan / G = m + (rem + xi nspan) / G with k nspan = m G + rem, so the offset is rounded once, at
// its own magnitude, instead of through the aperture coordinate.
__device__ __forceinline__ void sample_span(int k, float xi, int G, float inv_G, int nspan, int& m, float& t) {
    const int q = k * nspan;
    m = (int)((float)q * inv_G);
    int rem = q - m * G;
    if (rem < 0) { --m; rem += G; }
    if (rem >= G) { ++m; rem -= G; }
    t = fmaf(xi, (float)nspan, (float)rem) * inv_G;
    if (t >= 1.0f && m < nspan - 1) { ++m; t -= 1.0f; }
    m = min(max(m, 0), nspan - 1);   // k in [0, G) keeps m there; a stray k stays inside the net
}

// KIND bit 0 clear: collimated source; set: point source or grid of point sources (D.kind 1 or 2).  Bit 1
// selects the triangle-mesh intersection of sec. 2.2.2 instead of the exact root (see below).
template <int KIND>
__device__ __forceinline__ RayIn ray_entry(const DesignDev& D, int e, int ku, int kv, uint64_t ctr) {
    RayIn r;
    r.status = ST_HIT;
    float x1 = 0.5f, x2 = 0.5f;
    if (D.jitter) two_uniforms(splitmix_mix(ctr), x1, x2);
    if constexpr ((KIND & 1) == 0) {
        // Collimated bundle: samples on the grid of [0,1]^2, mapped linearly to the aperture; the ray meets
        // the flat face at normal incidence (Schlick weight 1 - R0) and travels along +z.
        float u = ((float)ku + x1) * D.inv_gu;
        float v = ((float)kv + x2) * D.inv_gv;
        r.ox = (2.0f * u - 1.0f) * D.r_x;
        r.oy = (2.0f * v - 1.0f) * D.r_y;
        sample_span(ku, x1, D.grid_u, D.inv_gu, D.nsu, r.su, r.tu);
        sample_span(kv, x2, D.grid_v, D.inv_gv, D.nsv, r.sv, r.tv);
        r.oz = D.z_in;
        r.dx = 0.0f;
        r.dy = 0.0f;
        r.dz = 1.0f;
        r.w = D.fresnel ? D.w0 * (1.0f - D.R0) : D.w0;
        return r;
    } else {
    // Point source: theta = 2 pi (k + xi) / S_theta, cos(phi) = 1 - (1 - cos phi_max) a (uniform in solid
    // angle), a = (k_a + xi) / S_a.  sin(phi) = sqrt(a' (2 - a')) with a' = (1 - cos phi_max) a avoids the
    // cancellation of 1 - cos^2.
    float sth, cth;
    sample_azimuth(ku, x1, D.grid_u, D.inv_gu, sth, cth);
    float a = ((float)kv + x2) * D.inv_gv;
    float ao = a * D.omc;
    float cphi = 1.0f - ao;
    float sphi = sqrt_hw(ao * (2.0f - ao));
    float px = D.pos_x, py = D.pos_y;
    if (D.kind == 2) {
        int ix = e / D.emit_ny, iy = e - ix * D.emit_ny;
        px += D.ex0 + (float)ix * D.edx;
        py += D.ey0 + (float)iy * D.edy;
    }
    float t0 = (D.z_in - D.pos_z) * rcpf(cphi);
    r.ox = px + t0 * cth * sphi;
    r.oy = py + t0 * sth * sphi;
    r.oz = D.z_in;
    if (fabsf(r.ox) > D.r_x || fabsf(r.oy) > D.r_y) {
        r.status = ST_MISS_ENTRY;
        return r;
    }
    // Refraction air -> glass at the normal (0,0,1): d1 = eta d0 + (sqrt(k) - eta cos) z, eta = 1/n, whose
    // z component is sqrt(k) = sqrt(1 - eta^2 sin^2).
    float eta = rcpf(D.n_lens);
    float k = 1.0f - eta * eta * sphi * sphi;
    r.dx = eta * cth * sphi;
    r.dy = eta * sth * sphi;
    r.dz = sqrt_hw(k);
    float w = D.w0;
    if (D.fresnel) {  // Schlick with the air-side cosine
        float m = 1.0f - cphi, m2 = m * m;
        w *= 1.0f - (D.R0 + (1.0f - D.R0) * m2 * m2 * m);
    }
    r.w = w;
    return r;
    }
}

// ------------------------------------------------------------------------------------------------
// Freeform intersection (sec. 2.2.1 root problem; sec. 2.2.2 bounding box).
// f(t) = h(o_xy + t d_xy) - o_z - t d_z.  Bracket from the global convex-hull box [min P^z, max P^z]
// intersected with the aperture; f > 0 below it and f < 0 above.  When the slope bound proves f strictly
// decreasing the root is unique; otherwise the bracket is scanned for its first sign change (64 samples per
// projected knot span), which is the smallest root even where the ray meets the surface again before it
// leaves the aperture.  Safeguarded
// Newton (bisection when a step leaves the bracket), at most newton_max iterations.  Grazing hits
// (|f'| small) get their residual re-evaluated in double precision and one double Newton correction.
// ------------------------------------------------------------------------------------------------
constexpr float GRAZING_FP = 0.05f;

// oz_rel = o_z - zref (heights in LDS are relative to zref).
template <int P, int Q>
__device__ __forceinline__ float f_and_slope(const DesignDev& D, const float* sP, const float* sKu,
                                             const float* sKv, const RayIn& r, float oz_rel, float t,
                                             float& fp) {
    SurfEval<P, Q, float> S;
    eval_surface<P, Q, false, float, true>(D, sP, sKu, sKv, r.ox + t * r.dx, r.oy + t * r.dy, S);
    fp = S.hx * r.dx + S.hy * r.dy - r.dz;
    return S.h - oz_rel - t * r.dz;
}

struct RootOut {
    int status;
    float t;
    int iters;
    int failed, nonmono, refined;
};

// t_guess: a start for Newton inside the final bracket (the root of a neighbouring ray), else the midpoint.
template <int P, int Q>
__device__ RootOut intersect(const DesignDev& D, const BoundsDev& B, const float* sP, const float* sKu,
                             const float* sKv, const float* sS, const RayIn& r, float t_guess = -1.0f) {
    RootOut R;
    R.status = ST_HIT;
    R.t = 0.0f;
    R.iters = 0;
    R.failed = R.nonmono = R.refined = 0;
    float inv_dz = rcpf(r.dz);
    float pad = 4e-6f * (1.0f + fabsf(B.zmax - r.oz)) * inv_dz;
    float t_lo = fmaxf(0.0f, (B.zmin - r.oz) * inv_dz - pad);
    float t_hi = (B.zmax - r.oz) * inv_dz + pad;
    // where the ray leaves the aperture prism, needed only when that happens before the bracket's top: the ray
    // starts inside the prism, which is convex, so a point inside at t_hi keeps the whole bracket inside
    float t_ap = INFINITY;
    if (!(fabsf(r.ox + t_hi * r.dx) < D.r_x && fabsf(r.oy + t_hi * r.dy) < D.r_y)) {
        if (r.dx > 0.0f) t_ap = fminf(t_ap, (D.r_x - r.ox) * rcpf(r.dx));
        if (r.dx < 0.0f) t_ap = fminf(t_ap, (-D.r_x - r.ox) * rcpf(r.dx));
        if (r.dy > 0.0f) t_ap = fminf(t_ap, (D.r_y - r.oy) * rcpf(r.dy));
        if (r.dy < 0.0f) t_ap = fminf(t_ap, (-D.r_y - r.oy) * rcpf(r.dy));
    }
    float t_end = fminf(t_hi, t_ap);
    if (t_end < t_lo) {
        R.status = ST_SIDE_WALL;
        return R;
    }
    const float ozr = r.oz - B.zref;
    float a = t_lo, b = t_end, fp;
    // the aperture ends the search: a ray still below the surface where it leaves the aperture has no root,
    // unless (f not monotone) it crossed the surface and met it again before the aperture edge
    const bool end_below = t_ap <= t_hi && f_and_slope<P, Q>(D, sP, sKu, sKv, r, ozr, t_end, fp) > 0.0f;
    float gx = B.gx, gy = B.gy;
    // A ray that the design's global slope bounds already prove monotone and that has a start for Newton
    // needs neither the narrowed bracket nor the local bounds.
    const bool mono_global = gx * fabsf(r.dx) + gy * fabsf(r.dy) < r.dz;
    if (sS && !(mono_global && t_guess >= 0.0f)) {
        // Local bounds: over [t_lo, t_end] the ray stays above the few span products its (x, y) segment
        // crosses, so every root lies where the ray height is inside their height range, and the slope
        // bounds of those spans alone decide monotonicity.  Signs at the narrowed ends stay known: the ray
        // is below the surface where its height is at most their minimum and above it at their maximum.
        const float x0 = r.ox + t_lo * r.dx, y0 = r.oy + t_lo * r.dy;
        const float x1 = r.ox + t_end * r.dx, y1 = r.oy + t_end * r.dy;
        const int u0 = min(max((int)floorf(x0 * D.sxu + D.ubar0), 0), D.nsu - 1);
        const int u1 = min(max((int)floorf(x1 * D.sxu + D.ubar0), 0), D.nsu - 1);
        const int v0 = min(max((int)floorf(y0 * D.syv + D.vbar0), 0), D.nsv - 1);
        const int v1 = min(max((int)floorf(y1 * D.syv + D.vbar0), 0), D.nsv - 1);
        const int ua = min(u0, u1), ub = max(u0, u1), va = min(v0, v1), vb = max(v0, v1);
        if ((ub - ua + 1) * (vb - va + 1) <= 9) {
            float zl = INFINITY, zh = -INFINITY, gxl = 0.0f, gyl = 0.0f;
            for (int su = ua; su <= ub; ++su)
                for (int sv = va; sv <= vb; ++sv) {
                    const float* rec = sS + 4 * (su * D.nsv + sv);
                    zl = fminf(zl, rec[0]);
                    zh = fmaxf(zh, rec[1]);
                    gxl = fmaxf(gxl, rec[2]);
                    gyl = fmaxf(gyl, rec[3]);
                }
            const float a2 = fmaxf(a, (zl - r.oz) * inv_dz - pad), b2 = fminf(b, (zh - r.oz) * inv_dz + pad);
            if (a2 <= b2) {
                a = a2;
                b = b2;
            }
            gx = gxl;
            gy = gyl;
        }
    }
    const bool mono = gx * fabsf(r.dx) + gy * fabsf(r.dy) < r.dz;
    if (mono) {
        if (end_below) {
            R.status = ST_SIDE_WALL;
            return R;
        }
    } else {
        // the first sign change, sampled at 64 points per knot span the segment [a, b] projects onto (at least
        // 64, at most 4096); no sign change at any sample: the ray leaves through the side wall
        R.nonmono = 1;
        const float du = fabsf(r.dx) * (b - a) * D.sxu, dv = fabsf(r.dy) * (b - a) * D.syv;
        const int M = min(max(64, (int)ceilf(64.0f * (du + dv)) + 1), 4096);
        const float a0 = a, len = b - a, inv_m = 1.0f / (float)M;
        float prev = a0;
        bool found = false;
        for (int s = 1; s <= M; ++s) {
            const float ts = s == M ? a0 + len : a0 + len * ((float)s * inv_m);
            if (f_and_slope<P, Q>(D, sP, sKu, sKv, r, ozr, ts, fp) <= 0.0f) {
                a = prev;
                b = ts;
                found = true;
                break;
            }
            prev = ts;
        }
        if (!found) {
            R.status = ST_SIDE_WALL;
            return R;
        }
    }
    // A neighbouring sample's root, when inside the bracket, starts Newton ~1e-3 of the ray length from this
    // root instead of half a bracket away: one iteration fewer on average.
    float t = t_guess > a && t_guess < b ? t_guess : 0.5f * (a + b);
    bool done = false;
    float f = 0.0f;
    int it = 0;
    for (; it < D.newton_max && !done; ++it) {
        f = f_and_slope<P, Q>(D, sP, sKu, sKv, r, ozr, t, fp);
        if (f > 0.0f) a = t; else b = t;
        float tn = t - f * rcpf(fp);
        if (!(tn >= a && tn <= b) || !(fp < 0.0f)) tn = 0.5f * (a + b);
        done = fabsf(tn - t) <= 2e-6f * (1.0f + fabsf(t));
        t = tn;
    }
    R.iters = it;
    R.failed = done ? 0 : 1;
    if (fabsf(fp) < GRAZING_FP) {
        // double-precision residual at the root and one Newton correction
        SurfEval<P, Q, double> S;
        double td = (double)t;
        eval_surface<P, Q, false, double>(D, sP, sKu, sKv, (double)r.ox + td * (double)r.dx,
                                          (double)r.oy + td * (double)r.dy, S);
        double fd = S.h - ((double)r.oz - (double)B.zref) - td * (double)r.dz;
        double fpd = S.hx * (double)r.dx + S.hy * (double)r.dy - (double)r.dz;
        if (fpd < 0.0) {
            double tn = td - fd / fpd;
            if (tn >= (double)a - 1e-6 && tn <= (double)b + 1e-6) t = (float)tn;
        }
        R.refined = 1;
    }
    R.t = t;
    return R;
}

// ------------------------------------------------------------------------------------------------
// Freeform entry face (both faces freeform): the entry face is a second B-spline whose net follows the exit
// net; its LDS copy holds heights relative to zref_in.  A point-source ray meets it at the smallest root over
// the aperture prism (it must enter the prism below the face and leave it above, else it passes the lens:
// ST_MISS_ENTRY), found like the exit root: bracket from the face's height range, monotonicity from its slope
// bounds or a scan, safeguarded Newton.  A collimated ray meets it at its sampled (x, y).  The ray refracts
// into the glass with the vector Snell law at n_hat = (-g_x, -g_y, 1)/|.| and takes the Schlick weight with
// the air-side cosine d0 . n_hat.
// ------------------------------------------------------------------------------------------------
struct EntryHit {
    float sx, sy, sz, d0x, d0y, d0z;  // source ray in air
    float t;                          // its parameter at the entry hit
};

template <int P, int Q, bool POINT>
__device__ __forceinline__ RayIn ray_entry_ff(const DesignDev& D, const BoundsDev& B, const float* sPin,
                                              const float* sKu, const float* sKv, int e, int ku, int kv,
                                              uint64_t ctr, EntryHit& H) {
    RayIn r;
    r.status = ST_HIT;
    float x1 = 0.5f, x2 = 0.5f;
    if (D.jitter) two_uniforms(splitmix_mix(ctr), x1, x2);
    if constexpr (!POINT) {
        const float u = ((float)ku + x1) * D.inv_gu, v = ((float)kv + x2) * D.inv_gv;
        H.sx = (2.0f * u - 1.0f) * D.r_x;
        H.sy = (2.0f * v - 1.0f) * D.r_y;
        H.sz = B.zmin_in - 1.0f;
        H.d0x = 0.0f;
        H.d0y = 0.0f;
        H.d0z = 1.0f;
    } else {
        float sth, cth;
        sample_azimuth(ku, x1, D.grid_u, D.inv_gu, sth, cth);
        const float ao = ((float)kv + x2) * D.inv_gv * D.omc;
        const float cphi = 1.0f - ao, sphi = sqrt_hw(ao * (2.0f - ao));
        float px = D.pos_x, py = D.pos_y;
        if (D.kind == 2) {
            int ix = e / D.emit_ny, iy = e - ix * D.emit_ny;
            px += D.ex0 + (float)ix * D.edx;
            py += D.ey0 + (float)iy * D.edy;
        }
        H.sx = px;
        H.sy = py;
        H.sz = D.pos_z;
        H.d0x = cth * sphi;
        H.d0y = sth * sphi;
        H.d0z = cphi;
    }
    RayIn s0;  // the source ray, in the form the surface evaluation takes
    s0.ox = H.sx;
    s0.oy = H.sy;
    s0.oz = H.sz;
    s0.dx = H.d0x;
    s0.dy = H.d0y;
    s0.dz = H.d0z;
    const float ozr = H.sz - B.zref_in;
    float t;
    if constexpr (!POINT) {
        SurfEval<P, Q, float> S;
        eval_surface<P, Q, false, float>(D, sPin, sKu, sKv, H.sx, H.sy, S);
        t = S.h - ozr;
    } else {
        float t_a = 0.0f, t_b = INFINITY;
        if (H.d0x != 0.0f) {
            const float ta = (-D.r_x - H.sx) * rcpf(H.d0x), tb = (D.r_x - H.sx) * rcpf(H.d0x);
            t_a = fmaxf(t_a, fminf(ta, tb));
            t_b = fminf(t_b, fmaxf(ta, tb));
        } else if (fabsf(H.sx) > D.r_x) {
            t_b = -1.0f;
        }
        if (H.d0y != 0.0f) {
            const float ta = (-D.r_y - H.sy) * rcpf(H.d0y), tb = (D.r_y - H.sy) * rcpf(H.d0y);
            t_a = fmaxf(t_a, fminf(ta, tb));
            t_b = fminf(t_b, fmaxf(ta, tb));
        } else if (fabsf(H.sy) > D.r_y) {
            t_b = -1.0f;
        }
        const float inv_dz = rcpf(H.d0z);
        const float pad = 4e-6f * (1.0f + fabsf(B.zmax_in - H.sz)) * inv_dz;
        float a = fmaxf(t_a, (B.zmin_in - H.sz) * inv_dz - pad), b = fminf(t_b, (B.zmax_in - H.sz) * inv_dz + pad);
        if (!(a <= b)) {
            r.status = ST_MISS_ENTRY;
            return r;
        }
        float fp;
        // enter the prism below the face (else through the side wall) and cross it before leaving the prism
        // (else the ray passes the lens): with a monotone f the sign where it leaves decides, otherwise the
        // first sign change of the scan, as at the exit face
        if (f_and_slope<P, Q>(D, sPin, sKu, sKv, s0, ozr, a, fp) < 0.0f) {
            r.status = ST_MISS_ENTRY;
            return r;
        }
        const bool exit_below = f_and_slope<P, Q>(D, sPin, sKu, sKv, s0, ozr, b, fp) > 0.0f;
        if (B.gx_in * fabsf(H.d0x) + B.gy_in * fabsf(H.d0y) < H.d0z) {
            if (exit_below) {
                r.status = ST_MISS_ENTRY;
                return r;
            }
        } else {
            const float du = fabsf(H.d0x) * (b - a) * D.sxu, dv = fabsf(H.d0y) * (b - a) * D.syv;
            const int M = min(max(64, (int)ceilf(64.0f * (du + dv)) + 1), 4096);
            const float a0 = a, len = b - a, inv_m = 1.0f / (float)M;
            float prev = a0;
            bool found = false;
            for (int k = 1; k <= M; ++k) {
                const float ts = k == M ? a0 + len : a0 + len * ((float)k * inv_m);
                if (f_and_slope<P, Q>(D, sPin, sKu, sKv, s0, ozr, ts, fp) <= 0.0f) {
                    a = prev;
                    b = ts;
                    found = true;
                    break;
                }
                prev = ts;
            }
            if (!found) {
                r.status = ST_MISS_ENTRY;
                return r;
            }
        }
        t = 0.5f * (a + b);
        bool done = false;
        for (int it = 0; it < D.newton_max && !done; ++it) {
            const float f = f_and_slope<P, Q>(D, sPin, sKu, sKv, s0, ozr, t, fp);
            if (f > 0.0f) a = t; else b = t;
            float tn = t - f * rcpf(fp);
            if (!(tn >= a && tn <= b) || !(fp < 0.0f)) tn = 0.5f * (a + b);
            done = fabsf(tn - t) <= 2e-6f * (1.0f + fabsf(t));
            t = tn;
        }
        if (fabsf(fp) < GRAZING_FP) {
            // grazing hit: double-precision residual at the root and one Newton correction, as at the exit
            SurfEval<P, Q, double> S;
            const double td = (double)t;
            eval_surface<P, Q, false, double>(D, sPin, sKu, sKv, (double)H.sx + td * (double)H.d0x,
                                              (double)H.sy + td * (double)H.d0y, S);
            const double fd = S.h - ((double)H.sz - (double)B.zref_in) - td * (double)H.d0z;
            const double fpd = S.hx * (double)H.d0x + S.hy * (double)H.d0y - (double)H.d0z;
            if (fpd < 0.0) {
                const double tn = td - fd / fpd;
                if (tn >= (double)a - 1e-6 && tn <= (double)b + 1e-6) t = (float)tn;
            }
        }
    }
    H.t = t;
    r.ox = H.sx + t * H.d0x;
    r.oy = H.sy + t * H.d0y;
    r.oz = H.sz + t * H.d0z;
    SurfEval<P, Q, float> S;
    eval_surface<P, Q, false, float>(D, sPin, sKu, sKv, r.ox, r.oy, S);
    const float inv = rsqrtf(S.hx * S.hx + S.hy * S.hy + 1.0f);
    const float nx = -S.hx * inv, ny = -S.hy * inv, nz = inv;
    const float eta = rcpf(D.n_lens);
    const float c = H.d0x * nx + H.d0y * ny + H.d0z * nz;
    const float k = 1.0f - eta * eta * (1.0f - c * c);
    const float beta = sqrt_hw(k) - eta * c;
    r.dx = eta * H.d0x + beta * nx;
    r.dy = eta * H.d0y + beta * ny;
    r.dz = eta * H.d0z + beta * nz;
    float w = D.w0;
    if (D.fresnel) {
        const float m = 1.0f - c, m2 = m * m;
        w *= 1.0f - (D.R0 + (1.0f - D.R0) * m2 * m2 * m);
    }
    r.w = w;
    return r;
}

// ------------------------------------------------------------------------------------------------
// Triangle mesh of sec. 2.2.2, the paper's own intersector (an alternative to the exact root): each knot
// span product is divided into mesh_u x mesh_v equal rectangles, each into a lower-left triangle (left and
// lower edges closed) and an upper-right one (diagonal closed) whose corners lie on the surface.  In cell
// units c_u = ubar mesh_u, c_v = vbar mesh_v (ubar in knot spans), cell (K, L) = (floor c_u, floor c_v)
// belongs to span product (K / mesh_u, L / mesh_v); a = c_u - K, b = c_v - L place a point in its cell and
// the lower-left triangle is a + b < 1.  Corner heights are B-spline values at the cell's nodes, from the
// basis functions at the two node columns and rows of the cell (they depend on the node only, not on P).
// ------------------------------------------------------------------------------------------------
template <int P, int Q>
struct MeshCell {
    int su, sv;                                              // span product of the cell
    float Nu0[P + 1], Nu1[P + 1], Nv0[Q + 1], Nv1[Q + 1];    // basis at the cell's node columns / rows
    float z00, z10, z01, z11;                                // corner heights relative to zref
};

template <int P, int Q>
__device__ __forceinline__ void mesh_cell(const DesignDev& D, const float* sP, const float* sKu, const float* sKv,
                                          int K, int L, MeshCell<P, Q>& C) {
    C.su = K / D.mesh_u;
    C.sv = L / D.mesh_v;
    const float tu0 = (float)(K - C.su * D.mesh_u) * D.inv_mesh_u, tu1 = tu0 + D.inv_mesh_u;
    const float tv0 = (float)(L - C.sv * D.mesh_v) * D.inv_mesh_v, tv1 = tv0 + D.inv_mesh_v;
    float dn[P + 1 > Q + 1 ? P + 1 : Q + 1];
    if (C.su >= P - 1 && C.su <= D.nsu - P) {
        span_basis<P, false, true, float>(nullptr, tu0, C.Nu0, dn, nullptr);
        span_basis<P, false, true, float>(nullptr, tu1, C.Nu1, dn, nullptr);
    } else {
        span_basis<P, false, false, float>(sKu + C.su * kt_stride(P), tu0, C.Nu0, dn, nullptr);
        span_basis<P, false, false, float>(sKu + C.su * kt_stride(P), tu1, C.Nu1, dn, nullptr);
    }
    if (C.sv >= Q - 1 && C.sv <= D.nsv - Q) {
        span_basis<Q, false, true, float>(nullptr, tv0, C.Nv0, dn, nullptr);
        span_basis<Q, false, true, float>(nullptr, tv1, C.Nv1, dn, nullptr);
    } else {
        span_basis<Q, false, false, float>(sKv + C.sv * kt_stride(Q), tv0, C.Nv0, dn, nullptr);
        span_basis<Q, false, false, float>(sKv + C.sv * kt_stride(Q), tv1, C.Nv1, dn, nullptr);
    }
    const float* row = sP + C.su * D.n_v + C.sv;
    float z00 = 0.0f, z10 = 0.0f, z01 = 0.0f, z11 = 0.0f;
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        float r0 = 0.0f, r1 = 0.0f;
#pragma unroll
        for (int b = 0; b <= Q; ++b) {
            const float pz = row[a * D.n_v + b];
            r0 += C.Nv0[b] * pz;
            r1 += C.Nv1[b] * pz;
        }
        z00 += C.Nu0[a] * r0;
        z10 += C.Nu1[a] * r0;
        z01 += C.Nu0[a] * r1;
        z11 += C.Nu1[a] * r1;
    }
    C.z00 = z00;
    C.z10 = z10;
    C.z01 = z01;
    C.z11 = z11;
}

// Slopes of a triangle's plane per cell unit: T = z00 + A a + B b (lower-left, through corners 00, 10, 01)
// or T = z11 + A (a - 1) + B (b - 1) (upper-right, through corners 11, 01, 10).
template <int P, int Q>
__device__ __forceinline__ void tri_slopes(const MeshCell<P, Q>& C, int upper, float& A, float& B) {
    A = upper ? C.z11 - C.z01 : C.z10 - C.z00;
    B = upper ? C.z11 - C.z10 : C.z01 - C.z00;
}

struct MeshRoot {
    int status;
    float t;
    int K, L, upper, cells;
};

// First hit of a point-source ray on the mesh.  The ray is bracketed by the global height box as for the
// exact root; its (u, v) track is then walked cell by cell in order of t (a 2-D DDA), and in each cell the
// plane of either triangle is intersected; the first cell with a hit inside one of its triangles holds the
// smallest t.  The triangle tests accept a rounding margin (a hit on a shared edge has the same t on both
// sides), so no ray slips between triangles.  A ray whose track leaves the aperture or the bracket without
// a hit leaves through the side wall.
template <int P, int Q>
__device__ MeshRoot intersect_mesh(const DesignDev& D, const BoundsDev& B, const float* sP, const float* sKu,
                                   const float* sKv, const RayIn& r) {
    MeshRoot R;
    R.status = ST_SIDE_WALL;
    R.t = 0.0f;
    R.K = R.L = R.upper = R.cells = 0;
    const float inv_dz = rcpf(r.dz);
    const float pad = 4e-6f * (1.0f + fabsf(B.zmax - r.oz)) * inv_dz;
    const float t_lo = fmaxf(0.0f, (B.zmin - r.oz) * inv_dz - pad);
    const float t_hi = (B.zmax - r.oz) * inv_dz + pad;
    // where the ray leaves the aperture prism, needed only when that happens before the bracket's top: the ray
    // starts inside the prism, which is convex, so a point inside at t_hi keeps the whole bracket inside
    float t_ap = INFINITY;
    if (!(fabsf(r.ox + t_hi * r.dx) < D.r_x && fabsf(r.oy + t_hi * r.dy) < D.r_y)) {
        if (r.dx > 0.0f) t_ap = fminf(t_ap, (D.r_x - r.ox) * rcpf(r.dx));
        if (r.dx < 0.0f) t_ap = fminf(t_ap, (-D.r_x - r.ox) * rcpf(r.dx));
        if (r.dy > 0.0f) t_ap = fminf(t_ap, (D.r_y - r.oy) * rcpf(r.dy));
        if (r.dy < 0.0f) t_ap = fminf(t_ap, (-D.r_y - r.oy) * rcpf(r.dy));
    }
    const float t_end = fminf(t_hi, t_ap);
    if (t_end < t_lo) return R;
    const int NK = D.nsu * D.mesh_u, NL = D.nsv * D.mesh_v;
    const float cu0 = ((r.ox + t_lo * r.dx) * D.sxu + D.ubar0) * (float)D.mesh_u;
    const float cv0 = ((r.oy + t_lo * r.dy) * D.syv + D.vbar0) * (float)D.mesh_v;
    const float dcu = r.dx * D.sxu * (float)D.mesh_u, dcv = r.dy * D.syv * (float)D.mesh_v;  // cells per unit t
    int K = min(max((int)floorf(cu0), 0), NK - 1), L = min(max((int)floorf(cv0), 0), NL - 1);
    const int stK = dcu > 0.0f ? 1 : -1, stL = dcv > 0.0f ? 1 : -1;
    float tK = dcu != 0.0f ? t_lo + ((float)(K + (dcu > 0.0f ? 1 : 0)) - cu0) * rcpf(dcu) : INFINITY;
    float tL = dcv != 0.0f ? t_lo + ((float)(L + (dcv > 0.0f ? 1 : 0)) - cv0) * rcpf(dcv) : INFINITY;
    const float dtK = dcu != 0.0f ? fabsf(rcpf(dcu)) : INFINITY, dtL = dcv != 0.0f ? fabsf(rcpf(dcv)) : INFINITY;
    const float zr0 = (r.oz - B.zref) + t_lo * r.dz;  // ray height above zref at t_lo
    constexpr float EPS = 2e-5f;                      // cell units
    const float s_max = t_end - t_lo + pad;
    for (int it = 0; it <= NK + NL; ++it) {
        MeshCell<P, Q> C;
        mesh_cell<P, Q>(D, sP, sKu, sKv, K, L, C);
        R.cells++;
        const float a0 = cu0 - (float)K, b0 = cv0 - (float)L;  // the ray's cell coordinates at t_lo
        float best = INFINITY;
        int up = 0;
#pragma unroll
        for (int tri = 0; tri < 2; ++tri) {
            float A, Bs;
            tri_slopes<P, Q>(C, tri, A, Bs);
            // z at s = t - t_lo: zr0 + dz s = T(a0 + dcu s, b0 + dcv s)
            const float den = r.dz - A * dcu - Bs * dcv;
            const float num = tri ? C.z11 + A * (a0 - 1.0f) + Bs * (b0 - 1.0f) - zr0 : C.z00 + A * a0 + Bs * b0 - zr0;
            if (den == 0.0f) continue;
            const float sh = num * rcpf(den);
            const float a = a0 + dcu * sh, b = b0 + dcv * sh;
            const bool inside = tri ? (a + b >= 1.0f - EPS && a <= 1.0f + EPS && b <= 1.0f + EPS)
                                    : (a >= -EPS && b >= -EPS && a + b <= 1.0f + EPS);
            if (inside && sh >= -pad && sh <= s_max && sh < best) {
                best = sh;
                up = tri;
            }
        }
        if (best < INFINITY) {
            R.status = ST_HIT;
            R.t = t_lo + best;
            R.K = K;
            R.L = L;
            R.upper = up;
            return R;
        }
        if (fminf(tK, tL) > t_end) break;
        if (tK < tL) {
            K += stK;
            tK += dtK;
            if (K < 0 || K >= NK) break;
        } else {
            L += stL;
            tL += dtL;
            if (L < 0 || L >= NL) break;
        }
    }
    return R;
}

// Cell, triangle and in-cell coordinates of a point (x, y).
__device__ __forceinline__ void mesh_locate(const DesignDev& D, float x, float y, int& K, int& L, float& a,
                                            float& b) {
    const float cu = (x * D.sxu + D.ubar0) * (float)D.mesh_u, cv = (y * D.syv + D.vbar0) * (float)D.mesh_v;
    K = min(max((int)floorf(cu), 0), D.nsu * D.mesh_u - 1);
    L = min(max((int)floorf(cv), 0), D.nsv * D.mesh_v - 1);
    a = cu - (float)K;
    b = cv - (float)L;
}

// ------------------------------------------------------------------------------------------------
// Exit face (sec. 2.2): vector Snell glass -> air at n_hat = (-h_x, -h_y, 1)/|.|, TIR dropped, Schlick
// weight with the air-side cosine sqrt(k), propagation to the screen plane (sec. 2.3).
// ------------------------------------------------------------------------------------------------
struct ExitState {
    int status;
    float nxh, nyh, nzh, inv_m;   // unit normal and 1/|m|
    float k;                      // Snell discriminant 1 - n^2 sin^2 (negative: TIR)
    float c, sk, beta;            // d.n_hat, sqrt(k), sqrt(k) - n c
    float ex, ey, ez;             // direction in air
    float tau, T;                 // screen distance parameter, Schlick transmittance
    float X, Y, w;                // landing (NaN when the ray does not reach the screen plane)
};

__device__ __forceinline__ ExitState exit_face(const DesignDev& D, float qx, float qy, float qz, float dx,
                                               float dy, float dz, float hx, float hy, float w1) {
    ExitState E;
    E.status = ST_HIT;
    E.X = E.Y = __builtin_nanf("");
    float inv = rsqrtf(hx * hx + hy * hy + 1.0f);
    E.inv_m = inv;
    E.nxh = -hx * inv;
    E.nyh = -hy * inv;
    E.nzh = inv;
    E.c = dx * E.nxh + dy * E.nyh + dz * E.nzh;
    // sin^2 of the incidence angle as |d x n_hat|^2 (no cancellation near normal incidence)
    float cx = dy * E.nzh - dz * E.nyh, cy = dz * E.nxh - dx * E.nzh, cz = dx * E.nyh - dy * E.nxh;
    float s2 = cx * cx + cy * cy + cz * cz;
    float n = D.n_lens;
    float k = 1.0f - n * n * s2;
    E.k = k;
    if (!(k >= 0.0f)) {
        E.status = ST_TIR;
        return E;
    }
    E.sk = sqrt_hw(k);
    E.beta = E.sk - n * E.c;
    E.ex = n * dx + E.beta * E.nxh;
    E.ey = n * dy + E.beta * E.nyh;
    E.ez = n * dz + E.beta * E.nzh;
    E.T = 1.0f;
    if (D.fresnel) {
        float m = 1.0f - E.sk, m2 = m * m;
        E.T = 1.0f - (D.R0 + (1.0f - D.R0) * m2 * m2 * m);
    }
    E.w = w1 * E.T;
    if (!(E.ez > 0.0f)) {
        E.status = ST_OFF_SCREEN;
        return E;
    }
    E.tau = (D.z_screen - qz) * rcpf(E.ez);
    E.X = qx + E.tau * E.ex;
    E.Y = qy + E.tau * E.ey;
    if (!(E.X >= -D.Rx && E.X < D.Rx && E.Y >= -D.Ry && E.Y < D.Ry)) E.status = ST_OFF_SCREEN;
    return E;
}

// ------------------------------------------------------------------------------------------------
// Gaussian reconstruction filter along one axis (sec. 2.3, filter eq.):
//   f_i = exp(-alpha ((X - c_i)/w)^2) - exp(-alpha (nu/2)^2) inside the support, c_i = (i + 1/2) w - R,
// window = the NU pixels centred on the landing pixel i0, pixels outside the grid excluded, normalised (with
// NORM = false the weights stay unnormalised and their sum goes to *Sout, so that a caller normalising the
// product of two axes takes one reciprocal instead of two).
// F[m] is the weight of pixel i0 - (NU-1)/2 + m; dF[m] = dF/dX.  With box (the simplest reconstruction of
// sec. 2.3, the indicator of the pixel) the window holds the landing pixel alone, with weight 1 and no
// derivative.
// ------------------------------------------------------------------------------------------------
template <int NU, bool DERIV, bool NORM = true>
__device__ __forceinline__ int filter_axis(float X, float R, float w, float inv_w, int n, float alpha,
                                           float edge, float* F, float* dF, bool box, float* Sout = nullptr) {
    constexpr int H = (NU - 1) / 2;
    int i0 = (int)floorf((X + R) * inv_w);
    i0 = min(max(i0, 0), n - 1);
    if (box) {
#pragma unroll
        for (int m = 0; m < NU; ++m) {
            F[m] = m == H ? 1.0f : 0.0f;
            if constexpr (DERIV) dF[m] = 0.0f;
        }
        if constexpr (!NORM) *Sout = 1.0f;
        return i0;
    }
    float c0 = ((float)i0 + 0.5f) * w - R;
    float delta = (X - c0) * inv_w;  // offset from the centre of pixel i0, in pixel widths
    float S = 0.0f, Sp = 0.0f;
    float fp[NU];
    const float alpha_l2 = alpha * 1.44269504f;  // exp(-alpha d^2) = 2^(-alpha log2(e) d^2)
#pragma unroll
    for (int m = 0; m < NU; ++m) {
        int i = i0 + m - H;
        float dm = delta - (float)(m - H);
        float e = DERIV ? __expf(-alpha * dm * dm) : __builtin_amdgcn_exp2f(-alpha_l2 * dm * dm);
        if constexpr (DERIV) {
            bool in = (i >= 0) && (i < n) && (fabsf(dm) < 0.5f * (float)NU);
            F[m] = in ? e - edge : 0.0f;
            fp[m] = in ? -2.0f * alpha * dm * e * inv_w : 0.0f;
            Sp += fp[m];
        } else {
            // the window is centred on the landing pixel, so |dm| <= nu / 2 and the support test is e >= edge
            F[m] = (i >= 0) && (i < n) ? fmaxf(e - edge, 0.0f) : 0.0f;
        }
        S += F[m];
    }
    if constexpr (!NORM) {
        *Sout = S;
        return i0;
    }
    float invS = rcpf(S);
#pragma unroll
    for (int m = 0; m < NU; ++m) {
        F[m] *= invS;
        if constexpr (DERIV) dF[m] = (fp[m] - F[m] * Sp) * invS;
    }
    return i0;
}

// ------------------------------------------------------------------------------------------------
// One ray, forward.
// ------------------------------------------------------------------------------------------------
struct FwdRay {
    int status;
    float X, Y, w;
    float t, u, v;
    int iters, failed, nonmono, refined;
};

template <int P, int Q, int KIND>
__device__ __forceinline__ FwdRay trace_forward(const DesignDev& D, const BoundsDev& B, const float* sP,
                                                const float* sKu, const float* sKv, const float* sS, int e, int ku,
                                                int kv, uint64_t ctr,
                                                float* tsave = nullptr, float t_guess = -1.0f) {
    FwdRay o;
    o.iters = o.failed = o.nonmono = o.refined = 0;
    o.X = o.Y = o.w = o.t = o.u = o.v = 0.0f;
    constexpr bool POINT = (KIND & 1) != 0, MESH = (KIND & 2) != 0, ENTRY = (KIND & 4) != 0;
    // with a freeform entry face every ray reaches the exit face from an arbitrary point and direction: the
    // exit hit needs the root search for collimated rays too
    constexpr bool SEARCH = POINT || ENTRY;
    RayIn r;
    if constexpr (ENTRY) {
        EntryHit H;
        r = ray_entry_ff<P, Q, POINT>(D, B, sP + D.n_u * D.n_v, sKu, sKv, e, ku, kv, ctr, H);
    } else {
        r = ray_entry<KIND>(D, e, ku, kv, ctr);
    }
    o.status = r.status;
    // exit root for the adjoint of the same step (point sources, exact root, flat entry): -1 when none
    constexpr bool STORE = POINT && !MESH && !ENTRY;
    if constexpr (STORE)
        if (tsave && r.status != ST_HIT) *tsave = -1.0f;
    if (r.status != ST_HIT) return o;
    float t;
    if constexpr (MESH) {
        // the hit on the triangle mesh; the normal is the B-spline's at the hit, on the triangle's span
        int K, L, upper = 0;
        float qz;
        if constexpr (POINT) {
            MeshRoot M = intersect_mesh<P, Q>(D, B, sP, sKu, sKv, r);
            o.iters = M.cells;
            if (M.status != ST_HIT) {
                o.status = M.status;
                return o;
            }
            t = M.t;
            K = M.K;
            L = M.L;
            qz = r.oz + t * r.dz;
        } else {
            float a, b;
            mesh_locate(D, r.ox, r.oy, K, L, a, b);
            upper = a + b >= 1.0f;
            MeshCell<P, Q> C;
            mesh_cell<P, Q>(D, sP, sKu, sKv, K, L, C);
            float A, Bs;
            tri_slopes<P, Q>(C, upper, A, Bs);
            qz = (upper ? C.z11 + A * (a - 1.0f) + Bs * (b - 1.0f) : C.z00 + A * a + Bs * b) + B.zref;
            t = qz - r.oz;
        }
        const float qx = r.ox + t * r.dx, qy = r.oy + t * r.dy;
        SurfEval<P, Q, float> S;
        eval_surface_on<P, Q, false, float>(D, sP, sKu, sKv, qx, qy, K / D.mesh_u, L / D.mesh_v, S);
        o.t = t;
        o.u = qx * (0.5f / D.r_x) + 0.5f;
        o.v = qy * (0.5f / D.r_y) + 0.5f;
        ExitState E = exit_face(D, qx, qy, qz, r.dx, r.dy, r.dz, S.hx, S.hy, r.w);
        o.status = E.status;
        if (E.status == ST_TIR) return o;
        o.X = E.X;
        o.Y = E.Y;
        o.w = E.w;
        return o;
    }
    if constexpr (SEARCH) {
        RootOut R = intersect<P, Q>(D, B, sP, sKu, sKv, sS, r, t_guess);
        if constexpr (STORE)
            if (tsave) *tsave = R.status == ST_HIT ? R.t : -1.0f;
        o.iters = R.iters;
        o.failed = R.failed;
        o.nonmono = R.nonmono;
        o.refined = R.refined;
        if (R.status != ST_HIT) {
            o.status = R.status;
            return o;
        }
        t = R.t;
    } else {
        t = 0.0f;
    }
    float qx = r.ox + t * r.dx, qy = r.oy + t * r.dy;
    SurfEval<P, Q, float> S;
    if constexpr (SEARCH)
        eval_surface<P, Q, false, float>(D, sP, sKu, sKv, qx, qy, S);
    else
        eval_surface_local<P, Q, false, float>(D, sP, sKu, sKv, r.su, r.sv, r.tu, r.tv, S);
    float qz = SEARCH ? r.oz + t * r.dz : S.h + B.zref;
    if constexpr (!SEARCH) t = qz - r.oz;
    o.t = t;
    o.u = qx * (0.5f / D.r_x) + 0.5f;
    o.v = qy * (0.5f / D.r_y) + 0.5f;
    ExitState E = exit_face(D, qx, qy, qz, r.dx, r.dy, r.dz, S.hx, S.hy, r.w);
    o.status = E.status;
    if (E.status == ST_TIR) return o;
    o.X = E.X;
    o.Y = E.Y;
    o.w = E.w;
    return o;
}

// ------------------------------------------------------------------------------------------------
// Rays whose pathwise derivative single precision cannot resolve.  The derivative of a ray's contribution
// jumps where its landing crosses a pixel edge (for odd nu the filter's support edges are pixel edges, where
// the filter is only continuous) or the screen edge, and it grows as 1 / sqrt(k) towards total internal
// reflection; on the triangle mesh it also jumps where the hit crosses a triangle's edge.  A landing carries
// ~1e-5 pixel of single-precision error (at most ~1e-3 on the stated workloads, 4e-4 for 1 ray in 10^4), so
// single precision may take the other side of such a kink.  The adjoint (every kernel group) leaves these rays
// out and queues them; k_adjoint_fp64 re-traces them in double precision from their samples and adds their
// contributions to the same fixed-point sums.
// ------------------------------------------------------------------------------------------------
constexpr float FLAG_EDGE_PX = 5e-4f;   // landing within this many pixel widths of a pixel edge
constexpr float FLAG_K_HIT = 1e-4f;     // a kept ray with k below this: derivative error above ~1e-3 of it
constexpr float FLAG_K_TIR = 1e-5f;     // a ray dropped for TIR with k above -this may be kept in double
constexpr float FLAG_TRI = 1e-4f;       // mesh: a hit within this many cell units of its triangle's edge

__device__ __forceinline__ bool near_pixel_edge(float X, float R, float inv_w, int n) {
    const float px = (X + R) * inv_w;
    const float r = rintf(px);
    return r >= 0.0f && r <= (float)n && fabsf(px - r) < FLAG_EDGE_PX;
}

// ------------------------------------------------------------------------------------------------
// One ray, adjoint: re-trace, gather dL/dI over the filter window, reverse sweep.  Returns false when the
// ray does not reach the screen.  With tload (point sources, exact root, flat entry) the exit root comes from
// the forward of the same step instead of the search.  g[] receives dL/dP for control point (ku + a, kv + b) at a * (Q+1) + b;
// with a freeform entry face gin[] receives dL/dP of the entry net's points (cku_in + a, ckv_in + b).
// ------------------------------------------------------------------------------------------------
struct NoQueue {
    __device__ bool operator()(float, float) const { return false; }
};

template <int P, int Q, int NU, int KIND, class Enqueue = NoQueue>
__device__ __forceinline__ bool trace_adjoint(const DesignDev& D, const BoundsDev& B, const float* sP,
                                              const float* sKu, const float* sKv, const float* sS,
                                              const float* __restrict__ G,
                                              int e, int ku, int kv, uint64_t ctr, int& cku, int& ckv,
                                              float* g, int& cku_in, int& ckv_in, float* gin,
                                              const float* tload = nullptr, Enqueue enqueue = Enqueue()) {
    constexpr bool point = (KIND & 1) != 0, MESH = (KIND & 2) != 0, ENTRY = (KIND & 4) != 0;
    constexpr bool SEARCH = point || ENTRY;
    EntryHit EH;
    RayIn r;
    if constexpr (ENTRY) {
        r = ray_entry_ff<P, Q, point>(D, B, sP + D.n_u * D.n_v, sKu, sKv, e, ku, kv, ctr, EH);
    } else {
        r = ray_entry<KIND>(D, e, ku, kv, ctr);
    }
    if (r.status != ST_HIT) return false;
    float t = 0.0f;
    // mesh: the hit triangle, its cell (corner heights and node basis) and the hit's in-cell coordinates
    MeshCell<P, Q> C;
    int mK = 0, mL = 0, mup = 0;
    float ma = 0.0f, mb = 0.0f, mqz = 0.0f;
    if constexpr (MESH) {
        if constexpr (point) {
            MeshRoot M = intersect_mesh<P, Q>(D, B, sP, sKu, sKv, r);
            if (M.status != ST_HIT) return false;
            t = M.t;
            mK = M.K;
            mL = M.L;
            mup = M.upper;
            ma = ((r.ox + t * r.dx) * D.sxu + D.ubar0) * (float)D.mesh_u - (float)mK;
            mb = ((r.oy + t * r.dy) * D.syv + D.vbar0) * (float)D.mesh_v - (float)mL;
        } else {
            mesh_locate(D, r.ox, r.oy, mK, mL, ma, mb);
            mup = ma + mb >= 1.0f;
        }
        mesh_cell<P, Q>(D, sP, sKu, sKv, mK, mL, C);
        if constexpr (!point) {
            float A, Bs;
            tri_slopes<P, Q>(C, mup, A, Bs);
            mqz = (mup ? C.z11 + A * (ma - 1.0f) + Bs * (mb - 1.0f) : C.z00 + A * ma + Bs * mb) + B.zref;
        }
    } else if constexpr (SEARCH) {
        bool found = false;
        if constexpr (!ENTRY) {
            // the exit root the forward of this step stored (-1: no hit), instead of searching again
            if (tload) {
                t = *tload;
                if (!(t >= 0.0f)) return false;
                found = true;
            }
        }
        if (!found) {
            RootOut R = intersect<P, Q>(D, B, sP, sKu, sKv, sS, r);
            if (R.status != ST_HIT) return false;
            t = R.t;
        }
    }
    float qx = r.ox + t * r.dx, qy = r.oy + t * r.dy;
    SurfEval<P, Q, float> S;
    if constexpr (MESH) {
        // the normal is the B-spline's at the hit, on the triangle's span product
        eval_surface_on<P, Q, point, float>(D, sP, sKu, sKv, qx, qy, C.su, C.sv, S);
    } else if constexpr (SEARCH) {
        eval_surface<P, Q, true, float>(D, sP, sKu, sKv, qx, qy, S);
    } else {
        // the hit of a collimated ray does not move with P: no second derivatives needed
        eval_surface_local<P, Q, false, float>(D, sP, sKu, sKv, r.su, r.sv, r.tu, r.tv, S);
    }
    float qz = SEARCH ? r.oz + t * r.dz : (MESH ? mqz : S.h + B.zref);
    ExitState E = exit_face(D, qx, qy, qz, r.dx, r.dy, r.dz, S.hx, S.hy, r.w);
    {
        // a derivative single precision cannot resolve (see FLAG_EDGE_PX): enqueue() may take the ray for the
        // double-precision re-trace (with its roots), which then makes the contribution instead of this sweep.
        // On the mesh the derivative also jumps where the hit crosses a triangle's edge (the slopes change).
        bool flag = E.status == ST_TIR ? E.k > -FLAG_K_TIR
                                       : E.k < FLAG_K_HIT || near_pixel_edge(E.X, D.Rx, D.inv_wx, D.nx) ||
                                             near_pixel_edge(E.Y, D.Ry, D.inv_wy, D.ny);
        if constexpr (MESH)
            flag = flag || fminf(fminf(ma, mb), fminf(1.0f - ma, 1.0f - mb)) < FLAG_TRI ||
                   fabsf(ma + mb - 1.0f) < FLAG_TRI;
        if (flag && !D.box && enqueue(t, ENTRY ? EH.t : 0.0f)) return false;
    }
    if (E.status != ST_HIT) return false;

    // ---- splat, reverse: I_ij += w Fx_i Fy_j
    float Fx[NU], dFx[NU], Fy[NU], dFy[NU];
    int i0 = filter_axis<NU, true>(E.X, D.Rx, D.wx, D.inv_wx, D.nx, D.alpha, D.edge_x, Fx, dFx, D.box);
    int j0 = filter_axis<NU, true>(E.Y, D.Ry, D.wy, D.inv_wy, D.ny, D.alpha, D.edge_y, Fy, dFy, D.box);
    constexpr int H = (NU - 1) / 2;
    float wbar = 0.0f, Xbar = 0.0f, Ybar = 0.0f;
#pragma unroll
    for (int a = 0; a < NU; ++a) {
        int i = min(max(i0 + a - H, 0), D.nx - 1);
        float gb = 0.0f, gbp = 0.0f;
#pragma unroll
        for (int b = 0; b < NU; ++b) {
            int j = min(max(j0 + b - H, 0), D.ny - 1);
            float Gij = G[(int64_t)i * D.ny + j];
            gb += Gij * Fy[b];
            gbp += Gij * dFy[b];
        }
        wbar += Fx[a] * gb;
        Xbar += dFx[a] * gb;
        Ybar += Fx[a] * gbp;
    }
    Xbar *= E.w;
    Ybar *= E.w;

    // ---- screen: X = q_x + tau e_x, Y = q_y + tau e_y, tau = (z_s - q_z) / e_z
    float qxb = Xbar, qyb = Ybar;
    float taub = Xbar * E.ex + Ybar * E.ey;
    float inv_ez = rcpf(E.ez);
    float exb = Xbar * E.tau, eyb = Ybar * E.tau, ezb = -taub * E.tau * inv_ez;
    float qzb = -taub * inv_ez;
    // ---- Schlick: w = w1 T(sk)
    float skb = 0.0f;
    if (D.fresnel) {
        float m = 1.0f - E.sk, m2 = m * m;
        skb = wbar * r.w * 5.0f * (1.0f - D.R0) * m2 * m2;
    }
    // ---- refraction: e = n d + beta n_hat, beta = sk - n c, sk = sqrt(k), k = 1 - n^2 (1 - c^2), c = d.n_hat
    float n = D.n_lens;
    float betab = exb * E.nxh + eyb * E.nyh + ezb * E.nzh;
    float nxb = E.beta * exb, nyb = E.beta * eyb, nzb = E.beta * ezb;
    skb += betab;
    float cb = -n * betab;
    float kb = skb * 0.5f * rcpf(fmaxf(E.sk, 1e-30f));
    cb += 2.0f * n * n * E.c * kb;
    nxb += cb * r.dx;
    nyb += cb * r.dy;
    nzb += cb * r.dz;
    // ---- n_hat = m / |m|, m = (-h_x, -h_y, 1)
    float ndot = nxb * E.nxh + nyb * E.nyh + nzb * E.nzh;
    float mxb = (nxb - ndot * E.nxh) * E.inv_m;
    float myb = (nyb - ndot * E.nyh) * E.inv_m;
    float hxb = -mxb, hyb = -myb;
    // ---- hit point: coefficient of N_a M_b in dL/dP
    float g0;
    if (SEARCH) {
        // q = o + t d; t moves with P through f(t, P) = 0: dt/dP_ab = -N_a M_b / f'(t)
        float tb = qxb * r.dx + qyb * r.dy + qzb * r.dz + hxb * (S.hxx * r.dx + S.hxy * r.dy) +
                   hyb * (S.hxy * r.dx + S.hyy * r.dy);
        float fp = S.hx * r.dx + S.hy * r.dy - r.dz;
        if constexpr (MESH) {
            // on the mesh f(t) = T(q(t)) - q_z(t): f' = T_x d_x + T_y d_y - d_z, and T moves with the corner
            // heights, dT/dz_c = the barycentric weight of corner c (applied below)
            float A, Bs;
            tri_slopes<P, Q>(C, mup, A, Bs);
            fp = A * D.sxu * (float)D.mesh_u * r.dx + Bs * D.syv * (float)D.mesh_v * r.dy - r.dz;
        }
        g0 = -tb * rcpf(fp);
    } else {
        g0 = qzb;  // q_z = h(x, y), or the triangle's height on the mesh
    }
    // h_x = sum dN_a/du M_b P_ab * sxu, h_y = sum N_a dM_b/dv P_ab * syv
    float gx = hxb * D.sxu, gy = hyb * D.syv;
    if constexpr (MESH) {
        // the hit (and the height of a collimated hit) follows the triangle: its corner heights carry the
        // weights l_c of the hit, z_c = sum_ab N_a(u_c) M_b(v_c) P_ab, so dP_ab gets
        // g0 sum_c l_c N_a(u_c) M_b(v_c) = g0 (X0_a Nv0_b + X1_a Nv1_b); the normal's terms are the exact ones
        float X0[P + 1], X1[P + 1];
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            if (mup) {  // corners 11 (a + b - 1), 01 (1 - a), 10 (1 - b)
                X0[a] = (1.0f - mb) * C.Nu1[a];
                X1[a] = (ma + mb - 1.0f) * C.Nu1[a] + (1.0f - ma) * C.Nu0[a];
            } else {    // corners 00 (1 - a - b), 10 (a), 01 (b)
                X0[a] = (1.0f - ma - mb) * C.Nu0[a] + ma * C.Nu1[a];
                X1[a] = mb * C.Nu0[a];
            }
        }
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            float du = gx * S.dNu[a];
#pragma unroll
            for (int b = 0; b <= Q; ++b)
                g[a * (Q + 1) + b] = g0 * (X0[a] * C.Nv0[b] + X1[a] * C.Nv1[b]) + S.Nu[a] * gy * S.dNv[b] +
                                     du * S.Nv[b];
        }
        cku = S.ku;
        ckv = S.kv;
        return true;
    }
    float cv[Q + 1];
#pragma unroll
    for (int b = 0; b <= Q; ++b) cv[b] = g0 * S.Nv[b] + gy * S.dNv[b];
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        float du = gx * S.dNu[a];
#pragma unroll
        for (int b = 0; b <= Q; ++b) g[a * (Q + 1) + b] = S.Nu[a] * cv[b] + du * S.Nv[b];
    }
    cku = S.ku;
    ckv = S.kv;
    if constexpr (ENTRY) {
        // ---- back through the exit root into the ray inside the glass, q = o + t d with f(t; o, d) = 0:
        // dt/do = -(h_x, h_y, -1) / f', dt/dd = t dt/do; q_bar includes the exit normal's dependence on q
        const float qbx = qxb + hxb * S.hxx + hyb * S.hxy, qby = qyb + hxb * S.hxy + hyb * S.hyy;
        const float obx = qbx + g0 * S.hx, oby = qby + g0 * S.hy, obz = qzb - g0;
        // d: directly through the exit refraction (e = n d + beta n_hat, c = d . n_hat) and through q
        const float dbx = n * exb + cb * E.nxh + t * obx;
        const float dby = n * eyb + cb * E.nyh + t * oby;
        const float dbz = n * ezb + cb * E.nzh + t * obz;
        // ---- entry refraction, air -> glass: d = eta d0 + beta_i m_hat, beta_i = sqrt(k_i) - eta c_i,
        // c_i = d0 . m_hat, k_i = 1 - eta^2 (1 - c_i^2); weight w1 = w0 (1 - Schlick(c_i)); final w = w1 T_exit
        const float* sPin = sP + D.n_u * D.n_v;
        SurfEval<P, Q, float> Si;
        eval_surface<P, Q, point, float>(D, sPin, sKu, sKv, r.ox, r.oy, Si);
        const float inv_i = rsqrtf(Si.hx * Si.hx + Si.hy * Si.hy + 1.0f);
        const float mx = -Si.hx * inv_i, my = -Si.hy * inv_i, mz = inv_i;
        const float eta = rcpf(D.n_lens);
        const float ci = EH.d0x * mx + EH.d0y * my + EH.d0z * mz;
        const float ski = sqrt_hw(fmaxf(1.0f - eta * eta * (1.0f - ci * ci), 1e-30f));
        const float betai = ski - eta * ci;
        float cib = (dbx * mx + dby * my + dbz * mz) * (eta * eta * ci / ski - eta);
        if (D.fresnel) {
            const float mm = 1.0f - ci, mm2 = mm * mm;
            cib += wbar * E.T * D.w0 * 5.0f * (1.0f - D.R0) * mm2 * mm2;
        }
        const float nbx = betai * dbx + cib * EH.d0x, nby = betai * dby + cib * EH.d0y,
                    nbz = betai * dbz + cib * EH.d0z;
        const float nd = nbx * mx + nby * my + nbz * mz;
        const float gxb_i = -(nbx - nd * mx) * inv_i, gyb_i = -(nby - nd * my) * inv_i;
        // ---- entry hit: collimated rays meet the face at fixed (x, y), so only its height moves; point-source
        // rays move along s + t_i d0 with g(s + t_i d0) = s_z + t_i d0_z (the entry normal's dependence on the
        // hit included, as at the exit face)
        float c0;
        if constexpr (point) {
            const float pbx = obx + gxb_i * Si.hxx + gyb_i * Si.hxy, pby = oby + gxb_i * Si.hxy + gyb_i * Si.hyy;
            const float tbi = pbx * EH.d0x + pby * EH.d0y + obz * EH.d0z;
            const float fpi = Si.hx * EH.d0x + Si.hy * EH.d0y - EH.d0z;
            c0 = -tbi * rcpf(fpi);
        } else {
            c0 = obz;
        }
        const float gxi = gxb_i * D.sxu, gyi = gyb_i * D.syv;
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            const float du = gxi * Si.dNu[a];
#pragma unroll
            for (int b = 0; b <= Q; ++b)
                gin[a * (Q + 1) + b] = Si.Nu[a] * (c0 * Si.Nv[b] + gyi * Si.dNv[b]) + du * Si.Nv[b];
        }
        cku_in = Si.ku;
        ckv_in = Si.kv;
    }
    return true;
}

// B-spline basis of span k (0-based) of nspan on the clamped uniform knots, in double precision, with the
// local knots and reciprocals of the Cox-de Boor recursion formed in double (the knot table in LDS holds
// single-precision reciprocals).  t = ubar - k in [0, 1].
template <int P, bool D2>
__device__ inline void basis_f64(int k, int nspan, double t, double* N, double* dN, double* d2N) {
    if (k >= P - 1 && k <= nspan - P) {  // unclamped knots: the uniform B-spline
        span_basis<P, D2, true, double>(nullptr, t, N, dN, d2N);
        return;
    }
    int kap[2 * P];
#pragma unroll
    for (int i = 0; i < 2 * P; ++i) kap[i] = min(max(i + 1 - P, -k), nspan - k);
    auto KAP = [&](int o) { return (double)kap[o + P - 1]; };
    auto REC = [&](int deg, int j) {  // 1 / (kap(j) - kap(j - deg)), a knot difference of 0 .. P units
        const int d = kap[j + P - 1] - kap[j - deg + P - 1];
        return d == 1 ? 1.0 : d == 2 ? 0.5 : d == 3 ? 1.0 / 3.0 : d == 4 ? 0.25 : d == 5 ? 0.2 : 0.0;
    };
    double tb[P + 1][P + 1];
    tb[0][0] = 1.0;
#pragma unroll
    for (int deg = 1; deg <= P; ++deg) {
#pragma unroll
        for (int m = 0; m <= deg; ++m) {
            double acc = 0.0;
            if (m >= 1) acc += (t - KAP(m - deg)) * REC(deg, m) * tb[deg - 1][m - 1];
            if (m <= deg - 1) acc += (KAP(m + 1) - t) * REC(deg, m + 1) * tb[deg - 1][m];
            tb[deg][m] = acc;
        }
    }
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        N[m] = tb[P][m];
        const double a = m >= 1 ? REC(P, m) * tb[P - 1][m - 1] : 0.0;
        const double b = m <= P - 1 ? REC(P, m + 1) * tb[P - 1][m] : 0.0;
        dN[m] = (double)P * (a - b);
    }
    if constexpr (D2) {
        if constexpr (P >= 2) {
            double d1[P];
#pragma unroll
            for (int m = 0; m <= P - 1; ++m) {
                const double a = m >= 1 ? REC(P - 1, m) * tb[P - 2][m - 1] : 0.0;
                const double b = m <= P - 2 ? REC(P - 1, m + 1) * tb[P - 2][m] : 0.0;
                d1[m] = (double)(P - 1) * (a - b);
            }
#pragma unroll
            for (int m = 0; m <= P; ++m) {
                const double a = m >= 1 ? REC(P, m) * d1[m - 1] : 0.0;
                const double b = m <= P - 1 ? REC(P, m + 1) * d1[m] : 0.0;
                d2N[m] = (double)P * (a - b);
            }
        } else {
#pragma unroll
            for (int m = 0; m <= P; ++m) d2N[m] = 0.0;
        }
    }
}

// Surface and derivatives in double precision from the device control heights (absolute), on the span
// product containing (x, y).
template <int P, int Q, bool D2>
__device__ inline void surface_f64(const DesignDev& D, const DesignDev64& E, const float* __restrict__ Pz, double x,
                                   double y, SurfEval<P, Q, double>& S) {
    const double ub = x * E.sxu + E.ubar0, vb = y * E.syv + E.vbar0;
    const int ku = min(max((int)floor(ub), 0), D.nsu - 1), kv = min(max((int)floor(vb), 0), D.nsv - 1);
    S.ku = ku;
    S.kv = kv;
    basis_f64<P, D2>(ku, D.nsu, ub - (double)ku, S.Nu, S.dNu, S.d2Nu);
    basis_f64<Q, D2>(kv, D.nsv, vb - (double)kv, S.Nv, S.dNv, S.d2Nv);
    const float* row = Pz + D.cp_off + (int64_t)ku * D.n_v + kv;
    double h = 0.0, hu = 0.0, hv = 0.0, huu = 0.0, huv = 0.0, hvv = 0.0;
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        double r0 = 0.0, r1 = 0.0, r2 = 0.0;
#pragma unroll
        for (int b = 0; b <= Q; ++b) {
            const double pz = (double)row[a * D.n_v + b];
            r0 += S.Nv[b] * pz;
            r1 += S.dNv[b] * pz;
            if constexpr (D2) r2 += S.d2Nv[b] * pz;
        }
        h += S.Nu[a] * r0;
        hu += S.dNu[a] * r0;
        hv += S.Nu[a] * r1;
        if constexpr (D2) {
            huu += S.d2Nu[a] * r0;
            huv += S.dNu[a] * r1;
            hvv += S.Nu[a] * r2;
        }
    }
    S.h = h;
    S.hx = hu * E.sxu;
    S.hy = hv * E.syv;
    if constexpr (D2) {
        S.hxx = huu * E.sxu * E.sxu;
        S.hxy = huv * E.sxu * E.syv;
        S.hyy = hvv * E.syv * E.syv;
    }
}

// The normalised filter of one axis and its derivative in double precision (as filter_axis).
template <int NU>
__device__ inline int filter_axis_f64(double X, double R, double w, int n, double alpha, double edge, double* F,
                                      double* dF) {
    constexpr int H = (NU - 1) / 2;
    int i0 = (int)floor((X + R) / w);
    i0 = min(max(i0, 0), n - 1);
    const double delta = (X - (((double)i0 + 0.5) * w - R)) / w;
    double S = 0.0, Sp = 0.0, fp[NU];
#pragma unroll
    for (int m = 0; m < NU; ++m) {
        const int i = i0 + m - H;
        const double dm = delta - (double)(m - H);
        const bool in = i >= 0 && i < n && fabs(dm) < 0.5 * NU;
        const double e = exp(-alpha * dm * dm);
        F[m] = in ? e - edge : 0.0;
        fp[m] = in ? -2.0 * alpha * dm * e / w : 0.0;
        S += F[m];
        Sp += fp[m];
    }
#pragma unroll
    for (int m = 0; m < NU; ++m) {
        F[m] /= S;
        dF[m] = (fp[m] - F[m] * Sp) / S;
    }
    return i0;
}

// Surface and derivatives in double precision on a given span product (su, sv) at (x, y) (the mesh's normal is
// the B-spline's on the hit triangle's span product).
template <int P, int Q, bool D2>
__device__ inline void surface_f64_on(const DesignDev& D, const DesignDev64& E, const float* __restrict__ Pz, double x,
                                      double y, int su, int sv, SurfEval<P, Q, double>& S) {
    S.ku = su;
    S.kv = sv;
    basis_f64<P, D2>(su, D.nsu, x * E.sxu + E.ubar0 - (double)su, S.Nu, S.dNu, S.d2Nu);
    basis_f64<Q, D2>(sv, D.nsv, y * E.syv + E.vbar0 - (double)sv, S.Nv, S.dNv, S.d2Nv);
    const float* row = Pz + D.cp_off + (int64_t)su * D.n_v + sv;
    double h = 0.0, hu = 0.0, hv = 0.0, huu = 0.0, huv = 0.0, hvv = 0.0;
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        double r0 = 0.0, r1 = 0.0, r2 = 0.0;
#pragma unroll
        for (int b = 0; b <= Q; ++b) {
            const double pz = (double)row[a * D.n_v + b];
            r0 += S.Nv[b] * pz;
            r1 += S.dNv[b] * pz;
            if constexpr (D2) r2 += S.d2Nv[b] * pz;
        }
        h += S.Nu[a] * r0;
        hu += S.dNu[a] * r0;
        hv += S.Nu[a] * r1;
        if constexpr (D2) {
            huu += S.d2Nu[a] * r0;
            huv += S.dNu[a] * r1;
            hvv += S.Nu[a] * r2;
        }
    }
    S.h = h;
    S.hx = hu * E.sxu;
    S.hy = hv * E.syv;
    if constexpr (D2) {
        S.hxx = huu * E.sxu * E.sxu;
        S.hxy = huv * E.sxu * E.syv;
        S.hyy = hvv * E.syv * E.syv;
    }
}

// The hit of a ray on the triangle mesh in double precision, found near the single-precision hit t32 (a
// collimated ray, d = (0, 0, 1), meets the mesh above its sample): the cell holding that hit first, then, while neither of a cell's triangles holds its plane's hit, the
// neighbouring cell where the lower triangle's plane is met.  Triangles as in intersect_mesh, with the
// partition's closed and open edges (the lower triangle's diagonal open, the upper one's right and upper edges
// open but on the border of the net).  Out: t, the triangle (span product su, sv; upper), the hit's in-cell
// coordinates (a, b), the triangle's slopes per cell unit (A, B) and the basis at the cell's node columns
// and rows.
template <int P, int Q>
struct MeshHit64 {
    double t, a, b, A, B;
    int su, sv, upper;
    double Nu0[P + 1], Nu1[P + 1], Nv0[Q + 1], Nv1[Q + 1];
};

template <int P, int Q>
__device__ bool mesh_hit_f64(const DesignDev& D, const DesignDev64& E, const float* __restrict__ Pz, double ox,
                             double oy, double oz, double dx, double dy, double dz, float t32, MeshHit64<P, Q>& M) {
    const int MU = D.mesh_u, MV = D.mesh_v, NK = D.nsu * MU, NL = D.nsv * MV;
    const double cu = (ox * E.sxu + E.ubar0) * MU, dcu = dx * E.sxu * MU;  // cell coordinates at t: cu + dcu t
    const double cv = (oy * E.syv + E.vbar0) * MV, dcv = dy * E.syv * MV;
    const double t0 = (double)t32;
    int K = min(max((int)floor(cu + dcu * t0), 0), NK - 1), L = min(max((int)floor(cv + dcv * t0), 0), NL - 1);
    double dn[(P > Q ? P : Q) + 1];
    for (int it = 0; it < 8; ++it) {
        const int su = K / MU, sv = L / MV;
        basis_f64<P, false>(su, D.nsu, (double)(K - su * MU) / MU, M.Nu0, dn, nullptr);
        basis_f64<P, false>(su, D.nsu, (double)(K - su * MU + 1) / MU, M.Nu1, dn, nullptr);
        basis_f64<Q, false>(sv, D.nsv, (double)(L - sv * MV) / MV, M.Nv0, dn, nullptr);
        basis_f64<Q, false>(sv, D.nsv, (double)(L - sv * MV + 1) / MV, M.Nv1, dn, nullptr);
        const float* row = Pz + D.cp_off + (int64_t)su * D.n_v + sv;
        double z00 = 0.0, z10 = 0.0, z01 = 0.0, z11 = 0.0;
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            double r0 = 0.0, r1 = 0.0;
#pragma unroll
            for (int b = 0; b <= Q; ++b) {
                const double pz = (double)row[a * D.n_v + b];
                r0 += M.Nv0[b] * pz;
                r1 += M.Nv1[b] * pz;
            }
            z00 += M.Nu0[a] * r0;
            z10 += M.Nu1[a] * r0;
            z01 += M.Nu0[a] * r1;
            z11 += M.Nu1[a] * r1;
        }
        const bool last_u = K == NK - 1, last_v = L == NL - 1;
        const double a0 = cu - (double)K, b0 = cv - (double)L;
        int mK = 0, mL = 0;
        double t_up = -1.0, a_up = 0.0, b_up = 0.0;
        for (int tri = 0; tri < 2; ++tri) {
            const double A = tri ? z11 - z01 : z10 - z00, B = tri ? z11 - z10 : z01 - z00;
            const double den = dz - A * dcu - B * dcv;
            if (den == 0.0) continue;
            const double num = tri ? z11 + A * (a0 - 1.0) + B * (b0 - 1.0) - oz : z00 + A * a0 + B * b0 - oz;
            const double t = num / den, a = a0 + dcu * t, b = b0 + dcv * t;
            const bool in = tri ? (a + b >= 1.0 && (a < 1.0 || (last_u && a <= 1.0)) && (b < 1.0 || (last_v && b <= 1.0)))
                                : (a >= 0.0 && b >= 0.0 && a + b < 1.0);
            if (in && t >= 0.0) {
                M.t = t;
                M.a = a;
                M.b = b;
                M.A = A;
                M.B = B;
                M.su = su;
                M.sv = sv;
                M.upper = tri;
                return true;
            }
            if (tri == 0) {
                mK = a < 0.0 ? -1 : (a >= 1.0 ? 1 : 0);
                mL = b < 0.0 ? -1 : (b >= 1.0 ? 1 : 0);
            } else {
                t_up = t;
                a_up = a;
                b_up = b;
            }
        }
        if (mK == 0 && mL == 0) {
            // both planes met inside the cell, each on the other triangle's side: the ray crosses the fold at
            // the diagonal, which belongs to the upper triangle
            if (!(t_up >= 0.0)) return false;
            M.t = t_up;
            M.a = a_up;
            M.b = b_up;
            M.A = z11 - z01;
            M.B = z11 - z10;
            M.su = su;
            M.sv = sv;
            M.upper = 1;
            return true;
        }
        K += mK;
        L += mL;
        if (K < 0 || K >= NK || L < 0 || L >= NL) return false;
    }
    return false;
}

// One queued ray in double precision: the whole trace from its sample (exact roots polished from the
// single-precision ones by Newton steps on the double-precision surfaces) and the reverse sweep of
// trace_adjoint.  Returns false when, in double precision, the ray does not reach the screen; else g[] holds
// dL/dP of the exit net's control points (ku + a, kv + b) at a (Q+1) + b.  MODE 0: flat entry face, exact
// root.  MODE 1 (F64_TWO), 3 (F64_TWO_COLL): a point-source (collimated) ray through a lens whose entry face is
// freeform too (a point-source ray's entry root ti32 queued beside the exit root; a collimated ray meets the
// entry face above its sample); gin[] then holds dL/dP of the entry net's points (cku_in + a, ckv_in + b).  MODE 2 (F64_MESH): a ray on the triangle mesh of
// sec. 2.2.2, whose hit triangle is found again in double precision near the single-precision hit.
template <int P, int Q, int NU, int MODE = F64_FLAT>
__device__ bool trace_adjoint_f64(const DesignDev& D, const DesignDev64& E, const float* __restrict__ Pz,
                                  const float* __restrict__ G, int64_t id, float t32, int& cku, int& ckv, double* g,
                                  float ti32 = 0.0f, int* cku_in = nullptr, int* ckv_in = nullptr,
                                  double* gin = nullptr) {
    const int64_t per = (int64_t)D.grid_u * D.grid_v;
    const int e = (int)(id / per);
    const int64_t rr = id - (int64_t)e * per;
    const int ku = (int)(rr / D.grid_v), kv = (int)(rr - (rr / D.grid_v) * D.grid_v);
    float x1f = 0.5f, x2f = 0.5f;
    if (D.jitter) two_uniforms(splitmix_at(D.rng_state0, (uint64_t)id), x1f, x2f);  // exact 24-bit values
    const double x1 = x1f, x2 = x2f;
    constexpr bool TWOC = MODE == F64_TWO_COLL, TWO = MODE == F64_TWO || TWOC, MESH = MODE == F64_MESH;
    const bool point = TWO || D.kind != 0;
    double ox, oy, oz, dx, dy, dz, w1;
    // (TWO) the source ray d0, the entry face at the entry hit (Si, unit normal m) and its refraction
    SurfEval<P, Q, double> Si;
    double d0x = 0.0, d0y = 0.0, d0z = 0.0, mx = 0.0, my = 0.0, mz = 0.0, inv_i = 0.0, ci = 0.0, ski = 1.0,
           betai = 0.0;
    const float* Pin = Pz + D.n_u * D.n_v;  // the entry net follows the exit net
    if constexpr (TWOC) {
        // collimated through two freeform faces: the ray meets the entry face above its sample, along +z
        ox = (2.0 * (((double)ku + x1) / (double)D.grid_u) - 1.0) * E.r_x;
        oy = (2.0 * (((double)kv + x2) / (double)D.grid_v) - 1.0) * E.r_y;
        d0z = 1.0;
        surface_f64<P, Q, true>(D, E, Pin, ox, oy, Si);
        oz = Si.h;
    } else if (!point) {
        ox = (2.0 * (((double)ku + x1) / (double)D.grid_u) - 1.0) * E.r_x;
        oy = (2.0 * (((double)kv + x2) / (double)D.grid_v) - 1.0) * E.r_y;
        oz = E.z_in;
        dx = dy = 0.0;
        dz = 1.0;
        w1 = D.fresnel ? E.w0 * (1.0 - E.R0) : E.w0;
    } else {
        double sth, cth;
        sincospi(2.0 * ((double)ku + x1) / (double)D.grid_u, &sth, &cth);
        const double ao = ((double)kv + x2) / (double)D.grid_v * E.omc;
        const double cphi = 1.0 - ao, sphi = sqrt(ao * (2.0 - ao));
        double px = E.pos_x, py = E.pos_y;
        if (D.kind == 2) {
            const int ix = e / D.emit_ny, iy = e - ix * D.emit_ny;
            px += E.ex0 + (double)ix * E.edx;
            py += E.ey0 + (double)iy * E.edy;
        }
        const double eta = 1.0 / E.n_lens;
        if constexpr (TWO) {
            // entry root: g(s + t d0) = s_z + t d0_z on the entry face, polished from the single-precision one
            d0x = cth * sphi;
            d0y = sth * sphi;
            d0z = cphi;
            const double sz = E.pos_z;
            double ti = (double)ti32;
            for (int it = 0; it < 2; ++it) {
                surface_f64<P, Q, false>(D, E, Pin, px + ti * d0x, py + ti * d0y, Si);
                const double f = Si.h - sz - ti * d0z, fp = Si.hx * d0x + Si.hy * d0y - d0z;
                if (!(fp < 0.0)) break;
                ti -= f / fp;
            }
            ox = px + ti * d0x;
            oy = py + ti * d0y;
            oz = sz + ti * d0z;
            if (fabs(ox) > E.r_x || fabs(oy) > E.r_y) return false;
            surface_f64<P, Q, true>(D, E, Pin, ox, oy, Si);
        } else {
            const double t0 = (E.z_in - E.pos_z) / cphi;
            ox = px + t0 * cth * sphi;
            oy = py + t0 * sth * sphi;
            oz = E.z_in;
            if (fabs(ox) > E.r_x || fabs(oy) > E.r_y) return false;
            dx = eta * cth * sphi;
            dy = eta * sth * sphi;
            dz = sqrt(1.0 - eta * eta * sphi * sphi);
            w1 = E.w0;
            if (D.fresnel) {
                const double m = 1.0 - cphi, m2 = m * m;
                w1 *= 1.0 - (E.R0 + (1.0 - E.R0) * m2 * m2 * m);
            }
        }
    }
    if constexpr (TWO) {
        // refraction air -> glass at the entry hit at m = (-g_x, -g_y, 1) / |.|, Schlick with the air-side cosine
        const double eta = 1.0 / E.n_lens;
        inv_i = 1.0 / sqrt(Si.hx * Si.hx + Si.hy * Si.hy + 1.0);
        mx = -Si.hx * inv_i;
        my = -Si.hy * inv_i;
        mz = inv_i;
        ci = d0x * mx + d0y * my + d0z * mz;
        ski = sqrt(fmax(1.0 - eta * eta * (1.0 - ci * ci), 1e-300));
        betai = ski - eta * ci;
        dx = eta * d0x + betai * mx;
        dy = eta * d0y + betai * my;
        dz = eta * d0z + betai * mz;
        w1 = E.w0;
        if (D.fresnel) {
            const double m = 1.0 - ci, m2 = m * m;
            w1 *= 1.0 - (E.R0 + (1.0 - E.R0) * m2 * m2 * m);
        }
    }
    SurfEval<P, Q, double> S;
    double t = 0.0, qx = ox, qy = oy, qz;
    MeshHit64<P, Q> M;  // (MESH) the hit triangle
    if (MESH) {
        if (!mesh_hit_f64<P, Q>(D, E, Pz, ox, oy, oz, dx, dy, dz, t32, M)) return false;
        t = M.t;
        qx = ox + t * dx;
        qy = oy + t * dy;
        qz = oz + t * dz;
        surface_f64_on<P, Q, true>(D, E, Pz, qx, qy, M.su, M.sv, S);
    } else if (point) {
        t = (double)t32;
        for (int it = 0; it < 2; ++it) {  // from ~1e-6 relative: ~1e-12 after one step, rounding after two
            surface_f64<P, Q, false>(D, E, Pz, ox + t * dx, oy + t * dy, S);
            const double f = S.h - oz - t * dz, fp = S.hx * dx + S.hy * dy - dz;
            if (!(fp < 0.0)) break;
            t -= f / fp;
        }
        qx = ox + t * dx;
        qy = oy + t * dy;
        qz = oz + t * dz;
        surface_f64<P, Q, true>(D, E, Pz, qx, qy, S);
    } else {
        surface_f64<P, Q, false>(D, E, Pz, qx, qy, S);
        qz = S.h;
    }
    // ---- exit face: vector Snell, TIR dropped, Schlick with the air-side cosine, screen
    const double n = E.n_lens;
    const double inv_m = 1.0 / sqrt(S.hx * S.hx + S.hy * S.hy + 1.0);
    const double nxh = -S.hx * inv_m, nyh = -S.hy * inv_m, nzh = inv_m;
    const double c = dx * nxh + dy * nyh + dz * nzh;
    const double cx = dy * nzh - dz * nyh, cy = dz * nxh - dx * nzh, cz = dx * nyh - dy * nxh;
    const double k = 1.0 - n * n * (cx * cx + cy * cy + cz * cz);
    if (!(k >= 0.0)) return false;
    const double sk = sqrt(k), beta = sk - n * c;
    const double ex = n * dx + beta * nxh, ey = n * dy + beta * nyh, ez = n * dz + beta * nzh;
    double T = 1.0;
    if (D.fresnel) {
        const double m = 1.0 - sk, m2 = m * m;
        T = 1.0 - (E.R0 + (1.0 - E.R0) * m2 * m2 * m);
    }
    const double w = w1 * T;
    if (!(ez > 0.0)) return false;
    const double tau = (E.z_screen - qz) / ez;
    const double X = qx + tau * ex, Y = qy + tau * ey;
    if (!(X >= -E.Rx && X < E.Rx && Y >= -E.Ry && Y < E.Ry)) return false;
    // ---- splat, reverse
    double Fx[NU], dFx[NU], Fy[NU], dFy[NU];
    const int i0 = filter_axis_f64<NU>(X, E.Rx, E.wx, D.nx, E.alpha, E.edge_x, Fx, dFx);
    const int j0 = filter_axis_f64<NU>(Y, E.Ry, E.wy, D.ny, E.alpha, E.edge_y, Fy, dFy);
    constexpr int H = (NU - 1) / 2;
    const float* Gd = G + D.img_off;
    double wbar = 0.0, Xbar = 0.0, Ybar = 0.0;
#pragma unroll
    for (int a = 0; a < NU; ++a) {
        const int i = min(max(i0 + a - H, 0), D.nx - 1);
        double gb = 0.0, gbp = 0.0;
#pragma unroll
        for (int b = 0; b < NU; ++b) {
            const int j = min(max(j0 + b - H, 0), D.ny - 1);
            const double Gij = (double)Gd[(int64_t)i * D.ny + j];
            gb += Gij * Fy[b];
            gbp += Gij * dFy[b];
        }
        wbar += Fx[a] * gb;
        Xbar += dFx[a] * gb;
        Ybar += Fx[a] * gbp;
    }
    Xbar *= w;
    Ybar *= w;
    const double taub = Xbar * ex + Ybar * ey;
    const double exb = Xbar * tau, eyb = Ybar * tau, ezb = -taub * tau / ez;
    const double qxb = Xbar, qyb = Ybar, qzb = -taub / ez;
    double skb = 0.0;
    if (D.fresnel) {
        const double m = 1.0 - sk, m2 = m * m;
        skb = wbar * w1 * 5.0 * (1.0 - E.R0) * m2 * m2;
    }
    const double betab = exb * nxh + eyb * nyh + ezb * nzh;
    double nxb = beta * exb, nyb = beta * eyb, nzb = beta * ezb;
    skb += betab;
    double cb = -n * betab;
    const double kb = skb * 0.5 / fmax(sk, 1e-300);
    cb += 2.0 * n * n * c * kb;
    nxb += cb * dx;
    nyb += cb * dy;
    nzb += cb * dz;
    const double ndot = nxb * nxh + nyb * nyh + nzb * nzh;
    const double hxb = -(nxb - ndot * nxh) * inv_m, hyb = -(nyb - ndot * nyh) * inv_m;
    double g0;
    if (point) {
        const double tb = qxb * dx + qyb * dy + qzb * dz + hxb * (S.hxx * dx + S.hxy * dy) +
                          hyb * (S.hxy * dx + S.hyy * dy);
        // on the mesh f(t) = T(q(t)) - q_z(t), whose slope is the triangle's
        const double fp = MESH ? M.A * E.sxu * D.mesh_u * dx + M.B * E.syv * D.mesh_v * dy - dz
                               : S.hx * dx + S.hy * dy - dz;
        g0 = -tb / fp;
    } else {
        g0 = qzb;
    }
    const double gx = hxb * E.sxu, gy = hyb * E.syv;
    if constexpr (MESH) {
        // the hit follows the triangle, whose corner heights carry the hit's barycentric weights l_c:
        // dP_ab gets g0 (X0_a Nv0_b + X1_a Nv1_b) (as in trace_adjoint); the normal's terms are the B-spline's
        double X0[P + 1], X1[P + 1];
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            if (M.upper) {
                X0[a] = (1.0 - M.b) * M.Nu1[a];
                X1[a] = (M.a + M.b - 1.0) * M.Nu1[a] + (1.0 - M.a) * M.Nu0[a];
            } else {
                X0[a] = (1.0 - M.a - M.b) * M.Nu0[a] + M.a * M.Nu1[a];
                X1[a] = M.b * M.Nu0[a];
            }
        }
#pragma unroll
        for (int a = 0; a <= P; ++a)
#pragma unroll
            for (int b = 0; b <= Q; ++b)
                g[a * (Q + 1) + b] = g0 * (X0[a] * M.Nv0[b] + X1[a] * M.Nv1[b]) + S.Nu[a] * gy * S.dNv[b] +
                                     gx * S.dNu[a] * S.Nv[b];
    } else {
#pragma unroll
        for (int a = 0; a <= P; ++a)
#pragma unroll
            for (int b = 0; b <= Q; ++b)
                g[a * (Q + 1) + b] = S.Nu[a] * (g0 * S.Nv[b] + gy * S.dNv[b]) + gx * S.dNu[a] * S.Nv[b];
    }
    cku = S.ku;
    ckv = S.kv;
    if constexpr (TWO) {
        // ---- back through the exit root into the ray inside the glass, q = o + t d with f(t; o, d) = 0 (as in
        // trace_adjoint): the exit normal's dependence on q, then o and d
        const double qbx = qxb + hxb * S.hxx + hyb * S.hxy, qby = qyb + hxb * S.hxy + hyb * S.hyy;
        const double obx = qbx + g0 * S.hx, oby = qby + g0 * S.hy, obz = qzb - g0;
        const double dbx = n * exb + cb * nxh + t * obx;
        const double dby = n * eyb + cb * nyh + t * oby;
        const double dbz = n * ezb + cb * nzh + t * obz;
        // ---- entry refraction d = eta d0 + beta_i m, beta_i = sqrt(k_i) - eta c_i, c_i = d0 . m; w1 = w0 (1 -
        // Schlick(c_i)) and w = w1 T
        const double eta = 1.0 / n;
        double cib = (dbx * mx + dby * my + dbz * mz) * (eta * eta * ci / ski - eta);
        if (D.fresnel) {
            const double mm = 1.0 - ci, mm2 = mm * mm;
            cib += wbar * T * E.w0 * 5.0 * (1.0 - E.R0) * mm2 * mm2;
        }
        const double nbx = betai * dbx + cib * d0x, nby = betai * dby + cib * d0y, nbz = betai * dbz + cib * d0z;
        const double nd = nbx * mx + nby * my + nbz * mz;
        const double gxb_i = -(nbx - nd * mx) * inv_i, gyb_i = -(nby - nd * my) * inv_i;
        // ---- a point-source ray's entry hit moves along s + t_i d0 with g(s + t_i d0) = s_z + t_i d0_z; a
        // collimated ray meets the face at fixed (x, y), so only its height moves
        const double pbx = obx + gxb_i * Si.hxx + gyb_i * Si.hxy, pby = oby + gxb_i * Si.hxy + gyb_i * Si.hyy;
        const double tbi = pbx * d0x + pby * d0y + obz * d0z;
        const double c0 = TWOC ? obz : -tbi / (Si.hx * d0x + Si.hy * d0y - d0z);
        const double gxi = gxb_i * E.sxu, gyi = gyb_i * E.syv;
#pragma unroll
        for (int a = 0; a <= P; ++a)
#pragma unroll
            for (int b = 0; b <= Q; ++b)
                gin[a * (Q + 1) + b] = Si.Nu[a] * (c0 * Si.Nv[b] + gyi * Si.dNv[b]) + gxi * Si.dNu[a] * Si.Nv[b];
        *cku_in = Si.ku;
        *ckv_in = Si.kv;
    }
    return true;
}

// The double-precision re-trace of the queued rays.  A workgroup takes 64 consecutive queue segments (one per
// wave of a logical block, ~2 rays each), forms the prefix sums of their counts in LDS and gives its threads the
// rays densely, one per thread.  Their contributions are summed in an LDS copy of the control net of the
// round's design (the design of its first ray; rays of another design, at a design boundary, add to the
// device accumulator directly), which is then added to the device accumulator once: one atomic per touched
// control point and round instead of one per ray.  Both sums are in the design's fixed-point unit, so the result
// does not depend on which kernel adds them or in which order.
// MODE (F64_FLAT, F64_TWO, F64_TWO_COLL, F64_MESH): the instance for the segments of one kind of queued rays
// (seg0 on).
template <int P, int Q, int NU, int MODE>
__global__ __launch_bounds__(WG) void k_adjoint_fp64(TraceArgs A, const DesignDev64* d64, int shape, int64_t seg0,
                                                     int64_t nseg) {
    constexpr int SPW = 64;  // segments per workgroup and round
    __shared__ int s_off[SPW + 1];
    __shared__ int s_design;
    extern __shared__ unsigned long long sG[];  // A.lds_cp entries
    const int per_wave = queue_cap(shape) / 4;
    A.queue += seg0 * per_wave;
    A.queue_tin += seg0 * per_wave;
    A.qcount += seg0;
    for (int64_t s0 = (int64_t)blockIdx.x * SPW; s0 < nseg; s0 += (int64_t)gridDim.x * SPW) {
        if (threadIdx.x < SPW) {  // inclusive scan of the counts over wave 0
            int c = s0 + threadIdx.x < nseg ? A.qcount[s0 + threadIdx.x] : 0;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(c, o);
                if ((int)threadIdx.x >= o) c += u;
            }
            s_off[threadIdx.x + 1] = c;
            if (threadIdx.x == 0) s_off[0] = 0;
        }
        __syncthreads();
        const int total = s_off[SPW];
        if (total == 0) {
            __syncthreads();  // s_off is rewritten by the next round
            continue;
        }
        if (threadIdx.x == 0) {
            int k = 0;  // the segment of the round's first ray
            while (s_off[k + 1] == 0) ++k;
            s_design = A.queue[(s0 + k) * per_wave].design;
        }
        __syncthreads();
        const int dmain = s_design;
        const DesignDev Dm = load_uniform(A.designs, dmain);
        for (int i = threadIdx.x; i < Dm.ncp; i += WG) sG[i] = 0ull;
        __syncthreads();
        for (int i = threadIdx.x; i < total; i += WG) {
            int lo = 0, hi = SPW - 1;  // the segment of ray i: the last k with s_off[k] <= i
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= i) lo = mid; else hi = mid - 1;
            }
            const int64_t qi = (s0 + lo) * per_wave + (i - s_off[lo]);
            const QEntry q = A.queue[qi];
            const int qd = q.design;
            const DesignDev D = A.designs[qd];
            const DesignDev64 E = d64[qd];
            double g[(P + 1) * (Q + 1)], gin[(P + 1) * (Q + 1)];
            int cku = 0, ckv = 0, cku_in = -1, ckv_in = -1;
            if (!trace_adjoint_f64<P, Q, NU, MODE>(D, E, A.Pz, A.dLdI, q.id, q.t, cku, ckv, g,
                                                   MODE == F64_TWO ? A.queue_tin[qi] : 0.0f, &cku_in, &ckv_in, gin))
                continue;
            const double inv_unit = ldexp(1.0, -fixed_point_exponent(A.gmax[qd], D.w0));
            unsigned long long* acc = qd == dmain ? sG : A.gacc + D.cp_off;
#pragma unroll
            for (int a = 0; a <= P; ++a)
#pragma unroll
                for (int b = 0; b <= Q; ++b) {
                    const double v = g[a * (Q + 1) + b];
                    if (v != 0.0)
                        atomicAdd(&acc[(int64_t)(cku + a) * D.n_v + ckv + b],
                                  (unsigned long long)__double2ll_rn(v * inv_unit));
                }
            if (cku_in >= 0) {  // the entry net follows the exit net in the accumulator too
                unsigned long long* acc_in = acc + D.n_u * D.n_v;
#pragma unroll
                for (int a = 0; a <= P; ++a)
#pragma unroll
                    for (int b = 0; b <= Q; ++b) {
                        const double v = gin[a * (Q + 1) + b];
                        if (v != 0.0)
                            atomicAdd(&acc_in[(int64_t)(cku_in + a) * D.n_v + ckv_in + b],
                                      (unsigned long long)__double2ll_rn(v * inv_unit));
                    }
            }
        }
        __syncthreads();
        unsigned long long* gacc = A.gacc + Dm.cp_off;
        for (int i = threadIdx.x; i < Dm.ncp; i += WG) {
            const unsigned long long v = sG[i];
            if (v != 0ull) atomicAdd(&gacc[i], v);
        }
        __syncthreads();  // s_off and sG are rewritten by the next round
    }
}

// ------------------------------------------------------------------------------------------------
// Block decoding
// ------------------------------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs of the chip; give each XCD a contiguous range of
// logical blocks so that its L2 sees neighbouring rays (same control points, same pixels).
__device__ __forceinline__ int64_t xcd_remap(int64_t pb, int64_t nblocks) {
    constexpr int NX = 8;
    int64_t per = nblocks / NX, rem = nblocks % NX;
    int64_t x = pb % NX, slot = pb / NX;
    return x * per + min(x, rem) + slot;
}

__device__ __forceinline__ int find_design(const BlockMap* bm, int n, int64_t b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (load_uniform(bm, mid).first <= b) lo = mid; else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Stage design d in LDS: the knot tables, and P^z relative to a reference height zref inside the lens's
// height range (single-precision sums of B-spline terms then cancel far less).  With `bracket` (sources
// whose rays need the root search) the bounds of sec. 2.2.2 come from launch_bounds and zref is the middle of
// the convex-hull box; otherwise (collimated rays meet the surface at a known (x, y)) zref is the height of
// the middle control point and no bounds are used.  Every thread calls it; it ends with a barrier.
__device__ BoundsDev stage_design(const TraceArgs& A, const DesignDev& D, int d, float* sP, float* sK, int p, int q,
                                  bool bracket) {
    const float* P = A.Pz + D.cp_off;
    const int ncp = D.n_u * D.n_v;  // exit net; a freeform entry net follows it, relative to zref_in
    const int nku = D.nsu * kt_stride(p), nkv = D.nsv * kt_stride(q);
    const float* ku = A.knots + D.kt_u;
    const float* kv = A.knots + D.kt_v;
    BoundsDev B;
    if (bracket) {
        B = load_uniform(A.bounds, d);
        if (A.lds_sb) {  // span bounds follow the knot tables
            const float* src = reinterpret_cast<const float*>(A.span_bounds + D.sb_off);
            float* sS = sK + A.lds_kt;
            for (int i = threadIdx.x; i < 4 * D.nsu * D.nsv; i += WG) sS[i] = src[i];
        }
    } else {
        B.zmin = B.zmax = B.gx = B.gy = 0.0f;
        const float zc = load_uniform(P, (D.n_u / 2) * D.n_v + D.n_v / 2);
        B.zref = isfinite(zc) ? zc : D.zmin_allowed;
    }
    for (int i = threadIdx.x; i < ncp; i += WG) sP[i] = P[i] - B.zref;
    if (D.entry_ff)
        for (int i = threadIdx.x; i < ncp; i += WG) sP[ncp + i] = P[ncp + i] - B.zref_in;
    for (int i = threadIdx.x; i < nku; i += WG) sK[i] = ku[i];
    for (int i = threadIdx.x; i < nkv; i += WG) sK[nku + i] = kv[i];
    __syncthreads();
    return B;
}

// ------------------------------------------------------------------------------------------------
// Forward kernel
// ------------------------------------------------------------------------------------------------
// Add a pixel contribution v >= 0 in fixed point, either to the workgroup's LDS tile or, when the block's
// footprint does not fit the tile, directly to the device image.  The image unit is 1 / scale (2^-26 w0,
// 64-bit); the tile unit is 2^TSH image units (32-bit), chosen so that a workgroup's sum for one pixel stays
// below 2^31.  Integer LDS atomics are far cheaper than float ones on gfx950 (and 32-bit ones cheaper than
// 64-bit ones when lanes collide), and integer sums do not depend on the order of the additions, so the
// irradiance is reproducible bit for bit.
template <int TSH>
__device__ __forceinline__ void splat_add(bool to_tile, uint32_t* tile, int tile_ld, int ilo, int jlo, float scale,
                                          unsigned long long* img, int ny, int i, int j, float v) {
    if (to_tile) {
        const uint32_t q = (uint32_t)__float2int_rn(v * (scale * (1.0f / (float)(1 << TSH))));
        __hip_atomic_fetch_add(&tile[(i - ilo) * tile_ld + (j - jlo)], q, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        const unsigned long long q = (unsigned long long)(long long)__float2int_rn(v * scale);
        __hip_atomic_fetch_add(&img[(int64_t)i * ny + j], q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int P, int Q, int NU, int SHAPE, int KIND>
__device__ __forceinline__ void forward_body(TraceArgs A) {
    constexpr int MU = shape_mu(SHAPE), MV = shape_mv(SHAPE), RPT = MU * MV;
    constexpr int BU = 16 * MU, BV = 16 * MV;
    constexpr int H = (NU - 1) / 2;
    // tile unit 2^TSH image units: 256 RPT rays of at most 2^26 units each then sum to at most 2^30 per pixel
    constexpr int TSH = 4 + (RPT >= 2) + (RPT >= 4) + (RPT >= 8) + (RPT >= 16);
    // per-thread accumulation window of WN x WN pixels: the filter windows of a thread's neighbouring rays
    // usually fall inside one such window, so most rays cost no atomic at all
    // Per-thread accumulation pays where a thread's neighbouring samples land within a pixel of each other
    // (collimated bundles); the searched rays of point sources fan out, and a wave whose lanes leave their
    // windows takes the direct path anyway: they add each ray's window to the tile directly.
    constexpr bool ACCUM = NU <= 5 && (KIND & 5) == 0;
    constexpr int SLACK = 1;  // a thread's rays whose filter windows start up to SLACK pixels apart share one window
    constexpr int WN = NU + SLACK;
    extern __shared__ float smem[];
    float* sP = smem;
    float* sK = sP + A.lds_cp;
    float* sS = sK + A.lds_kt;  // span bounds (exit root searches, when they fit)
    uint32_t* tile = reinterpret_cast<uint32_t*>(sS + A.lds_sb);
    const float* sSb = (KIND & 5) != 0 && A.lds_sb ? sS : nullptr;
    __shared__ int s_box[4][4];
    __shared__ float s_red[4][11];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int cur = -1;
    BoundsDev B;
    for (int64_t pb = blockIdx.x; pb < A.n_blocks; pb += gridDim.x) {
        const int64_t b = xcd_remap(pb, A.n_blocks);
        const int d = find_design(A.bmap, A.n_designs, b);
        const DesignDev D = load_uniform(A.designs, d);
        if (d != cur) {
            __syncthreads();
            B = stage_design(A, D, d, sP, sK, P, Q, (KIND & 5) != 0);
            cur = d;
        }
        const float* sKu = sK;
        const float* sKv = sK + D.nsu * kt_stride(P);
        const BlockMap bm = load_uniform(A.bmap, d);
        int64_t local = b - bm.first;
        int e = (int)(local / bm.per_emitter);
        int rb = (int)(local - (int64_t)e * bm.per_emitter);
        int bu = rb / bm.nbv, bv = rb - (rb / bm.nbv) * bm.nbv;
        int64_t ebase = (int64_t)e * D.grid_u * D.grid_v;
        const int ku0 = bu * BU + (wave >> 1) * 8 * MU + (lane >> 3) * MU;
        const int kv0 = bv * BV + (wave & 1) * 8 * MV + (lane & 7) * MV;

        float X[RPT], Y[RPT], W[RPT];
        uint32_t c_hit = 0, c_miss = 0, c_side = 0, c_tir = 0, c_off = 0, c_fail = 0, c_ref = 0, c_nm = 0,
                 c_tr = 0, c_it = 0;
        float flux = 0.0f;
        int imin = 1 << 30, imax = -1, jmin = 1 << 30, jmax = -1;
        float t_prev = -1.0f;  // the exit root of the thread's previous ray (its samples are adjacent)
        // ray (ku0 + r / MV, kv0 + r % MV) is id0 + off: its id and RNG counter from the first ray's by additions
        // of workgroup-uniform offsets
        const int64_t id0 = ebase + (int64_t)ku0 * D.grid_v + kv0;
        const uint64_t ctr0 = rng_counter(D.rng_state0, id0);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int ku = ku0 + r / MV, kv = kv0 + r % MV;
            W[r] = 0.0f;
            X[r] = 0.0f;
            Y[r] = 0.0f;
            if (ku < D.grid_u && kv < D.grid_v) {
                const int64_t off = (int64_t)(r / MV) * D.grid_v + r % MV;
                float* ts = nullptr;
                if constexpr (KIND == 1)
                    if (A.roots) ts = A.roots + D.root_off + id0 + off;
                FwdRay o = trace_forward<P, Q, KIND>(D, B, sP, sKu, sKv, sSb, e, ku, kv,
                                                     ctr0 + (uint64_t)off * SPLITMIX_GAMMA, ts, t_prev);
                if (o.t > 0.0f) t_prev = o.t;
                c_tr++;
                c_fail += o.failed;
                c_ref += o.refined;
                c_nm += o.nonmono;
                c_it += o.iters;
                switch (o.status) {
                    case ST_HIT: c_hit++; break;
                    case ST_MISS_ENTRY: c_miss++; break;
                    case ST_SIDE_WALL: c_side++; break;
                    case ST_TIR: c_tir++; break;
                    default: c_off++; break;
                }
                if (o.status == ST_HIT) {
                    X[r] = o.X;
                    Y[r] = o.Y;
                    W[r] = o.w;
                    flux += o.w;
                    int i0 = min(max((int)floorf((o.X + D.Rx) * D.inv_wx), 0), D.nx - 1);
                    int j0 = min(max((int)floorf((o.Y + D.Ry) * D.inv_wy), 0), D.ny - 1);
                    imin = min(imin, i0);
                    imax = max(imax, i0);
                    jmin = min(jmin, j0);
                    jmax = max(jmax, j0);
                }
            }
        }
        // ---- statistics: reduced over the workgroup, then one atomic per counter into one of NSLOT slots
        if (A.slots) {
            // the ten counters (exact in float: a wave traces at most 1024 rays of at most 8192 search steps
            // each) and the flux, summed over the wave by one reduce-scatter
            float v[16] = {(float)c_tr, (float)c_hit, (float)c_miss, (float)c_side, (float)c_tir, (float)c_off,
                           (float)c_fail, (float)c_ref, (float)c_nm, (float)c_it, flux, 0.0f, 0.0f, 0.0f, 0.0f,
                           0.0f};
            const float sum = wave_reduce_scatter<16>(v, lane);
            if ((lane & 3) == 0 && (lane >> 2) < 11) s_red[wave][lane >> 2] = sum;
            __syncthreads();
            ffrt_stats* slot = A.slots + (size_t)d * NSLOT + (blockIdx.x % NSLOT);
            if (threadIdx.x < 10) {
                uint32_t tot = (uint32_t)s_red[0][threadIdx.x] + (uint32_t)s_red[1][threadIdx.x] +
                               (uint32_t)s_red[2][threadIdx.x] + (uint32_t)s_red[3][threadIdx.x];
                // fields n_traced .. n_search_steps follow flux_on_screen in ffrt_stats
                if (tot) atomicAdd(reinterpret_cast<uint32_t*>(slot) + 1 + threadIdx.x, tot);
            } else if (threadIdx.x == 10) {
                float tot = s_red[0][10] + s_red[1][10] + s_red[2][10] + s_red[3][10];
                if (tot != 0.0f) atomicAdd(&slot->flux_on_screen, tot);
            }
            __syncthreads();
        }
        // ---- footprint of the block: the landing pixels widened by the filter half-width, and by one more
        // row and column for the per-thread windows below.  The tile is not clipped to the image, so every
        // window of a thread with a hit lies inside it and needs no per-pixel test; pixels outside the
        // image only ever receive zero weights, and the flush skips them.  A footprint larger than the tile
        // is splatted in slabs of whole rows, one pass each (every pass clears the tile, adds the block's
        // contributions to the slab's rows and flushes them), so that the device image still receives one
        // atomic per touched pixel and pass instead of one per ray and pixel.
        unsigned long long* img = A.img64 + D.img_off;
        bool use_tile = false;
        int ilo = 0, jlo = 0, tw = 0, rows = 0, slab = 0;
        if (A.use_tile) {
            int a0 = wave_min(imin), a1 = wave_max(imax), b0 = wave_min(jmin), b1 = wave_max(jmax);
            if (lane == 0) {
                s_box[wave][0] = a0;
                s_box[wave][1] = a1;
                s_box[wave][2] = b0;
                s_box[wave][3] = b1;
            }
            __syncthreads();
            // workgroup-uniform: kept in scalar registers, with everything derived from them below
            a0 = __builtin_amdgcn_readfirstlane(min(min(s_box[0][0], s_box[1][0]), min(s_box[2][0], s_box[3][0])));
            a1 = __builtin_amdgcn_readfirstlane(max(max(s_box[0][1], s_box[1][1]), max(s_box[2][1], s_box[3][1])));
            b0 = __builtin_amdgcn_readfirstlane(min(min(s_box[0][2], s_box[1][2]), min(s_box[2][2], s_box[3][2])));
            b1 = __builtin_amdgcn_readfirstlane(max(max(s_box[0][3], s_box[1][3]), max(s_box[2][3], s_box[3][3])));
            __syncthreads();
            if (a1 < 0) continue;  // no ray of the block reached the screen
            constexpr int PAD = ACCUM ? 1 : 0;
            ilo = a0 - H;
            jlo = b0 - H;
            tw = b1 + H + PAD - jlo + 1;
            rows = a1 + H + PAD - ilo + 1;
            // slabs for the searched rays (point sources, freeform entry faces), whose blocks may fan out over
            // the screen; a collimated block's footprint stays compact, and its kernels keep a single pass (a
            // footprint beyond the tile then goes to the device image directly)
            constexpr bool SLABS = (KIND & 5) != 0;
            use_tile = SLABS ? tw <= TILE_CAP : rows * tw <= TILE_CAP;
            if (use_tile) slab = min(rows, TILE_CAP / tw);
        }
        const int npass = (KIND & 5) != 0 && use_tile ? (rows + slab - 1) / slab : 1;
        for (int pass = 0; pass < npass; ++pass) {
            // the slab: image rows [r0, r0 + nrow) of the footprint, in the tile at (i - r0) tw + (j - jlo)
            const int r0 = ilo + pass * slab;
            const int nrow = use_tile ? min(slab, rows - pass * slab) : 0;
            const int area = nrow * tw;
            uint32_t* mytile = tile;
            if (use_tile) {
                for (int i = threadIdx.x; i < area; i += WG) tile[i] = 0u;
                __syncthreads();
            }
            auto in_slab = [&](int i) { return !use_tile || (i >= r0 && i < r0 + nrow); };
            // ---- splat.  Every pass evaluates the filter weights of the thread's rays again (cheap beside the
            // trace) and keeps the contributions to the slab's rows; registers then carry only the landings
            // from one pass to the next.  The empty asm makes each landing look pass-dependent, so that the
            // compiler does not hoist the weights of every ray out of the pass loop.
            if constexpr (ACCUM) {
                // Per-thread accumulation window anchored at the thread's lowest landing pixel (imin, jmin): rays
                // whose filter window starts at most SLACK pixels further along each axis are summed in registers,
                // the others are added directly.  With the tile the sums are kept in tile units.  A wave takes
                // the direct path when any of its lanes needs it, so the slack covers the landing spread of a
                // thread's neighbouring samples on fanned-out footprints.
                const int ai = imin - H, aj = jmin - H;
                const float wsc = use_tile ? D.fx_scale * (1.0f / (float)(1 << TSH)) : 1.0f;
                float acc[WN * WN];
#pragma unroll
                for (int k = 0; k < WN * WN; ++k) acc[k] = 0.0f;
                int used_r = 0, used_c = 0;  // the largest window offsets of the thread's rays
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    if (W[r] == 0.0f) continue;
                    float xr = X[r], yr = Y[r];
                    if (npass > 1) asm volatile("" : "+v"(xr), "+v"(yr));
                    float Fx[NU], Fy[NU], Sx, Sy;
                    const int di = filter_axis<NU, false, false>(xr, D.Rx, D.wx, D.inv_wx, D.nx, D.alpha, D.edge_x,
                                                                 Fx, nullptr, D.box, &Sx) - H - ai;
                    const int dj = filter_axis<NU, false, false>(yr, D.Ry, D.wy, D.inv_wy, D.ny, D.alpha, D.edge_y,
                                                                 Fy, nullptr, D.box, &Sy) - H - aj;
                    const float Wn = W[r] * rcpf(Sx * Sy);
                    if (di > SLACK || dj > SLACK) {
#pragma unroll
                        for (int a = 0; a < NU; ++a) {
                            if (!in_slab(ai + di + a)) continue;
#pragma unroll
                            for (int bb = 0; bb < NU; ++bb) {
                                const float v = Wn * Fx[a] * Fy[bb];
                                if (v != 0.0f)
                                    splat_add<TSH>(use_tile, mytile, tw, r0, jlo, D.fx_scale, img, D.ny, ai + di + a,
                                                   aj + dj + bb, v);
                            }
                        }
                        continue;
                    }
                    used_r = max(used_r, di);
                    used_c = max(used_c, dj);
                    // add the NU x NU window at offset (di, dj) in [0, SLACK]^2 without indexing registers
                    // dynamically
                    const float wr = Wn * wsc;
                    float fx[WN], fy[WN];
#pragma unroll
                    for (int k = 0; k < WN; ++k) {
                        float xa = 0.0f, ya = 0.0f;
#pragma unroll
                        for (int o = 0; o <= SLACK; ++o) {
                            if (k - o < 0 || k - o >= NU) continue;
                            xa = di == o ? Fx[k - o] : xa;
                            ya = dj == o ? Fy[k - o] : ya;
                        }
                        fx[k] = wr * xa;
                        fy[k] = ya;
                    }
#pragma unroll
                    for (int k = 0; k < WN * WN; ++k) acc[k] += fx[k / WN] * fy[k % WN];
                }
                if (use_tile) {
                    if (imax >= 0) {  // the window lies inside the footprint: one row address per window row
                        auto add = [](uint32_t* p, float v) {
                            __hip_atomic_fetch_add(p, (uint32_t)__float2int_rn(v), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                        };
#pragma unroll
                        for (int a = 0; a < WN; ++a) {
                            if (a >= used_r + NU || !in_slab(ai + a)) continue;
                            uint32_t* row = mytile + (ai + a - r0) * tw + (aj - jlo);
#pragma unroll
                            for (int bb = 0; bb < WN; ++bb)
                                if (bb < used_c + NU) add(row + bb, acc[a * WN + bb]);
                        }
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < WN * WN; ++k)
                        if (acc[k] != 0.0f)
                            splat_add<TSH>(false, mytile, tw, r0, jlo, D.fx_scale, img, D.ny, ai + k / WN,
                                           aj + k % WN, acc[k]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    if (W[r] == 0.0f) continue;
                    float xr = X[r], yr = Y[r];
                    if (npass > 1) asm volatile("" : "+v"(xr), "+v"(yr));
                    float Fx[NU], Fy[NU], Sx, Sy;
                    const int i0 = filter_axis<NU, false, false>(xr, D.Rx, D.wx, D.inv_wx, D.nx, D.alpha, D.edge_x,
                                                                 Fx, nullptr, D.box, &Sx);
                    const int j0 = filter_axis<NU, false, false>(yr, D.Ry, D.wy, D.inv_wy, D.ny, D.alpha, D.edge_y,
                                                                 Fy, nullptr, D.box, &Sy);
                    const float Wn = W[r] * rcpf(Sx * Sy);
                    if (use_tile) {
                        // the tile holds every row and column of the window (pixels off the image get zero
                        // weights, which the flush skips): nine adds without a test, rows outside the slab aside.
                        // Tile offsets fit 24-bit products; the weights are >= 0, so adding one half and
                        // truncating rounds them to the nearest unit.
                        const float wr = Wn * (D.fx_scale * (1.0f / (float)(1 << TSH)));
                        const int base = __mul24(i0 - H - r0, tw) + (j0 - H - jlo);
#pragma unroll
                        for (int a = 0; a < NU; ++a) {
                            if (npass > 1 && !in_slab(i0 + a - H)) continue;
                            uint32_t* row = mytile + base + a * tw;
                            const float wa = wr * Fx[a];
#pragma unroll
                            for (int bb = 0; bb < NU; ++bb)
                                __hip_atomic_fetch_add(row + bb, __float2uint_rz(fmaf(wa, Fy[bb], 0.5f)),
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        continue;
                    }
#pragma unroll
                    for (int a = 0; a < NU; ++a) {
                        const int i = i0 + a - H;
                        if (i < 0 || i >= D.nx) continue;
#pragma unroll
                        for (int bb = 0; bb < NU; ++bb) {
                            const int j = j0 + bb - H;
                            if (j < 0 || j >= D.ny) continue;
                            splat_add<TSH>(false, mytile, tw, r0, jlo, D.fx_scale, img, D.ny, i, j,
                                           Wn * Fx[a] * Fy[bb]);
                        }
                    }
                }
            }
            if (use_tile) {
                __syncthreads();
                // element i = ti tw + tj of the slab: row and column follow from the previous element's
                // (WG = qs tw + rs), one division per pass instead of one per element
                const int qs = WG / tw, rs = WG - qs * tw;
                int ti = (int)threadIdx.x / tw, tj = (int)threadIdx.x - ti * tw;
                for (int i = threadIdx.x; i < area; i += WG) {
                    const uint32_t v = tile[i];
                    const int gi = r0 + ti, gj = jlo + tj;
                    if (v != 0u && gi >= 0 && gi < D.nx && gj >= 0 && gj < D.ny)
                        __hip_atomic_fetch_add(&img[(int64_t)gi * D.ny + gj], (unsigned long long)v << TSH,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ti += qs;
                    tj += rs;
                    if (tj >= tw) {
                        tj -= tw;
                        ++ti;
                    }
                }
                __syncthreads();
            }
        }
    }
}

template <int P, int Q, int NU, int SHAPE, int KIND>
__global__ __launch_bounds__(WG) void k_forward(TraceArgs A) {
    forward_body<P, Q, NU, SHAPE, KIND>(A);
}

// The same with at least three waves per SIMD, for the point-source forward at 8 rays per thread: uncapped it
// takes ~174 VGPRs (two waves); capped it fits 168 without a spill and runs faster than at 4 rays per thread
// (its first, cold-started Newton search is one ray in 8 instead of one in 4).
template <int P, int Q, int NU, int SHAPE, int KIND>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(3))) void k_forward_w3(TraceArgs A) {
    forward_body<P, Q, NU, SHAPE, KIND>(A);
}

// ------------------------------------------------------------------------------------------------
// Adjoint kernel
// ------------------------------------------------------------------------------------------------
// The adjoint sums its gradient contributions as signed 64-bit integers (fixed point): integer additions do
// not depend on their order, so dL/dP is reproducible bit for bit whatever order the lanes, waves and
// workgroups add in.  The unit is set per design from the size of a single ray's weighted cotangent,
// S = max |dL/dI| w0, as 2^(floor(log2 S) - 32) (fixed_point_exponent): a contribution of size S keeps 32
// bits below its leading bit, and a sum of up to 2^31 S fits (the gradient itself stays far below: on the
// stated workloads max |dL/dP| < 2^22 S).  Two's-complement sums wrap around, so only the final value has to
// fit.
__device__ __forceinline__ unsigned long long to_fixed(float v, float inv_unit) {
    return (unsigned long long)__float2ll_rn(v * inv_unit);
}

// Add a thread's control-point accumulator (span product (ku, kv)) to the LDS copy of the control net.
template <int P, int Q, int NV>
__device__ __forceinline__ void cp_flush_lane(unsigned long long* sG, int n_v, int ku, int kv, const float* acc,
                                              float inv_unit) {
#pragma unroll
    for (int a = 0; a <= P; ++a)
#pragma unroll
        for (int b = 0; b <= Q; ++b) {
            float v = acc[a * (Q + 1) + b];
            if (v != 0.0f) atomicAdd(&sG[(ku + a) * n_v + kv + b], to_fixed(v, inv_unit));
        }
}

// End of a workgroup's run of blocks of design d: add its LDS control-net gradient to the device
// accumulator (cleared again by the finishing kernel that reads it).
__device__ void adjoint_flush(const TraceArgs& A, int d, const unsigned long long* sG) {
    __syncthreads();
    const DesignDev D = load_uniform(A.designs, d);
    unsigned long long* acc = A.gacc + D.cp_off;
    for (int i = threadIdx.x; i < D.ncp; i += WG) {
        const unsigned long long v = sG[i];
        if (v != 0ull) atomicAdd(&acc[i], v);
    }
}

template <int P, int Q, int NU, int KIND>
__device__ __forceinline__ void adjoint_body(const TraceArgs& A, int shape) {
    constexpr int NT = (P + 1) * (Q + 1);
    constexpr int NV = NT <= 16 ? 16 : (NT <= 32 ? 32 : 64);
    constexpr int LOG_NV = NV == 16 ? 4 : (NV == 32 ? 5 : 6);
    extern __shared__ float smem[];
    float* sP = smem;
    float* sK = sP + A.lds_cp;
    float* sS = sK + A.lds_kt;  // span bounds (exit root searches, when they fit)
    unsigned long long* sG = reinterpret_cast<unsigned long long*>(sS + A.lds_sb);  // 64-bit fixed point
    const float* sSb = (KIND & 5) != 0 && A.lds_sb ? sS : nullptr;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int MU = shape_mu(shape), MV = shape_mv(shape), RPT = MU * MV;
    const int BU = 16 * MU, BV = 16 * MV;
    const int mv_shift = MV == 1 ? 0 : (MV == 2 ? 1 : 2);
    // per-wave count of the block's rays queued for the double-precision re-trace (KIND 0 and 1)
    __shared__ int s_qn[WG / 64];
    const int qcap_w = queue_cap(shape) / 4;
    if (lane == 0) s_qn[wave] = 0;
    int cur = -1;
    BoundsDev B;
    for (int64_t pb = blockIdx.x; pb < A.n_blocks; pb += gridDim.x) {
        const int64_t b = xcd_remap(pb, A.n_blocks);
        const int d = find_design(A.bmap, A.n_designs, b);
        const DesignDev D = load_uniform(A.designs, d);
        const BlockMap bm = load_uniform(A.bmap, d);
        int64_t local = b - bm.first;
        if (d != cur) {
            if (cur >= 0) adjoint_flush(A, cur, sG);
            __syncthreads();
            for (int i = threadIdx.x; i < D.ncp; i += WG) sG[i] = 0ull;
            B = stage_design(A, D, d, sP, sK, P, Q, (KIND & 5) != 0);
            cur = d;
        }
        const float* G = A.dLdI + D.img_off;
        const float* sKu = sK;
        const float* sKv = sK + D.nsu * kt_stride(P);
        int e = (int)(local / bm.per_emitter);
        int rb = (int)(local - (int64_t)e * bm.per_emitter);
        int bu = rb / bm.nbv, bv = rb - (rb / bm.nbv) * bm.nbv;
        int64_t ebase = (int64_t)e * D.grid_u * D.grid_v;
        const int ku0 = bu * BU + (wave >> 1) * 8 * MU + (lane >> 3) * MU;
        const int kv0 = bv * BV + (wave & 1) * 8 * MV + (lane & 7) * MV;
        // per-thread accumulator of the span product its rays hit; flushed when the span changes (a second one
        // for the entry net of a lens with a freeform entry face, whose LDS gradient follows the exit net's)
        constexpr bool ENTRY = (KIND & 4) != 0;
        float acc[NV], acc_in[ENTRY ? NV : 1];
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < (ENTRY ? NV : 1); ++i) acc_in[i] = 0.0f;
        int aku = -1, akv = -1, aku_in = -1, akv_in = -1;
        unsigned long long* sG_in = sG + D.n_u * D.n_v;
        const float inv_unit = ldexpf(1.0f, -fixed_point_exponent(load_uniform(A.gmax, d), D.w0));
        // ray r is id0 + off (a workgroup-uniform offset): its RNG counter follows by an addition.  The
        // point-source instance with stored roots computes both per ray instead (its registers are full).
        const uint64_t ctr0 = rng_counter(D.rng_state0, ebase + (int64_t)ku0 * D.grid_v + kv0);
        for (int r = 0; r < RPT; ++r) {
            const int ku = ku0 + (r >> mv_shift), kv = kv0 + (r & (MV - 1));
            if (ku >= D.grid_u || kv >= D.grid_v) continue;
            float g[NT], gin[ENTRY ? NT : 1];
            int cku = -1, ckv = -1, cku_in = -1, ckv_in = -1;
            uint64_t ctr;
            const float* tl = nullptr;
            if constexpr (KIND == 1) {
                const int64_t id = ebase + (int64_t)ku * D.grid_v + kv;
                ctr = rng_counter(D.rng_state0, id);
                if (A.roots) tl = A.roots + D.root_off + id;
            } else {
                ctr = ctr0 + (uint64_t)((int64_t)(r >> mv_shift) * D.grid_v + (r & (MV - 1))) * SPLITMIX_GAMMA;
            }
            // queued for the double-precision re-trace while the wave's segment of the queue has room
            auto enqueue = [&](float tq, float tq_in) {
                if (!A.queue) return false;
                const int slot = atomicAdd(&s_qn[wave], 1);
                if (slot >= qcap_w) return false;
                // the ray id again from the block's base and the ray's place (cheaper than keeping it live)
                const int kq = ku0 + (r >> mv_shift), lq = kv0 + (r & (MV - 1));
                const int64_t qi = ((A.qbase + b) * 4 + wave) * qcap_w + slot;
                A.queue[qi] = QEntry{d, tq, ebase + (int64_t)kq * D.grid_v + lq};
                if constexpr (KIND == 5) A.queue_tin[qi] = tq_in;
                return true;
            };
            if (!trace_adjoint<P, Q, NU, KIND>(D, B, sP, sKu, sKv, sSb, G, e, ku, kv, ctr, cku, ckv, g, cku_in, ckv_in,
                                               gin, tl, enqueue))
                continue;
            if (aku >= 0 && (cku != aku || ckv != akv)) {
                cp_flush_lane<P, Q, NV>(sG, D.n_v, aku, akv, acc, inv_unit);
#pragma unroll
                for (int i = 0; i < NV; ++i) acc[i] = 0.0f;
            }
            aku = cku;
            akv = ckv;
#pragma unroll
            for (int i = 0; i < NT; ++i) acc[i] += g[i];
            if constexpr (ENTRY) {
                if (aku_in >= 0 && (cku_in != aku_in || ckv_in != akv_in)) {
                    cp_flush_lane<P, Q, NV>(sG_in, D.n_v, aku_in, akv_in, acc_in, inv_unit);
#pragma unroll
                    for (int i = 0; i < NV; ++i) acc_in[i] = 0.0f;
                }
                aku_in = cku_in;
                akv_in = ckv_in;
#pragma unroll
                for (int i = 0; i < NT; ++i) acc_in[i] += gin[i];
            }
        }
        if constexpr (ENTRY) {
            if (aku_in >= 0) cp_flush_lane<P, Q, NV>(sG_in, D.n_v, aku_in, akv_in, acc_in, inv_unit);
        }
        // end of the block: one round per distinct span product held in the wave, in which the lanes of the
        // leader's span product sum their accumulators with a butterfly (one LDS atomic per control point)
        bool pend = aku >= 0;
        if (A.butterfly) {
            const int key = (aku << 16) | (akv & 0xFFFF);
            for (uint64_t m = __ballot(pend); m != 0; m = __ballot(pend)) {
                const int lkey = __builtin_amdgcn_readlane(key, __ffsll((unsigned long long)m) - 1);
                const bool take = pend && key == lkey;
                float v[NV];
#pragma unroll
                for (int i = 0; i < NV; ++i) v[i] = take ? acc[i] : 0.0f;
                const float sum = wave_reduce_scatter<NV>(v, lane);
                const int idx = lane >> (6 - LOG_NV);
                if ((lane & ((1 << (6 - LOG_NV)) - 1)) == 0 && idx < NT && sum != 0.0f) {
                    const int a = idx / (Q + 1), bb = idx - (idx / (Q + 1)) * (Q + 1);
                    atomicAdd(&sG[((lkey >> 16) + a) * D.n_v + (lkey & 0xFFFF) + bb], to_fixed(sum, inv_unit));
                }
                pend = pend && !take;
            }
        } else if (pend) {
            cp_flush_lane<P, Q, NV>(sG, D.n_v, aku, akv, acc, inv_unit);
        }
        {
            // the wave's queued rays of this block (its lanes' LDS atomics completed in order before this read)
            if (A.queue && lane == 0) {
                A.qcount[(A.qbase + b) * 4 + wave] = min(s_qn[wave], qcap_w);
                s_qn[wave] = 0;
            }
        }
    }
    if (cur >= 0) adjoint_flush(A, cur, sG);
}

template <int P, int Q, int NU, int KIND>
__global__ __launch_bounds__(WG) void k_adjoint(TraceArgs A, int shape) {
    adjoint_body<P, Q, NU, KIND>(A, shape);
}

// The same with at least three waves per SIMD, for the instances where that costs (almost) no spill: the
// bicubic, nu = 3 point-source adjoint would otherwise take ~190 VGPRs (two waves) and stall on latency.
template <int P, int Q, int NU, int KIND>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(3))) void k_adjoint_w3(TraceArgs A, int shape) {
    adjoint_body<P, Q, NU, KIND>(A, shape);
}

// ------------------------------------------------------------------------------------------------
// Individual rays (inspection)
// ------------------------------------------------------------------------------------------------
template <int P, int Q>
__global__ __launch_bounds__(WG) void k_trace_rays(TraceArgs A, int design, const int64_t* ids, int64_t n,
                                                   float* out8) {
    extern __shared__ float smem[];
    float* sP = smem;
    float* sK = sP + A.lds_cp;
    float* sS = sK + A.lds_kt;
    const DesignDev D = load_uniform(A.designs, design);
    const BoundsDev B = stage_design(A, D, design, sP, sK, P, Q, D.kind != 0 || D.entry_ff);
    int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    int64_t id = ids[i];
    int64_t per = (int64_t)D.grid_u * D.grid_v;
    int e = (int)(id / per);
    int64_t rr = id - (int64_t)e * per;
    int ku = (int)(rr / D.grid_v), kv = (int)(rr - (rr / D.grid_v) * D.grid_v);
    const float* sKv = sK + D.nsu * kt_stride(P);
    const float* sSb = A.lds_sb && (D.kind != 0 || D.entry_ff) ? sS : nullptr;
    const uint64_t c = rng_counter(D.rng_state0, id);
    FwdRay o;
    if (D.entry_ff) o = D.kind == 0 ? trace_forward<P, Q, 4>(D, B, sP, sK, sKv, sSb, e, ku, kv, c)
                                    : trace_forward<P, Q, 5>(D, B, sP, sK, sKv, sSb, e, ku, kv, c);
    else if (D.mesh_u) o = D.kind == 0 ? trace_forward<P, Q, 2>(D, B, sP, sK, sKv, nullptr, e, ku, kv, c)
                                       : trace_forward<P, Q, 3>(D, B, sP, sK, sKv, nullptr, e, ku, kv, c);
    else o = D.kind == 0 ? trace_forward<P, Q, 0>(D, B, sP, sK, sKv, nullptr, e, ku, kv, c)
                         : trace_forward<P, Q, 1>(D, B, sP, sK, sKv, sSb, e, ku, kv, c);
    float* dst = out8 + 8 * i;
    dst[0] = (float)o.status;
    dst[1] = o.X;
    dst[2] = o.Y;
    dst[3] = o.status == ST_HIT ? o.w : 0.0f;
    dst[4] = o.u;
    dst[5] = o.v;
    dst[6] = o.t;
    dst[7] = (float)o.iters;
}

// ------------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------------
inline size_t trace_lds_bytes(const TraceArgs& A, int extra_floats) {
    return sizeof(float) * (size_t)(A.lds_cp + A.lds_kt + A.lds_sb + extra_floats);
}

template <int P, int Q, int NU>
struct KernelsFor {
    template <int SHAPE>
    static hipError_t fwd_shape(const TraceArgs& A, int grid, hipStream_t s) {
        size_t lds = trace_lds_bytes(A, A.use_tile ? TILE_CAP : 0);
        switch (A.kind_group) {
            case 0: hipLaunchKernelGGL((k_forward<P, Q, NU, SHAPE, 0>), dim3(grid), dim3(WG), lds, s, A); break;
            case 1:
                if constexpr (SHAPE == 3 && P == 3 && Q == 3 && NU == 3)
                    hipLaunchKernelGGL((k_forward_w3<P, Q, NU, SHAPE, 1>), dim3(grid), dim3(WG), lds, s, A);
                else
                    hipLaunchKernelGGL((k_forward<P, Q, NU, SHAPE, 1>), dim3(grid), dim3(WG), lds, s, A);
                break;
            case 2: hipLaunchKernelGGL((k_forward<P, Q, NU, SHAPE, 2>), dim3(grid), dim3(WG), lds, s, A); break;
            case 3: hipLaunchKernelGGL((k_forward<P, Q, NU, SHAPE, 3>), dim3(grid), dim3(WG), lds, s, A); break;
            case 4: hipLaunchKernelGGL((k_forward<P, Q, NU, SHAPE, 4>), dim3(grid), dim3(WG), lds, s, A); break;
            case 5: hipLaunchKernelGGL((k_forward<P, Q, NU, SHAPE, 5>), dim3(grid), dim3(WG), lds, s, A); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    static hipError_t forward(const TraceArgs& A, int shape, int grid, hipStream_t s) {
        switch (shape) {
            case 0: return fwd_shape<0>(A, grid, s);
            case 1: return fwd_shape<1>(A, grid, s);
            case 2: return fwd_shape<2>(A, grid, s);
            case 3: return fwd_shape<3>(A, grid, s);
            default: return hipErrorInvalidValue;
        }
    }
    static hipError_t adjoint(const TraceArgs& A, int shape, int grid, hipStream_t s) {
        size_t lds = trace_lds_bytes(A, 2 * A.lds_cp);  // the gradient net in 64-bit fixed point
        constexpr bool cap = P == 3 && Q == 3 && NU == 3;
        switch (A.kind_group) {
            case 0: hipLaunchKernelGGL((k_adjoint<P, Q, NU, 0>), dim3(grid), dim3(WG), lds, s, A, shape); break;
            case 1:
                if constexpr (cap)
                    hipLaunchKernelGGL((k_adjoint_w3<P, Q, NU, 1>), dim3(grid), dim3(WG), lds, s, A, shape);
                else
                    hipLaunchKernelGGL((k_adjoint<P, Q, NU, 1>), dim3(grid), dim3(WG), lds, s, A, shape);
                break;
            case 2: hipLaunchKernelGGL((k_adjoint<P, Q, NU, 2>), dim3(grid), dim3(WG), lds, s, A, shape); break;
            case 3: hipLaunchKernelGGL((k_adjoint<P, Q, NU, 3>), dim3(grid), dim3(WG), lds, s, A, shape); break;
            case 4: hipLaunchKernelGGL((k_adjoint<P, Q, NU, 4>), dim3(grid), dim3(WG), lds, s, A, shape); break;
            case 5: hipLaunchKernelGGL((k_adjoint<P, Q, NU, 5>), dim3(grid), dim3(WG), lds, s, A, shape); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    static hipError_t adjoint_fp64(const TraceArgs& A, const DesignDev64* d64, int shape, int64_t first,
                                   int64_t nblocks, int mode, hipStream_t s) {
        const int64_t nseg = 4 * nblocks, seg0 = 4 * first;  // one segment per (logical block, wave)
        const int grid = (int)std::min<int64_t>((nseg + 63) / 64, 4096);
        if (grid <= 0) return hipSuccess;
        const size_t lds = sizeof(unsigned long long) * (size_t)A.lds_cp;  // the round design's control net(s)
        switch (mode) {
            case F64_FLAT:
                hipLaunchKernelGGL((k_adjoint_fp64<P, Q, NU, F64_FLAT>), dim3(grid), dim3(WG), lds, s, A, d64, shape,
                                   seg0, nseg);
                break;
            case F64_TWO:
                hipLaunchKernelGGL((k_adjoint_fp64<P, Q, NU, F64_TWO>), dim3(grid), dim3(WG), lds, s, A, d64, shape,
                                   seg0, nseg);
                break;
            case F64_MESH:
                hipLaunchKernelGGL((k_adjoint_fp64<P, Q, NU, F64_MESH>), dim3(grid), dim3(WG), lds, s, A, d64, shape,
                                   seg0, nseg);
                break;
            case F64_TWO_COLL:
                hipLaunchKernelGGL((k_adjoint_fp64<P, Q, NU, F64_TWO_COLL>), dim3(grid), dim3(WG), lds, s, A, d64,
                                   shape, seg0, nseg);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    static hipError_t trace_rays(const TraceArgs& A, int design, const int64_t* ids, int64_t n, float* out8,
                                 hipStream_t s) {
        if (n <= 0) return hipSuccess;
        size_t lds = trace_lds_bytes(A, 0);
        int grid = (int)((n + WG - 1) / WG);
        hipLaunchKernelGGL((k_trace_rays<P, Q>), dim3(grid), dim3(WG), lds, s, A, design, ids, n, out8);
        return hipGetLastError();
    }
    static const KernelSet* get() {
        static const KernelSet ks = {&forward, &adjoint, &adjoint_fp64, &trace_rays};
        return &ks;
    }
};

}  // namespace ffrt
