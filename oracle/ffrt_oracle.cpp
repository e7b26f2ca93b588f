// FP64 CPU oracle for differentiable non-sequential ray tracing through a plano-freeform B-spline lens.
//
// TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU-baseline leg of the benchmark.
// It shares no code with the HIP library.  Every step follows the paper (de Koning et al. 2023) in its
// order and notation; where the paper is silent or garbled the reading taken is stated at the step.
//
// Structure of one ray (sec. 2.2 - 2.3):
//   sample (sec. 2.2.1) -> [point sources: flat entry face, refraction air->glass]
//   -> freeform hit (collimated: sampled on the surface; point: smallest root of f(t), sec. 2.2.1 eq. for f)
//   -> exit refraction glass->air, TIR dropped (sec. 2.2), Schlick weight (sec. 2.3)
//   -> screen plane (sec. 2.3) -> Gaussian reconstruction filter (sec. 2.3, eq. for f_i^x)
// The gradient (sec. 2.5, back-propagated in the paper) is the same pathwise derivative computed here in
// forward mode: the ray is re-evaluated with dual numbers whose tangents are the control points of the hit
// knot-span product.  At a point-source hit the root t is differentiated by Newton steps taken in dual
// arithmetic from the converged root (implicit function theorem).
#include "oracle.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

constexpr int MAXDEG = 5;
constexpr int MAXT = (MAXDEG + 1) * (MAXDEG + 1);

// ---------------------------------------------------------------------------------------------------
// Dual numbers: value plus tl_nt tangents (tl_nt is fixed for the duration of one ray).
// ---------------------------------------------------------------------------------------------------
thread_local int tl_nt = 0;

struct NoInit {};

struct Dual {
    double v;
    double d[2 * MAXT];  // both faces' local control points when the entry face is freeform too
    Dual() : v(0.0) { for (int k = 0; k < tl_nt; ++k) d[k] = 0.0; }
    Dual(double x) : v(x) { for (int k = 0; k < tl_nt; ++k) d[k] = 0.0; }
    Dual(double x, NoInit) : v(x) {}
};

inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = -a.d[k]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) { Dual r(a.v / b.v, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v); return r; }
inline Dual operator+(const Dual& a, double b) { Dual r(a.v + b, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = a.d[k]; return r; }
inline Dual operator+(double a, const Dual& b) { return b + a; }
inline Dual operator-(const Dual& a, double b) { return a + (-b); }
inline Dual operator-(double a, const Dual& b) { Dual r(a - b.v, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = -b.d[k]; return r; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = a.d[k] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
inline Dual operator/(double a, const Dual& b) { Dual r(a / b.v, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = -a * b.d[k] / (b.v * b.v); return r; }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); Dual r(s, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = a.d[k] / (2.0 * s); return r; }
inline Dual exp(const Dual& a) { double e = std::exp(a.v); Dual r(e, NoInit{}); for (int k = 0; k < tl_nt; ++k) r.d[k] = a.d[k] * e; return r; }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::exp;
using std::sqrt;

// ---------------------------------------------------------------------------------------------------
// B-spline basis (sec. 2.1)
// ---------------------------------------------------------------------------------------------------

// Clamped knot vector with p+1 zeros, p+1 ones and equispaced interior knots u_i = (i-p)/(n-p), where n is
// the number of control points (the paper's n_1 + 1), length n + p + 1.
std::vector<double> make_knots(int p, int n) {
    std::vector<double> U(n + p + 1);
    for (int i = 0; i < n + p + 1; ++i) {
        if (i <= p) U[i] = 0.0;
        else if (i >= n) U[i] = 1.0;
        else U[i] = double(i - p) / double(n - p);
    }
    return U;
}

// Knot span s with U[s] <= u < U[s+1]; u = 1 belongs to the last span s = n-1 so that N_{n-1,p}(1) = 1.
int find_span(int p, int n, double u) {
    int s = p + int(std::floor(u * double(n - p)));
    if (s < p) s = p;
    if (s > n - 1) s = n - 1;
    return s;
}

// Degree-k derivative-type combination used by the textbook derivative formula:
//   D_{i,k} = k * ( X_{i,k-1} / (U[i+k]-U[i]) - X_{i+1,k-1} / (U[i+k+1]-U[i+1]) ),  0/0 := 0,
// where X holds the k nonzero degree-(k-1) entries of span s (index m <-> function s-k+1+m).
template <class S>
void deriv_step(int k, const double* U, int s, const S* X, S* D) {
    for (int m = 0; m <= k; ++m) {
        int i = s - k + m;
        S acc = 0.0;
        double d1 = U[i + k] - U[i];
        double d2 = U[i + k + 1] - U[i + 1];
        if (m >= 1 && d1 != 0.0) acc = acc + X[m - 1] / d1;
        if (m <= k - 1 && d2 != 0.0) acc = acc - X[m] / d2;
        D[m] = acc * double(k);
    }
}

// Nonzero basis functions N_{s-p..s,p}(u) on span s, by the Cox-de Boor recursion (sec. 2.1; the second
// denominator is read as u_{i+p+1} - u_{i+1}, and 0/0 := 0), with first and second u-derivatives.
template <class S>
void basis(int p, const double* U, int s, const S& u, S* N, S* dN, S* d2N) {
    S T[MAXDEG + 1][MAXDEG + 1];  // T[k][m] = N_{s-k+m,k}(u)
    T[0][0] = 1.0;
    for (int k = 1; k <= p; ++k) {
        for (int m = 0; m <= k; ++m) {
            int i = s - k + m;
            S acc = 0.0;
            double d1 = U[i + k] - U[i];
            double d2 = U[i + k + 1] - U[i + 1];
            if (m >= 1 && d1 != 0.0) acc = acc + (u - U[i]) / d1 * T[k - 1][m - 1];
            if (m <= k - 1 && d2 != 0.0) acc = acc + (U[i + k + 1] - u) / d2 * T[k - 1][m];
            T[k][m] = acc;
        }
    }
    for (int m = 0; m <= p; ++m) N[m] = T[p][m];
    if (dN) deriv_step(p, U, s, T[p - 1], dN);
    if (d2N) {
        if (p >= 2) {
            S D1[MAXDEG + 1];
            deriv_step(p - 1, U, s, T[p - 2], D1);
            deriv_step(p, U, s, D1, d2N);
        } else {
            for (int m = 0; m <= p; ++m) d2N[m] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------------------------------
// Problem geometry
// ---------------------------------------------------------------------------------------------------
struct Geo {
    orc_problem pr;
    int p, q, nu, nv;
    std::vector<double> U, V;
    double zmin, zmax;      // global convex-hull bounds of P^z (sec. 2.2.2, whole-surface test)
    double Gx, Gy;          // bounds of |h_x|, |h_y| from the derivative control points
    int K;                  // control points of one face
    double zmin_in, zmax_in, Gx_in, Gy_in;  // the same for a freeform entry face (its net follows the exit's)
    int nxe, nye;           // effective detector resolution
    double Rxe, Rye, wx, wy;
    double R0;              // Schlick reflectance at normal incidence
    int64_t nrays;
    double w0;              // initial ray weight
};

bool valid_problem(const orc_problem* pr) {
    if (!pr) return false;
    if (pr->p < 1 || pr->q < 1 || pr->p > MAXDEG || pr->q > MAXDEG) return false;
    if (pr->n_u <= pr->p || pr->n_v <= pr->q) return false;
    if (!(pr->n_lens > 1.0) || !(pr->r_x > 0) || !(pr->r_y > 0)) return false;
    if (pr->grid_u < 1 || pr->grid_v < 1 || pr->n_x < 1 || pr->n_y < 1) return false;
    if (pr->nu_x < 1 || pr->nu_y < 1 || pr->nu_x % 2 == 0 || pr->nu_y % 2 == 0) return false;
    if (!(pr->R_x > 0) || !(pr->R_y > 0) || !(pr->alpha > 0)) return false;
    if (pr->kind < 0 || pr->kind > 2) return false;
    if (pr->filter != 0 && pr->filter != 1) return false;
    if (pr->entry_freeform != 0 && pr->entry_freeform != 1) return false;
    if (pr->loss != 0 && pr->loss != 1) return false;
    if (pr->entry_freeform && pr->mesh_u) return false;  // the mesh option covers the exit face only
    if (pr->mesh_u < 0 || pr->mesh_v < 0 || pr->mesh_u > 64 || pr->mesh_v > 64 || (pr->mesh_u == 0) != (pr->mesh_v == 0))
        return false;
    if (pr->kind != 0) {
        if (!(pr->pos_z < pr->z_in)) return false;
        if (!(pr->half_angle >= 0.0 && pr->half_angle < M_PI / 2)) return false;
        if (pr->kind == 2 && (pr->emit_nx < 1 || pr->emit_ny < 1)) return false;
    }
    return true;
}

// Height range of one face's control net and bounds of |h_x|, |h_y| from its derivative control points:
// Z_u = sum N_{i,p-1} N_{j,q} p (P_{i+1,j} - P_{i,j}) / (U[i+p+1] - U[i+1]) (likewise in v).
void face_bounds(const Geo& g, const double* Pz, double* zmin, double* zmax, double* Gx, double* Gy) {
    *zmin = *zmax = Pz[0];
    *Gx = *Gy = 0.0;
    for (int i = 0; i < g.nu * g.nv; ++i) { *zmin = std::min(*zmin, Pz[i]); *zmax = std::max(*zmax, Pz[i]); }
    for (int i = 0; i + 1 < g.nu; ++i)
        for (int j = 0; j < g.nv; ++j) {
            double den = g.U[i + g.p + 1] - g.U[i + 1];
            double Q = g.p * (Pz[(i + 1) * g.nv + j] - Pz[i * g.nv + j]) / den;
            *Gx = std::max(*Gx, std::fabs(Q) / (2.0 * g.pr.r_x));
        }
    for (int i = 0; i < g.nu; ++i)
        for (int j = 0; j + 1 < g.nv; ++j) {
            double den = g.V[j + g.q + 1] - g.V[j + 1];
            double Q = g.q * (Pz[i * g.nv + j + 1] - Pz[i * g.nv + j]) / den;
            *Gy = std::max(*Gy, std::fabs(Q) / (2.0 * g.pr.r_y));
        }
}

Geo make_geo(const orc_problem* pr, const double* Pz) {
    Geo g;
    g.pr = *pr;
    g.p = pr->p; g.q = pr->q; g.nu = pr->n_u; g.nv = pr->n_v;
    g.U = make_knots(g.p, g.nu);
    g.V = make_knots(g.q, g.nv);
    g.K = g.nu * g.nv;
    g.zmin = g.zmax = g.Gx = g.Gy = 0.0;
    g.zmin_in = g.zmax_in = g.Gx_in = g.Gy_in = 0.0;
    if (Pz) {
        face_bounds(g, Pz, &g.zmin, &g.zmax, &g.Gx, &g.Gy);
        if (pr->entry_freeform) face_bounds(g, Pz + g.K, &g.zmin_in, &g.zmax_in, &g.Gx_in, &g.Gy_in);
    }
    double wx = 2.0 * pr->R_x / pr->n_x, wy = 2.0 * pr->R_y / pr->n_y;
    g.wx = wx; g.wy = wy;
    if (pr->ghost) {  // ghost pixels (sec. 2.3): R* = R + (nu-1)/2 w, resolution n + nu - 1
        g.nxe = pr->n_x + pr->nu_x - 1; g.nye = pr->n_y + pr->nu_y - 1;
        g.Rxe = pr->R_x + 0.5 * (pr->nu_x - 1) * wx; g.Rye = pr->R_y + 0.5 * (pr->nu_y - 1) * wy;
    } else {
        g.nxe = pr->n_x; g.nye = pr->n_y; g.Rxe = pr->R_x; g.Rye = pr->R_y;
    }
    double r0 = (pr->n_lens - 1.0) / (pr->n_lens + 1.0);
    g.R0 = r0 * r0;
    int64_t per = int64_t(pr->grid_u) * pr->grid_v;
    if (pr->kind == 2) per *= int64_t(pr->emit_nx) * pr->emit_ny;
    g.nrays = per;
    g.w0 = 1.0 / double(per);
    return g;
}

// Surface derivatives at (u, v) on span (su, sv) with local control points Pl[(a)*(q+1)+b] =
// P^z_{su-p+a, sv-q+b}.  Returns h and its x/y derivatives (X = (2u-1) r_x, so d/dx = d/du / (2 r_x)).
template <class S>
struct Surf { S h, hx, hy, hxx, hxy, hyy; };

template <class S>
Surf<S> eval_surface(const Geo& g, const S* Pl, int su, int sv, const S& u, const S& v, bool second) {
    S Nu[MAXDEG + 1], dNu[MAXDEG + 1], d2Nu[MAXDEG + 1];
    S Nv[MAXDEG + 1], dNv[MAXDEG + 1], d2Nv[MAXDEG + 1];
    basis(g.p, g.U.data(), su, u, Nu, dNu, second ? d2Nu : nullptr);
    basis(g.q, g.V.data(), sv, v, Nv, dNv, second ? d2Nv : nullptr);
    // S(u,v) = sum_i sum_j N_i(u) N_j(v) P_ij (sec. 2.1, tensor-product surface)
    S h = 0.0, hu = 0.0, hv = 0.0, huu = 0.0, huv = 0.0, hvv = 0.0;
    for (int a = 0; a <= g.p; ++a)
        for (int b = 0; b <= g.q; ++b) {
            const S& P = Pl[a * (g.q + 1) + b];
            h = h + Nu[a] * Nv[b] * P;
            hu = hu + dNu[a] * Nv[b] * P;
            hv = hv + Nu[a] * dNv[b] * P;
            if (second) {
                huu = huu + d2Nu[a] * Nv[b] * P;
                huv = huv + dNu[a] * dNv[b] * P;
                hvv = hvv + Nu[a] * d2Nv[b] * P;
            }
        }
    Surf<S> r;
    double sx = 1.0 / (2.0 * g.pr.r_x), sy = 1.0 / (2.0 * g.pr.r_y);
    r.h = h; r.hx = hu * sx; r.hy = hv * sy;
    r.hxx = huu * (sx * sx); r.hxy = huv * (sx * sy); r.hyy = hvv * (sy * sy);
    return r;
}

// Local control points of the span product containing (u, v), as doubles.
void local_cps(const Geo& g, const double* Pz, int su, int sv, double* Pl) {
    for (int a = 0; a <= g.p; ++a)
        for (int b = 0; b <= g.q; ++b)
            Pl[a * (g.q + 1) + b] = Pz[(su - g.p + a) * g.nv + (sv - g.q + b)];
}

// h(x, y) and derivatives in double precision from the full control net.
Surf<double> surface_at(const Geo& g, const double* Pz, double x, double y, bool second) {
    double u = 0.5 * (x / g.pr.r_x + 1.0), v = 0.5 * (y / g.pr.r_y + 1.0);  // X^{-1}, Y^{-1} (sec. 2.1.1)
    int su = find_span(g.p, g.nu, u), sv = find_span(g.q, g.nv, v);
    double Pl[MAXT];
    local_cps(g, Pz, su, sv, Pl);
    return eval_surface<double>(g, Pl, su, sv, u, v, second);
}

// ---------------------------------------------------------------------------------------------------
// Random numbers: counter-based SplitMix64 (Steele, Lea, Flood 2014).  Output i of the SplitMix64 sequence
// whose state starts at mix(seed + stream * gamma).
// ---------------------------------------------------------------------------------------------------
constexpr uint64_t GOLDEN_GAMMA = 0x9E3779B97F4A7C15ull;
uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
uint64_t rng_at(uint64_t seed, uint64_t stream, uint64_t index) {
    uint64_t state = mix64(seed + stream * GOLDEN_GAMMA);
    return mix64(state + (index + 1) * GOLDEN_GAMMA);
}
constexpr uint64_t RAY_STREAM = 2;

// Two 24-bit uniforms in [0,1) from one output.
void two_uniforms(uint64_t h, double* a, double* b) {
    *a = double(h >> 40) * (1.0 / 16777216.0);
    *b = double((h >> 16) & 0xFFFFFFull) * (1.0 / 16777216.0);
}

// ---------------------------------------------------------------------------------------------------
// Sources (sec. 2.2.1; grid of point sources, sec. 3.3)
// ---------------------------------------------------------------------------------------------------
// Collimated: rays sampled on a square grid of [0,1]^2 directly on the B-spline surface.  Reading: samples
// are cell-centred (k + 1/2)/N, or (k + xi)/N when jittered.  Ray id = k_u * N_v + k_v.
void sample_collimated(const Geo& g, int64_t id, double* u, double* v) {
    int64_t ku = id / g.pr.grid_v, kv = id % g.pr.grid_v;
    double xu = 0.5, xv = 0.5;
    if (g.pr.jitter) two_uniforms(rng_at(g.pr.seed, RAY_STREAM, uint64_t(id)), &xu, &xv);
    *u = (double(ku) + xu) / double(g.pr.grid_u);
    *v = (double(kv) + xv) / double(g.pr.grid_v);
}

// Point source: theta uniform in [0, 2 pi), a uniform in [0,1], phi = arccos(1 - (1 - cos phi_max) a)
// (uniform in solid angle).  Reading: the "uniform" draws are stratified, k_theta and k_a being the strata.
// Ray id = e * (S_theta S_a) + k_theta * S_a + k_a for emitter e (kind 2: grid of emitters, endpoints
// included, row-major in (x, y)).
void sample_point(const Geo& g, int64_t id, double* theta, double* a, double* ex, double* ey) {
    int64_t per = int64_t(g.pr.grid_u) * g.pr.grid_v;
    int64_t e = id / per, r = id % per;
    int64_t kt = r / g.pr.grid_v, ka = r % g.pr.grid_v;
    double x1 = 0.5, x2 = 0.5;
    if (g.pr.jitter) two_uniforms(rng_at(g.pr.seed, RAY_STREAM, uint64_t(id)), &x1, &x2);
    *theta = 2.0 * M_PI * (double(kt) + x1) / double(g.pr.grid_u);
    *a = (double(ka) + x2) / double(g.pr.grid_v);
    *ex = g.pr.pos_x; *ey = g.pr.pos_y;
    if (g.pr.kind == 2) {
        int64_t ix = e / g.pr.emit_ny, iy = e % g.pr.emit_ny;
        if (g.pr.emit_nx > 1) *ex += -0.5 * g.pr.emit_wx + double(ix) * g.pr.emit_wx / double(g.pr.emit_nx - 1);
        if (g.pr.emit_ny > 1) *ey += -0.5 * g.pr.emit_wy + double(iy) * g.pr.emit_wy / double(g.pr.emit_ny - 1);
    }
}

// ---------------------------------------------------------------------------------------------------
// Optics
// ---------------------------------------------------------------------------------------------------
// Schlick's approximation, R = R0 + (1 - R0)(1 - c)^5.  Reading: c is the cosine on the air side.
template <class S>
S schlick(const S& c, double R0) {
    S m = 1.0 - c;
    S m2 = m * m;
    return R0 + (1.0 - R0) * (m2 * m2 * m);
}

// Vector Snell law (the paper does not print it; textbook form): n_hat on the transmitted side,
// eta = n_i / n_t, c = d . n_hat, k = 1 - eta^2 (1 - c^2); k < 0 is TIR; d_t = eta d + (sqrt(k) - eta c) n_hat.
// ---------------------------------------------------------------------------------------------------

struct Entry {          // the ray up to the exit face: origin/direction inside the glass and weight
    int status;         // ORC_HIT (continues) or ORC_MISS_ENTRY
    double o[3], d[3], w;
    bool collimated;    // sampled on the exit face itself (flat entry face): no root search there
    double u, v;        // collimated: the sample on the surface
    double margin;      // distance of the entry point to the aperture edge (point sources)
    // freeform entry face: the source ray (air) and where it met the entry face
    bool freeform;
    double s[3], d0[3]; // point of departure (source, or the collimated sample below the lens) and direction
    double t_in;        // parameter of the entry hit along s + t d0
    int su_in, sv_in;   // its knot span product
};

// Entry face z = g(x, y) as a second B-spline (its control net follows the exit face's in Pz): the source ray
// s + t d0 meets it at the smallest t whose point lies over the aperture.  The aperture prism is crossed for
// t in [t_a, t_b]; the ray must enter it below the face and leave it above, else it passes the lens
// (ORC_MISS_ENTRY).  Root: bracket by the face's height range, strict monotonicity from its slope bounds, or
// a scan for the first sign change; bisection, then Newton polish (as for the exit face).
double f_in_of_t(const Geo& g, const double* Pz_in, const double* s, const double* d0, double t);
bool find_entry_root(const Geo& g, const double* Pz_in, const double* s, const double* d0, double* t_out,
                     double* margin) {
    double t_a = 0.0, t_b = std::numeric_limits<double>::infinity();
    const double r[2] = {g.pr.r_x, g.pr.r_y};
    for (int ax = 0; ax < 2; ++ax) {
        if (d0[ax] == 0.0) {
            if (std::fabs(s[ax]) > r[ax]) return false;
            continue;
        }
        double ta = (-r[ax] - s[ax]) / d0[ax], tb = (r[ax] - s[ax]) / d0[ax];
        if (ta > tb) std::swap(ta, tb);
        t_a = std::max(t_a, ta);
        t_b = std::min(t_b, tb);
    }
    double pad = 1e-9 * (1.0 + std::fabs(g.zmax_in - s[2])) / d0[2];
    double a = std::max(t_a, (g.zmin_in - s[2]) / d0[2] - pad), b = std::min(t_b, (g.zmax_in - s[2]) / d0[2] + pad);
    a = std::max(a, 0.0);
    if (!(a <= b)) { *margin = 0.0; return false; }
    double fa = f_in_of_t(g, Pz_in, s, d0, a), fb = f_in_of_t(g, Pz_in, s, d0, b);
    // The signs of f at the bracket ends are decisions (side wall, passed the lens) only where an end is the
    // aperture prism's wall; an end set by the face's height range has its sign by construction.
    *margin = std::numeric_limits<double>::infinity();
    if (a == t_a) *margin = std::fabs(fa);
    if (b == t_b) *margin = std::min(*margin, std::fabs(fb));
    if (fa < 0.0) return false;  // entered the prism above the face (through the side wall)
    bool monotone = g.Gx_in * std::fabs(d0[0]) + g.Gy_in * std::fabs(d0[1]) < d0[2];
    if (monotone) {
        if (fb > 0.0) return false;  // left the prism below the face: passed the lens
    } else {
        // the first sign change (a ray that crossed the face and met it again before leaving the prism has
        // its smallest root in between); none at any sample: the ray passed the lens
        double du = std::fabs(d0[0]) * (b - a) / (2.0 * g.pr.r_x) * (g.nu - g.p);
        double dv = std::fabs(d0[1]) * (b - a) / (2.0 * g.pr.r_y) * (g.nv - g.q);
        int64_t M = std::max<int64_t>(64, int64_t(std::ceil(64.0 * (du + dv))) + 1);
        double prev = a;
        bool found = false;
        for (int64_t k = 1; k <= M; ++k) {
            double t = a + (b - a) * double(k) / double(M);
            if (f_in_of_t(g, Pz_in, s, d0, t) <= 0.0) { b = t; a = prev; found = true; break; }
            prev = t;
        }
        if (!found) return false;
    }
    for (int it = 0; it < 200 && (b - a) > 1e-11 * (1.0 + b); ++it) {
        double m = 0.5 * (a + b);
        if (f_in_of_t(g, Pz_in, s, d0, m) > 0.0) a = m; else b = m;
    }
    double t = 0.5 * (a + b);
    double slack = b - a;
    for (int it = 0; it < 6; ++it) {
        Surf<double> sf = surface_at(g, Pz_in, s[0] + t * d0[0], s[1] + t * d0[1], false);
        double f = sf.h - s[2] - t * d0[2];
        double fp = sf.hx * d0[0] + sf.hy * d0[1] - d0[2];
        if (fp == 0.0) break;
        double tn = t - f / fp;
        if (!(tn >= a - slack && tn <= b + slack)) break;
        bool done = std::fabs(tn - t) <= 1e-15 * (1.0 + std::fabs(t));
        t = tn;
        if (done) break;
    }
    *t_out = t;
    return true;
}

double f_in_of_t(const Geo& g, const double* Pz_in, const double* s, const double* d0, double t) {
    return surface_at(g, Pz_in, s[0] + t * d0[0], s[1] + t * d0[1], false).h - s[2] - t * d0[2];
}

// Refraction air -> glass at the freeform entry face (normal (-g_x, -g_y, 1)/|.|, pointing into the glass)
// and the Schlick weight with the air-side cosine d0 . n.
template <class S>
void refract_in(const Geo& g, const S* d0, const S& gx, const S& gy, S* d1, S* wfac) {
    S nn = sqrt(gx * gx + gy * gy + 1.0);
    S n0 = -gx / nn, n1 = -gy / nn, n2 = 1.0 / nn;
    double eta = 1.0 / g.pr.n_lens;
    S c = d0[0] * n0 + d0[1] * n1 + d0[2] * n2;
    S k = 1.0 - eta * eta * (1.0 - c * c);
    S beta = sqrt(k) - eta * c;
    d1[0] = eta * d0[0] + beta * n0;
    d1[1] = eta * d0[1] + beta * n1;
    d1[2] = eta * d0[2] + beta * n2;
    *wfac = g.pr.fresnel ? 1.0 - schlick(c, g.R0) : S(1.0);
}

Entry ray_entry(const Geo& g, const double* Pz, int64_t id) {
    Entry E;
    E.status = ORC_HIT;
    E.margin = 1e300;
    E.freeform = false;
    E.t_in = 0.0;
    E.su_in = E.sv_in = 0;
    const orc_problem& pr = g.pr;
    if (pr.entry_freeform) {
        // both faces freeform: the ray crosses the entry B-spline, then searches the exit face like any ray
        E.freeform = true;
        E.collimated = false;
        const double* Pin = Pz + g.K;
        if (pr.kind == 0) {
            sample_collimated(g, id, &E.u, &E.v);
            E.s[0] = (2.0 * E.u - 1.0) * pr.r_x;
            E.s[1] = (2.0 * E.v - 1.0) * pr.r_y;
            E.s[2] = g.zmin_in - 1.0;
            E.d0[0] = 0.0; E.d0[1] = 0.0; E.d0[2] = 1.0;
            Surf<double> sf = surface_at(g, Pin, E.s[0], E.s[1], false);
            E.t_in = sf.h - E.s[2];
        } else {
            double theta, a, ex, ey;
            sample_point(g, id, &theta, &a, &ex, &ey);
            double cphi = 1.0 - (1.0 - std::cos(pr.half_angle)) * a;
            double sphi = std::sqrt(std::max(0.0, 1.0 - cphi * cphi));
            E.s[0] = ex; E.s[1] = ey; E.s[2] = pr.pos_z;
            E.d0[0] = std::cos(theta) * sphi; E.d0[1] = std::sin(theta) * sphi; E.d0[2] = cphi;
            double margin = 0.0;
            bool ok = find_entry_root(g, Pin, E.s, E.d0, &E.t_in, &margin);
            E.margin = margin;
            if (!ok) { E.status = ORC_MISS_ENTRY; return E; }
        }
        double p0[3];
        for (int i = 0; i < 3; ++i) p0[i] = E.s[i] + E.t_in * E.d0[i];
        if (pr.kind != 0)
            E.margin = std::min(E.margin, std::min(pr.r_x - std::fabs(p0[0]), pr.r_y - std::fabs(p0[1])));
        double u = 0.5 * (p0[0] / pr.r_x + 1.0), v = 0.5 * (p0[1] / pr.r_y + 1.0);
        E.su_in = find_span(g.p, g.nu, u);
        E.sv_in = find_span(g.q, g.nv, v);
        Surf<double> sf = surface_at(g, Pin, p0[0], p0[1], false);
        double wfac;
        refract_in<double>(g, E.d0, sf.hx, sf.hy, E.d, &wfac);
        for (int i = 0; i < 3; ++i) E.o[i] = p0[i];
        E.w = g.w0 * wfac;
        return E;
    }
    if (pr.kind == 0) {
        // Collimated bundle: the path to the freeform is parallel to z, rays start on the surface with
        // d = (0,0,1).  They cross the flat face at normal incidence: Schlick weight 1 - R0.
        E.collimated = true;
        sample_collimated(g, id, &E.u, &E.v);
        E.o[0] = (2.0 * E.u - 1.0) * pr.r_x;
        E.o[1] = (2.0 * E.v - 1.0) * pr.r_y;
        E.o[2] = pr.z_in;
        E.d[0] = 0.0; E.d[1] = 0.0; E.d[2] = 1.0;
        E.w = g.w0 * (pr.fresnel ? 1.0 - g.R0 : 1.0);
        return E;
    }
    E.collimated = false;
    double theta, a, ex, ey;
    sample_point(g, id, &theta, &a, &ex, &ey);
    double cphi = 1.0 - (1.0 - std::cos(pr.half_angle)) * a;
    double sphi = std::sqrt(std::max(0.0, 1.0 - cphi * cphi));
    double d0[3] = {std::cos(theta) * sphi, std::sin(theta) * sphi, cphi};
    // Flat entry face z = z_in over the aperture; rays outside it are dropped (other paths ignored, sec 2.2).
    double t0 = (pr.z_in - pr.pos_z) / d0[2];
    double p0[3] = {ex + t0 * d0[0], ey + t0 * d0[1], pr.z_in};
    E.margin = std::min(pr.r_x - std::fabs(p0[0]), pr.r_y - std::fabs(p0[1]));
    if (std::fabs(p0[0]) > pr.r_x || std::fabs(p0[1]) > pr.r_y) { E.status = ORC_MISS_ENTRY; return E; }
    // Refraction air -> glass at normal (0,0,1), eta = 1/n.
    double eta = 1.0 / pr.n_lens;
    double c = d0[2];
    double k = 1.0 - eta * eta * (1.0 - c * c);
    double sk = std::sqrt(k);
    for (int i = 0; i < 3; ++i) E.d[i] = eta * d0[i] + (i == 2 ? (sk - eta * c) : 0.0);
    for (int i = 0; i < 3; ++i) E.o[i] = p0[i];
    E.w = g.w0 * (pr.fresnel ? 1.0 - schlick(c, g.R0) : 1.0);  // air-side cosine is the incidence cosine
    return E;
}

// f(t) = h(o_xy + t d_xy) - o_z - t d_z  (sec. 2.2.1, the root problem, written in x,y instead of u,v).
double f_of_t(const Geo& g, const double* Pz, const Entry& E, double t) {
    double x = E.o[0] + t * E.d[0], y = E.o[1] + t * E.d[1];
    return surface_at(g, Pz, x, y, false).h - E.o[2] - t * E.d[2];
}

struct Root { int status; double t; double margin; };

// Smallest positive root of f whose point lies in the lens aperture.  Exact in double precision:
// the bracket comes from the global convex-hull bounds (sec. 2.2.2); when the derivative bound proves f
// strictly decreasing the root is unique and found by bisection, otherwise the bracket is scanned in steps
// of 1/64 of a projected knot span for the first sign change.  Newton steps polish the root.
Root find_root(const Geo& g, const double* Pz, const Entry& E, bool ignore_aperture = false) {
    Root R; R.status = ORC_HIT; R.t = 0.0; R.margin = 1e300;
    const double* o = E.o; const double* d = E.d;
    // Bracket widened by a rounding margin so that f(t_lo) > 0 > f(t_hi) also for a flat surface.
    double pad = 1e-9 * (1.0 + std::fabs(g.zmax - o[2])) / d[2];
    double t_lo = std::max(0.0, (g.zmin - o[2]) / d[2] - pad);
    double t_hi = (g.zmax - o[2]) / d[2] + pad;
    double t_ap = std::numeric_limits<double>::infinity();
    const double r[2] = {g.pr.r_x, g.pr.r_y};
    for (int ax = 0; ax < 2; ++ax) {
        if (d[ax] > 0) t_ap = std::min(t_ap, (r[ax] - o[ax]) / d[ax]);
        else if (d[ax] < 0) t_ap = std::min(t_ap, (-r[ax] - o[ax]) / d[ax]);
    }
    if (ignore_aperture) t_ap = std::numeric_limits<double>::infinity();
    double t_end = std::min(t_hi, t_ap);
    if (t_end < t_lo) { R.status = ORC_SIDE_WALL; R.margin = (t_lo - t_end) * d[2]; return R; }
    double f_end = f_of_t(g, Pz, E, t_end);
    if (t_ap <= t_hi) R.margin = std::fabs(f_end);
    double a = t_lo, b = t_end;
    bool monotone = g.Gx * std::fabs(d[0]) + g.Gy * std::fabs(d[1]) < d[2];
    if (monotone) {
        // f strictly decreasing: still below the surface where the ray leaves the aperture means no root
        if (f_end > 0.0) { R.status = ORC_SIDE_WALL; return R; }
    } else {
        // the first sign change; a ray that crossed the surface and met it again before leaving the aperture
        // (f back above zero at t_end) has its smallest root in between, and only a ray that stays below the
        // surface at every sample leaves through the side wall
        double du = std::fabs(d[0]) * (t_end - t_lo) / (2.0 * g.pr.r_x) * (g.nu - g.p);
        double dv = std::fabs(d[1]) * (t_end - t_lo) / (2.0 * g.pr.r_y) * (g.nv - g.q);
        int64_t M = std::max<int64_t>(64, int64_t(std::ceil(64.0 * (du + dv))) + 1);
        double prev = t_lo;
        bool found = false;
        for (int64_t k = 1; k <= M; ++k) {
            double t = t_lo + (t_end - t_lo) * double(k) / double(M);
            if (f_of_t(g, Pz, E, t) <= 0.0) { a = prev; b = t; found = true; break; }
            prev = t;
        }
        if (!found) { R.status = ORC_SIDE_WALL; return R; }
    }
    // Bisection: f(a) > 0 >= f(b).
    for (int it = 0; it < 200 && (b - a) > 1e-11 * (1.0 + b); ++it) {
        double m = 0.5 * (a + b);
        if (f_of_t(g, Pz, E, m) > 0.0) a = m; else b = m;
    }
    double t = 0.5 * (a + b);
    double slack = b - a;              // the root may sit on a bracket end up to rounding of f
    for (int it = 0; it < 6; ++it) {  // guarded Newton polish
        double x = o[0] + t * d[0], y = o[1] + t * d[1];
        Surf<double> s = surface_at(g, Pz, x, y, false);
        double f = s.h - o[2] - t * d[2];
        double fp = s.hx * d[0] + s.hy * d[1] - d[2];
        if (fp == 0.0) break;
        double tn = t - f / fp;
        if (!(tn >= a - slack && tn <= b + slack)) break;
        bool done = std::fabs(tn - t) <= 1e-15 * (1.0 + std::fabs(t));
        t = tn;
        if (done) break;
    }
    R.t = t;
    return R;
}

// ---------------------------------------------------------------------------------------------------
// Triangle-mesh intersection (sec. 2.2.2, the paper's own intersector).  Each knot span product is divided
// into mesh_u x mesh_v rectangles of equal size in (u, v); each rectangle into a lower-left triangle (its
// left and lower edges closed, the diagonal open) and an upper-right one (the diagonal closed, its right and
// upper edges open, except on the border of [0,1]^2), whose corners lie on the surface: together they
// partition the domain.  The hit is the ray's first point (smallest t >= 0) on that piecewise-linear
// surface.  Work in (u, v, z): o_u = (o_x / r_x + 1) / 2, d_u = d_x / (2 r_x), likewise v.
//   Phase 1: the ray must cross the box [0,1]^2 x [min P^z, max P^z]; then rectangles of knot span
//            products are split into at most four and tested against their own boxes (the heights of the
//            control points acting on them, by the strong convex hull property) down to single products.
//   Phase 2/3: every triangle of a surviving span product is intersected as a plane T(u,v) = A u + B v + C
//            through its three corners, and the hit kept if it lies in the triangle's (u, v) domain.  (The
//            paper first selects candidate triangles by where the ray's (u, v) line crosses the grid lines;
//            testing all of them here gives the same first hit.)
// ---------------------------------------------------------------------------------------------------
struct MeshHit {
    bool hit;
    double t;
    int su, sv;      // knot span indices (U[su] <= u < U[su + 1])
    int k, l;        // rectangle within the span product
    int upper;       // 0 lower-left, 1 upper-right triangle
};

// Height Z(u, v) at a mesh node of span product (su, sv), evaluated with that product's basis functions
// (which the paper notes depend on the node only, not on P).
template <class S>
S node_height(const Geo& g, const S* Pl, int su, int sv, double u, double v) {
    double Nu[MAXDEG + 1], dNu[MAXDEG + 1], Nv[MAXDEG + 1], dNv[MAXDEG + 1];
    basis<double>(g.p, g.U.data(), su, u, Nu, dNu, nullptr);
    basis<double>(g.q, g.V.data(), sv, v, Nv, dNv, nullptr);
    S h = 0.0;
    for (int a = 0; a <= g.p; ++a)
        for (int b = 0; b <= g.q; ++b) h = h + Pl[a * (g.q + 1) + b] * (Nu[a] * Nv[b]);
    return h;
}

// Corner coordinates of rectangle (k, l) of span product (su, sv).
void mesh_cell(const Geo& g, int su, int sv, int k, int l, double* u0, double* du, double* v0, double* dv) {
    *du = (g.U[su + 1] - g.U[su]) / g.pr.mesh_u;
    *dv = (g.V[sv + 1] - g.V[sv]) / g.pr.mesh_v;
    *u0 = g.U[su] + k * *du;
    *v0 = g.V[sv] + l * *dv;
}

// Plane of a triangle: T(u, v) = z_c + A (u - u_c) + B (v - v_c) through corner c, from the corner heights
// z00 = Z(u_k, v_l), z10 = Z(u_k+1, v_l), z01 = Z(u_k, v_l+1), z11 = Z(u_k+1, v_l+1).
template <class S>
void tri_plane(int upper, const S* z, double du, double dv, S* A, S* B) {
    if (!upper) { *A = (z[1] - z[0]) / du; *B = (z[2] - z[0]) / dv; }   // corners 00, 10, 01
    else { *A = (z[3] - z[2]) / du; *B = (z[3] - z[1]) / dv; }          // corners 11, 01, 10
}

// Whether (a, b) = ((u - u_k)/du, (v - v_l)/dv) lies in the triangle; last_u / last_v close the open edges
// on the border u = 1 / v = 1 of the domain.
bool in_triangle(int upper, double a, double b, bool last_u, bool last_v) {
    if (!upper) return a >= 0.0 && b >= 0.0 && a + b < 1.0;
    return a + b >= 1.0 && (a < 1.0 || (last_u && a <= 1.0)) && (b < 1.0 || (last_v && b <= 1.0));
}

// The ray's hit on triangle (k, l, upper) of span product (su, sv), if any, with t in [t0, t1].
bool mesh_triangle_hit(const Geo& g, const double* Pz, const double* o, const double* d, int su, int sv, int k,
                       int l, int upper, double t0, double t1, double* t_out) {
    double u0, du, v0, dv;
    mesh_cell(g, su, sv, k, l, &u0, &du, &v0, &dv);
    double Pl[MAXT];
    local_cps(g, Pz, su, sv, Pl);
    double z[4] = {node_height(g, Pl, su, sv, u0, v0), node_height(g, Pl, su, sv, u0 + du, v0),
                   node_height(g, Pl, su, sv, u0, v0 + dv), node_height(g, Pl, su, sv, u0 + du, v0 + dv)};
    double A, B;
    tri_plane(upper, z, du, dv, &A, &B);
    double uc = upper ? u0 + du : u0, vc = upper ? v0 + dv : v0, zc = upper ? z[3] : z[0];
    double ou = 0.5 * (o[0] / g.pr.r_x + 1.0), ov = 0.5 * (o[1] / g.pr.r_y + 1.0);
    double du_t = d[0] / (2.0 * g.pr.r_x), dv_t = d[1] / (2.0 * g.pr.r_y);
    // o_z + d_z t = zc + A (o_u + d_u t - uc) + B (o_v + d_v t - vc)
    double den = d[2] - A * du_t - B * dv_t;
    if (den == 0.0) return false;  // ray parallel to the triangle
    double t = (zc + A * (ou - uc) + B * (ov - vc) - o[2]) / den;
    if (!(t >= t0 && t <= t1)) return false;
    double a = (ou + du_t * t - u0) / du, b = (ov + dv_t * t - v0) / dv;
    bool last_u = su == g.nu - 1 && k == g.pr.mesh_u - 1, last_v = sv == g.nv - 1 && l == g.pr.mesh_v - 1;
    if (!in_triangle(upper, a, b, last_u, last_v)) return false;
    *t_out = t;
    return true;
}

// Ray parameters where the (u, v, z) ray crosses the box [ua, ub] x [va, vb] x [za, zb] (slab method).
bool ray_box(const double* ouvz, const double* duvz, const double* lo, const double* hi, double* t0, double* t1) {
    double a = *t0, b = *t1;
    for (int ax = 0; ax < 3; ++ax) {
        if (duvz[ax] == 0.0) {
            if (ouvz[ax] < lo[ax] || ouvz[ax] > hi[ax]) return false;
            continue;
        }
        double ta = (lo[ax] - ouvz[ax]) / duvz[ax], tb = (hi[ax] - ouvz[ax]) / duvz[ax];
        if (ta > tb) std::swap(ta, tb);
        a = std::max(a, ta);
        b = std::min(b, tb);
    }
    *t0 = a; *t1 = b;
    return a <= b;
}

// Phase 1 recursion over the rectangle of span products [a0, a1) x [b0, b1) (span indices counted from 0).
void mesh_boxes(const Geo& g, const double* Pz, const double* o, const double* d, const double* ouvz,
                const double* duvz, int a0, int a1, int b0, int b1, double t0, double t1, MeshHit* best) {
    double zl = 1e300, zh = -1e300;
    for (int i = a0; i <= a1 - 1 + g.p; ++i)       // control points acting on these products
        for (int j = b0; j <= b1 - 1 + g.q; ++j) {
            zl = std::min(zl, Pz[i * g.nv + j]);
            zh = std::max(zh, Pz[i * g.nv + j]);
        }
    double pad = 1e-12 * (1.0 + std::fabs(zh));
    double lo[3] = {g.U[g.p + a0], g.V[g.q + b0], zl - pad}, hi[3] = {g.U[g.p + a1], g.V[g.q + b1], zh + pad};
    double ta = t0, tb = best->hit ? std::min(t1, best->t) : t1;
    if (!ray_box(ouvz, duvz, lo, hi, &ta, &tb)) return;
    if (a1 - a0 == 1 && b1 - b0 == 1) {
        int su = g.p + a0, sv = g.q + b0;
        for (int k = 0; k < g.pr.mesh_u; ++k)
            for (int l = 0; l < g.pr.mesh_v; ++l)
                for (int up = 0; up < 2; ++up) {
                    double t;
                    if (mesh_triangle_hit(g, Pz, o, d, su, sv, k, l, up, t0, t1, &t) && (!best->hit || t < best->t))
                        *best = MeshHit{true, t, su, sv, k, l, up};
                }
        return;
    }
    int am = a1 - a0 > 1 ? (a0 + a1) / 2 : a1, bm = b1 - b0 > 1 ? (b0 + b1) / 2 : b1;
    const int ra[3] = {a0, am, a1}, rb[3] = {b0, bm, b1};
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            if (ra[x] < ra[x + 1] && rb[y] < rb[y + 1])
                mesh_boxes(g, Pz, o, d, ouvz, duvz, ra[x], ra[x + 1], rb[y], rb[y + 1], t0, t1, best);
}

MeshHit find_mesh_hit(const Geo& g, const double* Pz, const Entry& E) {
    MeshHit best{false, 0.0, 0, 0, 0, 0, 0};
    const double* o = E.o; const double* d = E.d;
    double ouvz[3] = {0.5 * (o[0] / g.pr.r_x + 1.0), 0.5 * (o[1] / g.pr.r_y + 1.0), o[2]};
    double duvz[3] = {d[0] / (2.0 * g.pr.r_x), d[1] / (2.0 * g.pr.r_y), d[2]};
    mesh_boxes(g, Pz, o, d, ouvz, duvz, 0, g.nu - g.p, 0, g.nv - g.q, 0.0, 1e300, &best);
    return best;
}

// The triangle containing the sample (u, v) of a collimated ray, and the hit's height on it.
MeshHit mesh_cell_of(const Geo& g, double u, double v) {
    MeshHit h{true, 0.0, find_span(g.p, g.nu, u), find_span(g.q, g.nv, v), 0, 0, 0};
    double du = (g.U[h.su + 1] - g.U[h.su]) / g.pr.mesh_u, dv = (g.V[h.sv + 1] - g.V[h.sv]) / g.pr.mesh_v;
    h.k = std::min(g.pr.mesh_u - 1, std::max(0, int(std::floor((u - g.U[h.su]) / du))));
    h.l = std::min(g.pr.mesh_v - 1, std::max(0, int(std::floor((v - g.V[h.sv]) / dv))));
    double a = (u - g.U[h.su]) / du - h.k, b = (v - g.V[h.sv]) / dv - h.l;
    h.upper = a + b >= 1.0 ? 1 : 0;
    return h;
}

// Ray parameter of the hit on triangle h: o_z + d_z t = T(o_u + d_u t, o_v + d_v t) (values or duals).
template <class S>
S mesh_t(const Geo& g, const S* Pl, const MeshHit& h, const double* o, const double* d) {
    double u0, du, v0, dv;
    mesh_cell(g, h.su, h.sv, h.k, h.l, &u0, &du, &v0, &dv);
    S z[4] = {node_height(g, Pl, h.su, h.sv, u0, v0), node_height(g, Pl, h.su, h.sv, u0 + du, v0),
              node_height(g, Pl, h.su, h.sv, u0, v0 + dv), node_height(g, Pl, h.su, h.sv, u0 + du, v0 + dv)};
    S A, B;
    tri_plane(h.upper, z, du, dv, &A, &B);
    double uc = h.upper ? u0 + du : u0, vc = h.upper ? v0 + dv : v0;
    S zc = h.upper ? z[3] : z[0];
    double ou = 0.5 * (o[0] / g.pr.r_x + 1.0), ov = 0.5 * (o[1] / g.pr.r_y + 1.0);
    double du_t = d[0] / (2.0 * g.pr.r_x), dv_t = d[1] / (2.0 * g.pr.r_y);
    return (zc + A * (ou - uc) + B * (ov - vc) - o[2]) / (d[2] - A * du_t - B * dv_t);
}

// Height of the mesh at (u, v) on triangle h (values or duals over the product's control points).
template <class S>
S mesh_height(const Geo& g, const S* Pl, const MeshHit& h, const S& u, const S& v) {
    double u0, du, v0, dv;
    mesh_cell(g, h.su, h.sv, h.k, h.l, &u0, &du, &v0, &dv);
    S z[4] = {node_height(g, Pl, h.su, h.sv, u0, v0), node_height(g, Pl, h.su, h.sv, u0 + du, v0),
              node_height(g, Pl, h.su, h.sv, u0, v0 + dv), node_height(g, Pl, h.su, h.sv, u0 + du, v0 + dv)};
    S A, B;
    tri_plane(h.upper, z, du, dv, &A, &B);
    if (!h.upper) return z[0] + A * (u - u0) + B * (v - v0);
    return z[3] + A * (u - (u0 + du)) + B * (v - (v0 + dv));
}

// Result of the P-dependent part of a ray (templated: double for values, Dual for derivatives).
template <class S>
struct Exit {
    int status;
    S X, Y, w;
    double k;        // Snell discriminant at the exit face (TIR margin)
    double gain;     // landing displacement per radian of rotation of the ray inside the glass (mm)
};

// Exit refraction at the freeform, Schlick weight, propagation to the screen.
template <class S>
Exit<S> exit_and_screen(const Geo& g, const S* q, const S* d, const S& hx, const S& hy, const S& w_in,
                        bool ignore_tir) {
    Exit<S> X;
    X.status = ORC_HIT;
    X.gain = 0.0;
    // Outward unit normal of z = h(x,y): (-h_x, -h_y, 1) / |.|
    S m0 = -hx, m1 = -hy;
    S nn = sqrt(m0 * m0 + m1 * m1 + 1.0);
    S n0 = m0 / nn, n1 = m1 / nn, n2 = 1.0 / nn;
    double eta = g.pr.n_lens;  // glass -> air
    S c = n0 * d[0] + n1 * d[1] + n2 * d[2];
    S k = 1.0 - eta * eta * (1.0 - c * c);
    X.k = val(k);
    if (val(k) < 0.0) {
        if (!ignore_tir) { X.status = ORC_TIR; return X; }
        k = S(0.0);
    }
    S sk = sqrt(k);
    S beta = sk - eta * c;
    S e0 = eta * d[0] + beta * n0, e1 = eta * d[1] + beta * n1, e2 = eta * d[2] + beta * n2;
    S T = g.pr.fresnel ? 1.0 - schlick(sk, g.R0) : S(1.0);
    X.w = T * w_in;
    if (!(val(e2) > 0.0)) { X.status = ORC_OFF_SCREEN; return X; }
    S tau = (g.pr.z_screen - q[2]) / e2;
    X.X = q[0] + tau * e0;
    X.Y = q[1] + tau * e1;
    // Conditioning of the landing: a rotation d(theta) of the ray inside the glass turns the exit ray by
    // eta c / sqrt(k) d(theta) (Snell's law differentiated), which moves the landing by L / e_z^2 per radian.
    X.gain = val(k) > 0.0 ? (g.pr.z_screen - val(q[2])) * eta * std::fabs(val(c)) /
                                (val(e2) * val(e2) * std::sqrt(val(k)))
                          : std::numeric_limits<double>::infinity();
    if (!(val(X.X) >= -g.Rxe && val(X.X) < g.Rxe && val(X.Y) >= -g.Rye && val(X.Y) < g.Rye))
        X.status = ORC_OFF_SCREEN;
    return X;
}

// Gaussian reconstruction filter (sec. 2.3):
//   f_i(x) = exp(-alpha (x - c_i)^2) - exp(-alpha (nu w / 2)^2) if |x - c_i| < nu w / 2, else 0,
//   c_i = (i + 1/2) w - R*, F_ij = f_i g_j / sum_{i',j'} f_i' g_j'.
// Reading: distances in pixel widths (alpha per pixel^2); pixel i is [i w - R*, (i+1) w - R*) (0-based);
// the sum runs over the pixels of the grid.  Window = the nu pixels centred on the landing pixel, which
// holds the whole support.  Fills idx[] with pixel indices and F[] with the normalised weights.
// With box (the simplest reconstruction of sec. 2.3) the filter of pixel i is the indicator of the pixel:
// the ray's weight goes to its landing pixel alone, and the pixel value does not move with X.
template <class S>
int filter_axis(int n, double R, double w, int nu, double alpha, const S& X, int* idx, S* F, bool box) {
    int i0 = int(std::floor((val(X) + R) / w));
    if (i0 < 0) i0 = 0;
    if (i0 > n - 1) i0 = n - 1;
    if (box) {
        idx[0] = i0;
        F[0] = S(1.0);
        return 1;
    }
    int h = (nu - 1) / 2;
    double edge = std::exp(-alpha * (0.5 * nu) * (0.5 * nu));
    S sum = 0.0;
    int cnt = 0;
    for (int a = -h; a <= h; ++a) {
        int i = i0 + a;
        if (i < 0 || i >= n) continue;
        double c = (i + 0.5) * w - R;
        S dx = (X - c) / w;
        S f = 0.0;
        if (std::fabs(val(dx)) < 0.5 * nu) f = exp(-alpha * dx * dx) - edge;
        idx[cnt] = i;
        F[cnt] = f;
        sum = sum + f;
        ++cnt;
    }
    for (int m = 0; m < cnt; ++m) F[m] = F[m] / sum;
    return cnt;
}

constexpr int MAXNU = 64;

// Splat: calls fn(pixel_index, weight) for every pixel of the window of a ray landing at (X, Y).
template <class S, class Fn>
void splat(const Geo& g, const S& X, const S& Y, const S& w, Fn fn) {
    int ix[MAXNU], iy[MAXNU];
    S Fx[MAXNU], Fy[MAXNU];
    int cx = filter_axis(g.nxe, g.Rxe, g.wx, g.pr.nu_x, g.pr.alpha, X, ix, Fx, g.pr.filter == 1);
    int cy = filter_axis(g.nye, g.Rye, g.wy, g.pr.nu_y, g.pr.alpha, Y, iy, Fy, g.pr.filter == 1);
    for (int a = 0; a < cx; ++a)
        for (int b = 0; b < cy; ++b) fn(int64_t(ix[a]) * g.nye + iy[b], w * Fx[a] * Fy[b]);
}

// ---------------------------------------------------------------------------------------------------
// One ray, values only.
// ---------------------------------------------------------------------------------------------------
struct RayOut {
    int status;
    double X, Y, w;
    double u, v, t;      // hit parameters
    int su, sv;          // hit span product
    bool marginal;
    double k;
    double gain;         // landing conditioning (mm per radian), exact-root and mesh hits
    Entry E;
    MeshHit mh;          // mesh mode: the triangle hit
};

// Rounding-distance thresholds for "marginal" rays whose discrete state may differ in single precision
// (about ten times the single-precision error of each quantity).
constexpr double EPS_APERTURE = 3e-5;  // mm, entry point to the aperture edge
constexpr double EPS_SIDE = 5e-6;      // mm, |f| at the aperture exit
constexpr double EPS_TIR = 3e-6;       // Snell discriminant k
constexpr double EPS_SCREEN = 3e-5;    // landing to the screen edge, relative to the screen radius

// force = true ignores the entry aperture and the side wall: used only to locate, for the pixel mask, where
// a marginal ray would land if single precision took the other side of such a decision.
RayOut trace_value(const Geo& g, const double* Pz, int64_t id, bool force = false) {
    RayOut R;
    R.marginal = false; R.X = R.Y = R.w = 0.0; R.u = R.v = R.t = 0.0; R.su = R.sv = 0; R.k = 1.0; R.gain = 0.0;
    R.mh = MeshHit{false, 0.0, 0, 0, 0, 0, 0};
    const bool mesh = g.pr.mesh_u > 0;
    R.E = ray_entry(g, Pz, id);
    Entry& E = R.E;
    if (std::fabs(E.margin) < EPS_APERTURE) R.marginal = true;
    if (force && E.status == ORC_MISS_ENTRY && !E.freeform) {  // continue as if the entry face were large enough
        double theta, a, ex, ey;
        sample_point(g, id, &theta, &a, &ex, &ey);
        double cphi = 1.0 - (1.0 - std::cos(g.pr.half_angle)) * a;
        double sphi = std::sqrt(std::max(0.0, 1.0 - cphi * cphi));
        double d0[3] = {std::cos(theta) * sphi, std::sin(theta) * sphi, cphi};
        double t0 = (g.pr.z_in - g.pr.pos_z) / d0[2];
        double eta = 1.0 / g.pr.n_lens, k = 1.0 - eta * eta * (1.0 - cphi * cphi);
        E.o[0] = ex + t0 * d0[0]; E.o[1] = ey + t0 * d0[1]; E.o[2] = g.pr.z_in;
        for (int i = 0; i < 3; ++i) E.d[i] = eta * d0[i] + (i == 2 ? std::sqrt(k) - eta * cphi : 0.0);
        E.w = g.w0;
        E.status = ORC_HIT;
    }
    if (E.status != ORC_HIT) { R.status = E.status; return R; }
    double q[3];
    if (E.collimated) {
        R.t = 0.0;
        q[0] = E.o[0]; q[1] = E.o[1];
        R.u = E.u; R.v = E.v;
        if (mesh) R.mh = mesh_cell_of(g, R.u, R.v);
    } else if (mesh) {
        // the first hit on the triangle mesh; a ray that meets no triangle leaves through the side wall
        R.mh = find_mesh_hit(g, Pz, E);
        if (!R.mh.hit) { R.status = ORC_SIDE_WALL; return R; }
        R.t = R.mh.t;
        q[0] = E.o[0] + R.t * E.d[0]; q[1] = E.o[1] + R.t * E.d[1];
        R.u = 0.5 * (q[0] / g.pr.r_x + 1.0); R.v = 0.5 * (q[1] / g.pr.r_y + 1.0);
    } else {
        Root rt = find_root(g, Pz, E, force);
        if (rt.margin < EPS_SIDE) R.marginal = true;
        if (rt.status != ORC_HIT) { R.status = rt.status; return R; }
        R.t = rt.t;
        q[0] = E.o[0] + rt.t * E.d[0]; q[1] = E.o[1] + rt.t * E.d[1];
        R.u = 0.5 * (q[0] / g.pr.r_x + 1.0); R.v = 0.5 * (q[1] / g.pr.r_y + 1.0);
    }
    // mesh mode: the normal is the B-spline's at the hit's (u, v), on the triangle's span product
    R.su = mesh ? R.mh.su : find_span(g.p, g.nu, R.u);
    R.sv = mesh ? R.mh.sv : find_span(g.q, g.nv, R.v);
    double Pl[MAXT];
    local_cps(g, Pz, R.su, R.sv, Pl);
    Surf<double> s = eval_surface<double>(g, Pl, R.su, R.sv, R.u, R.v, false);
    if (E.collimated) q[2] = mesh ? mesh_height<double>(g, Pl, R.mh, R.u, R.v) : s.h;
    else q[2] = E.o[2] + R.t * E.d[2];
    Exit<double> X = exit_and_screen<double>(g, q, E.d, s.hx, s.hy, E.w, false);
    R.k = X.k;
    R.gain = X.gain;
    if (std::fabs(X.k) < EPS_TIR) {
        R.marginal = true;
        if (X.status == ORC_TIR) {  // landing the ray would have had: for the mask only
            Exit<double> Y = exit_and_screen<double>(g, q, E.d, s.hx, s.hy, E.w, true);
            R.X = Y.X; R.Y = Y.Y;
        }
    }
    R.status = X.status;
    if (X.status == ORC_TIR) return R;
    R.X = X.X; R.Y = X.Y; R.w = X.w;
    if (std::fabs(g.Rxe - std::fabs(X.X)) < EPS_SCREEN * g.Rxe || std::fabs(g.Rye - std::fabs(X.Y)) < EPS_SCREEN * g.Rye)
        R.marginal = true;
    return R;
}

// ---------------------------------------------------------------------------------------------------
// One ray with dual numbers: tangents are the (p+1)(q+1) control points of the hit span product.
// Calls sink(local_cp_index, derivative) with d(sum_ij G_ij w F_ij)/dP for each local control point, or
// accumulates the image JVP when G is null.
// ---------------------------------------------------------------------------------------------------
Exit<Dual> trace_dual(const Geo& g, const double* Pz, const RayOut& R, Dual* Xo, Dual* Yo) {
    const Entry& E = R.E;
    int nt = (g.p + 1) * (g.q + 1);
    tl_nt = E.freeform ? 2 * nt : nt;
    Dual Pl[MAXT];
    for (int a = 0; a <= g.p; ++a)
        for (int b = 0; b <= g.q; ++b) {
            int l = a * (g.q + 1) + b;
            Pl[l] = Dual(Pz[(R.su - g.p + a) * g.nv + (R.sv - g.q + b)]);
            Pl[l].d[l] = 1.0;
        }
    // the ray inside the glass: fixed for a flat entry face; with a freeform entry it moves with the entry
    // net (tangents nt .. 2 nt - 1): the entry hit differentiated by Newton steps in dual arithmetic from the
    // converged root (a collimated ray meets the face at a fixed (x, y)), then the refraction and the weight
    Dual o[3], d[3], w(E.w);
    for (int i = 0; i < 3; ++i) { o[i] = Dual(E.o[i]); d[i] = Dual(E.d[i]); }
    if (E.freeform) {
        Dual Pin[MAXT];
        for (int a = 0; a <= g.p; ++a)
            for (int b = 0; b <= g.q; ++b) {
                int l = a * (g.q + 1) + b;
                Pin[l] = Dual(Pz[g.K + (E.su_in - g.p + a) * g.nv + (E.sv_in - g.q + b)]);
                Pin[l].d[nt + l] = 1.0;
            }
        Surf<Dual> si;
        if (g.pr.kind == 0) {
            Dual u(E.u), v(E.v);
            si = eval_surface<Dual>(g, Pin, E.su_in, E.sv_in, u, v, false);
            o[0] = Dual(E.s[0]); o[1] = Dual(E.s[1]); o[2] = si.h;
        } else {
            Dual t(E.t_in);
            for (int it = 0; it < 2; ++it) {
                Dual x = E.s[0] + t * E.d0[0], y = E.s[1] + t * E.d0[1];
                Dual u = 0.5 * (x / g.pr.r_x + 1.0), v = 0.5 * (y / g.pr.r_y + 1.0);
                Surf<Dual> sn = eval_surface<Dual>(g, Pin, E.su_in, E.sv_in, u, v, false);
                Dual f = sn.h - E.s[2] - t * E.d0[2];
                Dual fp = sn.hx * E.d0[0] + sn.hy * E.d0[1] - E.d0[2];
                t = t - f / fp;
            }
            for (int i = 0; i < 3; ++i) o[i] = E.s[i] + t * E.d0[i];
            Dual u = 0.5 * (o[0] / g.pr.r_x + 1.0), v = 0.5 * (o[1] / g.pr.r_y + 1.0);
            si = eval_surface<Dual>(g, Pin, E.su_in, E.sv_in, u, v, false);
        }
        Dual d0[3] = {Dual(E.d0[0]), Dual(E.d0[1]), Dual(E.d0[2])};
        Dual wfac;
        refract_in<Dual>(g, d0, si.hx, si.hy, d, &wfac);
        w = g.w0 * wfac;
    }
    Dual q[3];
    Surf<Dual> s;
    const bool mesh = g.pr.mesh_u > 0;
    if (E.collimated) {
        Dual u(R.u), v(R.v);
        s = eval_surface<Dual>(g, Pl, R.su, R.sv, u, v, false);
        q[0] = Dual(E.o[0]); q[1] = Dual(E.o[1]); q[2] = mesh ? mesh_height<Dual>(g, Pl, R.mh, u, v) : s.h;
    } else if (mesh) {
        // the plane of the hit triangle moves with its corner heights: t in dual arithmetic
        Dual t = mesh_t<Dual>(g, Pl, R.mh, E.o, E.d);
        for (int i = 0; i < 3; ++i) q[i] = E.o[i] + t * E.d[i];
        Dual u = 0.5 * (q[0] / g.pr.r_x + 1.0), v = 0.5 * (q[1] / g.pr.r_y + 1.0);
        s = eval_surface<Dual>(g, Pl, R.su, R.sv, u, v, false);
    } else {
        // Differentiate the root: two Newton steps in dual arithmetic from the converged root.
        Dual t(R.t);
        for (int it = 0; it < 2; ++it) {
            Dual x = o[0] + t * d[0], y = o[1] + t * d[1];
            Dual u = 0.5 * (x / g.pr.r_x + 1.0), v = 0.5 * (y / g.pr.r_y + 1.0);
            Surf<Dual> sn = eval_surface<Dual>(g, Pl, R.su, R.sv, u, v, false);
            Dual f = sn.h - o[2] - t * d[2];
            Dual fp = sn.hx * d[0] + sn.hy * d[1] - d[2];
            t = t - f / fp;
        }
        for (int i = 0; i < 3; ++i) q[i] = o[i] + t * d[i];
        Dual u = 0.5 * (q[0] / g.pr.r_x + 1.0), v = 0.5 * (q[1] / g.pr.r_y + 1.0);
        s = eval_surface<Dual>(g, Pl, R.su, R.sv, u, v, false);
    }
    Exit<Dual> X = exit_and_screen<Dual>(g, q, d, s.hx, s.hy, w, false);
    *Xo = X.X; *Yo = X.Y;
    return X;
}

// Control point of tangent l: the exit face's local points first, then (freeform entry) the entry face's,
// whose net follows the exit net in Pz.
int64_t cp_index(const Geo& g, const RayOut& R, int l) {
    const int nt = (g.p + 1) * (g.q + 1);
    if (l >= nt) {
        l -= nt;
        int a = l / (g.q + 1), b = l % (g.q + 1);
        return g.K + int64_t(R.E.su_in - g.p + a) * g.nv + (R.E.sv_in - g.q + b);
    }
    int a = l / (g.q + 1), b = l % (g.q + 1);
    return int64_t(R.su - g.p + a) * g.nv + (R.sv - g.q + b);
}

// ---------------------------------------------------------------------------------------------------
// Parallel loop over rays: blocks of 4096 rays, block b handled by thread b mod T (static, so results are
// summed in a fixed order and are reproducible).
// ---------------------------------------------------------------------------------------------------
template <class Fn>
void parallel_rays(int64_t n, int threads, Fn fn) {
    if (threads <= 0) threads = int(std::max(1u, std::thread::hardware_concurrency()));
    const int64_t B = 4096;
    int64_t nb = (n + B - 1) / B;
    if (threads > nb) threads = int(std::max<int64_t>(1, nb));
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t) {
        pool.emplace_back([=, &fn]() {
            for (int64_t b = t; b < nb; b += threads) {
                int64_t lo = b * B, hi = std::min(n, lo + B);
                for (int64_t id = lo; id < hi; ++id) fn(t, id);
            }
        });
    }
    for (auto& th : pool) th.join();
}

int nthreads(int t, int64_t n) {
    if (t <= 0) t = int(std::max(1u, std::thread::hardware_concurrency()));
    int64_t nb = (n + 4095) / 4096;
    return int(std::max<int64_t>(1, std::min<int64_t>(t, nb)));
}

void mark_window(const Geo& g, double X, double Y, double* mask) {
    splat<double>(g, X, Y, 1.0, [&](int64_t pix, double) { mask[pix] = 1.0; });
}

}  // namespace

// ===================================================================================================
// C ABI
// ===================================================================================================
extern "C" {

int64_t orc_num_rays(const orc_problem* pr) {
    if (!valid_problem(pr)) return -1;
    return make_geo(pr, nullptr).nrays;
}

void orc_image_size(const orc_problem* pr, int32_t* nx, int32_t* ny) {
    Geo g = make_geo(pr, nullptr);
    *nx = g.nxe; *ny = g.nye;
}

int orc_knots(int32_t p, int32_t n, double* U) {
    if (p < 1 || n <= p) return ORC_E_ARG;
    std::vector<double> k = make_knots(p, n);
    std::copy(k.begin(), k.end(), U);
    return ORC_OK;
}

int orc_basis_all(int32_t p, int32_t n, double u, int32_t der, double* out) {
    if (p < 1 || p > MAXDEG || n <= p || der < 0 || der > 2) return ORC_E_ARG;
    std::vector<double> U = make_knots(p, n);
    int s = find_span(p, n, u);
    double N[MAXDEG + 1], dN[MAXDEG + 1], d2N[MAXDEG + 1];
    basis<double>(p, U.data(), s, u, N, dN, d2N);
    for (int i = 0; i < n; ++i) out[i] = 0.0;
    const double* src = der == 0 ? N : (der == 1 ? dN : d2N);
    for (int m = 0; m <= p; ++m) out[s - p + m] = src[m];
    return ORC_OK;
}

int orc_surface(const orc_problem* pr, const double* Pz, double x, double y, double* out) {
    if (!valid_problem(pr)) return ORC_E_ARG;
    Geo g = make_geo(pr, Pz);
    Surf<double> s = surface_at(g, Pz, x, y, true);
    out[0] = s.h; out[1] = s.hx; out[2] = s.hy; out[3] = s.hxx; out[4] = s.hxy; out[5] = s.hyy;
    return ORC_OK;
}

int orc_samples(const orc_problem* pr, const int64_t* ids, int64_t n, double* out4) {
    if (!valid_problem(pr)) return ORC_E_ARG;
    Geo g = make_geo(pr, nullptr);
    for (int64_t r = 0; r < n; ++r) {
        double* o = out4 + 4 * r;
        if (pr->kind == 0) { sample_collimated(g, ids[r], &o[0], &o[1]); o[2] = o[3] = 0.0; }
        else sample_point(g, ids[r], &o[0], &o[1], &o[2], &o[3]);
    }
    return ORC_OK;
}

int orc_refract(const double* d, const double* nrm, double eta, double* out) {
    double c = d[0] * nrm[0] + d[1] * nrm[1] + d[2] * nrm[2];
    double k = 1.0 - eta * eta * (1.0 - c * c);
    if (k < 0.0) return 1;
    double sk = std::sqrt(k);
    for (int i = 0; i < 3; ++i) out[i] = eta * d[i] + (sk - eta * c) * nrm[i];
    return 0;
}

double orc_schlick(double c, double n_lens) {
    double r0 = (n_lens - 1.0) / (n_lens + 1.0);
    return schlick(c, r0 * r0);
}

int orc_splat_one(const orc_problem* pr, double X, double Y, double* img) {
    if (!valid_problem(pr)) return ORC_E_ARG;
    Geo g = make_geo(pr, nullptr);
    if (!(X >= -g.Rxe && X < g.Rxe && Y >= -g.Rye && Y < g.Rye)) return ORC_OK;
    splat<double>(g, X, Y, 1.0, [&](int64_t pix, double F) { img[pix] += F; });
    return ORC_OK;
}

int orc_trace_rays(const orc_problem* pr, const double* Pz, const int64_t* ids, int64_t n, double* out8) {
    if (!valid_problem(pr)) return ORC_E_ARG;
    Geo g = make_geo(pr, Pz);
    for (int64_t r = 0; r < n; ++r) {
        RayOut R = trace_value(g, Pz, ids[r]);
        double* o = out8 + 8 * r;
        o[0] = R.status; o[1] = R.X; o[2] = R.Y; o[3] = R.status == ORC_HIT ? R.w : 0.0;
        o[4] = R.u; o[5] = R.v; o[6] = R.t; o[7] = R.marginal ? 1.0 : 0.0;
    }
    return ORC_OK;
}

int orc_landing_gain(const orc_problem* pr, const double* Pz, const int64_t* ids, int64_t n, double* out) {
    if (!valid_problem(pr)) return ORC_E_ARG;
    Geo g = make_geo(pr, Pz);
    for (int64_t r = 0; r < n; ++r) {
        RayOut R = trace_value(g, Pz, ids[r]);
        out[r] = R.status == ORC_HIT ? R.gain : 0.0;
    }
    return ORC_OK;
}

// Where a marginal ray lands, or would land if single precision took the other side of its decision (entry
// aperture, side wall, total internal reflection); false if it would not reach the screen plane.
static bool marginal_landing(const Geo& g, const double* Pz, int64_t id, const RayOut& R, double* X, double* Y) {
    RayOut F = (R.status == ORC_MISS_ENTRY || R.status == ORC_SIDE_WALL) ? trace_value(g, Pz, id, true) : R;
    bool landed = F.status == ORC_HIT || F.status == ORC_OFF_SCREEN || (F.status == ORC_TIR && std::fabs(F.k) < EPS_TIR);
    if (!landed) return false;
    *X = std::min(std::max(F.X, -g.Rxe), std::nextafter(g.Rxe, 0.0));
    *Y = std::min(std::max(F.Y, -g.Rye), std::nextafter(g.Rye, 0.0));
    return std::isfinite(*X) && std::isfinite(*Y);
}

int orc_marginal_rays(const orc_problem* pr, const double* Pz, int64_t cap, int64_t* ids, double* xy,
                      int64_t* count, int32_t threads) {
    if (!valid_problem(pr) || !Pz || !count || (cap > 0 && (!ids || !xy))) return ORC_E_ARG;
    Geo g = make_geo(pr, Pz);
    int T = nthreads(threads, g.nrays);
    std::vector<std::vector<int64_t>> found(T);
    parallel_rays(g.nrays, T, [&](int t, int64_t id) {
        RayOut R = trace_value(g, Pz, id);
        if (R.marginal) found[t].push_back(id);
    });
    std::vector<int64_t> all;
    for (auto& f : found) all.insert(all.end(), f.begin(), f.end());
    std::sort(all.begin(), all.end());
    *count = int64_t(all.size());
    for (int64_t i = 0; i < std::min<int64_t>(cap, *count); ++i) {
        ids[i] = all[i];
        RayOut R = trace_value(g, Pz, all[i]);
        double X, Y;
        bool landed = marginal_landing(g, Pz, all[i], R, &X, &Y);
        xy[2 * i] = landed ? X : std::numeric_limits<double>::quiet_NaN();
        xy[2 * i + 1] = landed ? Y : std::numeric_limits<double>::quiet_NaN();
    }
    return ORC_OK;
}

int orc_forward(const orc_problem* pr, const double* Pz, double* irr, orc_stats* st, double* mask,
                int32_t threads) {
    if (!valid_problem(pr) || !Pz || !irr) return ORC_E_ARG;
    Geo g = make_geo(pr, Pz);
    int64_t npix = int64_t(g.nxe) * g.nye;
    int T = nthreads(threads, g.nrays);
    std::vector<std::vector<double>> img(T, std::vector<double>(npix, 0.0));
    std::vector<std::vector<double>> msk(mask ? T : 0, std::vector<double>(npix, 0.0));
    std::vector<orc_stats> sts(T);
    for (auto& s : sts) std::memset(&s, 0, sizeof(s));
    parallel_rays(g.nrays, T, [&](int t, int64_t id) {
        RayOut R = trace_value(g, Pz, id);
        orc_stats& s = sts[t];
        s.n_rays++;
        if (R.marginal) {
            s.n_marginal++;
            double X, Y;
            if (mask && marginal_landing(g, Pz, id, R, &X, &Y)) mark_window(g, X, Y, msk[t].data());
        }
        switch (R.status) {
            case ORC_HIT: s.n_hit++; break;
            case ORC_MISS_ENTRY: s.n_miss_entry++; break;
            case ORC_SIDE_WALL: s.n_side_wall++; break;
            case ORC_TIR: s.n_tir++; break;
            default: s.n_off_screen++; break;
        }
        if (R.status != ORC_HIT) return;
        s.flux_on_screen += R.w;
        double* I = img[t].data();
        splat<double>(g, R.X, R.Y, R.w, [&](int64_t pix, double v) { I[pix] += v; });
    });
    for (int64_t i = 0; i < npix; ++i) {
        double acc = 0.0;
        for (int t = 0; t < T; ++t) acc += img[t][i];
        irr[i] = acc;
        if (mask) {
            double m = 0.0;
            for (int t = 0; t < T; ++t) m = std::max(m, msk[t][i]);
            mask[i] = m;
        }
    }
    if (st) {
        std::memset(st, 0, sizeof(*st));
        for (int t = 0; t < T; ++t) {
            st->flux_on_screen += sts[t].flux_on_screen;
            st->n_rays += sts[t].n_rays; st->n_hit += sts[t].n_hit; st->n_miss_entry += sts[t].n_miss_entry;
            st->n_side_wall += sts[t].n_side_wall; st->n_tir += sts[t].n_tir;
            st->n_off_screen += sts[t].n_off_screen; st->n_marginal += sts[t].n_marginal;
        }
    }
    return ORC_OK;
}

// Loss (sec. 2.5): I_hat = I / sum I, I_ref_hat likewise, L = ||I_hat - I_ref_hat||_F / sqrt(n_x n_y).
// dL/dI_kl = (D_kl - sum_ij D_ij I_hat_ij) / (s sqrt(n_x n_y) ||D||), with D = I_hat - I_ref_hat, s = sum I;
// reading: dL/dI = 0 where ||D|| = 0.  Kind 1, the sum of squares L = ||D||_F^2, has
// dL/dI_kl = 2 (D_kl - sum_ij D_ij I_hat_ij) / s (dD_ij/dI_kl = delta / s - I_ij / s^2).
int orc_loss(int32_t nx, int32_t ny, const double* irr, const double* target, double* loss, double* dL_dI) {
    return orc_loss_kind(0, nx, ny, irr, target, loss, dL_dI);
}

int orc_loss_kind(int32_t kind, int32_t nx, int32_t ny, const double* irr, const double* target, double* loss,
                  double* dL_dI) {
    if (kind != 0 && kind != 1) return ORC_E_ARG;
    int64_t n = int64_t(nx) * ny;
    double s = 0.0, sT = 0.0;
    for (int64_t i = 0; i < n; ++i) { s += irr[i]; sT += target[i]; }
    if (!(sT > 0.0)) return ORC_E_ARG;
    if (!(s > 0.0)) return ORC_E_NOFLUX;
    double d2 = 0.0, dot = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double D = irr[i] / s - target[i] / sT;
        d2 += D * D;
        dot += D * irr[i] / s;
    }
    double nrm = std::sqrt(d2), rn = std::sqrt(double(n));
    *loss = kind == 1 ? d2 : nrm / rn;
    if (dL_dI) {
        for (int64_t i = 0; i < n; ++i) {
            double D = irr[i] / s - target[i] / sT;
            if (kind == 1) dL_dI[i] = 2.0 * (D - dot) / s;
            else dL_dI[i] = nrm > 0.0 ? (D - dot) / (s * rn * nrm) : 0.0;
        }
    }
    return ORC_OK;
}

static int grad_impl(const orc_problem* pr, const double* Pz, const double* target, double k_min,
                     double* loss, double* dL_dP, double* dL_dP_ill, double* irr_out, double* dLdI_out,
                     int32_t threads) {
    if (!valid_problem(pr) || !Pz || !target || !dL_dP) return ORC_E_ARG;
    Geo g = make_geo(pr, Pz);
    int64_t npix = int64_t(g.nxe) * g.nye;
    std::vector<double> irr(npix), G(npix);
    int rc = orc_forward(pr, Pz, irr.data(), nullptr, nullptr, threads);
    if (rc) return rc;
    double L = 0.0;
    rc = orc_loss_kind(pr->loss, g.nxe, g.nye, irr.data(), target, &L, G.data());
    if (rc) return rc;
    if (loss) *loss = L;
    if (irr_out) std::copy(irr.begin(), irr.end(), irr_out);
    if (dLdI_out) std::copy(G.begin(), G.end(), dLdI_out);
    int64_t K = int64_t(g.K) * (g.pr.entry_freeform ? 2 : 1);
    int T = nthreads(threads, g.nrays);
    std::vector<std::vector<double>> gr(T, std::vector<double>(K, 0.0));
    std::vector<std::vector<double>> gi(T, std::vector<double>(K, 0.0));
    parallel_rays(g.nrays, T, [&](int t, int64_t id) {
        RayOut R = trace_value(g, Pz, id);
        if (R.status != ORC_HIT) return;
        Dual X, Y;
        Exit<Dual> E = trace_dual(g, Pz, R, &X, &Y);
        Dual acc = 0.0;
        splat<Dual>(g, X, Y, E.w, [&](int64_t pix, const Dual& v) { acc = acc + v * G[pix]; });
        bool ill = dL_dP_ill && std::fabs(R.k) < k_min;
        double* dst = ill ? gi[t].data() : gr[t].data();
        for (int l = 0; l < tl_nt; ++l) dst[cp_index(g, R, l)] += acc.d[l];
        tl_nt = 0;
    });
    for (int64_t k = 0; k < K; ++k) {
        double a = 0.0, b = 0.0;
        for (int t = 0; t < T; ++t) { a += gr[t][k]; b += gi[t][k]; }
        dL_dP[k] = a;
        if (dL_dP_ill) dL_dP_ill[k] = b;
    }
    return ORC_OK;
}

int orc_grad(const orc_problem* pr, const double* Pz, const double* target, double* loss, double* dL_dP,
             double* irr, double* dL_dI, int32_t threads) {
    return grad_impl(pr, Pz, target, 0.0, loss, dL_dP, nullptr, irr, dL_dI, threads);
}

int orc_grad_split(const orc_problem* pr, const double* Pz, const double* target, double k_min,
                   double* loss, double* dL_dP, double* dL_dP_ill, int32_t threads) {
    return grad_impl(pr, Pz, target, k_min, loss, dL_dP, dL_dP_ill, nullptr, nullptr, threads);
}

int orc_jvp(const orc_problem* pr, const double* Pz, const double* vdir, double* dI, int32_t threads) {
    if (!valid_problem(pr) || !Pz || !vdir || !dI) return ORC_E_ARG;
    Geo g = make_geo(pr, Pz);
    int64_t npix = int64_t(g.nxe) * g.nye;
    int T = nthreads(threads, g.nrays);
    std::vector<std::vector<double>> acc(T, std::vector<double>(npix, 0.0));
    parallel_rays(g.nrays, T, [&](int t, int64_t id) {
        RayOut R = trace_value(g, Pz, id);
        if (R.status != ORC_HIT) return;
        Dual X, Y;
        Exit<Dual> E = trace_dual(g, Pz, R, &X, &Y);
        double* A = acc[t].data();
        splat<Dual>(g, X, Y, E.w, [&](int64_t pix, const Dual& v) {
            double s = 0.0;
            for (int l = 0; l < tl_nt; ++l) s += v.d[l] * vdir[cp_index(g, R, l)];
            A[pix] += s;
        });
        tl_nt = 0;
    });
    for (int64_t i = 0; i < npix; ++i) {
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += acc[t][i];
        dI[i] = s;
    }
    return ORC_OK;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// P -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
int orc_adam(int64_t n, double* P, const double* g, double* m, double* v, int64_t t, double lr,
             double beta1, double beta2, double eps) {
    if (t < 1) return ORC_E_ARG;
    double bc1 = 1.0 - std::pow(beta1, double(t)), bc2 = 1.0 - std::pow(beta2, double(t));
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        P[i] -= lr * (m[i] / bc1) / (std::sqrt(v[i] / bc2) + eps);
    }
    return ORC_OK;
}

uint64_t orc_rng(uint64_t seed, uint64_t stream, uint64_t index) { return rng_at(seed, stream, index); }

}  // extern "C"
