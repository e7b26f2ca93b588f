/*
 * FP64 CPU oracle for differentiable freeform-lens ray tracing (de Koning, Heemels, Adam, Moller,
 * "Gradient descent-based freeform optics design using algorithmic differentiable non-sequential ray
 * tracing", 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or call this library; only the
 * tests, the smoke check and the benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * constant with the HIP library: its own structs are defined here.
 *
 * Everything is plain, slow, double precision and follows the paper's steps in order:
 *   sec. 2.1      B-spline surface (Cox-de Boor recursion, clamped uniform knots, tensor product)
 *   sec. 2.1.1    linear X, Y via Greville abscissae, so only P^z is free
 *   sec. 2.2.1    collimated and point sources (uniform in solid angle), grid of point sources (sec. 3.3)
 *   sec. 2.2.2    smallest positive root of f(t) = Z(o_uv + d_uv t) - d_z t - o_z, solved exactly, or
 *                 (mesh_u > 0) the first hit on the paper's triangle mesh of the surface
 *   sec. 2.2      refraction at both faces, TIR rays dropped, Schlick weights (sec. 2.3)
 *   sec. 2.3      Gaussian reconstruction filter, normalised, optional ghost pixels
 *   sec. 2.5      normalised images and the RMS Frobenius loss; Adam
 * The gradient is the pathwise derivative computed in forward mode with dual numbers (one tangent per
 * control point of the hit span), so it is independent of any reverse-mode adjoint.
 */
#ifndef FFRT_ORACLE_H
#define FFRT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One problem: lens, source, detector, options.  Lengths in mm, angles in radians. */
typedef struct {
    /* lens (sec. 2.1, 2.1.1, 2.1.2) */
    double n_lens, r_x, r_y, z_in, delta_min;
    int32_t p, q, n_u, n_v;          /* degrees and control-net size (n_u = n_1 + 1, n_v = n_2 + 1) */
    /* source (sec. 2.2.1, sec. 3.3) */
    int32_t kind;                    /* 0 collimated grid, 1 point source, 2 grid of point sources */
    int32_t grid_u, grid_v;          /* collimated: rays per axis; point: strata in (theta, a) */
    int32_t jitter;                  /* 0 cell-centred samples, 1 jittered within each cell/stratum */
    double pos_x, pos_y, pos_z;      /* point source (or emitter-grid centre) */
    double half_angle;               /* cone half angle phi_max */
    int32_t emit_nx, emit_ny;        /* kind 2: emitters per axis */
    double emit_wx, emit_wy;         /* kind 2: emitter-grid extent (endpoints included) */
    uint64_t seed;
    /* detector (sec. 2.3) */
    int32_t n_x, n_y;
    double R_x, R_y, z_screen, alpha;  /* alpha in units of (pixel width)^-2 */
    int32_t nu_x, nu_y, ghost;
    /* options */
    int32_t fresnel;                 /* 1: Schlick weights at both faces, 0: none */
    int32_t mesh_u, mesh_v;          /* 0: exact intersection; >= 1: the triangle mesh of sec. 2.2.2 with
                                        mesh_u x mesh_v rectangles per knot span product */
    int32_t filter;                  /* 0: Gaussian reconstruction filter, 1: box (indicator of the pixel) */
    int32_t entry_freeform;          /* 1: the entry face is a second B-spline (net after the exit's in Pz) */
    int32_t loss;                    /* 0: the RMS loss of sec. 2.5; 1: its sum of squares */
} orc_problem;

typedef struct {
    double flux_on_screen;           /* sum of final weights of accepted rays */
    int64_t n_rays, n_hit, n_miss_entry, n_side_wall, n_tir, n_off_screen, n_marginal;
} orc_stats;

/* Ray status codes. */
enum { ORC_HIT = 0, ORC_MISS_ENTRY = 1, ORC_SIDE_WALL = 2, ORC_TIR = 3, ORC_OFF_SCREEN = 4 };

/* Return codes. */
enum { ORC_OK = 0, ORC_E_ARG = 1, ORC_E_NOFLUX = 3 };

/* Total number of rays of the problem. */
int64_t orc_num_rays(const orc_problem* pr);

/* Effective image size (ghost pixels included when enabled). */
void orc_image_size(const orc_problem* pr, int32_t* nx, int32_t* ny);

/* Clamped uniform knot vector, length n + p + 1 (sec. 2.1). */
int orc_knots(int32_t p, int32_t n, double* U);

/* All n basis functions N_{i,p}(u) (der = 0) or their first / second u-derivatives (der = 1, 2). */
int orc_basis_all(int32_t p, int32_t n, double u, int32_t der, double* out);

/* Surface height field h(x, y) and its x/y derivatives: out = {h, h_x, h_y, h_xx, h_xy, h_yy}. */
int orc_surface(const orc_problem* pr, const double* Pz, double x, double y, double* out);

/* Ray samples: kind 0 -> (u, v, 0, 0); kinds 1/2 -> (theta, a, emitter x, emitter y), per ray id. */
int orc_samples(const orc_problem* pr, const int64_t* ids, int64_t n, double* out4);

/* Vector Snell refraction of unit d at unit normal nrm (pointing to the transmitted side), ratio eta =
 * n_incident / n_transmitted.  Returns 1 on total internal reflection (out untouched), else 0. */
int orc_refract(const double* d, const double* nrm, double eta, double* out);

/* Schlick reflectance for cosine c (taken on the air side) and index n. */
double orc_schlick(double c, double n_lens);

/* Splat one unit-weight ray landing at (X, Y) into a zeroed image of the effective size. */
int orc_splat_one(const orc_problem* pr, double X, double Y, double* img);

/* Trace the given rays.  out8 per ray: {status, X, Y, w, u_hit, v_hit, t_hit, marginal}. */
int orc_trace_rays(const orc_problem* pr, const double* Pz, const int64_t* ids, int64_t n, double* out8);

/* Conditioning of each ray's landing: the displacement (mm) of the landing point per radian of rotation of
 * the ray inside the glass (0 for rays that do not land). */
int orc_landing_gain(const orc_problem* pr, const double* Pz, const int64_t* ids, int64_t n, double* out);

/* The rays whose discrete state (status) is within rounding distance of flipping ("marginal"), in id order:
 * their number in *count, the first min(cap, count) ids, and where each lands or would land on the other side
 * of its decision (xy, NaN if nowhere on the screen plane). */
int orc_marginal_rays(const orc_problem* pr, const double* Pz, int64_t cap, int64_t* ids, double* xy,
                      int64_t* count, int32_t threads);

/* Irradiance image (row-major [n_x][n_y], i along x).  mask (optional): pixels touched by rays whose
 * discrete state is within rounding distance of flipping are set to 1.  threads <= 0 means all cores. */
int orc_forward(const orc_problem* pr, const double* Pz, double* irr, orc_stats* st, double* mask,
                int32_t threads);

/* Loss of sec. 2.5 and dL/dI.  Returns ORC_E_NOFLUX if sum(I) = 0. */
int orc_loss(int32_t nx, int32_t ny, const double* irr, const double* target, double* loss, double* dL_dI);
/* The same for loss kind 0 (the RMS loss of sec. 2.5) or 1 (its sum of squares, ||I_hat - T_hat||_F^2). */
int orc_loss_kind(int32_t kind, int32_t nx, int32_t ny, const double* irr, const double* target, double* loss,
                  double* dL_dI);

/* Forward, loss, and the pathwise gradient dL/dP^z (row-major [n_u][n_v]).  irr and dL_dI optional. */
int orc_grad(const orc_problem* pr, const double* Pz, const double* target, double* loss, double* dL_dP,
             double* irr, double* dL_dI, int32_t threads);

/* Same as orc_grad but only rays whose landing is well conditioned enter dL_dP; the ill-conditioned
 * remainder (rays close to TIR) is written to dL_dP_ill.  The sum of the two is orc_grad's dL_dP. */
int orc_grad_split(const orc_problem* pr, const double* Pz, const double* target, double k_min,
                   double* loss, double* dL_dP, double* dL_dP_ill, int32_t threads);

/* Directional derivative of the image: dI = sum_k v_k dI/dP_k (forward mode). */
int orc_jvp(const orc_problem* pr, const double* Pz, const double* v, double* dI, int32_t threads);

/* One Adam step (Kingma & Ba) in place; t is the new step count (>= 1). */
int orc_adam(int64_t n, double* P, const double* g, double* m, double* v, int64_t t, double lr,
             double beta1, double beta2, double eps);

/* The counter-based SplitMix64 output used for ray sampling (seed, stream, index). */
uint64_t orc_rng(uint64_t seed, uint64_t stream, uint64_t index);

#ifdef __cplusplus
}
#endif
#endif
