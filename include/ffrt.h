/*
 * ffrt - differentiable freeform-lens ray tracing on AMD Instinct MI355X (gfx950).
 *
 * The calls follow the design problem of de Koning, Heemels, Adam, Moller (2023), "Gradient descent-based
 * freeform optics design using algorithmic differentiable non-sequential ray tracing":
 *   sec. 2 (problem)          min over P of L(P; I_ref), solved by gradient descent
 *   sec. 2.1, 2.1.1, 2.1.2    plano-freeform lens: flat entry face z = z_in, exit face a clamped uniform
 *                             B-spline height field; X, Y linear (Greville), only P^z free; P^z >= z_in + delta
 *   sec. 2.2.1                collimated bundle, point source uniform in solid angle; sec. 3.3 grid of
 *                             point sources approximating an extended source
 *   sec. 2.2, 2.2.2           smallest positive root of the ray/height-field equation; refraction at both
 *                             faces; total internal reflection dropped
 *   sec. 2.3                  detector grid, Schlick weights, normalised Gaussian reconstruction filter,
 *                             optional ghost pixels
 *   sec. 2.5                  normalised images, RMS Frobenius loss, Adam on the control points
 *
 * Conventions for every call:
 *  - Lengths in mm, angles in radians.  Device arrays are float32 unless stated.
 *  - The caller owns every buffer.  A plan holds host metadata only; its device workspace is caller
 *    allocated (ffrt_plan_workspace_size) and handed over once (ffrt_plan_set_workspace).  The compute
 *    calls never allocate.  Calls on one plan share that workspace (bounds, loss partial sums and their
 *    arrival counters), so they must not overlap in time: issue them on one stream, or order the streams.
 *  - A plan holds one or more designs.  Their buffers are packed back to back at the offsets given by
 *    ffrt_plan_layout: control points P^z[i][j] row-major with i along u / x (sec. 2.1); images I[i][j]
 *    row-major with i along x (sec. 2.3).  Ghost pixels, when enabled, enlarge the stored image.
 *  - Compute calls are asynchronous on the given HIP stream (hipStream_t passed as void*, NULL = default
 *    stream).  Argument and shape errors are reported at plan creation or by the call's return code;
 *    data-dependent conditions (constraint violation, no flux, NaN, Newton non-convergence) are counted on
 *    the device in ffrt_stats.  Nothing crosses the ABI as an exception.
 *  - ffrt_last_error() returns a thread-local message for the last failing call.
 */
#ifndef FFRT_H
#define FFRT_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FFRT_OK = 0,
    FFRT_E_ARG = 1,          /* invalid argument or shape */
    FFRT_E_CONSTRAINT = 2,   /* lens constraint violated (host-side check of given values) */
    FFRT_E_NOFLUX = 3,       /* no ray reached the screen */
    FFRT_E_HIP = 4,          /* HIP runtime error (message in ffrt_last_error) */
    FFRT_E_OOM = 5,          /* workspace too small */
    FFRT_E_UNSUPPORTED = 6,  /* valid but not compiled for (degree / filter-size combination) */
    FFRT_E_STATE = 7         /* call order (e.g. no workspace set, no graph captured) */
} ffrt_status;

/* Lens (sec. 2.1 - 2.1.2).  n_u = n_1 + 1 and n_v = n_2 + 1 control points, degrees p, q.  The aperture is
 * [-r_x, r_x] x [-r_y, r_y]; the flat entry face is z = z_in; delta_min is the minimal thickness used by
 * the constraint count (P^z >= z_in + delta_min).  A face holds at most 4096 control points and 64 knot spans
 * along each axis (n_u - p <= 64, n_v - q <= 64); ffrt_plan_create returns FFRT_E_ARG beyond that.
 * entry_freeform = 1 makes the entry face a second B-spline height field on the same knots (the paper's
 * proposal for extended sources, sec. 3.3 and the conclusion): the design's control heights are then
 * 2 n_u n_v floats, the exit net followed by the entry net, and both are optimised.  Point-source rays meet
 * the entry face at its smallest root over the aperture (else they miss the lens), collimated rays at their
 * sampled (x, y); both faces refract with Schlick weights; the thickness check becomes
 * P_exit - P_entry >= delta_min per control point.  At most 2048 control points per face; not combined
 * with the triangle mesh; the sparse generator does not apply. */
typedef struct {
    double n_lens, r_x, r_y, z_in, delta_min;
    int32_t p, q, n_u, n_v;
    int32_t entry_freeform;  /* 0 or 1 */
    int32_t reserved;        /* 0 */
} ffrt_lens;

/* Source (sec. 2.2.1, sec. 3.3).
 * kind 0: collimated bundle along +z sampled on a grid_u x grid_v grid of [0,1]^2 directly on the
 *         freeform; ray id = k_u * grid_v + k_v.
 * kind 1: point source at pos, cone half angle half_angle; (theta, a) stratified grid_u x grid_v;
 *         ray id = k_theta * grid_v + k_a.
 * kind 2: emit_nx x emit_ny point sources evenly spaced (endpoints included) over emit_wx x emit_wy around
 *         pos, each sampled as kind 1; ray id = e * grid_u * grid_v + (per-emitter id), e = ix * emit_ny + iy.
 * jitter 0 places samples at cell centres; 1 jitters them with 24-bit uniforms from a counter-based
 * SplitMix64 keyed by (seed, stream 2, ray id). */
typedef struct {
    int32_t kind, grid_u, grid_v, jitter;
    double pos[3];
    double half_angle;
    int32_t emit_nx, emit_ny;
    double emit_wx, emit_wy;
    uint64_t seed;
} ffrt_source;

/* Detector (sec. 2.3): n_x x n_y pixels on [-R_x, R_x) x [-R_y, R_y) at z = z_screen.  Filter
 * f(x) = exp(-alpha ((x - c)/w)^2) - exp(-alpha (nu/2)^2) inside nu pixels (alpha per pixel width^2),
 * normalised over the grid.  ghost = 1 adds (nu-1)/2 ghost pixels on each side.  filter = 1 selects box
 * reconstruction instead (the pixel's indicator: a ray's weight goes to its landing pixel; the image then
 * has no derivative in the landing position, only through the Fresnel weights). */
typedef struct {
    int32_t n_x, n_y;
    double R_x, R_y, z_screen, alpha;
    int32_t nu_x, nu_y, ghost, filter;
} ffrt_detector;

/* fresnel: 1 applies Schlick's approximation at both faces (cosine taken on the air side), 0 does not.
 * loss: 0 the paper's loss of sec. 2.5, L = ||I/sum I - T/sum T||_F / sqrt(n_x n_y) (RMS Frobenius norm of the
 * difference of the normalised images); 1 its sum of squares, L = ||I/sum I - T/sum T||_F^2.
 * newton_max_iter: iteration cap of the freeform intersection (point sources), 1..32.
 * mesh_u, mesh_v: 0 (both) intersects the B-spline itself; 1..64 (both) intersects the paper's triangle
 * mesh instead (sec. 2.2.2): every knot span product divided into mesh_u x mesh_v equal rectangles, each
 * split into a lower-left and an upper-right triangle with corners on the surface.  The hit lies on the
 * mesh; the refraction uses the B-spline's normal at the hit, and the gradient follows the triangle's
 * corner heights. */
typedef struct {
    int32_t fresnel, newton_max_iter;
    int32_t mesh_u, mesh_v;
    int32_t loss;            /* 0 RMS (the paper's), 1 sum of squares */
    int32_t reserved;        /* 0 */
} ffrt_options;

typedef struct {
    ffrt_lens lens;
    ffrt_source src;
    ffrt_detector det;
    ffrt_options opt;
} ffrt_problem;

typedef struct ffrt_plan ffrt_plan;

/* Per-design counters written by ffrt_forward (device memory, one per design, zeroed by the call). */
typedef struct {
    float flux_on_screen;         /* sum of final weights of accepted rays (initial weight 1/N) */
    uint32_t n_traced, n_hit, n_miss_entry, n_side_wall, n_tir, n_off_screen;
    uint32_t n_newton_fail;       /* roots not converged within newton_max_iter */
    uint32_t n_fp64_refined;      /* grazing hits whose residual was re-checked in double precision */
    uint32_t n_nonmonotone;       /* rays whose root needed the bracket scan */
    uint32_t n_search_steps;      /* Newton iterations (exact root) or mesh cells visited, summed over rays */
    uint32_t n_constraint_viol;   /* control points below z_in + delta_min (sec. 2.1.2) */
    uint32_t n_nan;               /* non-finite control points */
} ffrt_stats;

typedef struct {
    float lr, beta1, beta2, eps;
} ffrt_adam_hparams;

/* ---- plan ------------------------------------------------------------------------------------------ */

/* Validate n_designs problems and build a plan (host only, no HIP call).  All designs of a plan share the
 * degrees (p, q) and filter sizes (nu_x, nu_y).  Supported: p, q in {2,3,5} pairs (3,3), (5,3), (2,2) and
 * nu in {3, 5, 11} with nu_x = nu_y; other valid values return FFRT_E_UNSUPPORTED.  Returns FFRT_E_ARG
 * with a message for invalid problems. */
ffrt_status ffrt_plan_create(const ffrt_problem* probs, int32_t n_designs, ffrt_plan** out);
ffrt_status ffrt_plan_destroy(ffrt_plan* plan);

/* Device workspace bytes the plan needs: design descriptors, knot tables, bounds, loss flags and partial
 * sums, a dL/dI buffer for steps, and the accumulators of the trace kernels (a 64-bit fixed-point
 * irradiance image and a gradient buffer, each kept at zero between calls).  When the rays of the point and
 * emitter-grid designs with the exact root and a flat entry face number at most 2^28 (1 GiB at 4 bytes per
 * ray), the workspace also holds their exit roots for the adjoint of a step (see ffrt_step). */
ffrt_status ffrt_plan_workspace_size(const ffrt_plan* plan, size_t* bytes);

/* Hand over caller-allocated device workspace (>= the size above, 256-byte aligned) on the current
 * device; uploads the plan's descriptors with a synchronous copy.  Must precede every compute call. */
ffrt_status ffrt_plan_set_workspace(ffrt_plan* plan, void* dev_ptr, size_t bytes);

/* Packed layout: cp_offsets[n_designs + 1] and img_offsets[n_designs + 1] (prefix sums, in elements);
 * either may be NULL. */
ffrt_status ffrt_plan_layout(const ffrt_plan* plan, int64_t* cp_offsets, int64_t* img_offsets);
ffrt_status ffrt_plan_num_designs(const ffrt_plan* plan, int32_t* n);
ffrt_status ffrt_plan_num_rays(const ffrt_plan* plan, int64_t* n);

/* ---- the hot path ---------------------------------------------------------------------------------- */

/* Irradiance of every design (sec. 2.3): traces all rays and splats them; irr and stats are overwritten.
 * Pz: packed control heights; irr: packed images (output); stats: n_designs ffrt_stats or NULL.  Pixel
 * sums are accumulated in 64-bit fixed point (unit 2^-26 w0, w0 = 1 / rays of the design), so the result
 * does not depend on the order in which rays are added. */
ffrt_status ffrt_forward(ffrt_plan* plan, const float* Pz, float* irr, ffrt_stats* stats, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): ffrt_forward without a caller workspace.  The plan need not have one
 * set (ffrt_plan_create makes no HIP call).  Its descriptor tables, the bounds, the statistics slots and the
 * fixed-point image live instead in a device array the library holds per GPU from module load until the
 * process ends: 32 MiB, so the call returns FFRT_E_OOM, with the size it needs in ffrt_last_error(), for a
 * plan whose images, control nets and tables do not fit (about 32 designs of 256 x 256 pixels).  Each call
 * copies the plan's host tables into the array with hipMemcpyAsync on `stream` and clears the slots and the
 * image with a kernel; it calls no allocating routine.  Every call on one GPU shares that array, whatever
 * the plan or stream: calls that overlap in time on one GPU race, so issue them on one stream or order them.
 * Results are those of ffrt_forward, bit for bit. */
ffrt_status ffrt_forward_static(ffrt_plan* plan, const float* Pz, float* irr, ffrt_stats* stats, void* stream);

/* Loss of sec. 2.5 per design and dL/dI.  loss: n_designs floats (NaN for a design without flux, whose
 * dL/dI is then zero and whose next Adam update is skipped); dL_dI: packed like irr. */
ffrt_status ffrt_loss(ffrt_plan* plan, const float* irr, const float* target, float* loss, float* dL_dI,
                      void* stream);

/* Loss value per design (n_designs doubles, device) with every reduction in double precision, no dL/dI.
 * For finite-difference gradients: a central difference over h = 1e-4 mm changes the loss by ~1e-5 of
 * itself, below what single-precision sums resolve.  Not used by the optimisation step. */
ffrt_status ffrt_loss_f64(ffrt_plan* plan, const float* irr, const float* target, double* loss, void* stream);

/* Pathwise gradient dL/dP^z (packed like Pz) of sum_ij dL_dI_ij I_ij: re-traces every ray (nothing per ray
 * is taken from an earlier call) and back-propagates through splat, screen, refraction and the root (implicit function
 * theorem).  dL_dP is overwritten. */
ffrt_status ffrt_adjoint(ffrt_plan* plan, const float* Pz, const float* dL_dI, float* dL_dP, void* stream);

/* Adam on P^z in place (Kingma & Ba; bias-corrected).  m, v: packed like Pz; t: n_designs step counters
 * in device memory, incremented by the call.  A design whose last ffrt_loss found no flux is skipped. */
ffrt_status ffrt_adam(ffrt_plan* plan, float* Pz, const float* dL_dP, float* m, float* v, int32_t* t,
                      const ffrt_adam_hparams* hp, void* stream);

/* One optimisation step: forward, loss, adjoint, Adam (all device-side, no host synchronisation).  irr,
 * loss, dL_dI, dL_dP and stats (if not NULL) receive the step's values before the update; Pz, m, v, t are
 * updated.  dL_dI may be NULL, in which case dL/dI is kept in the plan's workspace.  The forward keeps the
 * exit root of every point-source ray (exact root, flat entry face; when the workspace holds them) and the
 * adjoint of the same step starts from it instead of repeating the search of sec. 2.2.1. */
ffrt_status ffrt_step(ffrt_plan* plan, float* Pz, const float* target, float* irr, float* loss,
                      float* dL_dI, float* dL_dP, float* m, float* v, int32_t* t, ffrt_stats* stats,
                      const ffrt_adam_hparams* hp, void* stream);

/* Capture `steps` consecutive ffrt_step calls into a HIP graph owned by the plan (stream must not be the
 * NULL stream; dL_dI may be NULL as for ffrt_step).  The arguments are bound at capture.
 * ffrt_graph_launch replays it on `stream`. */
ffrt_status ffrt_graph_capture(ffrt_plan* plan, int32_t steps, float* Pz, const float* target, float* irr,
                               float* loss, float* dL_dI, float* dL_dP, float* m, float* v, int32_t* t,
                               ffrt_stats* stats, const ffrt_adam_hparams* hp, void* stream);
ffrt_status ffrt_graph_launch(ffrt_plan* plan, void* stream);

/* ---- range reparametrisation of the control heights (sec. 2.4.1, eq. of the output correction) ------ */
/* The paper optimises, per control point, a variable theta mapped through tanh onto an allowed range,
 * optionally offset by a function f of the control point's (x, y):  P^z = lo + (tanh(theta) + 1) span / 2,
 * with lo = z_min (+ f(P^x, P^y)) and span = z_max - z_min >= 0 (both may vary per control point).  theta,
 * lo, span, Pz, dL_dP, dL_dtheta: device float32, packed like Pz.  NULL buffers give FFRT_E_ARG. */
ffrt_status ffrt_reparam_apply(ffrt_plan* plan, const float* theta, const float* lo, const float* span, float* Pz,
                               void* stream);
/* dL_dtheta = dL_dP (1 - tanh^2(theta)) span / 2. */
ffrt_status ffrt_reparam_grad(ffrt_plan* plan, const float* theta, const float* span, const float* dL_dP,
                              float* dL_dtheta, void* stream);
/* One optimisation step on theta: as ffrt_step, with Adam (m, v, t) acting on theta through the chain rule
 * above; Pz must hold P(theta) on entry (ffrt_reparam_apply) and holds P of the updated theta on return.
 * dL_dP receives the gradient with respect to P^z. */
ffrt_status ffrt_step_reparam(ffrt_plan* plan, float* theta, const float* lo, const float* span, float* Pz,
                              const float* target, float* irr, float* loss, float* dL_dI, float* dL_dP, float* m,
                              float* v, int32_t* t, ffrt_stats* stats, const ffrt_adam_hparams* hp, void* stream);
/* ffrt_graph_capture for ffrt_step_reparam (replayed with ffrt_graph_launch). */
ffrt_status ffrt_graph_capture_reparam(ffrt_plan* plan, int32_t steps, float* theta, const float* lo,
                                       const float* span, float* Pz, const float* target, float* irr, float* loss,
                                       float* dL_dI, float* dL_dP, float* m, float* v, int32_t* t, ffrt_stats* stats,
                                       const ffrt_adam_hparams* hp, void* stream);
/* Host-side (x, y) of every control point, packed like Pz (host float64 arrays): the Greville positions
 * P^x_ij = (2 u*_i - 1) r_x, P^y_ij = (2 v*_j - 1) r_y of sec. 2.1.1, at which an offset function f is
 * evaluated. */
ffrt_status ffrt_plan_control_xy(const ffrt_plan* plan, double* x, double* y);

/* ---- control-point generators (sec. 2.4) ----------------------------------------------------------- */
/* Multi-layer perceptrons with the trivial input 1 and three tanh layers, each of the size K = n_u n_v of a
 * design's control net (k = i n_v + j, as in Pz), whose output y passes through the output correction above:
 *   h1 = tanh(w1 + b1),  h2 = tanh(W2 h1 + b2),  y = tanh(W3 h2 + b3),  P^z = lo + (y + 1) span / 2.
 * arch selects how W2 and W3 connect:
 *   FFRT_MLP_DENSE: fully connected; design d's parameters, packed: w1 (K), b1 (K), W2 (K x K, row-major: row i
 *     holds the input weights of neuron i), b2 (K), W3 (K x K), b3 (K): 2 K^2 + 4 K floats.  K <= 16384.
 *   FFRT_MLP_SPARSE: locally connected with the footprint of a (2p+1) x (2q+1) convolution (the control points
 *     whose basis functions share a knot span), a weight per connection and a bias per neuron.  Neuron (i, j)
 *     takes the layer input at (i + a - p, j + b - q), a in [0, 2p], b in [0, 2q]; packed: w1 (K), b1 (K),
 *     W2 (C x K: W2[c][k], c = a (2q + 1) + b), b2 (K), W3 (C x K), b3 (K), C = (2p+1)(2q+1): 2 C K + 4 K floats.
 *     A connection that would leave the net does not exist: its stored weight gets zero gradient.  K <= 6144.
 * params: device float32; design d's parameters start at offsets[d] (ffrt_mlp_layout); offsets[n_designs] is
 * the total.  acts: device float32 of 3 x (total control points), design d's h1, h2, y (K each) at 3 x its
 * control-point offset; written by ffrt_mlp_forward, read by the backward pass.  lo, span, Pz, dL_dP: packed
 * like Pz.  NULL buffers, an unknown arch or a control net above the limit give FFRT_E_ARG. */
#define FFRT_MLP_DENSE 0
#define FFRT_MLP_SPARSE 1
/* Host int64 offsets[n_designs + 1] of each design's parameters in params. */
ffrt_status ffrt_mlp_layout(const ffrt_plan* plan, int32_t arch, int64_t* offsets);
/* Forward pass: writes acts and Pz. */
ffrt_status ffrt_mlp_forward(ffrt_plan* plan, int32_t arch, const float* params, const float* lo, const float* span,
                             float* acts, float* Pz, void* stream);
/* Back-propagation of dL_dP (e.g. from ffrt_adjoint) through the output correction and the three layers:
 * grad (device float32, laid out like params) receives dL/d(params).  acts must come from ffrt_mlp_forward
 * on the same params.  Uses the plan's workspace. */
ffrt_status ffrt_mlp_backward(ffrt_plan* plan, int32_t arch, const float* params, const float* acts,
                              const float* span, const float* dL_dP, float* grad, void* stream);
/* One optimisation step of the generator: as ffrt_step, with Adam acting on params (m, v laid out like
 * params; t: one counter per design).  On entry acts and Pz must hold ffrt_mlp_forward of params; on return
 * they hold it for the updated params.  dL_dP receives the gradient with respect to P^z.  A design whose
 * loss found no flux keeps its params and counter. */
ffrt_status ffrt_step_mlp(ffrt_plan* plan, int32_t arch, float* params, float* m, float* v, int32_t* t,
                          const float* lo, const float* span, float* acts, float* Pz, const float* target, float* irr,
                          float* loss, float* dL_dI, float* dL_dP, ffrt_stats* stats, const ffrt_adam_hparams* hp,
                          void* stream);
/* ffrt_graph_capture for ffrt_step_mlp (replayed with ffrt_graph_launch). */
ffrt_status ffrt_graph_capture_mlp(ffrt_plan* plan, int32_t arch, int32_t steps, float* params, float* m, float* v,
                                   int32_t* t, const float* lo, const float* span, float* acts, float* Pz,
                                   const float* target, float* irr, float* loss, float* dL_dI, float* dL_dP,
                                   ffrt_stats* stats, const ffrt_adam_hparams* hp, void* stream);

/* ---- kernel shapes (autotuner) ------------------------------------------------------------------- */

/* Number of candidate shapes for the forward (which = 0) or adjoint (which = 1) kernel, and selection. */
ffrt_status ffrt_num_configs(int32_t which, int32_t* n);
ffrt_status ffrt_config_name(int32_t which, int32_t index, char* buf, int32_t buflen);
ffrt_status ffrt_plan_set_config(ffrt_plan* plan, int32_t which, int32_t index);
ffrt_status ffrt_plan_get_config(const ffrt_plan* plan, int32_t which, int32_t* index);

/* Mean duration (ms) of the forward and the adjoint trace kernel alone, each launched `reps` times back to
 * back between two HIP events recorded on `stream` with the plan's current shapes (the zeroing and bounds
 * kernels of the full calls run once before), as a step launches them (the adjoint reusing the exit roots).  Synchronises the stream.  irr and dL_dP are overwritten
 * (they accumulate over the repetitions). */
ffrt_status ffrt_plan_time_kernels(ffrt_plan* plan, const float* Pz, float* irr, const float* dL_dI,
                                   float* dL_dP, int32_t reps, float* fwd_ms, float* adj_ms, void* stream);

/* Time every candidate shape on the caller's buffers (reps launches each, HIP events, synchronises the
 * stream; the adjoint as a step launches it) and keep the fastest for each kernel.  irr and dL_dP are overwritten. */
ffrt_status ffrt_plan_autotune(ffrt_plan* plan, const float* Pz, float* irr, const float* dL_dI,
                               float* dL_dP, int32_t reps, void* stream);

/* Mean duration (ms) of the generator's forward pass, its back-propagation to the layer vectors, and its
 * gradient + Adam update, each launched `reps` times back to back between HIP events on `stream`
 * after one untimed pass.  params, m and v are updated reps + 1 times (pass copies); acts and Pz are
 * overwritten; t is read only.  Synchronises the stream. */
ffrt_status ffrt_plan_time_mlp(ffrt_plan* plan, int32_t arch, float* params, float* m, float* v, const int32_t* t,
                               const float* lo, const float* span, float* acts, float* Pz, const float* dL_dP,
                               const ffrt_adam_hparams* hp, int32_t reps, float* fwd_ms, float* bwd_ms,
                               float* upd_ms, void* stream);

/* ---- inspection ------------------------------------------------------------------------------------ */

/* Trace individual rays of one design.  ray_ids: n int64 (device); out8: n x 8 floats (device) =
 * {status, X, Y, w, u_hit, v_hit, t_hit, newton_iterations}; status 0 hit, 1 missed the entry face,
 * 2 left through the side wall, 3 TIR, 4 off screen. */
ffrt_status ffrt_trace_rays(ffrt_plan* plan, int32_t design, const float* Pz, const int64_t* ray_ids,
                            int64_t n, float* out8, void* stream);

/* Throughput of LDS atomic adds (ds_add_u32, workgroup scope) on the current device, in atomics per second
 * over the whole chip: 8 workgroups of 256 threads per compute unit each add 256 rounds of 9 values to a
 * tile of their own, launched reps times after one untimed launch (HIP events on `stream`, synchronised).
 * pattern 0: distinct addresses in distinct banks (the unit's peak); pattern 1: the forward's splat (an
 * 8 x 8 lane grid of rays two pixels apart, each adding its 3 x 3 filter window).  Allocates and frees a
 * small device buffer (hipMalloc), so it is not for graph capture.  A measurement aid for the roofline of the splat, not part of the method. */
ffrt_status ffrt_lds_atomic_rate(int32_t pattern, int32_t reps, double* atomics_per_s, void* stream);

/* The ray-sampling random numbers: out[i] = SplitMix64 output for (seed, stream, first + i) (device). */
ffrt_status ffrt_rng(uint64_t seed, uint64_t stream_id, uint64_t first, int64_t n, uint64_t* out,
                     void* stream);

const char* ffrt_status_string(ffrt_status s);
const char* ffrt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
