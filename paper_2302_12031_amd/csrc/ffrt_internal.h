// Internal descriptors shared by the host runtime and the gfx950 kernels of libffrt.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ffrt.h"

namespace ffrt {

constexpr int WG = 256;               // threads per workgroup: 4 wave64s
constexpr int TILE_CAP = 6144;        // 32-bit fixed-point pixels in the LDS irradiance tile of the forward kernel
constexpr int MAX_DEG = 5;
constexpr int MAX_CP = 4096;          // control points of one face (the net is at most 64 x 64)
constexpr int N_SHAPES = 5;           // block shapes: rays per thread 1, 2, 4, 8, 16
constexpr int N_KG = 8;               // kernel groups: bit 0 point source, bit 1 mesh, bit 2 freeform entry
constexpr int RPT_OF_SHAPE[N_SHAPES] = {1, 2, 4, 8, 16};
constexpr int NSLOT = 64;             // per-design partial-statistics slots (spreads the counter atomics)
constexpr size_t ROOTS_CAP = size_t(1) << 30;  // bytes of the per-ray exit-root buffer of a plan, at most
constexpr size_t STATIC_SCRATCH_BYTES = size_t(32) << 20;  // library-owned device array per GPU (ffrt_forward_static)

// Ray status codes (same meaning as the public ffrt_trace_rays status).
enum : int { ST_HIT = 0, ST_MISS_ENTRY = 1, ST_SIDE_WALL = 2, ST_TIR = 3, ST_OFF_SCREEN = 4 };

// Block shapes: every thread traces an MU x MV patch of adjacent samples (RPT = MU MV rays), a wave covers
// 8 x 8 such patches and a workgroup 2 x 2 waves, so a block is (16 MU) x (16 MV) samples.
__host__ __device__ constexpr int shape_mu(int s) { return s <= 1 ? 1 : (s <= 3 ? 2 : 4); }
__host__ __device__ constexpr int shape_mv(int s) { return s == 0 ? 1 : (s <= 2 ? 2 : 4); }

// Per-axis knot table stride (floats) for degree p: 2p local knots + p(p+1)/2 reciprocals, padded to 4.
__host__ __device__ constexpr int kt_stride(int p) { return ((2 * p + p * (p + 1) / 2) + 3) / 4 * 4; }

// One design, as the kernels see it (all float32 except layout and seed).
struct DesignDev {
    // lens
    float r_x, r_y, z_in, n_lens;
    float sxu, syv;          // d(ubar)/dx = (n_u - p) / (2 r_x), d(vbar)/dy: knot units per mm
    float ubar0, vbar0;      // ubar at x = 0: (n_u - p) / 2
    int32_t n_u, n_v, nsu, nsv;     // control points and knot spans per axis
    float zmin_allowed;      // z_in + delta_min
    // source
    int32_t kind, grid_u, grid_v, jitter;
    float pos_x, pos_y, pos_z, omc;  // omc = 1 - cos(phi_max)
    int32_t emit_nx, emit_ny;
    float ex0, edx, ey0, edy;        // emitter grid: pos + (ex0 + ix * edx, ey0 + iy * edy)
    float inv_gu, inv_gv;            // 1 / grid_u, 1 / grid_v
    uint64_t rng_state0;             // SplitMix64 state for (seed, stream 2)
    // detector (effective grid, ghost pixels included)
    int32_t nx, ny;
    float Rx, Ry, wx, wy, inv_wx, inv_wy, z_screen, alpha, edge_x, edge_y;  // edge = exp(-alpha (nu/2)^2)
    // options
    int32_t fresnel, newton_max;
    float R0, w0;                    // Schlick R0, initial ray weight 1/N
    // layout
    int64_t cp_off, img_off, n_rays;
    int64_t root_off;                // first slot of the design's rays in the exit-root buffer (-1: none)
    int32_t kt_u, kt_v;              // float offsets of the knot tables (workspace)
    // Fixed-point scale of the forward's LDS tile: a pixel contribution v (at most RPT w0) is added as the
    // integer rint(v fx_scale), fx_scale = 2^26 / w0, so that one addend stays below 2^31 and a workgroup's
    // sum for one pixel (at most 2^11 rays) below 2^37.
    float fx_scale, fx_unscale;
    int32_t sb_off;                  // first record of the design's span bounds (workspace)
    int32_t mesh_u, mesh_v;          // triangle mesh of sec. 2.2.2: rectangles per knot span (0: exact root)
    int32_t box;                     // box reconstruction (sec. 2.3) instead of the Gaussian filter
    float inv_mesh_u, inv_mesh_v;
    // freeform entry face: its control net follows the exit net (ncp = 2 n_u n_v heights per design); the
    // lens must stay at least delta_min thick between control points of equal index
    int32_t entry_ff, ncp;
    float delta_min;
    int32_t loss_kind;               // 0 RMS (sec. 2.5), 1 sum of squares
    float sxu_lo, syv_lo;            // (n_u - p) / (2 r_x) - sxu exactly, to a float: sxu + sxu_lo is the scale
};

// The same design's parameters in double precision, for the adjoint's double-precision re-trace of rays whose
// pathwise derivative single precision cannot resolve (see k_adjoint_fp64).
struct DesignDev64 {
    double r_x, r_y, z_in, n_lens, R0, w0;
    double sxu, syv, ubar0, vbar0;           // knot units per mm and at x = 0
    double pos_x, pos_y, pos_z, omc;         // point source (emitter-grid centre); omc = 1 - cos(phi_max)
    double ex0, edx, ey0, edy;               // emitter grid
    double Rx, Ry, wx, wy, z_screen, alpha, edge_x, edge_y;
};

// A ray queued by the adjoint for the double-precision re-trace: its design, its exit root in single
// precision (point sources; the start of the double-precision Newton polish) and its id.
struct QEntry {
    int32_t design;
    float t;
    int64_t id;
};

// Kernel group of a design: the trace kernels are instantiated per source kind and intersection mode.
inline int kind_group(const DesignDev& d) {
    return (d.entry_ff ? 4 : 0) + (d.mesh_u ? 2 : 0) + (d.kind != 0 ? 1 : 0);
}

// Per-design bounds of sec. 2.2.2 (global convex-hull box and slope bounds), formed by launch_bounds before
// the trace kernels of designs whose rays need the root search (point and grid sources).
struct BoundsDev {
    float zmin, zmax, gx, gy;        // gx, gy: bounds of |dh/dx|, |dh/dy| from derivative control points
    float zref;                      // reference height subtracted from P^z in LDS
    // the same for a freeform entry face (zero otherwise)
    float zmin_in, zmax_in, gx_in, gy_in, zref_in;
};

// The same bounds for one knot-span product (su, sv) of a design, record su * nsv + sv: the surface over
// that span lies in [zmin, zmax] and its slopes within gx, gy (convex hull of the span's control points and
// of its derivative control points).
struct SpanBounds {
    float zmin, zmax, gx, gy;
};

// Block map of one design for one block shape.
struct BlockMap {
    int64_t first;                   // first logical block of the design
    int32_t nbv, per_emitter;        // blocks along v; blocks per emitter
};

// Scalars of dL/dI for one design: dL/dI = ((I is - T isT) - dot) coef.
struct LossScalars {
    float is, isT, dot, coef;
};

// Adam applied by the finishing kernel after the adjoint (null Pz: plain gradient output).  With theta set
// the optimised variables are theta (sec. 2.4.1): P = lo + (tanh(theta) + 1) span / 2, Adam steps theta with
// dL/dtheta = dL/dP (1 - tanh^2 theta) span / 2, and Pz is rewritten from the new theta.
struct AdamArgs {
    float* Pz;
    float* m;
    float* v;
    int32_t* t;
    ffrt_adam_hparams hp;
    float* theta;
    const float* lo;
    const float* span;
};

struct TraceArgs {
    const DesignDev* designs;
    const BoundsDev* bounds;         // of the current Pz, for point and grid sources
    const SpanBounds* span_bounds;   // per span product, for point and grid sources
    int32_t lds_sb;                  // floats of the LDS span-bounds table (0: use the global bounds only)
    const float* knots;
    const BlockMap* bmap;            // n_designs entries for the launch's block shape
    int32_t n_designs;
    int64_t n_blocks;
    int32_t lds_cp;                  // floats of the LDS control-point array (max over designs)
    int32_t lds_kt;                  // floats of the LDS knot tables
    const float* Pz;
    unsigned long long* img64;       // forward: fixed-point irradiance accumulator (zero on entry)
    ffrt_stats* slots;               // forward: NSLOT partial-statistics slots per design (may be null)
    const float* dLdI;               // adjoint input
    // adjoint: gradient accumulator in 64-bit fixed point (zero on entry; launch_finish converts and clears
    // it), and per design the cotangent bound max |dL/dI| (float bits) that sets its unit
    unsigned long long* gacc;
    const uint32_t* gmax;
    int32_t use_tile;                // forward: LDS footprint tile
    int32_t butterfly;               // adjoint: wave-level reduce-scatter of control-point gradients
    int32_t kind_group;              // 0: collimated designs, 1: point-source designs (bmap covers only these)
    // Exit roots of the point-source rays of kernel group 1 (exact root, flat entry), one float per ray at
    // root_off + ray index (-1: no hit).  The forward stores them and the adjoint of the same step reads
    // them instead of searching again; null: every kernel searches.
    float* roots;
    // Adjoint, kernel groups 0, 1 and 5: rays whose derivative single precision cannot resolve (landing
    // within rounding of a pixel edge, near total internal reflection) are left out and queued for the
    // double-precision re-trace: logical block b of the launch writes up to queue_cap(shape) entries at
    // queue + (qbase + b) queue_cap and their number at qcount[qbase + b]; group 5 (two freeform faces) also
    // writes each ray's entry root at the same place of queue_tin.  Null: no queue.
    QEntry* queue;
    int32_t* qcount;
    float* queue_tin;
    int64_t qbase;
};

// Queue capacity per logical block of the adjoint: 1/64 of its rays (the re-traced rays are ~0.4 %).
__host__ __device__ constexpr int queue_cap(int shape) { return (WG << shape) / 64; }  // RPT = 2^shape

struct FwdCfg { int shape; int tile; int persistent; const char* name; };
struct AdjCfg { int shape; int butterfly; int persistent; const char* name; };

constexpr FwdCfg FWD_CFGS[] = {
    {2, 1, 0, "fwd rpt4 lds-tile"},
    {3, 1, 0, "fwd rpt8 lds-tile"},
    {1, 1, 0, "fwd rpt2 lds-tile"},
    {0, 1, 0, "fwd rpt1 lds-tile"},
    {3, 1, 1, "fwd rpt8 lds-tile persistent"},
    {2, 0, 0, "fwd rpt4 global-atomics"},
};
constexpr AdjCfg ADJ_CFGS[] = {
    {2, 1, 0, "adj rpt4 butterfly"},
    {3, 1, 0, "adj rpt8 butterfly"},
    {4, 1, 0, "adj rpt16 butterfly"},
    {1, 1, 0, "adj rpt2 butterfly"},
    {3, 0, 0, "adj rpt8 lds-atomics"},
    {4, 1, 1, "adj rpt16 butterfly persistent"},
};
constexpr int N_FWD_CFGS = sizeof(FWD_CFGS) / sizeof(FWD_CFGS[0]);
constexpr int N_ADJ_CFGS = sizeof(ADJ_CFGS) / sizeof(ADJ_CFGS[0]);

// Launchers of the templated trace kernels, one set per compiled (P, Q, NU).  adjoint_fp64 re-traces the queued
// rays of logical blocks [first, first + nblocks) (queue and qcount as in TraceArgs, qbase 0) in double
// precision; mode: which kind of rays those blocks queued, each with an instance of its own: F64_FLAT (flat entry
// face, exact root), F64_TWO and F64_TWO_COLL (point sources and collimated rays through two freeform faces),
// F64_MESH (the mesh).
constexpr int F64_FLAT = 0, F64_TWO = 1, F64_MESH = 2, F64_TWO_COLL = 3;
struct KernelSet {
    hipError_t (*forward)(const TraceArgs&, int shape, int grid, hipStream_t);
    hipError_t (*adjoint)(const TraceArgs&, int shape, int grid, hipStream_t);
    hipError_t (*adjoint_fp64)(const TraceArgs&, const DesignDev64* d64, int shape, int64_t first, int64_t nblocks,
                               int mode, hipStream_t);
    hipError_t (*trace_rays)(const TraceArgs&, int design, const int64_t* ids, int64_t n, float* out8,
                             hipStream_t);
};

// Returns null when (P, Q, NU) is not compiled.
const KernelSet* kernel_set(int P, int Q, int NU);

// Kernels that do not depend on the degrees (ffrt_common.hip).
// Bounds of sec. 2.2.2 of every design from Pz, globally and per span product (one workgroup per design).
hipError_t launch_bounds(const DesignDev* designs, int n_designs, const float* Pz, int p, int q, BoundsDev* bounds,
                         SpanBounds* span_bounds, hipStream_t s);
// Image slices: LB = loss_blocks_per_design(largest image) workgroups per design, LB <= 64.
int loss_blocks_per_design(int64_t max_pixels);
// img64 -> irr (float), img64 cleared.  With stats, the partial-statistics slots are summed into stats and
// cleared, and the lens checks of sec. 2.1.2 are counted from Pz.
hipError_t launch_resolve(const DesignDev* designs, int n_designs, int LB, unsigned long long* img64, float* irr,
                          const float* Pz, ffrt_stats* slots, ffrt_stats* stats, hipStream_t s);
// Slice sums of the loss into partial (n_designs * LB * 5 doubles), resolving the irradiance from img64
// first when img64 is not null (as launch_resolve, statistics included); then dL/dI, loss and valid.  With
// gmax set (zero on entry), the largest |dL/dI| of every design goes there too, for the adjoint's unit.
hipError_t launch_loss(const DesignDev* designs, int n_designs, int LB, unsigned long long* img64, float* irr,
                       const float* target, const float* Pz, ffrt_stats* slots, ffrt_stats* stats, double* partial,
                       float* loss, float* dLdI, int32_t* valid, uint32_t* gmax, hipStream_t s);
// The largest |dL/dI| of every design of a given dL/dI into gmax (one workgroup per design).
hipError_t launch_gscale(const DesignDev* designs, int n_designs, const float* dLdI, uint32_t* gmax, hipStream_t s);
// After the adjoint: dL/dP from the fixed-point gacc, gacc and gmax cleared; with adam.Pz set, Adam updates the
// designs whose loss found flux (valid).
hipError_t launch_finish(const DesignDev* designs, int n_designs, unsigned long long* gacc, uint32_t* gmax,
                         float* dLdP, const int32_t* valid, const AdamArgs& adam, hipStream_t s);
// Range reparametrisation of sec. 2.4.1 over n packed control points: mode 0 writes P from theta, mode 1
// writes dL/dtheta from dL/dP.
hipError_t launch_reparam(int mode, int64_t n, const float* theta, const float* lo, const float* span, float* P,
                          const float* dLdP, float* dLdtheta, hipStream_t s);
// The control-point generators of sec. 2.4 (ffrt_mlp.hip); arch: FFRT_MLP_DENSE or FFRT_MLP_SPARSE, P and Q
// the plan's degrees (the sparse footprint).  poff: device offsets of each design's parameters; acts: h1, h2,
// y per design at 3 cp_off.  Forward: activations and Pz (with t set, the step counter of every valid design
// advances).  Backward: dz3, dh2, dh1 (packed like Pz) are scratch; grad (may be null) receives the parameter
// gradient; with hp set, Adam updates the parameters of valid designs.  The sparse kernels hold 2 Kmax floats
// in LDS.  part: MLP_ALL, or (for timing) MLP_BACKPROP (vectors only) / MLP_UPDATE (gradient and Adam only).
enum { MLP_ALL = 0, MLP_BACKPROP = 1, MLP_UPDATE = 2 };
hipError_t launch_mlp_forward(int arch, int P, int Q, const DesignDev* designs, int nd, int Kmax,
                              const int64_t* poff, const float* par, float* acts, const float* lo, const float* span,
                              float* Pz, int32_t* t, const int32_t* valid, hipStream_t s);
hipError_t launch_mlp_backward(int arch, int part, int P, int Q, const DesignDev* designs, int nd, int Kmax,
                               const int64_t* poff, float* par, const float* acts, const float* span,
                               const float* dLdP, float* dz3, float* dh2, float* dh1, float* grad, float* m, float* v,
                               const int32_t* t, const int32_t* valid, const ffrt_adam_hparams* hp, hipStream_t s);
hipError_t launch_loss_f64(const DesignDev* designs, int n_designs, const float* irr, const float* target,
                           double* loss, hipStream_t s);
hipError_t launch_adam(const DesignDev* designs, int n_designs, float* Pz, const float* g, float* m,
                       float* v, int32_t* t, const int32_t* valid, ffrt_adam_hparams hp, hipStream_t s);
hipError_t launch_lds_atomics(int pattern, int iters, int grid, uint32_t* out, hipStream_t s);
hipError_t launch_rng(uint64_t seed, uint64_t stream_id, uint64_t first, int64_t n, uint64_t* out,
                      hipStream_t s);

// Address of this device's copy of the library's static scratch array (STATIC_SCRATCH_BYTES, 256-byte
// aligned), resolved with hipGetSymbolAddress on the first call per device, and the device's CU count.
hipError_t static_scratch(void** ptr, int* num_cu);
// n 32-bit words at p set to v by a kernel on stream s.
hipError_t launch_fill_u32(void* p, int64_t n, uint32_t v, hipStream_t s);

// Host-side SplitMix64 state (same published definition as the device generator).
uint64_t splitmix_state0(uint64_t seed, uint64_t stream_id);

}  // namespace ffrt
