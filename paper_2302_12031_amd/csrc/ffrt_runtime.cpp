// Host runtime of libffrt: plan validation, workspace layout, launches, HIP graph capture and the kernel
// shape autotuner.  Implements the C ABI declared in include/ffrt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ffrt_internal.h"

namespace ffrt {
const KernelSet* kernel_set_p3q3nu3();
const KernelSet* kernel_set_p3q3nu5();
const KernelSet* kernel_set_p3q3nu11();
const KernelSet* kernel_set_p5q3nu3();
const KernelSet* kernel_set_p2q2nu3();

const KernelSet* kernel_set(int P, int Q, int NU) {
    if (P == 3 && Q == 3 && NU == 3) return kernel_set_p3q3nu3();
    if (P == 3 && Q == 3 && NU == 5) return kernel_set_p3q3nu5();
    if (P == 3 && Q == 3 && NU == 11) return kernel_set_p3q3nu11();
    if (P == 5 && Q == 3 && NU == 3) return kernel_set_p5q3nu3();
    if (P == 2 && Q == 2 && NU == 3) return kernel_set_p2q2nu3();
    return nullptr;
}
}  // namespace ffrt

using namespace ffrt;

namespace {

thread_local std::string g_err;

ffrt_status fail(ffrt_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

ffrt_status hip_fail(hipError_t e, const char* where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return FFRT_E_HIP;
}

#define HIP_TRY(expr)                                      \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return hip_fail(_e, #expr);  \
    } while (0)

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct ShapeDims { int BU, BV; };
ShapeDims shape_dims(int shape) { return {16 * shape_mu(shape), 16 * shape_mv(shape)}; }

}  // namespace

struct ffrt_plan {
    std::vector<ffrt_problem> probs;
    int nd = 0, P = 3, Q = 3, NU = 3;
    const KernelSet* ks = nullptr;
    std::vector<DesignDev> dd;
    std::vector<DesignDev64> dd64;
    std::vector<int64_t> cp_off, img_off, mlp_off[2];
    int64_t total_cp = 0, total_img = 0, total_rays = 0;
    int max_cp = 0, max_kt = 0, loss_lb = 1, max_spans = 0;
    int64_t total_spans = 0;
    bool has_point = false;  // some design needs the root search (bounds kernel)
    int64_t root_rays = 0;   // rays of kernel group 1 (point source, exact root, flat entry)
    bool roots_on = false;   // their exit-root buffer fits the cap and is in the workspace
    int64_t max_img = 0;
    std::vector<float> knots;
    // block maps per shape and source-kind group (designs of the other group get no blocks)
    std::vector<BlockMap> bmaps[N_SHAPES][N_KG];
    int64_t nblocks[N_SHAPES][N_KG] = {};
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t off_designs = 0, off_bounds = 0, off_sb = 0, off_valid = 0, off_knots = 0, off_bmap = 0, off_slots = 0;
    size_t need = 0;
    size_t off_lpart = 0, off_img64 = 0, off_gacc = 0, off_gmax = 0, off_dldi = 0, off_mlpoff = 0, off_mlpvec = 0,
           off_roots = 0, off_d64 = 0, off_queue = 0, off_qcount = 0, off_qtin = 0;
    int num_cu = 256;
    int fwd_cfg = 0, adj_cfg = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    DesignDev* d_designs() const { return reinterpret_cast<DesignDev*>(ws + off_designs); }
    BoundsDev* d_bounds() const { return reinterpret_cast<BoundsDev*>(ws + off_bounds); }
    SpanBounds* d_sb() const { return reinterpret_cast<SpanBounds*>(ws + off_sb); }
    int32_t* d_valid() const { return reinterpret_cast<int32_t*>(ws + off_valid); }
    float* d_knots() const { return reinterpret_cast<float*>(ws + off_knots); }
    BlockMap* d_bmap(int shape, int kg) const {
        return reinterpret_cast<BlockMap*>(ws + off_bmap) + ((size_t)shape * N_KG + kg) * nd;
    }
    ffrt_stats* d_slots() const { return reinterpret_cast<ffrt_stats*>(ws + off_slots); }
    double* d_lpart() const { return reinterpret_cast<double*>(ws + off_lpart); }
    unsigned long long* d_img64() const { return reinterpret_cast<unsigned long long*>(ws + off_img64); }
    unsigned long long* d_gacc() const { return reinterpret_cast<unsigned long long*>(ws + off_gacc); }
    uint32_t* d_gmax() const { return reinterpret_cast<uint32_t*>(ws + off_gmax); }
    float* d_dldi() const { return reinterpret_cast<float*>(ws + off_dldi); }
    int64_t* d_mlpoff(int arch) const { return reinterpret_cast<int64_t*>(ws + off_mlpoff) + (size_t)arch * (nd + 1); }
    float* d_mlpvec(int k) const { return reinterpret_cast<float*>(ws + off_mlpvec) + (size_t)k * total_cp; }
    float* d_roots() const { return roots_on ? reinterpret_cast<float*>(ws + off_roots) : nullptr; }
    DesignDev64* d_d64() const { return reinterpret_cast<DesignDev64*>(ws + off_d64); }
    QEntry* d_queue() const { return reinterpret_cast<QEntry*>(ws + off_queue); }
    int32_t* d_qcount() const { return reinterpret_cast<int32_t*>(ws + off_qcount); }
    float* d_qtin() const { return reinterpret_cast<float*>(ws + off_qtin); }
};

namespace {

bool odd3(int v) { return v >= 3 && (v % 2) == 1; }

ffrt_status validate(const ffrt_problem& pr, int idx) {
    char b[256];
    auto bad = [&](const char* what) {
        snprintf(b, sizeof b, "design %d: %s", idx, what);
        return fail(FFRT_E_ARG, b);
    };
    const ffrt_lens& L = pr.lens;
    const ffrt_source& S = pr.src;
    const ffrt_detector& D = pr.det;
    if (L.p < 1 || L.q < 1 || L.p > MAX_DEG || L.q > MAX_DEG) return bad("degrees must be in [1, 5]");
    if (L.n_u <= L.p || L.n_v <= L.q) return bad("need more control points than the degree");
    if ((int64_t)L.n_u * L.n_v > MAX_CP || L.n_u - L.p > 64 || L.n_v - L.q > 64)
        return bad("control net above 4096 points or 64 knot spans along an axis");
    if (L.entry_freeform != 0 && L.entry_freeform != 1) return bad("entry_freeform must be 0 or 1");
    if (L.entry_freeform && (int64_t)L.n_u * L.n_v > 2048)
        return bad("a lens with two freeform faces allows at most 2048 control points per face");
    if (L.entry_freeform && pr.opt.mesh_u) return bad("the triangle mesh applies to a flat entry face only");
    if (!(L.n_lens > 1.0) || !std::isfinite(L.n_lens)) return bad("n_lens must be > 1");
    if (!(L.r_x > 0) || !(L.r_y > 0)) return bad("aperture half widths must be > 0");
    if (!(L.delta_min >= 0)) return bad("delta_min must be >= 0");
    if (S.kind < 0 || S.kind > 2) return bad("source kind must be 0, 1 or 2");
    if (S.grid_u < 1 || S.grid_v < 1 || S.grid_u > (1 << 24) || S.grid_v > (1 << 24)) return bad("bad sample grid");
    if (S.jitter != 0 && S.jitter != 1) return bad("jitter must be 0 or 1");
    if (S.kind != 0) {
        if (!(S.pos[2] < L.z_in)) return bad("point source must lie below the entry face");
        if (!(S.half_angle >= 0 && S.half_angle < M_PI / 2)) return bad("half angle must be in [0, pi/2)");
        if (S.kind == 2 && (S.emit_nx < 1 || S.emit_ny < 1 || !(S.emit_wx >= 0) || !(S.emit_wy >= 0)))
            return bad("bad emitter grid");
    }
    if (D.n_x < 1 || D.n_y < 1 || D.n_x > 8192 || D.n_y > 8192) return bad("bad detector resolution");
    if (!(D.R_x > 0) || !(D.R_y > 0)) return bad("screen radii must be > 0");
    if (!(D.alpha > 0)) return bad("alpha must be > 0");
    if (!odd3(D.nu_x) || !odd3(D.nu_y)) return bad("filter sizes must be odd and >= 3");
    if (D.ghost != 0 && D.ghost != 1) return bad("ghost must be 0 or 1");
    if (D.filter != 0 && D.filter != 1) return bad("filter must be 0 (Gaussian) or 1 (box)");
    if (!(D.z_screen > L.z_in)) return bad("screen must lie above the entry face");
    if (pr.opt.fresnel != 0 && pr.opt.fresnel != 1) return bad("fresnel must be 0 or 1");
    if (pr.opt.newton_max_iter < 1 || pr.opt.newton_max_iter > 32) return bad("newton_max_iter in [1, 32]");
    if (pr.opt.loss != 0 && pr.opt.loss != 1) return bad("loss must be 0 (RMS) or 1 (sum of squares)");
    if (pr.opt.reserved != 0) return bad("options.reserved must be 0");
    if (pr.opt.mesh_u < 0 || pr.opt.mesh_u > 64 || pr.opt.mesh_v < 0 || pr.opt.mesh_v > 64 ||
        (pr.opt.mesh_u == 0) != (pr.opt.mesh_v == 0))
        return bad("mesh_u, mesh_v: both 0 (exact root) or both in [1, 64]");
    int64_t n = (int64_t)S.grid_u * S.grid_v * (S.kind == 2 ? (int64_t)S.emit_nx * S.emit_ny : 1);
    // the forward's fixed-point pixel sums (at most 2^26 per ray) must stay below 2^63
    if (n > ((int64_t)1 << 36)) return bad("too many rays in one design (at most 2^36)");
    return FFRT_OK;
}

// Knot table of one axis (see span_basis): for span k, local knots kap(o) = clamp(o, -k, nspan - k) for
// o = 1-p..p, then 1 / (kap(j) - kap(j - deg)) for deg = 1..p, j = 1..deg (0 for zero-length intervals).
void build_knot_table(int p, int nspan, std::vector<float>& out) {
    const int st = kt_stride(p);
    for (int k = 0; k < nspan; ++k) {
        std::vector<float> row(st, 0.0f);
        auto kap = [&](int o) { return std::min(std::max(o, -k), nspan - k); };
        for (int o = 1 - p; o <= p; ++o) row[o + p - 1] = (float)kap(o);
        int idx = 2 * p;
        for (int deg = 1; deg <= p; ++deg)
            for (int j = 1; j <= deg; ++j) {
                int diff = kap(j) - kap(j - deg);
                row[idx++] = diff > 0 ? (float)(1.0 / diff) : 0.0f;
            }
        out.insert(out.end(), row.begin(), row.end());
    }
}

DesignDev make_design(const ffrt_problem& pr, int64_t cp_off, int64_t img_off, int kt_u, int kt_v) {
    DesignDev d;
    std::memset(&d, 0, sizeof d);
    const ffrt_lens& L = pr.lens;
    const ffrt_source& S = pr.src;
    const ffrt_detector& D = pr.det;
    d.r_x = (float)L.r_x;
    d.r_y = (float)L.r_y;
    d.z_in = (float)L.z_in;
    d.n_lens = (float)L.n_lens;
    d.n_u = L.n_u;
    d.n_v = L.n_v;
    d.nsu = L.n_u - L.p;
    d.nsv = L.n_v - L.q;
    d.sxu = (float)(d.nsu / (2.0 * L.r_x));
    d.syv = (float)(d.nsv / (2.0 * L.r_y));
    d.sxu_lo = (float)(d.nsu / (2.0 * L.r_x) - (double)d.sxu);
    d.syv_lo = (float)(d.nsv / (2.0 * L.r_y) - (double)d.syv);
    d.ubar0 = 0.5f * (float)d.nsu;
    d.vbar0 = 0.5f * (float)d.nsv;
    d.zmin_allowed = (float)(L.z_in + L.delta_min);
    d.entry_ff = L.entry_freeform;
    d.ncp = L.n_u * L.n_v * (L.entry_freeform ? 2 : 1);
    d.delta_min = (float)L.delta_min;
    d.kind = S.kind;
    d.grid_u = S.grid_u;
    d.grid_v = S.grid_v;
    d.jitter = S.jitter;
    d.pos_x = (float)S.pos[0];
    d.pos_y = (float)S.pos[1];
    d.pos_z = (float)S.pos[2];
    d.omc = (float)(1.0 - std::cos(S.half_angle));
    d.emit_nx = S.kind == 2 ? S.emit_nx : 1;
    d.emit_ny = S.kind == 2 ? S.emit_ny : 1;
    d.ex0 = (S.kind == 2 && S.emit_nx > 1) ? (float)(-0.5 * S.emit_wx) : 0.0f;
    d.edx = (S.kind == 2 && S.emit_nx > 1) ? (float)(S.emit_wx / (S.emit_nx - 1)) : 0.0f;
    d.ey0 = (S.kind == 2 && S.emit_ny > 1) ? (float)(-0.5 * S.emit_wy) : 0.0f;
    d.edy = (S.kind == 2 && S.emit_ny > 1) ? (float)(S.emit_wy / (S.emit_ny - 1)) : 0.0f;
    d.inv_gu = (float)(1.0 / S.grid_u);
    d.inv_gv = (float)(1.0 / S.grid_v);
    d.rng_state0 = splitmix_state0(S.seed, 2);
    double wx = 2.0 * D.R_x / D.n_x, wy = 2.0 * D.R_y / D.n_y;
    if (D.ghost) {
        d.nx = D.n_x + D.nu_x - 1;
        d.ny = D.n_y + D.nu_y - 1;
        d.Rx = (float)(D.R_x + 0.5 * (D.nu_x - 1) * wx);
        d.Ry = (float)(D.R_y + 0.5 * (D.nu_y - 1) * wy);
    } else {
        d.nx = D.n_x;
        d.ny = D.n_y;
        d.Rx = (float)D.R_x;
        d.Ry = (float)D.R_y;
    }
    d.wx = (float)wx;
    d.wy = (float)wy;
    d.inv_wx = (float)(1.0 / wx);
    d.inv_wy = (float)(1.0 / wy);
    d.z_screen = (float)D.z_screen;
    d.alpha = (float)D.alpha;
    d.edge_x = (float)std::exp(-D.alpha * 0.25 * D.nu_x * D.nu_x);
    d.edge_y = (float)std::exp(-D.alpha * 0.25 * D.nu_y * D.nu_y);
    d.fresnel = pr.opt.fresnel;
    d.newton_max = pr.opt.newton_max_iter;
    d.box = pr.det.filter;
    d.mesh_u = pr.opt.mesh_u;
    d.loss_kind = pr.opt.loss;
    d.mesh_v = pr.opt.mesh_v;
    d.inv_mesh_u = d.mesh_u ? 1.0f / (float)d.mesh_u : 0.0f;
    d.inv_mesh_v = d.mesh_v ? 1.0f / (float)d.mesh_v : 0.0f;
    double r0 = (L.n_lens - 1.0) / (L.n_lens + 1.0);
    d.R0 = (float)(r0 * r0);
    int64_t n = (int64_t)S.grid_u * S.grid_v * d.emit_nx * d.emit_ny;
    d.n_rays = n;
    d.w0 = (float)(1.0 / (double)n);
    d.fx_scale = (float)(std::ldexp(1.0, 26) / (double)d.w0);
    d.fx_unscale = (float)((double)d.w0 * std::ldexp(1.0, -26));
    d.cp_off = cp_off;
    d.img_off = img_off;
    d.kt_u = kt_u;
    d.kt_v = kt_v;
    return d;
}

// The design's parameters in double precision, for the adjoint's double-precision re-trace (the same
// quantities as make_design without the single-precision rounding).
DesignDev64 make_design64(const ffrt_problem& pr) {
    DesignDev64 d;
    std::memset(&d, 0, sizeof d);
    const ffrt_lens& L = pr.lens;
    const ffrt_source& S = pr.src;
    const ffrt_detector& D = pr.det;
    d.r_x = L.r_x;
    d.r_y = L.r_y;
    d.z_in = L.z_in;
    d.n_lens = L.n_lens;
    const double r0 = (L.n_lens - 1.0) / (L.n_lens + 1.0);
    d.R0 = r0 * r0;
    const int64_t n = (int64_t)S.grid_u * S.grid_v * (S.kind == 2 ? (int64_t)S.emit_nx * S.emit_ny : 1);
    d.w0 = 1.0 / (double)n;
    d.sxu = (double)(L.n_u - L.p) / (2.0 * L.r_x);
    d.syv = (double)(L.n_v - L.q) / (2.0 * L.r_y);
    d.ubar0 = 0.5 * (double)(L.n_u - L.p);
    d.vbar0 = 0.5 * (double)(L.n_v - L.q);
    d.pos_x = S.pos[0];
    d.pos_y = S.pos[1];
    d.pos_z = S.pos[2];
    d.omc = 1.0 - std::cos(S.half_angle);
    if (S.kind == 2 && S.emit_nx > 1) {
        d.ex0 = -0.5 * S.emit_wx;
        d.edx = S.emit_wx / (S.emit_nx - 1);
    }
    if (S.kind == 2 && S.emit_ny > 1) {
        d.ey0 = -0.5 * S.emit_wy;
        d.edy = S.emit_wy / (S.emit_ny - 1);
    }
    d.wx = 2.0 * D.R_x / D.n_x;
    d.wy = 2.0 * D.R_y / D.n_y;
    d.Rx = D.ghost ? D.R_x + 0.5 * (D.nu_x - 1) * d.wx : D.R_x;
    d.Ry = D.ghost ? D.R_y + 0.5 * (D.nu_y - 1) * d.wy : D.R_y;
    d.z_screen = D.z_screen;
    d.alpha = D.alpha;
    d.edge_x = std::exp(-D.alpha * 0.25 * D.nu_x * D.nu_x);
    d.edge_y = std::exp(-D.alpha * 0.25 * D.nu_y * D.nu_y);
    return d;
}

bool ready(ffrt_plan* p) { return p && p->ws; }

TraceArgs make_args(ffrt_plan* pl, int shape, int kg) {
    TraceArgs A;
    std::memset(&A, 0, sizeof A);
    A.designs = pl->d_designs();
    A.bounds = pl->d_bounds();
    A.span_bounds = pl->d_sb();
    A.knots = pl->d_knots();
    A.bmap = pl->d_bmap(shape, kg);
    A.n_designs = pl->nd;
    A.n_blocks = pl->nblocks[shape][kg];
    A.kind_group = kg;
    A.lds_cp = (pl->max_cp + 3) / 4 * 4;
    A.lds_kt = (pl->max_kt + 3) / 4 * 4;
    // point sources stage the span bounds too, when the kernels' LDS then stays within 64 KiB
    const int sb = 4 * pl->max_spans;
    const bool search = kg == 1 || kg >= 4;  // exact exit root search (point sources, freeform entry faces)
    // (the forward's tile, or the adjoint's gradient net in 64-bit fixed point)
    if (search && 4 * (A.lds_cp + A.lds_kt + sb + std::max(TILE_CAP, 2 * A.lds_cp)) <= 65536) A.lds_sb = sb;
    return A;
}

int grid_for(ffrt_plan* pl, int shape, int kg, int persistent) {
    int64_t nb = pl->nblocks[shape][kg];
    int64_t g = nb;
    if (persistent) g = std::min<int64_t>(nb, (int64_t)pl->num_cu * 4);
    // launches are limited to 2^31 work items; larger batches loop over blocks inside the kernel
    if (g > ((int64_t)1 << 22)) g = (int64_t)1 << 22;
    return (int)std::max<int64_t>(g, 1);
}

// The forward trace kernel, into the plan's fixed-point image; partial statistics go to the plan's slots
// when `stats` is set.  The image must be resolved (launch_resolve or the loss) before the next forward.
// With `roots` the exit roots of kernel group 1 go to the plan's root buffer (when it has one).
ffrt_status launch_forward(ffrt_plan* pl, const float* Pz, bool stats, hipStream_t s, bool roots = false) {
    const FwdCfg& c = FWD_CFGS[pl->fwd_cfg];
    for (int kg = 0; kg < N_KG; ++kg) {
        if (pl->nblocks[c.shape][kg] == 0) continue;
        TraceArgs A = make_args(pl, c.shape, kg);
        A.Pz = Pz;
        A.img64 = pl->d_img64();
        A.slots = stats ? pl->d_slots() : nullptr;
        A.use_tile = c.tile;
        A.roots = roots && kg == 1 ? pl->d_roots() : nullptr;
        HIP_TRY(pl->ks->forward(A, c.shape, grid_for(pl, c.shape, kg, c.persistent), s));
    }
    return FFRT_OK;
}

// The adjoint trace kernel, into the plan's gradient accumulator (launch_finish turns it into dL/dP).  With
// `roots` the rays of kernel group 1 take their exit roots from the root buffer, which a forward with the
// same Pz must have filled.
ffrt_status launch_adjoint(ffrt_plan* pl, const float* Pz, const float* dLdI, hipStream_t s, bool roots = false) {
    const AdjCfg& c = ADJ_CFGS[pl->adj_cfg];
    // the rays whose derivative single precision cannot resolve are queued per logical block, the groups' blocks
    // in the order 0, 1 (flat entry face), 5, 4 (two freeform faces), 3, 2 (the mesh), and re-traced in double
    // precision afterwards, one kernel instance per kind
    const int64_t qb0 = pl->nblocks[c.shape][0], qb1 = pl->nblocks[c.shape][1], qb5 = pl->nblocks[c.shape][5],
                  qb4 = pl->nblocks[c.shape][4], qb3 = pl->nblocks[c.shape][3], qb2 = pl->nblocks[c.shape][2];
    const int64_t qblocks = qb0 + qb1 + qb5 + qb4 + qb3 + qb2;
    auto qfirst = [&](int kg) -> int64_t {
        switch (kg) {
            case 0: return 0;
            case 1: return qb0;
            case 5: return qb0 + qb1;
            case 4: return qb0 + qb1 + qb5;
            case 3: return qb0 + qb1 + qb5 + qb4;
            default: return qb0 + qb1 + qb5 + qb4 + qb3;  // group 2
        }
    };
    for (int kg = 0; kg < N_KG; ++kg) {
        if (pl->nblocks[c.shape][kg] == 0) continue;
        TraceArgs A = make_args(pl, c.shape, kg);
        A.Pz = Pz;
        A.dLdI = dLdI;
        A.gacc = pl->d_gacc();
        A.gmax = pl->d_gmax();
        A.butterfly = c.butterfly;
        A.roots = roots && kg == 1 ? pl->d_roots() : nullptr;
        if (kg <= 5) {
            A.queue = pl->d_queue();
            A.qcount = pl->d_qcount();
            A.queue_tin = pl->d_qtin();
            A.qbase = qfirst(kg);
        }
        HIP_TRY(pl->ks->adjoint(A, c.shape, grid_for(pl, c.shape, kg, c.persistent), s));
    }
    if (qblocks > 0) {
        TraceArgs A = make_args(pl, c.shape, 0);
        A.Pz = Pz;
        A.dLdI = dLdI;
        A.gacc = pl->d_gacc();
        A.gmax = pl->d_gmax();
        A.queue = pl->d_queue();
        A.qcount = pl->d_qcount();
        A.queue_tin = pl->d_qtin();
        if (qb0 + qb1 > 0) HIP_TRY(pl->ks->adjoint_fp64(A, pl->d_d64(), c.shape, 0, qb0 + qb1, F64_FLAT, s));
        if (qb5 > 0) HIP_TRY(pl->ks->adjoint_fp64(A, pl->d_d64(), c.shape, qfirst(5), qb5, F64_TWO, s));
        if (qb4 > 0) HIP_TRY(pl->ks->adjoint_fp64(A, pl->d_d64(), c.shape, qfirst(4), qb4, F64_TWO_COLL, s));
        if (qb3 + qb2 > 0) HIP_TRY(pl->ks->adjoint_fp64(A, pl->d_d64(), c.shape, qfirst(3), qb3 + qb2, F64_MESH, s));
    }
    return FFRT_OK;
}

AdamArgs no_adam() {
    AdamArgs a;
    std::memset(&a, 0, sizeof a);
    return a;
}

// Bounds of sec. 2.2.2 for the current Pz (only plans with point or grid sources use them).
ffrt_status run_bounds(ffrt_plan* pl, const float* Pz, hipStream_t s) {
    if (pl->has_point)
        HIP_TRY(launch_bounds(pl->d_designs(), pl->nd, Pz, pl->P, pl->Q, pl->d_bounds(), pl->d_sb(), s));
    return FFRT_OK;
}

ffrt_status run_forward(ffrt_plan* pl, const float* Pz, float* irr, ffrt_stats* stats, hipStream_t s,
                        bool roots = false) {
    if (ffrt_status b = run_bounds(pl, Pz, s)) return b;
    ffrt_status st = launch_forward(pl, Pz, stats != nullptr, s, roots);
    if (st) return st;
    HIP_TRY(launch_resolve(pl->d_designs(), pl->nd, pl->loss_lb, pl->d_img64(), irr, Pz, pl->d_slots(), stats, s));
    return FFRT_OK;
}

ffrt_status run_adjoint(ffrt_plan* pl, const float* Pz, const float* dLdI, float* dLdP, hipStream_t s,
                        bool roots = false) {
    if (ffrt_status b = run_bounds(pl, Pz, s)) return b;
    // the cotangent bound that sets the unit of the fixed-point gradient sums, from the dL/dI given
    HIP_TRY(launch_gscale(pl->d_designs(), pl->nd, dLdI, pl->d_gmax(), s));
    if (ffrt_status a = launch_adjoint(pl, Pz, dLdI, s, roots)) return a;
    HIP_TRY(launch_finish(pl->d_designs(), pl->nd, pl->d_gacc(), pl->d_gmax(), dLdP, nullptr, no_adam(), s));
    return FFRT_OK;
}

// One optimisation step in five kernels (six with point or grid sources: their bounds of sec. 2.2.2 first):
// forward, loss slice sums (resolving the irradiance, statistics), dL/dI (plus loss and validity), adjoint,
// finish (dL/dP and Adam).  dL/dI goes to the plan's workspace when the caller passes no buffer for it.
// With theta set (lo, span too) the optimised variables are theta, and Pz must hold P(theta) on entry (it
// does again on exit).
ffrt_status run_step(ffrt_plan* pl, float* Pz, const float* target, float* irr, float* loss, float* dLdI,
                     float* dLdP, float* m, float* v, int32_t* t, ffrt_stats* stats, const ffrt_adam_hparams& hp,
                     hipStream_t s, float* theta = nullptr, const float* lo = nullptr, const float* span = nullptr,
                     bool adam_on_P = true) {
    if (!dLdI) dLdI = pl->d_dldi();
    if (ffrt_status b = run_bounds(pl, Pz, s)) return b;
    // the adjoint below sees the same Pz: it reuses the forward's exit roots
    ffrt_status st = launch_forward(pl, Pz, stats != nullptr, s, true);
    if (st) return st;
    HIP_TRY(launch_loss(pl->d_designs(), pl->nd, pl->loss_lb, pl->d_img64(), irr, target, Pz, pl->d_slots(), stats,
                        pl->d_lpart(), loss, dLdI, pl->d_valid(), pl->d_gmax(), s));
    AdamArgs adam;
    std::memset(&adam, 0, sizeof adam);
    adam.Pz = adam_on_P ? Pz : nullptr;
    adam.m = m;
    adam.v = v;
    adam.t = t;
    adam.hp = hp;
    adam.theta = theta;
    adam.lo = lo;
    adam.span = span;
    st = launch_adjoint(pl, Pz, dLdI, s, true);
    if (st) return st;
    HIP_TRY(launch_finish(pl->d_designs(), pl->nd, pl->d_gacc(), pl->d_gmax(), dLdP, pl->d_valid(), adam, s));
    return FFRT_OK;
}

// One step of the dense control-point generator (sec. 2.4): the trace step without Adam on P, then the
// generator's back-propagation with Adam on its parameters, and its forward pass for the next step's P.
ffrt_status run_step_mlp(ffrt_plan* pl, int arch, float* par, float* m, float* v, int32_t* t, const float* lo,
                         const float* span, float* acts, float* Pz, const float* target, float* irr, float* loss,
                         float* dLdI, float* dLdP, ffrt_stats* stats, const ffrt_adam_hparams& hp, hipStream_t s) {
    ffrt_status st = run_step(pl, Pz, target, irr, loss, dLdI, dLdP, nullptr, nullptr, nullptr, stats, hp, s, nullptr,
                              nullptr, nullptr, false);
    if (st) return st;
    const int64_t* po = pl->d_mlpoff(arch);
    HIP_TRY(launch_mlp_backward(arch, MLP_ALL, pl->P, pl->Q, pl->d_designs(), pl->nd, pl->max_cp, po, par, acts, span,
                                dLdP, pl->d_mlpvec(0), pl->d_mlpvec(1), pl->d_mlpvec(2), nullptr, m, v, t,
                                pl->d_valid(), &hp, s));
    HIP_TRY(launch_mlp_forward(arch, pl->P, pl->Q, pl->d_designs(), pl->nd, pl->max_cp, po, par, acts, lo, span, Pz, t,
                               pl->d_valid(), s));
    return FFRT_OK;
}

ffrt_status capture(ffrt_plan* plan, int32_t steps, float* Pz, const float* target, float* irr, float* loss,
                    float* dL_dI, float* dL_dP, float* m, float* v, int32_t* t, ffrt_stats* stats,
                    const ffrt_adam_hparams* hp, void* stream, float* theta, const float* lo, const float* span) {
    hipStream_t s = (hipStream_t)stream;
    if (plan->gexec) { (void)hipGraphExecDestroy(plan->gexec); plan->gexec = nullptr; }
    if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    ffrt_status st = FFRT_OK;
    for (int i = 0; i < steps && st == FFRT_OK; ++i)
        st = run_step(plan, Pz, target, irr, loss, dL_dI, dL_dP, m, v, t, stats, *hp, s, theta, lo, span);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e, "hipGraphInstantiate"); }
    plan->graph = g;
    plan->gexec = ge;
    return FFRT_OK;
}

}  // namespace

extern "C" {

const char* ffrt_status_string(ffrt_status s) {
    switch (s) {
        case FFRT_OK: return "ok";
        case FFRT_E_ARG: return "invalid argument";
        case FFRT_E_CONSTRAINT: return "lens constraint violated";
        case FFRT_E_NOFLUX: return "no flux on the screen";
        case FFRT_E_HIP: return "HIP error";
        case FFRT_E_OOM: return "workspace too small";
        case FFRT_E_UNSUPPORTED: return "unsupported configuration";
        case FFRT_E_STATE: return "invalid call order";
    }
    return "unknown status";
}

const char* ffrt_last_error(void) { return g_err.c_str(); }

ffrt_status ffrt_plan_create(const ffrt_problem* probs, int32_t n_designs, ffrt_plan** out) {
    if (!out) return fail(FFRT_E_ARG, "out is null");
    *out = nullptr;
    if (!probs || n_designs < 1) return fail(FFRT_E_ARG, "need at least one design");
    for (int i = 0; i < n_designs; ++i) {
        ffrt_status s = validate(probs[i], i);
        if (s) return s;
    }
    const ffrt_problem& p0 = probs[0];
    for (int i = 1; i < n_designs; ++i) {
        const ffrt_problem& pi = probs[i];
        if (pi.lens.p != p0.lens.p || pi.lens.q != p0.lens.q || pi.det.nu_x != p0.det.nu_x ||
            pi.det.nu_y != p0.det.nu_y)
            return fail(FFRT_E_ARG, "all designs of a plan must share degrees and filter sizes");
    }
    if (p0.det.nu_x != p0.det.nu_y) return fail(FFRT_E_UNSUPPORTED, "nu_x != nu_y is not compiled");
    const KernelSet* ks = kernel_set(p0.lens.p, p0.lens.q, p0.det.nu_x);
    if (!ks) return fail(FFRT_E_UNSUPPORTED, "(p, q, nu) combination not compiled");
    ffrt_plan* pl = new ffrt_plan();
    pl->probs.assign(probs, probs + n_designs);
    pl->nd = n_designs;
    pl->P = p0.lens.p;
    pl->Q = p0.lens.q;
    pl->NU = p0.det.nu_x;
    pl->ks = ks;
    int64_t cp = 0, img = 0;
    for (int i = 0; i < n_designs; ++i) {
        const ffrt_problem& pr = probs[i];
        int kt_u = (int)pl->knots.size();
        build_knot_table(pr.lens.p, pr.lens.n_u - pr.lens.p, pl->knots);
        int kt_v = (int)pl->knots.size();
        build_knot_table(pr.lens.q, pr.lens.n_v - pr.lens.q, pl->knots);
        DesignDev d = make_design(pr, cp, img, kt_u, kt_v);
        pl->dd64.push_back(make_design64(pr));
        d.root_off = -1;
        if (kind_group(d) == 1) {
            d.root_off = pl->root_rays;
            pl->root_rays += d.n_rays;
        }
        d.sb_off = (int32_t)pl->total_spans;
        pl->total_spans += (int64_t)d.nsu * d.nsv;
        pl->max_spans = std::max(pl->max_spans, d.nsu * d.nsv);
        pl->dd.push_back(d);
        pl->cp_off.push_back(cp);
        pl->img_off.push_back(img);
        cp += (int64_t)d.ncp;
        img += (int64_t)d.nx * d.ny;
        pl->total_rays += d.n_rays;
        pl->max_cp = std::max(pl->max_cp, d.ncp);
        pl->max_img = std::max<int64_t>(pl->max_img, (int64_t)d.nx * d.ny);
        if (d.kind != 0 || d.entry_ff) pl->has_point = true;
        pl->max_kt = std::max(pl->max_kt, d.nsu * kt_stride(pl->P) + d.nsv * kt_stride(pl->Q));
    }
    pl->cp_off.push_back(cp);
    pl->img_off.push_back(img);
    pl->total_cp = cp;
    int64_t mo[2] = {0, 0};
    for (const DesignDev& d : pl->dd) {
        // the dense generator outputs all of a design's heights (both nets of a freeform entry); the sparse one
        // is defined on one control net
        const int64_t K = d.ncp, K1 = (int64_t)d.n_u * d.n_v;
        const int64_t C = (int64_t)(2 * (d.n_u - d.nsu) + 1) * (2 * (d.n_v - d.nsv) + 1);
        for (int a = 0; a < 2; ++a) pl->mlp_off[a].push_back(mo[a]);
        mo[FFRT_MLP_DENSE] += 2 * K * K + 4 * K;
        mo[FFRT_MLP_SPARSE] += 2 * C * K1 + 4 * K1;
    }
    for (int a = 0; a < 2; ++a) pl->mlp_off[a].push_back(mo[a]);
    pl->total_img = img;
    for (int sh = 0; sh < N_SHAPES; ++sh) {
        ShapeDims sd = shape_dims(sh);
        for (int kg = 0; kg < N_KG; ++kg) {
            int64_t first = 0;
            for (int i = 0; i < n_designs; ++i) {
                const DesignDev& d = pl->dd[i];
                int nbu = (d.grid_u + sd.BU - 1) / sd.BU, nbv = (d.grid_v + sd.BV - 1) / sd.BV;
                BlockMap bm;
                bm.first = first;
                bm.nbv = nbv;
                bm.per_emitter = nbu * nbv;
                pl->bmaps[sh][kg].push_back(bm);
                if (kind_group(d) == kg) first += (int64_t)bm.per_emitter * d.emit_nx * d.emit_ny;
            }
            pl->nblocks[sh][kg] = first;
        }
    }
    size_t off = 0;
    pl->off_designs = off;
    off = align256(off + sizeof(DesignDev) * n_designs);
    pl->off_bounds = off;
    off = align256(off + sizeof(BoundsDev) * n_designs);
    pl->off_sb = off;
    off = align256(off + sizeof(SpanBounds) * (size_t)pl->total_spans);
    pl->off_valid = off;
    off = align256(off + sizeof(int32_t) * n_designs);
    pl->off_knots = off;
    off = align256(off + sizeof(float) * pl->knots.size());
    pl->off_bmap = off;
    off = align256(off + sizeof(BlockMap) * N_SHAPES * N_KG * n_designs);
    pl->off_slots = off;
    off = align256(off + sizeof(ffrt_stats) * NSLOT * n_designs);
    pl->loss_lb = loss_blocks_per_design(pl->max_img);
    pl->off_lpart = off;
    off = align256(off + sizeof(double) * 5 * pl->loss_lb * n_designs);
    pl->off_img64 = off;
    off = align256(off + sizeof(unsigned long long) * (size_t)pl->total_img);
    pl->off_gacc = off;  // 64-bit fixed point
    off = align256(off + sizeof(unsigned long long) * (size_t)pl->total_cp);
    pl->off_gmax = off;
    off = align256(off + sizeof(uint32_t) * n_designs);
    // the adjoint's double-precision re-trace: design parameters, and a queue segment of queue_cap / 4 rays
    // per wave of every logical block (sized over all kernel groups, of which 0 and 1 use it, for the adjoint
    // shape that needs most)
    pl->off_d64 = off;
    off = align256(off + sizeof(DesignDev64) * n_designs);
    int64_t qent = 0, qblk = 0;
    for (int sh = 0; sh < N_SHAPES; ++sh) {
        int64_t nb = 0;
        for (int kg = 0; kg < N_KG; ++kg) nb += pl->nblocks[sh][kg];
        qent = std::max<int64_t>(qent, nb * queue_cap(sh));
        qblk = std::max<int64_t>(qblk, nb);
    }
    pl->off_queue = off;
    off = align256(off + sizeof(QEntry) * (size_t)qent);
    pl->off_qtin = off;
    off = align256(off + sizeof(float) * (size_t)qent);
    pl->off_qcount = off;
    off = align256(off + sizeof(int32_t) * 4 * (size_t)qblk);
    pl->off_dldi = off;  // dL/dI of a step whose caller does not want it
    off = align256(off + sizeof(float) * (size_t)pl->total_img);
    pl->off_mlpoff = off;  // parameter offsets of the control-point generators (dense, sparse)
    off = align256(off + 2 * sizeof(int64_t) * (size_t)(n_designs + 1));
    pl->off_mlpvec = off;  // its back-propagation vectors dz3, dh2, dh1
    off = align256(off + sizeof(float) * 3 * (size_t)pl->total_cp);
    // exit roots of the exact-root point-source rays, reused by the adjoint of a step (at most ROOTS_CAP bytes;
    // larger plans search again in the adjoint)
    pl->off_roots = off;
    pl->roots_on = pl->root_rays > 0 && (size_t)pl->root_rays * sizeof(float) <= ROOTS_CAP;
    if (pl->roots_on) off = align256(off + sizeof(float) * (size_t)pl->root_rays);
    pl->need = off;
    *out = pl;
    return FFRT_OK;
}

ffrt_status ffrt_plan_destroy(ffrt_plan* plan) {
    if (!plan) return FFRT_OK;
    if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return FFRT_OK;
}

ffrt_status ffrt_plan_workspace_size(const ffrt_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(FFRT_E_ARG, "null argument");
    *bytes = plan->need;
    return FFRT_OK;
}

ffrt_status ffrt_plan_set_workspace(ffrt_plan* plan, void* dev_ptr, size_t bytes) {
    if (!plan || !dev_ptr) return fail(FFRT_E_ARG, "null argument");
    if (bytes < plan->need) return fail(FFRT_E_OOM, "workspace smaller than ffrt_plan_workspace_size");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) return fail(FFRT_E_ARG, "workspace must be 256-byte aligned");
    plan->ws = static_cast<char*>(dev_ptr);
    plan->ws_bytes = bytes;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int ncu = 0;
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    plan->num_cu = ncu > 0 ? ncu : 256;
    HIP_TRY(hipMemcpy(plan->d_designs(), plan->dd.data(), sizeof(DesignDev) * plan->nd, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(plan->d_d64(), plan->dd64.data(), sizeof(DesignDev64) * plan->nd, hipMemcpyHostToDevice));
    std::vector<int32_t> ones(plan->nd, 1);
    HIP_TRY(hipMemcpy(plan->d_valid(), ones.data(), sizeof(int32_t) * plan->nd, hipMemcpyHostToDevice));
    // accumulators and counters that the kernels expect to be zero on entry (and leave zero on exit)
    HIP_TRY(hipMemset(plan->d_slots(), 0, sizeof(ffrt_stats) * NSLOT * plan->nd));
    HIP_TRY(hipMemset(plan->d_img64(), 0, sizeof(unsigned long long) * plan->total_img));
    HIP_TRY(hipMemset(plan->d_gacc(), 0, sizeof(unsigned long long) * plan->total_cp));
    HIP_TRY(hipMemset(plan->d_gmax(), 0, sizeof(uint32_t) * plan->nd));
    for (int a = 0; a < 2; ++a)
        HIP_TRY(hipMemcpy(plan->d_mlpoff(a), plan->mlp_off[a].data(), sizeof(int64_t) * plan->mlp_off[a].size(),
                          hipMemcpyHostToDevice));
    if (!plan->knots.empty())
        HIP_TRY(hipMemcpy(plan->d_knots(), plan->knots.data(), sizeof(float) * plan->knots.size(),
                          hipMemcpyHostToDevice));
    for (int sh = 0; sh < N_SHAPES; ++sh)
        for (int kg = 0; kg < N_KG; ++kg)
            HIP_TRY(hipMemcpy(plan->d_bmap(sh, kg), plan->bmaps[sh][kg].data(), sizeof(BlockMap) * plan->nd,
                              hipMemcpyHostToDevice));
    return FFRT_OK;
}

ffrt_status ffrt_plan_layout(const ffrt_plan* plan, int64_t* cp_offsets, int64_t* img_offsets) {
    if (!plan) return fail(FFRT_E_ARG, "null plan");
    if (cp_offsets) std::copy(plan->cp_off.begin(), plan->cp_off.end(), cp_offsets);
    if (img_offsets) std::copy(plan->img_off.begin(), plan->img_off.end(), img_offsets);
    return FFRT_OK;
}

ffrt_status ffrt_plan_num_designs(const ffrt_plan* plan, int32_t* n) {
    if (!plan || !n) return fail(FFRT_E_ARG, "null argument");
    *n = plan->nd;
    return FFRT_OK;
}

ffrt_status ffrt_plan_num_rays(const ffrt_plan* plan, int64_t* n) {
    if (!plan || !n) return fail(FFRT_E_ARG, "null argument");
    *n = plan->total_rays;
    return FFRT_OK;
}

ffrt_status ffrt_forward(ffrt_plan* plan, const float* Pz, float* irr, ffrt_stats* stats, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!Pz || !irr) return fail(FFRT_E_ARG, "null buffer");
    return run_forward(plan, Pz, irr, stats, (hipStream_t)stream);
}

ffrt_status ffrt_forward_static(ffrt_plan* plan, const float* Pz, float* irr, ffrt_stats* stats, void* stream) {
    if (!plan) return fail(FFRT_E_ARG, "null plan");
    if (!Pz || !irr) return fail(FFRT_E_ARG, "null buffer");
    // the forward reads the plan's tables and uses the accumulators up to the fixed-point image; the layout is
    // the workspace's, so everything it touches ends where the gradient accumulator would begin
    const size_t need = plan->off_gacc;
    if (need > STATIC_SCRATCH_BYTES) {
        char b[160];
        snprintf(b, sizeof b, "ffrt_forward_static: the plan needs %zu bytes of scratch, at most %zu are available",
                 need, STATIC_SCRATCH_BYTES);
        return fail(FFRT_E_OOM, b);
    }
    void* base = nullptr;
    int ncu = 0;
    HIP_TRY(static_scratch(&base, &ncu));
    hipStream_t s = (hipStream_t)stream;
    char* saved_ws = plan->ws;
    const size_t saved_bytes = plan->ws_bytes;
    const int saved_cu = plan->num_cu;
    plan->ws = static_cast<char*>(base);
    plan->ws_bytes = STATIC_SCRATCH_BYTES;
    plan->num_cu = ncu;
    // the array keeps whatever the last call on this device left there: write this plan's tables and clear
    // the statistics slots and the fixed-point image, which the forward expects at zero
    ffrt_status st = FFRT_OK;
    hipError_t e = hipMemcpyAsync(plan->d_designs(), plan->dd.data(), sizeof(DesignDev) * plan->nd,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !plan->knots.empty())
        e = hipMemcpyAsync(plan->d_knots(), plan->knots.data(), sizeof(float) * plan->knots.size(),
                           hipMemcpyHostToDevice, s);
    for (int sh = 0; sh < N_SHAPES && e == hipSuccess; ++sh)
        for (int kg = 0; kg < N_KG && e == hipSuccess; ++kg)
            e = hipMemcpyAsync(plan->d_bmap(sh, kg), plan->bmaps[sh][kg].data(), sizeof(BlockMap) * plan->nd,
                               hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fill_u32(plan->d_slots(), (int64_t)(sizeof(ffrt_stats) / 4) * NSLOT * plan->nd, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(plan->d_img64(), 2 * plan->total_img, 0u, s);
    if (e != hipSuccess) st = hip_fail(e, "ffrt_forward_static set-up");
    if (!st) st = run_forward(plan, Pz, irr, stats, s);
    plan->ws = saved_ws;
    plan->ws_bytes = saved_bytes;
    plan->num_cu = saved_cu;
    return st;
}

ffrt_status ffrt_loss(ffrt_plan* plan, const float* irr, const float* target, float* loss, float* dL_dI,
                      void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!irr || !target || !loss || !dL_dI) return fail(FFRT_E_ARG, "null buffer");
    HIP_TRY(launch_loss(plan->d_designs(), plan->nd, plan->loss_lb, nullptr, const_cast<float*>(irr), target, nullptr,
                        plan->d_slots(), nullptr, plan->d_lpart(), loss, dL_dI, plan->d_valid(), nullptr,
                        (hipStream_t)stream));
    return FFRT_OK;
}

ffrt_status ffrt_loss_f64(ffrt_plan* plan, const float* irr, const float* target, double* loss, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!irr || !target || !loss) return fail(FFRT_E_ARG, "null buffer");
    HIP_TRY(launch_loss_f64(plan->d_designs(), plan->nd, irr, target, loss, (hipStream_t)stream));
    return FFRT_OK;
}

ffrt_status ffrt_adjoint(ffrt_plan* plan, const float* Pz, const float* dL_dI, float* dL_dP, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!Pz || !dL_dI || !dL_dP) return fail(FFRT_E_ARG, "null buffer");
    return run_adjoint(plan, Pz, dL_dI, dL_dP, (hipStream_t)stream);
}

ffrt_status ffrt_adam(ffrt_plan* plan, float* Pz, const float* dL_dP, float* m, float* v, int32_t* t,
                      const ffrt_adam_hparams* hp, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!Pz || !dL_dP || !m || !v || !t || !hp) return fail(FFRT_E_ARG, "null buffer");
    HIP_TRY(launch_adam(plan->d_designs(), plan->nd, Pz, dL_dP, m, v, t, plan->d_valid(), *hp, (hipStream_t)stream));
    return FFRT_OK;
}

ffrt_status ffrt_step(ffrt_plan* plan, float* Pz, const float* target, float* irr, float* loss, float* dL_dI,
                      float* dL_dP, float* m, float* v, int32_t* t, ffrt_stats* stats, const ffrt_adam_hparams* hp,
                      void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!Pz || !target || !irr || !loss || !dL_dP || !m || !v || !t || !hp)
        return fail(FFRT_E_ARG, "null buffer");
    return run_step(plan, Pz, target, irr, loss, dL_dI, dL_dP, m, v, t, stats, *hp, (hipStream_t)stream);
}

ffrt_status ffrt_graph_capture(ffrt_plan* plan, int32_t steps, float* Pz, const float* target, float* irr,
                               float* loss, float* dL_dI, float* dL_dP, float* m, float* v, int32_t* t,
                               ffrt_stats* stats, const ffrt_adam_hparams* hp, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!stream) return fail(FFRT_E_ARG, "graph capture needs a non-default stream");
    if (steps < 1) return fail(FFRT_E_ARG, "steps must be >= 1");
    if (!Pz || !target || !irr || !loss || !dL_dP || !m || !v || !t || !hp)
        return fail(FFRT_E_ARG, "null buffer");
    return capture(plan, steps, Pz, target, irr, loss, dL_dI, dL_dP, m, v, t, stats, hp, stream, nullptr, nullptr,
                   nullptr);
}


ffrt_status ffrt_reparam_apply(ffrt_plan* plan, const float* theta, const float* lo, const float* span, float* Pz,
                               void* stream) {
    if (!plan) return fail(FFRT_E_ARG, "null plan");
    if (!theta || !lo || !span || !Pz) return fail(FFRT_E_ARG, "null buffer");
    HIP_TRY(launch_reparam(0, plan->total_cp, theta, lo, span, Pz, nullptr, nullptr, (hipStream_t)stream));
    return FFRT_OK;
}

ffrt_status ffrt_reparam_grad(ffrt_plan* plan, const float* theta, const float* span, const float* dL_dP,
                              float* dL_dtheta, void* stream) {
    if (!plan) return fail(FFRT_E_ARG, "null plan");
    if (!theta || !span || !dL_dP || !dL_dtheta) return fail(FFRT_E_ARG, "null buffer");
    HIP_TRY(launch_reparam(1, plan->total_cp, theta, nullptr, span, nullptr, dL_dP, dL_dtheta, (hipStream_t)stream));
    return FFRT_OK;
}

ffrt_status ffrt_step_reparam(ffrt_plan* plan, float* theta, const float* lo, const float* span, float* Pz,
                              const float* target, float* irr, float* loss, float* dL_dI, float* dL_dP, float* m,
                              float* v, int32_t* t, ffrt_stats* stats, const ffrt_adam_hparams* hp, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!theta || !lo || !span || !Pz || !target || !irr || !loss || !dL_dP || !m || !v || !t || !hp)
        return fail(FFRT_E_ARG, "null buffer");
    return run_step(plan, Pz, target, irr, loss, dL_dI, dL_dP, m, v, t, stats, *hp, (hipStream_t)stream, theta, lo,
                    span);
}

ffrt_status ffrt_graph_capture_reparam(ffrt_plan* plan, int32_t steps, float* theta, const float* lo,
                                       const float* span, float* Pz, const float* target, float* irr, float* loss,
                                       float* dL_dI, float* dL_dP, float* m, float* v, int32_t* t, ffrt_stats* stats,
                                       const ffrt_adam_hparams* hp, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!stream) return fail(FFRT_E_ARG, "graph capture needs a non-default stream");
    if (steps < 1) return fail(FFRT_E_ARG, "steps must be >= 1");
    if (!theta || !lo || !span || !Pz || !target || !irr || !loss || !dL_dP || !m || !v || !t || !hp)
        return fail(FFRT_E_ARG, "null buffer");
    return capture(plan, steps, Pz, target, irr, loss, dL_dI, dL_dP, m, v, t, stats, hp, stream, theta, lo, span);
}

// The dense GEMV stages one layer's input vector (K floats) in LDS, the sparse kernels two such vectors.
static constexpr int MLP_MAX_K[2] = {16384, 6144};
static ffrt_status mlp_check(ffrt_plan* plan, int32_t arch) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (arch != FFRT_MLP_DENSE && arch != FFRT_MLP_SPARSE) return fail(FFRT_E_ARG, "unknown generator architecture");
    if (arch == FFRT_MLP_SPARSE)
        for (const DesignDev& d : plan->dd)
            if (d.entry_ff) return fail(FFRT_E_ARG, "sparse generator: defined for one control net per design");
    if (plan->max_cp > MLP_MAX_K[arch])
        return fail(FFRT_E_ARG, arch == FFRT_MLP_DENSE ? "dense generator: a control net exceeds 16384 points"
                                                       : "sparse generator: a control net exceeds 6144 points");
    return FFRT_OK;
}

ffrt_status ffrt_mlp_layout(const ffrt_plan* plan, int32_t arch, int64_t* offsets) {
    if (!plan || !offsets) return fail(FFRT_E_ARG, "null argument");
    if (arch != FFRT_MLP_DENSE && arch != FFRT_MLP_SPARSE) return fail(FFRT_E_ARG, "unknown generator architecture");
    std::copy(plan->mlp_off[arch].begin(), plan->mlp_off[arch].end(), offsets);
    return FFRT_OK;
}

ffrt_status ffrt_mlp_forward(ffrt_plan* plan, int32_t arch, const float* params, const float* lo, const float* span,
                             float* acts, float* Pz, void* stream) {
    if (ffrt_status st = mlp_check(plan, arch)) return st;
    if (!params || !lo || !span || !acts || !Pz) return fail(FFRT_E_ARG, "null buffer");
    HIP_TRY(launch_mlp_forward(arch, plan->P, plan->Q, plan->d_designs(), plan->nd, plan->max_cp,
                               plan->d_mlpoff(arch), params, acts, lo, span, Pz, nullptr, nullptr,
                               (hipStream_t)stream));
    return FFRT_OK;
}

ffrt_status ffrt_mlp_backward(ffrt_plan* plan, int32_t arch, const float* params, const float* acts, const float* span,
                              const float* dL_dP, float* grad, void* stream) {
    if (ffrt_status st = mlp_check(plan, arch)) return st;
    if (!params || !acts || !span || !dL_dP || !grad) return fail(FFRT_E_ARG, "null buffer");
    HIP_TRY(launch_mlp_backward(arch, MLP_ALL, plan->P, plan->Q, plan->d_designs(), plan->nd, plan->max_cp,
                                plan->d_mlpoff(arch), const_cast<float*>(params), acts, span, dL_dP,
                                plan->d_mlpvec(0), plan->d_mlpvec(1), plan->d_mlpvec(2), grad, nullptr, nullptr,
                                nullptr, nullptr, nullptr, (hipStream_t)stream));
    return FFRT_OK;
}

ffrt_status ffrt_step_mlp(ffrt_plan* plan, int32_t arch, float* params, float* m, float* v, int32_t* t, const float* lo,
                          const float* span, float* acts, float* Pz, const float* target, float* irr, float* loss,
                          float* dL_dI, float* dL_dP, ffrt_stats* stats, const ffrt_adam_hparams* hp, void* stream) {
    if (ffrt_status st = mlp_check(plan, arch)) return st;
    if (!params || !m || !v || !t || !lo || !span || !acts || !Pz || !target || !irr || !loss || !dL_dP || !hp)
        return fail(FFRT_E_ARG, "null buffer");
    return run_step_mlp(plan, arch, params, m, v, t, lo, span, acts, Pz, target, irr, loss, dL_dI, dL_dP, stats,
                        *hp, (hipStream_t)stream);
}

ffrt_status ffrt_graph_capture_mlp(ffrt_plan* plan, int32_t arch, int32_t steps, float* params, float* m, float* v,
                                   int32_t* t, const float* lo, const float* span, float* acts, float* Pz,
                                   const float* target, float* irr, float* loss, float* dL_dI, float* dL_dP,
                                   ffrt_stats* stats, const ffrt_adam_hparams* hp, void* stream) {
    if (ffrt_status st = mlp_check(plan, arch)) return st;
    if (!stream) return fail(FFRT_E_ARG, "graph capture needs a non-default stream");
    if (steps < 1) return fail(FFRT_E_ARG, "steps must be >= 1");
    if (!params || !m || !v || !t || !lo || !span || !acts || !Pz || !target || !irr || !loss || !dL_dP || !hp)
        return fail(FFRT_E_ARG, "null buffer");
    hipStream_t s = (hipStream_t)stream;
    if (plan->gexec) { (void)hipGraphExecDestroy(plan->gexec); plan->gexec = nullptr; }
    if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    ffrt_status st = FFRT_OK;
    for (int i = 0; i < steps && st == FFRT_OK; ++i)
        st = run_step_mlp(plan, arch, params, m, v, t, lo, span, acts, Pz, target, irr, loss, dL_dI, dL_dP, stats,
                          *hp, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e, "hipGraphInstantiate"); }
    plan->graph = g;
    plan->gexec = ge;
    return FFRT_OK;
}

ffrt_status ffrt_plan_control_xy(const ffrt_plan* plan, double* x, double* y) {
    if (!plan || !x || !y) return fail(FFRT_E_ARG, "null argument");
    for (int d = 0; d < plan->nd; ++d) {
        const ffrt_lens& L = plan->probs[d].lens;
        // Greville abscissae u*_i = (u_{i+1} + ... + u_{i+p}) / p of the clamped equispaced knots (sec. 2.1.1)
        auto greville = [](int p, int n, int i) {
            double acc = 0.0;
            for (int k = i + 1; k <= i + p; ++k) {
                const double u = k <= p ? 0.0 : (k >= n ? 1.0 : double(k - p) / double(n - p));
                acc += u;
            }
            return acc / p;
        };
        const int64_t K = (int64_t)L.n_u * L.n_v;
        for (int face = 0; face <= L.entry_freeform; ++face) {  // a freeform entry net repeats the positions
            const int64_t off = plan->cp_off[d] + face * K;
            for (int i = 0; i < L.n_u; ++i)
                for (int j = 0; j < L.n_v; ++j) {
                    x[off + (int64_t)i * L.n_v + j] = (2.0 * greville(L.p, L.n_u, i) - 1.0) * L.r_x;
                    y[off + (int64_t)i * L.n_v + j] = (2.0 * greville(L.q, L.n_v, j) - 1.0) * L.r_y;
                }
        }
    }
    return FFRT_OK;
}

ffrt_status ffrt_graph_launch(ffrt_plan* plan, void* stream) {
    if (!plan || !plan->gexec) return fail(FFRT_E_STATE, "no graph captured");
    HIP_TRY(hipGraphLaunch(plan->gexec, (hipStream_t)stream));
    return FFRT_OK;
}

ffrt_status ffrt_num_configs(int32_t which, int32_t* n) {
    if (!n || (which != 0 && which != 1)) return fail(FFRT_E_ARG, "which must be 0 or 1");
    *n = which == 0 ? N_FWD_CFGS : N_ADJ_CFGS;
    return FFRT_OK;
}

ffrt_status ffrt_config_name(int32_t which, int32_t index, char* buf, int32_t buflen) {
    int32_t n = 0;
    if (ffrt_num_configs(which, &n)) return FFRT_E_ARG;
    if (index < 0 || index >= n || !buf || buflen < 1) return fail(FFRT_E_ARG, "bad index or buffer");
    const char* name = which == 0 ? FWD_CFGS[index].name : ADJ_CFGS[index].name;
    snprintf(buf, (size_t)buflen, "%s", name);
    return FFRT_OK;
}

ffrt_status ffrt_plan_set_config(ffrt_plan* plan, int32_t which, int32_t index) {
    int32_t n = 0;
    if (!plan) return fail(FFRT_E_ARG, "null plan");
    if (ffrt_num_configs(which, &n)) return FFRT_E_ARG;
    if (index < 0 || index >= n) return fail(FFRT_E_ARG, "config index out of range");
    if (which == 0) plan->fwd_cfg = index; else plan->adj_cfg = index;
    return FFRT_OK;
}

ffrt_status ffrt_plan_get_config(const ffrt_plan* plan, int32_t which, int32_t* index) {
    if (!plan || !index || (which != 0 && which != 1)) return fail(FFRT_E_ARG, "bad argument");
    *index = which == 0 ? plan->fwd_cfg : plan->adj_cfg;
    return FFRT_OK;
}

ffrt_status ffrt_plan_autotune(ffrt_plan* plan, const float* Pz, float* irr, const float* dL_dI, float* dL_dP,
                               int32_t reps, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!Pz || !irr || !dL_dI || !dL_dP || reps < 1) return fail(FFRT_E_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    ffrt_status st = FFRT_OK;
    for (int which = 0; which < 2 && st == FFRT_OK; ++which) {
        int n = which == 0 ? N_FWD_CFGS : N_ADJ_CFGS;
        int best = 0;
        float best_ms = 1e30f;
        for (int c = 0; c < n && st == FFRT_OK; ++c) {
            if (which == 0) plan->fwd_cfg = c; else plan->adj_cfg = c;
            // one untimed launch, then reps timed
            st = which == 0 ? run_forward(plan, Pz, irr, nullptr, s, true)
                            : run_adjoint(plan, Pz, dL_dI, dL_dP, s, true);
            if (st) break;
            if (hipEventRecord(e0, s) != hipSuccess) { st = hip_fail(hipGetLastError(), "hipEventRecord"); break; }
            for (int r = 0; r < reps && st == FFRT_OK; ++r)
                st = which == 0 ? run_forward(plan, Pz, irr, nullptr, s, true)
                                : run_adjoint(plan, Pz, dL_dI, dL_dP, s, true);
            if (st) break;
            hipError_t e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { st = hip_fail(e, "autotune timing"); break; }
            if (ms < best_ms) { best_ms = ms; best = c; }
        }
        if (which == 0) plan->fwd_cfg = best; else plan->adj_cfg = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

ffrt_status ffrt_plan_time_kernels(ffrt_plan* plan, const float* Pz, float* irr, const float* dL_dI,
                                   float* dL_dP, int32_t reps, float* fwd_ms, float* adj_ms, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (!Pz || !irr || !dL_dI || !dL_dP || reps < 1 || !fwd_ms || !adj_ms) return fail(FFRT_E_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[4];
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    // the kernels as a step launches them: the adjoint reuses the forward's exit roots
    ffrt_status st = run_forward(plan, Pz, irr, nullptr, s, true);
    if (!st) st = run_adjoint(plan, Pz, dL_dI, dL_dP, s, true);
    hipError_t e = hipSuccess;
    if (!st) e = hipEventRecord(ev[0], s);
    for (int r = 0; r < reps && !st && e == hipSuccess; ++r) st = launch_forward(plan, Pz, false, s, true);
    if (!st && e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (!st && e == hipSuccess) e = hipEventRecord(ev[2], s);
    for (int r = 0; r < reps && !st && e == hipSuccess; ++r)
        st = launch_adjoint(plan, Pz, dL_dI, s, true);
    if (!st && e == hipSuccess) e = hipEventRecord(ev[3], s);
    if (!st && e == hipSuccess) e = hipEventSynchronize(ev[3]);
    // the timed launches accumulated into the fixed-point image and the gradient accumulator without
    // consuming them: clear both in any case
    hipError_t ez = hipMemsetAsync(plan->d_img64(), 0, sizeof(unsigned long long) * plan->total_img, s);
    if (ez == hipSuccess) ez = hipMemsetAsync(plan->d_gacc(), 0, sizeof(unsigned long long) * plan->total_cp, s);
    if (ez == hipSuccess) ez = hipMemsetAsync(plan->d_gmax(), 0, sizeof(uint32_t) * plan->nd, s);
    if (!st && e == hipSuccess) e = ez;
    if (!st && e == hipSuccess) e = hipStreamSynchronize(s);
    float f = 0.0f, a = 0.0f;
    if (!st && e == hipSuccess) e = hipEventElapsedTime(&f, ev[0], ev[1]);
    if (!st && e == hipSuccess) e = hipEventElapsedTime(&a, ev[2], ev[3]);
    for (auto x : ev) (void)hipEventDestroy(x);
    if (st) return st;
    if (e != hipSuccess) return hip_fail(e, "kernel timing");
    *fwd_ms = f / reps;
    *adj_ms = a / reps;
    return FFRT_OK;
}

ffrt_status ffrt_plan_time_mlp(ffrt_plan* plan, int32_t arch, float* params, float* m, float* v, const int32_t* t,
                               const float* lo, const float* span, float* acts, float* Pz, const float* dL_dP,
                               const ffrt_adam_hparams* hp, int32_t reps, float* fwd_ms, float* bwd_ms,
                               float* upd_ms, void* stream) {
    if (ffrt_status st = mlp_check(plan, arch)) return st;
    if (!params || !m || !v || !t || !lo || !span || !acts || !Pz || !dL_dP || !hp || reps < 1 || !fwd_ms ||
        !bwd_ms || !upd_ms)
        return fail(FFRT_E_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int64_t* po = plan->d_mlpoff(arch);
    auto fwd = [&]() {
        return launch_mlp_forward(arch, plan->P, plan->Q, plan->d_designs(), plan->nd, plan->max_cp, po, params, acts,
                                  lo, span, Pz, nullptr, nullptr, s);
    };
    auto bwd = [&](int part) {
        return launch_mlp_backward(arch, part, plan->P, plan->Q, plan->d_designs(), plan->nd, plan->max_cp, po,
                                   params, acts, span, dL_dP, plan->d_mlpvec(0), plan->d_mlpvec(1),
                                   plan->d_mlpvec(2), nullptr, m, v, t, nullptr, hp, s);
    };
    hipEvent_t ev[6];
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    hipError_t e = fwd();  // one untimed pass of each part
    if (e == hipSuccess) e = bwd(MLP_ALL);
    const int parts[2] = {MLP_BACKPROP, MLP_UPDATE};
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = fwd();
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    for (int k = 0; k < 2; ++k) {
        if (e == hipSuccess) e = hipEventRecord(ev[2 + 2 * k], s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = bwd(parts[k]);
        if (e == hipSuccess) e = hipEventRecord(ev[3 + 2 * k], s);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[5]);
    float ms[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventElapsedTime(&ms[k], ev[2 * k], ev[2 * k + 1]);
    for (auto x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(e, "generator timing");
    *fwd_ms = ms[0] / reps;
    *bwd_ms = ms[1] / reps;
    *upd_ms = ms[2] / reps;
    return FFRT_OK;
}

ffrt_status ffrt_trace_rays(ffrt_plan* plan, int32_t design, const float* Pz, const int64_t* ray_ids, int64_t n,
                            float* out8, void* stream) {
    if (!ready(plan)) return fail(FFRT_E_STATE, "no workspace set");
    if (design < 0 || design >= plan->nd || !Pz || (n > 0 && (!ray_ids || !out8)) || n < 0)
        return fail(FFRT_E_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    if (ffrt_status b = run_bounds(plan, Pz, s)) return b;
    TraceArgs A = make_args(plan, 0, kind_group(plan->dd[design]));  // the forward's LDS layout
    A.Pz = Pz;
    HIP_TRY(plan->ks->trace_rays(A, design, ray_ids, n, out8, s));
    return FFRT_OK;
}

ffrt_status ffrt_lds_atomic_rate(int32_t pattern, int32_t reps, double* atomics_per_s, void* stream) {
    if ((pattern != 0 && pattern != 1) || reps < 1 || !atomics_per_s) return fail(FFRT_E_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = 8 * ncu, iters = 256;
    uint32_t* out = nullptr;
    HIP_TRY(hipMalloc((void**)&out, sizeof(uint32_t) * grid));
    hipEvent_t ev[2];
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    hipError_t e = launch_lds_atomics(pattern, iters, grid, out, s);  // untimed warm-up
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_lds_atomics(pattern, iters, grid, out, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    hipError_t ef = hipStreamSynchronize(s);
    if (ef == hipSuccess) ef = hipFree(out);
    else (void)hipFree(out);
    for (auto x : ev) (void)hipEventDestroy(x);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return hip_fail(e, "LDS atomic timing");
    *atomics_per_s = (double)grid * 256.0 * iters * 9.0 * reps / (ms * 1e-3);
    return FFRT_OK;
}

ffrt_status ffrt_rng(uint64_t seed, uint64_t stream_id, uint64_t first, int64_t n, uint64_t* out, void* stream) {
    if (n < 0 || (n > 0 && !out)) return fail(FFRT_E_ARG, "bad argument");
    HIP_TRY(launch_rng(seed, stream_id, first, n, out, (hipStream_t)stream));
    return FFRT_OK;
}

}  // extern "C"
