// runtime.hip -- host side of liblbimb.so: the C ABI of include/lbimb.h.
//
// The caller hands over one device workspace; the context carves it into the
// population arrays, footprint records, particle arrays and cell list and
// never allocates device memory on the step path.  A step is a fixed sequence
// of kernels on the context's stream; runs of steps replay a captured HIP
// graph of two steps (one A->B->A swap), so small lattices are not
// launch-bound.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbimb.h"
#include "internal.h"

using namespace lbimb;

namespace {

constexpr size_t ALIGN = 256;
constexpr uint64_t SAVE_MAGIC = 0x314d4942494d424cull;  // "LBMIBIM1"

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int store_bytes(int storage) { return storage == LBM_FP64 ? 8 : (storage == LBM_FP32_SHIFTED ? 4 : 2); }

struct Layout {
    int D, Q, Smax;
    int64_t N;
    int P;
    int64_t cell_budget;
    size_t off_fA, off_fB, off_nown, off_slots, off_qr, off_beta, off_arel;
    size_t off_x, off_v, off_w, off_R, off_m, off_I, off_fixed, off_Fh, off_Th, off_Fc, off_bb;
    size_t off_list, off_list_len;
    int list_cap;
    double rmax;
    size_t off_cc, off_cid, off_flags, off_tab, off_stats, off_nl, off_nl_len, off_xb, off_nl_state;
    size_t off_gcount, off_glist, list_buf, total;
};

int validate(const lbm_config *c, std::string &msg) {
    if (!c) { msg = "null config"; return LBM_E_INVALID; }
    if (c->lattice != LBM_D2Q9 && c->lattice != LBM_D3Q19) { msg = "lattice must be D2Q9 or D3Q19"; return LBM_E_INVALID; }
    if (c->storage < LBM_FP64 || c->storage > LBM_FP16_STORE) { msg = "unknown storage"; return LBM_E_INVALID; }
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) { msg = "lattice sizes must be >= 1"; return LBM_E_INVALID; }
    if (c->lattice == LBM_D2Q9 && c->nz != 1) { msg = "D2Q9 needs nz == 1"; return LBM_E_INVALID; }
    if (c->ny > 65535 || c->nz > 65535) { msg = "ny and nz must be <= 65535"; return LBM_E_INVALID; }
    if ((int64_t)c->nx * c->ny * c->nz >= ((int64_t)1 << 40)) { msg = "lattice too large"; return LBM_E_INVALID; }
    if (!(c->tau > 0.5) || !std::isfinite(c->tau)) { msg = "tau must be > 1/2"; return LBM_E_INVALID; }
    if (c->eps_samples < 1 || c->eps_samples > 8) { msg = "eps_samples must be in 1..8"; return LBM_E_INVALID; }
    if (c->eps_mode != LBM_EPS_SAMPLING && c->eps_mode != LBM_EPS_TABLE) { msg = "unknown eps_mode"; return LBM_E_INVALID; }
    if (c->max_particles < 0 || c->max_particles > LBM_MAX_PARTICLES) { msg = "max_particles out of range"; return LBM_E_INVALID; }
    if (!(c->restitution > 0.0 && c->restitution <= 1.0)) { msg = "restitution must be in (0, 1]"; return LBM_E_INVALID; }
    if (!(c->kn >= 0.0)) { msg = "kn must be >= 0"; return LBM_E_INVALID; }
    if (!(c->max_radius <= 62.0) || std::isnan(c->max_radius)) { msg = "max_radius must be <= 62"; return LBM_E_INVALID; }
    for (int a = 0; a < 3; a++)
        if (!std::isfinite(c->fluid_force[a]) || !std::isfinite(c->particle_accel[a])) {
            msg = "non-finite force"; return LBM_E_INVALID;
        }
    return LBM_OK;
}

Layout make_layout(const lbm_config *c) {
    Layout L{};
    L.D = c->lattice == LBM_D2Q9 ? 2 : 3;
    L.Q = c->lattice == LBM_D2Q9 ? 9 : 19;
    L.Smax = L.D == 2 ? c->eps_samples * c->eps_samples : c->eps_samples * c->eps_samples * c->eps_samples;
    L.N = (int64_t)c->nx * c->ny * c->nz;
    L.P = c->max_particles > 0 ? c->max_particles : 1;
    L.cell_budget = std::max<int64_t>(65536, 8 * (int64_t)L.P);
    const size_t fs = (size_t)L.Q * (size_t)L.N * store_bytes(c->storage);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    L.off_fA = take(fs);
    L.off_fB = take(fs);
    // whole aligned 8-byte words: the footprint kernel claims owner slots
    // with 64-bit atomic adds
    L.off_nown = take(((size_t)L.N + 7) / 8 * 8);
    L.off_slots = take((size_t)MAX_OWNERS * L.N * 4);
    L.off_qr = take((size_t)L.N * (c->storage == LBM_FP64 ? sizeof(QRec) : sizeof(QRec32)));
    L.off_beta = take((size_t)(L.Smax + 1) * 8);
    L.off_arel = take((size_t)(L.Smax + 1) * 8);
    const size_t P = (size_t)L.P;
    L.off_x = take(3 * P * 8);
    L.off_v = take(3 * P * 8);
    L.off_w = take(3 * P * 8);
    L.off_R = take(P * 8);
    L.off_m = take(P * 8);
    L.off_I = take(P * 8);
    L.off_fixed = take(P);
    L.off_Fh = take(3 * P * 8);
    L.off_Th = take(3 * P * 8);
    L.off_Fc = take(3 * P * 8);
    // footprint records of two steps (the current and the last completed
    // one: the slab pipeline paints the next footprint before a step ends):
    // bounding boxes, lists of every node of the bounding box of the largest
    // particle, list lengths; buffer k starts k * list_buf bytes after the first
    L.rmax = c->max_radius > 0.0 ? c->max_radius : 8.0;
    const int ext = (int)std::floor(2.0 * L.rmax + 1.0) + 1;
    L.list_cap = L.D == 2 ? ext * ext : ext * ext * ext;
    {
        const size_t o0 = o;
        L.off_bb = take(6 * P * 4);
        L.off_list = take(P * (size_t)L.list_cap * 4);
        L.off_list_len = take(P * 4);
        L.list_buf = o - o0;
        o += L.list_buf;
    }
    L.off_cc = take((size_t)L.cell_budget * 4);
    L.off_cid = take((size_t)L.cell_budget * CELL_CAP * 4);
    L.off_flags = take(64);
    L.off_tab = take((size_t)EPS_TAB_NRHO * EPS_TAB_NT * EPS_TAB_NT * 2);
    // lbm_get_stats: node-pass partials, one row per particle, the totals
    L.off_stats = take(((size_t)STATS_NODE_GROUPS * 4 + P * STATS_PK + 4 + STATS_PK) * 8);
    // neighbour-list mode: lists, build positions, guard state and build count
    L.off_nl = take(P * NL_CAP * 4);
    L.off_nl_len = take(P * 4);
    L.off_xb = take(3 * P * 8);
    L.off_nl_state = take(64);
    // slab pipeline: group counts and lists of two steps
    L.off_gcount = take(2 * PIPE_MAX * 4);
    L.off_glist = take(2 * (size_t)PIPE_MAX * P * 4);
    L.total = o;
    return L;
}

struct TimedEvent {
    int phase;
    hipEvent_t a, b;
};

}  // namespace

struct lbm_ctx {
    lbm_config cfg;
    Layout L;
    char *ws;
    hipStream_t stream;
    hipStream_t cap_stream;
    // the DEM cell list and contact forces run on a side stream beside the
    // footprint, lattice and force kernels (they only read positions and
    // velocities, which change in the integration at the end of the step)
    hipStream_t side_stream;
    static constexpr int GS = 8;  // event slots (steps in flight at once in the pipeline)
    hipEvent_t ev_fork[GS], ev_join[GS], ev_L[GS][PIPE_MAX], ev_P[GS][PIPE_MAX];
    int cur;  // 0: state in fA, 1: state in fB
    int64_t t;
    int np;
    bool particles_set;
    Geom g;
    int ncx, ncy, ncz;
    double ce, arel0;
    double cg[19];
    hipGraphExec_t graph[2];
    bool graph_ok[2];
    int timing;  // 0 off, 1 every phase, 2 the lattice phase only
    int lb_width;  // lattice kernel workgroup width, 0 for the built-in rule
    int lb_order;  // lattice kernel workgroup order, LBM_ORDER_LINEAR / _XCD
    int lb_cu_groups;  // lattice kernel workgroups per CU at most, 0: no cap
    int pipe_req;      // slab pipeline requested: 0 automatic, 1 off, 2..PIPE_MAX slabs
    int pipe_K;        // slabs in use (1: the plain step)
    int nl_every;      // 0: cell list every step; else neighbour lists, rebuilt after nl_every steps at most
    double nl_skin;    // list margin beyond contact
    double prmax;      // largest radius of the current particles
    bool rec_open;
    std::vector<TimedEvent> events;
    size_t ev_used;
    double phase_ms[LBM_NPHASES];
    int64_t phase_n[LBM_NPHASES];
    char err[512];
};

namespace {

template <class T> T *wsp(lbm_ctx *c, size_t off) { return (T *)(c->ws + off); }

thread_local char g_err[512];  // last error of a call that has no context yet

int fail(lbm_ctx *c, int code, const char *fmt, ...) {
    char *dst = c ? c->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    if (c) memcpy(g_err, c->err, sizeof(g_err));
    return code;
}

#define HIPCHK(ctx, expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return fail(ctx, LBM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Particle arrays with the footprint records of buffer `buf` (a step's
// footprint lives in the buffer of its state parity).
Particles particles(lbm_ctx *c, int buf) {
    const size_t fb = (size_t)buf * c->L.list_buf;
    Particles P;
    P.x = wsp<double>(c, c->L.off_x);
    P.v = wsp<double>(c, c->L.off_v);
    P.w = wsp<double>(c, c->L.off_w);
    P.R = wsp<double>(c, c->L.off_R);
    P.m = wsp<double>(c, c->L.off_m);
    P.I = wsp<double>(c, c->L.off_I);
    P.fixed = wsp<uint8_t>(c, c->L.off_fixed);
    P.Fh = wsp<double>(c, c->L.off_Fh);
    P.Th = wsp<double>(c, c->L.off_Th);
    P.Fc = wsp<double>(c, c->L.off_Fc);
    P.bb = wsp<int>(c, c->L.off_bb + fb);
    P.list = wsp<uint32_t>(c, c->L.off_list + fb);
    P.list_len = wsp<int>(c, c->L.off_list_len + fb);
    P.list_cap = c->L.list_cap;
    P.np = c->np;
    return P;
}

void *state(lbm_ctx *c, int which) { return c->ws + (which == 0 ? c->L.off_fA : c->L.off_fB); }

uint32_t *flags(lbm_ctx *c) { return wsp<uint32_t>(c, c->L.off_flags); }

// DEM cell grid for np particles of largest radius rmax: cell edge >= 2 rmax
// (plus the skin in neighbour-list mode, where the lists reach that far), the
// count bounded by the reserved budget.
void cell_grid(const lbm_ctx *c, int np, double rmax, int nc[3]) {
    const double Lb[3] = {c->g.Lx, c->g.Ly, c->g.Lz};
    nc[0] = nc[1] = nc[2] = 1;
    if (np < 1) return;
    const double edge = 2.0 * rmax + (c->nl_every > 0 ? c->nl_skin : 0.0);
    for (int a = 0; a < c->L.D; a++) nc[a] = std::max(1, (int)std::floor(Lb[a] / edge));
    while ((int64_t)nc[0] * nc[1] * nc[2] > c->L.cell_budget)
        for (int a = 0; a < c->L.D; a++) nc[a] = std::max(1, nc[a] / 2);
}

// Checks one particle's radius and state against the context (the rules of
// lbm_set_particles; pos, vel, omega point at its three components): true if
// it passes, else a message in `why`.
bool particle_ok(const lbm_ctx *c, double r, const double *pos, const double *vel,
                 const double *omega, const char *&why) {
    const double Lb[3] = {c->g.Lx, c->g.Ly, c->g.Lz};
    if (!(r > 0.0) || !std::isfinite(r)) { why = "radius must be > 0"; return false; }
    if (r > c->L.rmax) { why = "radius above max_radius"; return false; }
    for (int a = 0; a < 3; a++)
        if ((a < c->L.D || a == 2) && !std::isfinite(omega[a])) { why = "non-finite angular velocity"; return false; }
    for (int a = 0; a < c->L.D; a++) {
        if (!std::isfinite(pos[a]) || !std::isfinite(vel[a])) { why = "non-finite state"; return false; }
        const bool periodic = !(a == 1 && c->g.wall_y);
        if (periodic && (pos[a] < 0.0 || pos[a] >= Lb[a])) { why = "centre outside the periodic box"; return false; }
        if (periodic && 2.0 * r + 2.0 > Lb[a]) { why = "wider than the periodic box"; return false; }
    }
    if (c->g.wall_y && (pos[1] < -0.5 || pos[1] > Lb[1] - 0.5)) { why = "centre beyond a wall"; return false; }
    return true;
}

CellArgs cell_args(lbm_ctx *c) {
    CellArgs a;
    a.P = particles(c, c->cur);  // positions and velocities only
    a.g = c->g;
    a.ncx = c->ncx; a.ncy = c->ncy; a.ncz = c->ncz;
    a.cell_count = wsp<int>(c, c->L.off_cc);
    a.cell_ids = wsp<int>(c, c->L.off_cid);
    a.flags = flags(c);
    a.D = c->L.D;
    a.kn = c->cfg.kn;
    a.ce = c->ce;
    for (int d = 0; d < 3; d++) a.ap[d] = c->cfg.particle_accel[d];
    a.every = c->nl_every;
    a.skin = c->nl_skin;
    a.nl = wsp<int>(c, c->L.off_nl);
    a.nl_len = wsp<int>(c, c->L.off_nl_len);
    a.xb = wsp<double>(c, c->L.off_xb);
    a.nl_state = wsp<int>(c, c->L.off_nl_state);
    a.nl_builds = wsp<int64_t>(c, c->L.off_nl_state + 8);
    a.ncell = (int64_t)c->ncx * c->ncy * c->ncz;
    return a;
}

// Neighbour-list mode: the next step rebuilds (new particles, a new cell grid
// or a mode change); the cell counts start at zero.
hipError_t nl_reset(lbm_ctx *c) {
    hipError_t e = launch_fill_u32(wsp<uint32_t>(c, c->L.off_nl_state), 0u, 4, c->stream);
    if (e == hipSuccess) e = launch_fill_u32(wsp<uint32_t>(c, c->L.off_nl_state), 1u, 1, c->stream);
    if (e == hipSuccess)
        e = launch_fill_u32(wsp<uint32_t>(c, c->L.off_cc), 0u, (int64_t)c->ncx * c->ncy * c->ncz, c->stream);
    return e;
}

// Slab-pipeline groups of the step reading state `from`: this step's group
// lists (filled by the previous step's integration) and the next step's.
Groups groups_of(lbm_ctx *c, int from, int g) {
    Groups G;
    const size_t stride = (size_t)c->L.P;
    int *cnt = wsp<int>(c, c->L.off_gcount);
    int *lst = wsp<int>(c, c->L.off_glist);
    G.count = cnt + from * PIPE_MAX;
    G.list = lst + (size_t)from * PIPE_MAX * stride;
    G.ncount = cnt + (1 - from) * PIPE_MAX;
    G.nlist = lst + (size_t)(1 - from) * PIPE_MAX * stride;
    G.K = c->pipe_K;
    G.g = g;
    G.stride = (int)stride;
    for (int k = 0; k <= PIPE_MAX; k++)
        G.ys[k] = k <= c->pipe_K ? (int)((int64_t)c->g.ny * k / c->pipe_K) : c->g.ny;
    return G;
}

// Footprint arguments painting into buffer `buf`; G.g = -1: every particle.
FootArgs foot_args(lbm_ctx *c, int buf, const Groups &G);
ForceArgs force_args(lbm_ctx *c, int buf, const Groups &G);
void drop_graphs(lbm_ctx *c);

// Slabs of the pipeline for the current particles: 1 (the plain step) without
// walls in y, without particles or when switched off; otherwise the requested
// number (4 when automatic), reduced until every slab is at least
// 2 R_max + 5 rows high (a particle's footprint then spans two slabs at most,
// also after a step of one node).
int resolve_pipe(const lbm_ctx *c) {
    if (!c->g.wall_y || c->np == 0 || c->pipe_req == 1) return 1;
    const int want = c->pipe_req == 0 ? 4 : c->pipe_req;
    const int minh = (int)std::ceil(2.0 * c->prmax) + 5;
    const int k = std::min(want, c->g.ny / std::max(minh, 1));
    return std::max(1, std::min(k, PIPE_MAX));
}

// Brings the footprint of the coming step in line with the slab count
// resolve_pipe gives (stream-ordered on the context's stream).  The pipeline
// paints a step's footprint during the step before, the plain step at its
// start; the owner counts are zero at the start of a plain step.
hipError_t pipe_setup(lbm_ctx *c) {
    const int K = resolve_pipe(c);
    hipError_t e = hipSuccess;
    if (c->pipe_K > 1 && K == 1) {  // painted ahead: forget it
        e = launch_fill_u32(wsp<uint32_t>(c, c->L.off_nown), 0u, (int64_t)((c->L.N + 7) / 8 * 2), c->stream);
    }
    // from the plain step: paint the coming step's footprint; to another
    // slab count: file the particles in the new groups
    const bool paint = K > 1 && c->pipe_K == 1;
    const bool regroup = K > 1 && K != c->pipe_K;
    if (K != c->pipe_K) drop_graphs(c);
    c->pipe_K = K;
    const int from = c->cur;
    if (e == hipSuccess && regroup) {
        const Groups G = groups_of(c, 1 - from, -1);  // its ncount / nlist are step `from`'s lists
        e = launch_fill_u32((uint32_t *)G.ncount, 0u, PIPE_MAX, c->stream);
        if (e == hipSuccess) e = launch_assign_groups(force_args(c, from, G), c->stream);
    }
    if (e == hipSuccess && paint)  // into the buffer of the step's parity
        e = launch_foot_paint(foot_args(c, from, groups_of(c, from, -1)), c->L.D, c->stream);
    return e;
}

FootArgs foot_args(lbm_ctx *c, int buf, const Groups &G) {
    FootArgs a;
    a.G = G;
    a.P = particles(c, buf);
    a.g = c->g;
    a.nown = wsp<uint8_t>(c, c->L.off_nown);
    a.slots = wsp<uint32_t>(c, c->L.off_slots);
    a.S = c->cfg.eps_samples;
    a.flags = flags(c);
    const int D = c->L.D;
    a.tab = c->cfg.eps_mode == LBM_EPS_TABLE ? wsp<uint16_t>(c, c->L.off_tab) : nullptr;
    a.tabH = std::sqrt((double)D) * 0.5;
    a.tabW = 2.0 * a.tabH / (double)EPS_TAB_NRHO;
    a.tabK1 = std::sqrt(2.0) * (double)EPS_TAB_NT;
    a.tabK2 = std::sqrt(3.0) * (double)EPS_TAB_NT;
    return a;
}

// Counts of the eps lookup table for radius R, layout [rho][t1][t2] (t2 only
// in 3D): the entry of a bin is the number of EPS_TAB_M^D reference points of
// the cell centred at the bin centre that lie inside the particle, put on the
// S^D scale with integer rounding (see LBM_EPS_TABLE in the header).
void build_eps_table(int D, int S, double R, std::vector<uint16_t> &tab) {
    const double H = std::sqrt((double)D) * 0.5;
    const double W = 2.0 * H / (double)EPS_TAB_NRHO;
    const double K1 = std::sqrt(2.0) * (double)EPS_TAB_NT, K2 = std::sqrt(3.0) * (double)EPS_TAB_NT;
    const int64_t smax = D == 3 ? (int64_t)S * S * S : (int64_t)S * S;
    const int M = EPS_TAB_M;
    const int64_t mtot = D == 3 ? (int64_t)M * M * M : (int64_t)M * M;
    const int n2 = D == 3 ? EPS_TAB_NT : 1;
    tab.assign((size_t)EPS_TAB_NRHO * EPS_TAB_NT * EPS_TAB_NT, 0);
    double off[EPS_TAB_M];
    for (int k = 0; k < M; k++) off[k] = ((double)k + 0.5) / (double)M - 0.5;
    const double R2 = R * R;
    for (int ir = 0; ir < EPS_TAB_NRHO; ir++)
        for (int i1 = 0; i1 < EPS_TAB_NT; i1++)
            for (int i2 = 0; i2 < n2; i2++) {
                const double rn = R + (-H + ((double)ir + 0.5) * W);
                const double b = ((double)i1 + 0.5) / K1 * rn;
                const double c3 = D == 3 ? ((double)i2 + 0.5) / K2 * rn : 0.0;
                const double a2 = rn * rn - b * b - c3 * c3;
                const double a = a2 > 0.0 ? std::sqrt(a2) : 0.0;
                int64_t kin = 0;
                for (int kz = 0; kz < (D == 3 ? M : 1); kz++)
                    for (int ky = 0; ky < M; ky++)
                        for (int kx = 0; kx < M; kx++) {
                            const double dx = a + off[kx], dy = b + off[ky];
                            double r2 = dx * dx + dy * dy;
                            if (D == 3) {
                                const double dz = c3 + off[kz];
                                r2 = r2 + dz * dz;
                            }
                            if (r2 <= R2) kin++;
                        }
                tab[((size_t)ir * EPS_TAB_NT + i1) * n2 + i2] = (uint16_t)((kin * smax + mtot / 2) / mtot);
            }
}

// Table-lookup eps: one radius (>= 1) for every particle; builds and uploads
// the table for it.
int upload_eps_table(lbm_ctx *c, const double *radius, int np) {
    if (np < 1) return LBM_OK;
    const double R = radius[0];
    for (int p = 1; p < np; p++)
        if (radius[p] != R) return fail(c, LBM_E_INVALID, "table-lookup eps needs one particle radius");
    if (!(R >= 1.0)) return fail(c, LBM_E_INVALID, "table-lookup eps needs a radius of at least 1");
    std::vector<uint16_t> tab;
    build_eps_table(c->L.D, c->cfg.eps_samples, R, tab);
    HIPCHK(c, hipMemcpy(wsp<uint16_t>(c, c->L.off_tab), tab.data(), tab.size() * 2, hipMemcpyHostToDevice));
    return LBM_OK;
}

LBArgs lb_args(lbm_ctx *c, int from) {
    LBArgs a;
    a.A = state(c, from);
    a.B = state(c, 1 - from);
    a.nown = wsp<uint8_t>(c, c->L.off_nown);
    a.slots = wsp<uint32_t>(c, c->L.off_slots);
    a.beta_tab = wsp<double>(c, c->L.off_beta);
    a.arel_tab = wsp<double>(c, c->L.off_arel);
    a.qr = wsp<char>(c, c->L.off_qr);
    a.px = wsp<double>(c, c->L.off_x);
    a.pv = wsp<double>(c, c->L.off_v);
    a.pw = wsp<double>(c, c->L.off_w);
    a.np = c->np;
    a.g = c->g;
    a.Smax = c->L.Smax;
    a.arel0 = c->arel0;
    for (int i = 0; i < 19; i++) {
        a.cg[i] = c->cg[i];
        a.cgf[i] = (float)c->cg[i];
    }
    a.arel0f = (float)c->arel0;
    a.tauf = (float)c->cfg.tau;
    a.flags = flags(c);
    a.y0 = 0;
    a.ny_run = c->g.ny;
    return a;
}

// Force-kernel arguments reading the footprint of buffer `buf`.
ForceArgs force_args(lbm_ctx *c, int buf, const Groups &G) {
    ForceArgs fo;
    fo.P = particles(c, buf);
    fo.g = c->g;
    fo.qr = wsp<char>(c, c->L.off_qr);
    fo.rec32 = c->cfg.storage != LBM_FP64;
    fo.D = c->L.D;
    fo.integrate = 1;
    for (int d = 0; d < 3; d++) fo.ap[d] = c->cfg.particle_accel[d];
    fo.flags = flags(c);
    fo.G = G;
    return fo;
}

// Phase markers for the timing mode.
void phase_begin(lbm_ctx *c, int phase, hipStream_t s) {
    c->rec_open = c->timing == 1 || (c->timing == 2 && phase == 1);
    if (!c->rec_open) return;
    if (c->ev_used == c->events.size()) {
        TimedEvent e{};
        (void)hipEventCreate(&e.a);
        (void)hipEventCreate(&e.b);
        c->events.push_back(e);
    }
    c->events[c->ev_used].phase = phase;
    (void)hipEventRecord(c->events[c->ev_used].a, s);
}

void phase_end(lbm_ctx *c, hipStream_t s) {
    if (!c->rec_open) return;
    c->rec_open = false;
    (void)hipEventRecord(c->events[c->ev_used].b, s);
    c->ev_used++;
}

// Queue one complete time step reading state `from` (the plain schedule):
// footprint, lattice, force and integration on stream s, the DEM on the side
// stream joined before the force kernel.  `slot` selects the step's events
// (up to GS steps are captured per graph).
hipError_t enqueue_plain(lbm_ctx *c, int from, hipStream_t s, int slot) {
    hipError_t e;
    const int lattice = c->cfg.lattice, storage = c->cfg.storage;
    if (c->np > 0) {
        CellArgs ca = cell_args(c);
        hipStream_t d = c->side_stream;
        if ((e = hipEventRecord(c->ev_fork[slot], s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(d, c->ev_fork[slot], 0)) != hipSuccess) return e;
        phase_begin(c, 3, d);
        if ((e = c->nl_every > 0 ? launch_nl_rebuild(ca, d) : launch_cells(ca, d)) != hipSuccess) return e;
        phase_end(c, d);
        phase_begin(c, 4, d);
        if ((e = c->nl_every > 0 ? launch_nl_contacts(ca, d) : launch_dem(ca, d)) != hipSuccess) return e;
        phase_end(c, d);
        if ((e = hipEventRecord(c->ev_join[slot], d)) != hipSuccess) return e;
        FootArgs fa = foot_args(c, from, groups_of(c, from, -1));
        phase_begin(c, 0, s);
        if ((e = launch_foot_paint(fa, c->L.D, s)) != hipSuccess) return e;
        phase_end(c, s);
    }
    phase_begin(c, 1, s);
    if ((e = launch_lb(lattice, storage, lb_args(c, from), c->lb_width, c->lb_order, c->lb_cu_groups, s)) != hipSuccess) return e;
    phase_end(c, s);
    if (c->np > 0) {
        ForceArgs fo = force_args(c, from, groups_of(c, from, -1));
        // the force kernel integrates: it needs the contact forces; the cell
        // list and the contacts overlap the footprint and lattice kernels
        if ((e = hipStreamWaitEvent(s, c->ev_join[slot], 0)) != hipSuccess) return e;
        phase_begin(c, 2, s);
        if ((e = launch_force(fo, s)) != hipSuccess) return e;
        phase_end(c, s);
    }
    return hipSuccess;
}

// Queue one time step of the slab pipeline (walls in y, K slabs) on two
// streams.  Stream s runs the lattice slabs in order; slab k of step t waits
// for the particle groups k and k + 1 of step t - 1 (their new footprints lie
// in slabs up to k + 1; slab k rewrites rows that the step-(t - 1) slabs
// k - 1 .. k + 1 read, which stream order already covers).  The side stream
// runs, in order, the DEM of step t (it needs every particle's position at t:
// the last group of step t - 1 precedes it on this stream) and then each
// group g (force and torque sums of step t, integration, filing into the
// next step's groups, footprint of step t + 1) once slab g is done (slab
// g - 1 precedes it on s).  `first`: no step of this schedule is pending (the
// side stream then also waits for the work queued on s before the step);
// `last`: join the side stream back into s at the end.  The footprint of step
// t was painted by step t - 1 (or by the set-up) into buffer `from`.
hipError_t enqueue_pipe(lbm_ctx *c, int from, hipStream_t s, int slot, bool first, bool last) {
    hipError_t e;
    const int K = c->pipe_K;
    const int prev = (slot + lbm_ctx::GS - 1) % lbm_ctx::GS;
    hipStream_t d = c->side_stream;
    const int lattice = c->cfg.lattice, storage = c->cfg.storage;
    if (first) {
        if ((e = hipEventRecord(c->ev_fork[slot], s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(d, c->ev_fork[slot], 0)) != hipSuccess) return e;
    }
    CellArgs ca = cell_args(c);
    phase_begin(c, 3, d);
    if ((e = c->nl_every > 0 ? launch_nl_rebuild(ca, d) : launch_cells(ca, d)) != hipSuccess) return e;
    phase_end(c, d);
    phase_begin(c, 4, d);
    if ((e = c->nl_every > 0 ? launch_nl_contacts(ca, d) : launch_dem(ca, d)) != hipSuccess) return e;
    phase_end(c, d);
    // the next step's groups are filed from empty (after the previous step's
    // groups, which read these counts, on this stream)
    const Groups G0 = groups_of(c, from, -1);
    if ((e = launch_fill_u32((uint32_t *)G0.ncount, 0u, PIPE_MAX, d)) != hipSuccess) return e;
    for (int k = 0; k < K; k++) {
        if (!first) {
            if ((e = hipStreamWaitEvent(s, c->ev_P[prev][k], 0)) != hipSuccess) return e;
            if (k + 1 < K && (e = hipStreamWaitEvent(s, c->ev_P[prev][k + 1], 0)) != hipSuccess) return e;
        }
        LBArgs la = lb_args(c, from);
        la.y0 = G0.ys[k];
        la.ny_run = G0.ys[k + 1] - G0.ys[k];
        phase_begin(c, 1, s);
        if ((e = launch_lb(lattice, storage, la, c->lb_width, c->lb_order, c->lb_cu_groups, s)) != hipSuccess)
            return e;
        phase_end(c, s);
        if ((e = hipEventRecord(c->ev_L[slot][k], s)) != hipSuccess) return e;
    }
    for (int g = 0; g < K; g++) {
        if ((e = hipStreamWaitEvent(d, c->ev_L[slot][g], 0)) != hipSuccess) return e;
        const Groups G = groups_of(c, from, g);
        ForceArgs fo = force_args(c, from, G);
        phase_begin(c, 2, d);
        if ((e = launch_force(fo, d)) != hipSuccess) return e;
        phase_end(c, d);
        FootArgs fa = foot_args(c, 1 - from, G);
        phase_begin(c, 0, d);
        if ((e = launch_foot_paint(fa, c->L.D, d)) != hipSuccess) return e;
        phase_end(c, d);
        if ((e = hipEventRecord(c->ev_P[slot][g], d)) != hipSuccess) return e;
    }
    if (last) {
        if ((e = hipEventRecord(c->ev_join[slot], d)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, c->ev_join[slot], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t enqueue_step(lbm_ctx *c, int from, hipStream_t s, int slot, bool first, bool last) {
    if (c->pipe_K > 1 && c->np > 0) return enqueue_pipe(c, from, s, slot, first, last);
    return enqueue_plain(c, from, s, slot);
}

// The step events (fork/join, lattice slabs, particle groups) of every
// slot; events that were not created are null.
bool create_step_events(lbm_ctx *c) {
    bool ok = true;
    auto mk = [&](hipEvent_t &ev) {
        ev = nullptr;
        if (ok) ok = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    };
    for (int k = 0; k < lbm_ctx::GS; k++) {
        mk(c->ev_fork[k]);
        mk(c->ev_join[k]);
        for (int g = 0; g < PIPE_MAX; g++) {
            mk(c->ev_L[k][g]);
            mk(c->ev_P[k][g]);
        }
    }
    return ok;
}

void destroy_step_events(lbm_ctx *c) {
    auto rm = [](hipEvent_t ev) { if (ev) (void)hipEventDestroy(ev); };
    for (int k = 0; k < lbm_ctx::GS; k++) {
        rm(c->ev_fork[k]);
        rm(c->ev_join[k]);
        for (int g = 0; g < PIPE_MAX; g++) {
            rm(c->ev_L[k][g]);
            rm(c->ev_P[k][g]);
        }
    }
}

void drop_graphs(lbm_ctx *c) {
    for (int k = 0; k < 2; k++) {
        if (c->graph_ok[k]) (void)hipGraphExecDestroy(c->graph[k]);
        c->graph_ok[k] = false;
    }
}

// Steps per captured graph of the plain schedule (one A -> B -> A swap, so the
// state parity returns to `from`).
constexpr int GRAPH_STEPS = 2;

int build_graph(lbm_ctx *c, int from) {
    hipGraph_t graph;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = hipSuccess;
    for (int k = 0; k < GRAPH_STEPS && e1 == hipSuccess; k++)
        e1 = enqueue_plain(c, (from + k) & 1, c->cap_stream, k);
    hipError_t e3 = hipStreamEndCapture(c->cap_stream, &graph);
    if (e1 != hipSuccess) return fail(c, LBM_E_HIP, "graph capture: %s", hipGetErrorString(e1));
    if (e3 != hipSuccess) return fail(c, LBM_E_HIP, "graph capture end: %s", hipGetErrorString(e3));
    hipError_t e4 = hipGraphInstantiate(&c->graph[from], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e4 != hipSuccess) return fail(c, LBM_E_HIP, "graph instantiate: %s", hipGetErrorString(e4));
    c->graph_ok[from] = true;
    return LBM_OK;
}

int check_flags(lbm_ctx *c) {
    uint32_t h[4] = {0, 0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(h, flags(c), sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h[0] & FLAG_SLOT_OVERFLOW)
        return fail(c, LBM_E_SLOT_OVERFLOW, "more than %d particles cover one node", MAX_OWNERS);
    if (h[0] & FLAG_CELL_OVERFLOW)
        return fail(c, LBM_E_CELL_OVERFLOW, "a DEM cell holds more than %d particles", CELL_CAP);
    if (h[0] & FLAG_CONTACT_OVERFLOW)
        return fail(c, LBM_E_CONTACT_OVERFLOW, "a particle has more than %d contacts", MAX_CONTACTS);
    if (h[0] & FLAG_NONFINITE) return fail(c, LBM_E_NONFINITE, "non-finite value in the state or a particle outside the box");
    if (h[0] & FLAG_FAST)
        return fail(c, LBM_E_NONFINITE, "a particle moved more than one node in y in one step (slab pipeline)");
    return LBM_OK;
}

// Runs `produce` into a device buffer (the caller's when ptr_kind is device,
// else a temporary) and copies to the host when needed.
template <class F>
int produce_to(lbm_ctx *c, void *out, size_t bytes, int kind, F produce) {
    if (kind != LBM_HOST && kind != LBM_DEVICE) return fail(c, LBM_E_INVALID, "bad ptr_kind");
    if (!out) return fail(c, LBM_E_INVALID, "null output");
    if (kind == LBM_DEVICE) {
        HIPCHK(c, produce(out));
        return LBM_OK;
    }
    void *tmp = nullptr;
    HIPCHK(c, hipMalloc(&tmp, bytes));
    hipError_t e = produce(tmp);
    if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(c, LBM_E_HIP, "%s", hipGetErrorString(e));
    return LBM_OK;
}


}  // namespace

// ====================================================================== ABI
extern "C" {

const char *lbm_error_string(int code) {
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_E_INVALID: return "invalid argument";
        case LBM_E_NOMEM: return "workspace too small";
        case LBM_E_HIP: return "HIP runtime error";
        case LBM_E_NONFINITE: return "non-finite value in the state or a particle outside the box";
        case LBM_E_SLOT_OVERFLOW: return "too many particles cover one node";
        case LBM_E_STATE: return "call out of order";
        case LBM_E_IO: return "file error";
        case LBM_E_CELL_OVERFLOW: return "DEM cell capacity exceeded";
        case LBM_E_CONTACT_OVERFLOW: return "too many contacts on one particle";
        default: return "unknown error";
    }
}

const char *lbm_last_error(const lbm_ctx *ctx) { return ctx ? ctx->err : g_err; }

int lbm_workspace_bytes(const lbm_config *cfg, size_t *bytes) {
    std::string msg;
    int rc = validate(cfg, msg);
    if (rc != LBM_OK) return rc;
    if (!bytes) return LBM_E_INVALID;
    *bytes = make_layout(cfg).total;
    return LBM_OK;
}

int lbm_create(const lbm_config *cfg, void *workspace, size_t ws_bytes, void *hip_stream,
               lbm_ctx **out) {
    if (!out) return LBM_E_INVALID;
    *out = nullptr;
    std::string msg;
    int rc = validate(cfg, msg);
    if (rc != LBM_OK) return fail(nullptr, rc, "%s", msg.c_str());
    Layout L = make_layout(cfg);
    if (!workspace || ws_bytes < L.total)
        return fail(nullptr, LBM_E_NOMEM, "workspace of %zu bytes needed", L.total);
    if (((uintptr_t)workspace) % ALIGN != 0) return fail(nullptr, LBM_E_INVALID, "workspace must be 256-byte aligned");
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    c->cfg = *cfg;
    c->L = L;
    c->ws = (char *)workspace;
    c->stream = (hipStream_t)hip_stream;
    c->cur = 0;
    c->t = 0;
    c->np = 0;
    c->particles_set = false;
    c->g.nx = cfg->nx; c->g.ny = cfg->ny; c->g.nz = cfg->nz;
    c->g.wall_y = cfg->wall_y ? 1 : 0;
    c->g.N = L.N;
    c->g.Lx = (double)cfg->nx; c->g.Ly = (double)cfg->ny; c->g.Lz = (double)cfg->nz;
    c->ncx = c->ncy = c->ncz = 1;
    const double le = std::log(cfg->restitution);
    c->ce = -2.0 * le / std::sqrt(M_PI * M_PI + le * le);
    c->arel0 = (1.0 - 0.0) / cfg->tau;
    // c_i . g_fluid in the direction order of the lattice
    const int *cx = cfg->lattice == LBM_D2Q9 ? D2Q9::cx : D3Q19::cx;
    const int *cy = cfg->lattice == LBM_D2Q9 ? D2Q9::cy : D3Q19::cy;
    const int *cz = cfg->lattice == LBM_D2Q9 ? D2Q9::cz : D3Q19::cz;
    for (int i = 0; i < 19; i++) c->cg[i] = 0.0;
    for (int i = 0; i < L.Q; i++) {
        double v = (double)cx[i] * cfg->fluid_force[0] + (double)cy[i] * cfg->fluid_force[1];
        if (L.D == 3) v = v + (double)cz[i] * cfg->fluid_force[2];
        c->cg[i] = v;
    }
    c->graph_ok[0] = c->graph_ok[1] = false;
    c->timing = 0;
    c->lb_width = 0;
    c->lb_order = LBM_ORDER_LINEAR;
    c->lb_cu_groups = 0;
    c->nl_every = 0;
    c->nl_skin = 1.0;
    c->prmax = 0.0;
    c->pipe_req = 1;  // off: measured slower than the plain step on MI355X
    c->pipe_K = 1;
    c->rec_open = false;
    c->ev_used = 0;
    for (int k = 0; k < LBM_NPHASES; k++) { c->phase_ms[k] = 0.0; c->phase_n[k] = 0; }
    c->err[0] = 0;
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(nullptr, LBM_E_HIP, "hipStreamCreateWithFlags failed");
    }
    if (hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(c->cap_stream);
        delete c;
        return fail(nullptr, LBM_E_HIP, "hipStreamCreateWithFlags failed");
    }
    if (!create_step_events(c)) {
        destroy_step_events(c);
        (void)hipStreamDestroy(c->side_stream);
        (void)hipStreamDestroy(c->cap_stream);
        delete c;
        return fail(nullptr, LBM_E_HIP, "hipEventCreateWithFlags failed");
    }
    // beta(eps) (Eq. 2) and (1 - beta)/tau for every possible clamped count
    std::vector<double> beta(L.Smax + 1), arel(L.Smax + 1);
    const double tau = cfg->tau;
    for (int k = 0; k <= L.Smax; k++) {
        const double eps = (double)k / (double)L.Smax;
        beta[k] = eps * (tau - 0.5) / ((1.0 - eps) + (tau - 0.5));
        arel[k] = (1.0 - beta[k]) / tau;
    }
    int r = LBM_OK;
    auto chk = [&](hipError_t e) { if (e != hipSuccess && r == LBM_OK) r = fail(c, LBM_E_HIP, "%s", hipGetErrorString(e)); };
    chk(hipMemcpyAsync(wsp<double>(c, L.off_beta), beta.data(), beta.size() * 8, hipMemcpyHostToDevice, c->stream));
    chk(hipMemcpyAsync(wsp<double>(c, L.off_arel), arel.data(), arel.size() * 8, hipMemcpyHostToDevice, c->stream));
    chk(launch_fill_u32(wsp<uint32_t>(c, L.off_nown), 0u, (int64_t)((L.N + 7) / 8 * 2), c->stream));
    chk(launch_fill_u32(wsp<uint32_t>(c, L.off_flags), 0u, 16, c->stream));
    chk(launch_fill_u32(wsp<uint32_t>(c, L.off_qr), 0u,
                        (int64_t)L.N * (int64_t)((cfg->storage == LBM_FP64 ? sizeof(QRec) : sizeof(QRec32)) / 4),
                        c->stream));
    // fluid at rest: f = f^eq(1, 0) = w_i  (shifted storage: g = 0)
    {
        const int Q = L.Q;
        if (cfg->storage == LBM_FP64) {
            // f^eq_i(1, 0) = w_i exactly (c.u = 0, u.u = 0)
            chk(launch_fill_rest_f64(cfg->lattice, c->g, wsp<double>(c, L.off_fA), c->stream));
        } else {
            const size_t bytes = (size_t)Q * L.N * store_bytes(cfg->storage);
            chk(launch_fill_u32(wsp<uint32_t>(c, L.off_fA), 0u, (int64_t)((bytes + 3) / 4), c->stream));
        }
    }
    chk(hipStreamSynchronize(c->stream));
    if (r != LBM_OK) {
        destroy_step_events(c);
        (void)hipStreamDestroy(c->side_stream);
        (void)hipStreamDestroy(c->cap_stream);
        delete c;
        return r;  // message already in the thread's last error
    }
    *out = c;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (auto &e : c->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    (void)hipStreamSynchronize(c->side_stream);
    destroy_step_events(c);
    (void)hipStreamDestroy(c->side_stream);
    (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

int lbm_set_particles(lbm_ctx *c, int64_t n, const double *pos, const double *vel,
                      const double *omega, const double *radius, const double *rho_s,
                      const uint8_t *fixed, int ptr_kind) {
    if (!c) return LBM_E_INVALID;
    if (ptr_kind != LBM_HOST) return fail(c, LBM_E_INVALID, "lbm_set_particles takes host pointers");
    if (n < 0 || n > c->cfg.max_particles) return fail(c, LBM_E_INVALID, "particle count %lld out of range", (long long)n);
    if (n > 0 && (!pos || !vel || !omega || !radius || !rho_s))
        return fail(c, LBM_E_INVALID, "null particle array");
    const int D = c->L.D;
    const double Lb[3] = {c->g.Lx, c->g.Ly, c->g.Lz};
    double rmax = 0.0;
    const int P = (int)n;
    for (int p = 0; p < P; p++) {
        const char *why = "";
        if (!particle_ok(c, radius[p], pos + 3 * p, vel + 3 * p, omega + 3 * p, why))
            return fail(c, LBM_E_INVALID, "particle %d: %s", p, why);
        if (!(rho_s[p] > 0.0) || !std::isfinite(rho_s[p]))
            return fail(c, LBM_E_INVALID, "particle %d: density must be > 0", p);
        rmax = std::max(rmax, radius[p]);
    }
    if (c->cfg.eps_mode == LBM_EPS_TABLE) {
        const int r = upload_eps_table(c, radius, P);
        if (r != LBM_OK) return r;
    }
    int nc[3];
    cell_grid(c, P, rmax, nc);
    // overlap check on the host with the same cell grid
    if (P > 1) {
        const int ncell = nc[0] * nc[1] * nc[2];
        std::vector<int> head(ncell, -1), next(P, -1);
        auto cellof = [&](int p, int a) {
            double t = pos[3 * p + a];
            if (a == 1 && c->g.wall_y) t = t + 0.5;
            int k = (int)std::floor(t * (double)nc[a] / Lb[a]);
            return k < 0 ? 0 : (k >= nc[a] ? nc[a] - 1 : k);
        };
        for (int p = 0; p < P; p++) {
            int ci[3] = {cellof(p, 0), cellof(p, 1), D == 3 ? cellof(p, 2) : 0};
            const int id = ci[0] + nc[0] * (ci[1] + nc[1] * ci[2]);
            next[p] = head[id];
            head[id] = p;
        }
        for (int p = 0; p < P; p++) {
            int ci[3] = {cellof(p, 0), cellof(p, 1), D == 3 ? cellof(p, 2) : 0};
            for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        int cc[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
                        bool skip = false;
                        for (int a = 0; a < 3; a++) {
                            if (a == 1 && c->g.wall_y) { if (cc[a] < 0 || cc[a] >= nc[a]) skip = true; }
                            else cc[a] = ((cc[a] % nc[a]) + nc[a]) % nc[a];
                        }
                        if (skip) continue;
                        for (int q = head[cc[0] + nc[0] * (cc[1] + nc[1] * cc[2])]; q >= 0; q = next[q]) {
                            if (q <= p) continue;
                            double d2 = 0.0;
                            for (int a = 0; a < D; a++) {
                                double d = pos[3 * p + a] - pos[3 * q + a];
                                if (!(a == 1 && c->g.wall_y)) {
                                    if (d > 0.5 * Lb[a]) d -= Lb[a];
                                    else if (d < -0.5 * Lb[a]) d += Lb[a];
                                }
                                d2 += d * d;
                            }
                            const double lim = radius[p] + radius[q] - 0.5 * std::min(radius[p], radius[q]);
                            if (d2 < lim * lim)
                                return fail(c, LBM_E_INVALID, "particles %d and %d overlap by more than half a radius", p, q);
                        }
                    }
        }
    }
    const size_t Pc = (size_t)c->L.P;
    std::vector<double> X(3 * Pc, 0.0), V(3 * Pc, 0.0), W(3 * Pc, 0.0), R(Pc, 0.0), M(Pc, 0.0), I(Pc, 0.0);
    std::vector<uint8_t> F(Pc, 0);
    for (int p = 0; p < P; p++) {
        for (int a = 0; a < 3; a++) {
            const bool used = a < D;
            X[a * Pc + p] = used ? pos[3 * p + a] : 0.0;
            V[a * Pc + p] = used ? vel[3 * p + a] : 0.0;
            W[a * Pc + p] = (D == 3 || a == 2) ? omega[3 * p + a] : 0.0;
        }
        const double r = radius[p];
        R[p] = r;
        if (D == 2) {
            M[p] = rho_s[p] * (M_PI * r * r);
            I[p] = 0.5 * M[p] * r * r;
        } else {
            M[p] = rho_s[p] * (4.0 / 3.0 * M_PI * r * r * r);
            I[p] = 0.4 * M[p] * r * r;
        }
        F[p] = fixed ? (fixed[p] ? 1 : 0) : 0;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    // particle arrays are [3][np] on the device: compact to the actual count
    const size_t np = (size_t)std::max(P, 1);
    std::vector<double> Xc(3 * np, 0.0), Vc(3 * np, 0.0), Wc(3 * np, 0.0);
    for (int a = 0; a < 3; a++)
        for (int p = 0; p < P; p++) {
            Xc[a * np + p] = X[a * Pc + p];
            Vc[a * np + p] = V[a * Pc + p];
            Wc[a * np + p] = W[a * Pc + p];
        }
    c->np = P;
    HIPCHK(c, hipMemcpy(wsp<double>(c, c->L.off_x), Xc.data(), 3 * np * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(wsp<double>(c, c->L.off_v), Vc.data(), 3 * np * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(wsp<double>(c, c->L.off_w), Wc.data(), 3 * np * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(wsp<double>(c, c->L.off_R), R.data(), np * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(wsp<double>(c, c->L.off_m), M.data(), np * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(wsp<double>(c, c->L.off_I), I.data(), np * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(wsp<uint8_t>(c, c->L.off_fixed), F.data(), np, hipMemcpyHostToDevice));
    c->ncx = nc[0]; c->ncy = nc[1]; c->ncz = nc[2];
    c->prmax = rmax;
    HIPCHK(c, nl_reset(c));
    // forget the old footprint, then record bounding boxes for the first clear
    HIPCHK(c, launch_fill_u32(wsp<uint32_t>(c, c->L.off_nown), 0u, (int64_t)((c->L.N + 7) / 8 * 2), c->stream));
    HIPCHK(c, launch_fill_u32(wsp<uint32_t>(c, c->L.off_Fh), 0u, (int64_t)(3 * np * 2), c->stream));
    HIPCHK(c, launch_fill_u32(wsp<uint32_t>(c, c->L.off_Th), 0u, (int64_t)(3 * np * 2), c->stream));
    HIPCHK(c, launch_fill_u32(wsp<uint32_t>(c, c->L.off_Fc), 0u, (int64_t)(3 * np * 2), c->stream));
    for (int b = 0; b < 2; b++)
        HIPCHK(c, launch_fill_u32(wsp<uint32_t>(c, c->L.off_list_len + (size_t)b * c->L.list_buf), 0u,
                                  (int64_t)np, c->stream));
    // a new particle set starts with clear health flags
    HIPCHK(c, launch_fill_u32(flags(c), 0u, 16, c->stream));
    c->particles_set = true;
    c->pipe_K = 1;  // the footprint is forgotten: set the pipeline up afresh
    HIPCHK(c, pipe_setup(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_set_distributions(lbm_ctx *c, const double *f, int ptr_kind) {
    if (!c || !f) return LBM_E_INVALID;
    const size_t bytes = (size_t)c->L.Q * c->L.N * 8;
    const double *src = f;
    void *tmp = nullptr;
    if (ptr_kind == LBM_HOST) {
        HIPCHK(c, hipMalloc(&tmp, bytes));
        hipError_t e = hipMemcpy(tmp, f, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) { (void)hipFree(tmp); return fail(c, LBM_E_HIP, "%s", hipGetErrorString(e)); }
        src = (const double *)tmp;
    } else if (ptr_kind != LBM_DEVICE) {
        return fail(c, LBM_E_INVALID, "bad ptr_kind");
    }
    hipError_t e = launch_set_f(c->cfg.lattice, c->cfg.storage, c->g, src, state(c, c->cur), c->stream);
    if (e == hipSuccess && tmp) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return fail(c, LBM_E_HIP, "%s", hipGetErrorString(e));
    return LBM_OK;
}

int lbm_get_distributions(lbm_ctx *c, double *f, int ptr_kind) {
    if (!c) return LBM_E_INVALID;
    const size_t bytes = (size_t)c->L.Q * c->L.N * 8;
    return produce_to(c, f, bytes, ptr_kind, [&](void *dst) {
        return launch_get_f(c->cfg.lattice, c->cfg.storage, c->g, state(c, c->cur), (double *)dst, c->stream);
    });
}

int lbm_get_macro(lbm_ctx *c, double *rho, double *u, int ptr_kind) {
    if (!c || !rho || !u) return LBM_E_INVALID;
    const int64_t N = c->L.N;
    if (ptr_kind == LBM_DEVICE) {
        HIPCHK(c, launch_macro(c->cfg.lattice, c->cfg.storage, c->g, state(c, c->cur), rho, u, c->stream));
        return LBM_OK;
    }
    if (ptr_kind != LBM_HOST) return fail(c, LBM_E_INVALID, "bad ptr_kind");
    void *tmp = nullptr;
    const size_t bytes = (size_t)(1 + c->L.D) * N * 8;
    HIPCHK(c, hipMalloc(&tmp, bytes));
    double *dr = (double *)tmp, *du = dr + N;
    hipError_t e = launch_macro(c->cfg.lattice, c->cfg.storage, c->g, state(c, c->cur), dr, du, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(rho, dr, N * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(u, du, (size_t)c->L.D * N * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(c, LBM_E_HIP, "%s", hipGetErrorString(e));
    return LBM_OK;
}

int lbm_get_q(lbm_ctx *c, double *q, int ptr_kind) {
    if (!c) return LBM_E_INVALID;
    const size_t bytes = (size_t)c->L.D * c->L.N * 8;
    return produce_to(c, q, bytes, ptr_kind, [&](void *dst) {
        ForceArgs fo;
        fo.P = particles(c, 1 - c->cur);  // the last completed step's footprint
        fo.g = c->g;
        fo.qr = wsp<char>(c, c->L.off_qr);
        fo.rec32 = c->cfg.storage != LBM_FP64;
        fo.D = c->L.D;
        fo.integrate = 0;
        return launch_list_q(fo, (double *)dst, c->stream);
    });
}

static int get_particle_vec(lbm_ctx *c, size_t off, double *out, int ptr_kind) {
    // device layout [3][np] -> caller layout [np][3]
    const int P = c->np;
    if (P == 0) return LBM_OK;
    std::vector<double> h(3 * (size_t)P);
    HIPCHK(c, hipMemcpyAsync(h.data(), wsp<double>(c, off), h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<double> t(3 * (size_t)P);
    for (int p = 0; p < P; p++)
        for (int a = 0; a < 3; a++) t[3 * p + a] = h[(size_t)a * P + p];
    if (ptr_kind == LBM_HOST) {
        memcpy(out, t.data(), t.size() * 8);
    } else if (ptr_kind == LBM_DEVICE) {
        HIPCHK(c, hipMemcpyAsync(out, t.data(), t.size() * 8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        return fail(c, LBM_E_INVALID, "bad ptr_kind");
    }
    return LBM_OK;
}

int lbm_get_forces(lbm_ctx *c, double *F, double *T, int ptr_kind) {
    if (!c || (c->np > 0 && (!F || !T))) return LBM_E_INVALID;
    int r = get_particle_vec(c, c->L.off_Fh, F, ptr_kind);
    if (r != LBM_OK) return r;
    return get_particle_vec(c, c->L.off_Th, T, ptr_kind);
}

int lbm_get_contact_forces(lbm_ctx *c, double *Fc, int ptr_kind) {
    if (!c || (c->np > 0 && !Fc)) return LBM_E_INVALID;
    return get_particle_vec(c, c->L.off_Fc, Fc, ptr_kind);
}

int lbm_get_particles(lbm_ctx *c, double *pos, double *vel, double *omega, int ptr_kind) {
    if (!c || (c->np > 0 && (!pos || !vel || !omega))) return LBM_E_INVALID;
    int r = get_particle_vec(c, c->L.off_x, pos, ptr_kind);
    if (r == LBM_OK) r = get_particle_vec(c, c->L.off_v, vel, ptr_kind);
    if (r == LBM_OK) r = get_particle_vec(c, c->L.off_w, omega, ptr_kind);
    return r;
}

int64_t lbm_time(const lbm_ctx *c) { return c ? c->t : -1; }

int64_t lbm_particle_count(const lbm_ctx *c) { return c ? c->np : -1; }

int lbm_step(lbm_ctx *c, int64_t nsteps) {
    if (!c || nsteps < 0) return LBM_E_INVALID;
    if (!c->particles_set)
        return fail(c, LBM_E_STATE, "lbm_step before lbm_set_particles (n may be 0) or lbm_load");
    if (nsteps == 0) return LBM_OK;
    hipError_t e;
    constexpr int GS = lbm_ctx::GS;
    // steps queued one by one (timing mode, or the steps beyond whole graphs)
    auto eager = [&](int64_t n) -> int {
        for (int64_t k = 0; k < n; k++) {
            if ((e = enqueue_step(c, c->cur, c->stream, (int)(k % GS), k == 0, k == n - 1)) != hipSuccess)
                return fail(c, LBM_E_HIP, "step: %s", hipGetErrorString(e));
            c->cur ^= 1;
            c->t++;
        }
        return LBM_OK;
    };
    // The slab pipeline always launches step by step: its three-stream
    // schedule is not captured as a graph (its capture crashed the host
    // runtime once and is switched off); a step's launches take far less host
    // time than the step takes on the GPU, so the queue stays ahead.
    if (c->timing || (c->pipe_K > 1 && c->np > 0)) {
        const int r = eager(nsteps);
        if (r != LBM_OK) return r;
        return check_flags(c);
    }
    int64_t left = nsteps;
    if (left >= GRAPH_STEPS) {
        if (!c->graph_ok[c->cur]) {
            int r = build_graph(c, c->cur);
            if (r != LBM_OK) return r;
        }
        const int64_t reps = left / GRAPH_STEPS;
        for (int64_t k = 0; k < reps; k++)
            if ((e = hipGraphLaunch(c->graph[c->cur], c->stream)) != hipSuccess)
                return fail(c, LBM_E_HIP, "graph launch: %s", hipGetErrorString(e));
        c->t += GRAPH_STEPS * reps;
        left -= GRAPH_STEPS * reps;
    }
    const int r = eager(left);
    if (r != LBM_OK) return r;
    return check_flags(c);
}

int lbm_set_timing(lbm_ctx *c, int enable) {
    if (!c) return LBM_E_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (enable < 0 || enable > 2) return LBM_E_INVALID;
    c->timing = enable;
    c->ev_used = 0;
    for (int k = 0; k < LBM_NPHASES; k++) { c->phase_ms[k] = 0.0; c->phase_n[k] = 0; }
    return LBM_OK;
}

int lbm_get_timing(lbm_ctx *c, double *ms, int64_t *launches) {
    if (!c || !ms || !launches) return LBM_E_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < c->ev_used; k++) {
        float t = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&t, c->events[k].a, c->events[k].b));
        c->phase_ms[c->events[k].phase] += (double)t;
        c->phase_n[c->events[k].phase] += 1;
    }
    c->ev_used = 0;
    for (int k = 0; k < LBM_NPHASES; k++) { ms[k] = c->phase_ms[k]; launches[k] = c->phase_n[k]; }
    return LBM_OK;
}

int lbm_set_lattice_block(lbm_ctx *c, int threads, int order, int cu_groups) {
    if (!c) return LBM_E_INVALID;
    if (!(threads == 0 || threads == 64 || threads == 128 || threads == 192 || threads == 256))
        return fail(c, LBM_E_INVALID, "lattice block width %d is not 0, 64, 128, 192 or 256", threads);
    if (order != LBM_ORDER_LINEAR && order != LBM_ORDER_XCD)
        return fail(c, LBM_E_INVALID, "unknown lattice block order %d", order);
    if (order == LBM_ORDER_XCD && !xcd_order_fits(c->g, threads))
        return fail(c, LBM_E_INVALID, "XCD order needs fewer than 2^32 workgroups");
    if (!(cu_groups == 0 || (cu_groups >= 3 && cu_groups <= 8)))
        return fail(c, LBM_E_INVALID, "workgroups per CU %d is not 0 or 3..8", cu_groups);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (threads != c->lb_width || order != c->lb_order || cu_groups != c->lb_cu_groups) {
        c->lb_width = threads;
        c->lb_order = order;
        c->lb_cu_groups = cu_groups;
        drop_graphs(c);  // captured steps hold the old launch shape
    }
    return LBM_OK;
}

int lbm_get_lattice_block(const lbm_ctx *c, int *threads, int *order, int *cu_groups) {
    if (!c || !threads || !order || !cu_groups) return LBM_E_INVALID;
    *threads = lattice_block_width(c->cfg.nx, c->lb_width);
    *order = c->lb_order;
    *cu_groups = c->lb_cu_groups;
    return LBM_OK;
}

int lbm_set_neighbour_list(lbm_ctx *c, int every, double skin) {
    if (!c) return LBM_E_INVALID;
    if (every < 0) return fail(c, LBM_E_INVALID, "every must be >= 0");
    if (every > 0 && !(skin > 0.0 && skin <= 2.0 * c->L.rmax))
        return fail(c, LBM_E_INVALID, "skin must be in (0, 2 max_radius]");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipStreamSynchronize(c->side_stream));
    const int old_every = c->nl_every;
    const double old_skin = c->nl_skin;
    c->nl_every = every;
    if (every > 0) c->nl_skin = skin;
    int nc[3];
    cell_grid(c, c->np, c->prmax, nc);
    if ((int64_t)nc[0] * nc[1] * nc[2] > c->L.cell_budget) {
        c->nl_every = old_every;
        c->nl_skin = old_skin;
        return fail(c, LBM_E_INVALID, "cell grid above the reserved budget");
    }
    drop_graphs(c);  // captured steps hold the other contact kernels
    c->ncx = nc[0]; c->ncy = nc[1]; c->ncz = nc[2];
    HIPCHK(c, nl_reset(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_get_neighbour_list(lbm_ctx *c, int *every, double *skin, int64_t *builds) {
    if (!c) return LBM_E_INVALID;
    if (every) *every = c->nl_every;
    if (skin) *skin = c->nl_skin;
    if (builds) {
        HIPCHK(c, hipStreamSynchronize(c->side_stream));
        HIPCHK(c, hipMemcpy(builds, c->ws + c->L.off_nl_state + 8, 8, hipMemcpyDeviceToHost));
    }
    return LBM_OK;
}

int lbm_set_pipeline(lbm_ctx *c, int slabs) {
    if (!c) return LBM_E_INVALID;
    if (slabs < 0 || slabs > PIPE_MAX) return fail(c, LBM_E_INVALID, "slabs must be in 0..%d", PIPE_MAX);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->pipe_req = slabs;
    if (c->particles_set) {
        HIPCHK(c, pipe_setup(c));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return LBM_OK;
}

int lbm_get_pipeline(const lbm_ctx *c, int *slabs) {
    if (!c || !slabs) return LBM_E_INVALID;
    *slabs = c->pipe_K;
    return LBM_OK;
}

// Every launch shape computes the same bits at every node, so the choice is by
// time alone: each candidate runs real steps with the lattice phase timed,
// twice in opposite orders so that a drift of the clock or of the state
// between the first and the last candidate does not favour one of them.
int lbm_autotune_lattice_block(lbm_ctx *c, int steps, int *best_threads, int *best_order,
                               int *best_cu_groups, double *ms_out) {
    if (!c || steps < 1 || steps > 100000) return LBM_E_INVALID;
    static const int widths[4] = {64, 128, 192, 256};
    static const int caps[3] = {0, 4, 3};
    // candidate k: width widths[k % 4], order (k / 4) % 2, cap caps[k / 8]
    constexpr int NC = 24;
    const int prev_timing = c->timing, prev_width = c->lb_width, prev_order = c->lb_order,
              prev_cap = c->lb_cu_groups;
    double best_ms[NC];
    for (int k = 0; k < NC; k++) best_ms[k] = HUGE_VAL;
    int r = LBM_OK;
    for (int pass = 0; pass < 2 && r == LBM_OK; pass++) {
        for (int j = 0; j < NC && r == LBM_OK; j++) {
            const int k = pass == 0 ? j : NC - 1 - j;
            const int order = (k / 4) % 2, width = widths[k % 4], cap = caps[k / 8];
            if (order == LBM_ORDER_XCD && !xcd_order_fits(c->g, width)) continue;
            if ((r = lbm_set_lattice_block(c, width, order, cap)) != LBM_OK) break;
            if ((r = lbm_set_timing(c, 2)) != LBM_OK) break;
            if ((r = lbm_step(c, 1)) != LBM_OK) break;  // first launch of this shape, untimed
            if ((r = lbm_set_timing(c, 2)) != LBM_OK) break;
            if ((r = lbm_step(c, steps)) != LBM_OK) break;
            double ms[LBM_NPHASES];
            int64_t n[LBM_NPHASES];
            if ((r = lbm_get_timing(c, ms, n)) != LBM_OK) break;
            if (n[1] > 0) best_ms[k] = std::min(best_ms[k], ms[1] / (double)n[1]);
        }
    }
    if (r != LBM_OK) {
        char msg[512];
        memcpy(msg, c->err, sizeof(msg));
        (void)lbm_set_lattice_block(c, prev_width, prev_order, prev_cap);
        (void)lbm_set_timing(c, prev_timing);
        memcpy(c->err, msg, sizeof(msg));
        memcpy(g_err, msg, sizeof(g_err));
        return r;
    }
    int best = 0;
    for (int k = 1; k < NC; k++)
        if (best_ms[k] < best_ms[best]) best = k;
    r = lbm_set_lattice_block(c, widths[best % 4], (best / 4) % 2, caps[best / 8]);
    if (r == LBM_OK) r = lbm_set_timing(c, prev_timing);
    if (r != LBM_OK) return r;
    if (best_threads) *best_threads = widths[best % 4];
    if (best_order) *best_order = (best / 4) % 2;
    if (best_cu_groups) *best_cu_groups = caps[best / 8];
    if (ms_out)
        for (int k = 0; k < NC; k++) ms_out[k] = best_ms[k];
    return LBM_OK;
}

int lbm_save(lbm_ctx *c, const char *path) {
    if (!c || !path) return LBM_E_INVALID;
    FILE *fp = fopen(path, "wb");
    if (!fp) return fail(c, LBM_E_IO, "cannot open %s", path);
    const size_t fbytes = (size_t)c->L.Q * c->L.N * store_bytes(c->cfg.storage);
    const size_t P = (size_t)std::max(c->np, 1);
    std::vector<char> buf(std::max(fbytes, 16 * P * 8));
    bool ok = true;
    auto put = [&](const void *p, size_t n) { ok = ok && fwrite(p, 1, n, fp) == n; };
    put(&SAVE_MAGIC, 8);
    put(&c->cfg, sizeof(lbm_config));
    put(&c->t, 8);
    put(&c->np, 4);
    if (hipMemcpy(buf.data(), state(c, c->cur), fbytes, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
    put(buf.data(), fbytes);
    const size_t offs[] = {c->L.off_x, c->L.off_v, c->L.off_w, c->L.off_Fh, c->L.off_Th, c->L.off_Fc};
    for (size_t o : offs) {
        if (hipMemcpy(buf.data(), c->ws + o, 3 * P * 8, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
        put(buf.data(), 3 * P * 8);
    }
    const size_t offs1[] = {c->L.off_R, c->L.off_m, c->L.off_I};
    for (size_t o : offs1) {
        if (hipMemcpy(buf.data(), c->ws + o, P * 8, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
        put(buf.data(), P * 8);
    }
    if (hipMemcpy(buf.data(), c->ws + c->L.off_fixed, P, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
    put(buf.data(), P);
    put(&c->ncx, 4); put(&c->ncy, 4); put(&c->ncz, 4);
    if (fclose(fp) != 0) ok = false;
    return ok ? LBM_OK : fail(c, LBM_E_IO, "write failed: %s", path);
}

// Reads the whole file and checks it before anything in the context
// changes: a truncated, foreign or inconsistent file leaves the context as it
// was.  The DEM cell grid is rebuilt from the loaded radii.
int lbm_load(lbm_ctx *c, const char *path) {
    if (!c || !path) return LBM_E_INVALID;
    FILE *fp = fopen(path, "rb");
    if (!fp) return fail(c, LBM_E_IO, "cannot open %s", path);
    bool ok = true;
    auto get = [&](void *p, size_t n) { ok = ok && fread(p, 1, n, fp) == n; };
    uint64_t magic = 0;
    lbm_config cfg;
    int64_t t = 0;
    int np = 0;
    get(&magic, 8);
    get(&cfg, sizeof(cfg));
    get(&t, 8);
    get(&np, 4);
    if (!ok || magic != SAVE_MAGIC) { fclose(fp); return fail(c, LBM_E_IO, "not a state file: %s", path); }
    if (memcmp(&cfg, &c->cfg, sizeof(cfg)) != 0) { fclose(fp); return fail(c, LBM_E_INVALID, "state file has another configuration"); }
    if (np < 0 || np > c->cfg.max_particles) { fclose(fp); return fail(c, LBM_E_INVALID, "bad particle count in file"); }
    if (t < 0) { fclose(fp); return fail(c, LBM_E_INVALID, "bad time in file"); }
    const size_t fbytes = (size_t)c->L.Q * c->L.N * store_bytes(c->cfg.storage);
    const size_t P = (size_t)std::max(np, 1);
    std::vector<char> fbuf(fbytes);
    get(fbuf.data(), fbytes);
    std::vector<double> vec[6];  // x, v, omega, F^h, T^h, F^c as [3][np]
    for (auto &v : vec) {
        v.resize(3 * P);
        get(v.data(), 3 * P * 8);
    }
    std::vector<double> R(P), M(P), I(P);
    get(R.data(), P * 8);
    get(M.data(), P * 8);
    get(I.data(), P * 8);
    std::vector<uint8_t> fixed(P);
    get(fixed.data(), P);
    int ncf[3];
    get(ncf, sizeof(ncf));  // recorded for reference; the grid is rebuilt below
    const bool at_end = ok && fgetc(fp) == EOF;
    fclose(fp);
    if (!ok) return fail(c, LBM_E_IO, "truncated state file: %s", path);
    if (!at_end) return fail(c, LBM_E_IO, "state file longer than its contents: %s", path);
    double rmax = 0.0;
    for (int p = 0; p < np; p++) {
        double pos[3], vel[3], om[3];
        for (int a = 0; a < 3; a++) {
            pos[a] = vec[0][(size_t)a * np + p];
            vel[a] = vec[1][(size_t)a * np + p];
            om[a] = vec[2][(size_t)a * np + p];
        }
        const char *why = "";
        if (!particle_ok(c, R[p], pos, vel, om, why))
            return fail(c, LBM_E_INVALID, "state file, particle %d: %s", p, why);
        if (!(M[p] > 0.0) || !std::isfinite(M[p]) || !(I[p] > 0.0) || !std::isfinite(I[p]))
            return fail(c, LBM_E_INVALID, "state file, particle %d: mass and inertia must be > 0", p);
        rmax = std::max(rmax, R[p]);
    }
    if (c->cfg.eps_mode == LBM_EPS_TABLE) {
        const int r = upload_eps_table(c, R.data(), np);
        if (r != LBM_OK) return r;
    }
    int nc[3];
    cell_grid(c, np, rmax, nc);
    // the file is sound: replace the state
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    HIPCHK(c, hipMemcpy(state(c, 0), fbuf.data(), fbytes, hipMemcpyHostToDevice));
    const size_t offs[6] = {c->L.off_x, c->L.off_v, c->L.off_w, c->L.off_Fh, c->L.off_Th, c->L.off_Fc};
    for (int k = 0; k < 6; k++) HIPCHK(c, hipMemcpy(c->ws + offs[k], vec[k].data(), 3 * P * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ws + c->L.off_R, R.data(), P * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ws + c->L.off_m, M.data(), P * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ws + c->L.off_I, I.data(), P * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ws + c->L.off_fixed, fixed.data(), P, hipMemcpyHostToDevice));
    c->np = np;
    c->ncx = nc[0]; c->ncy = nc[1]; c->ncz = nc[2];
    c->prmax = rmax;
    HIPCHK(c, nl_reset(c));
    c->cur = 0;
    c->t = t;
    c->particles_set = true;
    HIPCHK(c, launch_fill_u32(wsp<uint32_t>(c, c->L.off_nown), 0u, (int64_t)((c->L.N + 7) / 8 * 2), c->stream));
    for (int b = 0; b < 2; b++)
        HIPCHK(c, launch_fill_u32(wsp<uint32_t>(c, c->L.off_list_len + (size_t)b * c->L.list_buf), 0u,
                                  (int64_t)P, c->stream));
    HIPCHK(c, launch_fill_u32(flags(c), 0u, 16, c->stream));
    c->pipe_K = 1;  // the footprint is forgotten: set the pipeline up afresh
    HIPCHK(c, pipe_setup(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// Suspension-wide sums, reduced in a fixed order on the context's stream.
int lbm_get_stats(lbm_ctx *c, lbm_stats *out) {
    if (!c || !out) return LBM_E_INVALID;
    StatsArgs a;
    a.A = state(c, c->cur);
    a.g = c->g;
    a.P = particles(c, 1 - c->cur);  // the last completed step's footprint
    a.qr = wsp<char>(c, c->L.off_qr);
    a.rec32 = c->cfg.storage != LBM_FP64;
    a.Smax = c->L.Smax;
    double *base = wsp<double>(c, c->L.off_stats);
    a.node_part = base;
    a.part_rows = base + (size_t)STATS_NODE_GROUPS * 4;
    a.tot = a.part_rows + (size_t)c->L.P * STATS_PK;
    HIPCHK(c, launch_stats(c->cfg.lattice, c->cfg.storage, a, c->stream));
    double s[4 + STATS_PK];
    HIPCHK(c, hipMemcpyAsync(s, a.tot, sizeof(s), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int np = c->np;
    out->t = c->t;
    out->np = np;
    out->nodes = c->L.N;
    out->mass = s[0];
    const double *mv = s + 4, *vs = s + 7, *Fs = s + 10;
    const double wrho = s[13], *wj = s + 14, weps = s[17], msum = s[18];
    out->solid_fraction = weps / (double)c->L.N;
    const double fluid_mass = s[0] - wrho;
    for (int d = 0; d < 3; d++) {
        out->fluid_momentum[d] = s[1 + d];
        out->fluid_velocity[d] = (s[1 + d] - wj[d]) / fluid_mass;
        out->particle_momentum[d] = mv[d];
        out->particle_velocity[d] = np > 0 ? mv[d] / msum : 0.0;
        out->mean_particle_velocity[d] = np > 0 ? vs[d] / (double)np : 0.0;
        out->slip_velocity[d] = out->fluid_velocity[d] - out->particle_velocity[d];
        out->mean_drag[d] = np > 0 ? Fs[d] / (double)np : 0.0;
    }
    return LBM_OK;
}

}  // extern "C"
