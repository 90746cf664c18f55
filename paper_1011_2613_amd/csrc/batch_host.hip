// batch_host.hip -- host side of the batched drag ensemble (lbm_batch_* ABI).
//
// The caller's workspace holds the population pool (A and B, shifted FP32),
// the static per-node sample counts, q, the per-box tables and descriptors,
// the sphere footprint lists and forces.  Footprints are computed here once
// with the same sub-cell sampling rule as the single-box paint kernel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbimb.h"
#include "internal.h"

using namespace lbimb;

namespace {

constexpr size_t AL = 256;
size_t al(size_t v) { return (v + AL - 1) / AL * AL; }
constexpr int ROW_CHOICES[5] = {1, 2, 4, 8, 16};

struct BLayout {
    int nbox, nsph, Smax, ntiles;
    int64_t total_nodes, pool, list_total;
    size_t A, B, cnt, q, beta, arel, boxes, tile_box, queue, done, flags, sph_box, sph_x, lstart, list, F,
        T, U, Fprev, steady, stop, misc, Us, feat, total;
};

double pdisp(double d, double L) {
    if (d > 0.5 * L) d = d - L;
    else if (d < -0.5 * L) d = d + L;
    return d;
}

// Sub-cell sample count of node (ix,iy,iz) in a sphere (same rule and
// evaluation order as the single-box paint kernel).
int sample_count(int S, double d0, double d1, double d2, double R2) {
    int count = 0;
    for (int kz = 0; kz < S; kz++)
        for (int ky = 0; ky < S; ky++)
            for (int kx = 0; kx < S; kx++) {
                const double ox = ((double)kx + 0.5) / (double)S - 0.5;
                const double oy = ((double)ky + 0.5) / (double)S - 0.5;
                const double oz = ((double)kz + 0.5) / (double)S - 0.5;
                const double ex = d0 + ox, ey = d1 + oy, ez = d2 + oz;
                if (ex * ex + ey * ey + ez * ez <= R2) count++;
            }
    return count;
}

struct Footprint {
    std::vector<uint16_t> cnt;        // per node of the whole batch
    std::vector<int> start;           // per sphere
    std::vector<uint32_t> list;       // node | count << 20
    std::vector<uint8_t> owners;      // per node
};

int validate_boxes(const lbm_box *boxes, int nbox, int S) {
    if (!boxes || nbox < 1 || S < 1 || S > 8) return LBM_E_INVALID;
    for (int b = 0; b < nbox; b++) {
        const lbm_box &x = boxes[b];
        if (x.edge < 4 || x.edge > 1024 || !(x.tau > 0.5) || x.nspheres < 0) return LBM_E_INVALID;
        if ((int64_t)x.edge * x.edge * x.edge >= (1 << 20) && x.nspheres > 0) return LBM_E_INVALID;
        if (x.nspheres > 0 && (!x.pos || !(x.radius > 0.0) || 2.0 * x.radius + 2.0 > (double)x.edge))
            return LBM_E_INVALID;
        for (int p = 0; p < x.nspheres; p++)
            for (int a = 0; a < 3; a++)
                if (!(x.pos[3 * p + a] >= 0.0 && x.pos[3 * p + a] < (double)x.edge)) return LBM_E_INVALID;
        const double *u = x.init_velocity;
        if (!(u[0] * u[0] + u[1] * u[1] + u[2] * u[2] <= 0.04)) return LBM_E_INVALID;
    }
    return LBM_OK;
}

BLayout make_blayout(const lbm_box *boxes, int nbox, int S, int64_t list_total) {
    BLayout L{};
    L.nbox = nbox;
    L.Smax = S * S * S;
    int64_t nodes = 0;
    int nsph = 0, ntiles = 0;
    for (int b = 0; b < nbox; b++) {
        nodes += (int64_t)boxes[b].edge * boxes[b].edge * boxes[b].edge;
        nsph += boxes[b].nspheres;
        ntiles += boxes[b].edge * boxes[b].edge;  // worst case: one row per tile
    }
    L.total_nodes = nodes;
    L.pool = 19 * nodes;
    L.nsph = nsph;
    L.ntiles = ntiles;
    L.list_total = list_total;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = al(o + b); return r; };
    L.A = take((size_t)L.pool * 4);
    L.B = take((size_t)L.pool * 4);
    L.cnt = take((size_t)nodes * 2);
    L.q = take((size_t)nodes * 3 * 4);
    L.beta = take((size_t)nbox * (L.Smax + 1) * 4);
    L.arel = take((size_t)nbox * (L.Smax + 1) * 4);
    L.boxes = take((size_t)nbox * sizeof(BatchBox));
    L.tile_box = take((size_t)ntiles * 4);
    L.queue = take(64);
    L.done = take((size_t)nbox * 4);
    L.flags = take(64);
    L.sph_box = take((size_t)std::max(nsph, 1) * 4);
    L.sph_x = take((size_t)std::max(nsph, 1) * 24);
    L.lstart = take((size_t)(nsph + 1) * 4);
    L.list = take((size_t)std::max<int64_t>(list_total, 1) * 4);
    L.F = take((size_t)std::max(nsph, 1) * 24);
    L.T = take((size_t)std::max(nsph, 1) * 24);
    L.U = take((size_t)nbox * 24);
    L.Fprev = take((size_t)std::max(nsph, 1) * 24);
    L.steady = take((size_t)nbox * 4);
    L.stop = take((size_t)nbox * 8);
    L.misc = take(64);  // remaining (int), first check (int), check time (int64)
    L.Us = take((size_t)std::max(nsph, 1) * 24);
    L.feat = take((size_t)std::max(nsph, 1) * 40 * 4);
    L.total = o;
    return L;
}

// Footprint list length without storing it (for workspace sizing).
int64_t list_length(const lbm_box *boxes, int nbox, int S) {
    int64_t total = 0;
    for (int b = 0; b < nbox; b++) {
        const lbm_box &x = boxes[b];
        const int ext = (int)std::floor(2.0 * x.radius + 1.0) + 1;
        total += (int64_t)x.nspheres * ext * ext * ext;  // upper bound
    }
    (void)S;
    return total;
}

int compute_footprint(const lbm_box *boxes, int nbox, int S, Footprint &fp) {
    int64_t nodes = 0;
    std::vector<int64_t> noff(nbox);
    for (int b = 0; b < nbox; b++) {
        noff[b] = nodes;
        nodes += (int64_t)boxes[b].edge * boxes[b].edge * boxes[b].edge;
    }
    fp.cnt.assign((size_t)nodes, 0);
    fp.owners.assign((size_t)nodes, 0);
    fp.start.clear();
    fp.list.clear();
    for (int b = 0; b < nbox; b++) {
        const lbm_box &x = boxes[b];
        const int Lb = x.edge;
        const double Ld = (double)Lb, r = x.radius, R2 = r * r;
        for (int p = 0; p < x.nspheres; p++) {
            fp.start.push_back((int)fp.list.size());
            int lo[3], hi[3];
            for (int a = 0; a < 3; a++) {
                lo[a] = (int)std::ceil(x.pos[3 * p + a] - r - 0.5);
                hi[a] = (int)std::floor(x.pos[3 * p + a] + r + 0.5);
            }
            for (int cz = lo[2]; cz <= hi[2]; cz++)
                for (int cy = lo[1]; cy <= hi[1]; cy++)
                    for (int cx = lo[0]; cx <= hi[0]; cx++) {
                        const int ix = (cx % Lb + Lb) % Lb, iy = (cy % Lb + Lb) % Lb, iz = (cz % Lb + Lb) % Lb;
                        const double d0 = pdisp((double)ix - x.pos[3 * p], Ld);
                        const double d1 = pdisp((double)iy - x.pos[3 * p + 1], Ld);
                        const double d2 = pdisp((double)iz - x.pos[3 * p + 2], Ld);
                        const int c = sample_count(S, d0, d1, d2, R2);
                        if (c == 0) continue;
                        const int64_t node = (int64_t)ix + (int64_t)Lb * ((int64_t)iy + (int64_t)Lb * iz);
                        fp.cnt[(size_t)(noff[b] + node)] = (uint16_t)(fp.cnt[(size_t)(noff[b] + node)] + c);
                        if (++fp.owners[(size_t)(noff[b] + node)] > MAX_OWNERS) return LBM_E_SLOT_OVERFLOW;
                        fp.list.push_back((uint32_t)node | ((uint32_t)c << 20));
                    }
        }
    }
    fp.start.push_back((int)fp.list.size());
    return LBM_OK;
}

}  // namespace

struct lbm_batch {
    BLayout L;
    char *ws;
    hipStream_t s;
    hipStream_t cap;              // private stream the steady-run chunks are captured on
    hipGraphExec_t chunk[2];      // captured chunk (check_every steps, forces, check) per starting parity
    bool chunk_ok[2];
    int64_t chunk_k;              // steps, mode and tolerance the captured chunks hold
    int chunk_mode;
    double chunk_tol;
    std::vector<BatchBox> box;
    std::vector<int> tile_box;
    int ntiles;
    int cur;
    int64_t t;
    int pgrid;
    int mode_hint;
};

namespace {
template <class T> T *Pp(lbm_batch *c, size_t off) { return (T *)(c->ws + off); }

BatchArgs bargs(lbm_batch *c) {
    BatchArgs a;
    a.A = Pp<float>(c, c->L.A);
    a.B = Pp<float>(c, c->L.B);
    a.boxes = Pp<BatchBox>(c, c->L.boxes);
    a.tile_box = Pp<int>(c, c->L.tile_box);
    a.cnt = Pp<uint16_t>(c, c->L.cnt);
    a.beta = Pp<float>(c, c->L.beta);
    a.arel = Pp<float>(c, c->L.arel);
    a.q = Pp<float>(c, c->L.q);
    a.total_nodes = c->L.total_nodes;
    a.nbox = c->L.nbox;
    a.ntiles = c->ntiles;
    a.Smax = c->L.Smax;
    a.queue = Pp<int>(c, c->L.queue);
    a.done = Pp<int>(c, c->L.done);
    a.flags = Pp<uint32_t>(c, c->L.flags);
    a.nsph = c->L.nsph;
    a.sph_box = Pp<int>(c, c->L.sph_box);
    a.sph_x = Pp<double>(c, c->L.sph_x);
    a.list_start = Pp<int>(c, c->L.lstart);
    a.list = Pp<uint32_t>(c, c->L.list);
    a.F = Pp<double>(c, c->L.F);
    a.T = Pp<double>(c, c->L.T);
    return a;
}

BatchSteady steady_args(lbm_batch *c, double tol) {
    BatchSteady st;
    st.Fprev = Pp<double>(c, c->L.Fprev);
    st.steady = Pp<int>(c, c->L.steady);
    st.stop = Pp<int64_t>(c, c->L.stop);
    st.remaining = Pp<int>(c, c->L.misc);
    st.first = Pp<int>(c, c->L.misc + 4);
    st.tnow = Pp<int64_t>(c, c->L.misc + 8);
    st.tol = tol;
    return st;
}

void drop_chunks(lbm_batch *c) {
    for (int k = 0; k < 2; k++) {
        if (c->chunk_ok[k]) (void)hipGraphExecDestroy(c->chunk[k]);
        c->chunk_ok[k] = false;
    }
}

// Rebuild tile numbering after a tile-shape change and upload descriptors.
hipError_t upload_tiles(lbm_batch *c) {
    drop_chunks(c);  // captured launches hold the tile count
    c->tile_box.clear();
    int t = 0;
    for (int b = 0; b < c->L.nbox; b++) {
        BatchBox &x = c->box[b];
        x.ntiles = x.L * x.L / x.rows;
        x.tile0 = t;
        for (int k = 0; k < x.ntiles; k++) c->tile_box.push_back(b);
        t += x.ntiles;
    }
    c->ntiles = t;
    hipError_t e = hipMemcpyAsync(Pp<BatchBox>(c, c->L.boxes), c->box.data(), c->box.size() * sizeof(BatchBox),
                                  hipMemcpyHostToDevice, c->s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(Pp<int>(c, c->L.tile_box), c->tile_box.data(), c->tile_box.size() * 4,
                       hipMemcpyHostToDevice, c->s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->s);
}

hipError_t reset_state(lbm_batch *c) {
    int maxL = 0;
    for (auto &x : c->box) maxL = std::max(maxL, x.L);
    hipError_t e = launch_batch_init(bargs(c), c->L.nbox, maxL, c->s);
    if (e == hipSuccess) e = launch_fill_u32(Pp<uint32_t>(c, c->L.q), 0u, 3 * c->L.total_nodes, c->s);
    c->cur = 0;
    c->t = 0;
    return e;
}

// Queue nsteps steps starting from state `from` on stream s (no wait).
hipError_t enqueue_steps(lbm_batch *c, int64_t nsteps, int mode, int from, hipStream_t s) {
    BatchArgs a = bargs(c);
    hipError_t e = hipSuccess;
    int cur = from;
    if (mode == LBM_BATCH_PERSISTENT) {
        // items are counted in a 32-bit integer: keep nsteps * ntiles (plus one
        // overshoot per workgroup) far below 2^31
        const int chunk = std::max(1, (int)(((int64_t)1 << 30) / std::max(c->ntiles, 1)));
        for (int64_t done = 0; done < nsteps && e == hipSuccess;) {
            const int k = (int)std::min<int64_t>(nsteps - done, chunk);
            e = launch_fill_u32((uint32_t *)a.queue, 0u, 1, s);
            if (e == hipSuccess) e = launch_fill_u32((uint32_t *)a.done, 0u, c->L.nbox, s);
            if (e == hipSuccess) e = launch_batch_persistent(a, k, cur, c->pgrid, s);
            cur = (cur + k) & 1;
            done += k;
        }
    } else {
        for (int64_t k = 0; k < nsteps && e == hipSuccess; k++) {
            e = launch_batch_step(a, cur, s);
            cur ^= 1;
        }
    }
    return e;
}

// Health word of the batch (synchronises).
int read_flags(lbm_batch *c) {
    uint32_t h = 0;
    if (hipMemcpyAsync(&h, Pp<uint32_t>(c, c->L.flags), 4, hipMemcpyDeviceToHost, c->s) != hipSuccess)
        return LBM_E_HIP;
    if (hipStreamSynchronize(c->s) != hipSuccess) return LBM_E_HIP;
    if (h & FLAG_BATCH_TIMEOUT) return LBM_E_STATE;
    return LBM_OK;
}

int run_steps(lbm_batch *c, int64_t nsteps, int mode) {
    hipError_t e = enqueue_steps(c, nsteps, mode, c->cur, c->s);
    c->cur = (int)((c->cur + nsteps) & 1);
    c->t += nsteps;
    if (e != hipSuccess) return LBM_E_HIP;
    return read_flags(c);
}

// One chunk of a steady run: k steps from state `from`, the forces of the
// last step and the device-side steady check.
hipError_t enqueue_chunk(lbm_batch *c, int64_t k, int mode, int from, double tol, hipStream_t s) {
    hipError_t e = enqueue_steps(c, k, mode, from, s);
    if (e == hipSuccess) e = launch_batch_force(bargs(c), s);
    if (e == hipSuccess) e = launch_batch_check(bargs(c), Pp<BatchBox>(c, c->L.boxes), steady_args(c, tol), k, s);
    return e;
}

hipError_t build_chunk(lbm_batch *c, int64_t k, int mode, int from, double tol) {
    hipGraph_t g;
    hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t e1 = enqueue_chunk(c, k, mode, from, tol, c->cap);
    const hipError_t e2 = hipStreamEndCapture(c->cap, &g);
    if (e1 != hipSuccess) return e1;
    if (e2 != hipSuccess) return e2;
    e = hipGraphInstantiate(&c->chunk[from], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e == hipSuccess) c->chunk_ok[from] = true;
    return e;
}
}  // namespace

extern "C" {

int lbm_batch_workspace_bytes(const lbm_box *boxes, int nbox, int eps_samples, size_t *bytes) {
    if (!bytes) return LBM_E_INVALID;
    int rc = validate_boxes(boxes, nbox, eps_samples);
    if (rc != LBM_OK) return rc;
    *bytes = make_blayout(boxes, nbox, eps_samples, list_length(boxes, nbox, eps_samples)).total;
    return LBM_OK;
}

int lbm_batch_create(const lbm_box *boxes, int nbox, int eps_samples, void *workspace, size_t ws_bytes,
                     void *hip_stream, lbm_batch **out) {
    if (!out) return LBM_E_INVALID;
    *out = nullptr;
    int rc = validate_boxes(boxes, nbox, eps_samples);
    if (rc != LBM_OK) return rc;
    BLayout L = make_blayout(boxes, nbox, eps_samples, list_length(boxes, nbox, eps_samples));
    if (!workspace || ws_bytes < L.total) return LBM_E_NOMEM;
    if ((uintptr_t)workspace % AL) return LBM_E_INVALID;
    Footprint fp;
    rc = compute_footprint(boxes, nbox, eps_samples, fp);
    if (rc != LBM_OK) return rc;
    lbm_batch *c = new (std::nothrow) lbm_batch();
    if (!c) return LBM_E_NOMEM;
    c->L = L;
    c->ws = (char *)workspace;
    c->s = (hipStream_t)hip_stream;
    c->pgrid = batch_persistent_grid();
    c->mode_hint = LBM_BATCH_PER_STEP;
    c->chunk_ok[0] = c->chunk_ok[1] = false;
    c->chunk_k = 0;
    c->chunk_mode = -1;
    c->chunk_tol = 0.0;
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return LBM_E_HIP;
    }
    // per-box descriptors and tables
    const int S1 = L.Smax + 1;
    std::vector<float> beta((size_t)nbox * S1), arel((size_t)nbox * S1);
    std::vector<int> sph_box;
    std::vector<double> sph_x;
    int64_t off = 0, noff = 0;
    c->box.resize(nbox);
    for (int b = 0; b < nbox; b++) {
        const lbm_box &x = boxes[b];
        BatchBox &d = c->box[b];
        d.L = x.edge;
        d.radius = x.radius;
        d.rows = 1;
        d.off = off;
        d.noff = noff;
        d.table = b * S1;
        d.active = 1;
        d.tau = x.tau;
        d.sph0 = (int)sph_box.size();
        d.nsph = x.nspheres;
        const double tau = x.tau;
        d.arel0f = (float)((1.0 - 0.0) / tau);
        for (int i = 0; i < 19; i++) {
            static const int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
            static const int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
            static const int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
            double v = (double)cx[i] * x.fluid_force[0] + (double)cy[i] * x.fluid_force[1];
            v = v + (double)cz[i] * x.fluid_force[2];
            d.cgf[i] = (float)v;
            // f^eq_i(1, u0) - w_i = w_i (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
            const double *u = x.init_velocity;
            const double w = i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
            const double cu = (double)cx[i] * u[0] + (double)cy[i] * u[1] + (double)cz[i] * u[2];
            const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            d.g0[i] = (float)(w * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        }
        for (int k = 0; k <= L.Smax; k++) {
            const double eps = (double)k / (double)L.Smax;
            const double bt = eps * (tau - 0.5) / ((1.0 - eps) + (tau - 0.5));
            beta[(size_t)b * S1 + k] = (float)bt;
            arel[(size_t)b * S1 + k] = (float)((1.0 - bt) / tau);
        }
        for (int p = 0; p < x.nspheres; p++) {
            sph_box.push_back(b);
            for (int a = 0; a < 3; a++) sph_x.push_back(x.pos[3 * p + a]);
        }
        const int64_t N = (int64_t)x.edge * x.edge * x.edge;
        off += 19 * N;
        noff += N;
    }
    hipError_t e = hipSuccess;
    auto up = [&](size_t o, const void *src, size_t n) {
        if (e == hipSuccess && n) e = hipMemcpyAsync(c->ws + o, src, n, hipMemcpyHostToDevice, c->s);
    };
    up(L.cnt, fp.cnt.data(), fp.cnt.size() * 2);
    up(L.beta, beta.data(), beta.size() * 4);
    up(L.arel, arel.data(), arel.size() * 4);
    up(L.sph_box, sph_box.data(), sph_box.size() * 4);
    up(L.sph_x, sph_x.data(), sph_x.size() * 8);
    up(L.lstart, fp.start.data(), fp.start.size() * 4);
    up(L.list, fp.list.data(), fp.list.size() * 4);
    if (e == hipSuccess) e = launch_fill_u32(Pp<uint32_t>(c, L.flags), 0u, 16, c->s);
    if (e == hipSuccess) e = upload_tiles(c);  // box descriptors first: the initial state reads them
    if (e == hipSuccess) e = reset_state(c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->s);
    if (e != hipSuccess) {
        drop_chunks(c);
        (void)hipStreamDestroy(c->cap);
        delete c;
        return LBM_E_HIP;
    }
    *out = c;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    drop_chunks(c);
    (void)hipStreamDestroy(c->cap);
    delete c;
}

int lbm_batch_set_tile_rows(lbm_batch *c, int edge, int rows) {
    if (!c || rows < 1) return LBM_E_INVALID;
    bool any = false;
    for (auto &x : c->box)
        if (x.L == edge) {
            if ((x.L * x.L) % rows != 0) return LBM_E_INVALID;
            x.rows = rows;
            any = true;
        }
    if (!any) return LBM_E_INVALID;
    return upload_tiles(c) == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_batch_set_active(lbm_batch *c, const uint8_t *active) {
    if (!c || !active) return LBM_E_INVALID;
    for (int b = 0; b < c->L.nbox; b++) c->box[b].active = active[b] ? 1 : 0;
    return upload_tiles(c) == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_batch_run(lbm_batch *c, int64_t nsteps, int mode) {
    if (!c || nsteps < 0 || (mode != LBM_BATCH_PER_STEP && mode != LBM_BATCH_PERSISTENT)) return LBM_E_INVALID;
    if (nsteps == 0) return LBM_OK;
    int rc = run_steps(c, nsteps, mode);
    if (rc != LBM_OK) return rc;
    return launch_batch_force(bargs(c), c->s) == hipSuccess && hipStreamSynchronize(c->s) == hipSuccess
               ? LBM_OK : LBM_E_HIP;
}

int lbm_batch_forces(lbm_batch *c, double *F, double *T, int ptr_kind) {
    if (!c) return LBM_E_INVALID;
    const size_t n = (size_t)c->L.nsph * 24;
    if (n == 0) return LBM_OK;
    const hipMemcpyKind k = ptr_kind == LBM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (F && hipMemcpyAsync(F, c->ws + c->L.F, n, k, c->s) != hipSuccess) return LBM_E_HIP;
    if (T && hipMemcpyAsync(T, c->ws + c->L.T, n, k, c->s) != hipSuccess) return LBM_E_HIP;
    return hipStreamSynchronize(c->s) == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_batch_mean_velocity(lbm_batch *c, double *U, int ptr_kind) {
    if (!c || !U) return LBM_E_INVALID;
    if (launch_batch_mean(bargs(c), c->cur, Pp<double>(c, c->L.U), c->s) != hipSuccess) return LBM_E_HIP;
    const hipMemcpyKind k = ptr_kind == LBM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(U, c->ws + c->L.U, (size_t)c->L.nbox * 24, k, c->s) != hipSuccess) return LBM_E_HIP;
    return hipStreamSynchronize(c->s) == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_batch_shell_velocity(lbm_batch *c, double *u, int ptr_kind) {
    if (!c || !u) return LBM_E_INVALID;
    const size_t n = (size_t)c->L.nsph * 24;
    if (n == 0) return LBM_OK;
    double *dst = u;
    if (ptr_kind == LBM_HOST && hipMalloc(&dst, n) != hipSuccess) return LBM_E_HIP;
    hipError_t e = launch_batch_shell(bargs(c), c->cur, dst, c->s);
    if (e == hipSuccess && ptr_kind == LBM_HOST) e = hipMemcpyAsync(u, dst, n, hipMemcpyDeviceToHost, c->s);
    if (e == hipSuccess) e = hipStreamSynchronize(c->s);
    if (ptr_kind == LBM_HOST) (void)hipFree(dst);
    return e == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_batch_get_distributions(lbm_batch *c, int b, double *f, int ptr_kind) {
    if (!c || !f || b < 0 || b >= c->L.nbox) return LBM_E_INVALID;
    const int Lb = c->box[b].L;
    const size_t bytes = (size_t)19 * Lb * Lb * Lb * 8;
    double *dst = f;
    if (ptr_kind == LBM_HOST && hipMalloc(&dst, bytes) != hipSuccess) return LBM_E_HIP;
    hipError_t e = launch_batch_get_f(bargs(c), b, Lb, c->cur, dst, c->s);
    if (e == hipSuccess && ptr_kind == LBM_HOST) e = hipMemcpyAsync(f, dst, bytes, hipMemcpyDeviceToHost, c->s);
    if (e == hipSuccess) e = hipStreamSynchronize(c->s);
    if (ptr_kind == LBM_HOST) (void)hipFree(dst);
    return e == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_batch_run_steady(lbm_batch *c, int64_t max_steps, double tol, int check_every, int mode,
                         uint8_t *steady, int64_t *stop_step) {
    if (!c || max_steps < 0 || check_every < 1 || !(tol > 0.0) || !std::isfinite(tol) ||
        (mode != LBM_BATCH_PER_STEP && mode != LBM_BATCH_PERSISTENT))
        return LBM_E_INVALID;
    const int nb = c->L.nbox;
    const int64_t t0 = c->t;
    BatchSteady st = steady_args(c, tol);
    hipError_t e = launch_fill_u32((uint32_t *)st.steady, 0u, nb, c->s);
    if (e == hipSuccess) e = launch_fill_u64((uint64_t *)st.stop, (uint64_t)t0, nb, c->s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)st.first, 1u, 1, c->s);
    if (e == hipSuccess) e = launch_fill_u64((uint64_t *)st.tnow, (uint64_t)t0, 1, c->s);
    if (e != hipSuccess) return LBM_E_HIP;
    if (c->chunk_k != check_every || c->chunk_mode != mode || c->chunk_tol != tol) {
        drop_chunks(c);
        c->chunk_k = check_every;
        c->chunk_mode = mode;
        c->chunk_tol = tol;
    }
    std::vector<uint8_t> was_active(nb);
    int left = 0;
    for (int b = 0; b < nb; b++) left += (was_active[b] = (uint8_t)c->box[b].active);
    int64_t done = 0;
    while (done < max_steps && left > 0) {
        const int64_t k = std::min<int64_t>(check_every, max_steps - done);
        if (k == check_every) {
            if (!c->chunk_ok[c->cur] && build_chunk(c, k, mode, c->cur, tol) != hipSuccess) return LBM_E_HIP;
            if (hipGraphLaunch(c->chunk[c->cur], c->s) != hipSuccess) return LBM_E_HIP;
        } else if (enqueue_chunk(c, k, mode, c->cur, tol, c->s) != hipSuccess) {
            return LBM_E_HIP;
        }
        c->cur = (int)((c->cur + k) & 1);
        c->t += k;
        done += k;
        if (hipMemcpyAsync(&left, st.remaining, 4, hipMemcpyDeviceToHost, c->s) != hipSuccess) return LBM_E_HIP;
        const int rc = read_flags(c);  // synchronises
        if (rc != LBM_OK) return rc;
    }
    std::vector<int> st_h(nb);
    std::vector<int64_t> stop_h(nb);
    if (hipMemcpyAsync(st_h.data(), st.steady, (size_t)nb * 4, hipMemcpyDeviceToHost, c->s) != hipSuccess ||
        hipMemcpyAsync(stop_h.data(), st.stop, (size_t)nb * 8, hipMemcpyDeviceToHost, c->s) != hipSuccess ||
        hipStreamSynchronize(c->s) != hipSuccess)
        return LBM_E_HIP;
    for (int b = 0; b < nb; b++) {
        if (st_h[b]) c->box[b].active = 0;  // the device descriptor was cleared by the check
        else if (was_active[b]) stop_h[b] = c->t;
        if (steady) steady[b] = (uint8_t)(st_h[b] ? 1 : 0);
        if (stop_step) stop_step[b] = stop_h[b];
    }
    return LBM_OK;
}

int lbm_batch_get_drag(lbm_batch *c, double *F, float *feat, int ptr_kind) {
    if (!c || (ptr_kind != LBM_HOST && ptr_kind != LBM_DEVICE)) return LBM_E_INVALID;
    const int nsph = c->L.nsph;
    if (nsph == 0) return LBM_OK;
    const hipMemcpyKind k = ptr_kind == LBM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (F && hipMemcpyAsync(F, c->ws + c->L.F, (size_t)nsph * 24, k, c->s) != hipSuccess) return LBM_E_HIP;
    if (feat) {
        for (auto &x : c->box)
            if (x.nsph > 64) return LBM_E_INVALID;
        BatchArgs a = bargs(c);
        double *U = Pp<double>(c, c->L.U), *Us = Pp<double>(c, c->L.Us);
        float *X = Pp<float>(c, c->L.feat);
        hipError_t e = launch_batch_mean(a, c->cur, U, c->s);
        if (e == hipSuccess) e = launch_batch_shell(a, c->cur, Us, c->s);
        if (e == hipSuccess) e = launch_batch_features(a, U, Us, X, c->s);
        if (e == hipSuccess) e = hipMemcpyAsync(feat, X, (size_t)nsph * 160, k, c->s);
        if (e != hipSuccess) return LBM_E_HIP;
    }
    return hipStreamSynchronize(c->s) == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int64_t lbm_batch_time(const lbm_batch *c) { return c ? c->t : -1; }

int lbm_batch_autotune(lbm_batch *c, int steps, int *edges_out, int *rows_out, int *mode_out,
                       double *ms_out) {
    if (!c || steps < 1) return LBM_E_INVALID;
    std::vector<int> edges;
    for (auto &x : c->box)
        if (std::find(edges.begin(), edges.end(), x.L) == edges.end()) edges.push_back(x.L);
    std::sort(edges.begin(), edges.end());
    auto time_run = [&](int mode, double &ms) -> int {
        if (hipStreamSynchronize(c->s) != hipSuccess) return LBM_E_HIP;
        const auto t0 = std::chrono::steady_clock::now();
        int rc = run_steps(c, steps, mode);
        const auto t1 = std::chrono::steady_clock::now();
        ms = std::chrono::duration<double, std::milli>(t1 - t0).count() / steps;
        return rc;
    };
    double best_all = 0.0;
    for (size_t k = 0; k < edges.size(); k++) {
        int best_rows = 1;
        double best = 1e300;
        for (int r : ROW_CHOICES) {
            if ((edges[k] * edges[k]) % r != 0 || r * edges[k] > 4096) continue;
            int rc = lbm_batch_set_tile_rows(c, edges[k], r);
            if (rc != LBM_OK) return rc;
            double ms;
            if ((rc = time_run(LBM_BATCH_PER_STEP, ms)) != LBM_OK) return rc;
            if (ms < best) { best = ms; best_rows = r; }
        }
        int rc = lbm_batch_set_tile_rows(c, edges[k], best_rows);
        if (rc != LBM_OK) return rc;
        if (edges_out) edges_out[k] = edges[k];
        if (rows_out) rows_out[k] = best_rows;
        best_all = best;
    }
    double ms_step = 0.0, ms_pers = 0.0;
    int rc = time_run(LBM_BATCH_PER_STEP, ms_step);
    if (rc == LBM_OK) rc = time_run(LBM_BATCH_PERSISTENT, ms_pers);
    if (rc != LBM_OK) return rc;
    c->mode_hint = ms_pers < ms_step ? LBM_BATCH_PERSISTENT : LBM_BATCH_PER_STEP;
    if (mode_out) *mode_out = c->mode_hint;
    if (ms_out) *ms_out = std::min(ms_step, ms_pers);
    (void)best_all;
    if (reset_state(c) != hipSuccess || hipStreamSynchronize(c->s) != hipSuccess) return LBM_E_HIP;
    return LBM_OK;
}

}  // extern "C"
