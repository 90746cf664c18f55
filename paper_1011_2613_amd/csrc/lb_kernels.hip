// lb_kernels.hip -- fused pull-streaming + LBGK collision with the
// Noble-Torczynski immersed-moving-boundary terms, for gfx950.
//
// One thread updates one node.  The state array A holds the post-collision
// populations of the previous step; the kernel gathers f_i(x, t) = A_i(x - c_i)
// (halfway bounce-back: A_opp(i)(x) when x - c_i lies beyond a wall), applies
// Eq. 1 with the weight beta of Eq. 2 and the solid operator Omega^S, and
// writes the new post-collision populations to B at x.  Reads of the shifted
// neighbours are unaligned by one element but every population is read once
// and written once: 2 Q s bytes per node of HBM traffic.
//
// Layout f[z][y][i][x]: the Q direction rows of one lattice row are
// contiguous, so a wavefront's 64 consecutive x are contiguous lines, a
// workgroup (one lattice row) writes one contiguous block and reads from the
// nine neighbouring rows' blocks.  Compared with one array per direction this
// keeps far fewer DRAM streams open at a time (measured on gfx950: +3 % FP64,
// +6 % FP32, +12 % FP16 pull bandwidth).  Every address is a per-workgroup
// scalar row base plus the lane's x byte offset.
//
// Covered nodes (a particle's sub-cell samples fall in the cell) also read
// their owner records and the owners' velocities (small particle arrays that
// stay in L2), and write q_n, the momentum the IMB term hands to the fluid,
// which the force kernel sums per particle (Eq. 3).
//
// FP64 evaluation order is fixed: every sum runs over the directions in index
// order, every product and quotient is taken exactly as in the paper's
// formulas with no fused multiply-add (the library is built with
// -ffp-contract=off), so the result is reproducible bit for bit.
#include "internal.h"
#include "lb_shared.h"

namespace lbimb {

// Periodic minimum image of a displacement, as selects (no branches, so the
// loads that feed it can all be in flight together).
__device__ __forceinline__ double disp_periodic(double d, double L) {
    const double dm = d - L, dp = d + L;
    return d > 0.5 * L ? dm : (d < -0.5 * L ? dp : d);
}

// Displacement node coordinate - particle coordinate along axis a.
__device__ __forceinline__ double node_disp(const Geom &g, int axis, int coord, double xp) {
    const double d = (double)coord - xp;
    if (axis == 0) return disp_periodic(d, g.Lx);
    if (axis == 1) return g.wall_y ? d : disp_periodic(d, g.Ly);
    return disp_periodic(d, g.Lz);
}

// Sorts up to 4 owner records ascending (missing entries are 0xffffffff).
__device__ __forceinline__ void sort4(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d) {
#define LBIMB_CSWAP(p, q) { uint32_t lo_ = min(p, q), hi_ = max(p, q); p = lo_; q = hi_; }
    LBIMB_CSWAP(a, b); LBIMB_CSWAP(c, d); LBIMB_CSWAP(a, c); LBIMB_CSWAP(b, d); LBIMB_CSWAP(b, c);
#undef LBIMB_CSWAP
}

// Solid velocity V_S at node (x,y,z): count-weighted mean of the owners'
// rigid-body velocities v_p + omega_p x (x_n - x_p), owners in ascending id;
// also the total sub-sample count and the node's beta and (1 - beta)/tau from
// the tables.  Memory is read in three dependent rounds at most: the owner
// records (all at once), the two table entries together with the first
// owner's nine particle values, and one round per further owner.
template <class L>
__device__ __forceinline__ int solid_velocity(const LBArgs &a, int64_t n, int nown, int x, int y,
                                              int z, double V[3], double &beta, double &arel) {
    const int64_t N = a.g.N;
    const int k = nown < MAX_OWNERS ? nown : MAX_OWNERS;
    uint32_t r[4];
#pragma unroll
    for (int j = 0; j < MAX_OWNERS; j++) r[j] = j < k ? a.slots[(int64_t)j * N + n] : 0xffffffffu;
    sort4(r[0], r[1], r[2], r[3]);
    int total = 0;
#pragma unroll
    for (int j = 0; j < MAX_OWNERS; j++)
        if (j < k) total += (int)(r[j] & ((1u << SLOT_COUNT_BITS) - 1u));
    const int cc = total < a.Smax ? total : a.Smax;
    beta = a.beta_tab[cc];
    arel = a.arel_tab[cc];
    double num[3] = {0.0, 0.0, 0.0};
    const int P = a.np;
#pragma unroll
    for (int j = 0; j < MAX_OWNERS; j++) {
        if (j < k) {
            const int p = (int)(r[j] >> SLOT_COUNT_BITS);
            const int cnt = (int)(r[j] & ((1u << SLOT_COUNT_BITS) - 1u));
            const double X0 = a.px[p], X1 = a.px[P + p], X2 = L::D == 3 ? a.px[2 * P + p] : 0.0;
            const double U0 = a.pv[p], U1 = a.pv[P + p], U2 = L::D == 3 ? a.pv[2 * P + p] : 0.0;
            const double W0 = L::D == 3 ? a.pw[p] : 0.0, W1 = L::D == 3 ? a.pw[P + p] : 0.0;
            const double W2 = a.pw[2 * P + p];
            const double rx = node_disp(a.g, 0, x, X0);
            const double ry = node_disp(a.g, 1, y, X1);
            double vr[3];
            if (L::D == 3) {
                const double rz = node_disp(a.g, 2, z, X2);
                vr[0] = U0 + (W1 * rz - W2 * ry);
                vr[1] = U1 + (W2 * rx - W0 * rz);
                vr[2] = U2 + (W0 * ry - W1 * rx);
            } else {
                vr[0] = U0 - W2 * ry;
                vr[1] = U1 + W2 * rx;
                vr[2] = 0.0;
            }
            const double c = (double)cnt;
#pragma unroll
            for (int d = 0; d < L::D; d++) num[d] = num[d] + c * vr[d];
        }
    }
    const double den = (double)total;
#pragma unroll
    for (int d = 0; d < 3; d++) V[d] = d < L::D ? num[d] / den : 0.0;
    return total;
}

// The same in binary32 (half-precision storage path, whose collision is
// binary32): the node - centre displacement is formed in binary64 and rounded
// once, the rigid-body velocities and their count-weighted mean are binary32,
// beta and (1 - beta)/tau are the binary64 table entries rounded.  Holding no
// binary64 temporaries keeps that kernel at six wavefronts per SIMD.
template <class L>
__device__ __forceinline__ int solid_velocity_f32(const LBArgs &a, int64_t n, int nown, int x, int y,
                                                  int z, float V[3], float &beta, float &arel) {
    const int64_t N = a.g.N;
    const int k = nown < MAX_OWNERS ? nown : MAX_OWNERS;
    uint32_t r[4];
#pragma unroll
    for (int j = 0; j < MAX_OWNERS; j++) r[j] = j < k ? a.slots[(int64_t)j * N + n] : 0xffffffffu;
    sort4(r[0], r[1], r[2], r[3]);
    int total = 0;
#pragma unroll
    for (int j = 0; j < MAX_OWNERS; j++)
        if (j < k) total += (int)(r[j] & ((1u << SLOT_COUNT_BITS) - 1u));
    const int cc = total < a.Smax ? total : a.Smax;
    beta = (float)a.beta_tab[cc];
    arel = (float)a.arel_tab[cc];
    float num[3] = {0.0f, 0.0f, 0.0f};
    const int P = a.np;
#pragma unroll
    for (int j = 0; j < MAX_OWNERS; j++) {
        if (j < k) {
            const int p = (int)(r[j] >> SLOT_COUNT_BITS);
            const int cnt = (int)(r[j] & ((1u << SLOT_COUNT_BITS) - 1u));
            const float rx = (float)node_disp(a.g, 0, x, a.px[p]);
            const float ry = (float)node_disp(a.g, 1, y, a.px[P + p]);
            const float U0 = (float)a.pv[p], U1 = (float)a.pv[P + p];
            const float U2 = L::D == 3 ? (float)a.pv[2 * P + p] : 0.0f;
            const float W0 = L::D == 3 ? (float)a.pw[p] : 0.0f, W1 = L::D == 3 ? (float)a.pw[P + p] : 0.0f;
            const float W2 = (float)a.pw[2 * P + p];
            float vr[3];
            if (L::D == 3) {
                const float rz = (float)node_disp(a.g, 2, z, a.px[2 * P + p]);
                vr[0] = U0 + (W1 * rz - W2 * ry);
                vr[1] = U1 + (W2 * rx - W0 * rz);
                vr[2] = U2 + (W0 * ry - W1 * rx);
            } else {
                vr[0] = U0 - W2 * ry;
                vr[1] = U1 + W2 * rx;
                vr[2] = 0.0f;
            }
            const float c = (float)cnt;
#pragma unroll
            for (int d = 0; d < L::D; d++) num[d] = num[d] + c * vr[d];
        }
    }
    const float den = (float)total;
#pragma unroll
    for (int d = 0; d < 3; d++) V[d] = d < L::D ? num[d] / den : 0.0f;
    return total;
}

// ------------------------------------------------------------- pull gather
// Element (i, x, y, z) of a state array.
__device__ __forceinline__ uint64_t row_elem(const Geom &g, int Q, int i, int y, int z) {
    return (((uint64_t)z * (uint64_t)g.ny + (uint64_t)y) * (uint64_t)Q + (uint64_t)i) * (uint64_t)g.nx;
}

template <class T>
__device__ __forceinline__ const T *lane(const T *row, uint32_t xbytes) {
    return (const T *)((const char *)row + xbytes);
}

template <class T>
__device__ __forceinline__ T *lane(T *row, uint32_t xbytes) {
    return (T *)((char *)row + xbytes);
}

// f_i(x) = A_i(x - c_i), or A_opp(i)(x) when x - c_i lies beyond a wall.  All
// threads of a block share y and z (the grid is one block row per lattice row),
// so the bounce-back test and every source row base are uniform per block
// (scalar registers); a lane adds its x, x - 1 or x + 1 (wrapped) byte offset.
template <class L, class T>
__device__ __forceinline__ void gather(const T *__restrict__ A, const Geom &g, int x, int y, int z,
                                       T (&f)[L::Q]) {
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    int ym = y - 1, yp = y + 1;
    bool lo = false, hi = false;
    if (g.wall_y) {
        lo = (y == 0);
        hi = (y == ny - 1);
    } else {
        if (ym < 0) ym = ny - 1;
        if (yp >= ny) yp = 0;
    }
    const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
    const uint32_t sz = (uint32_t)sizeof(T);
    const uint32_t ox[3] = {(uint32_t)x * sz, (uint32_t)xm * sz, (uint32_t)xp * sz};
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const int sy = L::cy[i] == 0 ? y : (L::cy[i] > 0 ? ym : yp);
        const int szz = L::cz[i] == 0 ? z : (L::cz[i] > 0 ? zm : zp);
        const bool bb = (L::cy[i] > 0 && lo) || (L::cy[i] < 0 && hi);
        const uint32_t xo = ox[L::cx[i] == 0 ? 0 : (L::cx[i] > 0 ? 1 : 2)];
        const T *src = bb ? lane(A + row_elem(g, L::Q, L::opp[i], y, z), ox[0])
                          : lane(A + row_elem(g, L::Q, i, sy, szz), xo);
        // binary64 populations are read with the non-temporal hint (measured
        // faster for the 8-byte pull on gfx950; no gain for the narrower types)
        f[i] = sizeof(T) == 8 ? __builtin_nontemporal_load(src) : *src;
    }
}

// ------------------------------------------------------ FP64 collision
// Equilibria are evaluated where they are used and every post-collision value
// is stored as soon as it is known, so only the Q gathered populations stay
// live in registers.
template <class L>
struct Eq64 {
    double ux, uy, uz, t15, wr[3];
    __device__ __forceinline__ double operator()(int i) const {
        if (i == 0) return wr[0] * (1.0 - t15);
        const double cu = cdot<L>(i, ux, uy, uz);
        return wr[L::wc[i]] * (1.0 + 3.0 * cu + 4.5 * cu * cu - t15);
    }
};

template <class L>
__device__ __forceinline__ void collide_f64(const LBArgs &a, uint64_t n, int x, int y, int z,
                                            const double (&f)[L::Q], int nown) {
    double rho = f[0];
#pragma unroll
    for (int i = 1; i < L::Q; i++) rho = rho + f[i];
    const double jx = cmoment<L, 0>(f), jy = cmoment<L, 1>(f);
    const double jz = L::D == 3 ? cmoment<L, 2>(f) : 0.0;
    Eq64<L> eq;
    eq.ux = jx / rho;
    eq.uy = jy / rho;
    eq.uz = L::D == 3 ? jz / rho : 0.0;
    double usq = eq.ux * eq.ux + eq.uy * eq.uy;
    if (L::D == 3) usq = usq + eq.uz * eq.uz;
    eq.t15 = 1.5 * usq;
    eq.wr[0] = L::w[0] * rho;
    eq.wr[1] = L::w[1] * rho;
    eq.wr[2] = L::w[2] * rho;
    const double w3r[3] = {3.0 * L::w[0] * rho, 3.0 * L::w[1] * rho, 3.0 * L::w[2] * rho};
    double *const Brow = (double *)a.B + row_elem(a.g, L::Q, 0, y, z);
    const uint32_t xb = (uint32_t)x * 8u;

    // A wavefront with no covered node takes the plain BGK path.  Otherwise
    // every lane takes the IMB path; an uncovered lane then has beta = 0,
    // a = 1/tau and V_S = 0, for which the IMB formula gives the same bits as
    // the plain one (beta * Omega adds +-0).  Keeping the wavefront converged
    // keeps every population store a full-wavefront store.
    if (!__any(nown != 0)) {
        const double ar = a.arel0;
#pragma unroll
        for (int i = 0; i < L::Q; i++) {
            const double out = f[i] - ar * (f[i] - eq(i)) + w3r[L::wc[i]] * a.cg[i];
            __builtin_nontemporal_store(out, lane(Brow + (uint64_t)i * a.g.nx, xb));
        }
        return;
    }
    if (nown > MAX_OWNERS) atomicOr(a.flags, FLAG_SLOT_OVERFLOW);
    double V[3] = {0.0, 0.0, 0.0};
    int total = 0;
    double beta = 0.0, ar = a.arel0;
    if (nown != 0) total = solid_velocity<L>(a, (int64_t)n, nown, x, y, z, V, beta, ar);
    double VV = V[0] * V[0] + V[1] * V[1];
    if (L::D == 3) VV = VV + V[2] * V[2];
    Eq64<L> eqV = eq;
    eqV.ux = V[0];
    eqV.uy = V[1];
    eqV.uz = V[2];
    eqV.t15 = 1.5 * VV;
    double mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const int o = L::opp[i];
        const double Om = (f[o] - f[i]) + (eqV(i) - eq(o));
        const double out = f[i] - ar * (f[i] - eq(i)) + beta * Om + w3r[L::wc[i]] * a.cg[i];
        __builtin_nontemporal_store(out, lane(Brow + (uint64_t)i * a.g.nx, xb));
        if (L::cx[i] > 0) mx = mx + Om; else if (L::cx[i] < 0) mx = mx - Om;
        if (L::cy[i] > 0) my = my + Om; else if (L::cy[i] < 0) my = my - Om;
        if (L::D == 3) { if (L::cz[i] > 0) mz = mz + Om; else if (L::cz[i] < 0) mz = mz - Om; }
    }
    if (nown != 0) {
        QRec r;
        r.q[0] = beta * mx;
        r.q[1] = beta * my;
        r.q[2] = L::D == 3 ? beta * mz : 0.0;
        r.tot = total;
        r.pad = 0;
        ((QRec *)a.qr)[n] = r;
        a.nown[n] = 0;  // the next footprint starts from zero counts
    }
}

// ------------------------------------------- shifted storage, FP32 compute
// g_i = f_i - w_i (rho_0 = 1):  drho = sum g, rho = 1 + drho, u = sum g c / rho,
// g^eq_i = w_i (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2)); the solid operator
// keeps its exact form because the w_i terms cancel:
// Omega_i = (g_-i - g_i) + w_i rho [(3 cV + 4.5 cV^2 - 1.5 V^2) - (-3 cu + 4.5 cu^2 - 1.5 u^2)].
template <class L, int ST>
__device__ __forceinline__ void collide_shifted(const LBArgs &a, uint64_t n, int x, int y, int z,
                                                const float (&gg)[L::Q], int nown) {
    using T = typename Store<ST>::T;
    T *const Brow = (T *)a.B + row_elem(a.g, L::Q, 0, y, z);
    const uint32_t xb = (uint32_t)x * (uint32_t)sizeof(T);
    auto put = [&](int i, float v) {
        __builtin_nontemporal_store((T)v, lane(Brow + (uint64_t)i * a.g.nx, xb));
    };
    const bool wave_fluid = !__any(nown != 0);
    float beta = 0.0f, ar = a.arel0f;
    float V[3] = {0.0f, 0.0f, 0.0f};
    int total = 0;
    if (!wave_fluid && nown != 0) {
        if (nown > MAX_OWNERS) atomicOr(a.flags, FLAG_SLOT_OVERFLOW);
        if (ST == 2) {
            // half-precision storage: binary32 V_S (six wavefronts per SIMD
            // instead of five, measured faster); binary32 storage keeps the
            // binary64 V_S (measured faster there)
            total = solid_velocity_f32<L>(a, (int64_t)n, nown, x, y, z, V, beta, ar);
        } else {
            double Vd[3], bd, ad;
            total = solid_velocity<L>(a, (int64_t)n, nown, x, y, z, Vd, bd, ad);
            for (int d = 0; d < 3; d++) V[d] = (float)Vd[d];
            beta = (float)bd;
            ar = (float)ad;
        }
    }
    float mom[3];
    shifted_node<L, ST == 2>(gg, wave_fluid, beta, ar, V[0], V[1], V[2], a.cgf, put, mom);
    if (nown != 0) {
        QRec32 r;
        r.q[0] = mom[0];
        r.q[1] = mom[1];
        r.q[2] = L::D == 3 ? mom[2] : 0.0f;
        r.tot = total;
        ((QRec32 *)a.qr)[n] = r;
        a.nown[n] = 0;  // the next footprint starts from zero counts
    }
}

// Workgroup -> tile (x stretch, row y, z).  Linear order: the tile is the
// workgroup's own coordinates.  XCD order: the hardware deals workgroup ids
// (x fastest) to its 8 XCDs in turn, id mod 8; the ids one XCD receives are
// renumbered to one contiguous run of tiles, so that the stretches of a row
// and the neighbouring rows share that XCD's L2.  The renumbering is a
// bijection of [0, G) for any G (the first G mod 8 XCDs take one tile more);
// the launcher uses it only for grids of fewer than 2^32 workgroups.
template <bool XO>
__device__ __forceinline__ void tile_of(uint32_t &xt, int &y, int &z) {
    if (!XO) {
        xt = blockIdx.x;
        y = blockIdx.y;
        z = blockIdx.z;
        return;
    }
    const uint32_t gx = gridDim.x, G = gx * gridDim.y * gridDim.z;
    const uint32_t b = blockIdx.x + gx * (blockIdx.y + gridDim.y * blockIdx.z);
    const uint32_t k = b & 7u, q = G >> 3, r = G & 7u;
    const uint32_t t = (k < r ? k * (q + 1) : r * (q + 1) + (k - r) * q) + (b >> 3);
    const uint32_t row = t / gx;
    xt = t - row * gx;
    y = (int)(row % gridDim.y);
    z = (int)(row / gridDim.y);
}

template <class L, int ST, bool XO>
__global__ __launch_bounds__(256) void k_lb(LBArgs a) {
    uint32_t xt;
    int y, z;
    tile_of<XO>(xt, y, z);
    y += a.y0;  // the launch covers rows y0 .. y0 + ny_run - 1
    const int x = (int)xt * blockDim.x + threadIdx.x;
    if (x >= a.g.nx) return;
    const uint64_t n = (uint64_t)x + (uint64_t)a.g.nx * ((uint64_t)y + (uint64_t)a.g.ny * (uint64_t)z);
    using T = typename Store<ST>::T;
    // the owner count is read before the populations, so a wavefront with a
    // covered node can start its owner-record reads while they arrive
    const int nown = a.nown[n];
    T f[L::Q];
    gather<L, T>((const T *)a.A, a.g, x, y, z, f);
    if (ST == 0) {
        double fd[L::Q];
#pragma unroll
        for (int i = 0; i < L::Q; i++) fd[i] = (double)f[i];
        collide_f64<L>(a, n, x, y, z, fd, nown);
    } else {
        // FP32 storage holds g_i, FP16 storage g_i / w_i; the collision works
        // in the storage unit
        float gg[L::Q];
#pragma unroll
        for (int i = 0; i < L::Q; i++) gg[i] = (float)f[i];
        collide_shifted<L, ST>(a, n, x, y, z, gg, nown);
    }
}

// ---------------------------------------------- state conversion kernels
// Decoded population f_i = w_i + g_i in binary64.
template <class L, int ST>
__device__ __forceinline__ double decode(int i, typename Store<ST>::T v) {
    if (ST == 0) return (double)v;
    const float wf = (float)L::w[L::wc[i]];
    const float gv = ST == 1 ? (float)v : wf * (float)v;
    return L::w[L::wc[i]] + (double)gv;
}

template <class L, int ST>
__device__ __forceinline__ typename Store<ST>::T encode(int i, double fv) {
    using T = typename Store<ST>::T;
    if (ST == 0) return (T)fv;
    const float gv = (float)(fv - L::w[L::wc[i]]);
    if (ST == 1) return (T)gv;
    return (T)(gv * L::invw[L::wc[i]]);
}

template <class L, int ST>
__global__ void k_get_f(Geom g, const void *A, double *f) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const int64_t n = (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
    using T = typename Store<ST>::T;
    T v[L::Q];
    gather<L, T>((const T *)A, g, x, y, z, v);
#pragma unroll
    for (int i = 0; i < L::Q; i++) f[(int64_t)i * g.N + n] = decode<L, ST>(i, v[i]);
}

template <class L, int ST>
__global__ void k_macro(Geom g, const void *A, double *rho, double *u) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const int64_t n = (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
    using T = typename Store<ST>::T;
    T v[L::Q];
    gather<L, T>((const T *)A, g, x, y, z, v);
    double fd[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; i++) fd[i] = decode<L, ST>(i, v[i]);
    double r = fd[0];
#pragma unroll
    for (int i = 1; i < L::Q; i++) r = r + fd[i];
    rho[n] = r;
    u[n] = cmoment<L, 0>(fd) / r;
    u[g.N + n] = cmoment<L, 1>(fd) / r;
    if (L::D == 3) u[2 * g.N + n] = cmoment<L, 2>(fd) / r;
}

// Inverse of the pull streaming: A_j(x) = f_j(x + c_j), or f_opp(j)(x) when
// x + c_j lies beyond a wall.
template <class L, int ST>
__global__ void k_set_f(Geom g, const double *f, void *Av) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const int64_t n = (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
    using T = typename Store<ST>::T;
    T *A = (T *)Av;
#pragma unroll
    for (int j = 0; j < L::Q; j++) {
        int tx = x + L::cx[j], ty = y + L::cy[j], tz = z + L::cz[j];
        tx = tx < 0 ? tx + g.nx : (tx >= g.nx ? tx - g.nx : tx);
        tz = tz < 0 ? tz + g.nz : (tz >= g.nz ? tz - g.nz : tz);
        bool beyond = false;
        if (g.wall_y) beyond = ty < 0 || ty >= g.ny;
        else ty = ty < 0 ? ty + g.ny : (ty >= g.ny ? ty - g.ny : ty);
        double val;
        if (beyond) val = f[(int64_t)L::opp[j] * g.N + n];
        else val = f[(int64_t)j * g.N + (int64_t)tx + (int64_t)g.nx * ((int64_t)ty + (int64_t)g.ny * tz)];
        A[row_elem(g, L::Q, j, y, z) + (uint64_t)x] = encode<L, ST>(j, val);
    }
}

// FP64 rest state f_i = f^eq_i(1, 0) = w_i at every node, in the state layout.
template <class L>
__global__ void k_fill_rest_f64(Geom g, double *A) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
#pragma unroll
    for (int i = 0; i < L::Q; i++) A[row_elem(g, L::Q, i, y, z) + (uint64_t)x] = L::w[L::wc[i]];
}

__global__ void k_fill_u32(uint32_t *p, uint32_t value, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < count; k += stride) p[k] = value;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t value, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < count; k += stride) p[k] = value;
}

// ---------------------------------------------------------------- launchers
static dim3 lattice_grid(const Geom &g, int &block) {
    block = g.nx >= 256 ? 256 : ((g.nx + 63) / 64) * 64;
    return dim3((unsigned)((g.nx + block - 1) / block), (unsigned)g.ny, (unsigned)g.nz);
}

template <class L, int ST>
static hipError_t lb_dispatch(const LBArgs &a, int width, int order, int cu_groups, hipStream_t s) {
    int block;
    dim3 grid = lattice_grid(a.g, block);
    grid.y = (unsigned)a.ny_run;
    if (width > 0) {
        // a chosen workgroup width: part of one row per workgroup, the ragged
        // end of a row masked by the kernel's x < nx test
        block = width;
        grid.x = (unsigned)((a.g.nx + width - 1) / width);
    }
    const uint64_t groups = (uint64_t)grid.x * grid.y * grid.z;
    const unsigned lds = lds_reserve_bytes(cu_groups);
    if (order == 1 && groups < ((uint64_t)1 << 32))
        hipLaunchKernelGGL((k_lb<L, ST, true>), grid, dim3(block), lds, s, a);
    else
        hipLaunchKernelGGL((k_lb<L, ST, false>), grid, dim3(block), lds, s, a);
    return hipGetLastError();
}

// The lattice kernel uses no LDS.  Reserving an unused share of a CU's 160 KiB
// caps how many of its workgroups a CU holds at once (cu_groups, 3..8), below
// what its registers allow; 0 reserves nothing.
unsigned lds_reserve_bytes(int cu_groups) {
    if (cu_groups <= 0) return 0;
    return (unsigned)(163840 / cu_groups) / 512u * 512u;
}

bool xcd_order_fits(const Geom &g, int width) {
    const int w = lattice_block_width(g.nx, width);
    return (uint64_t)((g.nx + w - 1) / w) * (uint64_t)g.ny * (uint64_t)g.nz < ((uint64_t)1 << 32);
}

int lattice_block_width(int nx, int width) {
    if (width > 0) return width;
    Geom g{};
    g.nx = nx;
    int block;
    (void)lattice_grid(g, block);
    return block;
}

hipError_t launch_lb(int lattice, int storage, const LBArgs &a, int width, int order, int cu_groups,
                     hipStream_t s) {
    if (lattice == 0) {
        if (storage == 0) return lb_dispatch<D2Q9, 0>(a, width, order, cu_groups, s);
        if (storage == 1) return lb_dispatch<D2Q9, 1>(a, width, order, cu_groups, s);
        return lb_dispatch<D2Q9, 2>(a, width, order, cu_groups, s);
    }
    if (storage == 0) return lb_dispatch<D3Q19, 0>(a, width, order, cu_groups, s);
    if (storage == 1) return lb_dispatch<D3Q19, 1>(a, width, order, cu_groups, s);
    return lb_dispatch<D3Q19, 2>(a, width, order, cu_groups, s);
}

#define LBIMB_DISPATCH(KERNEL, ...)                                                          \
    do {                                                                                     \
        int block_;                                                                          \
        dim3 grid_ = lattice_grid(g, block_);                                                \
        if (lattice == 0) {                                                                  \
            if (storage == 0) hipLaunchKernelGGL((KERNEL<D2Q9, 0>), grid_, dim3(block_), 0, s, __VA_ARGS__); \
            else if (storage == 1) hipLaunchKernelGGL((KERNEL<D2Q9, 1>), grid_, dim3(block_), 0, s, __VA_ARGS__); \
            else hipLaunchKernelGGL((KERNEL<D2Q9, 2>), grid_, dim3(block_), 0, s, __VA_ARGS__); \
        } else {                                                                             \
            if (storage == 0) hipLaunchKernelGGL((KERNEL<D3Q19, 0>), grid_, dim3(block_), 0, s, __VA_ARGS__); \
            else if (storage == 1) hipLaunchKernelGGL((KERNEL<D3Q19, 1>), grid_, dim3(block_), 0, s, __VA_ARGS__); \
            else hipLaunchKernelGGL((KERNEL<D3Q19, 2>), grid_, dim3(block_), 0, s, __VA_ARGS__); \
        }                                                                                    \
    } while (0)

hipError_t launch_fill_rest_f64(int lattice, const Geom &g, double *A, hipStream_t s) {
    int block;
    dim3 grid = lattice_grid(g, block);
    if (lattice == 0) hipLaunchKernelGGL(k_fill_rest_f64<D2Q9>, grid, dim3(block), 0, s, g, A);
    else hipLaunchKernelGGL(k_fill_rest_f64<D3Q19>, grid, dim3(block), 0, s, g, A);
    return hipGetLastError();
}

hipError_t launch_get_f(int lattice, int storage, const Geom &g, const void *A, double *f,
                        hipStream_t s) {
    LBIMB_DISPATCH(k_get_f, g, A, f);
    return hipGetLastError();
}

hipError_t launch_set_f(int lattice, int storage, const Geom &g, const double *f, void *A,
                        hipStream_t s) {
    LBIMB_DISPATCH(k_set_f, g, f, A);
    return hipGetLastError();
}

hipError_t launch_macro(int lattice, int storage, const Geom &g, const void *A, double *rho,
                        double *u, hipStream_t s) {
    LBIMB_DISPATCH(k_macro, g, A, rho, u);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

}  // namespace lbimb
