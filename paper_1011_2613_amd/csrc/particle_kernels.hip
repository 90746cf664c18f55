// particle_kernels.hip -- particle side of the LB-IMB-DEM step on gfx950:
// footprint / solid fraction, hydrodynamic force and torque sums (Eq. 3),
// DEM cell list, contact forces (Eqs. 4-5) and time integration.
//
// All particle arithmetic is binary64 in every storage mode.  Sums whose
// order differs from a sequential loop (the per-particle force reduction) use
// error-free TwoSum accumulation (Ogita, Rump & Oishi 2005) so the rounded
// result does not depend on the reduction tree.
#include <algorithm>

#include "internal.h"

namespace lbimb {

__device__ __forceinline__ double pdisp(double d, double L) {
    if (d > 0.5 * L) d = d - L;
    else if (d < -0.5 * L) d = d + L;
    return d;
}

__device__ __forceinline__ double ndisp(const Geom &g, int axis, int coord, double xp) {
    double d = (double)coord - xp;
    if (axis == 0) return pdisp(d, g.Lx);
    if (axis == 1) return g.wall_y ? d : pdisp(d, g.Ly);
    return pdisp(d, g.Lz);
}

// Wrap an unwrapped node coordinate; -1 beyond a wall.
__device__ __forceinline__ int wrapc(const Geom &g, int axis, int c) {
    const int n = axis == 0 ? g.nx : (axis == 1 ? g.ny : g.nz);
    if (axis == 1 && g.wall_y) return (c < 0 || c >= n) ? -1 : c;
    c %= n;
    return c < 0 ? c + n : c;
}

// Bounding box of nodes whose cell may hold samples of the particle:
// ceil(x - R - 1/2) .. floor(x + R + 1/2) per axis.
__device__ __forceinline__ void bbox(const Particles &P, int p, int D, int lo[3], int hi[3]) {
    const double r = P.R[p];
    for (int a = 0; a < 3; a++) {
        if (a >= D) { lo[a] = hi[a] = 0; continue; }
        const double c = P.x[a * P.np + p];
        lo[a] = (int)ceil(c - r - 0.5);
        hi[a] = (int)floor(c + r + 0.5);
    }
}

// Number of sub-cell samples of a node inside a particle: offsets
// (k + 1/2)/S - 1/2 per axis from the node, inside test dx^2 + dy^2 (+ dz^2)
// <= R^2 evaluated left to right, d0/d1/d2 the node-minus-centre displacement.
// The squared offsets are separable, so a node needs S^D additions.  (Called
// only for nodes the distance bounds left undecided, so no shortcut for
// all-inside or all-outside nodes is taken here.)
template <int D, int S>
__device__ __forceinline__ int sample_count(double d0, double d1, double d2, double R2) {
    double sx[S], sz[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        const double off = ((double)s + 0.5) / (double)S - 0.5;
        const double ex = d0 + off;
        sx[s] = ex * ex;
        const double ez = d2 + off;
        sz[s] = D == 3 ? ez * ez : 0.0;
    }
    int count = 0;
    // one row of samples (fixed y offset) per iteration, kept rolled so
    // that only that row's partial sums are live
#pragma unroll 1
    for (int ky = 0; ky < S; ky++) {
        const double ey = d1 + (((double)ky + 0.5) / (double)S - 0.5);
        const double sy = ey * ey;
#pragma unroll
        for (int kx = 0; kx < S; kx++) {
            const double t = sx[kx] + sy;
            if (D == 2) {
                count += (t <= R2) ? 1 : 0;
            } else {
#pragma unroll
                for (int kz = 0; kz < S; kz++) count += (t + sz[kz] <= R2) ? 1 : 0;
            }
        }
    }
    return count;
}

// Unwrapped coordinate -> lattice coordinate.  A bounding box is narrower than
// the periodic box, so one conditional shift suffices; -1 beyond a wall.
__device__ __forceinline__ int wrap1(const Geom &g, int axis, int c) {
    const int n = axis == 0 ? g.nx : (axis == 1 ? g.ny : g.nz);
    if (axis == 1 && g.wall_y) return (c < 0 || c >= n) ? -1 : c;
    return c < 0 ? c + n : (c >= n ? c - n : c);
}

constexpr uint32_t LIST_COUNT_MASK = 1023u;

// floor(v / d) for 0 <= v < 2^24 and 1 <= d < 2^12: binary32 estimate from the
// reciprocal, then one exact integer correction step.
__device__ __forceinline__ int div_small(int v, int d, float inv_d) {
    int q = (int)((float)v * inv_d);
    const int r = v - q * d;
    if (r < 0) q -= 1;
    else if (r >= d) q += 1;
    return q;
}

__device__ __forceinline__ uint32_t list_entry(int count, int kx, int ky, int kz) {
    return (uint32_t)count | ((uint32_t)kx << 10) | ((uint32_t)ky << 17) | ((uint32_t)kz << 24);
}

// Exclusive prefix sum over the threads of a workgroup (<= 256 threads);
// `total` receives the sum.  Every thread of the workgroup must call it.
__device__ __forceinline__ int block_scan(int v, int &total) {
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63 || threadIdx.x == blockDim.x - 1) wsum[wave] = x;
    __syncthreads();
    int before = 0;
    total = 0;
    for (int w = 0; w < nw; w++) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    __syncthreads();
    return before + x - v;
}

// Conservative classification of a node from per-axis distance bounds: 0 when
// every sub-cell sample is certainly outside, S^D when every sample is
// certainly inside, -1 otherwise.  With h = 1/2 - 1/(2S) the largest sample
// offset, the sum of squares of every sample lies in [lo, hi] built from
// max(|d| - h, 0) and |d| + h; rounding moves the tested sums and the bounds
// by a few units in the last place, far inside the 1e-14 relative margins,
// so a decided node gets exactly the count the per-sample test gives.
template <int D, int S>
__device__ __forceinline__ int classify(double d0, double d1, double d2, double R2) {
    const double h = 0.5 - 0.5 / (double)S;
    const double a0 = fabs(d0), a1 = fabs(d1), a2 = fabs(d2);
    const double m0 = fmax(a0 - h, 0.0), m1 = fmax(a1 - h, 0.0), m2 = fmax(a2 - h, 0.0);
    const double M0 = a0 + h, M1 = a1 + h, M2 = a2 + h;
    double lo = m0 * m0 + m1 * m1, hi = M0 * M0 + M1 * M1;
    if (D == 3) {
        lo = lo + m2 * m2;
        hi = hi + M2 * M2;
    }
    if (lo * (1.0 - 1e-14) > R2) return 0;
    if (hi * (1.0 + 1e-14) <= R2) return D == 3 ? S * S * S : S * S;
    return -1;
}

// Table-lookup eps (Eq. 6): the count of a node at displacement (d0, d1, d2)
// from the centre, from rho = |r| - R and the folded direction of r (sorted
// magnitudes a >= b >= c, t1 = b/|r|, t2 = c/|r|); wholly inside for
// rho <= -H, outside for rho >= H (H = sqrt(D)/2, half a cell diagonal).
template <int D, int SMAX>
__device__ __forceinline__ int eps_lookup(const FootArgs &a, double d0, double d1, double d2, double R) {
    double r2 = d0 * d0 + d1 * d1;
    if (D == 3) r2 = r2 + d2 * d2;
    // wholly inside or outside by a relative margin of 1e-12 on |r|^2 (far
    // above the rounding of sqrt(|r|^2) - R): the same decision as below
    // without the square root
    const double ri = R - a.tabH, ro = R + a.tabH;
    if (r2 < ri * ri * (1.0 - 1e-12)) return SMAX;
    if (r2 > ro * ro * (1.0 + 1e-12)) return 0;
    const double r = sqrt(r2);
    const double rho = r - R;
    if (rho <= -a.tabH) return SMAX;
    if (rho >= a.tabH) return 0;
    int ir = (int)floor((rho + a.tabH) / a.tabW);
    ir = ir < 0 ? 0 : (ir > EPS_TAB_NRHO - 1 ? EPS_TAB_NRHO - 1 : ir);
    double x = fabs(d0), y = fabs(d1), z = D == 3 ? fabs(d2) : 0.0, t;
    if (y > x) { t = x; x = y; y = t; }
    if (z > y) { t = y; y = z; z = t; }
    if (y > x) { t = x; x = y; y = t; }
    int i1 = (int)floor(y / r * a.tabK1);
    i1 = i1 > EPS_TAB_NT - 1 ? EPS_TAB_NT - 1 : i1;
    if (D == 2) return a.tab[ir * EPS_TAB_NT + i1];
    int i2 = (int)floor(z / r * a.tabK2);
    i2 = i2 > EPS_TAB_NT - 1 ? EPS_TAB_NT - 1 : i2;
    return a.tab[(ir * EPS_TAB_NT + i1) * EPS_TAB_NT + i2];
}

// Footprint of one particle, one workgroup.  The bounding box is taken in
// chunks of nodes: (A) every node is classified by distance bounds, undecided
// nodes are queued in LDS; (B) the queued nodes get the exact per-sample count,
// the workgroup's lanes all busy with such nodes; (C1) a workgroup prefix sum
// lists the covered nodes of the chunk in node order (x fastest); (C2) the
// k-th covered node takes place k of the particle's list and an owner slot, so
// the list is the same on every run.
template <int D, int S, int NT, bool TAB>
__device__ __forceinline__ void foot_one(const FootArgs &a, int p) {
    constexpr int CHUNK = 1024;
    __shared__ uint16_t s_cnt[CHUNK];
    __shared__ uint16_t s_todo[CHUNK];
    __shared__ int s_ntodo;
    const int P = a.P.np;
    int lo[3], hi[3];
    bbox(a.P, p, D, lo, hi);
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; d++) {
            a.P.bb[d * P + p] = lo[d];
            a.P.bb[(3 + d) * P + p] = hi[d];
        }
    // A centre must lie in the box on periodic axes (integration keeps it
    // there unless a particle moves a box length in one step) and be finite:
    // otherwise the bounding box cannot be wrapped and the particle gets an
    // empty footprint and an error flag.
    bool placed = true;
    for (int d = 0; d < D; d++) {
        const double c = a.P.x[d * P + p];
        const double L = d == 0 ? a.g.Lx : (d == 1 ? a.g.Ly : a.g.Lz);
        placed = placed && ((d == 1 && a.g.wall_y) ? (c > -L && c < 2.0 * L) : (c >= 0.0 && c < L));
    }
    if (!placed && threadIdx.x == 0) atomicOr(a.flags, FLAG_NONFINITE);
    const int ext0 = hi[0] - lo[0] + 1, ext1 = hi[1] - lo[1] + 1;
    const int ext2 = D == 3 ? hi[2] - lo[2] + 1 : 1;
    const int items = placed ? ext0 * ext1 * ext2 : 0;
    const double r = a.P.R[p];
    const double R2 = r * r;
    const double xp0 = a.P.x[p], xp1 = a.P.x[P + p], xp2 = D == 3 ? a.P.x[2 * P + p] : 0.0;
    const int64_t N = a.g.N;
    const int cap = a.P.list_cap;
    uint32_t *list = a.P.list + (int64_t)p * cap;
    const float inv0 = 1.0f / (float)ext0, inv1 = 1.0f / (float)ext1;
    // node of a bounding-box item: lattice coordinates (iy < 0 beyond a wall)
    auto node_of = [&](int item, int &kx, int &ky, int &kz, int &ix, int &iy, int &iz) {
        const int rest = div_small(item, ext0, inv0);
        kx = item - rest * ext0;
        kz = div_small(rest, ext1, inv1);
        ky = rest - kz * ext1;
        iy = wrap1(a.g, 1, lo[1] + ky);
        ix = wrap1(a.g, 0, lo[0] + kx);
        iz = D == 3 ? wrap1(a.g, 2, lo[2] + kz) : 0;
    };
    int base = 0;
    for (int c0 = 0; c0 < items; c0 += CHUNK) {
        const int nc = items - c0 < CHUNK ? items - c0 : CHUNK;
        if (threadIdx.x == 0) s_ntodo = 0;
        __syncthreads();
        // (A) classify
#pragma unroll 1
        for (int i = threadIdx.x; i < nc; i += NT) {
            int kx, ky, kz, ix, iy, iz;
            node_of(c0 + i, kx, ky, kz, ix, iy, iz);
            int cls = 0;
            if (iy >= 0) {
                const double d0 = ndisp(a.g, 0, ix, xp0), d1 = ndisp(a.g, 1, iy, xp1);
                const double d2 = D == 3 ? ndisp(a.g, 2, iz, xp2) : 0.0;
                if (TAB) cls = eps_lookup<D, D == 3 ? S * S * S : S * S>(a, d0, d1, d2, r);
                else cls = classify<D, S>(d0, d1, d2, R2);
            }
            if (cls < 0) s_todo[atomicAdd(&s_ntodo, 1)] = (uint16_t)i;
            else s_cnt[i] = (uint16_t)cls;
        }
        __syncthreads();
        // (B) exact per-sample counts of the undecided nodes
        const int ntodo = s_ntodo;
#pragma unroll 1
        for (int j = threadIdx.x; j < ntodo; j += NT) {
            const int i = s_todo[j];
            int kx, ky, kz, ix, iy, iz;
            node_of(c0 + i, kx, ky, kz, ix, iy, iz);
            s_cnt[i] = (uint16_t)sample_count<D, S>(ndisp(a.g, 0, ix, xp0), ndisp(a.g, 1, iy, xp1),
                                                    D == 3 ? ndisp(a.g, 2, iz, xp2) : 0.0, R2);
        }
        __syncthreads();
        // (C1) the covered nodes of the chunk in node order into s_todo (the
        // queue of (B) is spent): each thread takes ceil(nc / NT) consecutive
        // nodes of the chunk (a disc's box fills a seventh of a chunk), one
        // workgroup prefix sum places them
        {
            const int per = (nc + NT - 1) / NT;
            const int j0 = min((int)threadIdx.x * per, nc), j1 = min(j0 + per, nc);
            int m = 0;
            for (int j = j0; j < j1; j++) m += s_cnt[j] > 0 ? 1 : 0;
            int ncov;
            int at = block_scan(m, ncov);
            for (int j = j0; j < j1; j++)
                if (s_cnt[j] > 0) s_todo[at++] = (uint16_t)j;
            __syncthreads();
            // (C2) owner slots and list entries, k-th covered node in lane
            // order.  Covered nodes that fall in one aligned 8-byte word of the
            // owner counts sit in consecutive lanes; the first lane of such a
            // run claims all of them with one 64-bit atomic add and every lane
            // of the run reads its own byte of the returned word, which is what
            // one atomic add per node in lane order would have returned.
            const int lane = threadIdx.x & 63;
#pragma unroll 1
            for (int k0 = 0; k0 < ncov; k0 += NT) {
                const int k = k0 + (int)threadIdx.x;
                int count = 0, kx = 0, ky = 0, kz = 0;
                int64_t n = 0;
                long long key = -1;  // owner-count word of a covered node
                if (k < ncov) {
                    const int i = s_todo[k];
                    count = s_cnt[i];
                    int ix, iy, iz;
                    node_of(c0 + i, kx, ky, kz, ix, iy, iz);
                    n = (int64_t)ix + (int64_t)a.g.nx * ((int64_t)iy + (int64_t)a.g.ny * iz);
                    key = (long long)(n >> 3);
                }
                const int byte = (int)(n & 7);
                uint32_t mask = key >= 0 ? 1u << byte : 0u;
                int back = 0;  // lanes between this one and the first of its run
                bool run = true;
#pragma unroll
                for (int j = 1; j < 8; j++) {
                    const long long kj = __shfl_up(key, j, 64);
                    run = run && lane >= j && kj == key;
                    back += run ? 1 : 0;
                }
                run = true;
#pragma unroll
                for (int j = 1; j < 8; j++) {
                    const long long kj = __shfl_down(key, j, 64);
                    const uint32_t mj = __shfl_down(mask, j, 64);
                    run = run && lane + j < 64 && kj == key;
                    if (run) mask |= mj;
                }
                unsigned long long old = 0ull;
                if (key >= 0 && back == 0) {
                    unsigned long long inc = 0ull;
#pragma unroll
                    for (int q = 0; q < 8; q++)
                        if ((mask >> q) & 1u) inc |= 1ull << (8 * q);
                    old = atomicAdd((unsigned long long *)(a.nown + ((int64_t)key << 3)), inc);
                }
                old = __shfl(old, lane - back, 64);
                if (k < ncov) {
                    const int slot = (int)((old >> (8 * byte)) & 0xffull);
                    if (slot < MAX_OWNERS)
                        a.slots[(int64_t)slot * N + n] = ((uint32_t)p << SLOT_COUNT_BITS) | (uint32_t)count;
                    else
                        atomicOr(a.flags, FLAG_SLOT_OVERFLOW);
                    if (base + k < cap) list[base + k] = list_entry(count, kx, ky, kz);
                }
            }
            base += ncov;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (base > cap) atomicOr(a.flags, FLAG_SLOT_OVERFLOW);
        a.P.list_len[p] = base < cap ? base : cap;
    }
}

// LDS written by some lanes of a wavefront and read by others, in a kernel
// of one wavefront per workgroup: order the accesses within the wavefront.
__device__ __forceinline__ void lane_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Footprints of 64 / LPP particles per wavefront (one wavefront per
// workgroup, LPP lanes per particle): the phases of foot_one for each
// particle in its own lanes and LDS buffers, prefix sums over the particle's
// lanes, and runs of owner-count words kept inside a particle's lanes (two
// particles may cover one node).  Each particle's list, owner claims and
// counts are those foot_one gives.
template <int D, int S, int LPP>
__global__ __launch_bounds__(64) void k_foot_sub(FootArgs a) {
    constexpr int G = 64 / LPP, CHUNK = D == 3 ? 1024 : 512;
    __shared__ uint16_t s_cnt[G][CHUNK];
    __shared__ uint16_t s_todo[G][CHUNK];
    __shared__ int s_ntodo[G];
    const int lane = (int)threadIdx.x, grp = lane / LPP, sub = lane % LPP;
    const int P = a.P.np;
    const int p = (int)blockIdx.x * G + grp;
    const bool live = p < P;
    const int q = live ? p : 0;  // the lanes of a missing disc run every loop empty
    int lo[3], hi[3];
    bbox(a.P, q, D, lo, hi);
    if (live && sub == 0)
        for (int d = 0; d < 3; d++) {
            a.P.bb[d * P + p] = lo[d];
            a.P.bb[(3 + d) * P + p] = hi[d];
        }
    bool placed = live;
    for (int d = 0; d < D; d++) {
        const double c = a.P.x[d * P + q];
        const double L = d == 0 ? a.g.Lx : (d == 1 ? a.g.Ly : a.g.Lz);
        placed = placed && ((d == 1 && a.g.wall_y) ? (c > -L && c < 2.0 * L) : (c >= 0.0 && c < L));
    }
    if (live && !placed && sub == 0) atomicOr(a.flags, FLAG_NONFINITE);
    const int ext0 = hi[0] - lo[0] + 1, ext1 = hi[1] - lo[1] + 1;
    const int ext2 = D == 3 ? hi[2] - lo[2] + 1 : 1;
    const int items = placed ? ext0 * ext1 * ext2 : 0;
    const double R2 = a.P.R[q] * a.P.R[q];
    const double xp0 = a.P.x[q], xp1 = a.P.x[P + q], xp2 = D == 3 ? a.P.x[2 * P + q] : 0.0;
    const int64_t N = a.g.N;
    const int cap = a.P.list_cap;
    uint32_t *list = a.P.list + (int64_t)q * cap;
    const float inv0 = 1.0f / (float)ext0, inv1 = 1.0f / (float)ext1;
    auto node_of = [&](int item, int &kx, int &ky, int &kz, int &ix, int &iy, int &iz) {
        const int rest = div_small(item, ext0, inv0);
        kx = item - rest * ext0;
        kz = D == 3 ? div_small(rest, ext1, inv1) : 0;
        ky = rest - kz * ext1;
        iy = wrap1(a.g, 1, lo[1] + ky);
        ix = wrap1(a.g, 0, lo[0] + kx);
        iz = D == 3 ? wrap1(a.g, 2, lo[2] + kz) : 0;
    };
    int base = 0;
    for (int c0 = 0; __any(c0 < items); c0 += CHUNK) {
        const int nc = items - c0 < 0 ? 0 : (items - c0 < CHUNK ? items - c0 : CHUNK);
        if (sub == 0) s_ntodo[grp] = 0;
        lane_sync();
        // (A) classify
#pragma unroll 1
        for (int i = sub; i < nc; i += LPP) {
            int kx, ky, kz, ix, iy, iz;
            node_of(c0 + i, kx, ky, kz, ix, iy, iz);
            int cls = 0;
            if (iy >= 0)
                cls = classify<D, S>(ndisp(a.g, 0, ix, xp0), ndisp(a.g, 1, iy, xp1),
                                     D == 3 ? ndisp(a.g, 2, iz, xp2) : 0.0, R2);
            if (cls < 0) s_todo[grp][atomicAdd(&s_ntodo[grp], 1)] = (uint16_t)i;
            else s_cnt[grp][i] = (uint16_t)cls;
        }
        lane_sync();
        // (B) exact per-sample counts of the undecided nodes
        const int ntodo = s_ntodo[grp];
#pragma unroll 1
        for (int j = sub; j < ntodo; j += LPP) {
            const int i = s_todo[grp][j];
            int kx, ky, kz, ix, iy, iz;
            node_of(c0 + i, kx, ky, kz, ix, iy, iz);
            s_cnt[grp][i] = (uint16_t)sample_count<D, S>(ndisp(a.g, 0, ix, xp0), ndisp(a.g, 1, iy, xp1),
                                                         D == 3 ? ndisp(a.g, 2, iz, xp2) : 0.0, R2);
        }
        lane_sync();
        // (C1) covered nodes in node order into s_todo: each lane takes
        // ceil(nc / LPP) consecutive nodes, a prefix sum over the disc's lanes
        const int per = (nc + LPP - 1) / LPP;
        const int j0 = min(sub * per, nc), j1 = min(j0 + per, nc);
        int m = 0;
        for (int j = j0; j < j1; j++) m += s_cnt[grp][j] > 0 ? 1 : 0;
        int incl = m;
#pragma unroll
        for (int d = 1; d < LPP; d <<= 1) {
            const int y = __shfl_up(incl, d, LPP);
            if (sub >= d) incl += y;
        }
        const int ncov = __shfl(incl, LPP - 1, LPP);
        int at = incl - m;
        for (int j = j0; j < j1; j++)
            if (s_cnt[grp][j] > 0) s_todo[grp][at++] = (uint16_t)j;
        lane_sync();
        // (C2) owner slots and list entries, as in foot_one, with each run of
        // lanes that share an owner-count word kept inside one disc's lanes
#pragma unroll 1
        for (int k0 = 0; __any(k0 < ncov); k0 += LPP) {
            const int k = k0 + sub;
            int count = 0, kx = 0, ky = 0, kz = 0;
            int64_t n = 0;
            long long key = -1;
            if (k < ncov) {
                const int i = s_todo[grp][k];
                count = s_cnt[grp][i];
                int ix, iy, iz;
                node_of(c0 + i, kx, ky, kz, ix, iy, iz);
                n = (int64_t)ix + (int64_t)a.g.nx * ((int64_t)iy + (int64_t)a.g.ny * iz);
                key = (long long)(n >> 3);
            }
            const int byte = (int)(n & 7);
            uint32_t mask = key >= 0 ? 1u << byte : 0u;
            int back = 0;
            bool run = true;
#pragma unroll
            for (int j = 1; j < 8; j++) {
                const long long kj = __shfl_up(key, j, 64);
                run = run && sub >= j && kj == key;
                back += run ? 1 : 0;
            }
            run = true;
#pragma unroll
            for (int j = 1; j < 8; j++) {
                const long long kj = __shfl_down(key, j, 64);
                const uint32_t mj = __shfl_down(mask, j, 64);
                run = run && sub + j < LPP && kj == key;
                if (run) mask |= mj;
            }
            unsigned long long old = 0ull;
            if (key >= 0 && back == 0) {
                unsigned long long inc = 0ull;
#pragma unroll
                for (int b = 0; b < 8; b++)
                    if ((mask >> b) & 1u) inc |= 1ull << (8 * b);
                old = atomicAdd((unsigned long long *)(a.nown + ((int64_t)key << 3)), inc);
            }
            old = __shfl(old, lane - back, 64);
            if (k < ncov) {
                const int slot = (int)((old >> (8 * byte)) & 0xffull);
                if (slot < MAX_OWNERS)
                    a.slots[(int64_t)slot * N + n] = ((uint32_t)p << SLOT_COUNT_BITS) | (uint32_t)count;
                else
                    atomicOr(a.flags, FLAG_SLOT_OVERFLOW);
                if (base + k < cap) list[base + k] = list_entry(count, kx, ky, kz);
            }
        }
        base += ncov;
        lane_sync();
    }
    if (live && sub == 0) {
        if (base > cap) atomicOr(a.flags, FLAG_SLOT_OVERFLOW);
        a.P.list_len[p] = base < cap ? base : cap;
    }
}

// Footprints of every particle (one workgroup each), or of the particles of
// group G.g (workgroups walk the group's list).
template <int D, int S, int NT, bool TAB>
__global__ __launch_bounds__(NT) void k_foot_paint(FootArgs a) {
    if (a.G.g < 0) {
        foot_one<D, S, NT, TAB>(a, (int)blockIdx.x);
        return;
    }
    const int n = a.G.count[a.G.g];
    const int *lst = a.G.list + (int64_t)a.G.g * a.G.stride;
    for (int i = (int)blockIdx.x; i < n; i += (int)gridDim.x) {
        foot_one<D, S, NT, TAB>(a, lst[i]);
        __syncthreads();  // the shared buffers are reused by the next particle
    }
}

__device__ __forceinline__ double wrap_pos(double x, double L) {
    if (x < 0.0) {
        x = x + L;
        if (x >= L) x = x - L;
    } else if (x >= L) {
        x = x - L;
    }
    return x;
}

// ------------------------------------------------- hydrodynamic force, Eq. 3
struct Acc {
    double s, c;
};

__device__ __forceinline__ void acc_add(Acc &A, double p) {
    const double x = A.s + p;
    const double bb = x - A.s;
    const double e = (A.s - (x - bb)) + (p - bb);
    A.s = x;
    A.c = A.c + e;
}

__device__ __forceinline__ void acc_merge(Acc &A, const Acc &B) {
    const double x = A.s + B.s;
    const double bb = x - A.s;
    const double e = (A.s - (x - bb)) + (B.s - bb);
    A.s = x;
    A.c = (A.c + B.c) + e;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
    return __shfl_xor(v, m, 64);
}

// LPP lanes of a wavefront per particle over its footprint list: each entry
// gives the node and the particle's sample count there; q_n and the node's
// total count come from the lattice kernel.  With `integrate` set, the
// group's first lane then advances the particle (the contact forces of the
// step are complete).  s_pn q_n and r_pn x (s_pn q_n) go into TwoSum
// accumulators, which the group's lanes merge with butterfly shuffles.
// F_p = -sum, T_p = -sum.  `sub` is the lane's index in its group (groups are
// aligned runs of LPP lanes); `live` is false for the groups past the last
// particle, which take part in the shuffles only.
template <int D, bool R32, int LPP>
__device__ __forceinline__ void force_lanes(const ForceArgs &a, int p, int sub, bool live) {
    static_assert(LPP >= 16 && LPP <= 64 && (LPP & (LPP - 1)) == 0, "lanes per particle");
    const int lane = threadIdx.x & 63;
    const int gbase = lane - sub;
    const int P = a.P.np;
    const int q = live ? p : 0;
    const int len = live ? a.P.list_len[q] : 0;
    const int cap = a.P.list_cap;
    const int lo0 = a.P.bb[q], lo1 = a.P.bb[P + q], lo2 = a.P.bb[2 * P + q];
    const uint32_t *list = a.P.list + (int64_t)q * cap;
    const double xp0 = a.P.x[q], xp1 = a.P.x[P + q], xp2 = D == 3 ? a.P.x[2 * P + q] : 0.0;
    // the integration inputs, one per lane of the group (v, omega, F^c, m, I,
    // fixed), loaded beside the sums and gathered by the first lane at the end
    double pre = 0.0;
    if (live && a.integrate && sub < 12) {
        if (sub < 3) pre = a.P.v[sub * P + p];
        else if (sub < 6) pre = a.P.w[(sub - 3) * P + p];
        else if (sub < 9) pre = a.P.Fc[(sub - 6) * P + p];
        else if (sub == 9) pre = a.P.m[p];
        else if (sub == 10) pre = a.P.I[p];
        else pre = a.P.fixed[p] ? 1.0 : 0.0;
    }
    Acc F[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    Acc T[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    // UN entries per lane per round: all q loads of a round are issued
    // before the first accumulation, and the list entries of the next round
    // are loaded while they are in flight (the first round's beside the list
    // length: loads below the capacity stay inside the particle's list).
    constexpr int UN = 2;
    const int stride = UN * LPP;
    uint32_t vn[UN];
#pragma unroll
    for (int u = 0; u < UN; u++) {
        const int e = u * LPP + sub;
        vn[u] = e < cap ? list[e] : 0u;
    }
    // lattice coordinates of an entry, formed again where needed (fewer
    // registers live across the loads)
    auto coords = [&](uint32_t e, int &ix, int &iy, int &iz) {
        ix = wrap1(a.g, 0, lo0 + (int)((e >> 10) & 127u));
        iy = wrap1(a.g, 1, lo1 + (int)((e >> 17) & 127u));
        iz = D == 3 ? wrap1(a.g, 2, lo2 + (int)((e >> 24) & 127u)) : 0;
    };
    for (int e0 = 0; e0 < len; e0 += stride) {
        uint32_t v[UN];
#pragma unroll
        for (int u = 0; u < UN; u++) {
            const int e = e0 + u * LPP + sub;
            v[u] = e < len ? vn[u] : 0u;
        }
        double q0[UN], q1[UN], q2[UN];
        int tot[UN];
#pragma unroll
        for (int u = 0; u < UN; u++) {
            q0[u] = q1[u] = q2[u] = 0.0;
            tot[u] = 1;
            if (v[u] != 0u) {
                int ix, iy, iz;
                coords(v[u], ix, iy, iz);
                const int64_t n = (int64_t)ix + (int64_t)a.g.nx * ((int64_t)iy + (int64_t)a.g.ny * iz);
                double qq[3];
                read_qrec(a.qr, R32, n, qq, tot[u]);
                q0[u] = qq[0];
                q1[u] = qq[1];
                q2[u] = qq[2];
            }
        }
#pragma unroll
        for (int u = 0; u < UN; u++) {
            const int e = e0 + stride + u * LPP + sub;
            vn[u] = e < len ? list[e] : 0u;
        }
#pragma unroll
        for (int u = 0; u < UN; u++) {
            if (v[u] == 0u) continue;
            const int cnt = (int)(v[u] & LIST_COUNT_MASK);
            int ix, iy, iz;
            coords(v[u], ix, iy, iz);
            // the particle's share of the node: exactly 1 where it is the
            // only owner (cnt = tot), the division only where a wavefront
            // holds a shared node
            double sh = 1.0;
            if (__any(cnt != tot[u]) && cnt != tot[u]) sh = (double)cnt / (double)tot[u];
            const double t0 = sh * q0[u], t1 = sh * q1[u];
            const double rx = ndisp(a.g, 0, ix, xp0);
            const double ry = ndisp(a.g, 1, iy, xp1);
            acc_add(F[0], t0);
            acc_add(F[1], t1);
            if (D == 3) {
                const double t2 = sh * q2[u];
                const double rz = ndisp(a.g, 2, iz, xp2);
                acc_add(F[2], t2);
                acc_add(T[0], ry * t2 - rz * t1);
                acc_add(T[1], rz * t0 - rx * t2);
                acc_add(T[2], rx * t1 - ry * t0);
            } else {
                acc_add(T[2], rx * t1 - ry * t0);
            }
        }
    }
    // butterfly over the group's lanes: the components that can be nonzero
    // (2D: F_x, F_y and T_z; the others stay zero and are not used)
#pragma unroll
    for (int m = LPP / 2; m >= 1; m >>= 1) {
#pragma unroll
        for (int d = 0; d < 3; d++) {
            Acc o;
            if (d < D) {
                o.s = shfl_xor_d(F[d].s, m);
                o.c = shfl_xor_d(F[d].c, m);
                acc_merge(F[d], o);
            }
            if (D == 3 || d == 2) {
                o.s = shfl_xor_d(T[d].s, m);
                o.c = shfl_xor_d(T[d].c, m);
                acc_merge(T[d], o);
            }
        }
    }
    double pv[3], pw[3], pfc[3];
    for (int d = 0; d < 3; d++) {
        pv[d] = __shfl(pre, gbase + d, 64);
        pw[d] = __shfl(pre, gbase + 3 + d, 64);
        pfc[d] = __shfl(pre, gbase + 6 + d, 64);
    }
    const double pm = __shfl(pre, gbase + 9, 64), pI = __shfl(pre, gbase + 10, 64);
    const double pfix = __shfl(pre, gbase + 11, 64);
    if (live && sub == 0) {
        double Fv[3], Tv[3];
        for (int d = 0; d < 3; d++) {
            double fv = -(F[d].s + F[d].c);
            double tv = -(T[d].s + T[d].c);
            if (D == 2 && d == 2) fv = 0.0;
            if (D == 2 && d < 2) tv = 0.0;
            a.P.Fh[d * P + p] = fv;
            a.P.Th[d * P + p] = tv;
            Fv[d] = fv;
            Tv[d] = tv;
        }
        // Symplectic Euler with dt = 1 for this particle (every reader of its
        // position in this kernel has read it): v += (F^h + F^c + m a)/m,
        // omega += T^h/I, x += v (new), periodic wrap.
        if (a.integrate && pfix == 0.0) {
            const double xo[3] = {xp0, xp1, xp2};
            for (int d = 0; d < D; d++) {
                const double ftot = Fv[d] + pfc[d] + pm * a.ap[d];
                const double vn = pv[d] + ftot / pm;
                a.P.v[d * P + p] = vn;
                double xn = xo[d] + vn;
                if (!(d == 1 && a.g.wall_y)) xn = wrap_pos(xn, d == 0 ? a.g.Lx : (d == 1 ? a.g.Ly : a.g.Lz));
                a.P.x[d * P + p] = xn;
            }
            if (D == 3) {
                for (int d = 0; d < 3; d++) a.P.w[d * P + p] = pw[d] + Tv[d] / pI;
            } else {
                a.P.w[2 * P + p] = pw[2] + Tv[2] / pI;
            }
            // the slab pipeline assumes at most one node of motion in y per step
            if (a.G.K > 1 && !(fabs(a.P.v[P + p]) <= 1.0)) atomicOr(a.flags, FLAG_FAST);
        }
        if (a.integrate && a.G.K > 1) {
            // file the particle in its group of the next step
            const int gn = slab_group(a.G, a.P.x[P + p], a.P.R[p]);
            const int slot = atomicAdd(&a.G.ncount[gn], 1);
            a.G.nlist[(int64_t)gn * a.G.stride + slot] = p;
        }
    }
}

// Force, torque and integration of every particle (64 / LPP particles per
// wavefront, one wavefront per workgroup), or of the particles of group G.g
// (one particle per wavefront; workgroups walk the group's list).
template <int D, bool R32, int LPP>
__global__ __launch_bounds__(64) void k_force(ForceArgs a) {
    const int lane = (int)threadIdx.x;
    if (a.G.g < 0) {
        const int p = (int)blockIdx.x * (64 / LPP) + lane / LPP;
        force_lanes<D, R32, LPP>(a, p, lane % LPP, p < a.P.np);
        return;
    }
    const int n = a.G.count[a.G.g];
    const int *lst = a.G.list + (int64_t)a.G.g * a.G.stride;
    for (int i = (int)blockIdx.x; i < n; i += (int)gridDim.x) force_lanes<D, R32, 64>(a, lst[i], lane, true);
}

// Files every particle in its group of the current positions.
__global__ void k_assign_groups(ForceArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = a.P.np;
    if (p >= P) return;
    const int g = slab_group(a.G, a.P.x[P + p], a.P.R[p]);
    const int slot = atomicAdd(&a.G.ncount[g], 1);
    a.G.nlist[(int64_t)g * a.G.stride + slot] = p;
}

// q_n of the last step at the nodes of the current footprint lists (the nodes
// the lattice kernel covered); `out` [D][N] is zero elsewhere beforehand.
template <int D>
__global__ void k_list_q(ForceArgs a, double *out) {
    const int p = blockIdx.x;
    const int P = a.P.np;
    const int len = a.P.list_len[p];
    const int lo0 = a.P.bb[p], lo1 = a.P.bb[P + p], lo2 = a.P.bb[2 * P + p];
    const uint32_t *list = a.P.list + (int64_t)p * a.P.list_cap;
    const int64_t N = a.g.N;
    for (int e = threadIdx.x; e < len; e += blockDim.x) {
        const uint32_t v = list[e];
        const int ix = wrap1(a.g, 0, lo0 + (int)((v >> 10) & 127u));
        const int iy = wrap1(a.g, 1, lo1 + (int)((v >> 17) & 127u));
        const int iz = D == 3 ? wrap1(a.g, 2, lo2 + (int)((v >> 24) & 127u)) : 0;
        const int64_t n = (int64_t)ix + (int64_t)a.g.nx * ((int64_t)iy + (int64_t)a.g.ny * iz);
        double qq[3];
        int tot;
        read_qrec(a.qr, a.rec32 != 0, n, qq, tot);
        for (int d = 0; d < D; d++) out[d * N + n] = qq[d];
    }
}

// ------------------------------------------------------------- cell list
__device__ __forceinline__ int cell_coord(const CellArgs &a, int axis, double x) {
    const int nc = axis == 0 ? a.ncx : (axis == 1 ? a.ncy : a.ncz);
    const double L = axis == 0 ? a.g.Lx : (axis == 1 ? a.g.Ly : a.g.Lz);
    double t = x;
    if (axis == 1 && a.g.wall_y) t = x + 0.5;
    int c = (int)floor(t * (double)nc / L);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_cells(CellArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = a.P.np;
    if (p >= P) return;
    const int cx = cell_coord(a, 0, a.P.x[p]);
    const int cy = cell_coord(a, 1, a.P.x[P + p]);
    const int cz = a.D == 3 ? cell_coord(a, 2, a.P.x[2 * P + p]) : 0;
    const int c = cx + a.ncx * (cy + a.ncy * cz);
    const int slot = atomicAdd(&a.cell_count[c], 1);
    if (slot < CELL_CAP) a.cell_ids[c * CELL_CAP + slot] = p;
    else atomicOr(a.flags, FLAG_CELL_OVERFLOW);
}

// Neighbour cell offsets along one axis: {-1,0,1} wrapped (periodic, >= 3
// cells), {0,1} (2 cells), {0} (1 cell), or {-1,0,1} clipped at walls.
__device__ __forceinline__ int axis_cells(int c, int nc, bool periodic, int out[3]) {
    if (periodic) {
        if (nc >= 3) { out[0] = c == 0 ? nc - 1 : c - 1; out[1] = c; out[2] = c == nc - 1 ? 0 : c + 1; return 3; }
        if (nc == 2) { out[0] = 0; out[1] = 1; return 2; }
        out[0] = 0;
        return 1;
    }
    int k = 0;
    for (int d = -1; d <= 1; d++)
        if (c + d >= 0 && c + d < nc) out[k++] = c + d;
    return k;
}

// Contact test and force of Eqs. 4-5 for the pair (i, j) with the overlap
// delta = R_i + R_j - |r_i - r_j| (minimum image).  Returns false when the
// particles do not touch.
__device__ __forceinline__ bool pair_force(const CellArgs &a, int i, int j, double F[3]) {
    const int P = a.P.np, D = a.D;
    double d[3] = {0.0, 0.0, 0.0};
    for (int ax = 0; ax < D; ax++) {
        double dd = a.P.x[ax * P + i] - a.P.x[ax * P + j];
        if (!(ax == 1 && a.g.wall_y)) dd = pdisp(dd, ax == 0 ? a.g.Lx : (ax == 1 ? a.g.Ly : a.g.Lz));
        d[ax] = dd;
    }
    double d2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) d2 = d2 + d[2] * d[2];
    const double dist = sqrt(d2);
    const double delta = (a.P.R[i] + a.P.R[j]) - dist;
    if (!(delta > 0.0)) return false;
    if (F) {
        double nrm[3] = {0.0, 0.0, 0.0};
        for (int ax = 0; ax < D; ax++) nrm[ax] = d[ax] / dist;
        double vn = (a.P.v[i] - a.P.v[j]) * nrm[0] + (a.P.v[P + i] - a.P.v[P + j]) * nrm[1];
        if (D == 3) vn = vn + (a.P.v[2 * P + i] - a.P.v[2 * P + j]) * nrm[2];
        const double meff = a.P.m[i] * a.P.m[j] / (a.P.m[i] + a.P.m[j]);
        const double eta = a.ce * sqrt(meff * a.kn);
        const double fmag = a.kn * delta - eta * vn;
        for (int ax = 0; ax < D; ax++) F[ax] = F[ax] + fmag * nrm[ax];
    }
    return true;
}

// Wall contacts of particle i (Eqs. 4-5 against a wall at rest, m_eff = m_i),
// added to F after the pair forces.
__device__ __forceinline__ void wall_force(const CellArgs &a, int i, double F[3]) {
    if (!a.g.wall_y) return;
    const int P = a.P.np;
    const double eta = a.ce * sqrt(a.P.m[i] * a.kn);
    const double y = a.P.x[P + i];
    const double vy = a.P.v[P + i];
    const double dl = a.P.R[i] - (y + 0.5);
    if (dl > 0.0) {
        const double fmag = a.kn * dl - eta * vy;
        F[1] = F[1] + fmag;
    }
    const double du = a.P.R[i] - ((a.g.Ly - 0.5) - y);
    if (du > 0.0) {
        const double fmag = a.kn * du - eta * (-vy);
        F[1] = F[1] - fmag;
    }
}

// One wavefront per particle: each lane scans one neighbour cell, touching
// neighbours are gathered in LDS, sorted by id, and the pair forces are added
// in ascending id (then the walls) by the first lane.
__global__ __launch_bounds__(256) void k_dem(CellArgs a) {
    __shared__ int list[4][MAX_CONTACTS];
    __shared__ int nlist[4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 4 + wave;
    const int P = a.P.np;
    const int D = a.D;
    if (lane == 0) nlist[wave] = 0;
    __syncthreads();
    if (i < P) {
        const int c0 = cell_coord(a, 0, a.P.x[i]);
        const int c1 = cell_coord(a, 1, a.P.x[P + i]);
        const int c2 = D == 3 ? cell_coord(a, 2, a.P.x[2 * P + i]) : 0;
        int ox[3], oy[3], oz[3];
        const int nxc = axis_cells(c0, a.ncx, true, ox);
        const int nyc = axis_cells(c1, a.ncy, !a.g.wall_y, oy);
        int nzc = 1;
        oz[0] = 0;
        if (D == 3) nzc = axis_cells(c2, a.ncz, true, oz);
        if (lane < nxc * nyc * nzc) {
            const int kx = lane % nxc, ky = (lane / nxc) % nyc, kz = lane / (nxc * nyc);
            const int c = ox[kx] + a.ncx * (oy[ky] + a.ncy * oz[kz]);
            const int cnt = min(a.cell_count[c], CELL_CAP);
            for (int s = 0; s < cnt; s++) {
                const int j = a.cell_ids[c * CELL_CAP + s];
                if (j == i) continue;
                if (!pair_force(a, i, j, nullptr)) continue;
                const int slot = atomicAdd(&nlist[wave], 1);
                if (slot < MAX_CONTACTS) list[wave][slot] = j;
                else atomicOr(a.flags, FLAG_CONTACT_OVERFLOW);
            }
        }
    }
    __syncthreads();
    if (i < P && lane == 0) {
        int *l = list[wave];
        const int nl = min(nlist[wave], MAX_CONTACTS);
        for (int s = 1; s < nl; s++) {
            const int v = l[s];
            int t = s - 1;
            while (t >= 0 && l[t] > v) {
                l[t + 1] = l[t];
                t--;
            }
            l[t + 1] = v;
        }
        double F[3] = {0.0, 0.0, 0.0};
        for (int s = 0; s < nl; s++) pair_force(a, i, l[s], F);
        wall_force(a, i, F);
        for (int d = 0; d < 3; d++) a.P.Fc[d * P + i] = F[d];
    }
}

// One thread per particle, for many particles (k_dem keeps a wavefront busy
// with 9 or 27 neighbour cells, most of its lanes idle in 2D): the thread
// walks the neighbour cells itself and inserts each touching neighbour into
// its own id-sorted column of LDS, then adds the pair forces in ascending id
// and the walls, the sum order of k_dem, so both kernels give the same bits.
template <int NT>
__global__ __launch_bounds__(NT) void k_dem_thread(CellArgs a) {
    __shared__ int list[MAX_CONTACTS][NT];
    const int t = threadIdx.x;
    const int i = blockIdx.x * NT + t;
    const int P = a.P.np;
    const int D = a.D;
    if (i >= P) return;  // no barrier below
    const int c0 = cell_coord(a, 0, a.P.x[i]);
    const int c1 = cell_coord(a, 1, a.P.x[P + i]);
    const int c2 = D == 3 ? cell_coord(a, 2, a.P.x[2 * P + i]) : 0;
    int ox[3], oy[3], oz[3];
    const int nxc = axis_cells(c0, a.ncx, true, ox);
    const int nyc = axis_cells(c1, a.ncy, !a.g.wall_y, oy);
    int nzc = 1;
    oz[0] = 0;
    if (D == 3) nzc = axis_cells(c2, a.ncz, true, oz);
    int nl = 0;
    bool overflow = false;
    for (int kz = 0; kz < nzc; kz++)
        for (int ky = 0; ky < nyc; ky++)
            for (int kx = 0; kx < nxc; kx++) {
                const int c = ox[kx] + a.ncx * (oy[ky] + a.ncy * oz[kz]);
                const int cnt = min(a.cell_count[c], CELL_CAP);
                for (int s = 0; s < cnt; s++) {
                    const int j = a.cell_ids[c * CELL_CAP + s];
                    if (j == i) continue;
                    if (!pair_force(a, i, j, nullptr)) continue;
                    if (nl >= MAX_CONTACTS) {
                        overflow = true;
                        continue;
                    }
                    int q = nl;
                    while (q > 0 && list[q - 1][t] > j) {
                        list[q][t] = list[q - 1][t];
                        q--;
                    }
                    list[q][t] = j;
                    nl++;
                }
            }
    if (overflow) atomicOr(a.flags, FLAG_CONTACT_OVERFLOW);
    double F[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < nl; s++) pair_force(a, i, list[s][t], F);
    wall_force(a, i, F);
    for (int d = 0; d < 3; d++) a.P.Fc[d * P + i] = F[d];
}

// ------------------------------------------------------ neighbour-list mode
// The lists hold, in ascending id, every j with |r_i - r_j| < R_i + R_j + skin
// (minimum image) at the last build.  A pair missing from the lists was at
// least that far apart, so it can only touch after one of the two moved at
// least skin / 2; the guard rebuilds before any particle has moved 0.49 skin
// since the build, and after `every` steps in any case.  Contacts then sum the
// touching listed neighbours in ascending id, the order of k_dem, so both
// modes give the same bits.

// Guard: raises the rebuild flag when a particle moved 0.49 skin or more since
// the last build, or the lists are `every` steps old.
__global__ void k_nl_check(CellArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = a.P.np;
    if (p == 0 && a.nl_state[1] >= a.every) atomicOr(&a.nl_state[0], 1);
    if (p >= P) return;
    double d2 = 0.0;
    for (int ax = 0; ax < a.D; ax++) {
        double dd = a.P.x[ax * P + p] - a.xb[ax * P + p];
        if (!(ax == 1 && a.g.wall_y)) dd = pdisp(dd, ax == 0 ? a.g.Lx : (ax == 1 ? a.g.Ly : a.g.Lz));
        d2 = d2 + dd * dd;
    }
    const double lim = 0.49 * a.skin;
    if (!(d2 < lim * lim)) atomicOr(&a.nl_state[0], 1);
}

// Cell binning, on rebuild steps only (the counts are zero on entry).
__global__ void k_nl_cells(CellArgs a) {
    if (!a.nl_state[0]) return;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = a.P.np;
    if (p >= P) return;
    const int cx = cell_coord(a, 0, a.P.x[p]);
    const int cy = cell_coord(a, 1, a.P.x[P + p]);
    const int cz = a.D == 3 ? cell_coord(a, 2, a.P.x[2 * P + p]) : 0;
    const int c = cx + a.ncx * (cy + a.ncy * cz);
    const int slot = atomicAdd(&a.cell_count[c], 1);
    if (slot < CELL_CAP) a.cell_ids[c * CELL_CAP + slot] = p;
    else atomicOr(a.flags, FLAG_CELL_OVERFLOW);
}

// True when j lies within R_i + R_j + skin of i (minimum image).
__device__ __forceinline__ bool nl_candidate(const CellArgs &a, int i, int j) {
    const int P = a.P.np;
    double d2 = 0.0;
    for (int ax = 0; ax < a.D; ax++) {
        double dd = a.P.x[ax * P + i] - a.P.x[ax * P + j];
        if (!(ax == 1 && a.g.wall_y)) dd = pdisp(dd, ax == 0 ? a.g.Lx : (ax == 1 ? a.g.Ly : a.g.Lz));
        d2 = d2 + dd * dd;
    }
    const double lim = (a.P.R[i] + a.P.R[j]) + a.skin;
    return d2 < lim * lim;
}

// List build, on rebuild steps only: one wavefront per particle, each lane
// scans one neighbour cell (cell edge >= 2 R_max + skin), the candidates are
// gathered in LDS and sorted by id; the build positions are recorded.
__global__ __launch_bounds__(256) void k_nl_build(CellArgs a) {
    if (!a.nl_state[0]) return;
    __shared__ int list[4][NL_CAP];
    __shared__ int nlist[4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 4 + wave;
    const int P = a.P.np;
    const int D = a.D;
    if (lane == 0) nlist[wave] = 0;
    __syncthreads();
    if (i < P) {
        const int c0 = cell_coord(a, 0, a.P.x[i]);
        const int c1 = cell_coord(a, 1, a.P.x[P + i]);
        const int c2 = D == 3 ? cell_coord(a, 2, a.P.x[2 * P + i]) : 0;
        int ox[3], oy[3], oz[3];
        const int nxc = axis_cells(c0, a.ncx, true, ox);
        const int nyc = axis_cells(c1, a.ncy, !a.g.wall_y, oy);
        int nzc = 1;
        oz[0] = 0;
        if (D == 3) nzc = axis_cells(c2, a.ncz, true, oz);
        if (lane < nxc * nyc * nzc) {
            const int kx = lane % nxc, ky = (lane / nxc) % nyc, kz = lane / (nxc * nyc);
            const int c = ox[kx] + a.ncx * (oy[ky] + a.ncy * oz[kz]);
            const int cnt = min(a.cell_count[c], CELL_CAP);
            for (int s = 0; s < cnt; s++) {
                const int j = a.cell_ids[c * CELL_CAP + s];
                if (j == i || !nl_candidate(a, i, j)) continue;
                const int slot = atomicAdd(&nlist[wave], 1);
                if (slot < NL_CAP) list[wave][slot] = j;
                else atomicOr(a.flags, FLAG_CONTACT_OVERFLOW);
            }
        }
        if (lane < D) a.xb[lane * P + i] = a.P.x[lane * P + i];
    }
    __syncthreads();
    if (i < P && lane == 0) {
        int *l = list[wave];
        const int nl = min(nlist[wave], NL_CAP);
        for (int s = 1; s < nl; s++) {
            const int v = l[s];
            int t = s - 1;
            while (t >= 0 && l[t] > v) {
                l[t + 1] = l[t];
                t--;
            }
            l[t + 1] = v;
        }
        for (int s = 0; s < nl; s++) a.nl[(int64_t)i * NL_CAP + s] = l[s];
        a.nl_len[i] = nl;
    }
}

// Contacts from the lists (Eqs. 4-5): one thread per particle, the touching
// listed neighbours in ascending id, then the walls.
__global__ void k_dem_list(CellArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = a.P.np;
    if (i >= P) return;
    const int n = a.nl_len[i];
    int touching = 0;
    double F[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < n; s++) touching += pair_force(a, i, a.nl[(int64_t)i * NL_CAP + s], F) ? 1 : 0;
    if (touching > MAX_CONTACTS) atomicOr(a.flags, FLAG_CONTACT_OVERFLOW);
    wall_force(a, i, F);
    for (int d = 0; d < 3; d++) a.P.Fc[d * P + i] = F[d];
}

// After a rebuild: clear the cell counts for the next one.
__global__ void k_nl_clear(CellArgs a) {
    if (!a.nl_state[0]) return;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.ncell;
         c += (int64_t)gridDim.x * blockDim.x)
        a.cell_count[c] = 0;
}

// Ages the lists and lowers the rebuild flag (one thread, after every other
// kernel of the step's neighbour work has read the flag).
__global__ void k_nl_finish(CellArgs a) {
    if (a.nl_state[0]) {
        a.nl_state[0] = 0;
        a.nl_state[1] = 1;
        *a.nl_builds = *a.nl_builds + 1;
    } else {
        a.nl_state[1] = a.nl_state[1] + 1;
    }
}


// ---------------------------------------------------------------- launchers
static unsigned blocks_for(int n, int per) { return (unsigned)((n + per - 1) / per); }

// workgroups of a launch that walks one group's list
constexpr int GROUP_GRID = 4096;

template <int D, int NT, bool TAB>
static hipError_t paint_s(const FootArgs &a, hipStream_t s) {
    const dim3 g((unsigned)(a.G.g < 0 ? a.P.np : std::min(a.P.np, GROUP_GRID))), b((unsigned)NT);
    switch (a.S) {
        case 1: hipLaunchKernelGGL((k_foot_paint<D, 1, NT, TAB>), g, b, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_foot_paint<D, 2, NT, TAB>), g, b, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_foot_paint<D, 3, NT, TAB>), g, b, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_foot_paint<D, 4, NT, TAB>), g, b, 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_foot_paint<D, 5, NT, TAB>), g, b, 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_foot_paint<D, 6, NT, TAB>), g, b, 0, s, a); break;
        case 7: hipLaunchKernelGGL((k_foot_paint<D, 7, NT, TAB>), g, b, 0, s, a); break;
        default: hipLaunchKernelGGL((k_foot_paint<D, 8, NT, TAB>), g, b, 0, s, a); break;
    }
    return hipGetLastError();
}

// Threads per particle of the footprint kernel (compile-time knobs for
// measurement).  Measured on MI355X at 4^D samples: a disc of radius 5 runs
// fastest with one wavefront (1.3-1.4x faster than two; four are slower
// still), a sphere of radius 4 with two (one or four are slower).
#ifndef FOOT_NT2
#define FOOT_NT2 64
#endif
#ifndef FOOT_NT3
#define FOOT_NT3 128
#endif

// Discs of the sampling footprint on the plain step: 16 lanes per disc, four
// discs per wavefront (k_foot_sub, 78 registers, six wavefronts per SIMD).
// Measured on MI355X (same bits in every shape): 1 166 400 discs 1.96
// against 2.75 ms with a wavefront per disc (32 lanes: 1.72 ms, but the step
// was slower), C2 47.6 against 52.7 us.
#ifndef FOOT_LPP2
#define FOOT_LPP2 16
#endif
// Spheres: one wavefront per sphere in k_foot_sub (8 317 spheres: 81 against
// 83 us for foot_one's two wavefronts, 85 us for two spheres per wavefront);
// a value above 64 keeps foot_one.
#ifndef FOOT_LPP3
#define FOOT_LPP3 64
#endif

template <int D, int LPP>
static hipError_t paint_sub(const FootArgs &a, hipStream_t s) {
    const dim3 g(blocks_for(a.P.np, 64 / LPP)), b(64);
    switch (a.S) {
        case 1: hipLaunchKernelGGL((k_foot_sub<D, 1, LPP>), g, b, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_foot_sub<D, 2, LPP>), g, b, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_foot_sub<D, 3, LPP>), g, b, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_foot_sub<D, 4, LPP>), g, b, 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_foot_sub<D, 5, LPP>), g, b, 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_foot_sub<D, 6, LPP>), g, b, 0, s, a); break;
        case 7: hipLaunchKernelGGL((k_foot_sub<D, 7, LPP>), g, b, 0, s, a); break;
        default: hipLaunchKernelGGL((k_foot_sub<D, 8, LPP>), g, b, 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_foot_paint(const FootArgs &a, int D, hipStream_t s) {
    if (a.P.np == 0) return hipSuccess;
    // the table lookup is a kernel of its own, so the sampling kernel keeps
    // its registers
    if (a.tab) return D == 2 ? paint_s<2, FOOT_NT2, true>(a, s) : paint_s<3, FOOT_NT3, true>(a, s);
    if (D == 2 && FOOT_LPP2 <= 64 && a.G.g < 0) return paint_sub<2, FOOT_LPP2 <= 64 ? FOOT_LPP2 : 64>(a, s);
    if (D == 3 && FOOT_LPP3 <= 64 && a.G.g < 0) return paint_sub<3, FOOT_LPP3 <= 64 ? FOOT_LPP3 : 64>(a, s);
    return D == 2 ? paint_s<2, FOOT_NT2, false>(a, s) : paint_s<3, FOOT_NT3, false>(a, s);
}

// Lanes per particle of the force kernel on the plain step (compile-time
// knobs for measurement); the slab pipeline's groups take one wavefront per
// particle.  Measured on MI355X (same bits in every shape): a disc's ~100
// list entries take 16 lanes, four discs per wavefront (1 166 400 discs:
// 1.18 against 1.62 ms with a wavefront each, C2: 30 against 37 us); a
// sphere's ~270 entries keep a whole wavefront (16 or 32 lanes: within 3 %).
#ifndef FORCE_LPP2
#define FORCE_LPP2 16
#endif
#ifndef FORCE_LPP3
#define FORCE_LPP3 64
#endif

hipError_t launch_force(const ForceArgs &a, hipStream_t s) {
    if (a.P.np == 0) return hipSuccess;
    const dim3 b(64);
    if (a.G.g >= 0) {
        const dim3 g((unsigned)std::min(a.P.np, GROUP_GRID));
        if (a.D == 2) {
            if (a.rec32) hipLaunchKernelGGL((k_force<2, true, 64>), g, b, 0, s, a);
            else hipLaunchKernelGGL((k_force<2, false, 64>), g, b, 0, s, a);
        } else {
            if (a.rec32) hipLaunchKernelGGL((k_force<3, true, 64>), g, b, 0, s, a);
            else hipLaunchKernelGGL((k_force<3, false, 64>), g, b, 0, s, a);
        }
        return hipGetLastError();
    }
    if (a.D == 2) {
        const dim3 g(blocks_for(a.P.np, 64 / FORCE_LPP2));
        if (a.rec32) hipLaunchKernelGGL((k_force<2, true, FORCE_LPP2>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_force<2, false, FORCE_LPP2>), g, b, 0, s, a);
    } else {
        const dim3 g(blocks_for(a.P.np, 64 / FORCE_LPP3));
        if (a.rec32) hipLaunchKernelGGL((k_force<3, true, FORCE_LPP3>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_force<3, false, FORCE_LPP3>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_assign_groups(const ForceArgs &a, hipStream_t s) {
    if (a.P.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_assign_groups, dim3(blocks_for(a.P.np, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_list_q(const ForceArgs &a, double *out, hipStream_t s) {
    hipError_t e = launch_fill_u64((uint64_t *)out, 0ull, (int64_t)a.D * a.g.N, s);
    if (e != hipSuccess || a.P.np == 0) return e;
    if (a.D == 2) hipLaunchKernelGGL(k_list_q<2>, dim3((unsigned)a.P.np), dim3(128), 0, s, a, out);
    else hipLaunchKernelGGL(k_list_q<3>, dim3((unsigned)a.P.np), dim3(256), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_cells(const CellArgs &a, hipStream_t s) {
    if (a.P.np == 0) return hipSuccess;
    hipError_t e = launch_fill_u32((uint32_t *)a.cell_count, 0u, (int64_t)a.ncx * a.ncy * a.ncz, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cells, dim3(blocks_for(a.P.np, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Contacts: a thread per particle for 2D runs of at least DEM_THREAD_MIN
// discs, else a wavefront per particle.  Measured on MI355X: 21 361 discs
// 25 against 65 us, 1 166 400 discs 0.54 against 4.4 ms; 8 317 spheres 168
// against 26 us (too few wavefronts to hide a thread's walk over 27 cells).
#ifndef DEM_THREAD_MIN
#define DEM_THREAD_MIN 16384
#endif

hipError_t launch_dem(const CellArgs &a, hipStream_t s) {
    if (a.P.np == 0) return hipSuccess;
    if (a.D == 2 && a.P.np >= DEM_THREAD_MIN)
        hipLaunchKernelGGL(k_dem_thread<128>, dim3(blocks_for(a.P.np, 128)), dim3(128), 0, s, a);
    else
        hipLaunchKernelGGL(k_dem, dim3(blocks_for(a.P.np, 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_nl_rebuild(const CellArgs &a, hipStream_t s) {
    if (a.P.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_nl_check, dim3(blocks_for(a.P.np, 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_nl_cells, dim3(blocks_for(a.P.np, 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_nl_build, dim3(blocks_for(a.P.np, 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_nl_contacts(const CellArgs &a, hipStream_t s) {
    if (a.P.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dem_list, dim3(blocks_for(a.P.np, 256)), dim3(256), 0, s, a);
    const unsigned cb = (unsigned)std::min<int64_t>((a.ncell + 255) / 256, 4096);
    hipLaunchKernelGGL(k_nl_clear, dim3(cb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_nl_finish, dim3(1), dim3(1), 0, s, a);
    return hipGetLastError();
}


}  // namespace lbimb
