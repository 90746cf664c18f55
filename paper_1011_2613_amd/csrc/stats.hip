// stats.hip -- suspension-wide diagnostics behind lbm_get_stats: fluid mass
// and momentum over the lattice, the fluid-phase (1 - eps)-weighted share of
// them, particle momentum and the mean hydrodynamic force.  The paper follows
// its suspensions through the area-averaged slip velocity between the phases
// and the mean drag ("Simulation results", Figs. 5 and 7); these sums give
// both.
//
// Every reduction has a fixed shape (a fixed number of workgroups, a fixed
// per-thread order, a fixed tree), so the result does not depend on the GPU
// or on timing.  Partial sums live in the context's workspace.
#include "internal.h"
#include "lb_shared.h"

namespace lbimb {

namespace {

// Pre-collision population i of node (x, y, z) in binary64: the value the
// previous step's pull streaming leaves for it, A_i(x - c_i), or A_opp(i)(x)
// when x - c_i lies beyond a wall; shifted storage decoded to w_i + g_i.
template <class L, int ST>
__device__ __forceinline__ double pre_pop(const void *A, const Geom &g, int i, int x, int y, int z) {
    using T = typename Store<ST>::T;
    int sx = x - L::cx[i], sy = y - L::cy[i], sz = z - L::cz[i];
    int j = i;
    if (g.wall_y && (sy < 0 || sy >= g.ny)) {
        sx = x; sy = y; sz = z; j = L::opp[i];
    } else {
        sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
        sy = sy < 0 ? sy + g.ny : (sy >= g.ny ? sy - g.ny : sy);
        sz = sz < 0 ? sz + g.nz : (sz >= g.nz ? sz - g.nz : sz);
    }
    const uint64_t e = (((uint64_t)sz * (uint64_t)g.ny + (uint64_t)sy) * (uint64_t)L::Q + (uint64_t)j) *
                           (uint64_t)g.nx + (uint64_t)sx;
    const T v = ((const T *)A)[e];
    if (ST == 0) return (double)v;
    const float wf = (float)L::w[L::wc[j]];
    const float gv = ST == 1 ? (float)v : wf * (float)v;
    return L::w[L::wc[j]] + (double)gv;
}

// rho and j = sum_i c_i f_i of one node, directions in index order.
template <class L, int ST>
__device__ __forceinline__ void node_moments(const void *A, const Geom &g, int x, int y, int z,
                                             double &rho, double j[3]) {
    rho = 0.0;
    j[0] = j[1] = j[2] = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const double f = pre_pop<L, ST>(A, g, i, x, y, z);
        rho = rho + f;
        if (L::cx[i]) j[0] = L::cx[i] > 0 ? j[0] + f : j[0] - f;
        if (L::cy[i]) j[1] = L::cy[i] > 0 ? j[1] + f : j[1] - f;
        if (L::cz[i]) j[2] = L::cz[i] > 0 ? j[2] + f : j[2] - f;
    }
}

// Fixed-order tree sum of K values per thread over a 256-thread workgroup;
// thread 0 ends up with the totals in s[0][..].
template <int K>
__device__ __forceinline__ void block_sum(double (*s)[K], const double (&v)[K]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; k++) s[t][k] = v[k];
    __syncthreads();
    for (int h = STATS_NT / 2; h >= 1; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int k = 0; k < K; k++) s[t][k] = s[t][k] + s[t + h][k];
        __syncthreads();
    }
}

// Node pass: workgroup b sums the lattice rows b, b + G, b + 2G, ...; each
// thread walks x = t, t + 256, ... of a row.  partial[b] = (mass, jx, jy, jz).
template <class L, int ST>
__global__ __launch_bounds__(STATS_NT) void k_stats_nodes(const void *A, Geom g, double *partial) {
    __shared__ double s[STATS_NT][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t rows = (int64_t)g.ny * g.nz;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = (int)(r % g.ny), z = (int)(r / g.ny);
        for (int x = threadIdx.x; x < g.nx; x += STATS_NT) {
            double rho, j[3];
            node_moments<L, ST>(A, g, x, y, z, rho, j);
            acc[0] = acc[0] + rho;
            acc[1] = acc[1] + j[0];
            acc[2] = acc[2] + j[1];
            acc[3] = acc[3] + j[2];
        }
    }
    block_sum<4>(s, acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; k++) partial[(int64_t)blockIdx.x * 4 + k] = s[0][k];
}

__device__ __forceinline__ int wrap_list(const Geom &g, int axis, int c) {
    const int n = axis == 0 ? g.nx : (axis == 1 ? g.ny : g.nz);
    return c < 0 ? c + n : (c >= n ? c - n : c);
}

// Particle pass, one thread per particle: its momentum, velocity and
// hydrodynamic force, and over the nodes of its last footprint the share
// s_pn eps_n of the node's mass and momentum (s_pn = count_pn / count_n, so
// the shares of a node's owners add up to eps_n).
template <class L, int ST>
__global__ __launch_bounds__(STATS_NT) void k_stats_particles(const void *A, Geom g, Particles P,
                                                              const void *qr, int rec32, int Smax,
                                                              double *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.np) return;
    const int np = P.np;
    double r[STATS_PK];
    const double m = P.m[p];
    for (int d = 0; d < 3; d++) {
        const double v = P.v[d * np + p];
        r[d] = m * v;
        r[3 + d] = v;
        r[6 + d] = P.Fh[d * np + p];
    }
    double wr = 0.0, wj[3] = {0.0, 0.0, 0.0}, we = 0.0;
    const int len = P.list_len[p];
    const int lo0 = P.bb[p], lo1 = P.bb[np + p], lo2 = P.bb[2 * np + p];
    const uint32_t *list = P.list + (int64_t)p * P.list_cap;
    for (int e = 0; e < len; e++) {
        const uint32_t v = list[e];
        const int x = wrap_list(g, 0, lo0 + (int)((v >> 10) & 127u));
        const int y = g.wall_y ? lo1 + (int)((v >> 17) & 127u) : wrap_list(g, 1, lo1 + (int)((v >> 17) & 127u));
        const int z = L::D == 3 ? wrap_list(g, 2, lo2 + (int)((v >> 24) & 127u)) : 0;
        const int64_t n = (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
        double q[3];
        int tot;
        read_qrec(qr, rec32 != 0, n, q, tot);
        const int cnt = (int)(v & 1023u);
        const double eps = (double)(tot < Smax ? tot : Smax) / (double)Smax;
        const double w = ((double)cnt / (double)tot) * eps;
        double rho, j[3];
        node_moments<L, ST>(A, g, x, y, z, rho, j);
        wr = wr + w * rho;
        for (int d = 0; d < 3; d++) wj[d] = wj[d] + w * j[d];
        we = we + w;
    }
    r[9] = wr;
    r[10] = wj[0];
    r[11] = wj[1];
    r[12] = wj[2];
    r[13] = we;
    r[14] = m;
    for (int k = 0; k < STATS_PK; k++) out[(int64_t)p * STATS_PK + k] = r[k];
}

// Final pass, one workgroup: totals of the node partials (4 per workgroup of
// the node pass) and of the particle rows (STATS_PK each).
__global__ __launch_bounds__(STATS_NT) void k_stats_final(const double *node_part, int groups,
                                                          const double *part_rows, int np,
                                                          double *tot) {
    __shared__ double s[STATS_NT][4 + STATS_PK];
    double acc[4 + STATS_PK];
    for (int k = 0; k < 4 + STATS_PK; k++) acc[k] = 0.0;
    for (int b = threadIdx.x; b < groups; b += STATS_NT)
        for (int k = 0; k < 4; k++) acc[k] = acc[k] + node_part[(int64_t)b * 4 + k];
    for (int p = threadIdx.x; p < np; p += STATS_NT)
        for (int k = 0; k < STATS_PK; k++) acc[4 + k] = acc[4 + k] + part_rows[(int64_t)p * STATS_PK + k];
    block_sum<4 + STATS_PK>(s, acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4 + STATS_PK; k++) tot[k] = s[0][k];
}

template <class L, int ST>
hipError_t stats_dispatch(const StatsArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_stats_nodes<L, ST>), dim3(STATS_NODE_GROUPS), dim3(STATS_NT), 0, s, a.A, a.g,
                       a.node_part);
    if (a.P.np > 0)
        hipLaunchKernelGGL((k_stats_particles<L, ST>), dim3((a.P.np + STATS_NT - 1) / STATS_NT),
                           dim3(STATS_NT), 0, s, a.A, a.g, a.P, a.qr, a.rec32, a.Smax, a.part_rows);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(STATS_NT), 0, s, (const double *)a.node_part,
                       STATS_NODE_GROUPS, (const double *)a.part_rows, a.P.np, a.tot);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stats(int lattice, int storage, const StatsArgs &a, hipStream_t s) {
    if (lattice == 0) {
        if (storage == 0) return stats_dispatch<D2Q9, 0>(a, s);
        if (storage == 1) return stats_dispatch<D2Q9, 1>(a, s);
        return stats_dispatch<D2Q9, 2>(a, s);
    }
    if (storage == 0) return stats_dispatch<D3Q19, 0>(a, s);
    if (storage == 1) return stats_dispatch<D3Q19, 1>(a, s);
    return stats_dispatch<D3Q19, 2>(a, s);
}

}  // namespace lbimb
