// batch.hip -- many small periodic D3Q19 boxes with fixed spheres advanced
// together (drag-data ensemble), shifted FP32 storage.
//
// All boxes live in one pool: box b's populations are [19][L_b^3] at element
// offset off_b of the A and B arrays.  A box is cut into tiles of `rows`
// lattice rows along x; a tile is one workgroup's work for one step.  The
// per-node arithmetic is the shifted-storage collision of the single-box
// kernel (shifted_node), with the solid velocity 0 and a static footprint, so a
// box advanced in a batch gives the same bits as the same box alone.
//
// Two ways to run K steps:
//  * one launch per step over every tile (the kernel boundary orders steps);
//  * one persistent launch: workgroups take items (step, tile) from a global
//    counter in step-major order; a tile of step s waits until every tile of its
//    own box has finished step s - 1.  The tiles it waits for were taken earlier
//    by running workgroups, so progress needs no assumption about how many
//    workgroups are resident; the wait is bounded and reports an error flag if
//    the bound is ever reached, so every workgroup terminates.
#include <math.h>

#include "internal.h"
#include "lb_shared.h"

namespace lbimb {

__device__ __forceinline__ int wrapL(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

// Element (i, x, row) of a box's state, row = y + L z: the 19 direction rows
// of one lattice row are contiguous (the single-box layout f[z][y][i][x]).
__device__ __forceinline__ uint32_t belem(int Lb, int i, int x, int row) {
    return ((uint32_t)row * 19u + (uint32_t)i) * (uint32_t)Lb + (uint32_t)x;
}

// One tile of one box for one step.
__device__ __forceinline__ void batch_tile(const BatchArgs &a, const BatchBox &bx, int tile, int parity) {
    using L = D3Q19;
    const int Lb = bx.L;
    const float *A = (parity ? a.B : a.A) + bx.off;
    float *B = (parity ? a.A : a.B) + bx.off;
    const int nodes = Lb * bx.rows;
    const int row0 = tile * bx.rows;
    const float *beta_t = a.beta + bx.table;
    const float *arel_t = a.arel + bx.table;
    for (int k0 = 0; k0 < nodes; k0 += blockDim.x) {
        const int k = k0 + threadIdx.x;
        if (k >= nodes) continue;
        const int x = k % Lb;
        const int row = row0 + k / Lb;
        const int y = row % Lb, z = row / Lb;
        const uint64_t n = (uint64_t)x + (uint64_t)Lb * (uint64_t)row;
        const int xm = wrapL(x - 1, Lb), xp = wrapL(x + 1, Lb);
        const int ym = wrapL(y - 1, Lb), yp = wrapL(y + 1, Lb);
        const int zm = wrapL(z - 1, Lb), zp = wrapL(z + 1, Lb);
        float gg[L::Q];
#pragma unroll
        for (int i = 0; i < L::Q; i++) {
            const int sx = L::cx[i] == 0 ? x : (L::cx[i] > 0 ? xm : xp);
            const int sy = L::cy[i] == 0 ? y : (L::cy[i] > 0 ? ym : yp);
            const int sz = L::cz[i] == 0 ? z : (L::cz[i] > 0 ? zm : zp);
            gg[i] = A[belem(Lb, i, sx, sy + Lb * sz)];
        }
        const int cnt = a.cnt[bx.noff + n];
        const bool wave_fluid = !__any(cnt != 0);
        const int cc = cnt < a.Smax ? cnt : a.Smax;
        const float beta = cnt != 0 ? beta_t[cc] : 0.0f;
        const float ar = cnt != 0 ? arel_t[cc] : bx.arel0f;
        auto put = [&](int i, float v) { __builtin_nontemporal_store(v, &B[belem(Lb, i, x, row)]); };
        float mom[3];
        shifted_node<L, false>(gg, wave_fluid, beta, ar, 0.0f, 0.0f, 0.0f, bx.cgf, put, mom);
        if (cnt != 0) {
            const uint64_t m = (uint64_t)bx.noff + n;
            a.q[m] = mom[0];
            a.q[a.total_nodes + m] = mom[1];
            a.q[2 * a.total_nodes + m] = mom[2];
        }
    }
}

__global__ __launch_bounds__(256) void k_batch_step(BatchArgs a, int parity) {
    const int t = blockIdx.x;
    const int b = a.tile_box[t];
    const BatchBox bx = a.boxes[b];
    if (!bx.active) return;
    batch_tile(a, bx, t - bx.tile0, parity);
}

__global__ __launch_bounds__(256) void k_batch_persistent(BatchArgs a, int nsteps, int parity0) {
    // Every thread-0 section below is followed by a barrier that all threads
    // reach, and the loop has a single latch (the barrier at the end of the
    // body).  With a thread-0 branch joining directly into the loop header the
    // compiler may split the loop into nested loops by backedge, which leaves
    // lane 0 and the rest of its wavefront in different loops around the
    // barriers.
    __shared__ int s_item;
    const int64_t total = (int64_t)nsteps * a.ntiles;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;
        const int s = (int)(item / a.ntiles);
        const int t = (int)(item % a.ntiles);
        const int b = a.tile_box[t];
        const BatchBox bx = a.boxes[b];
        if (bx.active) {
            if (s > 0) {
                if (threadIdx.x == 0) {
                    const int target = s * bx.ntiles;
                    int spins = 0;
                    while (__hip_atomic_load(&a.done[b], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                        if (++spins > (1 << 22)) {
                            atomicOr(a.flags, FLAG_BATCH_TIMEOUT);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
                __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            batch_tile(a, bx, t - bx.tile0, (parity0 + s) & 1);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&a.done[b], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        // also keeps s_item unchanged until every thread has read it
        __syncthreads();
    }
}

// Per-sphere hydrodynamic force and torque from the static footprint list
// (entries: local node | count << 20), TwoSum accumulation as in the
// single-box force kernel.  One wavefront per sphere.
__global__ __launch_bounds__(256) void k_batch_force(BatchArgs a) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= a.nsph) return;
    const int b = a.sph_box[p];
    const BatchBox bx = a.boxes[b];
    const int Lb = bx.L;
    const double Ld = (double)Lb;
    const double xp0 = a.sph_x[3 * p], xp1 = a.sph_x[3 * p + 1], xp2 = a.sph_x[3 * p + 2];
    const int e0 = a.list_start[p], e1 = a.list_start[p + 1];
    double Fs[3] = {0, 0, 0}, Fc[3] = {0, 0, 0}, Ts[3] = {0, 0, 0}, Tc[3] = {0, 0, 0};
    auto add = [](double &s, double &c, double v) {
        const double x = s + v, bb = x - s;
        c = c + ((s - (x - bb)) + (v - bb));
        s = x;
    };
    for (int e = e0 + lane; e < e1; e += 64) {
        const uint32_t v = a.list[e];
        const int node = (int)(v & 0xFFFFFu);
        const int cnt = (int)(v >> 20);
        const uint64_t m = (uint64_t)bx.noff + node;
        const int tot = a.cnt[m];
        const double sh = (double)cnt / (double)tot;
        const double t0 = sh * (double)a.q[m], t1 = sh * (double)a.q[a.total_nodes + m],
                     t2 = sh * (double)a.q[2 * a.total_nodes + m];
        const int x = node % Lb, y = (node / Lb) % Lb, z = node / (Lb * Lb);
        double rx = (double)x - xp0, ry = (double)y - xp1, rz = (double)z - xp2;
        rx = rx > 0.5 * Ld ? rx - Ld : (rx < -0.5 * Ld ? rx + Ld : rx);
        ry = ry > 0.5 * Ld ? ry - Ld : (ry < -0.5 * Ld ? ry + Ld : ry);
        rz = rz > 0.5 * Ld ? rz - Ld : (rz < -0.5 * Ld ? rz + Ld : rz);
        add(Fs[0], Fc[0], t0);
        add(Fs[1], Fc[1], t1);
        add(Fs[2], Fc[2], t2);
        add(Ts[0], Tc[0], ry * t2 - rz * t1);
        add(Ts[1], Tc[1], rz * t0 - rx * t2);
        add(Ts[2], Tc[2], rx * t1 - ry * t0);
    }
#pragma unroll
    for (int mk = 32; mk >= 1; mk >>= 1)
        for (int d = 0; d < 3; d++) {
            for (int w = 0; w < 2; w++) {
                double &s = w == 0 ? Fs[d] : Ts[d];
                double &c = w == 0 ? Fc[d] : Tc[d];
                const double os = __shfl_xor(s, mk, 64), oc = __shfl_xor(c, mk, 64);
                const double x = s + os, bb = x - s;
                const double er = (s - (x - bb)) + (os - bb);
                s = x;
                c = (c + oc) + er;
            }
        }
    if (lane == 0)
        for (int d = 0; d < 3; d++) {
            a.F[3 * p + d] = -(Fs[d] + Fc[d]);
            a.T[3 * p + d] = -(Ts[d] + Tc[d]);
        }
}

// Superficial mean momentum per box: U_b = (1/N_b) sum_n sum_i g_i c_i
// (binary64 sums, one workgroup per box, fixed order).
__global__ __launch_bounds__(256) void k_batch_mean(BatchArgs a, int parity, double *U) {
    using L = D3Q19;
    __shared__ double red[3][256];
    const int b = blockIdx.x;
    const BatchBox bx = a.boxes[b];
    const uint64_t N = (uint64_t)bx.L * bx.L * bx.L;
    const float *A = (parity ? a.B : a.A) + bx.off;
    double s[3] = {0.0, 0.0, 0.0};
    for (uint64_t n = threadIdx.x; n < N; n += blockDim.x) {
        // moments of the post-collision populations: the same total as the
        // streamed ones on a periodic box
        const int x = (int)(n % (uint64_t)bx.L), row = (int)(n / (uint64_t)bx.L);
#pragma unroll
        for (int i = 1; i < L::Q; i++) {
            const double g = (double)A[belem(bx.L, i, x, row)];
            if (L::cx[i]) s[0] += L::cx[i] * g;
            if (L::cy[i]) s[1] += L::cy[i] * g;
            if (L::cz[i]) s[2] += L::cz[i] * g;
        }
    }
    for (int d = 0; d < 3; d++) red[d][threadIdx.x] = s[d];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; d++) {
            double t = 0.0;
            for (int k = 0; k < (int)blockDim.x; k++) t += red[d][k];
            U[3 * b + d] = t / (double)N;
        }
}

// Pre-collision populations of one box: f_i(x) = w_i + A_i(x - c_i).
__global__ void k_batch_get_f(BatchArgs a, int b, int parity, double *f) {
    using L = D3Q19;
    const BatchBox bx = a.boxes[b];
    const int Lb = bx.L;
    const uint64_t N = (uint64_t)Lb * Lb * Lb;
    const uint64_t n = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const float *A = (parity ? a.B : a.A) + bx.off;
    const int x = (int)(n % Lb), y = (int)((n / Lb) % Lb), z = (int)(n / ((uint64_t)Lb * Lb));
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const int sx = wrapL(x - L::cx[i], Lb), sy = wrapL(y - L::cy[i], Lb), sz = wrapL(z - L::cz[i], Lb);
        const float g = A[belem(Lb, i, sx, sy + Lb * sz)];
        f[(uint64_t)i * N + n] = L::w[L::wc[i]] + (double)g;
    }
}

hipError_t launch_batch_get_f(const BatchArgs &a, int b, int L, int parity, double *f, hipStream_t s) {
    const uint64_t N = (uint64_t)L * L * L;
    hipLaunchKernelGGL(k_batch_get_f, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, a, b, parity, f);
    return hipGetLastError();
}

// Initial state of every box: the uniform populations g0 in both arrays.
__global__ void k_batch_init(BatchArgs a) {
    const BatchBox bx = a.boxes[blockIdx.y];
    const uint64_t N = (uint64_t)bx.L * bx.L * bx.L;
    const uint64_t n = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % (uint64_t)bx.L), row = (int)(n / (uint64_t)bx.L);
#pragma unroll
    for (int i = 0; i < 19; i++) {
        a.A[bx.off + belem(bx.L, i, x, row)] = bx.g0[i];
        a.B[bx.off + belem(bx.L, i, x, row)] = bx.g0[i];
    }
}

hipError_t launch_batch_init(const BatchArgs &a, int nbox, int maxL, hipStream_t s) {
    const uint64_t N = (uint64_t)maxL * maxL * maxL;
    hipLaunchKernelGGL(k_batch_init, dim3((unsigned)((N + 255) / 256), (unsigned)nbox), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Mean pre-collision fluid velocity u = (sum_i c_i f_i) / (sum_i f_i) over the
// fluid nodes (no sub-cell sample of any sphere) whose minimum-image distance
// to the sphere centre lies in [R + 1, 2R]: the local flow a sphere sees.  One
// workgroup per sphere over the cube of nodes around the centre; each node
// counted once, through its minimum image; fixed-order workgroup reduction.
__global__ __launch_bounds__(256) void k_batch_shell(BatchArgs a, int parity, double *out) {
    using L = D3Q19;
    __shared__ double red[4][256];
    const int p = blockIdx.x;
    const BatchBox bx = a.boxes[a.sph_box[p]];
    const int Lb = bx.L;
    const double Ld = (double)Lb;
    const double R = bx.radius, rin2 = (R + 1.0) * (R + 1.0), rout2 = 4.0 * R * R;
    const double xc[3] = {a.sph_x[3 * p], a.sph_x[3 * p + 1], a.sph_x[3 * p + 2]};
    const int h = (int)ceil(2.0 * R) + 1;
    const int w = 2 * h + 1;
    const int cube = w * w * w;
    int base[3];
    for (int d = 0; d < 3; d++) base[d] = (int)floor(xc[d]);
    const float *A = (parity ? a.B : a.A) + bx.off;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < cube; t += blockDim.x) {
        const int off[3] = {t % w - h, (t / w) % w - h, t / (w * w) - h};
        int c[3];
        double r2 = 0.0;
        bool once = true;
        for (int d = 0; d < 3; d++) {
            const double rd = (double)(base[d] + off[d]) - xc[d];
            once = once && rd > -0.5 * Ld && rd <= 0.5 * Ld;
            r2 += rd * rd;
            int cd = (base[d] + off[d]) % Lb;
            c[d] = cd < 0 ? cd + Lb : cd;
        }
        if (!once || r2 < rin2 || r2 > rout2) continue;
        const int row = c[1] + Lb * c[2];
        const uint64_t n = (uint64_t)c[0] + (uint64_t)Lb * (uint64_t)row;
        if (a.cnt[bx.noff + n] != 0) continue;
        double rho = 1.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < L::Q; i++) {
            const int sx = wrapL(c[0] - L::cx[i], Lb), sy = wrapL(c[1] - L::cy[i], Lb), sz = wrapL(c[2] - L::cz[i], Lb);
            const double g = (double)A[belem(Lb, i, sx, sy + Lb * sz)];
            rho += g;
            j[0] += L::cx[i] * g;
            j[1] += L::cy[i] * g;
            j[2] += L::cz[i] * g;
        }
        for (int d = 0; d < 3; d++) s[d] += j[d] / rho;
        s[3] += 1.0;
    }
    for (int d = 0; d < 4; d++) red[d][threadIdx.x] = s[d];
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k)
            for (int d = 0; d < 4; d++) red[d][threadIdx.x] += red[d][threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; d++) out[3 * p + d] = red[3][0] > 0.0 ? red[d][0] / red[3][0] : 0.0;
}

hipError_t launch_batch_shell(const BatchArgs &a, int parity, double *u, hipStream_t s) {
    if (a.nsph == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_shell, dim3((unsigned)a.nsph), dim3(256), 0, s, a, parity, u);
    return hipGetLastError();
}

// Steady-drag check after a chunk of steps, on the device: one workgroup,
// thread k takes the boxes k, k + 256, ...  An active box with spheres
// retires when max over its spheres and components of |F - F_prev| is below
// tol times the mean over its spheres of |F| (both from the force kernel of
// the chunk's last step); the first check of a run only records F_prev.
// Boxes without spheres never retire.  Each box's sums run in sphere order,
// so the decision is reproducible.  The check time and the first-check flag
// live on the device (*st.tnow advances by the chunk's k steps), so one
// captured chunk serves every replay.  *remaining receives the active boxes
// left.
__global__ __launch_bounds__(256) void k_batch_check(BatchArgs a, BatchBox *boxes, BatchSteady st, int64_t k) {
    __shared__ int live[256];
    const int64_t t = *st.tnow + k;
    const int first = *st.first;
    int n_live = 0;
    for (int b = threadIdx.x; b < a.nbox; b += blockDim.x) {
        if (!boxes[b].active) continue;
        const int p0 = boxes[b].sph0, np = boxes[b].nsph;
        bool retire = false;
        if (!first && np > 0) {
            double scale = 0.0, dmax = 0.0;
            for (int p = p0; p < p0 + np; p++) {
                const double f0 = a.F[3 * p], f1 = a.F[3 * p + 1], f2 = a.F[3 * p + 2];
                scale = scale + sqrt(f0 * f0 + f1 * f1 + f2 * f2);
                for (int d = 0; d < 3; d++) dmax = fmax(dmax, fabs(a.F[3 * p + d] - st.Fprev[3 * p + d]));
            }
            scale = scale / (double)np;
            retire = scale > 0.0 && dmax / scale < st.tol;
        }
        for (int p = p0; p < p0 + np; p++)
            for (int d = 0; d < 3; d++) st.Fprev[3 * p + d] = a.F[3 * p + d];
        if (retire) {
            boxes[b].active = 0;
            st.steady[b] = 1;
            st.stop[b] = t;
        } else {
            n_live++;
        }
    }
    live[threadIdx.x] = n_live;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) live[threadIdx.x] += live[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {  // every thread read *tnow and *first before the barriers above
        *st.remaining = live[0];
        *st.tnow = t;
        *st.first = 0;
    }
}

hipError_t launch_batch_check(const BatchArgs &a, BatchBox *boxes, const BatchSteady &st, int64_t k,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_batch_check, dim3(1), dim3(256), 0, s, a, boxes, st, k);
    return hipGetLastError();
}

// The 40 closure inputs of every sphere, binary32 [nsph][40]; one wavefront
// per sphere, lane j holding sphere j of the same box (at most 64 per box).
//   0      local solid fraction: spheres other than this one whose
//          minimum-image centre distance is below 3R, over 27
//   1      log10 of max(Re, 1e-6), Re = |U| d / nu, U the box's superficial
//          mean velocity, d = 2R, nu = (tau - 1/2) / 3
//   2..4   shell velocity Us of the sphere over |U| in the flow frame
//          (e_x = U / |U|; e_y = e_x x z-hat normalised, or e_x x y-hat when
//          that is shorter than 1e-8; e_z = e_x x e_y)
//   5..36  the 16 nearest other spheres (distance, then index), each as its
//          offset along e_x over d and its distance across e_x over d; the
//          slots beyond the box's other spheres hold L / d
//   37     box solid fraction n (4/3) pi R^3 / L^3
//   38     d / L
//   39     nearest surface gap (min distance - d) / d, or L / d alone in a box
// Arithmetic is binary64, rounded to binary32 at the store.
__global__ __launch_bounds__(256) void k_batch_features(BatchArgs a, const double *U, const double *Us,
                                                        float *feat) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= a.nsph) return;
    const int b = a.sph_box[p];
    const BatchBox bx = a.boxes[b];
    const int n = bx.nsph, me = p - bx.sph0;
    const double R = bx.radius, Ld = (double)bx.L, d = 2.0 * R, nu = (bx.tau - 0.5) / 3.0;
    const double u0 = U[3 * b], u1 = U[3 * b + 1], u2 = U[3 * b + 2];
    const double umag = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
    const double re = umag * d / nu;
    double ex[3] = {1.0, 0.0, 0.0};
    if (umag > 0.0) {
        ex[0] = u0 / umag;
        ex[1] = u1 / umag;
        ex[2] = u2 / umag;
    }
    const bool other = lane < n && lane != me;
    double dv[3] = {0.0, 0.0, 0.0}, dist = INFINITY;
    if (other) {
        const int j = bx.sph0 + lane;
        for (int k = 0; k < 3; k++) {
            const double v = a.sph_x[3 * j + k] - a.sph_x[3 * p + k];
            dv[k] = v - Ld * rint(v / Ld);
        }
        dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    }
    int rank = 0;
    double dmin = dist;
    for (int k = 0; k < 64; k++) {
        const double dk = __shfl(dist, k, 64);
        rank += (dk < dist || (dk == dist && k < lane)) ? 1 : 0;
        dmin = fmin(dmin, dk);
    }
    const int n_loc = __popcll(__ballot(other && dist < 3.0 * R));
    float *row = feat + (int64_t)40 * p;
    if (other && rank < 16) {
        const double along = dv[0] * ex[0] + dv[1] * ex[1] + dv[2] * ex[2];
        const double across = sqrt(fmax(dist * dist - along * along, 0.0));
        row[5 + 2 * rank] = (float)(along / d);
        row[6 + 2 * rank] = (float)(across / d);
    }
    if (lane >= n - 1 && lane < 16) {  // slots beyond the other spheres
        row[5 + 2 * lane] = (float)(Ld / d);
        row[6 + 2 * lane] = (float)(Ld / d);
    }
    if (lane == 0) {
        double ey[3] = {ex[1], -ex[0], 0.0};  // e_x x z-hat
        double ny = sqrt(ey[0] * ey[0] + ey[1] * ey[1] + ey[2] * ey[2]);
        if (ny < 1e-8) {  // e_x x y-hat
            ey[0] = -ex[2];
            ey[1] = 0.0;
            ey[2] = ex[0];
            ny = sqrt(ey[0] * ey[0] + ey[1] * ey[1] + ey[2] * ey[2]);
        }
        for (int k = 0; k < 3; k++) ey[k] = ey[k] / ny;
        const double ez[3] = {ex[1] * ey[2] - ex[2] * ey[1], ex[2] * ey[0] - ex[0] * ey[2],
                              ex[0] * ey[1] - ex[1] * ey[0]};
        const double um = fmax(umag, 1e-300);
        const double us[3] = {Us[3 * p] / um, Us[3 * p + 1] / um, Us[3 * p + 2] / um};
        row[0] = (float)((double)n_loc / 27.0);
        row[1] = (float)log10(fmax(re, 1e-6));
        row[2] = (float)(us[0] * ex[0] + us[1] * ex[1] + us[2] * ex[2]);
        row[3] = (float)(us[0] * ey[0] + us[1] * ey[1] + us[2] * ey[2]);
        row[4] = (float)(us[0] * ez[0] + us[1] * ez[1] + us[2] * ez[2]);
        const double vol = 4.0 / 3.0 * M_PI * R * R * R;
        row[37] = (float)((double)n * vol / (Ld * Ld * Ld));
        row[38] = (float)(d / Ld);
        row[39] = (float)(n > 1 ? (dmin - d) / d : Ld / d);
    }
}

hipError_t launch_batch_features(const BatchArgs &a, const double *U, const double *Us, float *feat,
                                 hipStream_t s) {
    if (a.nsph == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_features, dim3((unsigned)((a.nsph + 3) / 4)), dim3(256), 0, s, a, U, Us, feat);
    return hipGetLastError();
}

int batch_persistent_grid() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_persistent, 256, 0) != hipSuccess || per < 1)
        per = 1;
    return cus * per;
}

hipError_t launch_batch_step(const BatchArgs &a, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_step, dim3((unsigned)a.ntiles), dim3(256), 0, s, a, parity);
    return hipGetLastError();
}

hipError_t launch_batch_persistent(const BatchArgs &a, int nsteps, int parity0, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_persistent, dim3((unsigned)grid), dim3(256), 0, s, a, nsteps, parity0);
    return hipGetLastError();
}

hipError_t launch_batch_force(const BatchArgs &a, hipStream_t s) {
    if (a.nsph == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_force, dim3((unsigned)((a.nsph + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_mean(const BatchArgs &a, int parity, double *U, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_mean, dim3((unsigned)a.nbox), dim3(256), 0, s, a, parity, U);
    return hipGetLastError();
}

}  // namespace lbimb
