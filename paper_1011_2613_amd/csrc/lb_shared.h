// lb_shared.h -- device helpers shared by the single-box and the batched
// lattice kernels: storage types, lattice sums, addressing and the
// shifted-storage collision of one node.
#pragma once

#include "internal.h"

namespace lbimb {

// ------------------------------------------------------------ storage
template <int ST> struct Store;
template <> struct Store<0> { using T = double; };
template <> struct Store<1> { using T = float; };
template <> struct Store<2> { using T = _Float16; };

// c_i . u with the zero components of c_i dropped (exact for c in {-1,0,1}).
template <class L, class R>
__device__ __forceinline__ R cdot(int i, R ux, R uy, R uz) {
    R s = R(0);
    bool first = true;
    if (L::cx[i] != 0) { s = L::cx[i] > 0 ? ux : -ux; first = false; }
    if (L::cy[i] != 0) {
        if (first) { s = L::cy[i] > 0 ? uy : -uy; first = false; }
        else s = L::cy[i] > 0 ? s + uy : s - uy;
    }
    if (L::D == 3 && L::cz[i] != 0) {
        if (first) { s = L::cz[i] > 0 ? uz : -uz; first = false; }
        else s = L::cz[i] > 0 ? s + uz : s - uz;
    }
    return s;
}

// Sum over directions of c_ia * v_i, index order, zero terms dropped.
template <class L, int AX, class R>
__device__ __forceinline__ R cmoment(const R (&v)[L::Q]) {
    R s = R(0);
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const int c = AX == 0 ? L::cx[i] : (AX == 1 ? L::cy[i] : L::cz[i]);
        if (c > 0) s = s + v[i];
        else if (c < 0) s = s - v[i];
    }
    return s;
}

// ------------------------------------------------------------- addressing
// Every direction array has a base address that is uniform across the grid
// (scalar registers); a node is a 32-bit byte offset from it when the array is
// below 4 GiB, so loads and stores use the scalar-base + vector-offset form.
template <class T, bool OFF32>
__device__ __forceinline__ const T *at(const T *base, uint64_t idx) {
    if (OFF32) return (const T *)((const char *)base + (uint32_t)((uint32_t)idx * (uint32_t)sizeof(T)));
    return base + idx;
}

template <class T, bool OFF32>
__device__ __forceinline__ T *at(T *base, uint64_t idx) {
    if (OFF32) return (T *)((char *)base + (uint32_t)((uint32_t)idx * (uint32_t)sizeof(T)));
    return base + idx;
}

// Shifted-storage collision of one node.  `wave_fluid`: no node of the
// wavefront is covered (plain BGK path for all lanes); otherwise every lane
// runs the IMB formula with its own beta, relaxation factor ar and solid
// velocity V (an uncovered lane passes beta = 0, ar = 1/tau, V = 0).  Each
// post-collision value goes out through put(i, value); mom receives
// beta * sum_i Omega_i c_i.
template <class L, class Put>
__device__ __forceinline__ void shifted_node(const float (&gg)[L::Q], bool wave_fluid, float beta, float ar,
                                             float V0, float V1, float V2, const float *cgf, Put put,
                                             float mom[3]) {
    float drho = gg[0];
#pragma unroll
    for (int i = 1; i < L::Q; i++) drho = drho + gg[i];
    const float rho = 1.0f + drho;
    const float jx = cmoment<L, 0>(gg), jy = cmoment<L, 1>(gg);
    const float jz = L::D == 3 ? cmoment<L, 2>(gg) : 0.0f;
    const float ux = jx / rho, uy = jy / rho, uz = L::D == 3 ? jz / rho : 0.0f;
    float usq = ux * ux + uy * uy;
    if (L::D == 3) usq = usq + uz * uz;
    const float t15 = 1.5f * usq;
    const float wf[3] = {(float)L::w[0], (float)L::w[1], (float)L::w[2]};
    const float wrf[3] = {wf[0] * rho, wf[1] * rho, wf[2] * rho};
    const float w3r[3] = {3.0f * wf[0] * rho, 3.0f * wf[1] * rho, 3.0f * wf[2] * rho};
    auto cu_of = [&](int i) { return i == 0 ? 0.0f : cdot<L>(i, ux, uy, uz); };
    mom[0] = mom[1] = mom[2] = 0.0f;
    if (wave_fluid) {
#pragma unroll
        for (int i = 0; i < L::Q; i++) {
            const float cu = cu_of(i);
            const float geq = wf[L::wc[i]] * (drho + rho * (3.0f * cu + 4.5f * cu * cu - t15));
            put(i, gg[i] - ar * (gg[i] - geq) + w3r[L::wc[i]] * cgf[i]);
        }
        return;
    }
    float VV = V0 * V0 + V1 * V1;
    if (L::D == 3) VV = VV + V2 * V2;
    const float v15 = 1.5f * VV;
    float mx = 0.0f, my = 0.0f, mz = 0.0f;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const float cV = i == 0 ? 0.0f : cdot<L>(i, V0, V1, V2);
        const float cu = cu_of(i);
        const float pV = 3.0f * cV + 4.5f * cV * cV - v15;
        const float pu = -3.0f * cu + 4.5f * cu * cu - t15;
        const float Om = (gg[L::opp[i]] - gg[i]) + wrf[L::wc[i]] * (pV - pu);
        const float geq = wf[L::wc[i]] * (drho + rho * (3.0f * cu + 4.5f * cu * cu - t15));
        put(i, gg[i] - ar * (gg[i] - geq) + beta * Om + w3r[L::wc[i]] * cgf[i]);
        if (L::cx[i] > 0) mx = mx + Om; else if (L::cx[i] < 0) mx = mx - Om;
        if (L::cy[i] > 0) my = my + Om; else if (L::cy[i] < 0) my = my - Om;
        if (L::D == 3) { if (L::cz[i] > 0) mz = mz + Om; else if (L::cz[i] < 0) mz = mz - Om; }
    }
    mom[0] = beta * mx;
    mom[1] = beta * my;
    mom[2] = beta * mz;
}

}  // namespace lbimb
