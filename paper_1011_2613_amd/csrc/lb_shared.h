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

// Shifted-storage collision of one node, binary32, written per direction pair
// (i, opp(i)) so the parts of f^eq and of Omega^S that are even or odd in c_i
// are formed once per pair, with explicit fused multiply-adds.
//
// v_i is g_i = f_i - w_i (SCALED = false) or g_i / w_i (SCALED = true, the
// half-precision storage unit).  With drho = sum g, rho = 1 + drho,
// u = sum g c / rho, E = drho - 1.5 rho u.u and per pair cu = c_i . u:
//   g^eq_i / w_i = E + 4.5 rho cu^2 + 3 rho cu          (even + odd part)
//   g*_i = (1 - a) g_i + a g^eq_i + 3 w_i rho c_i . g_f + beta Omega_i
//   Omega_i / w_i = (v_opp - v_i) + rho (P + Q),   Omega_opp / w_i = (v_i - v_opp) + rho (P - Q)
//   P = 4.5 ((c.V)^2 - cu^2) - 1.5 (V.V - u.u),    Q = 3 (c.V + cu)
// (the w_i terms of the two equilibria cancel in Omega).  `wave_fluid`: no
// node of the wavefront is covered, plain BGK for all lanes; otherwise every
// lane runs the IMB form with its own beta, relaxation factor ar and solid
// velocity V (an uncovered lane passes beta = 0, ar = 1/tau, V = 0).  Each
// post-collision value goes out through put(i, value in storage units); mom
// receives beta * sum_i Omega_i c_i.
template <class L, bool SCALED, class Put>
__device__ __forceinline__ void shifted_node(const float (&v)[L::Q], bool wave_fluid, float beta, float ar,
                                             float V0, float V1, float V2, const float *cgf, Put put,
                                             float mom[3]) {
    const float wf[3] = {(float)L::w[0], (float)L::w[1], (float)L::w[2]};
    // moments, grouped by weight class in the scaled unit
    float s[3] = {v[0], 0.0f, 0.0f}, jx[3] = {0.0f, 0.0f, 0.0f}, jy[3] = {0.0f, 0.0f, 0.0f},
          jz[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const int k = L::wc[i];
        s[k] = s[k] + v[i];
        if (L::cx[i] > 0) jx[k] = jx[k] + v[i]; else if (L::cx[i] < 0) jx[k] = jx[k] - v[i];
        if (L::cy[i] > 0) jy[k] = jy[k] + v[i]; else if (L::cy[i] < 0) jy[k] = jy[k] - v[i];
        if (L::D == 3) { if (L::cz[i] > 0) jz[k] = jz[k] + v[i]; else if (L::cz[i] < 0) jz[k] = jz[k] - v[i]; }
    }
    float drho, Jx, Jy, Jz;
    if (SCALED) {
        drho = fmaf(wf[2], s[2], fmaf(wf[1], s[1], wf[0] * s[0]));
        Jx = fmaf(wf[2], jx[2], wf[1] * jx[1]);
        Jy = fmaf(wf[2], jy[2], wf[1] * jy[1]);
        Jz = fmaf(wf[2], jz[2], wf[1] * jz[1]);
    } else {
        drho = (s[0] + s[1]) + s[2];
        Jx = jx[1] + jx[2];
        Jy = jy[1] + jy[2];
        Jz = jz[1] + jz[2];
    }
    const float rho = 1.0f + drho;
    const float rinv = 1.0f / rho;
    const float ux = Jx * rinv, uy = Jy * rinv, uz = L::D == 3 ? Jz * rinv : 0.0f;
    float usq = fmaf(uy, uy, ux * ux);
    if (L::D == 3) usq = fmaf(uz, uz, usq);
    const float E = fmaf(-1.5f * rho, usq, drho);
    const float R3 = 3.0f * rho, R45 = 4.5f * rho;
    const float omr = 1.0f - ar;
    // per weight class: a * W and 3 rho * W, W = w (g unit) or 1 (scaled unit)
    float arW[3], R3W[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        arW[k] = SCALED ? ar : ar * wf[k];
        R3W[k] = SCALED ? R3 : R3 * wf[k];
    }
    mom[0] = mom[1] = mom[2] = 0.0f;
    if (wave_fluid) {
        put(0, fmaf(omr, v[0], arW[0] * E));
#pragma unroll
        for (int i = 1; i < L::Q; i++) {
            const int o = L::opp[i];
            if (o < i) continue;
            const int k = L::wc[i];
            const float cu = cdot<L>(i, ux, uy, uz);
            const float b = arW[k] * fmaf(R45 * cu, cu, E);
            const float a = R3W[k] * fmaf(ar, cu, cgf[i]);
            put(i, fmaf(omr, v[i], b + a));
            put(o, fmaf(omr, v[o], b - a));
        }
        return;
    }
    float VV = fmaf(V1, V1, V0 * V0);
    if (L::D == 3) VV = fmaf(V2, V2, VV);
    const float K = -1.5f * (VV - usq);
    const float rW0 = SCALED ? rho : rho * wf[0];
    const float bOm0 = beta * (rW0 * K);
    put(0, fmaf(omr, v[0], arW[0] * E) + bOm0);
    // sum_i Omega_i c_i per class in the storage unit: pairs contribute c_i (Omega_i - Omega_opp)
    float mx[3] = {0.0f, 0.0f, 0.0f}, my[3] = {0.0f, 0.0f, 0.0f}, mz[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const int o = L::opp[i];
        if (o < i) continue;
        const int k = L::wc[i];
        const float rW = SCALED ? rho : rho * wf[k];
        const float cu = cdot<L>(i, ux, uy, uz);
        const float cV = cdot<L>(i, V0, V1, V2);
        const float b = arW[k] * fmaf(R45 * cu, cu, E);
        const float a = R3W[k] * fmaf(ar, cu, cgf[i]);
        const float P = fmaf(4.5f, fmaf(cV, cV, -(cu * cu)), K);
        const float Q = 3.0f * (cV + cu);
        const float d = v[i] - v[o];
        const float Omi = fmaf(rW, P + Q, -d);
        const float Omo = fmaf(rW, P - Q, d);
        put(i, fmaf(beta, Omi, fmaf(omr, v[i], b + a)));
        put(o, fmaf(beta, Omo, fmaf(omr, v[o], b - a)));
        const float dm = Omi - Omo;
        if (L::cx[i] > 0) mx[k] = mx[k] + dm; else if (L::cx[i] < 0) mx[k] = mx[k] - dm;
        if (L::cy[i] > 0) my[k] = my[k] + dm; else if (L::cy[i] < 0) my[k] = my[k] - dm;
        if (L::D == 3) { if (L::cz[i] > 0) mz[k] = mz[k] + dm; else if (L::cz[i] < 0) mz[k] = mz[k] - dm; }
    }
    if (SCALED) {
        mom[0] = beta * fmaf(wf[2], mx[2], wf[1] * mx[1]);
        mom[1] = beta * fmaf(wf[2], my[2], wf[1] * my[1]);
        mom[2] = beta * fmaf(wf[2], mz[2], wf[1] * mz[1]);
    } else {
        mom[0] = beta * (mx[1] + mx[2]);
        mom[1] = beta * (my[1] + my[2]);
        mom[2] = beta * (mz[1] + mz[2]);
    }
}

}  // namespace lbimb
