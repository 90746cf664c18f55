// mlp.hip -- learned drag closure on gfx950 matrix cores.
//
// Network 40 -> 128 -> 128 -> 128 -> 1, SiLU on the hidden layers.  Every
// matrix product uses v_mfma_f32_16x16x32_bf16: bfloat16 operands, binary32
// accumulation.  Operand fragments (one wavefront, 64 lanes):
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + j], j = 0..7
//   B (32 x 16): lane l holds B[8 (l / 16) + j][l % 16]
//   D (16 x 16): lane l holds D[4 (l / 16) + i][l % 16], i = 0..3
//
// Forward: one workgroup of twelve wavefronts keeps all weights in LDS as
// bfloat16 (rows padded so the 16 rows a fragment touches fall in distinct LDS
// banks) and loops over 16-row tiles, one tile per wavefront; a layer's eight
// output tiles accumulate in registers (eight independent MFMA chains per A
// fragment) and then overwrite the wavefront's activation tile in LDS.  Training mode also writes pre-activations and the
// bfloat16 activations to HBM for the backward pass.
// Backward: weight gradients dW = dZ^T H and input gradients dH = dZ W are
// MFMA GEMMs where one wavefront owns one 16 x 16 output tile and runs over the
// whole reduction, so every gradient is summed in a fixed order (deterministic,
// no atomics).  Bias gradients and the width-1 output layer use binary32 sums
// in row order.  Adam updates binary32 master weights and refreshes the
// bfloat16 copies.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>

#include "../../include/lbimb.h"
#include "../../include/mlp_closure.h"
#include "internal.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int NIN = MLP_NIN, NH = MLP_NHID, KIN = 64;  // input padded to 64
constexpr int S1 = 72;   // LDS row stride (bf16) of W1 and of the padded input
constexpr int SH = 136;  // LDS row stride (bf16) of 128-wide rows
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH,
              OFF_W4 = OFF_B3 + NH, OFF_B4 = OFF_W4 + NH, NPAR = OFF_B4 + 1;
static_assert(NPAR == MLP_NPARAMS, "parameter count");

// bfloat16 weight copies used by the kernels (global memory):
//   w1 [128][64] (columns 40..63 zero), w2, w3 [128][128], w4 [16][128] (rows 1..15 zero)
struct Wbf {
    __bf16 *w1, *w2, *w3, *w4;
};

// LDS written by some lanes of a wavefront and read by others: order the
// accesses within the wavefront (no cross-wavefront barrier is needed because
// each wavefront owns its activation buffers).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SiLU of the forward pass from the hardware base-2 exponential and
// reciprocal (e^-z = 2^(-z log2 e)): a few ulp of binary32, far below the
// bfloat16 rounding that follows, and about a fifth of the instructions of
// the correctly rounded form, which made the forward pass ALU-bound.
__device__ __forceinline__ float silu_fwd(float z) {
    const float e = __builtin_amdgcn_exp2f(-z * 1.44269504088896341f);
    return z * __builtin_amdgcn_rcpf(1.0f + e);
}
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

struct FwdArgs {
    const float *X;      // [n][40]
    const float *nmu;    // inputs enter as (X - nmu) / nsd when not null
    const float *nsd;
    int64_t n;
    const float *p;      // master parameters (biases read from here)
    Wbf w;
    float *y;            // [n]
    // training outputs (row stride 128 / 64), may be null in inference
    __bf16 *h0, *h1, *h2, *h3;
    float *z1, *z2, *z3;
};

// One dense layer for a 16-row tile held in LDS (row stride SIN), computed
// transposed: acc[mt] = W[16 mt .. 16 mt + 15] in^T, so that a lane's four
// results are four consecutive output features of one row (row l mod 16,
// features 16 mt + 4 (l / 16) + i) and go to LDS as one 8-byte write.  The
// reduction index is outermost, so one fragment of the input feeds NT
// independent MFMA chains; each output element still accumulates its K/32
// products in ascending order.
template <int K, int SIN, int SW, int NT>
__device__ __forceinline__ void layer_tiles(const __bf16 *sin, const __bf16 *sw, f32x4 (&acc)[NT]) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int nt = 0; nt < NT; nt++) acc[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < K / 32; kt++) {
        const bf16x8 x = *(const bf16x8 *)(sin + (l & 15) * SIN + kt * 32 + 8 * (l >> 4));
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const bf16x8 w = *(const bf16x8 *)(sw + (nt * 16 + (l & 15)) * SW + kt * 32 + 8 * (l >> 4));
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x, acc[nt], 0, 0, 0);
        }
    }
}

// Forward workgroup: FWD_WAVES wavefronts share the bfloat16 weights, the
// hidden biases and the input normaliser in LDS; each wavefront owns one
// activation tile (16 rows) that every layer overwrites in place once its
// products are in registers.
constexpr int FWD_WAVES = 12;
constexpr int FWD_WAVES_TRAIN = 8;  // training also streams activations out

template <bool TRAIN>
__global__ __launch_bounds__(TRAIN ? 64 * FWD_WAVES_TRAIN : 64 * FWD_WAVES) void k_mlp_forward(FwdArgs a) {
    constexpr int NWV = TRAIN ? FWD_WAVES_TRAIN : FWD_WAVES;
    __shared__ __attribute__((aligned(16))) __bf16 sW1[NH * S1];
    __shared__ __attribute__((aligned(16))) __bf16 sW2[NH * SH];
    __shared__ __attribute__((aligned(16))) __bf16 sW3[NH * SH];
    __shared__ __attribute__((aligned(16))) __bf16 sW4[16 * SH];
    __shared__ __attribute__((aligned(16))) __bf16 sAct[FWD_WAVES][16 * SH];
    __shared__ __attribute__((aligned(16))) float sBias[3 * NH];
    __shared__ float sMu[NIN], sRsd[NIN];
    const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
    // weights -> LDS, 8 bf16 per copy
    for (int c = tid; c < NH * KIN / 8; c += blockDim.x) {
        const int r = c / (KIN / 8), k = (c % (KIN / 8)) * 8;
        *(bf16x8 *)(sW1 + r * S1 + k) = *(const bf16x8 *)(a.w.w1 + r * KIN + k);
    }
    for (int c = tid; c < NH * NH / 8; c += blockDim.x) {
        const int r = c / (NH / 8), k = (c % (NH / 8)) * 8;
        *(bf16x8 *)(sW2 + r * SH + k) = *(const bf16x8 *)(a.w.w2 + r * NH + k);
        *(bf16x8 *)(sW3 + r * SH + k) = *(const bf16x8 *)(a.w.w3 + r * NH + k);
    }
    for (int c = tid; c < 16 * NH / 8; c += blockDim.x) {
        const int r = c / (NH / 8), k = (c % (NH / 8)) * 8;
        *(bf16x8 *)(sW4 + r * SH + k) = *(const bf16x8 *)(a.w.w4 + r * NH + k);
    }
    for (int c = tid; c < 3 * NH; c += blockDim.x) {
        const int layer = c / NH, col = c % NH;
        sBias[c] = a.p[(layer == 0 ? OFF_B1 : (layer == 1 ? OFF_B2 : OFF_B3)) + col];
    }
    const bool norm = !TRAIN && a.nmu;
    if (norm)
        for (int k = tid; k < NIN; k += blockDim.x) {
            sMu[k] = a.nmu[k];
            sRsd[k] = 1.0f / a.nsd[k];
        }
    __syncthreads();
    __bf16 *buf = sAct[wv];
    const int64_t ntiles = (a.n + 15) / 16;
    // the 16 rows of a tile are 640 consecutive binary32 values of X: ten
    // coalesced loads per lane, issued one tile ahead in inference (training
    // loads the tile where it is used: its registers go to the extra stores)
    constexpr int XL = 16 * NIN / 64;
    auto load_tile = [&](int64_t t, float (&xv)[XL]) {
        const int64_t base = t * 16 * NIN, lim = a.n * NIN - base;
#pragma unroll
        for (int j = 0; j < XL; j++) {
            const int idx = j * 64 + l;
            xv[j] = (t < ntiles && idx < lim) ? a.X[base + idx] : 0.0f;
        }
    };
    float xv[XL];
    int64_t tile = (int64_t)blockIdx.x * NWV + wv;
    if (!TRAIN) load_tile(tile, xv);
    // this lane's row of a tile and the first of its four features
    const int lr = l & 15, lf = 4 * (l >> 4);
    for (; tile < ntiles; tile += (int64_t)gridDim.x * NWV) {
        const int64_t r0 = tile * 16;
        const bool row_in = r0 + lr < a.n;
        if (TRAIN) load_tile(tile, xv);
        // input tile: 16 rows x 64 (40 features, zero padded), binary32 -> bfloat16
#pragma unroll
        for (int j = 0; j < XL; j++) {
            const int idx = j * 64 + l, r = idx / NIN, k = idx % NIN;
            float xk = xv[j];
            if (norm && r0 + r < a.n) xk = (xk - sMu[k]) * sRsd[k];
            const __bf16 q = (__bf16)xk;
            buf[r * S1 + k] = q;
            if (TRAIN && r0 + r < a.n) a.h0[(r0 + r) * KIN + k] = q;
        }
        for (int c = l; c < 16 * (KIN - NIN); c += 64) {
            const int r = c / (KIN - NIN), k = NIN + c % (KIN - NIN);
            buf[r * S1 + k] = (__bf16)0.0f;
            if (TRAIN && r0 + r < a.n) a.h0[(r0 + r) * KIN + k] = (__bf16)0.0f;
        }
        if (!TRAIN) load_tile(tile + (int64_t)gridDim.x * NWV, xv);
        wave_sync();
        // hidden layers
#pragma unroll
        for (int layer = 0; layer < 3; layer++) {
            __bf16 *hg = layer == 0 ? a.h1 : (layer == 1 ? a.h2 : a.h3);
            float *zg = layer == 0 ? a.z1 : (layer == 1 ? a.z2 : a.z3);
            f32x4 acc[NH / 16];
            if (layer == 0) layer_tiles<KIN, S1, S1, NH / 16>(buf, sW1, acc);
            else layer_tiles<NH, SH, SH, NH / 16>(buf, layer == 1 ? sW2 : sW3, acc);
            wave_sync();  // every lane's reads of the input tile are done
#pragma unroll
            for (int nt = 0; nt < NH / 16; nt++) {
                const int f0 = nt * 16 + lf;
                const f32x4 b = *(const f32x4 *)(sBias + layer * NH + f0);
                f32x4 z;
                __bf16 h[4];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    z[i] = acc[nt][i] + b[i];
                    h[i] = (__bf16)silu_fwd(z[i]);
                }
                typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
                const bf16x4 hv = {h[0], h[1], h[2], h[3]};
                *(bf16x4 *)(buf + lr * SH + f0) = hv;
                if (TRAIN && row_in) {
                    *(f32x4 *)(zg + (r0 + lr) * NH + f0) = z;
                    *(bf16x4 *)(hg + (r0 + lr) * NH + f0) = hv;
                }
            }
            wave_sync();
        }
        // output layer: W4 padded to 16 rows; output feature 0 of row l
        // (l < 16) is y
        f32x4 acc[1];
        layer_tiles<NH, SH, SH, 1>(buf, sW4, acc);
        if (l < 16 && row_in) a.y[r0 + l] = acc[0][0] + a.p[OFF_B4];
        wave_sync();
    }
}

// C[M][N] = A^T B with A [K][M] (row stride lda), B [K][N] (ldb); K a
// multiple of 32; one wavefront per 16 x 16 tile of C over the full K.
__global__ __launch_bounds__(256) void k_gemm_tn(const __bf16 *A, int lda, const __bf16 *B, int ldb,
                                                 float *C, int ldc, int M, int N, int K) {
    const int l = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tn = N / 16;
    if (tile >= (M / 16) * tn) return;
    const int m0 = (tile / tn) * 16, n0 = (tile % tn) * 16;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 fa, fb;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = k0 + 8 * (l >> 4) + j;
            fa[j] = A[(int64_t)k * lda + m0 + (l & 15)];
            fb[j] = B[(int64_t)k * ldb + n0 + (l & 15)];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; i++) C[(int64_t)(m0 + 4 * (l >> 4) + i) * ldc + n0 + (l & 15)] = acc[i];
}

// C[M][N] = A B with A [M][K] (lda), B [K][N] (ldb).
__global__ __launch_bounds__(256) void k_gemm_nn(const __bf16 *A, int lda, const __bf16 *B, int ldb,
                                                 float *C, int ldc, int M, int N, int K) {
    const int l = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tn = N / 16;
    if (tile >= (M / 16) * tn) return;
    const int m0 = (tile / tn) * 16, n0 = (tile % tn) * 16;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 fa = *(const bf16x8 *)(A + (int64_t)(m0 + (l & 15)) * lda + k0 + 8 * (l >> 4));
        bf16x8 fb;
#pragma unroll
        for (int j = 0; j < 8; j++) fb[j] = B[(int64_t)(k0 + 8 * (l >> 4) + j) * ldb + n0 + (l & 15)];
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; i++) C[(int64_t)(m0 + 4 * (l >> 4) + i) * ldc + n0 + (l & 15)] = acc[i];
}

// Output-layer gradient: g = 2/n (y - t) (binary32), gq its bfloat16, loss
// terms; rows beyond n (padding up to a multiple of 32) get zeros.
__global__ void k_out_grad(const float *y, const float *t, int64_t n, int64_t npad, float *g,
                           __bf16 *gq, float *sq) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= npad) return;
    float gv = 0.0f, s = 0.0f;
    if (r < n) {
        const float d = y[r] - t[r];
        gv = (2.0f / (float)n) * d;
        s = d * d;
    }
    g[r] = gv;
    gq[r] = (__bf16)gv;
    sq[r] = s;
}

// dZ3[r][c] = (gq[r] w4q[c]) silu'(z3[r][c]); dZ of lower layers from dH.
__global__ void k_dz_top(const __bf16 *gq, const __bf16 *w4, const float *z, int64_t n, int64_t npad,
                         float *dz, __bf16 *dzq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad * NH) return;
    const int64_t r = i / NH;
    const int c = (int)(i % NH);
    float v = 0.0f;
    if (r < n) v = ((float)gq[r] * (float)w4[c]) * dsilu(z[r * NH + c]);
    dz[i] = v;
    dzq[i] = (__bf16)v;
}

__global__ void k_dz(const float *dh, const float *z, int64_t n, int64_t npad, float *dz, __bf16 *dzq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad * NH) return;
    const int64_t r = i / NH;
    float v = 0.0f;
    if (r < n) v = dh[i] * dsilu(z[i]);
    dz[i] = v;
    dzq[i] = (__bf16)v;
}

// out[c] = sum over rows r < n of M[r][c] (row order), c < ncol, row stride ld.
__global__ void k_colsum(const float *M, int ld, int64_t n, int ncol, float *out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    float s = 0.0f;
    for (int64_t r = 0; r < n; r++) s = s + M[r * ld + c];
    out[c] = s;
}

// dW4[c] = sum_r gq[r] h3[r][c]; db4 = sum_r g[r]; loss = sum_r sq[r] / n.
__global__ void k_top_grads(const __bf16 *gq, const float *g, const __bf16 *h3, const float *sq,
                            int64_t n, float *grads, float *loss) {
    const int c = threadIdx.x;
    if (c < NH) {
        float s = 0.0f;
        for (int64_t r = 0; r < n; r++) s = s + (float)gq[r] * (float)h3[r * NH + c];
        grads[OFF_W4 + c] = s;
    } else if (c == NH) {
        float s = 0.0f;
        for (int64_t r = 0; r < n; r++) s = s + g[r];
        grads[OFF_B4] = s;
    } else if (c == NH + 1) {
        float s = 0.0f;
        for (int64_t r = 0; r < n; r++) s = s + sq[r];
        *loss = s / (float)n;
    }
}

// Copy a weight gradient block [rows][cols] out of a wider GEMM result.
__global__ void k_take(const float *src, int lds, int rows, int cols, float *dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    dst[i] = src[(i / cols) * lds + i % cols];
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int n, float lr, float c1,
                       float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + (1.0f - 0.9f) * gi;
    const float vi = 0.999f * v[i] + (1.0f - 0.999f) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] = p[i] - lr * mh / (sqrtf(vh) + 1e-8f);
}

// binary32 masters -> padded bfloat16 copies.
__global__ void k_pack(const float *p, Wbf w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NH * KIN) {
        const int r = i / KIN, k = i % KIN;
        w.w1[i] = (__bf16)(k < NIN ? p[OFF_W1 + r * NIN + k] : 0.0f);
    }
    if (i < NH * NH) {
        w.w2[i] = (__bf16)p[OFF_W2 + i];
        w.w3[i] = (__bf16)p[OFF_W3 + i];
    }
    if (i < 16 * NH) w.w4[i] = (__bf16)(i < NH ? p[OFF_W4 + i] : 0.0f);
}

// out[r] = 1 when some input of row r lies outside [lo, hi] (or is NaN).
__global__ void k_envelope(const float *X, int64_t n, const float *lo, const float *hi, uint8_t *out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    bool inside = true;
    for (int k = 0; k < NIN; k++) {
        const float x = X[r * NIN + k];
        inside = inside && x >= lo[k] && x <= hi[k];
    }
    out[r] = inside ? 0 : 1;
}

constexpr size_t AL = 256;
constexpr size_t al(size_t v) { return (v + AL - 1) / AL * AL; }

struct Lay {
    int64_t B;  // batch capacity, multiple of 32
    size_t p, m, v, g, w1, w2, w3, w4, h0, h1, h2, h3, z1, z2, z3, y, gout, gq, sq, dz, dzq, dh,
        tmp, loss, norm, total;
};

// masters: whether the binary32 parameters, their gradient and the Adam
// moments live here too (a context) or stay with the caller (a bare gradient
// evaluation).
constexpr Lay layout(int64_t max_batch, bool masters = true) {
    Lay L{};
    L.B = (max_batch + 31) / 32 * 32;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = al(o + b); return r; };
    const size_t mp = masters ? (size_t)NPAR * 4 : 0;
    L.p = take(mp); L.m = take(mp); L.v = take(mp); L.g = take(mp);
    L.w1 = take(NH * KIN * 2); L.w2 = take(NH * NH * 2); L.w3 = take(NH * NH * 2); L.w4 = take(16 * NH * 2);
    const size_t B = (size_t)L.B;
    L.h0 = take(B * KIN * 2); L.h1 = take(B * NH * 2); L.h2 = take(B * NH * 2); L.h3 = take(B * NH * 2);
    L.z1 = take(B * NH * 4); L.z2 = take(B * NH * 4); L.z3 = take(B * NH * 4);
    L.y = take(B * 4); L.gout = take(B * 4); L.gq = take(B * 2); L.sq = take(B * 4);
    L.dz = take(B * NH * 4); L.dzq = take(B * NH * 2); L.dh = take(B * NH * 4);
    L.tmp = take(NH * KIN * 4); L.loss = take(64);
    L.norm = masters ? take(4 * NIN * 4) : 0;
    L.total = o;
    return L;
}

}  // namespace

struct mlp_ctx {
    Lay L;
    char *ws;
    hipStream_t s;
    int t;
    Wbf w;
    bool have_norm;  // mlp_set_normaliser was called
};

namespace {
template <class T> T *P(mlp_ctx *c, size_t off) { return (T *)(c->ws + off); }

// Where one gradient evaluation reads its parameters and keeps its
// intermediates (activations, pre-activations, output and hidden-layer
// gradients, the padded first-layer weight gradient), and where it writes the
// gradient and the loss.
struct GradBufs {
    char *base;        // intermediates at the offsets of L
    Lay L;
    const float *p;    // binary32 parameters (biases are read from here)
    Wbf w;             // their bfloat16 copies
    float *g;          // gradient out [NPAR]
    float *loss;       // loss out (one value)
    hipStream_t s;
};
template <class T> T *Q(const GradBufs &b, size_t off) { return (T *)(b.base + off); }

GradBufs bufs_of(mlp_ctx *c) {
    return GradBufs{c->ws, c->L, P<float>(c, c->L.p), c->w, P<float>(c, c->L.g), P<float>(c, c->L.loss), c->s};
}

hipError_t pack_to(const float *p, Wbf w, hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3((NH * NH + 255) / 256), dim3(256), 0, s, p, w);
    return hipGetLastError();
}

hipError_t pack(mlp_ctx *c) { return pack_to(P<float>(c, c->L.p), c->w, c->s); }

hipError_t zero(mlp_ctx *c, size_t off, size_t bytes) {
    return lbimb::launch_fill_u32(P<uint32_t>(c, off), 0u, (int64_t)(bytes / 4), c->s);
}

// Forward (training mode) + backward: the gradient of the mean squared error
// into b.g, the loss into *b.loss.  Every intermediate a kernel reads is
// written earlier in the same evaluation (the padding rows up to a multiple of
// 32 are cleared here), so the buffers may hold anything on entry.
hipError_t grads(const GradBufs &b, const float *X, const float *y, int64_t n) {
    const Lay &L = b.L;
    const int64_t npad = (n + 31) / 32 * 32;
    hipError_t e;
    // padding rows of the activations must be zero for the K-reductions
    if (npad > n) {
        const size_t hoff[4] = {L.h0, L.h1, L.h2, L.h3};
        for (int k = 0; k < 4; k++) {
            const size_t row = k == 0 ? KIN * 2 : NH * 2;
            if ((e = lbimb::launch_fill_u32(Q<uint32_t>(b, hoff[k] + (size_t)n * row), 0u,
                                            (int64_t)((size_t)(npad - n) * row / 4), b.s)) != hipSuccess)
                return e;
        }
    }
    FwdArgs fa{};
    fa.X = X; fa.n = n; fa.p = b.p; fa.w = b.w; fa.y = Q<float>(b, L.y);
    fa.h0 = Q<__bf16>(b, L.h0); fa.h1 = Q<__bf16>(b, L.h1); fa.h2 = Q<__bf16>(b, L.h2);
    fa.h3 = Q<__bf16>(b, L.h3);
    fa.z1 = Q<float>(b, L.z1); fa.z2 = Q<float>(b, L.z2); fa.z3 = Q<float>(b, L.z3);
    const int64_t tiles = (n + 15) / 16;
    const unsigned blocks = (unsigned)std::min<int64_t>((tiles + FWD_WAVES_TRAIN - 1) / FWD_WAVES_TRAIN, 1024);
    hipLaunchKernelGGL(k_mlp_forward<true>, dim3(blocks), dim3(64 * FWD_WAVES_TRAIN), 0, b.s, fa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    float *g = b.g;
    hipLaunchKernelGGL(k_out_grad, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, b.s,
                       (const float *)Q<float>(b, L.y), y, n, npad, Q<float>(b, L.gout), Q<__bf16>(b, L.gq),
                       Q<float>(b, L.sq));
    hipLaunchKernelGGL(k_top_grads, dim3(1), dim3(192), 0, b.s, (const __bf16 *)Q<__bf16>(b, L.gq),
                       (const float *)Q<float>(b, L.gout), (const __bf16 *)Q<__bf16>(b, L.h3),
                       (const float *)Q<float>(b, L.sq), n, g, b.loss);
    const unsigned ew = (unsigned)((npad * NH + 255) / 256);
    hipLaunchKernelGGL(k_dz_top, dim3(ew), dim3(256), 0, b.s, (const __bf16 *)Q<__bf16>(b, L.gq),
                       (const __bf16 *)b.w.w4, (const float *)Q<float>(b, L.z3), n, npad,
                       Q<float>(b, L.dz), Q<__bf16>(b, L.dzq));
    // layers 3, 2, 1: dW = dZ^T H_prev, db = colsum dZ, dH_prev = dZ W
    const size_t hprev[3] = {L.h2, L.h1, L.h0};
    const size_t zprev[2] = {L.z2, L.z1};
    const __bf16 *wk[3] = {b.w.w3, b.w.w2, b.w.w1};
    const int offW[3] = {OFF_W3, OFF_W2, OFF_W1}, offB[3] = {OFF_B3, OFF_B2, OFF_B1};
    for (int k = 0; k < 3; k++) {
        const int nin = k == 2 ? KIN : NH;
        float *dst = k == 2 ? Q<float>(b, L.tmp) : g + offW[k];
        hipLaunchKernelGGL(k_gemm_tn, dim3((NH / 16) * (nin / 16) / 4), dim3(256), 0, b.s,
                           (const __bf16 *)Q<__bf16>(b, L.dzq), NH, (const __bf16 *)Q<__bf16>(b, hprev[k]), nin,
                           dst, nin, NH, nin, (int)npad);
        if (k == 2)
            hipLaunchKernelGGL(k_take, dim3((NH * NIN + 255) / 256), dim3(256), 0, b.s,
                               (const float *)Q<float>(b, L.tmp), KIN, NH, NIN, g + OFF_W1);
        hipLaunchKernelGGL(k_colsum, dim3(1), dim3(NH), 0, b.s, (const float *)Q<float>(b, L.dz), NH, n, NH,
                           g + offB[k]);
        if (k < 2) {
            hipLaunchKernelGGL(k_gemm_nn, dim3((unsigned)((npad / 16) * (NH / 16) / 4)), dim3(256), 0, b.s,
                               (const __bf16 *)Q<__bf16>(b, L.dzq), NH, wk[k], NH, Q<float>(b, L.dh), NH,
                               (int)npad, NH, NH);
            hipLaunchKernelGGL(k_dz, dim3(ew), dim3(256), 0, b.s, (const float *)Q<float>(b, L.dh),
                               (const float *)Q<float>(b, zprev[k]), n, npad, Q<float>(b, L.dz),
                               Q<__bf16>(b, L.dzq));
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------ allocation-free gradients
// The intermediates of mlp_gradients_noalloc: one fixed array per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a kernel
// (on the host that name is only a stand-in); it passes the device address
// that hipGetSymbolAddress returns for the current GPU, looked up once per
// device and kept in scratch_ptr.
constexpr Lay NOALLOC_LAY = layout(MLP_NOALLOC_MAX_ROWS, false);
static_assert(NOALLOC_LAY.total == MLP_NOALLOC_SCRATCH_BYTES, "scratch size in mlp_closure.h");
static __device__ __align__(256) char scratch[NOALLOC_LAY.total];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
char *scratch_ptr[MAX_DEVICES];

// Device address of this GPU's scratch array (looked up on the first call on
// each device, with that device current).
hipError_t scratch_for_current_device(char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr || (uintptr_t)ptr % AL) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = (char *)ptr;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

extern "C" {

int mlp_workspace_bytes(int64_t max_batch, size_t *bytes) {
    if (max_batch < 1 || !bytes) return LBM_E_INVALID;
    *bytes = layout(max_batch).total;
    return LBM_OK;
}

int mlp_create(int64_t max_batch, void *workspace, size_t ws_bytes, void *hip_stream, mlp_ctx **out) {
    if (!out || max_batch < 1) return LBM_E_INVALID;
    Lay L = layout(max_batch);
    if (!workspace || ws_bytes < L.total) return LBM_E_NOMEM;
    if ((uintptr_t)workspace % AL) return LBM_E_INVALID;
    mlp_ctx *c = new (std::nothrow) mlp_ctx();
    if (!c) return LBM_E_NOMEM;
    c->L = L;
    c->ws = (char *)workspace;
    c->s = (hipStream_t)hip_stream;
    c->t = 0;
    c->have_norm = false;
    c->w.w1 = P<__bf16>(c, L.w1);
    c->w.w2 = P<__bf16>(c, L.w2);
    c->w.w3 = P<__bf16>(c, L.w3);
    c->w.w4 = P<__bf16>(c, L.w4);
    if (zero(c, 0, L.total) != hipSuccess || hipStreamSynchronize(c->s) != hipSuccess) {
        delete c;
        return LBM_E_HIP;
    }
    *out = c;
    return LBM_OK;
}

void mlp_destroy(mlp_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    delete c;
}

int mlp_set_params(mlp_ctx *c, const float *params, int ptr_kind) {
    if (!c || !params) return LBM_E_INVALID;
    const hipMemcpyKind k = ptr_kind == LBM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(P<float>(c, c->L.p), params, NPAR * 4, k, c->s) != hipSuccess) return LBM_E_HIP;
    if (zero(c, c->L.m, NPAR * 4) != hipSuccess || zero(c, c->L.v, NPAR * 4) != hipSuccess) return LBM_E_HIP;
    c->t = 0;
    if (pack(c) != hipSuccess) return LBM_E_HIP;
    if (ptr_kind == LBM_HOST && hipStreamSynchronize(c->s) != hipSuccess) return LBM_E_HIP;
    return LBM_OK;
}

int mlp_get_params(mlp_ctx *c, float *params, int ptr_kind) {
    if (!c || !params) return LBM_E_INVALID;
    const hipMemcpyKind k = ptr_kind == LBM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(params, P<float>(c, c->L.p), NPAR * 4, k, c->s) != hipSuccess) return LBM_E_HIP;
    if (ptr_kind == LBM_HOST && hipStreamSynchronize(c->s) != hipSuccess) return LBM_E_HIP;
    return LBM_OK;
}

int mlp_forward(mlp_ctx *c, const float *X, int64_t n, float *y) {
    if (!c || !X || !y || n < 0) return LBM_E_INVALID;
    if (n == 0) return LBM_OK;
    FwdArgs fa{};
    fa.X = X; fa.n = n; fa.p = P<float>(c, c->L.p); fa.w = c->w; fa.y = y;
    const int64_t tiles = (n + 15) / 16;
    const unsigned blocks = (unsigned)std::min<int64_t>((tiles + FWD_WAVES - 1) / FWD_WAVES, 1024);
    hipLaunchKernelGGL(k_mlp_forward<false>, dim3(blocks), dim3(64 * FWD_WAVES), 0, c->s, fa);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int mlp_set_normaliser(mlp_ctx *c, const float *mu, const float *sd, const float *lo, const float *hi,
                       int ptr_kind) {
    if (!c || !mu || !sd || !lo || !hi || (ptr_kind != LBM_HOST && ptr_kind != LBM_DEVICE)) return LBM_E_INVALID;
    if (ptr_kind == LBM_HOST)
        for (int k = 0; k < NIN; k++)
            if (!(sd[k] > 0.0f) || !std::isfinite(sd[k]) || !std::isfinite(mu[k])) return LBM_E_INVALID;
    const hipMemcpyKind kind = ptr_kind == LBM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const float *src[4] = {mu, sd, lo, hi};
    for (int j = 0; j < 4; j++)
        if (hipMemcpyAsync(P<float>(c, c->L.norm) + j * NIN, src[j], NIN * 4, kind, c->s) != hipSuccess)
            return LBM_E_HIP;
    if (ptr_kind == LBM_HOST && hipStreamSynchronize(c->s) != hipSuccess) return LBM_E_HIP;
    c->have_norm = true;
    return LBM_OK;
}

int mlp_infer(mlp_ctx *c, const float *X, int64_t n, float *y, uint8_t *out_of_envelope) {
    if (!c || !X || !y || n < 0) return LBM_E_INVALID;
    if (!c->have_norm) return LBM_E_STATE;
    if (n == 0) return LBM_OK;
    const float *nb = P<float>(c, c->L.norm);
    FwdArgs fa{};
    fa.X = X; fa.nmu = nb; fa.nsd = nb + NIN; fa.n = n; fa.p = P<float>(c, c->L.p); fa.w = c->w; fa.y = y;
    const int64_t tiles = (n + 15) / 16;
    const unsigned blocks = (unsigned)std::min<int64_t>((tiles + FWD_WAVES - 1) / FWD_WAVES, 1024);
    hipLaunchKernelGGL(k_mlp_forward<false>, dim3(blocks), dim3(64 * FWD_WAVES), 0, c->s, fa);
    if (out_of_envelope)
        hipLaunchKernelGGL(k_envelope, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->s, X, n, nb + 2 * NIN,
                           nb + 3 * NIN, out_of_envelope);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int mlp_gradients(mlp_ctx *c, const float *X, const float *y, int64_t n, float *out_grads, float *loss,
                  int ptr_kind) {
    if (!c || !X || !y || n < 1 || n > c->L.B) return LBM_E_INVALID;
    if (grads(bufs_of(c), X, y, n) != hipSuccess) return LBM_E_HIP;
    const hipMemcpyKind k = ptr_kind == LBM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (out_grads && hipMemcpyAsync(out_grads, P<float>(c, c->L.g), NPAR * 4, k, c->s) != hipSuccess) return LBM_E_HIP;
    if (loss && hipMemcpyAsync(loss, P<float>(c, c->L.loss), 4, k, c->s) != hipSuccess) return LBM_E_HIP;
    if (ptr_kind == LBM_HOST && hipStreamSynchronize(c->s) != hipSuccess) return LBM_E_HIP;
    return LBM_OK;
}

int mlp_train_step(mlp_ctx *c, const float *X, const float *y, int64_t n, float lr, float *loss) {
    if (!c || !X || !y || n < 1 || n > c->L.B) return LBM_E_INVALID;
    if (grads(bufs_of(c), X, y, n) != hipSuccess) return LBM_E_HIP;
    c->t += 1;
    const float c1 = 1.0f - powf(0.9f, (float)c->t), c2 = 1.0f - powf(0.999f, (float)c->t);
    hipLaunchKernelGGL(k_adam, dim3((NPAR + 255) / 256), dim3(256), 0, c->s, P<float>(c, c->L.p),
                       (const float *)P<float>(c, c->L.g), P<float>(c, c->L.m), P<float>(c, c->L.v), NPAR, lr, c1, c2);
    if (hipGetLastError() != hipSuccess || pack(c) != hipSuccess) return LBM_E_HIP;
    if (loss) {
        if (hipMemcpyAsync(loss, P<float>(c, c->L.loss), 4, hipMemcpyDeviceToHost, c->s) != hipSuccess) return LBM_E_HIP;
        if (hipStreamSynchronize(c->s) != hipSuccess) return LBM_E_HIP;
    }
    return LBM_OK;
}

int mlp_gradients_noalloc(const float *params, const float *X, const float *y, int64_t n, float *grads_out,
                          float *loss, void *hip_stream) {
    if (!params || !X || !y || !grads_out) return LBM_E_INVALID;
    if (n < 1 || n > MLP_NOALLOC_MAX_ROWS) return LBM_E_INVALID;
    char *base = nullptr;
    if (scratch_for_current_device(&base) != hipSuccess) return LBM_E_HIP;
    const Lay &L = NOALLOC_LAY;
    const hipStream_t s = (hipStream_t)hip_stream;
    GradBufs b{base, L, params,
               Wbf{(__bf16 *)(base + L.w1), (__bf16 *)(base + L.w2), (__bf16 *)(base + L.w3),
                   (__bf16 *)(base + L.w4)},
               grads_out, loss ? loss : (float *)(base + L.loss), s};
    if (pack_to(params, b.w, s) != hipSuccess) return LBM_E_HIP;
    if (grads(b, X, y, n) != hipSuccess) return LBM_E_HIP;
    return LBM_OK;
}

}  // extern "C"
