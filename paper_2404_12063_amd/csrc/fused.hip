// Fused single-launch FastVPINNs loss and gradient (Algorithm 3 and its backward
// pass) on gfx950.
//
// One launch computes, for all quadrature, boundary and sensor points: network
// values and spatial tangents, the contraction R = eps sum_q (u_x G_x + u_y G_y)
// - F, the loss, the adjoint of the contraction, the reverse sweep through the
// network, and the fixed-order reduction of every partial sum into the loss
// and gradient outputs.
//
// Work decomposition.  A work item is a contiguous range of elements plus a
// slice of the boundary/sensor points; 256-thread blocks (4 wavefronts, two
// blocks per CU) take items round-robin.  Per item:
//   1. forward (values + tangents) for all points of the item, tiles of 16
//      points spread over the wavefronts; u_x, u_y (or u) go to LDS;
//   2. contraction, thread per point over chunks of whole elements: every G
//      load of the chunk is in flight before the first use; the per-point
//      terms go through LDS to per-(element, test) row sums; 2 c_v R kept in
//      LDS; loss partials;
//   3. dL/du_x[q] = eps sum_k 2 c_v R[e,k] G_x[e,k,q] (and y) from the G values
//      still in registers (a generic path reloads them for large elements);
//   4. backward per tile: the forward pass is recomputed (tanh included) and
//      the activations kept in registers for the reverse sweep.
// The block's gradient accumulators live in registers across items.  At the
// end every block writes one partial row; a second small kernel sums the rows
// in block order and writes the outputs (no float atomics: bitwise
// reproducible; the kernel boundary orders the partial writes before the
// reads, which costs far less than a device-scope fence per block).
//
// Register layout of a 32-neuron vector over a 16-point tile ("chained"):
// lane l holds point j = l % 16 and neurons 16 m + 4 g + r (g = l / 16,
// m = 0..1, r = 0..3) in v[m][r].  This is exactly the output layout of
// V_MFMA_F32_16X16X4F32 for two 16-row tiles, and also the B-operand layout of
// the next product when its K index is walked as (m, r) with K-slot g, so every
// hidden-to-hidden product (forward, and backward with W transposed) chains
// from registers to registers.  Only the weight-gradient products, which
// contract over points, need the vectors transposed; that goes through a small
// per-wavefront LDS tile.
#include <cstdint>

#include "device_common.h"
#include "internal.h"

namespace vp {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kFThreads = 256;
constexpr int kFBlocksPerCU = 2;   // two co-resident blocks: one's contraction latency hides under the other's MFMAs
constexpr int kFWaves = kFThreads / 64;
constexpr int kTs = 36;            // transpose tile row stride (floats)
constexpr int kMaxBlocks = 1024;
constexpr int kKB = 32;            // test functions held in registers by the fast contraction
constexpr int kCbs = kFThreads + 1;  // row stride of the per-point term buffer

struct Vec {
    f4 v[2];
};

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int L>
struct FusedShared {
    // A-operand fragments of the hidden-to-hidden products, layers 2..L:
    // [layer][dir 0 = W (forward), 1 = W^T (backward)][out tile][k step][lane]
    float wf[L > 1 ? L - 1 : 1][2][2][8][64];
    float w1[PW][2];
    float b[L][PW];
    float wo[PW];
    float bo;
    // per-wavefront transpose tiles [2][16 points][kTs]
    float tt[kFWaves][2][16][kTs];
    // per-wavefront loss partials: sum R^2, sum R A, sum d_b^2, sum d_s^2
    double lp[kFWaves][4];
};

struct FusedArgs {
    const float *params;  // flat layout, width H
    int H;
    const float *Gx, *Gy, *F;
    const float2 *pts;    // interior points then boundary then sensors
    const float *tgt;     // boundary values then sensor observations
    const float *eps_ptr;
    int64_t n_elem, n_pts, n_bnd, n_sen;
    int nq, ntest;
    int64_t n_items;
    float two_cv, wb2, ws2;  // 2 c_v, 2 tau / N_D, 2 gamma / N_s
    double cv;
    float tau, gamma;
    int want_grad;
    int64_t n_params_flat;
    int item_cap_pts;        // LDS capacity for item points
    int fast_contract;       // nq <= kFThreads and ntest <= kKB: G stays in registers
    float *gpart;            // [blocks][kMaxPadded]
    double *lpart;           // [blocks][4]
};

// element and extra-point ranges of item i (even split, no work list needed)
__device__ __forceinline__ void item_range(const FusedArgs &A, int64_t i, int64_t &e0, int64_t &e1, int64_t &x0,
                                           int64_t &x1) {
    const int64_t nx = A.n_bnd + A.n_sen;
    e0 = i * A.n_elem / A.n_items;
    e1 = (i + 1) * A.n_elem / A.n_items;
    x0 = i * nx / A.n_items;
    x1 = (i + 1) * nx / A.n_items;
}

// ---------------------------------------------------------------------------
// forward through the network for one tile.  If `keep` is non-null the
// activations a_l and pre-activation tangents p_l (l >= 2) are stored there
// (layer 1 keeps a_1 only; its tangent is s_1 times a weight column).
// ---------------------------------------------------------------------------
template <int L>
struct Acts {
    Vec a[L];
    Vec px[L];  // px[0], py[0] unused (layer 1)
    Vec py[L];
};

template <int L, bool KEEP>
__device__ __forceinline__ void tile_forward(const FusedShared<L> &S, int lane, float x, float y, Vec &A_, Vec &TX,
                                             Vec &TY, Acts<L> &keep) {
    const int g = lane >> 4;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * m + 4 * g + r;
            const float w0 = S.w1[n][0], w1v = S.w1[n][1];
            const float a = tanh_f32(fmaf(w0, x, fmaf(w1v, y, S.b[0][n])));
            const float s = 1.0f - a * a;
            A_.v[m][r] = a;
            TX.v[m][r] = s * w0;
            TY.v[m][r] = s * w1v;
        }
    if (KEEP) keep.a[0] = A_;
#pragma unroll
    for (int l = 2; l <= L; ++l) {
        Vec Z, PX, PY;
#pragma unroll
        for (int mo = 0; mo < 2; ++mo) {
            f4 z, px = {0.f, 0.f, 0.f, 0.f}, py = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) z[r] = S.b[l - 1][16 * mo + 4 * g + r];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const float w = S.wf[l - 2][0][mo][s][lane];
                z = mfma(w, A_.v[s >> 2][s & 3], z);
                px = mfma(w, TX.v[s >> 2][s & 3], px);
                py = mfma(w, TY.v[s >> 2][s & 3], py);
            }
            Z.v[mo] = z;
            PX.v[mo] = px;
            PY.v[mo] = py;
        }
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float a = tanh_f32(Z.v[m][r]);
                const float s = 1.0f - a * a;
                A_.v[m][r] = a;
                TX.v[m][r] = s * PX.v[m][r];
                TY.v[m][r] = s * PY.v[m][r];
            }
        if (KEEP) {
            keep.a[l - 1] = A_;
            keep.px[l - 1] = PX;
            keep.py[l - 1] = PY;
        }
    }
}

// sum over the four K-slot groups (lanes j, j+16, j+32, j+48)
__device__ __forceinline__ float group_sum(float v) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

template <int L>
__device__ __forceinline__ void tile_outputs(const FusedShared<L> &S, int lane, const Vec &A_, const Vec &TX,
                                             const Vec &TY, float &u, float &ux, float &uy) {
    const int g = lane >> 4;
    float su = 0.f, sx = 0.f, sy = 0.f;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float w = S.wo[16 * m + 4 * g + r];
            su = fmaf(w, A_.v[m][r], su);
            sx = fmaf(w, TX.v[m][r], sx);
            sy = fmaf(w, TY.v[m][r], sy);
        }
    u = group_sum(su) + S.bo;
    ux = group_sum(sx);
    uy = group_sum(sy);
}

// write a chained vector transposed into tile T[j][n]
__device__ __forceinline__ void put_t(float (*T)[kTs], int lane, const Vec &V) {
    const int j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int m = 0; m < 2; ++m) *reinterpret_cast<f4 *>(&T[j][16 * m + 4 * g]) = V.v[m];
}

// acc += sum over this lane's 8 points of column (lane % 32) of T
__device__ __forceinline__ float col_sum(float (*T)[kTs], int lane) {
    const int n = lane & 31, j0 = (lane >> 5) * 8;
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += T[j0 + j][n];
    return s;
}

// weight gradient dW[o][i] += sum_points Zo[o] * Ai[i] via the transpose tiles;
// acc[mo * 2 + mi] holds the 16x16 tile (rows 16 mo + 4 g + r, column 16 mi + lane % 16)
__device__ __forceinline__ void wgrad(float (*T0)[kTs], float (*T1)[kTs], int lane, const Vec &Zo, const Vec &Ai,
                                      f4 acc[4], float *bias_acc) {
    put_t(T0, lane, Zo);
    put_t(T1, lane, Ai);
    wave_sync();
    const int c = lane & 15, k = lane >> 4;
#pragma unroll
    for (int kp = 0; kp < 4; ++kp) {
        const float a0 = T0[4 * kp + k][c], a1 = T0[4 * kp + k][16 + c];
        const float b0 = T1[4 * kp + k][c], b1 = T1[4 * kp + k][16 + c];
        acc[0] = mfma(a0, b0, acc[0]);
        acc[1] = mfma(a0, b1, acc[1]);
        acc[2] = mfma(a1, b0, acc[2]);
        acc[3] = mfma(a1, b1, acc[3]);
    }
    if (bias_acc) *bias_acc += col_sum(T0, lane);
    wave_sync();
}

__device__ __forceinline__ float colsum_vec(float (*T0)[kTs], int lane, const Vec &V) {
    put_t(T0, lane, V);
    wave_sync();
    const float s = col_sum(T0, lane);
    wave_sync();
    return s;
}

// gradient accumulators of one wavefront
template <int L>
struct GradAcc {
    f4 w[L > 1 ? L - 1 : 1][4];  // hidden-to-hidden weight tiles, layers 2..L
    float b[L];                   // bias columns (lane % 32), per half-wave
    float w1c0, w1c1;             // W1 columns
    float wo;                     // W_out column
    float bo;                     // b_out (lanes with g == 0)
};

template <int L>
__device__ __forceinline__ void tile_backward(const FusedShared<L> &S, float (*T0)[kTs], float (*T1)[kTs], int lane,
                                              float x, float y, float ub, float uxb, float uyb, const Acts<L> &K,
                                              GradAcc<L> &G) {
    const int g = lane >> 4;
    Vec abar, txbar, tybar;
    {
        // output layer: dW_out = sum_p ub a_L + uxb t_L^x + uyb t_L^y
        const Vec &aL = K.a[L - 1];
        Vec v;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * m + 4 * g + r;
                float tx, ty;
                const float s = 1.0f - aL.v[m][r] * aL.v[m][r];
                if (L == 1) {
                    tx = s * S.w1[n][0];
                    ty = s * S.w1[n][1];
                } else {
                    tx = s * K.px[L - 1].v[m][r];
                    ty = s * K.py[L - 1].v[m][r];
                }
                v.v[m][r] = ub * aL.v[m][r] + uxb * tx + uyb * ty;
                const float w = S.wo[n];
                abar.v[m][r] = ub * w;
                txbar.v[m][r] = uxb * w;
                tybar.v[m][r] = uyb * w;
            }
        G.wo += colsum_vec(T0, lane, v);
        if (g == 0) G.bo += ub;
    }
#pragma unroll
    for (int l = L; l >= 2; --l) {
        Vec zb, pxb, pyb;
        const Vec &al = K.a[l - 1];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float a = al.v[m][r];
                const float s = 1.0f - a * a;
                pxb.v[m][r] = s * txbar.v[m][r];
                pyb.v[m][r] = s * tybar.v[m][r];
                const float sbar = txbar.v[m][r] * K.px[l - 1].v[m][r] + tybar.v[m][r] * K.py[l - 1].v[m][r];
                zb.v[m][r] = s * (abar.v[m][r] - 2.0f * a * sbar);
            }
        // inputs of layer l: a_{l-1} and t_{l-1} = s_{l-1} p_{l-1} (layer 1: s_1 times W1 column)
        Vec ai, ti_x, ti_y;
        const Vec &ap = K.a[l - 2];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float a = ap.v[m][r];
                const float s = 1.0f - a * a;
                ai.v[m][r] = a;
                if (l - 1 == 1) {
                    const int n = 16 * m + 4 * g + r;
                    ti_x.v[m][r] = s * S.w1[n][0];
                    ti_y.v[m][r] = s * S.w1[n][1];
                } else {
                    ti_x.v[m][r] = s * K.px[l - 2].v[m][r];
                    ti_y.v[m][r] = s * K.py[l - 2].v[m][r];
                }
            }
        wgrad(T0, T1, lane, zb, ai, G.w[l - 2], &G.b[l - 1]);
        wgrad(T0, T1, lane, pxb, ti_x, G.w[l - 2], nullptr);
        wgrad(T0, T1, lane, pyb, ti_y, G.w[l - 2], nullptr);
        // propagate: abar = W_l^T zbar, tbar = W_l^T pbar
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
            f4 sa = {0.f, 0.f, 0.f, 0.f}, sx = {0.f, 0.f, 0.f, 0.f}, sy = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const float w = S.wf[l - 2][1][mi][s][lane];
                sa = mfma(w, zb.v[s >> 2][s & 3], sa);
                sx = mfma(w, pxb.v[s >> 2][s & 3], sx);
                sy = mfma(w, pyb.v[s >> 2][s & 3], sy);
            }
            abar.v[mi] = sa;
            txbar.v[mi] = sx;
            tybar.v[mi] = sy;
        }
    }
    // layer 1: t_1 = s_1 W1[:, c], z_1 = W1 (x, y) + b_1
    {
        Vec zb, c0, c1;
        const Vec &a1 = K.a[0];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * m + 4 * g + r;
                const float a = a1.v[m][r];
                const float s = 1.0f - a * a;
                const float w0 = S.w1[n][0], w1v = S.w1[n][1];
                const float pxb = s * txbar.v[m][r], pyb = s * tybar.v[m][r];
                const float sbar = txbar.v[m][r] * w0 + tybar.v[m][r] * w1v;
                const float z = s * (abar.v[m][r] - 2.0f * a * sbar);
                zb.v[m][r] = z;
                c0.v[m][r] = fmaf(z, x, pxb);
                c1.v[m][r] = fmaf(z, y, pyb);
            }
        G.w1c0 += colsum_vec(T0, lane, c0);
        G.w1c1 += colsum_vec(T0, lane, c1);
        G.b[0] += colsum_vec(T0, lane, zb);
    }
}

// ---------------------------------------------------------------------------
// the fused kernel
// ---------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(kFThreads, kFBlocksPerCU) void k_fused(FusedArgs A) {
    __shared__ FusedShared<L> S;
    extern __shared__ float dyn[];  // item data: float2 per item point, then 2 c_v R per (element, test)
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int H = A.H;

    // weights -> LDS (padded to 32, fragment order for the MFMA A operands)
    for (int t = tid; t < PW * 2; t += kFThreads) {
        const int o = t >> 1, i = t & 1;
        S.w1[o][i] = o < H ? A.params[o * 2 + i] : 0.f;
    }
    for (int t = tid; t < L * PW; t += kFThreads) {
        const int l = t / PW + 1, o = t % PW;
        const int64_t off = (l == 1) ? 2 * H : hoff_w(H, l) + (int64_t)H * H;
        S.b[l - 1][o] = o < H ? A.params[off + o] : 0.f;
    }
    for (int t = tid; t < PW; t += kFThreads) S.wo[t] = t < H ? A.params[hoff_w(H, L + 1) + t] : 0.f;
    if (tid == 0) S.bo = A.params[hoff_w(H, L + 1) + H];
    for (int t = tid; t < (L - 1) * 2 * 2 * 8 * 64; t += kFThreads) {
        const int ln = t & 63, s = (t >> 6) & 7, mt = (t >> 9) & 1, dir = (t >> 10) & 1, l = 2 + (t >> 11);
        const int m = s >> 2, r = s & 3;
        // forward: W[16 mt + ln % 16][16 m + 4 (ln / 16) + r]; backward: W[16 m + 4 (ln / 16) + r][16 mt + ln % 16]
        const int o = dir == 0 ? 16 * mt + (ln & 15) : 16 * m + 4 * (ln >> 4) + r;
        const int i = dir == 0 ? 16 * m + 4 * (ln >> 4) + r : 16 * mt + (ln & 15);
        S.wf[l - 2][dir][mt][s][ln] = (o < H && i < H) ? A.params[hoff_w(H, l) + (int64_t)o * H + i] : 0.f;
    }
    __syncthreads();

    const float eps = A.eps_ptr ? *A.eps_ptr : 1.0f;
    float2 *uxy = reinterpret_cast<float2 *>(dyn);
    float *rbar = dyn + 2 * A.item_cap_pts;
    float(*T0)[kTs] = S.tt[wave][0];
    float(*T1)[kTs] = S.tt[wave][1];

    GradAcc<L> G;
#pragma unroll
    for (int l = 0; l < (L > 1 ? L - 1 : 1); ++l)
#pragma unroll
        for (int t = 0; t < 4; ++t) G.w[l][t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int l = 0; l < L; ++l) G.b[l] = 0.f;
    G.w1c0 = G.w1c1 = G.wo = G.bo = 0.f;
    double lrr = 0.0, lra = 0.0, lbb = 0.0, lss = 0.0;  // per-thread loss partials

    for (int64_t item = blockIdx.x; item < A.n_items; item += gridDim.x) {
        int64_t e0, e1, x0, x1;
        item_range(A, item, e0, e1, x0, x1);
        const int ne = (int)(e1 - e0);
        const int n_int = ne * A.nq;                 // interior points of the item
        const int n_all = n_int + (int)(x1 - x0);     // plus boundary/sensor points
        const int n_tiles = (n_all + 15) >> 4;
        auto point_xy = [&](int idx) -> float2 {
            if (idx < n_int) return A.pts[e0 * A.nq + idx];
            return A.pts[A.n_pts + x0 + (idx - n_int)];
        };

        // tiles go to wavefronts starting at a block-dependent offset, so the two
        // blocks sharing a CU put their ragged extra tiles on different SIMDs
        const int wrot = (wave + (int)(blockIdx.x + item) % kFWaves) % kFWaves;
        // 1. forward
        for (int t = wrot; t < n_tiles; t += kFWaves) {
            const int idx = 16 * t + (lane & 15);
            const bool valid = idx < n_all;
            const float2 p = valid ? point_xy(idx) : make_float2(0.f, 0.f);
            Vec a, tx, ty;
            Acts<L> unused;
            tile_forward<L, false>(S, lane, p.x, p.y, a, tx, ty, unused);
            float u, ux, uy;
            tile_outputs<L>(S, lane, a, tx, ty, u, ux, uy);
            if (valid && lane < 16) uxy[idx] = idx < n_int ? make_float2(ux, uy) : make_float2(u, 0.f);
        }
        __syncthreads();

        if (A.fast_contract) {
            // 2+3. chunks of whole elements, thread (element, q); G of all tests in registers
            float *cbuf = rbar + ne * A.ntest;  // [kKB][kCbs] per-point terms
            const int epc = kFThreads / A.nq;
            for (int c0 = 0; c0 < ne; c0 += epc) {
                const int ce = min(epc, ne - c0);
                const int el = c0 + tid / A.nq, q = tid - (tid / A.nq) * A.nq;
                const bool act = tid < ce * A.nq;
                const int64_t gbase = ((e0 + el) * A.ntest) * (int64_t)A.nq + q;
                float gx[kKB], gy[kKB];
#pragma unroll
                for (int k = 0; k < kKB; ++k) {
                    const bool ok = act && k < A.ntest;
                    gx[k] = ok ? A.Gx[gbase + (int64_t)k * A.nq] : 0.f;
                    gy[k] = ok ? A.Gy[gbase + (int64_t)k * A.nq] : 0.f;
                }
                const float2 d = act ? uxy[el * A.nq + q] : make_float2(0.f, 0.f);
#pragma unroll
                for (int k = 0; k < kKB; ++k)
                    if (k < A.ntest) cbuf[k * kCbs + tid] = fmaf(d.x, gx[k], d.y * gy[k]);
                __syncthreads();
                // row sums, 8 lanes per (element, test) row
                for (int r8 = tid; r8 < 8 * ce * A.ntest; r8 += kFThreads) {
                    const int r = r8 >> 3, part = r8 & 7;
                    const int e2 = r / A.ntest, k = r - e2 * A.ntest;
                    const float *row = cbuf + k * kCbs + e2 * A.nq;
                    float a = 0.f;
                    for (int qq = part; qq < A.nq; qq += 8) a += row[qq];
                    a += __shfl_xor(a, 4, 8);
                    a += __shfl_xor(a, 2, 8);
                    a += __shfl_xor(a, 1, 8);
                    if (part == 0) {
                        const float R = eps * a - A.F[(e0 + c0 + e2) * A.ntest + k];
                        rbar[(c0 + e2) * A.ntest + k] = A.two_cv * R;
                        lrr += (double)R * (double)R;
                        lra += (double)R * (double)a;
                    }
                }
                __syncthreads();
                if (A.want_grad && act) {
                    // reload G (cache hits) rather than keep 2 kKB registers live across the barrier
                    const float *rb = rbar + el * A.ntest;
#pragma unroll
                    for (int k = 0; k < kKB; ++k) {
                        const bool ok = k < A.ntest;
                        gx[k] = ok ? A.Gx[gbase + (int64_t)k * A.nq] : 0.f;
                        gy[k] = ok ? A.Gy[gbase + (int64_t)k * A.nq] : 0.f;
                    }
                    float bx = 0.f, by = 0.f;
#pragma unroll
                    for (int k = 0; k < kKB; ++k)
                        if (k < A.ntest) {
                            bx = fmaf(rb[k], gx[k], bx);
                            by = fmaf(rb[k], gy[k], by);
                        }
                    uxy[el * A.nq + q] = make_float2(eps * bx, eps * by);
                }
            }
        } else {
        // 2. contraction: rows (element, test function), 16 lanes per row, two rows per
            //    batch, every load of a batch in flight before the first use
            {
                constexpr int kRG = kFThreads / 16;
                const int rg = tid >> 4, rl = tid & 15;
                const int n_rows = ne * A.ntest;
                for (int r0 = 0; r0 < n_rows; r0 += 2 * kRG) {
                    float acc[2] = {0.f, 0.f}, fv[2];
                    int row[2];
                    int64_t base[2];
                    int el[2];
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        row[i] = r0 + rg + i * kRG;
                        el[i] = row[i] / A.ntest;
                        const int k = row[i] - el[i] * A.ntest;
                        base[i] = ((e0 + el[i]) * A.ntest + k) * (int64_t)A.nq;
                        fv[i] = row[i] < n_rows ? A.F[(e0 + el[i]) * A.ntest + k] : 0.f;
                    }
                    for (int qc = 0; qc < A.nq; qc += 128) {
                        float gx[2][8], gy[2][8];
#pragma unroll
                        for (int i = 0; i < 2; ++i)
#pragma unroll
                            for (int t = 0; t < 8; ++t) {
                                const int q = qc + rl + 16 * t;
                                const bool ok = row[i] < n_rows && q < A.nq;
                                gx[i][t] = ok ? A.Gx[base[i] + q] : 0.f;
                                gy[i][t] = ok ? A.Gy[base[i] + q] : 0.f;
                            }
#pragma unroll
                        for (int i = 0; i < 2; ++i)
#pragma unroll
                            for (int t = 0; t < 8; ++t) {
                                const int q = qc + rl + 16 * t;
                                if (row[i] < n_rows && q < A.nq) {
                                    const float2 d = uxy[el[i] * A.nq + q];
                                    acc[i] = fmaf(d.x, gx[i][t], fmaf(d.y, gy[i][t], acc[i]));
                                }
                            }
                    }
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        float a = acc[i];
                        a += __shfl_xor(a, 8, 16);
                        a += __shfl_xor(a, 4, 16);
                        a += __shfl_xor(a, 2, 16);
                        a += __shfl_xor(a, 1, 16);
                        if (rl == 0 && row[i] < n_rows) {
                            const float R = eps * a - fv[i];
                            rbar[row[i]] = A.two_cv * R;
                            lrr += (double)R * (double)R;
                            lra += (double)R * (double)a;
                        }
                    }
                }
            }
        }
        for (int idx = n_int + tid; idx < n_all; idx += kFThreads) {
            const int64_t xi = x0 + (idx - n_int);
            const float d = uxy[idx].x - A.tgt[xi];
            const bool bnd = xi < A.n_bnd;
            if (bnd) lbb += (double)d * (double)d;
            else lss += (double)d * (double)d;
            uxy[idx] = make_float2((bnd ? A.wb2 : A.ws2) * d, 0.f);
        }
        __syncthreads();
        if (!A.want_grad) {
            __syncthreads();
            continue;
        }

        // 3. adjoint of the contraction (generic path), thread per point, 16 tests per batch
        for (int idx = tid; idx < (A.fast_contract ? 0 : n_int); idx += kFThreads) {
            const int el = idx / A.nq, q = idx - el * A.nq;
            const int64_t e = e0 + el;
            const float *rb = rbar + el * A.ntest;
            float bx = 0.f, by = 0.f;
            for (int k0 = 0; k0 < A.ntest; k0 += 16) {
                float gx[16], gy[16];
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const int k = k0 + t;
                    const int64_t o = (e * A.ntest + k) * (int64_t)A.nq + q;
                    gx[t] = k < A.ntest ? A.Gx[o] : 0.f;
                    gy[t] = k < A.ntest ? A.Gy[o] : 0.f;
                }
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const float r = (k0 + t < A.ntest) ? rb[k0 + t] : 0.f;
                    bx = fmaf(r, gx[t], bx);
                    by = fmaf(r, gy[t], by);
                }
            }
            uxy[idx] = make_float2(eps * bx, eps * by);
        }
        __syncthreads();

        // 4. backward with recompute
        for (int t = wrot; t < n_tiles; t += kFWaves) {
            const int idx = 16 * t + (lane & 15);
            const bool valid = idx < n_all;
            const float2 p = valid ? point_xy(idx) : make_float2(0.f, 0.f);
            float ub = 0.f, uxb = 0.f, uyb = 0.f;
            if (valid) {
                const float2 d = uxy[idx];
                if (idx < n_int) {
                    uxb = d.x;
                    uyb = d.y;
                } else {
                    ub = d.x;
                }
            }
            Acts<L> K;
            Vec a, tx, ty;
            tile_forward<L, true>(S, lane, p.x, p.y, a, tx, ty, K);
            tile_backward<L>(S, T0, T1, lane, p.x, p.y, ub, uxb, uyb, K, G);
        }
        __syncthreads();
    }

    // ---- block partial: loss terms (double) and the padded gradient row ----
    {
        double v0 = wave_sum(lrr), v1 = wave_sum(lra), v2 = wave_sum(lbb), v3 = wave_sum(lss);
        if (lane == 0) {
            S.lp[wave][0] = v0;
            S.lp[wave][1] = v1;
            S.lp[wave][2] = v2;
            S.lp[wave][3] = v3;
        }
    }
    float *red = dyn;  // n_padded(L) floats (dynamic LDS is at least this large)
    const int g = lane >> 4, c = lane & 15;
    // this lane's (padded index, value) pairs; waves add them in wave order
    constexpr int NW = 16 * (L - 1), NV = NW + L + 4;
    int pidx[NV];
    float pval[NV];
    {
        int n = 0;
#pragma unroll
        for (int l = 2; l <= L; ++l)
#pragma unroll
            for (int mo = 0; mo < 2; ++mo)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        pidx[n] = off_w(l) + (16 * mo + 4 * g + r) * PW + 16 * mi + c;
                        pval[n++] = G.w[l - 2][mo * 2 + mi][r];
                    }
        const bool lo = lane < 32;
#pragma unroll
        for (int l = 1; l <= L; ++l) {
            pidx[n] = lo ? off_b(l) + lane : -1;
            pval[n++] = G.b[l - 1] + __shfl_xor(G.b[l - 1], 32, 64);
        }
        pidx[n] = lo ? off_w(1) + 2 * lane : -1;
        pval[n++] = G.w1c0 + __shfl_xor(G.w1c0, 32, 64);
        pidx[n] = lo ? off_w(1) + 2 * lane + 1 : -1;
        pval[n++] = G.w1c1 + __shfl_xor(G.w1c1, 32, 64);
        pidx[n] = lo ? off_wout(L) + lane : -1;
        pval[n++] = G.wo + __shfl_xor(G.wo, 32, 64);
        const float bo = wave_sum(G.bo);
        pidx[n] = lane == 0 ? off_wout(L) + PW : -1;
        pval[n++] = bo;
    }
    for (int w = 0; w < kFWaves; ++w) {
        if (wave == w && A.want_grad) {
            float cur[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) cur[i] = (w > 0 && pidx[i] >= 0) ? red[pidx[i]] : 0.f;
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (pidx[i] >= 0) red[pidx[i]] = cur[i] + pval[i];
        }
        __syncthreads();
    }
    const int NP = n_padded(L);
    if (A.want_grad)
        for (int j = tid; j < NP; j += kFThreads) A.gpart[(int64_t)blockIdx.x * kMaxPadded + j] = red[j];
    if (tid < 4) {
        double s = 0.0;
        for (int w = 0; w < kFWaves; ++w) s += S.lp[w][tid];
        A.lpart[blockIdx.x * 4 + tid] = s;
    }
}

// ---------------------------------------------------------------------------
// fixed-order reduction of the block partials into the outputs
// ---------------------------------------------------------------------------
// block = 32 columns x 32 row slices; slice t sums rows t, t+32, ... in order,
// then the 32 slice sums of a column are added in slice order (fixed order
// for any launch).  Loss partials are summed by block 0 the same way.
constexpr int kFinCols = 32, kFinSlices = 32;
template <int L>
__global__ __launch_bounds__(kFinCols *kFinSlices) void k_fused_final(
    const float *__restrict__ gpart, const double *__restrict__ lpart, int rows, int H, int64_t npf, double cv,
    int64_t n_bnd, int64_t n_sen, float tau, float gamma, float *__restrict__ loss_out, float *__restrict__ grad_out,
    float *__restrict__ grad_eps_out) {
    __shared__ float part[kFinSlices][kFinCols + 1];
    __shared__ double lred[kFinSlices][4];
    const int c = threadIdx.x % kFinCols, t = threadIdx.x / kFinCols;
    const int64_t j = (int64_t)blockIdx.x * kFinCols + c;
    int pj = -1;  // padded index of flat parameter j
    if (grad_out && j < npf) {
        if (j < 2 * H) pj = (int)j;
        else if (j < 3 * H) pj = kOffB1 + (int)(j - 2 * H);
        else {
            const int64_t lay = (int64_t)H * H + H, r0 = j - 3 * H;
            if (r0 < (int64_t)(L - 1) * lay) {
                const int l = 2 + (int)(r0 / lay), r = (int)(r0 % lay);
                pj = r < H * H ? off_w(l) + (r / H) * PW + (r % H) : off_b(l) + (r - H * H);
            } else {
                const int r = (int)(r0 - (int64_t)(L - 1) * lay);
                pj = r < H ? off_wout(L) + r : off_wout(L) + PW;
            }
        }
    }
    float acc = 0.f;
    if (pj >= 0) {
        for (int b0 = t; b0 < rows; b0 += 16 * kFinSlices) {
            float v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int b = b0 + i * kFinSlices;
                v[i] = b < rows ? gpart[(int64_t)b * kMaxPadded + pj] : 0.f;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) acc += v[i];
        }
    }
    part[t][c] = acc;
    if (blockIdx.x == 0 && c < 4) {
        double l4 = 0.0;
        for (int b0 = t; b0 < rows; b0 += 16 * kFinSlices) {
            double v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int b = b0 + i * kFinSlices;
                v[i] = b < rows ? lpart[b * 4 + c] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) l4 += v[i];
        }
        lred[t][c] = l4;
    }
    __syncthreads();
    if (t == 0 && pj >= 0) {
        float s = 0.f;
        for (int q = 0; q < kFinSlices; ++q) s += part[q][c];
        grad_out[j] = s;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double tt[4] = {0, 0, 0, 0};
        for (int q = 0; q < kFinSlices; ++q)
            for (int i = 0; i < 4; ++i) tt[i] += lred[q][i];
        const double Lv = cv * tt[0];
        const double Lb = n_bnd ? tt[2] / (double)n_bnd : 0.0;
        const double Ls = n_sen ? tt[3] / (double)n_sen : 0.0;
        if (loss_out) {
            loss_out[0] = (float)(Lv + (double)tau * Lb + (double)gamma * Ls);
            loss_out[1] = (float)Lv;
            loss_out[2] = (float)Lb;
            loss_out[3] = (float)Ls;
        }
        if (grad_eps_out) *grad_eps_out = (float)(2.0 * cv * tt[1]);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct FusedWorkspace {
    DevBuf gpart, lpart;
    int blocks = 0;
};

static int cu_count(int dev) {
    static int cached[64] = {0};
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    hipDeviceProp_t prop;
    int n = 256;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n = prop.multiProcessorCount;
    if (dev >= 0 && dev < 64) cached[dev] = n;
    return n;
}

// dynamic LDS available next to the static part (the device limit per workgroup minus the static size)
template <int L>
static size_t dyn_budget(int dev) {
    hipDeviceProp_t prop;
    size_t lim = 64 * 1024;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) lim = prop.sharedMemPerBlock;
    const size_t stat = sizeof(FusedShared<L>) + 64;
    return lim > stat ? lim - stat : 0;
}

template <int L>
static hipError_t launch_fused(int blocks, size_t dyn_bytes, const FusedArgs &a, hipStream_t s) {
    static size_t attr_bytes = 0;
    if (dyn_bytes > 48 * 1024 && attr_bytes < dyn_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)k_fused<L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)dyn_bytes);
        if (e != hipSuccess) return e;
        attr_bytes = dyn_bytes;
    }
    k_fused<L><<<blocks, kFThreads, dyn_bytes, s>>>(a);
    return hipGetLastError();
}

static size_t dyn_budget_for(int L, int dev) {
    switch (L) {
    case 1: return dyn_budget<1>(dev);
    case 2: return dyn_budget<2>(dev);
    case 3: return dyn_budget<3>(dev);
    default: return dyn_budget<4>(dev);
    }
}

vpinn_status fused_loss_grad(vpinn_problem *p, const vpinn_loss_cfg *cfg, const float *d_params,
                             const float *d_eps, float *d_loss, float *d_grad, float *d_grad_eps, hipStream_t s) {
    const int L = cfg->n_hidden, H = cfg->width;
    const int64_t nx = p->n_bnd + p->n_sen;
    const int64_t total = p->n_pts + nx;
    const int cus = cu_count(p->device);
    // items: a multiple of the block count, each about total / n_items points (at most ~2048)
    int blocks = (int)std::min<int64_t>(std::min<int64_t>((int64_t)cus * kFBlocksPerCU, kMaxBlocks), p->n_elem);
    const int64_t per_block_pts = (total + blocks - 1) / blocks;
    const int64_t rounds = (per_block_pts + 2047) / 2048;
    int64_t n_items = std::min<int64_t>((int64_t)blocks * rounds, p->n_elem);
    if (n_items < blocks) blocks = (int)n_items;
    const int64_t max_e = (p->n_elem + n_items - 1) / n_items;
    const int64_t max_x = (nx + n_items - 1) / n_items;
    const int64_t cap_pts = max_e * p->nq + max_x;
    const bool fast = p->nq <= kFThreads && p->ntest <= kKB;
    size_t dyn = sizeof(float) * (2 * cap_pts + max_e * p->ntest + (fast ? (size_t)p->ntest * kCbs : 0));
    dyn = std::max(dyn, sizeof(float) * (size_t)kMaxPadded);
    if (dyn > dyn_budget_for(L, p->device))
        return fail(VPINN_E_UNSUPPORTED, "fused path: an element's quadrature and test data exceed the LDS budget");

    auto *ws = reinterpret_cast<FusedWorkspace *>(p->fused_ws);
    if (!ws) {
        ws = new FusedWorkspace();
        p->fused_ws = ws;
        p->fused_ws_free = [](void *w) { delete reinterpret_cast<FusedWorkspace *>(w); };
    }
    if (ws->blocks < blocks) {
        VP_HIP(ws->gpart.reserve(sizeof(float) * kMaxPadded * blocks));
        VP_HIP(ws->lpart.reserve(sizeof(double) * 4 * blocks));
        ws->blocks = blocks;
    }
    const double cv = cfg->loss_norm == VPINN_NORM_ELEM ? 1.0 / (double)p->n_elem : 1.0 / (double)p->ntest;
    FusedArgs a{};
    a.params = d_params;
    a.H = H;
    a.Gx = p->Gx.as<float>();
    a.Gy = p->Gy.as<float>();
    a.F = p->F.as<float>();
    a.pts = p->pts.as<float2>();
    a.tgt = p->tgt.as<float>();
    a.eps_ptr = d_eps;
    a.n_elem = p->n_elem;
    a.n_pts = p->n_pts;
    a.n_bnd = p->n_bnd;
    a.n_sen = p->n_sen;
    a.nq = p->nq;
    a.ntest = p->ntest;
    a.n_items = n_items;
    a.cv = cv;
    a.two_cv = (float)(2.0 * cv);
    a.wb2 = p->n_bnd ? (float)(2.0 * cfg->tau / (double)p->n_bnd) : 0.f;
    a.ws2 = p->n_sen ? (float)(2.0 * cfg->gamma / (double)p->n_sen) : 0.f;
    a.tau = cfg->tau;
    a.gamma = cfg->gamma;
    a.want_grad = d_grad != nullptr;
    a.n_params_flat = vpinn_n_params(H, L);
    a.item_cap_pts = (int)cap_pts;
    a.gpart = ws->gpart.as<float>();
    a.lpart = ws->lpart.as<double>();
    a.fast_contract = fast ? 1 : 0;
    hipError_t e;
    switch (L) {
    case 1: e = launch_fused<1>(blocks, dyn, a, s); break;
    case 2: e = launch_fused<2>(blocks, dyn, a, s); break;
    case 3: e = launch_fused<3>(blocks, dyn, a, s); break;
    case 4: e = launch_fused<4>(blocks, dyn, a, s); break;
    default: return fail(VPINN_E_UNSUPPORTED, "n_hidden out of range");
    }
    if (e != hipSuccess) return fail(VPINN_E_DEVICE, std::string("fused launch: ") + hipGetErrorString(e));
    const int64_t npf = vpinn_n_params(H, L);
    const unsigned fb = (unsigned)std::max<int64_t>(1, (npf + kFinCols - 1) / kFinCols);
    const float *gp = ws->gpart.as<float>();
    const double *lp = ws->lpart.as<double>();
    const int ft = kFinCols * kFinSlices;
    switch (L) {
    case 1: k_fused_final<1><<<fb, ft, 0, s>>>(gp, lp, blocks, H, npf, cv, p->n_bnd, p->n_sen, cfg->tau, cfg->gamma,
                                               d_loss, d_grad, d_grad_eps); break;
    case 2: k_fused_final<2><<<fb, ft, 0, s>>>(gp, lp, blocks, H, npf, cv, p->n_bnd, p->n_sen, cfg->tau, cfg->gamma,
                                               d_loss, d_grad, d_grad_eps); break;
    case 3: k_fused_final<3><<<fb, ft, 0, s>>>(gp, lp, blocks, H, npf, cv, p->n_bnd, p->n_sen, cfg->tau, cfg->gamma,
                                               d_loss, d_grad, d_grad_eps); break;
    default: k_fused_final<4><<<fb, ft, 0, s>>>(gp, lp, blocks, H, npf, cv, p->n_bnd, p->n_sen, cfg->tau, cfg->gamma,
                                                d_loss, d_grad, d_grad_eps); break;
    }
    VP_HIP(hipGetLastError());
    return VPINN_OK;
}

}  // namespace vp
