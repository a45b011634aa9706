// Fused FastVPINNs loss and gradient (Algorithm 3 and its backward pass) on
// gfx950, for one problem or a batch of independent problems.
//
// Four launches per evaluation, each shaped for its own bound:
//   k_fwd      network values and spatial tangents at every point (MFMA), tiles
//              of 16 points dealt round-robin over the wavefronts of one block
//              per CU; interior points store (u_x, u_y), boundary and sensor
//              points their mismatch loss partials and adjoint dL/du directly;
//   k_contract the contraction R = eps sum_q (u_x G_x + u_y G_y) - F, the loss
//              partials and the adjoint dL/du_x[q] = eps sum_k 2 c_v R_k G_x[k,q]
//              (and y), one block per chunk of whole elements: each thread keeps
//              its point's G values in registers between the two uses, so G is
//              streamed from HBM once, by many small blocks (latency hidden by
//              occupancy rather than by a register-heavy fused kernel);
//   k_bwd      the reverse sweep through the network, same tiling as k_fwd; the
//              forward pass of each tile is recomputed (tanh included) and the
//              activations kept in registers;
//   k_fused_final  fixed-order sum of the per-block partial rows into the
//              outputs (and optionally Adam).
// No float atomics anywhere: results are bitwise reproducible, and the kernel
// boundaries order partial writes before their reads at no fence cost.
//
// Register layout of a 32-neuron vector over a 16-point tile ("chained"):
// lane l holds point j = l % 16 and neurons 16 m + 4 g + r (g = l / 16,
// m = 0..1, r = 0..3) in v[m][r].  This is exactly the output layout of a
// 16x16 MFMA for two 16-row tiles, and, read as the eight K slots 4m + r of
// lane group g, the B-operand layout of V_MFMA_F32_16X16X32_BF16 with K = all
// 32 inputs, so every hidden-to-hidden product (forward, and backward with W
// transposed) chains from registers to registers.  The products are FP32
// products evaluated as split-bf16 MFMAs (see split_pair).  Only the
// weight-gradient products, which contract over points, need their operands
// transposed: the adjoint in registers (identity MFMAs), the layer input
// through a small per-wavefront LDS tile.
#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "device_common.h"
#include "internal.h"

namespace vp {

typedef float f4 __attribute__((ext_vector_type(4)));

// forward: one block per CU of 8, 12 or 16 wavefronts (a tuning choice); the
// forward alone needs ~140 registers (the 16-wavefront build is held to 128), so
// three or four wavefronts per SIMD hide each other's LDS and MFMA latencies
// contraction: many small blocks, one chunk of whole elements each
constexpr int kCThreads = 256;
constexpr int kCWaves = kCThreads / 64;
constexpr int kGThreads = 1024;  // large-element contraction: one element per block
constexpr int kGWaves = kGThreads / 64;
// backward: one block of eight wavefronts per CU (two per SIMD, register-limited at ~250
// VGPRs); tiles are dealt round-robin over the eight, which bounds every SIMD's share
// within one tile of the mean, and the weights are held once per CU
constexpr int kBThreads = 512;
constexpr int kBWaves = kBThreads / 64;
constexpr int kTs = 36;            // transpose tile row stride (floats)
constexpr int kMaxBlocks = 1024;
constexpr int kKB = 32;              // test functions held in registers by the fast contraction
constexpr int kRowQ = 4;             // quadrature points per lane in the row-streaming contraction
// contraction paths: thread per point with every test function in registers
// (nq <= kCThreads, ntest <= kKB); wavefront per test-function row, G read once,
// with Q = 1, 2 or 4 points a lane (nq <= 64 Q; one kernel per Q keeps each at
// the occupancy its registers allow); two launches (row sums, then adjoint) for
// larger elements (and a matrix-free path, wavefront per element, for problems that
// store no G)
enum { kPathFast = 0, kPathRows1 = 1, kPathRows2 = 2, kPathRows4 = 3, kPathGeneric = 4, kPathMF = 5, kNumPaths = 6 };
constexpr int kCbs = kCThreads + 1;  // row stride of the per-point term buffer

// NH = 2: the network has a second linear output, the space-dependent diffusion
// coefficient e(x, y) (Sec. 4.7.2); its weights follow the first output's in the
// padded layout, and its gradient takes two more column-sum slots
__host__ __device__ constexpr int n_pad_h(int L, int NH) { return NH == 2 ? n_padded2(L) : n_padded(L); }
__host__ __device__ constexpr int n_vslots(int L, int NH) { return L + 4 + 2 * (NH - 1); }

struct Vec {
    f4 v[2];
};

// FP32 products on the bf16 matrix cores.  Every operand x is split into three bf16
// pieces, x0 = rn(x), x1 = rn(x - x0), x2 = rn(x - x0 - x1) (each subtraction exact), so
// |x1| <= 2^-8 |x|, |x2| <= 2^-16 |x| and |x - x0 - x1 - x2| <= 2^-24 |x|; a product is the
// sum of the six piece products x_i y_j with i + j <= 2, each exact in FP32, accumulated
// smallest first (the three dropped ones are below 2^-23 |x y|).  Measured on random
// 16x32 by 32x16 products, its error is half that of the FP32 MFMA (16x16x4f32).  The
// point of it: bf16 MFMAs run on the matrix cores beside the vector ALU work of the other
// wavefront of a SIMD, while FP32 MFMAs hold the vector ALU for their whole duration,
// and a 16x16x32 bf16 product takes ~17 cycles against ~33 for 16x16x4 in FP32.
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef float fl2 __attribute__((ext_vector_type(2)));

// the piece pairs (i, j) of a product, smallest first
constexpr int kPi[6] = {0, 1, 2, 0, 1, 0};
constexpr int kPj[6] = {2, 1, 0, 1, 0, 0};

__device__ __forceinline__ unsigned pk_bf16(float x, float y) {
    const fl2 v = {x, y};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf2));
}

// x in the low half, y in the high half of each piece
struct Pieces3 {
    unsigned p0, p1, p2;
};
__device__ __forceinline__ Pieces3 split_pair(float x, float y) {
    Pieces3 r;
    r.p0 = pk_bf16(x, y);
    x -= __uint_as_float(r.p0 << 16);
    y -= __uint_as_float(r.p0 & 0xffff0000u);
    r.p1 = pk_bf16(x, y);
    x -= __uint_as_float(r.p1 << 16);
    y -= __uint_as_float(r.p1 & 0xffff0000u);
    r.p2 = pk_bf16(x, y);
    return r;
}

// the weight fragments are read from LDS again for every tile: reading them through an
// opaque copy of the lane index keeps the compiler from hoisting them out of the tile
// loops into registers, which would cost the occupancy of every network kernel
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// a K = 32 operand (eight values a lane) and a K = 16 operand (four), three pieces each
struct Split8 {
    u4 p[3];
};
struct Split4 {
    u2 p[3];
};

__device__ __forceinline__ f4 mfb(u4 a, u4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfb16(u2 a, u2 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4v, a), __builtin_bit_cast(s4v, b), c, 0, 0,
                                                     0);
}

__device__ __forceinline__ void split4(const float (&v)[4], Split4 &s) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const Pieces3 r = split_pair(v[2 * q], v[2 * q + 1]);
        s.p[0][q] = r.p0;
        s.p[1][q] = r.p1;
        s.p[2][q] = r.p2;
    }
}

// a chained vector as the K = 32 operand: slot 4m + r holds v[m][r] (neuron 16m + 4g + r)
__device__ __forceinline__ void split8(const Vec &v, Split8 &s) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const Pieces3 r = split_pair(v.v[m][2 * h], v.v[m][2 * h + 1]);
            s.p[0][2 * m + h] = r.p0;
            s.p[1][2 * m + h] = r.p1;
            s.p[2][2 * m + h] = r.p2;
        }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// network weights of the current instance in LDS
template <int L>
struct WeightsShared {
    // A-operand fragments of the hidden-to-hidden products, layers 2..L, as three bf16
    // pieces: [layer][dir 0 = W (forward), 1 = W^T (backward)][out tile][piece][lane];
    // lane (c, g) of out tile t holds in slot 4m + r the weight of output 16t + c and
    // input 16m + 4g + r (dir 0), or of output 16m + 4g + r and input 16t + c (dir 1)
    u4 wp[L > 1 ? L - 1 : 1][2][2][3][64];
    // layer 2's tangent products from s_1 = 1 - a_1^2: p_2 = W_2 (s_1 W_1[:, c]) =
    // (W_2 diag(W_1[:, c])) s_1, so both tangents share one split; [c][out tile][piece][lane]
    u4 wt2[2][2][3][64];
    float w1[PW][2];
    float b[L][PW];
    float wo[PW];
    float bo;
    float wo2[PW];  // second output (NH = 2 only)
    float bo2;
};

template <int L, int NW>
struct FwdShared {
    WeightsShared<L> W;
    float stage[n_padded2(L)];  // flat parameters, staged for load_weights
    double lp[NW][2];          // per-wavefront loss partials: sum d_b^2, sum d_s^2
};

template <int L, int NH>
struct BwdShared {
    WeightsShared<L> W;
    union {
        // per-wavefront transpose tiles [2][16 points][kTs]
        float tt[kBWaves][2][16][kTs];
        // during the flush: three of the four pair-sum regions (the fourth is red)
        float part[3][n_pad_h(L, NH)];
    };
    // per-wavefront column sums of the vector-shaped gradients, one slot per lane:
    // [0, L) biases b_l, L: W1 column 0, L+1: W1 column 1, L+2: W_out, L+3: b_out,
    // and with a second output L+4: its weights, L+5: its bias
    float vacc[kBWaves][n_vslots(L, NH)][64];
    float red[n_pad_h(L, NH)];
};

// static description of one problem instance (device resident)
struct InstDesc {
    const float *Gx, *Gy, *F;
    const float2 *pts;        // interior points then boundary then sensors
    const float *tgt;         // boundary values then sensor observations
    int64_t n_elem, n_pts, n_bnd, n_sen;
    int64_t n_tiles, tile0;   // tiles (16 points each) tile0 .. of the global tile list
    int64_t ubase;            // offset of this instance's points in the point buffer
    int64_t cblk0, n_chunks;  // contraction blocks cblk0 .. (epc elements each)
    int64_t gstride;          // floats between elements in G_x, G_y (0: one shared premultiplier)
    const float *M;           // space-dependent diffusion: convection weights w_q det J v_k (else null)
    float cbx, cby;           // and the velocity (also of a matrix-free problem)
    const float *geo, *tab;   // matrix-free: bilinear map coefficients [n_elem][8], 1D tables
    float kdiff;              // matrix-free: constant diffusion coefficient
    int qn, tn;               // matrix-free: quadrature points and test functions per direction
    // shared points (else null): slot e nq + q reads point umap[slot]; the adjoint of
    // the contraction goes per slot to adj (eadj: dL/de), and the slots of point u are
    // uslot[usoff[u] .. usoff[u + 1]).  Unshared, adj and eadj are the point buffers.
    const int *umap, *usoff, *uslot;
    float2 *adj;
    float *eadj;
    int nq, ntest, epc;
    int path;                 // contraction path (kPathFast .. kPathMF)
    // large elements (kPathGeneric): row-sum blocks rblk0 .. (element, row block of 16, point
    // block of kSplitQ; nkb x nqb per element) write partial sums at apart[abase ..]; the
    // adjoint blocks (npb per element, 64 points each) are this instance's contraction blocks
    int64_t rblk0, abase;
    int nkb, nqb, npb;
    int kw;                   // adjoint: wavefronts sharing one group of 64 points (1, 2, 4, 8 or 16)
    // loss partial rows lrow0 .. lrow0 + ln_rows - 1: first one per tile block
    // (gblk0 ..), then one per contraction block
    int lrow0, ln_rows;
    int grow0, gblk0, gn_rows;  // gradient partial rows (tile blocks gblk0 ..)
    int64_t grp0, n_grp;      // one-pass plans: the instance's groups grp0 .. of the global group list
    float two_cv, wb2, ws2;   // 2 c_v, 2 tau / N_D, 2 gamma / N_s
    float tau, gamma;
    double cv;
};

struct FwdArgs {
    const InstDesc *inst;
    const int64_t *blk_tiles;   // [blocks + 1] global tile range of each block (shared with k_bwd)
    const int *blk_inst0;       // instance of each block's first tile
    const float *params;        // [n_inst][param_stride] flat layout, width H
    int64_t param_stride;
    int H;
    float2 *ubuf;               // per point: (u_x, u_y) at interior points, (dL/du, 0) elsewhere
    double *lpart;              // [loss rows][4]
    int64_t *step;              // optional step counter, incremented once per launch
    float *ebuf;                // two outputs: second output e at interior points (point buffer order)
    float *act;                 // optional: activations a_1 .. a_L of every tile, [tile][L][2][64][4]
};

struct ContractArgs {
    const InstDesc *inst;
    const int *cblk_inst;       // [contraction blocks] instance of each block
    int64_t cblk_base;          // global contraction block of this launch's block 0
    const float *eps;           // [n_inst] or null (eps = 1)
    int want_grad;
    float2 *ubuf;               // in: (u_x, u_y); out: (dL/du_x, dL/du_y) at interior points
    double *lpart;
    float *ebuf;                // two outputs: in e, out dL/de at interior points
};

struct BwdArgs {
    const InstDesc *inst;
    const int64_t *blk_tiles;   // [blocks + 1] global tile range of each block
    const int *blk_inst0;       // instance of each block's first tile
    const float *params;
    int64_t param_stride;
    int H;
    const float2 *ubuf;
    float *gpart;               // [gradient rows][kMaxPadded]
    const float *ebuf;          // two outputs: dL/de at interior points
    const float *act;           // activations stored by k_fwd (with the loading instantiation of k_bwd)
};

// ---------------------------------------------------------------------------
// forward through the network for one tile.  With KEEP the activations a_l and
// the tangents t_l = s_l p_l (s_l = 1 - a_l^2, p_l = W_l t_{l-1}; l >= 2) are kept
// for the reverse sweep, which needs exactly these: t_{l-1} is the input of layer
// l's weight gradient, and s_l sbar_l = tbar_l . t_l (layer 1 keeps a_1 only; its
// tangent is s_1 times a weight column).
// ---------------------------------------------------------------------------
template <int L>
struct Acts {
    Vec a[L];
    Vec tx[L];  // tx[0], ty[0] unused (layer 1)
    Vec ty[L];
};

// activations of one tile in the layout [layer][m][lane][4]: each lane's chained
// vector is two 16-byte pieces, so a layer is two fully coalesced 1 KB accesses
constexpr int kActTile = 2 * 64 * 4;  // floats per layer and tile
// largest activation buffer the autotuner considers storing (the 256 MB last-level cache of the part)
constexpr size_t kActStoreMaxBytes = (size_t)256 << 20;

// tanh(x) = 1 - 2 / (1 + e^{2x}): one exponential, one reciprocal and three other
// operations against five for the sign-split form tanh_f32 (largest absolute error
// 1.8e-7 against 1.3e-7); the limits come out exactly (e = inf gives 1, e = 0
// gives -1).  Every network kernel of this file uses it (the forward and reverse
// sweeps therefore see the same activations); the plain path keeps tanh_f32.
__device__ __forceinline__ float tanh_lean(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
}

template <int L, bool KEEP>
__device__ __forceinline__ void tile_forward(const WeightsShared<L> &S, int lane, float x, float y, Vec &A_, Vec &TX,
                                             Vec &TY, Acts<L> &keep, float *act = nullptr) {
    const int g = lane >> 4;
    const int ln = opaque(lane);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * m + 4 * g + r;
            const float w0 = S.w1[n][0], w1v = S.w1[n][1];
            const float z = fmaf(w0, x, fmaf(w1v, y, S.b[0][n]));
            const float a = tanh_lean(z);
            const float s = 1.0f - a * a;
            A_.v[m][r] = a;
            if (L == 1) {
                TX.v[m][r] = s * w0;
                TY.v[m][r] = s * w1v;
            } else {
                TX.v[m][r] = s;  // s_1: layer 2 forms both tangents from it
            }
        }
    if (act) {
        f4 *o = reinterpret_cast<f4 *>(act);
        o[lane] = A_.v[0];
        o[64 + lane] = A_.v[1];
    }
    if (KEEP) keep.a[0] = A_;
#pragma unroll
    for (int l = 2; l <= L; ++l) {
        Vec Z, PX, PY;
        // the layer's inputs as bf16 pieces.  Layer 2's TX holds s_1 and its tangents use the two scaled weight sets.  One output
        // tile at a time (its three chains interleaved), its weights read just before its
        // products; in the forward pass alone a scheduling barrier keeps the next tile's reads
        // from being hoisted, which would hold every weight set in registers at once.
        const bool s1 = l == 2;
        Split8 sa, sx, sy;
        split8(A_, sa);
        split8(TX, sx);
        if (!s1) split8(TY, sy);
        f4 z[2], px[2], py[2];
#pragma unroll
        for (int mo = 0; mo < 2; ++mo) {
#pragma unroll
            for (int r = 0; r < 4; ++r) z[mo][r] = S.b[l - 1][16 * mo + 4 * g + r];
            px[mo] = f4{0.f, 0.f, 0.f, 0.f};
            py[mo] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int mo = 0; mo < 2; ++mo) {
            Split8 w, wx, wy;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                w.p[k] = S.wp[l - 2][0][mo][k][ln];
                if (s1) {
                    wx.p[k] = S.wt2[0][mo][k][ln];
                    wy.p[k] = S.wt2[1][mo][k][ln];
                }
            }
#pragma unroll
            for (int t = 0; t < 6; ++t) {
                z[mo] = mfb(w.p[kPi[t]], sa.p[kPj[t]], z[mo]);
                if (s1) {
                    px[mo] = mfb(wx.p[kPi[t]], sx.p[kPj[t]], px[mo]);
                    py[mo] = mfb(wy.p[kPi[t]], sx.p[kPj[t]], py[mo]);
                } else {
                    px[mo] = mfb(w.p[kPi[t]], sx.p[kPj[t]], px[mo]);
                    py[mo] = mfb(w.p[kPi[t]], sy.p[kPj[t]], py[mo]);
                }
            }
            if (!KEEP) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int mo = 0; mo < 2; ++mo) {
            Z.v[mo] = z[mo];
            PX.v[mo] = px[mo];
            PY.v[mo] = py[mo];
        }
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float a = tanh_lean(Z.v[m][r]);
                const float s = 1.0f - a * a;
                A_.v[m][r] = a;
                TX.v[m][r] = s * PX.v[m][r];
                TY.v[m][r] = s * PY.v[m][r];
            }
        if (act) {
            f4 *o = reinterpret_cast<f4 *>(act + (l - 1) * kActTile);
            o[lane] = A_.v[0];
            o[64 + lane] = A_.v[1];
        }
        if (KEEP) {
            keep.a[l - 1] = A_;
            keep.tx[l - 1] = TX;
            keep.ty[l - 1] = TY;
        }
    }
}

// the reverse sweep's forward state from stored activations: a_l is read, s_l =
// 1 - a_l^2, and only the tangents are recomputed (no tanh, no value products)
template <int L>
__device__ __forceinline__ void tile_forward_loaded(const WeightsShared<L> &S, int lane, const float *act,
                                                    Acts<L> &K) {
    const int g = lane >> 4;
    const int ln = opaque(lane);
    const f4 *in = reinterpret_cast<const f4 *>(act);
#pragma unroll
    for (int l = 0; l < L; ++l) {
        K.a[l].v[0] = in[l * (kActTile / 4) + lane];
        K.a[l].v[1] = in[l * (kActTile / 4) + 64 + lane];
    }
    Vec TX, TY;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * m + 4 * g + r;
            const float a = K.a[0].v[m][r];
            const float s = 1.0f - a * a;
            TX.v[m][r] = s * S.w1[n][0];
            TY.v[m][r] = s * S.w1[n][1];
        }
#pragma unroll
    for (int l = 2; l <= L; ++l) {
        Vec PX, PY;
        Split8 sx, sy;
        split8(TX, sx);
        split8(TY, sy);
        Split8 w[2];
#pragma unroll
        for (int mo = 0; mo < 2; ++mo)
#pragma unroll
            for (int k = 0; k < 3; ++k) w[mo].p[k] = S.wp[l - 2][0][mo][k][ln];
        f4 px[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}}, py[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int t = 0; t < 6; ++t)
#pragma unroll
            for (int mo = 0; mo < 2; ++mo) {
                px[mo] = mfb(w[mo].p[kPi[t]], sx.p[kPj[t]], px[mo]);
                py[mo] = mfb(w[mo].p[kPi[t]], sy.p[kPj[t]], py[mo]);
            }
#pragma unroll
        for (int mo = 0; mo < 2; ++mo) {
            PX.v[mo] = px[mo];
            PY.v[mo] = py[mo];
        }
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float a = K.a[l - 1].v[m][r];
                const float s = 1.0f - a * a;
                TX.v[m][r] = s * PX.v[m][r];
                TY.v[m][r] = s * PY.v[m][r];
            }
        K.tx[l - 1] = TX;
        K.ty[l - 1] = TY;
    }
}

// sum over the four K-slot groups (lanes j, j+16, j+32, j+48)
__device__ __forceinline__ float group_sum(float v) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

template <int L>
__device__ __forceinline__ void tile_outputs(const WeightsShared<L> &S, int lane, const Vec &A_, const Vec &TX,
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

// the second output e = W_out2 . a_L + b_out2 (no tangents needed)
template <int L>
__device__ __forceinline__ float tile_second(const WeightsShared<L> &S, int lane, const Vec &A_) {
    const int g = lane >> 4;
    float se = 0.f;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) se = fmaf(S.wo2[16 * m + 4 * g + r], A_.v[m][r], se);
    return group_sum(se) + S.bo2;
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

__device__ __forceinline__ float colsum_vec(float (*T0)[kTs], int lane, const Vec &V) {
    put_t(T0, lane, V);
    wave_sync();
    const float s = col_sum(T0, lane);
    wave_sync();
    return s;
}

// gradient accumulators of one wavefront: the hidden-to-hidden weight tiles of
// layers 2..L in registers (MFMA accumulators); the vector-shaped gradients are
// column sums kept in LDS (FusedShared::vacc) to spare registers
template <int L>
struct GradAcc {
    f4 w[L > 1 ? L - 1 : 1][4];
};

// layer-1 tangent s_1 * W1[:, col] transposed into T
template <int L>
__device__ __forceinline__ void put_t_tangent1(float (*T)[kTs], int lane, const Vec &a, const WeightsShared<L> &S,
                                               int col) {
    const int j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        f4 t;
#pragma unroll
        for (int r = 0; r < 4; ++r) t[r] = (1.0f - a.v[m][r] * a.v[m][r]) * S.w1[16 * m + 4 * g + r][col];
        *reinterpret_cast<f4 *>(&T[j][16 * m + 4 * g]) = t;
    }
}

// identity operand of the in-register transposes (K = 16): lane (n, g) holds 1 in slot j
// where 4g + j = n
__device__ __forceinline__ u2 ident16(int lane) {
    const int j = (lane & 15) - 4 * (lane >> 4);
    const unsigned one = 0x3f80u;  // bf16 1.0
    return u2{(j == 0 ? one : 0u) | (j == 1 ? one << 16 : 0u), (j == 2 ? one : 0u) | (j == 3 ? one << 16 : 0u)};
}

// a split chained vector transposed in registers: per half m and piece k, D = A I with A
// the piece's half (rows = the 16 points, K = the half's 16 neurons), so lane (n, g) gets
// neuron 16m + n at points 4g + r, the K = points operand of the weight-gradient products
// (slot r = point 4g + r).  Every value is a bf16 times 1, so D and its repacking are exact.
__device__ __forceinline__ void transpose_split(const Split8 &s, u2 id, Split4 (&t)[2]) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const f4 d = mfb16(u2{s.p[k][2 * m], s.p[k][2 * m + 1]}, id, f4{0.f, 0.f, 0.f, 0.f});
            t[m].p[k] = u2{pk_bf16(d[0], d[1]), pk_bf16(d[2], d[3])};
        }
}

// the in-side operand of one weight-gradient product from the transpose tile T1[point][n]:
// lane (c, g) holds neurons c and 16 + c at points 4g + j (slot j)
__device__ __forceinline__ void wgrad_read(float (*T1)[kTs], int lane, float (&b0)[4], float (&b1)[4]) {
    wave_sync();
    const int c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        b0[j] = T1[4 * g + j][c];
        b1[j] = T1[4 * g + j][16 + c];
    }
}

// one stream of a layer's reverse sweep: its propagation W_l^T vbar (into out) and its
// weight gradient vbar x in (into acc, K = the tile's 16 points).  The transpose tile of
// the in-side vector is read first and the split of vbar, which needs no LDS, runs while
// those reads are in flight; then the in-side split, and then every product of the stream
// (propagation, the in-register transpose, the weight gradient) as one cluster at raised
// wave priority, so the matrix cores are fed while the other wavefront of the SIMD issues
// its vector work beside them.
__device__ __forceinline__ void stream_back(float (*T1)[kTs], int lane, u2 id, const Split8 (&wt)[2], const Vec &vb,
                                            f4 (&out)[2], f4 acc[4]) {
    float b0[4], b1[4];
    wgrad_read(T1, lane, b0, b1);
    Split8 sv;
    split8(vb, sv);
    Split4 a[2], sb[2];
    split4(b0, sb[0]);
    split4(b1, sb[1]);
    f4 v[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int t = 0; t < 6; ++t)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) v[mi] = mfb(wt[mi].p[kPi[t]], sv.p[kPj[t]], v[mi]);
    out[0] = v[0];
    out[1] = v[1];
    transpose_split(sv, id, a);
    // two piece products per K = 32 product (slots 0-3 one pair of pieces, 4-7 the other),
    // smallest first: (0,2)+(2,0), (1,1)+(0,1), (1,0)+(0,0)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int i0 = kPi[2 * q], j0 = kPj[2 * q], i1 = kPi[2 * q + 1], j1 = kPj[2 * q + 1];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
                acc[2 * m + n] = mfb(u4{a[m].p[i0][0], a[m].p[i0][1], a[m].p[i1][0], a[m].p[i1][1]},
                                     u4{sb[n].p[j0][0], sb[n].p[j0][1], sb[n].p[j1][0], sb[n].p[j1][1]},
                                     acc[2 * m + n]);
    }
    __builtin_amdgcn_s_setprio(0);
}

// padb (width below 32): the hidden layers' bias gradients come out of the weight-gradient
// products as column 31 (see tile_backward); otherwise they are column sums in VA
template <int L, int NH>
__device__ __forceinline__ void tile_backward(WeightsShared<L> &S, float (*T0)[kTs], float (*T1)[kTs], int lane,
                                              float x, float y, float ub, float uxb, float uyb, float eb,
                                              const Acts<L> &K, GradAcc<L> &G, float (*VA)[64], bool padb) {
    const int g = lane >> 4;
    const int ln = opaque(lane);
    const u2 id = ident16(lane);
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
                if (L == 1) {
                    const float s = 1.0f - aL.v[m][r] * aL.v[m][r];
                    tx = s * S.w1[n][0];
                    ty = s * S.w1[n][1];
                } else {
                    tx = K.tx[L - 1].v[m][r];
                    ty = K.ty[L - 1].v[m][r];
                }
                v.v[m][r] = ub * aL.v[m][r] + uxb * tx + uyb * ty;
                const float w = S.wo[n];
                abar.v[m][r] = NH == 2 ? fmaf(eb, S.wo2[n], ub * w) : ub * w;
                txbar.v[m][r] = uxb * w;
                tybar.v[m][r] = uyb * w;
            }
        VA[L + 2][lane] += colsum_vec(T0, lane, v);
        if (g == 0) VA[L + 3][lane] += ub;
        if (NH == 2) {
            // second output: dW_out2 = sum_p eb a_L, db_out2 = sum_p eb
            Vec ve;
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) ve.v[m][r] = eb * aL.v[m][r];
            VA[L + 4][lane] += colsum_vec(T0, lane, ve);
            if (g == 0) VA[L + 5][lane] += eb;
        }
    }
#pragma unroll
    for (int l = L; l >= 2; --l) {
        Vec zb, pxb, pyb;
        const Vec &al = K.a[l - 1];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // z_bar = s (abar - 2 a sbar) with sbar = tbar . p, and s sbar = tbar . t
                const float a = al.v[m][r];
                const float s = 1.0f - a * a;
                pxb.v[m][r] = s * txbar.v[m][r];
                pyb.v[m][r] = s * tybar.v[m][r];
                const float ssbar = txbar.v[m][r] * K.tx[l - 1].v[m][r] + tybar.v[m][r] * K.ty[l - 1].v[m][r];
                zb.v[m][r] = fmaf(-2.0f * a, ssbar, s * abar.v[m][r]);
            }
        // weight gradient with the inputs of layer l: a_{l-1} and t_{l-1} = s_{l-1} p_{l-1}
        // (layer 1: s_1 times a W1 column), formed while writing the transpose tile.  With a
        // padding neuron (width below 32) its input slot 31 is set to 1 in the transpose tile
        // of the value stream, so dW_l[:, 31] = sum_p zbar = db_l comes out of the same
        // products (the slot's weights are zero and its gradient is otherwise unused)
        // W_l^T fragments of the propagation (abar = W_l^T zbar, tbar = W_l^T pbar), read once
        // for the three streams
        Split8 wv[2];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int k = 0; k < 3; ++k) wv[mi].p[k] = S.wp[l - 2][1][mi][k][ln];
        f4 pa[2], px[2], py[2];
        // stream 1: zbar with a_{l-1}; 2: pbar^x with t^x_{l-1}; 3: pbar^y with t^y_{l-1}
        if (padb) {
            Vec ab = K.a[l - 2];
            if ((lane >> 4) == 3) ab.v[1][3] = 1.0f;  // neuron 16 + 4*3 + 3 = 31
            put_t(T1, lane, ab);
        } else {
            put_t(T1, lane, K.a[l - 2]);
            VA[l - 1][lane] += colsum_vec(T0, lane, zb);
        }
        stream_back(T1, lane, id, wv, zb, pa, G.w[l - 2]);
        wave_sync();
        if (l - 1 == 1) put_t_tangent1<L>(T1, lane, K.a[0], S, 0);
        else put_t(T1, lane, K.tx[l - 2]);
        stream_back(T1, lane, id, wv, pxb, px, G.w[l - 2]);
        wave_sync();
        if (l - 1 == 1) put_t_tangent1<L>(T1, lane, K.a[0], S, 1);
        else put_t(T1, lane, K.ty[l - 2]);
        stream_back(T1, lane, id, wv, pyb, py, G.w[l - 2]);
        wave_sync();
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
            abar.v[mi] = pa[mi];
            txbar.v[mi] = px[mi];
            tybar.v[mi] = py[mi];
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
        VA[L][lane] += colsum_vec(T0, lane, c0);
        VA[L + 1][lane] += colsum_vec(T0, lane, c1);
        VA[0][lane] += colsum_vec(T0, lane, zb);
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// weights of one instance -> LDS (padded to 32, fragment order for the MFMA A operands).
// The flat parameters are first copied into `stage` with every thread's loads in
// flight at once (npf <= n_padded(L)), then rearranged LDS to LDS.
template <int L, int NT, int NH>
__device__ __forceinline__ void load_weights(WeightsShared<L> &S, float *stage, const float *__restrict__ P, int H,
                                             int tid) {
    // addresses are formed here at every call: hoisted to the kernel's start, they would be
    // spilled by the tile loops and reloaded at every instance change
    tid = opaque(tid);
    // flat tail: W_out[NH][H], b_out[NH]
    const int npf = 3 * H + (L - 1) * (H * H + H) + NH * (H + 1);
    constexpr int kLoads = (n_pad_h(L, NH) + NT - 1) / NT;
    float v[kLoads];
#pragma unroll
    for (int i = 0; i < kLoads; ++i) {
        const int j = tid + i * NT;
        v[i] = j < npf ? P[j] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < kLoads; ++i) {
        const int j = tid + i * NT;
        if (j < npf) stage[j] = v[i];
    }
    __syncthreads();
    for (int t = tid; t < PW * 2; t += NT) {
        const int o = t >> 1, i = t & 1;
        S.w1[o][i] = o < H ? stage[o * 2 + i] : 0.f;
    }
    for (int t = tid; t < L * PW; t += NT) {
        const int l = t / PW + 1, o = t % PW;
        const int off = (l == 1) ? 2 * H : (int)hoff_w(H, l) + H * H;
        S.b[l - 1][o] = o < H ? stage[off + o] : 0.f;
    }
    const int ho = (int)hoff_w(H, L + 1);
    for (int t = tid; t < PW; t += NT) S.wo[t] = t < H ? stage[ho + t] : 0.f;
    if (tid == 0) S.bo = stage[ho + NH * H];
    if (NH == 2) {
        for (int t = tid; t < PW; t += NT) S.wo2[t] = t < H ? stage[ho + H + t] : 0.f;
        if (tid == 0) S.bo2 = stage[ho + 2 * H + 1];
    }
    // fragments: thread t takes (layer, dir, out tile, lane) = t, gathers its eight
    // weights from the staged parameters and writes their three pieces
    static_assert(NT % 64 == 0, "whole wavefronts");
    constexpr int kTot = (L - 1) * 2 * 2 * 64;
    for (int t = tid; t < kTot; t += NT) {
        const int ln = t & 63, mt = (t >> 6) & 1, dir = (t >> 7) & 1, l = 2 + (t >> 8);
        const int c = ln & 15, g = ln >> 4;
        Vec w;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = 16 * m + 4 * g + r;
                const int o = dir == 0 ? 16 * mt + c : q;
                const int i = dir == 0 ? q : 16 * mt + c;
                w.v[m][r] = (o < H && i < H) ? stage[hoff_w(H, l) + o * H + i] : 0.f;
            }
        Split8 sp;
        split8(w, sp);
#pragma unroll
        for (int k = 0; k < 3; ++k) S.wp[l - 2][dir][mt][k][ln] = sp.p[k];
    }
    if (L >= 2) {
        for (int t = tid; t < 2 * 2 * 64; t += NT) {
            const int ln = t & 63, mt = (t >> 6) & 1, col = t >> 7;
            const int c = ln & 15, g = ln >> 4, o = 16 * mt + c;
            Vec w;
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int q = 16 * m + 4 * g + r;
                    w.v[m][r] = (o < H && q < H) ? stage[hoff_w(H, 2) + o * H + q] * stage[2 * q + col] : 0.f;
                }
            Split8 sp;
            split8(w, sp);
#pragma unroll
            for (int k = 0; k < 3; ++k) S.wt2[col][mt][k][ln] = sp.p[k];
        }
    }
}

template <int L>
__device__ __forceinline__ void zero_acc(GradAcc<L> &G) {
#pragma unroll
    for (int l = 0; l < (L > 1 ? L - 1 : 1); ++l)
#pragma unroll
        for (int t = 0; t < 4; ++t) G.w[l][t] = f4{0.f, 0.f, 0.f, 0.f};
}

// 1: forward values and tangents at every point.  Blocks own contiguous tile ranges
// (the same ranges as k_bwd), possibly spanning instances; the tiles of a range go
// round-robin over the block's wavefronts.
template <int L, int NW, int NH, bool ST>
__global__ __launch_bounds__(NW * 64, 1) void k_fwd(FwdArgs A) {
    constexpr int kFwThreads = NW * 64, kFwWaves = NW;
    __shared__ FwdShared<L, NW> S;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (A.step && blockIdx.x == 0 && tid == 0) *A.step += 1;
    int64_t t = A.blk_tiles[blockIdx.x];
    const int64_t t_end = A.blk_tiles[blockIdx.x + 1], t_blk = t;
    int cur = A.blk_inst0[blockIdx.x];
    while (t < t_end) {
        const InstDesc *Ip = A.inst + cur;
        const int64_t tile0 = Ip->tile0, n_pts = Ip->n_pts, n_bnd = Ip->n_bnd;
        const int64_t n_all = n_pts + n_bnd + Ip->n_sen;
        const float2 *__restrict__ pts = Ip->pts;
        const float *__restrict__ tgt = Ip->tgt;
        float2 *__restrict__ ub_i = A.ubuf + Ip->ubase;
        float *__restrict__ e_i = NH == 2 ? A.ebuf + Ip->ubase : nullptr;
        const float wb2 = Ip->wb2, ws2 = Ip->ws2;
        const int64_t seg_end = min(t_end, tile0 + Ip->n_tiles);
        const int64_t row = Ip->lrow0 + (int64_t)(blockIdx.x - Ip->gblk0);
        __syncthreads();
        load_weights<L, kFwThreads, NH>(S.W, S.stage, A.params + (int64_t)cur * A.param_stride, A.H, tid);
        __syncthreads();
        double lbb = 0.0, lss = 0.0;
        // the next tile's point is loaded while this tile computes
        auto fetch = [&](int64_t tt) -> float2 {
            const int64_t idx = 16 * (tt - tile0) + (lane & 15);
            return (tt < seg_end && idx < n_all) ? pts[idx] : make_float2(0.f, 0.f);
        };
        const int64_t first = t + (int64_t)((wave - (int)((t - t_blk) % kFwWaves) + kFwWaves) % kFwWaves);
        float2 pn = fetch(first);
        for (int64_t tt = first; tt < seg_end; tt += kFwWaves) {
            const int64_t idx = 16 * (tt - tile0) + (lane & 15);
            const float2 p = pn;
            pn = fetch(tt + kFwWaves);
            Vec a, tx, ty;
            Acts<L> unused;
            // ST: keep every layer's activations for the reverse sweep
            tile_forward<L, false>(S.W, lane, p.x, p.y, a, tx, ty, unused,
                                   ST ? A.act + tt * (int64_t)(L * kActTile) : nullptr);
            float u, ux, uy;
            tile_outputs<L>(S.W, lane, a, tx, ty, u, ux, uy);
            const float e = NH == 2 ? tile_second<L>(S.W, lane, a) : 0.f;
            if (lane < 16 && idx < n_all) {
                if (idx < n_pts) {
                    ub_i[idx] = make_float2(ux, uy);
                    if (NH == 2) e_i[idx] = e;
                } else {
                    // boundary (Sec. 2.3) or sensor (Sec. 4.7) mismatch: loss term and its adjoint
                    const int64_t xi = idx - n_pts;
                    const float d = u - tgt[xi];
                    const bool bnd = xi < n_bnd;
                    if (bnd) lbb += (double)d * (double)d;
                    else lss += (double)d * (double)d;
                    ub_i[idx] = make_float2((bnd ? wb2 : ws2) * d, 0.f);
                }
            }
        }
        // loss partials of the block for this instance, wavefronts added in order
        const double vb = wave_sum(lbb), vs = wave_sum(lss);
        if (lane == 0) {
            S.lp[wave][0] = vb;
            S.lp[wave][1] = vs;
        }
        __syncthreads();
        if (tid < 4) {
            double v = 0.0;
            if (tid >= 2)
                for (int w = 0; w < kFwWaves; ++w) v += S.lp[w][tid - 2];
            A.lpart[row * 4 + tid] = v;
        }
        t = seg_end;
        ++cur;
    }
}

// Contraction, variational loss terms and the adjoint of the contraction
// (Algorithm 3 and its reverse), one block per chunk of epc whole elements, three
// kernels for three element shapes (each instance's chunks go to one of them):
//   fast (nq <= kCThreads, ntest <= kKB): thread (element, q) holds G_x[e,k,q],
//     G_y[e,k,q] for all k in registers; the per-point terms u_x G_x + u_y G_y go
//     through LDS to per-(element, test) row sums (eight lanes a row); then dL/du
//     at q from the same registers.  With a space-dependent diffusion e(x, y) (the
//     network's second output) and velocity b the term is
//     e_q (u_x G_x + u_y G_y) + (b . grad u)_q M, M = w_q det J v_k also held in
//     registers, and the adjoint adds dL/de_q = sum_k 2 c_v R_k (u_x G_x + u_y G_y);
//   rows (nq <= 64 kRowQ, any ntest): one element per block, G streamed row by row,
//     each row used twice from registers;
//   split (larger elements): two launches, row sums by (element, rows, points) into
//     partials, then R, loss and the adjoint by (element, points), G read again
//     (cache-resident by then), so even one element spreads over the chip.
// In every case G is read from HBM once; loss partials go to one row per block.

// point of slot s (shared points) or the slot itself
__device__ __forceinline__ int64_t upoint(const InstDesc *I, int64_t s) { return I->umap ? (int64_t)I->umap[s] : s; }

struct ContractCtx {
    const InstDesc *I;
    int64_t chunk, e0;
    float eps;
};

__device__ __forceinline__ ContractCtx contract_ctx(const ContractArgs &A) {
    const int64_t b = A.cblk_base + blockIdx.x;
    const int inst = A.cblk_inst[b];
    ContractCtx c;
    c.I = A.inst + inst;
    c.chunk = b - c.I->cblk0;
    c.e0 = c.chunk * c.I->epc;
    c.eps = A.eps ? A.eps[inst] : 1.0f;
    return c;
}

// the block's loss sums (sum R^2, sum R A), wavefronts added in order -> its loss row
template <int NWV = kCWaves>
__device__ __forceinline__ void contract_flush(const ContractArgs &A, const ContractCtx &c, double lrr, double lra,
                                               double (*lp)[2], int tid, int wave, int lane) {
    const double vr = wave_sum(lrr), va = wave_sum(lra);
    if (lane == 0) {
        lp[wave][0] = vr;
        lp[wave][1] = va;
    }
    __syncthreads();
    if (tid < 4) {
        double v = 0.0;
        if (tid < 2)
            for (int w = 0; w < NWV; ++w) v += lp[w][tid];
        A.lpart[(c.I->lrow0 + c.I->gn_rows + c.chunk) * 4 + tid] = v;
    }
}

template <bool VAR>
__global__ __launch_bounds__(kCThreads) void k_contract_fast(ContractArgs A) {
    extern __shared__ float dyn[];
    __shared__ double lp[kCWaves][2];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const ContractCtx c = contract_ctx(A);
    const InstDesc *Ip = c.I;
    const int nq = Ip->nq, ntest = Ip->ntest;
    const int64_t e0 = c.e0;
    const int ne = (int)min((int64_t)Ip->epc, Ip->n_elem - e0);
    const float *__restrict__ Gx = Ip->Gx;
    const float *__restrict__ Gy = Ip->Gy;
    const float *__restrict__ F = Ip->F;
    const float two_cv = Ip->two_cv, eps = c.eps;
    // not restrict: unshared, the adjoint is written in place over these entries
    const float2 *ub = A.ubuf + Ip->ubase;
    double lrr = 0.0, lra = 0.0;
    float *cbuf = dyn;                  // [ntest][kCbs] per-point terms
    float *rbar = dyn + ntest * kCbs;   // [ne][ntest] 2 c_v R
    const int el = tid / nq, q = tid - el * nq;
    const bool act = el < ne;
    const int64_t gbase = (e0 + el) * Ip->gstride + q;
    const float *__restrict__ Mw = Ip->M;
    float gx[kKB], gy[kKB], gm[VAR ? kKB : 1];
#pragma unroll
    for (int k = 0; k < kKB; ++k) {
        const bool ok = act && k < ntest;
        gx[k] = ok ? Gx[gbase + (int64_t)k * nq] : 0.f;
        gy[k] = ok ? Gy[gbase + (int64_t)k * nq] : 0.f;
        if (VAR) gm[k] = ok ? Mw[gbase + (int64_t)k * nq] : 0.f;
    }
    const int64_t pi = (e0 + el) * nq + q;  // the thread's slot
    const int64_t pu = act ? upoint(Ip, pi) : 0;
    const float2 d = act ? ub[pu] : make_float2(0.f, 0.f);
    float ev = 0.f, bgu = 0.f;  // e_q and (b . grad u)_q
    if (VAR) {
        ev = act ? A.ebuf[Ip->ubase + pu] : 0.f;
        bgu = fmaf(Ip->cbx, d.x, Ip->cby * d.y);
    }
#pragma unroll
    for (int k = 0; k < kKB; ++k)
        if (k < ntest)
            cbuf[k * kCbs + tid] =
                VAR ? fmaf(ev, fmaf(d.x, gx[k], d.y * gy[k]), bgu * gm[k]) : fmaf(d.x, gx[k], d.y * gy[k]);
    __syncthreads();
    for (int r8 = tid; r8 < 8 * ne * ntest; r8 += kCThreads) {
        const int r = r8 >> 3, part = r8 & 7;
        const int e2 = r / ntest, k = r - e2 * ntest;
        const float *rowp = cbuf + k * kCbs + e2 * nq;
        float a = 0.f;
        for (int qq = part; qq < nq; qq += 8) a += rowp[qq];
        a += __shfl_xor(a, 4, 8);
        a += __shfl_xor(a, 2, 8);
        a += __shfl_xor(a, 1, 8);
        if (part == 0) {
            const float R = eps * a - F[(e0 + e2) * ntest + k];
            rbar[e2 * ntest + k] = two_cv * R;
            lrr += (double)R * (double)R;
            lra += (double)R * (double)a;
        }
    }
    __syncthreads();
    if (A.want_grad && act) {
        const float *rb = rbar + el * ntest;
        float bx = 0.f, by = 0.f, bm = 0.f;
#pragma unroll
        for (int k = 0; k < kKB; ++k)
            if (k < ntest) {
                bx = fmaf(rb[k], gx[k], bx);
                by = fmaf(rb[k], gy[k], by);
                if (VAR) bm = fmaf(rb[k], gm[k], bm);
            }
        if (VAR) {
            Ip->adj[pi] = make_float2(fmaf(ev, bx, Ip->cbx * bm), fmaf(ev, by, Ip->cby * bm));
            Ip->eadj[pi] = fmaf(d.x, bx, d.y * by);
        } else {
            Ip->adj[pi] = make_float2(eps * bx, eps * by);
        }
    }
    contract_flush(A, c, lrr, lra, lp, tid, wave, lane);
}

// row-streaming contraction of one element: wavefront w takes test-function rows
// k = w, w + kCWaves, ..., kRP rows per pass (a tuning choice) with all their loads in flight; a row's G values (lane holds q = lane + 64 i, i < Q) give A_k by
// a wavefront sum and then, still in registers, the row's share 2 c_v R_k G[k, q] of
// the adjoint; the wavefront partials are added in wavefront order at the end.
template <int Q, int kRP>
struct RowBuf {
    float gx[kRP][Q], gy[kRP][Q];
};

template <int Q, int kRP>
__device__ __forceinline__ void rows_load(RowBuf<Q, kRP> &B, const float *__restrict__ Gx, const float *__restrict__ Gy,
                                          int64_t gbase, int k0, int ntest, int nq, int lane) {
#pragma unroll
    for (int r = 0; r < kRP; ++r) {
        const int k = k0 + r * kCWaves;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int q = lane + 64 * i;
            const bool ok = k < ntest && q < nq;
            const int64_t o = gbase + (int64_t)k * nq + q;
            B.gx[r][i] = ok ? Gx[o] : 0.f;
            B.gy[r][i] = ok ? Gy[o] : 0.f;
        }
    }
}

template <int Q, int kRP>
__device__ __forceinline__ void rows_use(const RowBuf<Q, kRP> &B, const float *ux, const float *uy, float *bx, float *by,
                                         const float *__restrict__ F, int64_t ebase, int k0, int ntest, float eps,
                                         float two_cv, int lane, double &lrr, double &lra) {
#pragma unroll
    for (int r = 0; r < kRP; ++r) {
        const int k = k0 + r * kCWaves;
        float a = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) a = fmaf(ux[i], B.gx[r][i], fmaf(uy[i], B.gy[r][i], a));
        a = wave_sum(a);
        if (k < ntest) {
            const float R = eps * a - F[ebase + k];
            const float rb = two_cv * R;
            if (lane == 0) {
                lrr += (double)R * (double)R;
                lra += (double)R * (double)a;
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                bx[i] = fmaf(rb, B.gx[r][i], bx[i]);
                by[i] = fmaf(rb, B.gy[r][i], by[i]);
            }
        }
    }
}

template <int Q, int kRP>
__device__ __forceinline__ void contract_rows(const ContractArgs &A, const ContractCtx &c, float *bsum, int tid,
                                              int wave, int lane, double &lrr, double &lra) {
    const InstDesc *Ip = c.I;
    const int nq = Ip->nq, ntest = Ip->ntest;
    const float *__restrict__ Gx = Ip->Gx;
    const float *__restrict__ Gy = Ip->Gy;
    const float *__restrict__ F = Ip->F;
    const float two_cv = Ip->two_cv, eps = c.eps;
    // not restrict: unshared, the adjoint is written in place over these entries
    const float2 *ub = A.ubuf + Ip->ubase;
    const int64_t e0 = c.e0, ebase = e0 * ntest, gbase = e0 * Ip->gstride;
    float ux[Q], uy[Q], bx[Q], by[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int q = lane + 64 * i;
        const float2 d = q < nq ? ub[upoint(Ip, e0 * nq + q)] : make_float2(0.f, 0.f);
        ux[i] = d.x;
        uy[i] = d.y;
        bx[i] = 0.f;
        by[i] = 0.f;
    }
    // high occupancy (few registers a wavefront) keeps many rows in flight per SIMD
    constexpr int kStep = kRP * kCWaves;
    for (int k0 = wave; k0 < ntest; k0 += kStep) {
        RowBuf<Q, kRP> B;
        rows_load<Q, kRP>(B, Gx, Gy, gbase, k0, ntest, nq, lane);
        rows_use<Q, kRP>(B, ux, uy, bx, by, F, ebase, k0, ntest, eps, two_cv, lane, lrr, lra);
    }
    if (A.want_grad) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            bsum[((wave * 2 + 0) * Q + i) * 64 + lane] = bx[i];
            bsum[((wave * 2 + 1) * Q + i) * 64 + lane] = by[i];
        }
        __syncthreads();
        for (int t = tid; t < Q * 64; t += kCThreads) {
            const int i = t >> 6, l = t & 63, q = l + 64 * i;
            if (q < nq) {
                float sx = 0.f, sy = 0.f;
                for (int w = 0; w < kCWaves; ++w) {
                    sx += bsum[((w * 2 + 0) * Q + i) * 64 + l];
                    sy += bsum[((w * 2 + 1) * Q + i) * 64 + l];
                }
                Ip->adj[e0 * nq + q] = make_float2(eps * sx, eps * sy);
            }
        }
    }
}

template <int Q, int RP>
__global__ __launch_bounds__(kCThreads) void k_contract_rows(ContractArgs A) {
    __shared__ float bsum[kCWaves * 2 * Q * 64];
    __shared__ double lp[kCWaves][2];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const ContractCtx c = contract_ctx(A);
    double lrr = 0.0, lra = 0.0;
    contract_rows<Q, RP>(A, c, bsum, tid, wave, lane, lrr, lra);
    contract_flush(A, c, lrr, lra, lp, tid, wave, lane);
}

// Large elements (N_quad > 256) in two launches, so that any number of blocks share an
// element and a problem of one large element still fills the chip.  k_split_rows: block
// (element, 16 test-function rows, kSplitQ points), a wavefront per row, sixteen points a
// lane with every load issued before the products, the lane sums added by a fixed
// butterfly -> partial row sums apart[e][point block][k].  k_split_adj: block (element,
// 64 x 16 / kw points) adds an element's partials in point-block order, forms R = eps A - F,
// 2 c_v R and (in the element's first block only) the loss terms, then the adjoint of its
// points: the 16 wavefronts form groups of kw, each group 64 points with the test functions
// split over its kw wavefronts, whose sums are added in order (kw grows with the test
// count, and with the blocks a small problem needs).  The adjoint is written over the point
// buffer, whose readers (the row sums) have finished.
constexpr int kSplitQ = 64 * 16;

__global__ __launch_bounds__(kGThreads) void k_split_rows(ContractArgs A, const int *__restrict__ rblk_inst,
                                                          float *__restrict__ apart) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b = blockIdx.x;
    const InstDesc *Ip = A.inst + rblk_inst[b];
    const int nq = Ip->nq, ntest = Ip->ntest, nkb = Ip->nkb, nqb = Ip->nqb;
    const int64_t r = b - Ip->rblk0;
    const int qb = (int)(r % nqb), kb = (int)((r / nqb) % nkb);
    const int64_t e = r / ((int64_t)nqb * nkb);
    const int k = kb * kGWaves + wave;
    if (k >= ntest) return;  // whole wavefronts; nothing below synchronises the block
    const int64_t gbase = e * Ip->gstride;
    const float *gxr = Ip->Gx + gbase + (int64_t)k * nq, *gyr = Ip->Gy + gbase + (int64_t)k * nq;
    const float2 *ub = A.ubuf + Ip->ubase;
    const int q0 = qb * kSplitQ, q1 = min(nq, q0 + kSplitQ);
    float2 d[16];
    float gx[16], gy[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = q0 + lane + 64 * i;
        const bool ok = q < q1;
        d[i] = ok ? ub[upoint(Ip, e * nq + q)] : make_float2(0.f, 0.f);
        gx[i] = ok ? gxr[q] : 0.f;
        gy[i] = ok ? gyr[q] : 0.f;
    }
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc = fmaf(d[i].x, gx[i], fmaf(d[i].y, gy[i], acc));
    acc = wave_sum(acc);
    if (lane == 0) apart[Ip->abase + (e * nqb + qb) * ntest + k] = acc;
}

__global__ __launch_bounds__(kGThreads) void k_split_adj(ContractArgs A, const float *__restrict__ apart) {
    extern __shared__ float dyn[];
    __shared__ double lp[kGWaves][2];
    __shared__ float2 red[kGWaves][64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const ContractCtx c = contract_ctx(A);
    const InstDesc *Ip = c.I;
    const int nq = Ip->nq, ntest = Ip->ntest, npb = Ip->npb, nqb = Ip->nqb;
    const int64_t e = c.chunk / npb;
    const int pb = (int)(c.chunk % npb);
    const float two_cv = Ip->two_cv, eps = c.eps;
    float *rbar = dyn;  // [ntest] 2 c_v R of the element
    double lrr = 0.0, lra = 0.0;
    const float *ap = apart + Ip->abase + e * nqb * ntest;
    for (int k = tid; k < ntest; k += kGThreads) {
        float a = 0.f;
        for (int j = 0; j < nqb; ++j) a += ap[(int64_t)j * ntest + k];
        const float R = eps * a - Ip->F[e * ntest + k];
        rbar[k] = two_cv * R;
        if (pb == 0) {
            lrr += (double)R * (double)R;
            lra += (double)R * (double)a;
        }
    }
    __syncthreads();
    if (A.want_grad) {
        const int kw = Ip->kw, pg = wave / kw, ks = wave - pg * kw;
        const int q = pb * (64 * (kGWaves / kw)) + pg * 64 + lane;
        const int kc = (ntest + kw - 1) / kw;
        const int k0 = min(ntest, ks * kc), k1 = min(ntest, k0 + kc);
        float bx = 0.f, by = 0.f;
        if (q < nq) {
            const int64_t gbase = e * Ip->gstride;
            int k = k0;
            for (; k + 7 < k1; k += 8) {
                float gx[8], gy[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int64_t o = gbase + (int64_t)(k + i) * nq + q;
                    gx[i] = Ip->Gx[o];
                    gy[i] = Ip->Gy[o];
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    bx = fmaf(rbar[k + i], gx[i], bx);
                    by = fmaf(rbar[k + i], gy[i], by);
                }
            }
            for (; k < k1; ++k) {
                const int64_t o = gbase + (int64_t)k * nq + q;
                bx = fmaf(rbar[k], Ip->Gx[o], bx);
                by = fmaf(rbar[k], Ip->Gy[o], by);
            }
        }
        red[wave][lane] = make_float2(bx, by);
        __syncthreads();
        if (ks == 0 && q < nq) {
            float sx = 0.f, sy = 0.f;
            for (int w = wave; w < wave + kw; ++w) {
                sx += red[w][lane].x;
                sy += red[w][lane].y;
            }
            Ip->adj[e * nq + q] = make_float2(eps * sx, eps * sy);
        }
    }
    contract_flush<kGWaves>(A, c, lrr, lra, lp, tid, wave, lane);
}

// Matrix-free contraction: no stored G; one wavefront per element rebuilds it from
// the element's bilinear map by sum factorisation.  With v_k = phi_r(xi) phi_s(eta)
// (k = s N_t + r), Jacobian entries a, b, c, d at point (i, j) and w = w_i w_j,
//   sum_q (u_x G_x + u_y G_y)[k, q]
//     = sum_{i,j} P_ij phi_r'(xi_i) phi_s(eta_j) + Q_ij phi_r(xi_i) phi_s'(eta_j),
//   P = kd w (d u_x - c u_y),  Q = kd w (a u_y - b u_x),
// kd the constant diffusion coefficient (or e_q of a space-dependent one); the
// convection term adds Mq = w det J (b . grad u) against phi_r phi_s.  Each double
// sum runs along xi first (N_t n partial sums per array, in LDS), then along eta:
// 2 (N_t n^2 + N_t^2 n) multiply-adds an element instead of 2 N_t^2 n^2, and no G
// from HBM.  The adjoint applies the transposed transforms to 2 c_v R.
template <bool VAR>
__global__ __launch_bounds__(kCThreads) void k_contract_mf(ContractArgs A) {
    extern __shared__ float dyn[];
    __shared__ double lp[kCWaves][2];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const ContractCtx c = contract_ctx(A);
    const InstDesc *Ip = c.I;
    const int n = Ip->qn, nt = Ip->tn, nq = n * n, ntest = nt * nt, nn = nt * n;
    const int ntab = 2 * n + 2 * nn;
    float *tab = dyn;  // nodes [n], weights [n], phi [nt][n], phi' [nt][n]
    for (int t = tid; t < ntab; t += kCThreads) tab[t] = Ip->tab[t];
    const float *xg = tab, *wg = tab + n, *ph = tab + 2 * n, *dph = tab + 2 * n + nn;
    // per wavefront: P, Q, Mq [nq] | V, W [nt][n] (then the adjoint's X1, X2) | 2 c_v R [ntest]
    float *Pv = dyn + ntab + wave * (3 * nq + 2 * nn + ntest);
    float *Qv = Pv + nq, *Mv = Qv + nq, *Vv = Mv + nq, *Wv = Vv + nn, *rb = Wv + nn;
    __syncthreads();
    const int64_t e = c.e0 + wave;
    double lrr = 0.0, lra = 0.0;
    if (e < Ip->n_elem) {
        const float *gp = Ip->geo + e * 8;
        const float x1 = gp[0], x2 = gp[1], x3 = gp[2], y1 = gp[3], y2 = gp[4], y3 = gp[5];
        const float eps = c.eps, two_cv = Ip->two_cv, kdiff = Ip->kdiff, cbx = Ip->cbx, cby = Ip->cby;
        // not restrict: unshared, adj and eadj are these buffers
        const float2 *ub = A.ubuf + Ip->ubase;
        const float *eb = VAR ? A.ebuf + Ip->ubase : nullptr;
        float2 *adj = Ip->adj + e * nq;
        float *eadj = VAR ? Ip->eadj + e * nq : nullptr;
        // Jacobian entries and weight at point q = j n + i
        auto geom = [&](int q, float &a, float &b, float &cc, float &d, float &w) {
            const int j = q / n, i = q - j * n;
            const float xi = xg[i], eta = xg[j];
            w = wg[i] * wg[j];
            a = fmaf(x3, eta, x1);
            b = fmaf(y3, eta, y1);
            cc = fmaf(x3, xi, x2);
            d = fmaf(y3, xi, y2);
        };
        for (int q = lane; q < nq; q += 64) {
            float a, b, cc, d, w;
            geom(q, a, b, cc, d, w);
            const int64_t pu = upoint(Ip, e * nq + q);
            const float2 g = ub[pu];
            const float kd = VAR ? eb[pu] : kdiff;
            Pv[q] = kd * w * (d * g.x - cc * g.y);
            Qv[q] = kd * w * (a * g.y - b * g.x);
            Mv[q] = w * (a * d - b * cc) * fmaf(cbx, g.x, cby * g.y);
        }
        wave_sync();
        // along xi: V[r][j] = sum_i P_ij phi_r'(xi_i) + Mq_ij phi_r(xi_i),  W[r][j] = sum_i Q_ij phi_r(xi_i)
        for (int t = lane; t < nn; t += 64) {
            const int r = t / n, j = t - r * n;
            const float *pr = ph + r * n, *dpr = dph + r * n;
            const float *Pj = Pv + j * n, *Qj = Qv + j * n, *Mj = Mv + j * n;
            float v = 0.f, wv = 0.f;
            for (int i = 0; i < n; ++i) {
                v = fmaf(Pj[i], dpr[i], fmaf(Mj[i], pr[i], v));
                wv = fmaf(Qj[i], pr[i], wv);
            }
            Vv[t] = v;
            Wv[t] = wv;
        }
        wave_sync();
        // along eta: A_k = sum_j V[r][j] phi_s(eta_j) + W[r][j] phi_s'(eta_j)
        const float *__restrict__ F = Ip->F + e * ntest;
        for (int k = lane; k < ntest; k += 64) {
            const int s = k / nt, r = k - s * nt;
            const float *Vr = Vv + r * n, *Wr = Wv + r * n, *ps = ph + s * n, *dps = dph + s * n;
            float a = 0.f;
            for (int j = 0; j < n; ++j) a = fmaf(Vr[j], ps[j], fmaf(Wr[j], dps[j], a));
            const float R = eps * a - F[k];
            rb[k] = two_cv * R;
            lrr += (double)R * (double)R;
            lra += (double)R * (double)a;
        }
        if (A.want_grad) {
            wave_sync();
            // transposed, along eta: X1[r][j] = sum_s rb_rs phi_s(eta_j), X2[r][j] = sum_s rb_rs phi_s'(eta_j)
            for (int t = lane; t < nn; t += 64) {
                const int r = t / n, j = t - r * n;
                float s1 = 0.f, s2 = 0.f;
                for (int s = 0; s < nt; ++s) {
                    const float rv = rb[s * nt + r];
                    s1 = fmaf(rv, ph[s * n + j], s1);
                    s2 = fmaf(rv, dph[s * n + j], s2);
                }
                Vv[t] = s1;
                Wv[t] = s2;
            }
            wave_sync();
            // along xi at each point: S_xi = sum_r phi_r'(xi_i) X1, S_eta = sum_r phi_r(xi_i) X2,
            // S_v = sum_r phi_r(xi_i) X1; then dL/du = eps (kd (G_x, G_y)-sums + b Mq-sum)
            for (int q = lane; q < nq; q += 64) {
                float a, b, cc, d, w;
                geom(q, a, b, cc, d, w);
                const int j = q / n, i = q - j * n;
                float sxi = 0.f, seta = 0.f, sv = 0.f;
                for (int r = 0; r < nt; ++r) {
                    const float x1v = Vv[r * n + j], x2v = Wv[r * n + j], p = ph[r * n + i];
                    sxi = fmaf(dph[r * n + i], x1v, sxi);
                    seta = fmaf(p, x2v, seta);
                    sv = fmaf(p, x1v, sv);
                }
                const float gx = w * (d * sxi - b * seta), gy = w * (a * seta - cc * sxi);
                const float gm = w * (a * d - b * cc) * sv;
                const int64_t pu = upoint(Ip, e * nq + q);
                const float2 g = ub[pu];
                const float kd = VAR ? eb[pu] : kdiff;
                adj[q] = make_float2(eps * fmaf(kd, gx, cbx * gm), eps * fmaf(kd, gy, cby * gm));
                if (VAR) eadj[q] = fmaf(g.x, gx, g.y * gy);
            }
        }
    }
    contract_flush(A, c, lrr, lra, lp, tid, wave, lane);
}

// one wavefront's gradient sums in padded order -> P (op: store, or add to what P holds).
// padb: the biases of layers 2..L are column 31 of the weight-gradient tiles (tile_backward)
template <int L, bool ADD, int NH>
__device__ __forceinline__ void put_partial(float *P, const GradAcc<L> &G, const float (*VA)[64], int lane,
                                            bool padb) {
    const int g = lane >> 4, c = lane & 15, hi = lane ^ 32;
    const bool lo = lane < 32;
    constexpr int NW = 16 * (L > 1 ? L - 1 : 0);
    float cw[NW > 0 ? NW : 1], cv[L + 3], cb = 0.f;
#pragma unroll
    for (int i = 0; i < (NW > 0 ? NW : 1); ++i) cw[i] = 0.f;
#pragma unroll
    for (int i = 0; i < L + 3; ++i) cv[i] = 0.f;
    if (ADD) {
#pragma unroll
        for (int l = 2; l <= L; ++l)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    cw[16 * (l - 2) + 4 * t + r] = P[off_w(l) + (16 * (t >> 1) + 4 * g + r) * PW + 16 * (t & 1) + c];
        if (lo) {
#pragma unroll
            for (int l = 1; l <= L; ++l) cv[l - 1] = P[off_b(l) + lane];
            cv[L] = P[off_w(1) + 2 * lane];
            cv[L + 1] = P[off_w(1) + 2 * lane + 1];
            cv[L + 2] = P[off_wout(L) + lane];
        }
        if (lane == 0) cb = P[off_wout(L) + PW];
    }
    float cw2 = 0.f, cb2 = 0.f;
    if (ADD && NH == 2) {
        if (lo) cw2 = P[off_wout2(L) + lane];
        if (lane == 0) cb2 = P[off_wout2(L) + PW];
    }
    const float bo = wave_sum(VA[L + 3][lane]);
    const float bo2 = NH == 2 ? wave_sum(VA[NH == 2 ? L + 5 : 0][lane]) : 0.f;
    // the partner's sum comes first, so the pair adds as (lower wave) + (upper wave)
#pragma unroll
    for (int l = 2; l <= L; ++l)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                P[off_w(l) + (16 * (t >> 1) + 4 * g + r) * PW + 16 * (t & 1) + c] =
                    ADD ? G.w[l - 2][t][r] + cw[16 * (l - 2) + 4 * t + r] : G.w[l - 2][t][r];
    if (padb && c == 15) {
        // column 31 (t odd, c = 15) of layer l's tile is db_l at row 16 (t >> 1) + 4 g + r
#pragma unroll
        for (int l = 2; l <= L; ++l)
#pragma unroll
            for (int t = 1; t < 4; t += 2)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float *d = P + off_b(l) + 16 * (t >> 1) + 4 * g + r;
                    *d = ADD ? G.w[l - 2][t][r] + *d : G.w[l - 2][t][r];
                }
    }
    if (lo) {
#pragma unroll
        for (int l = 1; l <= L; ++l) {
            if (padb && l >= 2) continue;
            const float v = VA[l - 1][lane] + VA[l - 1][hi];
            P[off_b(l) + lane] = ADD ? v + cv[l - 1] : v;
        }
        const float v0 = VA[L][lane] + VA[L][hi], v1 = VA[L + 1][lane] + VA[L + 1][hi];
        const float vo = VA[L + 2][lane] + VA[L + 2][hi];
        P[off_w(1) + 2 * lane] = ADD ? v0 + cv[L] : v0;
        P[off_w(1) + 2 * lane + 1] = ADD ? v1 + cv[L + 1] : v1;
        P[off_wout(L) + lane] = ADD ? vo + cv[L + 2] : vo;
    }
    if (lane == 0) P[off_wout(L) + PW] = ADD ? bo + cb : bo;
    if (NH == 2) {
        if (lo) {
            const float v2 = VA[NH == 2 ? L + 4 : 0][lane] + VA[NH == 2 ? L + 4 : 0][hi];
            P[off_wout2(L) + lane] = ADD ? v2 + cw2 : v2;
        }
        if (lane == 0) P[off_wout2(L) + PW] = ADD ? bo2 + cb2 : bo2;
    }
}

// the block's gradient sums for one instance -> gradient row `row`; accumulators reset.
// Fixed order ((w0 + w1) + (w2 + w3)) + ((w4 + w5) + (w6 + w7)): odd wavefronts store
// into four LDS regions (red, and three over the transpose tiles, idle here), even ones
// add theirs, and the four regions are added on the way out.
template <int L, int NH, class SH>
__device__ __forceinline__ void flush_grad(SH &S, float *gpart, int64_t row, GradAcc<L> &G, int tid, int wave,
                                           int lane, bool padb) {
    static_assert(kBWaves == 8, "pairwise flush assumes eight wavefronts");
    float *mine = (wave >> 1) == 0 ? S.red : S.part[(wave >> 1) - 1];
    __syncthreads();
    if (wave & 1) put_partial<L, false, NH>(mine, G, S.vacc[wave], lane, padb);
    __syncthreads();
    if (!(wave & 1)) put_partial<L, true, NH>(mine, G, S.vacc[wave], lane, padb);
    __syncthreads();
    for (int j = tid; j < n_pad_h(L, NH); j += kBThreads)
        gpart[row * kMaxPadded + j] = (S.red[j] + S.part[0][j]) + (S.part[1][j] + S.part[2][j]);
    zero_acc<L>(G);
    for (int t = tid; t < kBWaves * n_vslots(L, NH) * 64; t += kBThreads) (&S.vacc[0][0][0])[t] = 0.f;
    __syncthreads();
}

// 4: reverse sweep, tiles of 16 points spread evenly over all wavefronts; the
// forward pass of each tile is recomputed (tanh included) and kept in registers
template <int L, int NH, bool LOADA>
__global__ __launch_bounds__(kBThreads, 1) void k_bwd(BwdArgs A) {
    __shared__ BwdShared<L, NH> S;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    float(*T0)[kTs] = S.tt[wave][0];
    float(*T1)[kTs] = S.tt[wave][1];
    GradAcc<L> G;
    zero_acc<L>(G);
    for (int t = tid; t < kBWaves * n_vslots(L, NH) * 64; t += kBThreads) (&S.vacc[0][0][0])[t] = 0.f;
    int64_t t = A.blk_tiles[blockIdx.x];
    const int64_t t_blk = t;
    const int64_t t_end = A.blk_tiles[blockIdx.x + 1];
    int cur = A.blk_inst0[blockIdx.x];
    while (t < t_end) {
        // only the fields the tile loop needs (the whole descriptor would pin registers)
        const InstDesc *Ip = A.inst + cur;
        const int64_t tile0 = Ip->tile0, n_pts = Ip->n_pts, n_all = Ip->n_pts + Ip->n_bnd + Ip->n_sen;
        const float2 *__restrict__ pts = Ip->pts;
        const float2 *__restrict__ ub_i = A.ubuf + Ip->ubase;
        const float *__restrict__ eb_i = NH == 2 ? A.ebuf + Ip->ubase : nullptr;
        // shared points: the adjoints of a point's slots are added in slot order
        const int *__restrict__ usoff = Ip->usoff;
        const int *__restrict__ uslot = Ip->uslot;
        const float2 *__restrict__ adj = Ip->adj;
        const float *__restrict__ eadj = Ip->eadj;
        const int64_t seg_end = min(t_end, tile0 + Ip->n_tiles);
        const int64_t row = Ip->grow0 + (int64_t)(blockIdx.x - Ip->gblk0);
        __syncthreads();
        load_weights<L, kBThreads, NH>(S.W, S.red, A.params + (int64_t)cur * A.param_stride, A.H, tid);
        __syncthreads();
        // the next tile's point and adjoint are loaded while this tile computes
        auto fetch = [&](int64_t tt, float2 &p, float2 &d, float &ev) {
            const int64_t idx = 16 * (tt - tile0) + (lane & 15);
            const bool ok = tt < seg_end && idx < n_all;
            p = ok ? pts[idx] : make_float2(0.f, 0.f);
            if (usoff && ok && idx < n_pts) {
                d = make_float2(0.f, 0.f);
                ev = 0.f;
                for (int k = usoff[idx], k1 = usoff[idx + 1]; k < k1; ++k) {
                    const int s = uslot[k];
                    const float2 a = adj[s];
                    d.x += a.x;
                    d.y += a.y;
                    if (NH == 2) ev += eadj[s];
                }
            } else {
                d = ok ? ub_i[idx] : make_float2(0.f, 0.f);
                ev = (NH == 2 && ok && idx < n_pts) ? eb_i[idx] : 0.f;
            }
        };
        float2 pn, dn;
        float en;
        // the block's tiles go round-robin over its wavefronts, continuing across instances
        const int64_t first = t + (int64_t)((wave - (int)((t - t_blk) % kBWaves) + kBWaves) % kBWaves);
        fetch(first, pn, dn, en);
        for (int64_t tt = first; tt < seg_end; tt += kBWaves) {
            const int64_t idx = 16 * (tt - tile0) + (lane & 15);
            const float2 p = pn, d = dn;
            const float eb = en;
            fetch(tt + kBWaves, pn, dn, en);
            const bool interior = idx < n_pts;
            const float ub = interior ? 0.f : d.x, uxb = interior ? d.x : 0.f, uyb = interior ? d.y : 0.f;
            Acts<L> K;
            if (LOADA) {
                tile_forward_loaded<L>(S.W, lane, A.act + tt * (int64_t)(L * kActTile), K);
            } else {
                Vec a, tx, ty;
                tile_forward<L, true>(S.W, lane, p.x, p.y, a, tx, ty, K);
            }
            tile_backward<L, NH>(S.W, T0, T1, lane, p.x, p.y, ub, uxb, uyb, eb, K, G, S.vacc[wave], A.H < PW);
        }
        flush_grad<L, NH>(S, A.gpart, row, G, tid, wave, lane, A.H < PW);
        t = seg_end;
        ++cur;
    }
}

// ---------------------------------------------------------------------------
// one launch for the forward pass, the contraction and the reverse sweep (the
// one-pass tuning): a block of eight wavefronts owns groups of whole elements of
// at most kGroupPts points, one 16-point tile per wavefront, and keeps each tile's
// forward state (activations and post-activation tangents) in registers through
// the contraction of its elements, so the reverse sweep starts from it: no forward
// recomputation, no point buffer, no separate contraction launch.  Boundary and
// sensor points come in groups of their own (mismatch terms, no contraction).
// The contraction of a group: lane (point j, slice g) holds G_x, G_y of its point
// for test functions k = g, g + 4, ... (loaded before the forward products, so
// their latency hides behind them); the per-point terms go through LDS to
// per-(element, test) row sums, eight lanes a row, added in a fixed order; 2 c_v R
// comes back through LDS and each lane forms its slice of the adjoint, the four
// slices added across lanes.  Limits: N_quad <= kGroupPts, N_test <= kKB, one
// network output, no shared points, stored G.
// ---------------------------------------------------------------------------
constexpr int kGroupPts = 16 * kBWaves;          // points of a group: one tile per wavefront
constexpr int kGroupMaxElem = kGroupPts / 4;     // elements of a group (N_quad >= 4)
constexpr int kSlice = kKB / 4;                  // test functions a lane holds

struct GroupDesc {
    int64_t p0;  // first point of the group in the instance's point list
    int64_t e0;  // first element (interior groups)
    int np;      // points
    int ne;      // elements; 0: boundary and sensor points
};

struct StepArgs {
    const InstDesc *inst;
    const GroupDesc *grp;
    const int64_t *blk_grp;   // [blocks + 1] group range of each block
    const int *blk_inst0;     // instance of each block's first group
    const float *params;
    int64_t param_stride;
    int H;
    const float *eps;         // [n_inst] or null (eps = 1)
    int want_grad;
    float *gpart;
    double *lpart;
    int64_t *step;            // optional step counter, incremented once per launch
};

template <int L>
struct StepShared {
    WeightsShared<L> W;
    union {
        float tt[kBWaves][2][16][kTs];
        float part[3][n_pad_h(L, 1)];
    };
    float vacc[kBWaves][n_vslots(L, 1)][64];
    float red[n_pad_h(L, 1)];
    float cs[kGroupPts][kKB + 1];    // per-point terms u_x G_x + u_y G_y, by test function
    float rb[kGroupMaxElem][kKB];    // 2 c_v R of the group's elements
    float fs[kGroupMaxElem * kKB];   // F of the group's elements, [element][test]
    // per-wavefront loss sums of the current instance (sum R^2, sum R A, boundary, sensor),
    // one wavefront sum added per group, in group order
    double lp[kBWaves][4];
};

// add this lane's loss terms of one group to its wavefront's running sums (lane 0 writes)
__device__ __forceinline__ void add_loss(double (*lp)[4], int wave, int lane, int slot, double v0, double v1) {
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    if (lane == 0) {
        lp[wave][slot] += v0;
        lp[wave][slot + 1] += v1;
    }
}

template <int L>
__global__ __launch_bounds__(kBThreads, 1) void k_step(StepArgs A) {
    __shared__ StepShared<L> S;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int j = lane & 15, gq = lane >> 4;
    const int pl = 16 * wave + j;  // the lane's point within a group
    if (A.step && blockIdx.x == 0 && tid == 0) *A.step += 1;
    float(*T0)[kTs] = S.tt[wave][0];
    float(*T1)[kTs] = S.tt[wave][1];
    GradAcc<L> G;
    zero_acc<L>(G);
    for (int t = tid; t < kBWaves * n_vslots(L, 1) * 64; t += kBThreads) (&S.vacc[0][0][0])[t] = 0.f;
    int64_t g = A.blk_grp[blockIdx.x];
    const int64_t g_end = A.blk_grp[blockIdx.x + 1];
    int cur = A.blk_inst0[blockIdx.x];
    while (g < g_end) {
        const InstDesc *Ip = A.inst + cur;
        const int64_t seg_end = min(g_end, Ip->grp0 + Ip->n_grp);
        const int64_t n_pts = Ip->n_pts, n_bnd = Ip->n_bnd;
        const float2 *__restrict__ pts = Ip->pts;
        const float *__restrict__ tgt = Ip->tgt;
        const float *__restrict__ Gx = Ip->Gx;
        const float *__restrict__ Gy = Ip->Gy;
        const float *__restrict__ F = Ip->F;
        const int nq = Ip->nq, ntest = Ip->ntest;
        const int64_t gstride = Ip->gstride;
        const float two_cv = Ip->two_cv, wb2 = Ip->wb2, ws2 = Ip->ws2;
        const float eps = A.eps ? A.eps[cur] : 1.0f;
        const int64_t rel = (int64_t)(blockIdx.x - Ip->gblk0);
        __syncthreads();
        load_weights<L, kBThreads, 1>(S.W, S.red, A.params + (int64_t)cur * A.param_stride, A.H, tid);
        if (tid < kBWaves * 4) (&S.lp[0][0])[tid] = 0.0;
        __syncthreads();
        // the next group's point is loaded while this group computes
        auto fetch = [&](int64_t gg) -> float2 {
            if (gg >= seg_end) return make_float2(0.f, 0.f);
            const GroupDesc D = A.grp[gg];
            return pl < D.np ? pts[D.p0 + pl] : make_float2(0.f, 0.f);
        };
        float2 xyn = fetch(g);
        for (; g < seg_end; ++g) {
            const GroupDesc D = A.grp[g];
            const bool valid = pl < D.np;
            const bool active = 16 * wave < D.np;  // uniform in the wavefront
            const bool interior = D.ne > 0;        // uniform in the block
            const float2 xy = xyn;
            const int el = interior ? pl / nq : 0, q = pl - el * nq;
            float gx[kSlice], gy[kSlice];
            const int64_t gb = (D.e0 + el) * gstride + q;
#pragma unroll
            for (int t = 0; t < kSlice; ++t) {
                const int k = gq + 4 * t;
                const bool ok = interior && valid && k < ntest;
                gx[t] = ok ? Gx[gb + (int64_t)k * nq] : 0.f;
                gy[t] = ok ? Gy[gb + (int64_t)k * nq] : 0.f;
            }
            xyn = fetch(g + 1);
            // the group's rows of F (contiguous), loaded now and staged in LDS after the forward pass
            constexpr int kFr = kGroupMaxElem * kKB / kBThreads;
            float fr[kFr];
#pragma unroll
            for (int i = 0; i < kFr; ++i) {
                const int f = tid + i * kBThreads;
                fr[i] = (interior && f < D.ne * ntest) ? F[D.e0 * ntest + f] : 0.f;
            }
            Acts<L> K;
            float u = 0.f, ux = 0.f, uy = 0.f;
            if (active) {
                Vec a, tx, ty;
                tile_forward<L, true>(S.W, lane, xy.x, xy.y, a, tx, ty, K);
                tile_outputs<L>(S.W, lane, a, tx, ty, u, ux, uy);
            }
            float ub = 0.f, uxb = 0.f, uyb = 0.f;
            if (interior) {
#pragma unroll
                for (int t = 0; t < kSlice; ++t) {
                    const int k = gq + 4 * t;
                    if (valid && k < ntest) S.cs[pl][k] = fmaf(ux, gx[t], uy * gy[t]);
                }
#pragma unroll
                for (int i = 0; i < kFr; ++i) {
                    const int f = tid + i * kBThreads;
                    if (f < D.ne * ntest) S.fs[f] = fr[i];
                }
                __syncthreads();
                double lrr = 0.0, lra = 0.0;
                for (int r8 = tid; r8 < 8 * D.ne * ntest; r8 += kBThreads) {
                    const int r = r8 >> 3, part = r8 & 7;
                    const int e2 = r / ntest, k = r - e2 * ntest;
                    float a = 0.f;
                    for (int qq = part; qq < nq; qq += 8) a += S.cs[e2 * nq + qq][k];
                    a += __shfl_xor(a, 4, 8);
                    a += __shfl_xor(a, 2, 8);
                    a += __shfl_xor(a, 1, 8);
                    if (part == 0) {
                        const float R = eps * a - S.fs[e2 * ntest + k];
                        S.rb[e2][k] = two_cv * R;
                        lrr += (double)R * (double)R;
                        lra += (double)R * (double)a;
                    }
                }
                add_loss(S.lp, wave, lane, 0, lrr, lra);
                __syncthreads();
                // dL/du_x = eps sum_k 2 c_v R_k G_x[k, q]: this lane's slice, then the four slices
                float bx = 0.f, by = 0.f;
#pragma unroll
                for (int t = 0; t < kSlice; ++t) {
                    const int k = gq + 4 * t;
                    if (k < ntest) {
                        const float rk = S.rb[el][k];
                        bx = fmaf(rk, gx[t], bx);
                        by = fmaf(rk, gy[t], by);
                    }
                }
                bx = group_sum(bx);
                by = group_sum(by);
                if (valid) {
                    uxb = eps * bx;
                    uyb = eps * by;
                }
            } else {
                // boundary (Sec. 2.3) or sensor (Sec. 4.7) mismatch: loss term and its adjoint
                double lbb = 0.0, lss = 0.0;
                if (valid) {
                    const int64_t xi = D.p0 + pl - n_pts;
                    const float d = u - tgt[xi];
                    const bool bnd = xi < n_bnd;
                    if (gq == 0) {
                        if (bnd) lbb = (double)d * (double)d;
                        else lss = (double)d * (double)d;
                    }
                    ub = (bnd ? wb2 : ws2) * d;
                }
                add_loss(S.lp, wave, lane, 2, lbb, lss);
            }
            if (A.want_grad && active)
                tile_backward<L, 1>(S.W, T0, T1, lane, xy.x, xy.y, ub, uxb, uyb, 0.f, K, G, S.vacc[wave],
                                    A.H < PW);
        }
        // the block's loss sums for this instance, wavefronts added in order -> its loss row
        __syncthreads();
        if (tid < 4) {
            double v = 0.0;
            for (int w = 0; w < kBWaves; ++w) v += S.lp[w][tid];
            A.lpart[(Ip->lrow0 + rel) * 4 + tid] = v;
        }
        if (A.want_grad) flush_grad<L, 1>(S, A.gpart, Ip->grow0 + rel, G, tid, wave, lane, A.H < PW);
        ++cur;
    }
}

// ---------------------------------------------------------------------------
// fixed-order reduction of the block partials into the outputs, one instance
// per blockIdx.y; optionally followed by Adam (Kingma and Ba, Algorithm 1) on
// that instance's parameters with the step count read from device memory
// ---------------------------------------------------------------------------
// block = 64 columns (one per lane) x 16 wavefronts: wavefront w sums rows w,
// w + 16, ... of its lane's column in order, then a column's 16 wavefront sums
// are added in wavefront order.  Loss rows: the x = 0 block spreads them over
// all its threads (thread i sums rows i, i + 1024, ...), adds each wavefront's
// values with a fixed butterfly and the 16 wavefront sums in order.  The order
// is fixed for a given plan, so results are bitwise reproducible.
constexpr int kFinCols = 64, kFinWaves = 16, kFinThreads = kFinCols * kFinWaves;
constexpr int kFinBatch = 16;  // row loads in flight per lane
struct AdamArgs {
    float *params, *m, *v;
    const int64_t *step;
    float lr, b1, b2, eps;
    // optional: a trainable diffusion coefficient per instance and its moments, updated
    // with the same hyperparameters from dL/deps = 2 c_v sum R A
    float *ep, *em, *ev;
};

// one bias-corrected Adam update (Kingma and Ba, Algorithm 1) of a single value
__device__ __forceinline__ void adam_one(float &p, float &m, float &v, float g, float t, const AdamArgs &ad) {
    const float c1 = 1.0f - powf(ad.b1, t), c2 = 1.0f - powf(ad.b2, t);
    m = fmaf(ad.b1, m, (1.0f - ad.b1) * g);
    v = fmaf(ad.b2, v, (1.0f - ad.b2) * g * g);
    p = p - ad.lr * (m / c1) / (sqrtf(v / c2) + ad.eps);
}

template <int L, int NH>
__global__ __launch_bounds__(kFinThreads) void k_fused_final(
    const InstDesc *__restrict__ inst, const float *__restrict__ gpart, const double *__restrict__ lpart, int H,
    int64_t npf, float *__restrict__ loss_out, float *__restrict__ grad_out, float *__restrict__ grad_eps_out,
    AdamArgs ad) {
    __shared__ float part[kFinWaves][kFinCols];
    __shared__ double lred[kFinWaves][4];
    const int ii = blockIdx.y;
    const InstDesc &I = inst[ii];
    const int rows = I.gn_rows, lrows = I.ln_rows;
    const float *gp = gpart + (int64_t)I.grow0 * kMaxPadded;
    const double *lp = lpart + (int64_t)I.lrow0 * 4;
    const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * kFinCols + c;
    const bool want = (grad_out || ad.params) && j < npf;
    int pj = -1;  // padded index of flat parameter j
    if (want) {
        if (j < 2 * H) pj = (int)j;
        else if (j < 3 * H) pj = kOffB1 + (int)(j - 2 * H);
        else {
            const int64_t lay = (int64_t)H * H + H, r0 = j - 3 * H;
            if (r0 < (int64_t)(L - 1) * lay) {
                const int l = 2 + (int)(r0 / lay), r = (int)(r0 % lay);
                pj = r < H * H ? off_w(l) + (r / H) * PW + (r % H) : off_b(l) + (r - H * H);
            } else {
                // W_out[NH][H], b_out[NH]
                const int r = (int)(r0 - (int64_t)(L - 1) * lay);
                if (r < H) pj = off_wout(L) + r;
                else if (NH == 2 && r < 2 * H) pj = off_wout2(L) + (r - H);
                else pj = (r == NH * H) ? off_wout(L) + PW : off_wout2(L) + PW;
            }
        }
    }
    // Adam's operands are loaded now, so their latency overlaps the row sums
    float am = 0.f, av = 0.f, ap = 0.f, ast = 0.f;
    if (w == 0 && pj >= 0 && ad.params) {
        const int64_t k = (int64_t)ii * npf + j;
        am = ad.m[k];
        av = ad.v[k];
        ap = ad.params[k];
        ast = (float)*ad.step;
    }
    float acc = 0.f;
    if (pj >= 0) {
        for (int b0 = w; b0 < rows; b0 += kFinBatch * kFinWaves) {
            float v[kFinBatch];
#pragma unroll
            for (int i = 0; i < kFinBatch; ++i) {
                const int b = b0 + i * kFinWaves;
                v[i] = b < rows ? gp[(int64_t)b * kMaxPadded + pj] : 0.f;
            }
#pragma unroll
            for (int i = 0; i < kFinBatch; ++i) acc += v[i];
        }
    }
    part[w][c] = acc;
    if (blockIdx.x == 0) {
        double l4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b = threadIdx.x; b < lrows; b += kFinThreads) {
#pragma unroll
            for (int i = 0; i < 4; ++i) l4[i] += lp[(int64_t)b * 4 + i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double v = wave_sum(l4[i]);
            if (c == 0) lred[w][i] = v;
        }
    }
    __syncthreads();
    if (w == 0 && pj >= 0) {
        float pv[kFinWaves];
#pragma unroll
        for (int q = 0; q < kFinWaves; ++q) pv[q] = part[q][c];
        float g = 0.f;
#pragma unroll
        for (int q = 0; q < kFinWaves; ++q) g += pv[q];
        if (grad_out) grad_out[(int64_t)ii * npf + j] = g;
        if (ad.params) {
            const int64_t k = (int64_t)ii * npf + j;
            adam_one(ap, am, av, g, ast, ad);
            ad.m[k] = am;
            ad.v[k] = av;
            ad.params[k] = ap;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 64) {
        double tt[4] = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < kFinWaves; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) tt[i] += lred[q][i];
        const double Lv = I.cv * tt[0];
        const double Lb = I.n_bnd ? tt[2] / (double)I.n_bnd : 0.0;
        const double Ls = I.n_sen ? tt[3] / (double)I.n_sen : 0.0;
        if (loss_out) {
            float *lo = loss_out + 4 * (int64_t)ii;
            lo[0] = (float)(Lv + (double)I.tau * Lb + (double)I.gamma * Ls);
            lo[1] = (float)Lv;
            lo[2] = (float)Lb;
            lo[3] = (float)Ls;
        }
        const float ge = (float)(2.0 * I.cv * tt[1]);
        if (grad_eps_out) grad_eps_out[ii] = ge;
        if (ad.ep) {
            // the contraction read ep[ii] in this step and has finished: update it in place
            float pe = ad.ep[ii], me = ad.em[ii], ve = ad.ev[ii];
            adam_one(pe, me, ve, ge, (float)*ad.step, ad);
            ad.em[ii] = me;
            ad.ev[ii] = ve;
            ad.ep[ii] = pe;
        }
    }
}

// ---------------------------------------------------------------------------
// prediction: the network (and optionally its tangents, and its second output)
// at n arbitrary points, tiles of 16 points dealt round-robin over the
// wavefronts of one block per CU, weights read once per block
// ---------------------------------------------------------------------------
// values only: the hidden-to-hidden value products, no tangents
template <int L>
__device__ __forceinline__ void tile_values(const WeightsShared<L> &S, int lane, float x, float y, Vec &A_) {
    const int g = lane >> 4;
    const int ln = opaque(lane);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * m + 4 * g + r;
            A_.v[m][r] = tanh_lean(fmaf(S.w1[n][0], x, fmaf(S.w1[n][1], y, S.b[0][n])));
        }
#pragma unroll
    for (int l = 2; l <= L; ++l) {
        Vec Z;
        Split8 sa;
        split8(A_, sa);
        f4 z[2];
#pragma unroll
        for (int mo = 0; mo < 2; ++mo)
#pragma unroll
            for (int r = 0; r < 4; ++r) z[mo][r] = S.b[l - 1][16 * mo + 4 * g + r];
#pragma unroll
        for (int t = 0; t < 6; ++t)
#pragma unroll
            for (int mo = 0; mo < 2; ++mo) z[mo] = mfb(S.wp[l - 2][0][mo][kPi[t]][ln], sa.p[kPj[t]], z[mo]);
#pragma unroll
        for (int mo = 0; mo < 2; ++mo) Z.v[mo] = z[mo];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) A_.v[m][r] = tanh_lean(Z.v[m][r]);
    }
}

struct EvalArgs {
    const float *params;  // flat layout, width H, NH outputs
    int H;
    int64_t n;
    const float2 *xy;
    float *u, *ux, *uy, *e;  // any may be null (ux, uy only with TAN)
};

constexpr int kEvalWaves = 12;

template <int L, int NH, bool TAN>
__global__ __launch_bounds__(kEvalWaves * 64, 1) void k_eval(EvalArgs A) {
    __shared__ FwdShared<L, kEvalWaves> S;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    load_weights<L, kEvalWaves * 64, NH>(S.W, S.stage, A.params, A.H, tid);
    __syncthreads();
    const int64_t tiles = (A.n + 15) / 16;
    const int64_t t0 = (int64_t)blockIdx.x * tiles / gridDim.x, t1 = (int64_t)(blockIdx.x + 1) * tiles / gridDim.x;
    for (int64_t tt = t0 + wave; tt < t1; tt += kEvalWaves) {
        const int64_t idx = 16 * tt + (lane & 15);
        const bool ok = idx < A.n;
        const float2 p = ok ? A.xy[idx] : make_float2(0.f, 0.f);
        Vec a;
        float u, ux = 0.f, uy = 0.f;
        if (TAN) {
            Vec tx, ty;
            Acts<L> unused;
            tile_forward<L, false>(S.W, lane, p.x, p.y, a, tx, ty, unused);
            tile_outputs<L>(S.W, lane, a, tx, ty, u, ux, uy);
        } else {
            tile_values<L>(S.W, lane, p.x, p.y, a);
            const int g = lane >> 4;
            float su = 0.f;
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) su = fmaf(S.W.wo[16 * m + 4 * g + r], a.v[m][r], su);
            u = group_sum(su) + S.W.bo;
        }
        const float e = NH == 2 ? tile_second<L>(S.W, lane, a) : 0.f;
        if (lane < 16 && ok) {
            if (A.u) A.u[idx] = u;
            if (TAN && A.ux) A.ux[idx] = ux;
            if (TAN && A.uy) A.uy[idx] = uy;
            if (NH == 2 && A.e) A.e[idx] = e;
        }
    }
}

template <int L>
static void launch_eval(int nh, bool tan, unsigned blocks, const EvalArgs &a, hipStream_t s) {
    const int th = kEvalWaves * 64;
    if (nh == 2) {
        if (tan) k_eval<L, 2, true><<<blocks, th, 0, s>>>(a);
        else k_eval<L, 2, false><<<blocks, th, 0, s>>>(a);
    } else {
        if (tan) k_eval<L, 1, true><<<blocks, th, 0, s>>>(a);
        else k_eval<L, 1, false><<<blocks, th, 0, s>>>(a);
    }
}

static int cu_count(int dev);

vpinn_status eval_mfma(int L, int H, int nh, const float *params, int64_t n, const float2 *xy, float *u, float *ux,
                       float *uy, float *e, hipStream_t s) {
    if (n == 0) return VPINN_OK;
    int dev = 0;
    VP_HIP(hipGetDevice(&dev));
    const int64_t tiles = (n + 15) / 16;
    const unsigned blocks = (unsigned)std::min<int64_t>(cu_count(dev), tiles);
    EvalArgs a{params, H, n, xy, u, ux, uy, e};
    const bool tan = ux != nullptr || uy != nullptr;
    switch (L) {
    case 1: launch_eval<1>(nh, tan, blocks, a, s); break;
    case 2: launch_eval<2>(nh, tan, blocks, a, s); break;
    case 3: launch_eval<3>(nh, tan, blocks, a, s); break;
    default: launch_eval<4>(nh, tan, blocks, a, s); break;
    }
    VP_HIP(hipGetLastError());
    return VPINN_OK;
}

// ---------------------------------------------------------------------------
// host side: work plans
// ---------------------------------------------------------------------------
static int cu_count(int dev) {
    static int cached[64] = {0};
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    hipDeviceProp_t prop;
    int n = 256;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n = prop.multiProcessorCount;
    if (dev >= 0 && dev < 64) cached[dev] = n;
    return n;
}

// A plan fixes, for a set of instances with one network shape and loss
// weighting: the global tile list (16 points a tile, instance-major) and the
// contiguous tile range of each of the one-per-CU blocks of k_fwd and k_bwd
// (equal tile counts), the contraction chunks of every instance, and which loss
// and gradient partial rows each block writes.
// tile shapes a plan is built with (vpinn_tuning): forward wavefronts per block,
// elements per small-element contraction block (shift), rows per pass of the
// row-streaming contraction
static const vpinn_tuning kDefaultTuning = {12, 0, 4, 0, 0};
static bool tuning_valid(const vpinn_tuning &t) {
    return (t.fwd_waves == 8 || t.fwd_waves == 12 || t.fwd_waves == 16) && t.chunk_shift >= 0 && t.chunk_shift <= 2 &&
           (t.rows_per_pass == 2 || t.rows_per_pass == 4 || t.rows_per_pass == 8) &&
           (t.store_activations == 0 || t.store_activations == 1) && (t.one_pass == 0 || t.one_pass == 1) &&
           !(t.one_pass && t.store_activations);
}

struct FusedPlan {
    DevBuf inst, blk_tiles, blk_inst0, cblk_inst, ubuf, gpart, lpart;
    DevBuf ebuf;  // two outputs: e, then dL/de, per point (point buffer order)
    // shared points: the instances' point lists, and the per-slot adjoints of the contraction
    DevBuf dpts, abuf, eabuf;
    DevBuf act;  // store_activations: [tiles][L][kActTile]
    DevBuf rblk_inst, apart;  // large elements: instance of each row-sum block; partial row sums
    DevBuf grp;               // one-pass: the group list (GroupDesc); blk_tiles then holds group ranges
    int64_t n_grp = 0;
    int64_t rblocks = 0;
    int nh = 1;   // network outputs
    vpinn_tuning tune = kDefaultTuning;
    std::vector<InstDesc> host_inst;
    int tblocks = 0, n_inst = 0, grows = 0, lrows = 0, L = 0, H = 0;
    int64_t cblocks = 0, tiles = 0, npf = 0;
    int64_t cpath_blocks[kNumPaths] = {};  // contraction blocks of each path, in path order
    size_t cdyn_fast = 0, cdyn_generic = 0;  // dynamic LDS of k_contract_fast / k_split_adj
    size_t cdyn_mf = 0;                      // and of k_contract_mf
};

// which of the four-kernel plan's contraction kernels takes a problem's elements
static int contraction_path(const vpinn_problem *p) {
    return p->matfree                               ? kPathMF
           : (p->nq <= kCThreads && p->ntest <= kKB) ? kPathFast
           : (p->nq <= 64)                          ? kPathRows1
           : (p->nq <= 128)                         ? kPathRows2
           : (p->nq <= 64 * kRowQ)                  ? kPathRows4
                                                    : kPathGeneric;
}

// One-pass plan: every instance's elements in groups of whole elements of at most
// kGroupPts points (floor(kGroupPts / N_quad) elements each, the last one shorter),
// then its boundary and sensor points in groups of kGroupPts; the global group list
// is dealt in equal contiguous shares to one block per CU, and instance i gets one
// loss row and one gradient row per block whose share meets its groups.
static vpinn_status build_one_pass(vpinn_problem *const *probs, int n, int nh, int cus, std::vector<InstDesc> &D,
                                   FusedPlan &P) {
    if (nh != 1) return fail(VPINN_E_UNSUPPORTED, "the one-pass step has one network output");
    std::vector<GroupDesc> grp;
    for (int i = 0; i < n; ++i) {
        const vpinn_problem *p = probs[i];
        if (p->matfree || p->n_uniq > 0 || p->nq > kGroupPts || p->ntest > kKB)
            return fail(VPINN_E_UNSUPPORTED, "problem " + std::to_string(i) +
                                                 ": the one-pass step needs stored G, no shared points, N_quad <= " +
                                                 std::to_string(kGroupPts) + " and N_test <= " + std::to_string(kKB));
        InstDesc &d = D[i];
        d.grp0 = (int64_t)grp.size();
        const int epg = std::min(kGroupMaxElem, kGroupPts / p->nq);
        for (int64_t e0 = 0; e0 < p->n_elem; e0 += epg) {
            const int ne = (int)std::min<int64_t>(epg, p->n_elem - e0);
            grp.push_back(GroupDesc{e0 * p->nq, e0, ne * p->nq, ne});
        }
        const int64_t nx = p->n_bnd + p->n_sen;
        for (int64_t x0 = 0; x0 < nx; x0 += kGroupPts)
            grp.push_back(GroupDesc{p->n_pts + x0, 0, (int)std::min<int64_t>(kGroupPts, nx - x0), 0});
        d.n_grp = (int64_t)grp.size() - d.grp0;
    }
    const int64_t ng = (int64_t)grp.size();
    const int nblk = (int)std::min<int64_t>(std::min<int64_t>((int64_t)cus, kMaxBlocks), ng);
    std::vector<int64_t> bg(nblk + 1);
    std::vector<int> binst(nblk);
    for (int b = 0; b <= nblk; ++b) bg[b] = (int64_t)b * ng / nblk;
    int rows = 0, bb = 0;
    for (int i = 0; i < n; ++i) {
        InstDesc &d = D[i];
        const int64_t gf = d.grp0, gl = d.grp0 + d.n_grp - 1;
        while (bg[bb + 1] <= gf) ++bb;
        int bl = bb;
        while (bg[bl + 1] <= gl) ++bl;
        d.gblk0 = bb;
        d.gn_rows = bl - bb + 1;
        d.grow0 = rows;
        d.lrow0 = rows;
        d.ln_rows = d.gn_rows;
        rows += d.gn_rows;
    }
    for (int b = 0, i = 0; b < nblk; ++b) {
        while (D[i].grp0 + D[i].n_grp <= bg[b]) ++i;
        binst[b] = i;
    }
    VP_ALLOC(P.inst.reserve(sizeof(InstDesc) * n));
    VP_ALLOC(P.grp.reserve(sizeof(GroupDesc) * (size_t)ng));
    VP_ALLOC(P.blk_tiles.reserve(sizeof(int64_t) * (nblk + 1)));
    VP_ALLOC(P.blk_inst0.reserve(sizeof(int) * nblk));
    VP_ALLOC(P.gpart.reserve(sizeof(float) * kMaxPadded * (size_t)rows));
    VP_ALLOC(P.lpart.reserve(sizeof(double) * 4 * (size_t)rows));
    VP_HIP(hipMemcpy(P.inst.ptr, D.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(P.grp.ptr, grp.data(), sizeof(GroupDesc) * (size_t)ng, hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(P.blk_tiles.ptr, bg.data(), sizeof(int64_t) * (nblk + 1), hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(P.blk_inst0.ptr, binst.data(), sizeof(int) * nblk, hipMemcpyHostToDevice));
    P.host_inst = D;
    P.tblocks = nblk;
    P.cblocks = 0;
    P.n_inst = n;
    P.grows = rows;
    P.lrows = rows;
    P.n_grp = ng;
    P.tiles = 0;
    P.rblocks = 0;
    for (int k = 0; k < kNumPaths; ++k) P.cpath_blocks[k] = 0;
    return VPINN_OK;
}

static vpinn_status build_plan(vpinn_problem *const *probs, int n, const vpinn_loss_cfg *cfg, int dev,
                               const vpinn_tuning &tune, FusedPlan &P) {
    P.tune = tune;
    const int L = cfg->n_hidden, H = cfg->width;
    const int nh = cfg->n_outputs == 2 ? 2 : 1;
    const int cus = cu_count(dev);
    std::vector<InstDesc> D(n);
    // shared-point instances: their point list (distinct points, boundary, sensors) at
    // dbase[i] of the plan's dpts, their adjoint slots at sbase[i] of abuf (eabuf)
    std::vector<int64_t> dbase(n, -1), sbase(n, -1);
    int64_t n_dpts = 0, n_slots = 0;
    int64_t tiles = 0, ubase = 0, cblocks = 0, rblocks = 0, n_apart = 0;
    size_t cdyn_fast = 16, cdyn_generic = 16, cdyn_mf = 16;
    for (int i = 0; i < n; ++i) {
        const vpinn_problem *p = probs[i];
        const bool shared = p->n_uniq > 0;
        const int64_t n_int = shared ? p->n_uniq : p->n_pts;
        const int64_t tot = n_int + p->n_bnd + p->n_sen;
        InstDesc &d = D[i];
        d = InstDesc{};
        d.Gx = p->Gx.as<float>();
        d.Gy = p->Gy.as<float>();
        d.F = p->F.as<float>();
        d.pts = p->pts.as<float2>();
        d.tgt = p->tgt.as<float>();
        d.n_elem = p->n_elem;
        d.n_pts = n_int;
        if (shared) {
            d.umap = p->umap.as<int>();
            d.usoff = p->usoff.as<int>();
            d.uslot = p->uslot.as<int>();
            dbase[i] = n_dpts;
            n_dpts += tot;
            sbase[i] = n_slots;
            n_slots += p->n_pts;
        }
        d.n_bnd = p->n_bnd;
        d.n_sen = p->n_sen;
        d.n_tiles = (tot + 15) / 16;
        d.tile0 = tiles;
        tiles += d.n_tiles;
        d.ubase = ubase;
        ubase += tot;
        d.nq = p->nq;
        d.ntest = p->ntest;
        d.gstride = p->gstride();
        if (nh == 2) {
            // the small-element and matrix-free contractions are the ones with the space-dependent term
            if (!p->vardiff) return fail(VPINN_E_INVALID, "two network outputs need space-dependent diffusion problems");
            if (!p->matfree && !(p->nq <= kCThreads && p->ntest <= kKB))
                return fail(VPINN_E_UNSUPPORTED, "space-dependent diffusion needs N_quad <= " +
                                                     std::to_string(kCThreads) + " and N_test <= " +
                                                     std::to_string(kKB));
            d.M = p->M.as<float>();
            d.cbx = (float)p->vd_bx;
            d.cby = (float)p->vd_by;
        }
        if (p->matfree) {
            d.geo = p->geo.as<float>();
            d.tab = p->tab.as<float>();
            d.kdiff = (float)p->diff;
            d.cbx = (float)(p->vardiff ? p->vd_bx : p->conv_x);
            d.cby = (float)(p->vardiff ? p->vd_by : p->conv_y);
            d.qn = p->n;
            d.tn = p->nt;
        }
        d.path = contraction_path(p);
        d.epc = d.path == kPathFast ? std::max(1, (kCThreads / p->nq) >> tune.chunk_shift)
                : d.path == kPathMF ? kCWaves
                                    : 1;
        d.n_chunks = (p->n_elem + d.epc - 1) / d.epc;
        if (d.path == kPathGeneric) {
            d.nkb = (p->ntest + kGWaves - 1) / kGWaves;
            d.nqb = (p->nq + kSplitQ - 1) / kSplitQ;
            // wavefronts per point group: enough that each takes at most 32 test functions, and
            // more while the problem has fewer than 512 adjoint blocks
            d.kw = 1;
            while (d.kw < kGWaves && (d.kw * 32 < p->ntest ||
                                      p->n_elem * ((p->nq + 64 * (kGWaves / d.kw) - 1) / (64 * (kGWaves / d.kw))) < 512))
                d.kw *= 2;
            d.npb = (p->nq + 64 * (kGWaves / d.kw) - 1) / (64 * (kGWaves / d.kw));
            d.n_chunks = p->n_elem * d.npb;
            d.rblk0 = rblocks;
            rblocks += p->n_elem * d.nkb * d.nqb;
            d.abase = n_apart;
            n_apart += p->n_elem * d.nqb * p->ntest;
        }
        if (d.path == kPathFast)
            cdyn_fast = std::max(cdyn_fast, sizeof(float) * ((size_t)d.ntest * kCbs + (size_t)d.epc * d.ntest));
        if (d.path == kPathGeneric) cdyn_generic = std::max(cdyn_generic, sizeof(float) * (size_t)d.ntest);
        if (d.path == kPathMF) {
            const size_t nn = (size_t)p->n * p->nt;
            cdyn_mf = std::max(cdyn_mf, sizeof(float) * (2 * (size_t)p->n + 2 * nn +
                                                         kCWaves * (3 * (size_t)p->nq + 2 * nn + (size_t)p->ntest)));
        }
        d.cv = cfg->loss_norm == VPINN_NORM_ELEM ? 1.0 / (double)p->n_elem : 1.0 / (double)p->ntest;
        d.two_cv = (float)(2.0 * d.cv);
        d.wb2 = p->n_bnd ? (float)(2.0 * cfg->tau / (double)p->n_bnd) : 0.f;
        d.ws2 = p->n_sen ? (float)(2.0 * cfg->gamma / (double)p->n_sen) : 0.f;
        d.tau = cfg->tau;
        d.gamma = cfg->gamma;
    }
    if (tune.one_pass) {
        vpinn_status st = build_one_pass(probs, n, nh, cus, D, P);
        if (st) return st;
        P.tiles = tiles;  // the four-kernel tile count, for the stored-activation footprint
        P.L = L;
        P.H = H;
        P.nh = nh;
        P.npf = vpinn_n_params_out(H, L, nh);
        return VPINN_OK;
    }
    // contraction blocks grouped by path (one launch each), instance order within a path
    int64_t cpath_blocks[kNumPaths] = {};
    for (int path = 0; path < kNumPaths; ++path)
        for (int i = 0; i < n; ++i)
            if (D[i].path == path) {
                D[i].cblk0 = cblocks;
                cblocks += D[i].n_chunks;
                cpath_blocks[path] += D[i].n_chunks;
            }
    if (cblocks > (int64_t)INT32_MAX || rblocks > (int64_t)INT32_MAX)
        return fail(VPINN_E_UNSUPPORTED, "fused path: too many elements for one launch");
    if (cdyn_fast > 64 * 1024 || cdyn_generic > 64 * 1024 || cdyn_mf > 64 * 1024)
        return fail(VPINN_E_UNSUPPORTED, "fused path: test-function count exceeds the LDS budget");
    // tile blocks (k_fwd and k_bwd): one per CU, equal shares of the tile list
    const int tblocks = (int)std::min<int64_t>(std::min<int64_t>((int64_t)cus, kMaxBlocks), tiles);
    std::vector<int64_t> bt(tblocks + 1);
    std::vector<int> binst(tblocks);
    for (int b = 0; b <= tblocks; ++b) bt[b] = (int64_t)b * tiles / tblocks;
    // rows: instance i gets one loss row and one gradient row per tile block whose
    // range meets its tiles, then one loss row per contraction block
    int lrows = 0, grows = 0;
    std::vector<int> cinst((size_t)cblocks);
    {
        int bb = 0;
        for (int i = 0; i < n; ++i) {
            InstDesc &d = D[i];
            const int64_t tf = d.tile0, tl = d.tile0 + d.n_tiles - 1;
            while (bt[bb + 1] <= tf) ++bb;
            int bl = bb;
            while (bt[bl + 1] <= tl) ++bl;
            d.gblk0 = bb;
            d.gn_rows = bl - bb + 1;
            d.grow0 = grows;
            grows += d.gn_rows;
            d.lrow0 = lrows;
            d.ln_rows = d.gn_rows + (int)d.n_chunks;
            lrows += d.ln_rows;
            for (int64_t c = 0; c < d.n_chunks; ++c) cinst[(size_t)(d.cblk0 + c)] = i;
        }
        int i = 0;
        for (int b = 0; b < tblocks; ++b) {
            while (D[i].tile0 + D[i].n_tiles <= bt[b]) ++i;
            binst[b] = i;
        }
    }
    VP_ALLOC(P.inst.reserve(sizeof(InstDesc) * n));
    VP_ALLOC(P.blk_tiles.reserve(sizeof(int64_t) * (tblocks + 1)));
    VP_ALLOC(P.blk_inst0.reserve(sizeof(int) * tblocks));
    VP_ALLOC(P.cblk_inst.reserve(sizeof(int) * (size_t)cblocks));
    if (rblocks) {
        VP_ALLOC(P.rblk_inst.reserve(sizeof(int) * (size_t)rblocks));
        VP_ALLOC(P.apart.reserve(sizeof(float) * (size_t)n_apart));
        std::vector<int> rinst((size_t)rblocks);
        for (int i = 0; i < n; ++i)
            if (D[i].path == kPathGeneric)
                for (int64_t j = 0; j < D[i].n_elem * D[i].nkb * D[i].nqb; ++j) rinst[(size_t)(D[i].rblk0 + j)] = i;
        VP_HIP(hipMemcpy(P.rblk_inst.ptr, rinst.data(), sizeof(int) * (size_t)rblocks, hipMemcpyHostToDevice));
    }
    P.rblocks = rblocks;
    VP_ALLOC(P.ubuf.reserve(sizeof(float2) * (size_t)ubase));
    VP_ALLOC(P.gpart.reserve(sizeof(float) * kMaxPadded * (size_t)grows));
    VP_ALLOC(P.lpart.reserve(sizeof(double) * 4 * (size_t)lrows));
    if (nh == 2) VP_ALLOC(P.ebuf.reserve(sizeof(float) * (size_t)ubase));
    if (tune.store_activations) VP_ALLOC(P.act.reserve(sizeof(float) * (size_t)tiles * L * kActTile));
    if (n_slots) {
        VP_ALLOC(P.dpts.reserve(sizeof(float2) * (size_t)n_dpts));
        VP_ALLOC(P.abuf.reserve(sizeof(float2) * (size_t)n_slots));
        if (nh == 2) VP_ALLOC(P.eabuf.reserve(sizeof(float) * (size_t)n_slots));
    }
    for (int i = 0; i < n; ++i) {
        const vpinn_problem *p = probs[i];
        InstDesc &d = D[i];
        if (dbase[i] >= 0) {
            float2 *dp = P.dpts.as<float2>() + dbase[i];
            VP_HIP(hipMemcpy(dp, p->upts.ptr, sizeof(float2) * p->n_uniq, hipMemcpyDeviceToDevice));
            if (p->n_bnd + p->n_sen)
                VP_HIP(hipMemcpy(dp + p->n_uniq, p->pts.as<float2>() + p->n_pts, sizeof(float2) * (p->n_bnd + p->n_sen),
                                 hipMemcpyDeviceToDevice));
            d.pts = dp;
            d.adj = P.abuf.as<float2>() + sbase[i];
            d.eadj = nh == 2 ? P.eabuf.as<float>() + sbase[i] : nullptr;
        } else {
            d.adj = P.ubuf.as<float2>() + d.ubase;
            d.eadj = nh == 2 ? P.ebuf.as<float>() + d.ubase : nullptr;
        }
    }
    VP_HIP(hipMemcpy(P.inst.ptr, D.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(P.blk_tiles.ptr, bt.data(), sizeof(int64_t) * (tblocks + 1), hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(P.blk_inst0.ptr, binst.data(), sizeof(int) * tblocks, hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(P.cblk_inst.ptr, cinst.data(), sizeof(int) * (size_t)cblocks, hipMemcpyHostToDevice));
    if (cdyn_fast > 48 * 1024) {
        const void *fn = nh == 2 ? (const void *)k_contract_fast<true> : (const void *)k_contract_fast<false>;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cdyn_fast);
        if (e != hipSuccess) return fail(VPINN_E_DEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
    if (cdyn_mf > 48 * 1024) {
        const void *fn = nh == 2 ? (const void *)k_contract_mf<true> : (const void *)k_contract_mf<false>;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cdyn_mf);
        if (e != hipSuccess) return fail(VPINN_E_DEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
    P.host_inst = D;
    P.tblocks = tblocks;
    P.cblocks = cblocks;
    P.n_inst = n;
    P.grows = grows;
    P.lrows = lrows;
    P.tiles = tiles;
    P.L = L;
    P.H = H;
    P.nh = nh;
    P.npf = vpinn_n_params_out(H, L, nh);
    for (int k = 0; k < kNumPaths; ++k) P.cpath_blocks[k] = cpath_blocks[k];
    P.cdyn_fast = cdyn_fast;
    P.cdyn_generic = cdyn_generic;
    P.cdyn_mf = cdyn_mf;
    return VPINN_OK;
}

template <int Q>
static void launch_rows(int rp, unsigned blocks, const ContractArgs &c, hipStream_t s) {
    switch (rp) {
    case 2: k_contract_rows<Q, 2><<<blocks, kCThreads, 0, s>>>(c); break;
    case 8: k_contract_rows<Q, 8><<<blocks, kCThreads, 0, s>>>(c); break;
    default: k_contract_rows<Q, 4><<<blocks, kCThreads, 0, s>>>(c); break;
    }
}

template <int L, int NH>
static void launch_all(const FusedPlan &P, const FwdArgs &fa, const ContractArgs &ca, const BwdArgs &ba,
                       bool want_grad, dim3 fg, int ft, float *loss, float *grad, float *grad_eps, const AdamArgs &ad,
                       hipEvent_t const *ev, hipStream_t s) {
    if (ev && ev[0]) (void)hipEventRecord(ev[0], s);
    const bool st = fa.act != nullptr;
    switch (P.tune.fwd_waves * 2 + (st ? 1 : 0)) {
    case 16: k_fwd<L, 8, NH, false><<<P.tblocks, 8 * 64, 0, s>>>(fa); break;
    case 17: k_fwd<L, 8, NH, true><<<P.tblocks, 8 * 64, 0, s>>>(fa); break;
    case 32: k_fwd<L, 16, NH, false><<<P.tblocks, 16 * 64, 0, s>>>(fa); break;
    case 33: k_fwd<L, 16, NH, true><<<P.tblocks, 16 * 64, 0, s>>>(fa); break;
    case 25: k_fwd<L, 12, NH, true><<<P.tblocks, 12 * 64, 0, s>>>(fa); break;
    default: k_fwd<L, 12, NH, false><<<P.tblocks, 12 * 64, 0, s>>>(fa); break;
    }
    if (ev && ev[1]) (void)hipEventRecord(ev[1], s);
    {
        ContractArgs c = ca;
        c.cblk_base = 0;
        if (P.cpath_blocks[kPathFast])
            k_contract_fast<NH == 2><<<(unsigned)P.cpath_blocks[kPathFast], kCThreads, P.cdyn_fast, s>>>(c);
        c.cblk_base += P.cpath_blocks[kPathFast];
        const int rp = P.tune.rows_per_pass;
        if (P.cpath_blocks[kPathRows1]) launch_rows<1>(rp, (unsigned)P.cpath_blocks[kPathRows1], c, s);
        c.cblk_base += P.cpath_blocks[kPathRows1];
        if (P.cpath_blocks[kPathRows2]) launch_rows<2>(rp, (unsigned)P.cpath_blocks[kPathRows2], c, s);
        c.cblk_base += P.cpath_blocks[kPathRows2];
        if (P.cpath_blocks[kPathRows4]) launch_rows<4>(rp, (unsigned)P.cpath_blocks[kPathRows4], c, s);
        c.cblk_base += P.cpath_blocks[kPathRows4];
        if (P.cpath_blocks[kPathGeneric]) {
            k_split_rows<<<(unsigned)P.rblocks, kGThreads, 0, s>>>(c, P.rblk_inst.as<int>(), P.apart.as<float>());
            k_split_adj<<<(unsigned)P.cpath_blocks[kPathGeneric], kGThreads, P.cdyn_generic, s>>>(c, P.apart.as<float>());
        }
        c.cblk_base += P.cpath_blocks[kPathGeneric];
        if (P.cpath_blocks[kPathMF])
            k_contract_mf<NH == 2><<<(unsigned)P.cpath_blocks[kPathMF], kCThreads, P.cdyn_mf, s>>>(c);
    }
    if (ev && ev[2]) (void)hipEventRecord(ev[2], s);
    if (want_grad) {
        if (P.tune.store_activations) k_bwd<L, NH, true><<<P.tblocks, kBThreads, 0, s>>>(ba);
        else k_bwd<L, NH, false><<<P.tblocks, kBThreads, 0, s>>>(ba);
    }
    if (ev && ev[3]) (void)hipEventRecord(ev[3], s);
    k_fused_final<L, NH><<<fg, ft, 0, s>>>(P.inst.as<InstDesc>(), P.gpart.as<float>(), P.lpart.as<double>(), P.H, P.npf,
                                        loss, grad, grad_eps, ad);
    if (ev && ev[4]) (void)hipEventRecord(ev[4], s);
}

// launch forward, contraction, backward, and the per-instance reduction (with optional Adam)
static vpinn_status run_plan(const FusedPlan &P, const float *params, const float *eps, bool want_grad,
                             float *loss, float *grad, float *grad_eps, const AdamArgs &ad, int64_t *step,
                             hipEvent_t const *ev, hipStream_t s) {
    FwdArgs fa{};
    fa.inst = P.inst.as<InstDesc>();
    fa.blk_tiles = P.blk_tiles.as<int64_t>();
    fa.blk_inst0 = P.blk_inst0.as<int>();
    fa.params = params;
    fa.param_stride = P.npf;
    fa.H = P.H;
    fa.ubuf = P.ubuf.as<float2>();
    fa.lpart = P.lpart.as<double>();
    fa.step = step;
    fa.ebuf = P.ebuf.as<float>();
    // activations are stored only when the reverse sweep will read them
    fa.act = (want_grad && P.tune.store_activations) ? P.act.as<float>() : nullptr;
    ContractArgs ca{};
    ca.inst = P.inst.as<InstDesc>();
    ca.cblk_inst = P.cblk_inst.as<int>();
    ca.eps = eps;
    ca.want_grad = want_grad ? 1 : 0;
    ca.ubuf = P.ubuf.as<float2>();
    ca.lpart = P.lpart.as<double>();
    ca.ebuf = P.ebuf.as<float>();
    BwdArgs ba{};
    ba.inst = P.inst.as<InstDesc>();
    ba.blk_tiles = P.blk_tiles.as<int64_t>();
    ba.blk_inst0 = P.blk_inst0.as<int>();
    ba.params = params;
    ba.param_stride = P.npf;
    ba.H = P.H;
    ba.ubuf = P.ubuf.as<float2>();
    ba.gpart = P.gpart.as<float>();
    ba.ebuf = P.ebuf.as<float>();
    ba.act = P.act.as<float>();
    const dim3 fg((unsigned)std::max<int64_t>(1, (P.npf + kFinCols - 1) / kFinCols), (unsigned)P.n_inst);
    const int ft = kFinThreads;
    if (P.tune.one_pass) {
        StepArgs sa{};
        sa.inst = P.inst.as<InstDesc>();
        sa.grp = P.grp.as<GroupDesc>();
        sa.blk_grp = P.blk_tiles.as<int64_t>();
        sa.blk_inst0 = P.blk_inst0.as<int>();
        sa.params = params;
        sa.param_stride = P.npf;
        sa.H = P.H;
        sa.eps = eps;
        sa.want_grad = want_grad ? 1 : 0;
        sa.gpart = P.gpart.as<float>();
        sa.lpart = P.lpart.as<double>();
        sa.step = step;
        // profiling events: the one kernel is timed between the first two, the reduction between the last two
        if (ev && ev[0]) (void)hipEventRecord(ev[0], s);
        switch (P.L) {
        case 1: k_step<1><<<P.tblocks, kBThreads, 0, s>>>(sa); break;
        case 2: k_step<2><<<P.tblocks, kBThreads, 0, s>>>(sa); break;
        case 3: k_step<3><<<P.tblocks, kBThreads, 0, s>>>(sa); break;
        default: k_step<4><<<P.tblocks, kBThreads, 0, s>>>(sa); break;
        }
        for (int k = 1; k <= 3; ++k)
            if (ev && ev[k]) (void)hipEventRecord(ev[k], s);
        switch (P.L) {
        case 1: k_fused_final<1, 1><<<fg, ft, 0, s>>>(P.inst.as<InstDesc>(), P.gpart.as<float>(), P.lpart.as<double>(), P.H, P.npf, loss, grad, grad_eps, ad); break;
        case 2: k_fused_final<2, 1><<<fg, ft, 0, s>>>(P.inst.as<InstDesc>(), P.gpart.as<float>(), P.lpart.as<double>(), P.H, P.npf, loss, grad, grad_eps, ad); break;
        case 3: k_fused_final<3, 1><<<fg, ft, 0, s>>>(P.inst.as<InstDesc>(), P.gpart.as<float>(), P.lpart.as<double>(), P.H, P.npf, loss, grad, grad_eps, ad); break;
        default: k_fused_final<4, 1><<<fg, ft, 0, s>>>(P.inst.as<InstDesc>(), P.gpart.as<float>(), P.lpart.as<double>(), P.H, P.npf, loss, grad, grad_eps, ad); break;
        }
        if (ev && ev[4]) (void)hipEventRecord(ev[4], s);
        VP_HIP(hipGetLastError());
        return VPINN_OK;
    }
    switch (P.L * 2 + P.nh - 1) {
    case 2: launch_all<1, 1>(P, fa, ca, ba, want_grad, fg, ft, loss, grad, grad_eps, ad, ev, s); break;
    case 3: launch_all<1, 2>(P, fa, ca, ba, want_grad, fg, ft, loss, grad, grad_eps, ad, ev, s); break;
    case 4: launch_all<2, 1>(P, fa, ca, ba, want_grad, fg, ft, loss, grad, grad_eps, ad, ev, s); break;
    case 5: launch_all<2, 2>(P, fa, ca, ba, want_grad, fg, ft, loss, grad, grad_eps, ad, ev, s); break;
    case 6: launch_all<3, 1>(P, fa, ca, ba, want_grad, fg, ft, loss, grad, grad_eps, ad, ev, s); break;
    case 7: launch_all<3, 2>(P, fa, ca, ba, want_grad, fg, ft, loss, grad, grad_eps, ad, ev, s); break;
    case 9: launch_all<4, 2>(P, fa, ca, ba, want_grad, fg, ft, loss, grad, grad_eps, ad, ev, s); break;
    default: launch_all<4, 1>(P, fa, ca, ba, want_grad, fg, ft, loss, grad, grad_eps, ad, ev, s); break;
    }
    VP_HIP(hipGetLastError());
    return VPINN_OK;
}

// ---------------------------------------------------------------------------
// single problem: a cached plan, rebuilt when the point sets or the loss
// weighting change
// ---------------------------------------------------------------------------
struct SingleCache {
    FusedPlan plan;
    bool valid = false;
    int64_t n_bnd = -1, n_sen = -1;
    const void *pts = nullptr;
    int L = 0, H = 0, norm = -1, nh = 0;
    float tau = -1.f, gamma = -1.f;
    int64_t gen = -1;
};

vpinn_status fused_loss_grad(vpinn_problem *p, const vpinn_loss_cfg *cfg, const float *d_params,
                             const float *d_eps, float *d_loss, float *d_grad, float *d_grad_eps, hipStream_t s) {
    auto *c = reinterpret_cast<SingleCache *>(p->fused_ws);
    if (!c) {
        c = new SingleCache();
        p->fused_ws = c;
        p->fused_ws_free = [](void *w) { delete reinterpret_cast<SingleCache *>(w); };
    }
    if (!c->valid || c->n_bnd != p->n_bnd || c->n_sen != p->n_sen || c->pts != p->pts.ptr || c->L != cfg->n_hidden ||
        c->H != cfg->width || c->norm != cfg->loss_norm || c->tau != cfg->tau || c->gamma != cfg->gamma ||
        c->nh != (cfg->n_outputs == 2 ? 2 : 1) || c->gen != p->gen) {
        // the plan's device buffers are rewritten in place (descriptor copies on the null stream), so the
        // kernels of earlier calls, on whatever stream, must have finished reading them
        if (c->valid) VP_HIP(hipDeviceSynchronize());
        c->valid = false;
        vpinn_problem *one[1] = {p};
        vpinn_status st = build_plan(one, 1, cfg, p->device, kDefaultTuning, c->plan);
        if (st) return st;
        c->valid = true;
        c->n_bnd = p->n_bnd;
        c->n_sen = p->n_sen;
        c->pts = p->pts.ptr;
        c->L = cfg->n_hidden;
        c->H = cfg->width;
        c->norm = cfg->loss_norm;
        c->tau = cfg->tau;
        c->gamma = cfg->gamma;
        c->nh = cfg->n_outputs == 2 ? 2 : 1;
        c->gen = p->gen;
    }
    AdamArgs none{};
    return run_plan(c->plan, d_params, d_eps, d_grad != nullptr || d_grad_eps != nullptr, d_loss, d_grad, d_grad_eps,
                    none, nullptr, p->prof, s);
}

}  // namespace vp

// ---------------------------------------------------------------------------
// batches of independent problems
// ---------------------------------------------------------------------------
struct vpinn_batch {
    int device = 0;
    vpinn_loss_cfg cfg{};
    std::vector<vpinn_problem *> probs;  // borrowed; kept to rebuild the plan with another tuning
    std::vector<int64_t> gens;           // the problems' generations the plan was built from
    vp::FusedPlan plan;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t prof[VPINN_PROFILE_EVENTS] = {};
    ~vpinn_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace vp {

vpinn_status batch_create(int32_t n, vpinn_problem *const *problems, const vpinn_loss_cfg *cfg, vpinn_batch **out) {
    vpinn_batch *b = new (std::nothrow) vpinn_batch();
    if (!b) return fail(VPINN_E_NOMEM, "host allocation failed");
    b->device = problems[0]->device;
    b->cfg = *cfg;
    b->probs.assign(problems, problems + n);
    vpinn_status st = build_plan(problems, n, cfg, b->device, kDefaultTuning, b->plan);
    if (st) {
        delete b;
        return st;
    }
    for (const vpinn_problem *p : b->probs) b->gens.push_back(p->gen);
    *out = b;
    return VPINN_OK;
}

// the plan holds pointers into the problems' point buffers: after a problem's
// point sets or sharing changed, only a rebuilt plan (a new batch, or a new tuning)
// may run
static vpinn_status batch_fresh(const vpinn_batch *b) {
    for (size_t i = 0; i < b->probs.size(); ++i)
        if (b->probs[i]->gen != b->gens[i])
            return fail(VPINN_E_INVALID, "problem " + std::to_string(i) +
                                             " changed its boundary, sensors or shared points after the batch "
                                             "was planned: create the batch again");
    return VPINN_OK;
}

vpinn_status batch_loss_and_grad(vpinn_batch *b, const float *d_params, const float *d_eps, float *d_losses,
                                 float *d_grads, float *d_grad_eps, hipStream_t s) {
    vpinn_status fr = batch_fresh(b);
    if (fr) return fr;
    if (d_eps || d_grad_eps)
        for (const vpinn_problem *p : b->probs)
            if (p->folded() || p->vardiff)
                return fail(VPINN_E_INVALID, "a problem assembled with fixed or space-dependent "
                                             "convection-diffusion coefficients takes no eps");
    AdamArgs none{};
    return run_plan(b->plan, d_params, d_eps, d_grads != nullptr || d_grad_eps != nullptr, d_losses, d_grads,
                    d_grad_eps, none, nullptr, b->prof, s);
}

vpinn_status batch_step(vpinn_batch *b, float *d_params, float *d_m, float *d_v, int64_t *d_step, float lr, float b1,
                        float b2, float eps, float *d_losses, float *d_eps, float *d_eps_m, float *d_eps_v,
                        hipStream_t s) {
    vpinn_status fr = batch_fresh(b);
    if (fr) return fr;
    if (d_eps)
        for (const vpinn_problem *p : b->probs)
            if (p->folded() || p->vardiff)
                return fail(VPINN_E_INVALID, "a problem assembled with fixed or space-dependent "
                                             "convection-diffusion coefficients takes no eps");
    AdamArgs ad{d_params, d_m, d_v, d_step, lr, b1, b2, eps, d_eps, d_eps_m, d_eps_v};
    return run_plan(b->plan, d_params, d_eps, true, d_losses, nullptr, nullptr, ad, d_step, b->prof, s);
}

vpinn_status batch_capture(vpinn_batch *b, float *d_params, float *d_m, float *d_v, int64_t *d_step, float lr,
                           float b1, float b2, float eps, float *d_losses, float *d_eps, float *d_eps_m,
                           float *d_eps_v, hipStream_t s) {
    if (!s) return fail(VPINN_E_INVALID, "capture needs a non-null stream");
    vpinn_status fr = batch_fresh(b);
    if (fr) return fr;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    hipEvent_t saved[VPINN_PROFILE_EVENTS];
    for (int i = 0; i < VPINN_PROFILE_EVENTS; ++i) {
        saved[i] = b->prof[i];
        b->prof[i] = nullptr;
    }
    VP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    vpinn_status st = batch_step(b, d_params, d_m, d_v, d_step, lr, b1, b2, eps, d_losses, d_eps, d_eps_m, d_eps_v, s);
    for (int i = 0; i < VPINN_PROFILE_EVENTS; ++i) b->prof[i] = saved[i];
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(VPINN_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    b->graph = g;
    VP_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return VPINN_OK;
}

int batch_device(const vpinn_batch *b) { return b->device; }

void batch_set_profile_events(vpinn_batch *b, void *const *events) {
    for (int i = 0; i < VPINN_PROFILE_EVENTS; ++i) b->prof[i] = events ? (hipEvent_t)events[i] : nullptr;
}

void batch_destroy(vpinn_batch *b) { delete b; }

static void drop_graph(vpinn_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

vpinn_status batch_get_tuning(const vpinn_batch *b, vpinn_tuning *out) {
    *out = b->plan.tune;
    return VPINN_OK;
}

vpinn_status batch_set_tuning(vpinn_batch *b, const vpinn_tuning *t) {
    if (!tuning_valid(*t)) return fail(VPINN_E_INVALID, "tuning value outside the supported lists");
    FusedPlan np;
    vpinn_status st = build_plan(b->probs.data(), (int)b->probs.size(), &b->cfg, b->device, *t, np);
    if (st) return st;
    drop_graph(b);
    b->plan = std::move(np);
    for (size_t i = 0; i < b->probs.size(); ++i) b->gens[i] = b->probs[i]->gen;
    return VPINN_OK;
}

// Time every tuning that can matter for this batch on its own data and keep the
// fastest (median of `reps` loss-and-gradient evaluations after one warm-up).
vpinn_status batch_autotune(vpinn_batch *b, const float *d_params, int32_t reps, vpinn_tuning *best_out,
                            hipStream_t s) {
    const FusedPlan &P0 = b->plan;
    bool has_fast = false, has_rows = false;
    for (const vpinn_problem *p : b->probs) {
        const int path = contraction_path(p);
        has_fast = has_fast || path == kPathFast;
        has_rows = has_rows || path == kPathRows1 || path == kPathRows2 || path == kPathRows4;
    }
    // storing the activations is a candidate only while their buffer fits the last-level cache: beyond
    // it the round trip is HBM traffic, and the reverse sweep recomputes them instead
    const bool may_store = (size_t)P0.tiles * P0.L * kActTile * sizeof(float) <= kActStoreMaxBytes;
    std::vector<vpinn_tuning> cand;
    for (int fw : {8, 12, 16})
        for (int cs = 0; cs <= (has_fast ? 2 : 0); ++cs)
            for (int rp : {2, 4, 8})
                for (int sa : {0, 1})
                    if ((has_rows || rp == 4) && (sa == 0 || may_store)) cand.push_back(vpinn_tuning{fw, cs, rp, sa, 0});
    // the one-pass step (its kernels ignore the other fields) where every problem fits it
    bool one_pass_ok = b->cfg.n_outputs != 2;
    for (const vpinn_problem *p : b->probs)
        one_pass_ok = one_pass_ok && !p->matfree && p->n_uniq == 0 && p->nq <= kGroupPts && p->ntest <= kKB;
    if (one_pass_ok) cand.push_back(vpinn_tuning{12, 0, 4, 0, 1});
    const int n = (int)b->probs.size();
    DevBuf losses, grads;
    VP_ALLOC(losses.reserve(sizeof(float) * 4 * (size_t)n));
    VP_ALLOC(grads.reserve(sizeof(float) * (size_t)P0.npf * (size_t)n));
    std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
    for (auto &e : ev) VP_HIP(hipEventCreate(&e));
    auto free_events = [&]() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    vpinn_tuning best = P0.tune;
    float best_ms = -1.f;
    AdamArgs none{};
    vpinn_status first_err = VPINN_OK;
    std::string first_msg;
    for (const vpinn_tuning &c : cand) {
        FusedPlan P;
        vpinn_status st = build_plan(b->probs.data(), n, &b->cfg, b->device, c, P);
        if (!st) st = run_plan(P, d_params, nullptr, true, losses.as<float>(), grads.as<float>(), nullptr, none,
                               nullptr, nullptr, s);
        for (int r = 0; r < reps && !st; ++r) {
            if (hipEventRecord(ev[2 * r], s) != hipSuccess) st = fail(VPINN_E_DEVICE, "hipEventRecord failed");
            if (!st) st = run_plan(P, d_params, nullptr, true, losses.as<float>(), grads.as<float>(), nullptr, none,
                                   nullptr, nullptr, s);
            if (!st && hipEventRecord(ev[2 * r + 1], s) != hipSuccess) st = fail(VPINN_E_DEVICE, "hipEventRecord failed");
        }
        if (!st && hipStreamSynchronize(s) != hipSuccess) st = fail(VPINN_E_DEVICE, "hipStreamSynchronize failed");
        if (st == VPINN_E_NOMEM) {
            // a candidate whose plan does not fit (stored activations of a large batch) is skipped; the
            // failed allocation's error is cleared so later launches do not report it
            (void)hipGetLastError();
            if (!first_err) {
                first_err = st;
                first_msg = vpinn_last_error();
            }
            continue;
        }
        if (st) {
            free_events();
            return st;
        }
        std::vector<float> t(reps);
        for (int r = 0; r < reps; ++r) (void)hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]);
        std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
        const float med = t[reps / 2];
        if (best_ms < 0.f || med < best_ms) {
            best_ms = med;
            best = c;
        }
    }
    free_events();
    if (best_ms < 0.f) return fail(first_err ? first_err : VPINN_E_NOMEM, "no tuning fits: " + first_msg);
    vpinn_status st = batch_set_tuning(b, &best);
    if (st) return st;
    if (best_out) *best_out = best;
    return VPINN_OK;
}

vpinn_status batch_replay(vpinn_batch *b, hipStream_t s) {
    if (!b->exec) return fail(VPINN_E_INVALID, "no captured step: call vpinn_batch_capture first");
    vpinn_status fr = batch_fresh(b);
    if (fr) return fr;
    VP_HIP(hipGraphLaunch(b->exec, s));
    return VPINN_OK;
}

}  // namespace vp
