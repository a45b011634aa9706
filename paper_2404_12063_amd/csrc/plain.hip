// The unfused ("plain") HIP path: one kernel per stage of Algorithm 3 and its
// backward pass, with every intermediate materialised in device memory, as a
// tensor framework would run it:
//   k_plain_fwd          network values and the two spatial tangents at every point,
//                  storing the activations (Sec. 2.2; forward-mode derivatives)
//   k_plain_contract     A[e,k] = sum_q (u_x G_x + u_y G_y), R = eps A - F, sum_k R^2
//   k_plain_adj_contract dL/du_x[e,q] = eps sum_k 2 c_v R[e,k] G_x[e,k,q] (and y)
//   k_plain_bwd          reverse sweep through value and tangent graphs, per-block
//                  weight-gradient partials
//   k_final_*      fixed-order reductions of the loss and gradient partials
// One lane owns one point; weights are wavefront-uniform (scalar loads).
#include <mutex>

#include "device_common.h"
#include "internal.h"

namespace vp {

// ---------------------------------------------------------------------------
// parameter layout conversion
// ---------------------------------------------------------------------------
// output `head` of a network with `heads` linear outputs goes to the W_out, b_out slots
__global__ void k_plain_pack(const float *__restrict__ src, int H, int L, int heads, int head,
                             float *__restrict__ dst) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_padded(L)) return;
    float v = 0.0f;
    if (t < 64) {
        const int o = t / 2, i = t % 2;
        if (o < H) v = src[o * 2 + i];
    } else if (t < 96) {
        const int o = t - 64;
        if (o < H) v = src[2 * H + o];
    } else if (t < off_wout(L)) {
        const int l = 2 + (t - 96) / kLayerStride, r = (t - 96) % kLayerStride;
        const int64_t base = hoff_w(H, l);
        if (r < PW * PW) {
            const int o = r / PW, i = r % PW;
            if (o < H && i < H) v = src[base + o * H + i];
        } else {
            const int o = r - PW * PW;
            if (o < H) v = src[base + (int64_t)H * H + o];
        }
    } else {
        const int r = t - off_wout(L);
        const int64_t base = hoff_w(H, L + 1);
        if (r < PW) {
            if (r < H) v = src[base + (int64_t)head * H + r];
        } else {
            v = src[base + (int64_t)heads * H + head];
        }
    }
    dst[t] = v;
}

// padded index of flat parameter j (width H, L hidden layers)
__device__ inline int padded_index(int H, int L, int64_t j) {
    if (j < 2 * H) return (int)j;
    if (j < 3 * H) return kOffB1 + (int)(j - 2 * H);
    const int64_t lay = (int64_t)H * H + H;
    const int64_t r0 = j - 3 * H;
    if (r0 < (int64_t)(L - 1) * lay) {
        const int l = 2 + (int)(r0 / lay);
        const int r = (int)(r0 % lay);
        if (r < H * H) return off_w(l) + (r / H) * PW + (r % H);
        return off_b(l) + (r - H * H);
    }
    const int r = (int)(r0 - (int64_t)(L - 1) * lay);
    return r < H ? off_wout(L) + r : off_wout(L) + PW;
}

// grad[j] = sum over partial rows of the padded entry of j, in row order
__global__ void k_plain_final_grad(const float *__restrict__ gpart, int rows, int H, int L, int64_t np_flat,
                             float *__restrict__ grad) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= np_flat) return;
    const int pj = padded_index(H, L, j);
    double acc = 0.0;
    for (int r = 0; r < rows; ++r) acc += (double)gpart[(int64_t)r * kMaxPadded + pj];
    grad[j] = (float)acc;
}

// loss components from per-element (or per-block) partials, fixed-order tree
constexpr int kFinThreads = 1024;
__device__ inline double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kFinThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kFinThreads) void k_plain_final_loss(
    const double *__restrict__ lv_part, int64_t n_lv, double cv, const double *__restrict__ ep_part, int64_t n_ep,
    const float *__restrict__ u, const float *__restrict__ tgt, int64_t n_int, int64_t n_bnd, int64_t n_sen,
    float tau, float gamma, float *__restrict__ loss_out, float *__restrict__ grad_eps) {
    __shared__ double red[kFinThreads];
    double s_lv = 0.0, s_ep = 0.0, s_b = 0.0, s_s = 0.0;
    for (int64_t i = threadIdx.x; i < n_lv; i += kFinThreads) s_lv += lv_part[i];
    if (ep_part)
        for (int64_t i = threadIdx.x; i < n_ep; i += kFinThreads) s_ep += ep_part[i];
    for (int64_t i = threadIdx.x; i < n_bnd + n_sen; i += kFinThreads) {
        const double d = (double)u[n_int + i] - (double)tgt[i];
        if (i < n_bnd) s_b += d * d;
        else s_s += d * d;
    }
    s_lv = block_sum(s_lv, red);
    s_ep = block_sum(s_ep, red);
    s_b = block_sum(s_b, red);
    s_s = block_sum(s_s, red);
    if (threadIdx.x == 0) {
        const double Lv = cv * s_lv;
        const double Lb = n_bnd ? s_b / (double)n_bnd : 0.0;
        const double Ls = n_sen ? s_s / (double)n_sen : 0.0;
        if (loss_out) {
            loss_out[0] = (float)(Lv + (double)tau * Lb + (double)gamma * Ls);
            loss_out[1] = (float)Lv;
            loss_out[2] = (float)Lb;
            loss_out[3] = (float)Ls;
        }
        if (grad_eps) *grad_eps = (float)(2.0 * cv * s_ep);
    }
}

// ---------------------------------------------------------------------------
// forward: values and tangents, lane per point
// act layout (slot-major, point-minor): layer 1 a in slots 0..31; layer l >= 2
// a, p_x, p_y (pre-activation tangents) in slots 32 + 96 (l-2) + {0, 32, 64}.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int act_slots(int L) { return 32 + 96 * (L - 1); }

template <int L>
__global__ __launch_bounds__(256) void k_plain_fwd(const float *__restrict__ w, const float2 *__restrict__ pts,
                                             int64_t np, float *__restrict__ u, float *__restrict__ ux,
                                             float *__restrict__ uy, float *__restrict__ act) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= np) return;
    const float2 xy = pts[p];
    float a[PW], tx[PW], ty[PW];
#pragma unroll
    for (int o = 0; o < PW; ++o) {
        const float w0 = w[2 * o], w1 = w[2 * o + 1];
        const float av = tanh_f32(fmaf(w0, xy.x, fmaf(w1, xy.y, w[kOffB1 + o])));
        const float s = 1.0f - av * av;
        a[o] = av;
        tx[o] = s * w0;
        ty[o] = s * w1;
        if (act) act[(int64_t)o * np + p] = av;
    }
#pragma unroll
    for (int l = 2; l <= L; ++l) {
        const float *W = w + off_w(l);
        const float *b = w + off_b(l);
        float na[PW], ntx[PW], nty[PW];
#pragma unroll
        for (int o = 0; o < PW; ++o) {
            float z = b[o], px = 0.0f, py = 0.0f;
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                const float wv = W[o * PW + i];
                z = fmaf(wv, a[i], z);
                px = fmaf(wv, tx[i], px);
                py = fmaf(wv, ty[i], py);
            }
            const float av = tanh_f32(z);
            const float s = 1.0f - av * av;
            na[o] = av;
            ntx[o] = s * px;
            nty[o] = s * py;
            if (act) {
                const int64_t slot = 32 + 96 * (l - 2) + o;
                act[slot * np + p] = av;
                act[(slot + 32) * np + p] = px;
                act[(slot + 64) * np + p] = py;
            }
        }
#pragma unroll
        for (int o = 0; o < PW; ++o) {
            a[o] = na[o];
            tx[o] = ntx[o];
            ty[o] = nty[o];
        }
    }
    const float *Wo = w + off_wout(L);
    float uu = Wo[PW], gx = 0.0f, gy = 0.0f;
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        uu = fmaf(Wo[i], a[i], uu);
        gx = fmaf(Wo[i], tx[i], gx);
        gy = fmaf(Wo[i], ty[i], gy);
    }
    if (u) u[p] = uu;
    if (ux) ux[p] = gx;
    if (uy) uy[p] = gy;
}

// ---------------------------------------------------------------------------
// contraction (Alg. 3): wavefront per element, lanes over quadrature points
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_plain_contract(const float *__restrict__ Gx, const float *__restrict__ Gy,
                                                  const float *__restrict__ F, const float *__restrict__ ux,
                                                  const float *__restrict__ uy, const float *__restrict__ eps_ptr,
                                                  int64_t n_elem, int nq, int ntest, int64_t gstride,
                                                  float *__restrict__ A,
                                                  float *__restrict__ R, double *__restrict__ lv_e,
                                                  double *__restrict__ ep_e) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 4 + wave;
    if (e >= n_elem) return;
    const float eps = eps_ptr ? *eps_ptr : 1.0f;
    double le = 0.0, lp = 0.0;
    for (int k = 0; k < ntest; ++k) {
        const int64_t base = e * gstride + (int64_t)k * nq;
        float acc = 0.0f;
        for (int q = lane; q < nq; q += 64)
            acc = fmaf(ux[e * nq + q], Gx[base + q], fmaf(uy[e * nq + q], Gy[base + q], acc));
        acc = wave_sum(acc);
        const float r = eps * acc - F[e * ntest + k];
        if (lane == 0) {
            if (A) A[e * ntest + k] = acc;
            R[e * ntest + k] = r;
        }
        le += (double)r * (double)r;
        lp += (double)r * (double)acc;
    }
    if (lane == 0) {
        if (lv_e) lv_e[e] = le;
        if (ep_e) ep_e[e] = lp;
    }
}

// adjoint of the contraction, thread per interior point
__global__ __launch_bounds__(256) void k_plain_adj_contract(const float *__restrict__ Gx, const float *__restrict__ Gy,
                                                      const float *__restrict__ R, const float *__restrict__ eps_ptr,
                                                      float two_cv, int64_t n_elem, int nq, int ntest,
                                                      int64_t gstride, float *__restrict__ uxb,
                                                      float *__restrict__ uyb) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_elem * nq) return;
    const int64_t e = t / nq;
    const int q = (int)(t - e * nq);
    const float ce = two_cv * (eps_ptr ? *eps_ptr : 1.0f);
    float bx = 0.0f, by = 0.0f;
    for (int k = 0; k < ntest; ++k) {
        const float rb = R[e * ntest + k];
        const int64_t o = e * gstride + (int64_t)k * nq + q;
        bx = fmaf(rb, Gx[o], bx);
        by = fmaf(rb, Gy[o], by);
    }
    uxb[t] = ce * bx;
    uyb[t] = ce * by;
}

// ---------------------------------------------------------------------------
// backward: lane per point; the cross-point sums of weight gradients are
// formed per wavefront through shared memory (each lane owns a 4x4 block of
// every 32x32 weight-gradient matrix), then per block.
// ---------------------------------------------------------------------------
constexpr int kBwdThreads = 256;
constexpr int kLs = 36;  // shared row stride (floats), keeps float4 alignment

template <int L>
struct BwdShared {
    float z[4][64][kLs];
    float a[4][64][kLs];
};

__device__ inline void load_raw(const float *__restrict__ act, int64_t np, int64_t p, bool valid, int l,
                                const float *__restrict__ w, float a[PW], float px[PW], float py[PW]) {
    if (l == 1) {
#pragma unroll
        for (int o = 0; o < PW; ++o) {
            a[o] = valid ? act[(int64_t)o * np + p] : 0.0f;
            px[o] = w[2 * o];
            py[o] = w[2 * o + 1];
        }
    } else {
        const int64_t slot = 32 + 96 * (l - 2);
#pragma unroll
        for (int o = 0; o < PW; ++o) {
            a[o] = valid ? act[(slot + o) * np + p] : 0.0f;
            px[o] = valid ? act[(slot + 32 + o) * np + p] : 0.0f;
            py[o] = valid ? act[(slot + 64 + o) * np + p] : 0.0f;
        }
    }
}

__device__ inline void load_tangent(const float *__restrict__ act, int64_t np, int64_t p, bool valid, int l,
                                    const float *__restrict__ w, float a[PW], float tx[PW], float ty[PW]) {
    float px[PW], py[PW];
    load_raw(act, np, p, valid, l, w, a, px, py);
#pragma unroll
    for (int o = 0; o < PW; ++o) {
        const float s = 1.0f - a[o] * a[o];
        tx[o] = s * px[o];
        ty[o] = s * py[o];
    }
}

// acc[r*4+c] += sum over the wave's 64 points of out[4*ob+r] * in[4*ib+c]
__device__ inline void wave_gemm(float (*Zs)[kLs], float (*As)[kLs], int lane, const float out[PW],
                                 const float in[PW], float acc[16]) {
#pragma unroll
    for (int o = 0; o < PW; o += 4) {
        *reinterpret_cast<float4 *>(&Zs[lane][o]) = make_float4(out[o], out[o + 1], out[o + 2], out[o + 3]);
        *reinterpret_cast<float4 *>(&As[lane][o]) = make_float4(in[o], in[o + 1], in[o + 2], in[o + 3]);
    }
    __syncthreads();
    const int ob = lane >> 3, ib = lane & 7;
    for (int p = 0; p < 64; ++p) {
        const float4 z = *reinterpret_cast<const float4 *>(&Zs[p][4 * ob]);
        const float4 a = *reinterpret_cast<const float4 *>(&As[p][4 * ib]);
        const float zz[4] = {z.x, z.y, z.z, z.w}, aa[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r * 4 + c] = fmaf(zz[r], aa[c], acc[r * 4 + c]);
    }
    __syncthreads();
}

// acc += sum over the wave's points in this lane's half of column (lane % 32) of v
__device__ inline void column_sum(float (*Zs)[kLs], int lane, const float v[PW], float &acc) {
#pragma unroll
    for (int o = 0; o < PW; o += 4)
        *reinterpret_cast<float4 *>(&Zs[lane][o]) = make_float4(v[o], v[o + 1], v[o + 2], v[o + 3]);
    __syncthreads();
    const int col = lane & 31, p0 = (lane >> 5) * 32;
    float s = 0.0f;
#pragma unroll 8
    for (int p = 0; p < 32; ++p) s += Zs[p0 + p][col];
    acc += s;
    __syncthreads();
}

template <int L>
__global__ __launch_bounds__(kBwdThreads) void k_plain_bwd(const float *__restrict__ w, const float2 *__restrict__ pts,
                                                     int64_t n_int, int64_t np, const float *__restrict__ act,
                                                     const float *__restrict__ uxb_in,
                                                     const float *__restrict__ uyb_in, const float *__restrict__ u,
                                                     const float *__restrict__ tgt, int64_t n_bnd, float wb2,
                                                     float ws2, float *__restrict__ gpart) {
    __shared__ BwdShared<L> sh;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float(*Zs)[kLs] = sh.z[wave];
    float(*As)[kLs] = sh.a[wave];
    constexpr int NW = L > 1 ? L - 1 : 1;
    float accW[NW][16];
#pragma unroll
    for (int m = 0; m < NW; ++m)
#pragma unroll
        for (int r = 0; r < 16; ++r) accW[m][r] = 0.0f;
    // column sums: [l-1] b_l for l = 1..L, [L] W1 column 0, [L+1] W1 column 1, [L+2] W_out
    float accV[L + 3];
#pragma unroll
    for (int m = 0; m < L + 3; ++m) accV[m] = 0.0f;
    float accBo = 0.0f;

    for (int64_t base = (int64_t)blockIdx.x * kBwdThreads; base < np; base += (int64_t)gridDim.x * kBwdThreads) {
        const int64_t p = base + threadIdx.x;
        const bool valid = p < np;
        float ub = 0.0f, uxb = 0.0f, uyb = 0.0f;
        float2 xy = make_float2(0.0f, 0.0f);
        if (valid) {
            xy = pts[p];
            if (p < n_int) {
                uxb = uxb_in[p];
                uyb = uyb_in[p];
            } else {
                const int64_t r = p - n_int;
                ub = (r < n_bnd ? wb2 : ws2) * (u[p] - tgt[r]);
            }
        }
        float abar[PW], txbar[PW], tybar[PW];
        {
            float aL[PW], txL[PW], tyL[PW], v[PW];
            load_tangent(act, np, p, valid, L, w, aL, txL, tyL);
            const float *Wo = w + off_wout(L);
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                v[i] = ub * aL[i] + uxb * txL[i] + uyb * tyL[i];
                abar[i] = ub * Wo[i];
                txbar[i] = uxb * Wo[i];
                tybar[i] = uyb * Wo[i];
            }
            column_sum(Zs, lane, v, accV[L + 2]);
            accBo += ub;
        }
#pragma unroll
        for (int l = L; l >= 1; --l) {
            float zbar[PW], pxbar[PW], pybar[PW];
            {
                float al[PW], pxl[PW], pyl[PW];
                load_raw(act, np, p, valid, l, w, al, pxl, pyl);
#pragma unroll
                for (int o = 0; o < PW; ++o) {
                    const float s = 1.0f - al[o] * al[o];
                    pxbar[o] = s * txbar[o];
                    pybar[o] = s * tybar[o];
                    const float sbar = txbar[o] * pxl[o] + tybar[o] * pyl[o];
                    zbar[o] = s * (abar[o] - 2.0f * al[o] * sbar);
                }
            }
            column_sum(Zs, lane, zbar, accV[l - 1]);
            if (l >= 2) {
                float ai[PW], txi[PW], tyi[PW];
                load_tangent(act, np, p, valid, l - 1, w, ai, txi, tyi);
                wave_gemm(Zs, As, lane, zbar, ai, accW[l - 2]);
                wave_gemm(Zs, As, lane, pxbar, txi, accW[l - 2]);
                wave_gemm(Zs, As, lane, pybar, tyi, accW[l - 2]);
                const float *W = w + off_w(l);
#pragma unroll
                for (int i = 0; i < PW; ++i) {
                    float sa = 0.0f, sx = 0.0f, sy = 0.0f;
#pragma unroll
                    for (int o = 0; o < PW; ++o) {
                        const float wv = W[o * PW + i];
                        sa = fmaf(wv, zbar[o], sa);
                        sx = fmaf(wv, pxbar[o], sx);
                        sy = fmaf(wv, pybar[o], sy);
                    }
                    abar[i] = sa;
                    txbar[i] = sx;
                    tybar[i] = sy;
                }
            } else {
                float c0[PW], c1[PW];
#pragma unroll
                for (int o = 0; o < PW; ++o) {
                    c0[o] = fmaf(zbar[o], xy.x, pxbar[o]);
                    c1[o] = fmaf(zbar[o], xy.y, pybar[o]);
                }
                column_sum(Zs, lane, c0, accV[L]);
                column_sum(Zs, lane, c1, accV[L + 1]);
            }
        }
    }

    // block combine: each wave writes its full padded partial, then fixed-order sum over waves
    float *red = &sh.z[0][0][0];  // 4 * kMaxPadded floats fit in the shared buffers
    static_assert(sizeof(BwdShared<L>) >= 4 * kMaxPadded * sizeof(float), "shared scratch too small");
    float *mine = red + wave * kMaxPadded;
    __syncthreads();
    {
        const int ob = lane >> 3, ib = lane & 7;
#pragma unroll
        for (int l = 2; l <= L; ++l)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) mine[off_w(l) + (4 * ob + r) * PW + 4 * ib + c] = accW[l - 2][r * 4 + c];
        float full[L + 3];
#pragma unroll
        for (int m = 0; m < L + 3; ++m) full[m] = accV[m] + __shfl_xor(accV[m], 32, 64);
        const float bo = wave_sum(accBo);
        if (lane < 32) {
#pragma unroll
            for (int l = 1; l <= L; ++l) mine[off_b(l) + lane] = full[l - 1];
            mine[off_w(1) + 2 * lane] = full[L];
            mine[off_w(1) + 2 * lane + 1] = full[L + 1];
            mine[off_wout(L) + lane] = full[L + 2];
        }
        if (lane == 0) mine[off_wout(L) + PW] = bo;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n_padded(L); j += kBwdThreads)
        gpart[(int64_t)blockIdx.x * kMaxPadded + j] = ((red[j] + red[kMaxPadded + j]) + red[2 * kMaxPadded + j]) +
                                                      red[3 * kMaxPadded + j];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
vpinn_status pack_params(const float *d_params, int H, int L, int heads, int head, float *d_wpad, hipStream_t s) {
    k_plain_pack<<<(n_padded(L) + 255) / 256, 256, 0, s>>>(d_params, H, L, heads, head, d_wpad);
    VP_HIP(hipGetLastError());
    return VPINN_OK;
}

template <int L>
static void launch_fwd(const float *w, const float2 *pts, int64_t np, float *u, float *ux, float *uy, float *act,
                       hipStream_t s) {
    k_plain_fwd<L><<<dim3((unsigned)((np + 255) / 256)), 256, 0, s>>>(w, pts, np, u, ux, uy, act);
}

static vpinn_status fwd_dispatch(int L, const float *w, const float2 *pts, int64_t np, float *u, float *ux, float *uy,
                                 float *act, hipStream_t s) {
    if (np == 0) return VPINN_OK;
    switch (L) {
    case 1: launch_fwd<1>(w, pts, np, u, ux, uy, act, s); break;
    case 2: launch_fwd<2>(w, pts, np, u, ux, uy, act, s); break;
    case 3: launch_fwd<3>(w, pts, np, u, ux, uy, act, s); break;
    case 4: launch_fwd<4>(w, pts, np, u, ux, uy, act, s); break;
    default: return fail(VPINN_E_UNSUPPORTED, "n_hidden out of range");
    }
    VP_HIP(hipGetLastError());
    return VPINN_OK;
}

// prediction error against reference values: blocks stride over the points and keep
// FP64 sums of |d|, d^2, ref^2 and the max |d| (d = p - ref); each block's four
// values go to part[block] (wavefronts added in order), and one block adds the
// partials in block order, so the result does not depend on timing
constexpr int kErrThreads = 256, kErrMaxBlocks = 512;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(kErrThreads) void k_err_partial(const float *__restrict__ p, const float *__restrict__ ref,
                                                              int64_t n, double *__restrict__ part) {
    __shared__ double red[kErrThreads / 64][4];
    double sa = 0.0, mx = 0.0, sd = 0.0, sr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kErrThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kErrThreads) {
        const double r = (double)ref[i], d = (double)p[i] - r;
        sa += fabs(d);
        mx = fmax(mx, fabs(d));
        sd += d * d;
        sr += r * r;
    }
    sa = wave_sum(sa);
    sd = wave_sum(sd);
    sr = wave_sum(sr);
    mx = wave_max(mx);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = sa;
        red[w][1] = mx;
        red[w][2] = sd;
        red[w][3] = sr;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = red[0][threadIdx.x];
        for (int k = 1; k < kErrThreads / 64; ++k)
            v = threadIdx.x == 1 ? fmax(v, red[k][1]) : v + red[k][threadIdx.x];
        part[blockIdx.x * 4 + threadIdx.x] = v;
    }
}

__global__ void k_err_final(const double *__restrict__ part, int blocks, int64_t n, double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double sa = 0.0, mx = 0.0, sd = 0.0, sr = 0.0;
    for (int b = 0; b < blocks; ++b) {
        sa += part[4 * b];
        mx = fmax(mx, part[4 * b + 1]);
        sd += part[4 * b + 2];
        sr += part[4 * b + 3];
    }
    out[0] = sa / (double)n;
    out[1] = mx;
    out[2] = sqrt(sd) / sqrt(sr);
}

vpinn_status error_stats(int64_t n, const float *d_p, const float *d_ref, double *d_part, double *d_out,
                         hipStream_t s) {
    const int blocks = (int)std::min<int64_t>(kErrMaxBlocks, (n + kErrThreads - 1) / kErrThreads);
    k_err_partial<<<blocks, kErrThreads, 0, s>>>(d_p, d_ref, n, d_part);
    k_err_final<<<1, 64, 0, s>>>(d_part, blocks, n, d_out);
    VP_HIP(hipGetLastError());
    return VPINN_OK;
}

// workspace of the allocation-free prediction error: the network values of up to
// VPINN_NOALLOC_MAX_POINTS points, then the block partials of error_stats.  A file-scope
// device array: every device the library runs on holds its own copy, at its own address,
// until the process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: only the address hipGetSymbolAddress returns for the current device is
// passed to kernels.
constexpr size_t kNoAllocValueBytes = sizeof(float) * (size_t)VPINN_NOALLOC_MAX_POINTS;
constexpr size_t kNoAllocBytes = kNoAllocValueBytes + sizeof(double) * 4 * kErrMaxBlocks;
static_assert(kNoAllocValueBytes % sizeof(double) == 0, "partials must stay 8-byte aligned");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

vpinn_status noalloc_workspace(float **values, double **partials) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    VP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(VPINN_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // once per device, with that device current
        void *p = nullptr;
        VP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(VPINN_E_DEVICE, "hipGetSymbolAddress returned no address for the workspace");
        addr[dev] = p;
    }
    *values = static_cast<float *>(addr[dev]);
    *partials = reinterpret_cast<double *>(static_cast<unsigned char *>(addr[dev]) + kNoAllocValueBytes);
    return VPINN_OK;
}

constexpr int kBwdMaxBlocks = 512;

template <int L>
static void launch_bwd(int blocks, const float *w, const float2 *pts, int64_t n_int, int64_t np, const float *act,
                       const float *uxb, const float *uyb, const float *u, const float *tgt, int64_t n_bnd,
                       float wb2, float ws2, float *gpart, hipStream_t s) {
    k_plain_bwd<L><<<blocks, kBwdThreads, 0, s>>>(w, pts, n_int, np, act, uxb, uyb, u, tgt, n_bnd, wb2, ws2, gpart);
}

vpinn_status plain_loss_grad(vpinn_problem *p, const vpinn_loss_cfg *cfg, const float *d_params,
                             const float *d_eps, float *d_loss, float *d_grad, float *d_grad_eps, float *d_R_out,
                             hipStream_t s) {
    const int L = cfg->n_hidden, H = cfg->width;
    const int64_t np = p->all_pts(), n_int = p->n_pts;
    const bool want_grad = d_grad != nullptr;
    const int64_t nRA = p->n_elem * p->ntest;
    const int bwd_blocks = (int)std::min<int64_t>(kBwdMaxBlocks, (np + kBwdThreads - 1) / kBwdThreads);
    VP_HIP(p->wpad.reserve(sizeof(float) * kMaxPadded));
    VP_HIP(p->u.reserve(sizeof(float) * np));
    VP_HIP(p->ux.reserve(sizeof(float) * np));
    VP_HIP(p->uy.reserve(sizeof(float) * np));
    VP_HIP(p->A.reserve(sizeof(float) * nRA));
    VP_HIP(p->R.reserve(sizeof(float) * nRA));
    VP_HIP(p->loss_e.reserve(sizeof(double) * p->n_elem));
    VP_HIP(p->eps_part.reserve(sizeof(double) * p->n_elem));
    if (want_grad) {
        VP_HIP(p->act.reserve(sizeof(float) * act_slots(L) * np));
        VP_HIP(p->uxb.reserve(sizeof(float) * n_int));
        VP_HIP(p->uyb.reserve(sizeof(float) * n_int));
        VP_HIP(p->gpart.reserve(sizeof(float) * kMaxPadded * kBwdMaxBlocks));
    }
    float *w = p->wpad.as<float>();
    vpinn_status st = pack_params(d_params, H, L, 1, 0, w, s);
    if (st) return st;
    st = fwd_dispatch(L, w, p->pts.as<float2>(), np, p->u.as<float>(), p->ux.as<float>(), p->uy.as<float>(),
                      want_grad ? p->act.as<float>() : nullptr, s);
    if (st) return st;
    float *R = d_R_out ? d_R_out : p->R.as<float>();
    k_plain_contract<<<dim3((unsigned)((p->n_elem + 3) / 4)), 256, 0, s>>>(
        p->Gx.as<float>(), p->Gy.as<float>(), p->F.as<float>(), p->ux.as<float>(), p->uy.as<float>(), d_eps,
        p->n_elem, p->nq, p->ntest, p->gstride(), p->A.as<float>(), R, p->loss_e.as<double>(),
        p->eps_part.as<double>());
    VP_HIP(hipGetLastError());
    if (d_R_out && !d_loss) return VPINN_OK;
    const double cv = cfg->loss_norm == VPINN_NORM_ELEM ? 1.0 / (double)p->n_elem : 1.0 / (double)p->ntest;
    if (want_grad) {
        k_plain_adj_contract<<<dim3((unsigned)((n_int + 255) / 256)), 256, 0, s>>>(
            p->Gx.as<float>(), p->Gy.as<float>(), R, d_eps, (float)(2.0 * cv), p->n_elem, p->nq, p->ntest,
            p->gstride(), p->uxb.as<float>(), p->uyb.as<float>());
        VP_HIP(hipGetLastError());
        const float wb2 = p->n_bnd ? (float)(2.0 * cfg->tau / (double)p->n_bnd) : 0.0f;
        const float ws2 = p->n_sen ? (float)(2.0 * cfg->gamma / (double)p->n_sen) : 0.0f;
        switch (L) {
        case 1: launch_bwd<1>(bwd_blocks, w, p->pts.as<float2>(), n_int, np, p->act.as<float>(), p->uxb.as<float>(),
                              p->uyb.as<float>(), p->u.as<float>(), p->tgt.as<float>(), p->n_bnd, wb2, ws2,
                              p->gpart.as<float>(), s); break;
        case 2: launch_bwd<2>(bwd_blocks, w, p->pts.as<float2>(), n_int, np, p->act.as<float>(), p->uxb.as<float>(),
                              p->uyb.as<float>(), p->u.as<float>(), p->tgt.as<float>(), p->n_bnd, wb2, ws2,
                              p->gpart.as<float>(), s); break;
        case 3: launch_bwd<3>(bwd_blocks, w, p->pts.as<float2>(), n_int, np, p->act.as<float>(), p->uxb.as<float>(),
                              p->uyb.as<float>(), p->u.as<float>(), p->tgt.as<float>(), p->n_bnd, wb2, ws2,
                              p->gpart.as<float>(), s); break;
        case 4: launch_bwd<4>(bwd_blocks, w, p->pts.as<float2>(), n_int, np, p->act.as<float>(), p->uxb.as<float>(),
                              p->uyb.as<float>(), p->u.as<float>(), p->tgt.as<float>(), p->n_bnd, wb2, ws2,
                              p->gpart.as<float>(), s); break;
        default: return fail(VPINN_E_UNSUPPORTED, "n_hidden out of range");
        }
        VP_HIP(hipGetLastError());
        const int64_t npf = vpinn_n_params(H, L);
        k_plain_final_grad<<<dim3((unsigned)((npf + 255) / 256)), 256, 0, s>>>(p->gpart.as<float>(), bwd_blocks, H, L, npf,
                                                                      d_grad);
        VP_HIP(hipGetLastError());
    }
    if (d_loss || d_grad_eps) {
        k_plain_final_loss<<<1, kFinThreads, 0, s>>>(p->loss_e.as<double>(), p->n_elem, cv, p->eps_part.as<double>(),
                                               p->n_elem, p->u.as<float>(), p->tgt.as<float>(), n_int, p->n_bnd,
                                               p->n_sen, cfg->tau, cfg->gamma, d_loss, d_grad_eps);
        VP_HIP(hipGetLastError());
    }
    return VPINN_OK;
}

}  // namespace vp
