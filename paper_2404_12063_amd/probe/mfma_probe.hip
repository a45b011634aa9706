// Measurements behind the network kernels' product design, callable through a C ABI
// (tests/test_gpu_mfma_probe.py drives them; they are not part of the training path).
//
// 1. Accuracy: a 16x32 by 32x16 product per block as the FP32 MFMA (16x16x4, eight K
//    steps) and as split-bf16 MFMAs (16x16x32, three round-to-nearest pieces per operand,
//    the six piece products with i + j <= 2, and all nine), returned to the host, which
//    compares them with the FP64 product.
// 2. Co-execution: one block of eight wavefronts on one CU; wavefronts w and w + 4 share a
//    SIMD.  Waves 0-3 issue independent MFMA chains, waves 4-7 independent v_fma_f32
//    chains; each wave's span is read with s_memtime.  Running either role alone and both
//    together shows whether the matrix products take vector-ALU time.
#include <hip/hip_runtime.h>
#include <cstdint>

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ unsigned pk(float x, float y) {
    const fl2 v = {x, y};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf2));
}

__device__ __forceinline__ void split(const float (&v)[8], u4 (&p)[3]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float x = v[2 * q], y = v[2 * q + 1];
        const unsigned h = pk(x, y);
        x -= __uint_as_float(h << 16);
        y -= __uint_as_float(h & 0xffff0000u);
        const unsigned m = pk(x, y);
        x -= __uint_as_float(m << 16);
        y -= __uint_as_float(m & 0xffff0000u);
        p[0][q] = h;
        p[1][q] = m;
        p[2][q] = pk(x, y);
    }
}

__device__ __forceinline__ f4 mb(u4 a, u4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// W: [blocks][16][32], V: [blocks][32][16], outputs [blocks][16][16] each
__global__ __launch_bounds__(64) void k_products(const float *W, const float *V, float *d32, float *d6, float *d9) {
    const int b = blockIdx.x, l = threadIdx.x, i = l & 15, g = l >> 4;
    const float *w = W + (size_t)b * 512, *v = V + (size_t)b * 512;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int kk = 16 * (s >> 2) + 4 * g + (s & 3);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[i * 32 + kk], v[kk * 16 + i], acc, 0, 0, 0);
    }
    float a8[8], b8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int kk = 16 * (j >> 2) + 4 * g + (j & 3);
        a8[j] = w[i * 32 + kk];
        b8[j] = v[kk * 16 + i];
    }
    u4 A[3], B[3];
    split(a8, A);
    split(b8, B);
    f4 c6 = {0.f, 0.f, 0.f, 0.f}, c9 = {0.f, 0.f, 0.f, 0.f};
    c6 = mb(A[0], B[2], c6);
    c6 = mb(A[1], B[1], c6);
    c6 = mb(A[2], B[0], c6);
    c6 = mb(A[0], B[1], c6);
    c6 = mb(A[1], B[0], c6);
    c6 = mb(A[0], B[0], c6);
    c9 = mb(A[2], B[2], c9);
    c9 = mb(A[1], B[2], c9);
    c9 = mb(A[2], B[1], c9);
    c9 = mb(A[0], B[2], c9);
    c9 = mb(A[1], B[1], c9);
    c9 = mb(A[2], B[0], c9);
    c9 = mb(A[0], B[1], c9);
    c9 = mb(A[1], B[0], c9);
    c9 = mb(A[0], B[0], c9);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const size_t o = (size_t)b * 256 + (4 * g + r) * 16 + i;
        d32[o] = acc[r];
        d6[o] = c6[r];
        d9[o] = c9[r];
    }
}

template <int KIND>
__device__ __forceinline__ f4 op(f4 c, float a, float b, bf8 av, bf8 bv, s4v as, s4v bs) {
    if (KIND == 0) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    if (KIND == 1) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as, bs, c, 0, 0, 0);
}

template <int KIND>
__device__ void mfma_loop(int iters, float seed, float *out) {
    f4 acc[8];
    for (int j = 0; j < 8; ++j) acc[j] = f4{seed, 0.f, 0.f, (float)j};
    const float a = seed, b = seed * 0.5f;
    bf8 av, bv;
    s4v as, bs;
    for (int j = 0; j < 8; ++j) {
        av[j] = (__bf16)(seed + j);
        bv[j] = (__bf16)(seed - j);
    }
    for (int j = 0; j < 4; ++j) {
        as[j] = (short)(0x3f80 + j);
        bs[j] = (short)(0x3f00 + j);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = op<KIND>(acc[j], a, b, av, bv, as, bs);
    }
    float s = 0.f;
    for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[threadIdx.x] = s;
}

// 64 independent FMAs per iteration (eight chains, unrolled), so the loop branch is rare
__device__ void valu_loop(int iters, float seed, float *out) {
    float x[8];
    for (int j = 0; j < 8; ++j) x[j] = seed + j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = fmaf(x[j], 0.9999f, 1e-4f);
    }
    float s = 0.f;
    for (int j = 0; j < 8; ++j) s += x[j];
    out[threadIdx.x] = s;
}

template <int KIND>
__global__ __launch_bounds__(512) void k_coexec(int mode, int im, int iv, float seed, float *out, uint64_t *t) {
    const int w = threadIdx.x >> 6;
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    if (w < 4) {
        if (mode & 1) mfma_loop<KIND>(im, seed, out);
    } else {
        if (mode & 2) valu_loop(iv, seed, out);
    }
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    if ((threadIdx.x & 63) == 0) {
        t[2 * w] = t0;
        t[2 * w + 1] = t1;
    }
}

}  // namespace

extern "C" {

// products of n_blocks random 16x32 by 32x16 pairs (host W [n][16][32], V [n][32][16]);
// writes the three device results to host d32, d6, d9 ([n][16][16]).  0 on success.
int mfma_probe_products(int n_blocks, const float *W, const float *V, float *d32, float *d6, float *d9) {
    if (n_blocks <= 0 || n_blocks > 65536 || !W || !V || !d32 || !d6 || !d9) return 1;
    const size_t ni = (size_t)n_blocks * 512, no = (size_t)n_blocks * 256;
    float *dW = nullptr, *dV = nullptr, *o = nullptr;
    int rc = 0;
    if (hipMalloc(&dW, ni * 4) != hipSuccess || hipMalloc(&dV, ni * 4) != hipSuccess ||
        hipMalloc(&o, 3 * no * 4) != hipSuccess) {
        rc = 2;
    } else if (hipMemcpy(dW, W, ni * 4, hipMemcpyHostToDevice) != hipSuccess ||
               hipMemcpy(dV, V, ni * 4, hipMemcpyHostToDevice) != hipSuccess) {
        rc = 3;
    } else {
        hipLaunchKernelGGL(k_products, dim3(n_blocks), dim3(64), 0, 0, dW, dV, o, o + no, o + 2 * no);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) rc = 4;
        else if (hipMemcpy(d32, o, no * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                 hipMemcpy(d6, o + no, no * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                 hipMemcpy(d9, o + 2 * no, no * 4, hipMemcpyDeviceToHost) != hipSuccess)
            rc = 5;
    }
    (void)hipFree(dW);
    (void)hipFree(dV);
    (void)hipFree(o);
    return rc;
}

// one block of eight wavefronts: kind 0 FP32 16x16x4, 1 bf16 16x16x32, 2 bf16 16x16x16;
// mode 1 MFMA waves only, 2 VALU waves only, 3 both; im iterations of 8 MFMAs, iv of 64
// FMAs.  Writes the span in shader-clock cycles (first start to last end over the waves
// that ran) to *cycles.  0 on success.
int mfma_probe_coexec(int kind, int mode, int im, int iv, double *cycles) {
    if (kind < 0 || kind > 2 || mode < 1 || mode > 3 || im < 1 || iv < 1 || im > (1 << 20) || iv > (1 << 20) ||
        !cycles)
        return 1;
    float *out = nullptr;
    uint64_t *t = nullptr, h[16];
    int rc = 0;
    if (hipMalloc(&out, 512 * sizeof(float)) != hipSuccess || hipMalloc(&t, 16 * sizeof(uint64_t)) != hipSuccess) {
        rc = 2;
    } else {
        for (int rep = 0; rep < 2 && rc == 0; ++rep) {  // the second run is the one measured
            if (kind == 0) hipLaunchKernelGGL(k_coexec<0>, dim3(1), dim3(512), 0, 0, mode, im, iv, 1.0f, out, t);
            if (kind == 1) hipLaunchKernelGGL(k_coexec<1>, dim3(1), dim3(512), 0, 0, mode, im, iv, 1.0f, out, t);
            if (kind == 2) hipLaunchKernelGGL(k_coexec<2>, dim3(1), dim3(512), 0, 0, mode, im, iv, 1.0f, out, t);
            if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) rc = 4;
        }
        if (rc == 0 && hipMemcpy(h, t, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) rc = 5;
        if (rc == 0) {
            uint64_t lo = ~0ull, hi = 0;
            for (int w = 0; w < 8; ++w) {
                if ((w < 4 && !(mode & 1)) || (w >= 4 && !(mode & 2))) continue;
                lo = h[2 * w] < lo ? h[2 * w] : lo;
                hi = h[2 * w + 1] > hi ? h[2 * w + 1] : hi;
            }
            *cycles = (double)(hi - lo);
        }
    }
    (void)hipFree(out);
    (void)hipFree(t);
    return rc;
}

}  // extern "C"
