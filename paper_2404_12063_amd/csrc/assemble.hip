// One-time assembly of the premultiplied tensors G_x, G_y, the forcing matrix F
// and the physical quadrature points (Sec. 4.2 and 4.4, Appendix A.1 and A.2),
// computed in FP64 on the device and stored in FP32.
//
// For element e with counter-clockwise vertices (x_c, y_c), c = 0..3, the
// bilinear map of Appendix A.1 is x = xc0 + xc1 xi + xc2 eta + xc3 xi eta (same
// for y).  With a = dx/dxi, b = dy/dxi, c = dx/deta, d = dy/deta and
// D = ad - bc, the physical gradient of a reference function is
//   (v_x, v_y) = (d v_xi - b v_eta, -c v_xi + a v_eta) / D,
// so the premultiplied entries w_q D (v_x, v_y) need no division:
//   G_x = w_q (d v_xi - b v_eta),   G_y = w_q (-c v_xi + a v_eta).
#include <cmath>
#include <vector>

#include "device_common.h"
#include "internal.h"

namespace vp {

// --------------------------------------------------------------------------
// Gauss-Lobatto-Legendre nodes and weights on [-1, 1] (n points).  Fixed-point
// iteration of the Legendre-Vandermonde form: with N = n - 1,
//   x <- x - (x P_N(x) - P_{N-1}(x)) / ((N + 1) P_N(x)),
// started from the Chebyshev-Gauss-Lobatto points; its fixed points are +-1 and
// the roots of P'_N.  Weights 2 / (N (N + 1) P_N(x)^2).
// --------------------------------------------------------------------------
static void gll_rule(int n, std::vector<double> &x, std::vector<double> &w) {
    const int N = n - 1;
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) x[i] = -std::cos(M_PI * i / N);
    for (int it = 0; it < 200; ++it) {
        double change = 0.0;
        for (int i = 0; i < n; ++i) {
            double p0 = 1.0, p1 = x[i];
            for (int k = 2; k <= N; ++k) {
                double p2 = ((2 * k - 1) * x[i] * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_N, p0 = P_{N-1}; Newton on x P_N - P_{N-1}, whose derivative is (N + 1) P_N
            double nx = x[i] - (x[i] * p1 - p0) / ((N + 1) * p1);
            change = std::fmax(change, std::fabs(nx - x[i]));
            x[i] = nx;
        }
        if (change < 1e-16) break;
    }
    for (int i = 0; i < n; ++i) {
        double p0 = 1.0, p1 = x[i];
        for (int k = 2; k <= N; ++k) {
            double p2 = ((2 * k - 1) * x[i] * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        w[i] = 2.0 / (N * (N + 1.0) * p1 * p1);
    }
}

// 1D test functions phi_r = P_{r+1} - P_{r-1} and their derivatives
// phi_r' = (2r + 1) P_r at the n nodes; tables [r-1][i], r = 1..nt.
__global__ void k_basis_tables(const double *__restrict__ xg, int n, int nt, double *__restrict__ phi,
                               double *__restrict__ dphi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = xg[i];
    double pm1 = 1.0, p = t;  // P_0, P_1
    // walk the Bonnet recurrence, emitting phi_r once P_{r+1} is known
    for (int r = 1; r <= nt; ++r) {
        const double pp = ((2.0 * r + 1.0) * t * p - r * pm1) / (r + 1.0);  // P_{r+1}
        phi[(r - 1) * n + i] = pp - pm1;
        dphi[(r - 1) * n + i] = (2.0 * r + 1.0) * p;
        pm1 = p;
        p = pp;
    }
}

struct Geo {
    double xc[4], yc[4];
};

__device__ inline Geo load_geo(const double *__restrict__ nodes, const int32_t *__restrict__ quad, int64_t e) {
    double vx[4], vy[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int32_t id = quad[e * 4 + c];
        vx[c] = nodes[2 * (int64_t)id];
        vy[c] = nodes[2 * (int64_t)id + 1];
    }
    Geo g;
    g.xc[0] = 0.25 * (vx[0] + vx[1] + vx[2] + vx[3]);
    g.xc[1] = 0.25 * (-vx[0] + vx[1] + vx[2] - vx[3]);
    g.xc[2] = 0.25 * (-vx[0] - vx[1] + vx[2] + vx[3]);
    g.xc[3] = 0.25 * (vx[0] - vx[1] + vx[2] - vx[3]);
    g.yc[0] = 0.25 * (vy[0] + vy[1] + vy[2] + vy[3]);
    g.yc[1] = 0.25 * (-vy[0] + vy[1] + vy[2] - vy[3]);
    g.yc[2] = 0.25 * (-vy[0] - vy[1] + vy[2] + vy[3]);
    g.yc[3] = 0.25 * (vy[0] - vy[1] + vy[2] - vy[3]);
    return g;
}

// physical quadrature points, FP64 (for a host forcing callback) and FP32
__global__ void k_points(const double *__restrict__ nodes, const int32_t *__restrict__ quad, int64_t n_elem,
                         int n, const double *__restrict__ xg, double *__restrict__ xq64,
                         float2 *__restrict__ xq32) {
    const int nq = n * n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_elem * nq) return;
    const int64_t e = t / nq;
    const int q = (int)(t - e * nq);
    const Geo g = load_geo(nodes, quad, e);
    const double xi = xg[q % n], eta = xg[q / n];
    const double x = g.xc[0] + g.xc[1] * xi + g.xc[2] * eta + g.xc[3] * xi * eta;
    const double y = g.yc[0] + g.yc[1] * xi + g.yc[2] * eta + g.yc[3] * xi * eta;
    if (xq64) {
        xq64[2 * t] = x;
        xq64[2 * t + 1] = y;
    }
    xq32[t] = make_float2((float)x, (float)y);
}

// G_x, G_y, F for one element per block.  Threads stride over quadrature points;
// F[e,k] is reduced over q in fixed order through shared memory.  With a
// convection-diffusion operator -diff Lap u + (cx, cy) . grad u the convection
// term's weights w_q det J v_k are folded in: G_x = w_q det J (diff v_x + cx v),
// G_y = w_q det J (diff v_y + cy v) (Poisson: diff = 1, cx = cy = 0).  With M
// non-null (space-dependent diffusion, nothing folded) the convection weights
// w_q det J v_k are stored there instead.
constexpr int kAsmThreads = 256;
__global__ __launch_bounds__(kAsmThreads) void k_assemble(
    const double *__restrict__ nodes, const int32_t *__restrict__ quad, int n, int nt,
    const double *__restrict__ xg, const double *__restrict__ wg, const double *__restrict__ phi,
    const double *__restrict__ dphi, int f_kind, double f_amp, double f_kx, double f_ky,
    const double *__restrict__ f_vals, double diff, double cx, double cy, int shared_g, float *__restrict__ Gx,
    float *__restrict__ Gy, float *__restrict__ F, float *__restrict__ M) {
    __shared__ double wdf[kAsmThreads];
    const int64_t e = blockIdx.x;
    const int nq = n * n, ntest = nt * nt;
    const Geo g = load_geo(nodes, quad, e);
    constexpr int kMaxK = (VPINN_MAX_TEST_ORDER * VPINN_MAX_TEST_ORDER + kAsmThreads - 1) / kAsmThreads;
    double Fk[kMaxK];  // thread t accumulates F[e, t + m * kAsmThreads]
#pragma unroll
    for (int m = 0; m < kMaxK; ++m) Fk[m] = 0.0;
    for (int q0 = 0; q0 < nq; q0 += kAsmThreads) {
        const int q = q0 + threadIdx.x;
        if (q < nq) {
            const int i = q % n, j = q / n;
            const double xi = xg[i], eta = xg[j];
            const double w = wg[i] * wg[j];
            const double a = g.xc[1] + g.xc[3] * eta, b = g.yc[1] + g.yc[3] * eta;
            const double c = g.xc[2] + g.xc[3] * xi, d = g.yc[2] + g.yc[3] * xi;
            const double D = a * d - b * c;
            double f;
            if (f_kind == VPINN_FORCING_SINSIN) {
                const double x = g.xc[0] + g.xc[1] * xi + g.xc[2] * eta + g.xc[3] * xi * eta;
                const double y = g.yc[0] + g.yc[1] * xi + g.yc[2] * eta + g.yc[3] * xi * eta;
                f = f_amp * sin(f_kx * x) * sin(f_ky * y);
            } else {
                f = f_vals[e * nq + q];
            }
            wdf[threadIdx.x] = w * D * f;
            // a shared premultiplier is written once, from element 0; none for matrix-free problems
            for (int s = 0; s < ((Gx == nullptr || (shared_g && e > 0)) ? 0 : nt); ++s) {
                const double ps = phi[s * n + j], dps = dphi[s * n + j];
                for (int r = 0; r < nt; ++r) {
                    const double pr = phi[r * n + i], dpr = dphi[r * n + i];
                    const double vxi = dpr * ps, veta = pr * dps, dv = D * pr * ps;
                    const int64_t o = ((shared_g ? 0 : e * ntest) + s * nt + r) * (int64_t)nq + q;
                    // det J * physical gradient = (d v_xi - b v_eta, -c v_xi + a v_eta)
                    Gx[o] = (float)(w * (diff * (d * vxi - b * veta) + cx * dv));
                    Gy[o] = (float)(w * (diff * (-c * vxi + a * veta) + cy * dv));
                    if (M) M[o] = (float)(w * dv);
                }
            }
        }
        __syncthreads();
        const int lim = min(kAsmThreads, nq - q0);
#pragma unroll
        for (int m = 0; m < kMaxK; ++m) {
            const int k = threadIdx.x + m * kAsmThreads;
            if (k < ntest) {
                const int rk = k % nt, sk = k / nt;
                for (int t = 0; t < lim; ++t) {
                    const int q = q0 + t;
                    Fk[m] += wdf[t] * phi[rk * n + q % n] * phi[sk * n + q / n];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < kMaxK; ++m) {
        const int k = threadIdx.x + m * kAsmThreads;
        if (k < ntest) F[e * ntest + k] = (float)Fk[m];
    }
}

// The same for problems with fewer elements than CUs: one block per element and
// test-function index s along eta (grid: elements x N_t), so a few large elements
// still spread over the chip (each block re-evaluates the forcing at its points).
// Threads stride over quadrature points; F[e, s N_t + r] is reduced over q in fixed
// order through shared memory, thread r per entry.  With a
// convection-diffusion operator -diff Lap u + (cx, cy) . grad u the convection
// term's weights w_q det J v_k are folded in: G_x = w_q det J (diff v_x + cx v),
// G_y = w_q det J (diff v_y + cy v) (Poisson: diff = 1, cx = cy = 0).  With M
// non-null (space-dependent diffusion, nothing folded) the convection weights
// w_q det J v_k are stored there instead.
__global__ __launch_bounds__(kAsmThreads) void k_assemble_split(
    const double *__restrict__ nodes, const int32_t *__restrict__ quad, int n, int nt,
    const double *__restrict__ xg, const double *__restrict__ wg, const double *__restrict__ phi,
    const double *__restrict__ dphi, int f_kind, double f_amp, double f_kx, double f_ky,
    const double *__restrict__ f_vals, double diff, double cx, double cy, int shared_g, float *__restrict__ Gx,
    float *__restrict__ Gy, float *__restrict__ F, float *__restrict__ M) {
    __shared__ double wdf[kAsmThreads];
    const int64_t e = blockIdx.x;
    const int s = blockIdx.y;  // test function phi_s along eta
    const int nq = n * n, ntest = nt * nt;
    const Geo g = load_geo(nodes, quad, e);
    double Fr = 0.0;  // thread r < nt accumulates F[e, s nt + r]
    for (int q0 = 0; q0 < nq; q0 += kAsmThreads) {
        const int q = q0 + threadIdx.x;
        if (q < nq) {
            const int i = q % n, j = q / n;
            const double xi = xg[i], eta = xg[j];
            const double w = wg[i] * wg[j];
            const double a = g.xc[1] + g.xc[3] * eta, b = g.yc[1] + g.yc[3] * eta;
            const double c = g.xc[2] + g.xc[3] * xi, d = g.yc[2] + g.yc[3] * xi;
            const double D = a * d - b * c;
            double f;
            if (f_kind == VPINN_FORCING_SINSIN) {
                const double x = g.xc[0] + g.xc[1] * xi + g.xc[2] * eta + g.xc[3] * xi * eta;
                const double y = g.yc[0] + g.yc[1] * xi + g.yc[2] * eta + g.yc[3] * xi * eta;
                f = f_amp * sin(f_kx * x) * sin(f_ky * y);
            } else {
                f = f_vals[e * nq + q];
            }
            wdf[threadIdx.x] = w * D * f;
            // a shared premultiplier is written once, from element 0; none for matrix-free problems
            if (Gx != nullptr && !(shared_g && e > 0)) {
                const double ps = phi[s * n + j], dps = dphi[s * n + j];
                for (int r = 0; r < nt; ++r) {
                    const double pr = phi[r * n + i], dpr = dphi[r * n + i];
                    const double vxi = dpr * ps, veta = pr * dps, dv = D * pr * ps;
                    const int64_t o = ((shared_g ? 0 : e * ntest) + s * nt + r) * (int64_t)nq + q;
                    // det J * physical gradient = (d v_xi - b v_eta, -c v_xi + a v_eta)
                    Gx[o] = (float)(w * (diff * (d * vxi - b * veta) + cx * dv));
                    Gy[o] = (float)(w * (diff * (-c * vxi + a * veta) + cy * dv));
                    if (M) M[o] = (float)(w * dv);
                }
            }
        }
        __syncthreads();
        const int lim = min(kAsmThreads, nq - q0);
        if (threadIdx.x < nt) {
            const int r = threadIdx.x;
            for (int t = 0; t < lim; ++t) {
                const int q = q0 + t;
                Fr += wdf[t] * phi[r * n + q % n] * phi[s * n + q / n];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < nt) F[e * ntest + s * nt + threadIdx.x] = (float)Fr;
}

// matrix-free problems: the bilinear map's coefficients of each element (xc1, xc2, xc3,
// yc1, yc2, yc3, xc0, yc0; the Jacobian needs only the first six) ...
__global__ void k_geometry(const double *__restrict__ nodes, const int32_t *__restrict__ quad, int64_t n_elem,
                           float *__restrict__ geo) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elem) return;
    const Geo g = load_geo(nodes, quad, e);
    float *o = geo + e * 8;
    o[0] = (float)g.xc[1];
    o[1] = (float)g.xc[2];
    o[2] = (float)g.xc[3];
    o[3] = (float)g.yc[1];
    o[4] = (float)g.yc[2];
    o[5] = (float)g.yc[3];
    o[6] = (float)g.xc[0];
    o[7] = (float)g.yc[0];
}

// ... and the 1D tables in FP32: nodes [n], weights [n], phi [nt][n], phi' [nt][n]
__global__ void k_tables_f32(const double *__restrict__ xg, const double *__restrict__ wg,
                             const double *__restrict__ phi, const double *__restrict__ dphi, int n, int nt,
                             float *__restrict__ tab) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nn = n * nt;
    if (t >= 2 * n + 2 * nn) return;
    double v;
    if (t < n) v = xg[t];
    else if (t < 2 * n) v = wg[t - n];
    else if (t < 2 * n + nn) v = phi[t - 2 * n];
    else v = dphi[t - 2 * n - nn];
    tab[t] = (float)v;
}

vpinn_status assemble_device(vpinn_problem *p, const double *d_nodes, int64_t n_nodes, const int32_t *d_quad,
                             const vpinn_forcing *f, hipStream_t s) {
    (void)n_nodes;
    const int n = p->n, nt = p->nt, nq = p->nq;
    std::vector<double> xg, wg;
    gll_rule(n, xg, wg);
    DevBuf d_xg, d_wg, d_phi, d_dphi, d_x64, d_f;
    VP_HIP(d_xg.reserve(sizeof(double) * n));
    VP_HIP(d_wg.reserve(sizeof(double) * n));
    VP_HIP(d_phi.reserve(sizeof(double) * n * nt));
    VP_HIP(d_dphi.reserve(sizeof(double) * n * nt));
    VP_HIP(hipMemcpyAsync(d_xg.ptr, xg.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    VP_HIP(hipMemcpyAsync(d_wg.ptr, wg.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    k_basis_tables<<<1, 128, 0, s>>>(d_xg.as<double>(), n, nt, d_phi.as<double>(), d_dphi.as<double>());
    VP_HIP(hipGetLastError());

    const int64_t npts = p->n_pts;
    const bool callback = f->kind == VPINN_FORCING_CALLBACK;
    if (callback) VP_HIP(d_x64.reserve(sizeof(double) * 2 * npts));
    {
        const int64_t blocks = (npts + 255) / 256;
        k_points<<<dim3((unsigned)blocks), 256, 0, s>>>(d_nodes, d_quad, p->n_elem, n, d_xg.as<double>(),
                                                        callback ? d_x64.as<double>() : nullptr,
                                                        p->pts.as<float2>());
        VP_HIP(hipGetLastError());
    }
    if (callback) {
        std::vector<double> hx(2 * npts), hf(npts);
        VP_HIP(hipMemcpyAsync(hx.data(), d_x64.ptr, sizeof(double) * 2 * npts, hipMemcpyDeviceToHost, s));
        VP_HIP(hipStreamSynchronize(s));
        for (int64_t t = 0; t < npts; ++t) {
            hf[t] = f->fn(hx[2 * t], hx[2 * t + 1], f->user);
            if (!std::isfinite(hf[t]))
                return fail(VPINN_E_NONFINITE, "forcing is not finite at quadrature point " + std::to_string(t % nq) +
                                                   " of element " + std::to_string(t / nq));
        }
        VP_HIP(d_f.reserve(sizeof(double) * npts));
        VP_HIP(hipMemcpyAsync(d_f.ptr, hf.data(), sizeof(double) * npts, hipMemcpyHostToDevice, s));
        VP_HIP(hipStreamSynchronize(s));
    }
    int cus = 0;
    VP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device));
    // one block per element when there are enough elements to fill the CUs, else one per
    // element and test-function row (a few large elements)
    if (p->n_elem >= cus) {
        k_assemble<<<dim3((unsigned)p->n_elem), kAsmThreads, 0, s>>>(
            d_nodes, d_quad, n, nt, d_xg.as<double>(), d_wg.as<double>(), d_phi.as<double>(), d_dphi.as<double>(),
            f->kind, f->amp, f->kx, f->ky, callback ? d_f.as<double>() : nullptr, p->diff, p->conv_x, p->conv_y,
            p->shared_g ? 1 : 0, p->matfree ? nullptr : p->Gx.as<float>(), p->matfree ? nullptr : p->Gy.as<float>(),
            p->F.as<float>(), (p->vardiff && !p->matfree) ? p->M.as<float>() : nullptr);
    } else {
        k_assemble_split<<<dim3((unsigned)p->n_elem, (unsigned)nt), kAsmThreads, 0, s>>>(
            d_nodes, d_quad, n, nt, d_xg.as<double>(), d_wg.as<double>(), d_phi.as<double>(), d_dphi.as<double>(),
            f->kind, f->amp, f->kx, f->ky, callback ? d_f.as<double>() : nullptr, p->diff, p->conv_x, p->conv_y,
            p->shared_g ? 1 : 0, p->matfree ? nullptr : p->Gx.as<float>(), p->matfree ? nullptr : p->Gy.as<float>(),
            p->F.as<float>(), (p->vardiff && !p->matfree) ? p->M.as<float>() : nullptr);
    }
    VP_HIP(hipGetLastError());
    if (p->matfree) {
        k_geometry<<<dim3((unsigned)((p->n_elem + 255) / 256)), 256, 0, s>>>(d_nodes, d_quad, p->n_elem,
                                                                          p->geo.as<float>());
        VP_HIP(hipGetLastError());
        const int ntab = 2 * n + 2 * n * nt;
        k_tables_f32<<<dim3((unsigned)((ntab + 255) / 256)), 256, 0, s>>>(
            d_xg.as<double>(), d_wg.as<double>(), d_phi.as<double>(), d_dphi.as<double>(), n, nt, p->tab.as<float>());
        VP_HIP(hipGetLastError());
    }
    VP_HIP(hipStreamSynchronize(s));
    return VPINN_OK;
}

}  // namespace vp
