// Internal declarations shared by the host API and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/vpinn.h"

namespace vp {

// ---------------------------------------------------------------------------
// padded parameter layout used inside every kernel: width padded to 32, so
// weight rows are 32 floats and padded neurons carry zero weights and biases
// (their activation is tanh(0) = 0 and they feed nothing).
//   W1 [32][2] at 0, b1 [32] at 64,
//   layer l = 2..L: W_l [32][32] at 96 + (l-2)*1056, b_l [32] right after,
//   W_out [32] at 96 + (L-1)*1056, b_out after it;
//   a second output head (the space-dependent diffusion coefficient):
//   W_out2 [32] right after b_out, then b_out2.
// ---------------------------------------------------------------------------
constexpr int PW = 32;
constexpr int kOffB1 = 64;
constexpr int kLayerStride = PW * PW + PW;  // 1056
__host__ __device__ constexpr int off_w(int l) { return l == 1 ? 0 : 96 + (l - 2) * kLayerStride; }
__host__ __device__ constexpr int off_b(int l) { return l == 1 ? kOffB1 : off_w(l) + PW * PW; }
__host__ __device__ constexpr int off_wout(int L) { return 96 + (L - 1) * kLayerStride; }
__host__ __device__ constexpr int n_padded(int L) { return off_wout(L) + PW + 1; }
__host__ __device__ constexpr int off_wout2(int L) { return n_padded(L); }
__host__ __device__ constexpr int n_padded2(int L) { return n_padded(L) + PW + 1; }
constexpr int kMaxPadded = n_padded2(VPINN_MAX_HIDDEN);

// flat (unpadded) layout offsets for width H
__host__ __device__ inline int64_t hoff_w(int H, int l) {
    return l == 1 ? 0 : (int64_t)3 * H + (int64_t)(l - 2) * (H * H + H);
}

// status helpers ------------------------------------------------------------
void set_error(const std::string &msg);
vpinn_status fail(vpinn_status code, const std::string &msg);
#define VP_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::vp::fail(VPINN_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// an allocation: running out of device memory is VPINN_E_NOMEM, any other failure VPINN_E_DEVICE
#define VP_ALLOC(call)                                                                \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::vp::fail(e_ == hipErrorOutOfMemory ? VPINN_E_NOMEM : VPINN_E_DEVICE, \
                              std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

// device buffer that frees itself --------------------------------------------
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes) {
        o.ptr = nullptr;
        o.bytes = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            ptr = o.ptr;
            bytes = o.bytes;
            o.ptr = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    // grow to at least `b` bytes (contents are not preserved)
    hipError_t reserve(size_t b) {
        if (b <= bytes) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&ptr, b);
        if (e == hipSuccess) bytes = b;
        else ptr = nullptr;
        return e;
    }
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

}  // namespace vp

struct vpinn_problem {
    int device = 0;
    int64_t n_elem = 0;
    int n = 0, nt = 0, nq = 0, ntest = 0;
    int64_t n_pts = 0;       // interior points n_elem * nq
    int64_t n_bnd = 0, n_sen = 0;
    // convection-diffusion coefficients folded into G at assembly (1, 0, 0: Poisson)
    double diff = 1.0, conv_x = 0.0, conv_y = 0.0;
    bool folded() const { return diff != 1.0 || conv_x != 0.0 || conv_y != 0.0; }
    // every element a translate of one shape: G is the same for all of them and is
    // stored once (Algorithm 2's single reference premultiplier), element stride 0
    bool shared_g = false;
    // space-dependent diffusion (the network's second output): G holds the plain
    // diffusion weights, M the convection weights w_q det J v_k, b the velocity
    bool vardiff = false;
    double vd_bx = 0.0, vd_by = 0.0;
    vp::DevBuf M;            // float [n_elem][ntest][nq] (vardiff only)
    // matrix-free: no G or M; the bilinear map's coefficients and the 1D tables
    bool matfree = false;
    vp::DevBuf geo;          // float [n_elem][8]: xc1, xc2, xc3, yc1, yc2, yc3, xc0, yc0
    vp::DevBuf tab;          // float [2 n + 2 nt n]: GLL nodes, weights, phi_r(x_i), phi_r'(x_i)
    int64_t gstride() const { return shared_g ? 0 : (int64_t)ntest * nq; }
    // shared quadrature points (vpinn_set_shared_points): the fused path evaluates the
    // network once per distinct interior point; slot (e, q) reads point umap[e nq + q],
    // and the slots of point u are uslot[usoff[u] .. usoff[u + 1]) in increasing order
    int64_t n_uniq = 0;      // 0: every slot is its own point
    vp::DevBuf umap;         // int32 [n_pts]
    vp::DevBuf usoff;        // int32 [n_uniq + 1]
    vp::DevBuf uslot;        // int32 [n_pts]
    vp::DevBuf upts;         // float2 [n_uniq]
    // bumped whenever the point sets or their sharing change: a cached single-problem
    // plan rebuilds, and a batch built before the change refuses to run
    int64_t gen = 0;
    vp::DevBuf Gx, Gy, F;    // float
    vp::DevBuf pts;          // float2 [n_pts + n_bnd + n_sen]: interior, boundary, sensors
    vp::DevBuf tgt;          // float [n_bnd + n_sen]: g_b then d_s
    // workspace (grown on demand)
    vp::DevBuf wpad;         // float [kMaxPadded]: padded parameters
    vp::DevBuf u, ux, uy;    // float [all points]
    vp::DevBuf act;          // float [(32 + 96 (L-1))][all points]: stored activations (plain path)
    vp::DevBuf uxb, uyb;     // float [n_pts]: adjoint of the contraction
    vp::DevBuf A, R;         // float [n_elem * ntest]
    vp::DevBuf loss_e;       // double [n_elem]: per-element sum_k R^2 (or per-block partials)
    vp::DevBuf gpart;        // float [blocks][kMaxPadded]: per-block gradient partials
    vp::DevBuf eps_part;     // double [blocks]
    hipEvent_t prof[VPINN_PROFILE_EVENTS] = {};  // optional timing events (caller-owned)
    void *fused_ws = nullptr;              // fused-path workspace (owned)
    void (*fused_ws_free)(void *) = nullptr;
    int64_t all_pts() const { return n_pts + n_bnd + n_sen; }
    ~vpinn_problem() {
        if (fused_ws && fused_ws_free) fused_ws_free(fused_ws);
    }
};

namespace vp {

// kernel launchers (defined in the .hip files) --------------------------------
// builds G (with p->diff, p->conv_x, p->conv_y folded in), F and the points
vpinn_status assemble_device(vpinn_problem *p, const double *d_nodes, int64_t n_nodes, const int32_t *d_quad,
                             const vpinn_forcing *f, hipStream_t s);
// output `head` (0-based) of a network with `heads` outputs, padded, as a one-output network
vpinn_status pack_params(const float *d_params, int H, int L, int heads, int head, float *d_wpad, hipStream_t s);
// the network with `nh` outputs (flat parameters, width H) at n points: u and, if
// either is non-null, its tangents; e the second output (nh = 2); null outputs are skipped
vpinn_status eval_mfma(int L, int H, int nh, const float *d_params, int64_t n, const float2 *d_xy, float *d_u,
                       float *d_ux, float *d_uy, float *d_e, hipStream_t s);
// mean |p - ref|, max |p - ref|, ||p - ref|| / ||ref|| -> d_out[3]; d_part [512][4] workspace
vpinn_status error_stats(int64_t n, const float *d_p, const float *d_ref, double *d_part, double *d_out,
                         hipStream_t s);
// the fixed workspace of the allocation-free error call on the current device: room for
// VPINN_NOALLOC_MAX_POINTS values and error_stats' partials (looked up, never allocated)
vpinn_status noalloc_workspace(float **values, double **partials);
vpinn_status plain_loss_grad(vpinn_problem *p, const vpinn_loss_cfg *cfg, const float *d_params,
                             const float *d_eps, float *d_loss, float *d_grad, float *d_grad_eps,
                             float *d_R_out, hipStream_t s);
vpinn_status fused_loss_grad(vpinn_problem *p, const vpinn_loss_cfg *cfg, const float *d_params,
                             const float *d_eps, float *d_loss, float *d_grad, float *d_grad_eps,
                             hipStream_t s);
vpinn_status adam_step(int64_t n, float *p, const float *g, float *m, float *v, int64_t step, float lr,
                       float b1, float b2, float eps, hipStream_t s);
vpinn_status batch_create(int32_t n, vpinn_problem *const *problems, const vpinn_loss_cfg *cfg, vpinn_batch **out);
vpinn_status batch_loss_and_grad(vpinn_batch *b, const float *d_params, const float *d_eps, float *d_losses,
                                 float *d_grads, float *d_grad_eps, hipStream_t s);
vpinn_status batch_step(vpinn_batch *b, float *d_params, float *d_m, float *d_v, int64_t *d_step, float lr, float b1,
                        float b2, float eps, float *d_losses, float *d_eps, float *d_eps_m, float *d_eps_v,
                        hipStream_t s);
vpinn_status batch_capture(vpinn_batch *b, float *d_params, float *d_m, float *d_v, int64_t *d_step, float lr,
                           float b1, float b2, float eps, float *d_losses, float *d_eps, float *d_eps_m,
                           float *d_eps_v, hipStream_t s);
vpinn_status batch_replay(vpinn_batch *b, hipStream_t s);
void batch_set_profile_events(vpinn_batch *b, void *const *events);
vpinn_status batch_get_tuning(const vpinn_batch *b, vpinn_tuning *out);
vpinn_status batch_set_tuning(vpinn_batch *b, const vpinn_tuning *t);
vpinn_status batch_autotune(vpinn_batch *b, const float *d_params, int32_t reps, vpinn_tuning *best, hipStream_t s);
int batch_device(const vpinn_batch *b);
void batch_destroy(vpinn_batch *b);

}  // namespace vp
