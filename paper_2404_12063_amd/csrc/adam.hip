// Adam (Kingma and Ba, Algorithm 1), the optimiser the paper trains with
// (Sec. 4.6.3): bias-corrected first and second moment estimates, in place.
#include <cmath>

#include "internal.h"

namespace vp {

__global__ void k_adam(int64_t n, float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

vpinn_status adam_step(int64_t n, float *p, const float *g, float *m, float *v, int64_t step, float lr, float b1,
                       float b2, float eps, hipStream_t s) {
    if (n == 0) return VPINN_OK;
    // bias corrections in double on the host: 1 - beta^t
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    k_adam<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(n, p, g, m, v, lr, b1, b2, eps, c1, c2);
    VP_HIP(hipGetLastError());
    return VPINN_OK;
}

}  // namespace vp
