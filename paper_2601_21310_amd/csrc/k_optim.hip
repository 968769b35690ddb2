// AdamW parameter update for the inner loop (Sec. 3.3: AdamW with weight decay and a
// cosine learning-rate decay), with the step counter and the learning rate kept on the
// device so that a whole optimisation step can be captured in a HIP graph and replayed.
//
//   t   = step[0] + 1 (a single-thread kernel after the update stores t back)
//   lr  = lr_min + (lr_max - lr_min) (1 + cos(pi min(t, T) / T)) / 2
//   m   <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2
//   theta <- theta - lr ( m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd theta )
#include "dnqs_device.h"
#include "dnqs_kernels.h"

namespace dnqs {

__global__ void k_adamw(float *__restrict__ theta, const float *__restrict__ grad, float *__restrict__ m,
                        float *__restrict__ v, int64_t n, AdamCfg c, const int *__restrict__ step) {
    const int t = step[0] + 1;
    const double tc = (double)(t < c.decay_steps ? t : c.decay_steps);
    const float lr = (float)(c.lr_min + 0.5 * (c.lr_max - c.lr_min) * (1.0 + cos(3.14159265358979323846 * tc /
                                                                                  (double)c.decay_steps)));
    const float bc1 = 1.0f - powf(c.beta1, (float)t), bc2 = 1.0f - powf(c.beta2, (float)t);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float g = grad[i];
        const float mi = c.beta1 * m[i] + (1.0f - c.beta1) * g;
        const float vi = c.beta2 * v[i] + (1.0f - c.beta2) * g * g;
        m[i] = mi;
        v[i] = vi;
        const float upd = (mi / bc1) / (sqrtf(vi / bc2) + c.eps) + c.weight_decay * theta[i];
        theta[i] -= lr * upd;
    }
}

__global__ void k_step_incr(int *step) { step[0] += 1; }

void launch_adamw(hipStream_t st, float *theta, const float *grad, float *m, float *v, int64_t n, const AdamCfg &c,
                  int *step) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_adamw, dim3((unsigned)blocks), dim3(256), 0, st, theta, grad, m, v, n, c, step);
    hipLaunchKernelGGL(k_step_incr, dim3(1), dim3(1), 0, st, step);
}

}  // namespace dnqs
