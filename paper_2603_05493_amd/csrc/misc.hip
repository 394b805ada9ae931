// Small per-state kernels of the optimizer iteration: the hinge adjoint of
// self-collision, the cost head and the gradient step.  All are one state
// per lane over [k][B] arrays (coalesced in B); nb is the number of states
// and B the row length of the arrays (the ABI's ld >= nb).
#include <algorithm>
#include "spatial.h"

namespace wb {

// Hinge h = max(0, max_pen + margin) at the most penetrating pair: its
// subgradient moves the two spheres of that pair apart along their centre
// line (cuRoboV2 Sec. 6.2 reduces to one most-penetrating pair per state).
// One thread per (sphere coordinate row, state), the state fastest, so the
// whole [3S][B] output -- zero but for the pair's six entries -- is written
// in coalesced rows; the argmax and the penetration of a state are read by
// every row from the cache.
__global__ void __launch_bounds__(256) k_sc_backward(DevRobot rb, int64_t nb, int64_t B, const float *__restrict__ sph,
                                                     const int32_t *__restrict__ argmax,
                                                     const float *__restrict__ max_pen, float margin,
                                                     const float *__restrict__ g_cost,
                                                     float *__restrict__ g_sph) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int p = argmax[b];
    const bool on = p >= 0 && p < rb.n_pairs && max_pen[b] + margin > 0.0f;
    const int s = on ? rb.pair_s[p] : -1, t = on ? rb.pair_t[p] : -1;
    for (int row = blockIdx.y; row < 3 * rb.S; row += gridDim.y) {   // sphere * 3 + coordinate
        const int sphere = row / 3, c = row - 3 * sphere;
        float out = 0.0f;
        if (sphere == s || sphere == t) {
            const float *cs = sph + (int64_t)s * 3 * B + b;
            const float *ct = sph + (int64_t)t * 3 * B + b;
            const V3 d = v3(cs[0] - ct[0], cs[B] - ct[B], cs[2 * B] - ct[2 * B]);
            const float n = sqrtf(dot(d, d));
            if (n > 0.0f) {
                const float g = g_cost[b] / n;
                const float dc = c == 0 ? d.x : (c == 1 ? d.y : d.z);
                out = sphere == s ? -g * dc : g * dc;
            }
        }
        g_sph[(int64_t)row * B + b] = out;
    }
}

__global__ void __launch_bounds__(256) k_cost_head(int64_t nb, int64_t B, int n, const float *__restrict__ tau,
                                                   const float *__restrict__ w, float tw,
                                                   const float *__restrict__ max_pen, float margin,
                                                   float hw, float *__restrict__ cost,
                                                   float *__restrict__ g_tau, float *__restrict__ g_mp) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    float c = 0.0f;
    for (int j = 0; j < n; ++j) {
        const int64_t o = (int64_t)j * B + b;
        const float t = tau[o];
        if (w) {
            c = __builtin_fmaf(w[o], t, c);
            if (g_tau) g_tau[o] = w[o];
        } else {
            c = __builtin_fmaf(tw * t, t, c);
            if (g_tau) g_tau[o] = 2.0f * tw * t;
        }
    }
    if (max_pen) {
        const float h = max_pen[b] + margin;
        c += hw * fmaxf(h, 0.0f);
        if (g_mp) g_mp[b] = h > 0.0f ? hw : 0.0f;
    }
    if (cost) cost[b] = c;
}

// One thread per (joint, state): i = j * nb + b, at element j * B + b.
__global__ void __launch_bounds__(256) k_sgd_step(int64_t nb, int64_t B, int64_t total, float lr,
                                                  float *__restrict__ q, float *__restrict__ qd,
                                                  float *__restrict__ qdd, const float *__restrict__ g_q,
                                                  const float *__restrict__ g_q2, const float *__restrict__ g_qd,
                                                  const float *__restrict__ g_qdd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int64_t j = t / nb, i = j * B + (t - j * nb);
    const float gq = g_q[i] + (g_q2 ? g_q2[i] : 0.0f);
    q[i] -= lr * gq;
    qd[i] -= lr * g_qd[i];
    qdd[i] -= lr * g_qdd[i];
}

hipError_t launch_self_collision_backward(const DevRobot &rb, int64_t B, int64_t ld, const float *spheres,
                                          const int32_t *argmax, const float *max_pen,
                                          float margin, const float *g_cost, float *g_sph,
                                          hipStream_t s) {
    if (B == 0 || rb.S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sc_backward, dim3((unsigned)((B + 255) / 256), (unsigned)std::min(3 * rb.S, 65535)),
                       dim3(256), 0, s, rb,
                       B, ld, spheres, argmax, max_pen, margin, g_cost, g_sph);
    return hipGetLastError();
}

hipError_t launch_cost_head(int64_t B, int64_t ld, int32_t n, const float *tau, const float *w, float tw,
                            const float *max_pen, float margin, float hw, float *cost,
                            float *g_tau, float *g_maxpen, hipStream_t s) {
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cost_head, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, B, ld, n, tau, w, tw,
                       max_pen, margin, hw, cost, g_tau, g_maxpen);
    return hipGetLastError();
}

hipError_t launch_sgd_step(int64_t B, int64_t ld, int32_t n, float lr, float *q, float *qd, float *qdd,
                           const float *g_q, const float *g_q2, const float *g_qd,
                           const float *g_qdd, hipStream_t s) {
    const int64_t total = B * (int64_t)n;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sgd_step, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, B, ld, total, lr, q,
                       qd, qdd, g_q, g_q2, g_qd, g_qdd);
    return hipGetLastError();
}

}  // namespace wb
