// B-spline trajectory front end (cuRoboV2 Sec. 4): uniform cubic B-spline
// evaluation of joint states from control points (Eq. 10) and its transpose,
// the control-point gradient summed over every sample of a control point's
// support (Eqs. 13-14), with ghost knots for the initial state and a
// repeated final knot for a static goal.
//
// Knots of one trajectory and joint (extended index e):
//   e = 0..2        ghost knots from (theta_0, theta_dot_0, theta_ddot_0)
//   e = 3..K+2      control points u_0 .. u_{K-1}
//   e = K+3..K+5    copies of u_{K-1}
// Segment s (0 <= s < K+3) uses the window e = s..s+3 and is sampled at
// alpha = i / n_interp; sample t = s * n_interp + i, H = (K+3) n_interp per
// trajectory, state b = traj * H + t.
//
// Control points are stored [d][T][K] (a trajectory's knots contiguous).
// Evaluation: one lane per (joint, state), so the three state arrays are
// written coalesced; the lanes of one trajectory read its few knots from the
// same cache lines.
// Gradient: one lane per (joint, trajectory, control point), the control
// point fastest, sums the samples of the (at most seven) segments containing
// its knot, reading the trajectory's samples through the cache, and writes
// its gradient (contiguous across the wavefront), optionally taking the
// gradient step.  Both kernels are bound by HBM.
#include "spline.h"

namespace wb {


__global__ void __launch_bounds__(256) k_bspline_eval(int64_t T, int32_t K, int32_t n_interp, float dt,
                                                      int32_t printed, const float *__restrict__ U,
                                                      const float *__restrict__ th0,
                                                      const float *__restrict__ dth0,
                                                      const float *__restrict__ ddth0, float *__restrict__ q,
                                                      float *__restrict__ qd, float *__restrict__ qdd) {
    // 32-bit index arithmetic: the host keeps T * H below 2^31
    const int H = (K + 3) * n_interp, NB = (int)T * H;
    const int b = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (b >= NB) return;
    const int traj = b / H;
    const int t = b - traj * H;
    const int seg = t / n_interp, i = t - seg * n_interp;
    const float alpha = (float)i / (float)n_interp;
    const int64_t o0 = (int64_t)j * T + traj;
    const float *pv = dth0 ? dth0 : th0, *pa = ddth0 ? ddth0 : th0;
    const float th = th0[o0];
    const float v = pv[o0] * (dth0 ? dt : 0.f);
    const float a = pa[o0] * (ddth0 ? dt * dt : 0.f);
    float w[4], c[4];
    segment_window(U + ((int64_t)j * T + traj) * K, K, seg, th, v, a, printed != 0, w);
    window_coefficients(w, c);
    float p, pd, pdd;
    sample_at(c, alpha, 1.f / dt, p, pd, pdd);
    const int64_t o = (int64_t)j * NB + b;
    q[o] = p;
    if (qd) qd[o] = pd;
    if (qdd) qdd[o] = pdd;
}

// One lane per (joint, trajectory, control point), the control point
// fastest: lane (j, traj, k) sums the window products of the segments that
// contain its knot (extended index k + 3; for the final control point also
// its three copies), reading the trajectory's samples from cache.  Every
// sum runs in segment order, so the result is deterministic.
__global__ void __launch_bounds__(256) k_bspline_backward(int64_t T, int32_t K, int32_t n_interp, float dt,
                                                          const float *__restrict__ g_q,
                                                          const float *__restrict__ g_qd,
                                                          const float *__restrict__ g_qdd,
                                                          float *__restrict__ g_U, float lr,
                                                          float *__restrict__ U) {
    // 32-bit index arithmetic: the host keeps T * H below 2^31
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (idx >= (int)T * K) return;
    const int traj = idx / K;
    const int k = idx - traj * K;
    const int64_t H = (int64_t)(K + 3) * n_interp, NB = T * H;
    const int64_t base = (int64_t)j * NB + traj * H;
    const float inv = 1.f / dt, inv2 = inv * inv, rn = 1.f / (float)n_interp;
    // segments touching the knot (and its copies): s from k to k + 3, or to K + 2
    const int s_end = (k == K - 1) ? K + 2 : k + 3;
    float g = 0.f;
    for (int seg = k; seg <= s_end; ++seg) {
        // window positions of this control point in segment seg: e - seg for
        // e = k + 3 and, for the final control point, its copies K+3..K+5
        float w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f;   // 1 where the window slot holds the knot
        const int m = k + 3 - seg;
        if (m == 0) w0 = 1.f; else if (m == 1) w1 = 1.f; else if (m == 2) w2 = 1.f; else if (m == 3) w3 = 1.f;
        if (k == K - 1) {
            for (int e = K + 3; e <= K + 5; ++e) {
                const int mm = e - seg;
                if (mm == 0) w0 = 1.f; else if (mm == 1) w1 = 1.f; else if (mm == 2) w2 = 1.f; else if (mm == 3) w3 = 1.f;
            }
        }
        float r0 = 0.f, r1 = 0.f, r2 = 0.f, r3 = 0.f;
        for (int i = 0; i < n_interp; ++i) {
            const int64_t o = base + (int64_t)seg * n_interp + i;
            const float gp = g_q ? g_q[o] : 0.f;
            const float gv = g_qd ? g_qd[o] * inv : 0.f;
            const float ga = g_qdd ? g_qdd[o] * inv2 : 0.f;
            window_grad((float)i * rn, gp, gv, ga, r0, r1, r2, r3);
        }
        // the window slots holding the knot
        g += w0 * r0 + w1 * r1 + w2 * r2 + w3 * r3;
    }
    const int64_t o = ((int64_t)j * T + traj) * K + k;
    if (g_U) g_U[o] = g;
    if (lr != 0.f) U[o] -= lr * g;
}

// Four samples per knot interval (alpha = 0, 1/4, 1/2, 3/4), the paper's
// n_interp: one lane per (joint, trajectory, segment).  The evaluation forms
// the segment's window and coefficients once and stores its four samples of
// each output as one 16-byte vector.
__global__ void __launch_bounds__(256) k_bspline_eval4(int32_t T, int32_t K, float dt, int32_t printed,
                                                       const float *__restrict__ U, const float *__restrict__ th0,
                                                       const float *__restrict__ dth0,
                                                       const float *__restrict__ ddth0, float *__restrict__ q,
                                                       float *__restrict__ qd, float *__restrict__ qdd) {
    const int S = K + 3, NS = T * S;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (idx >= NS) return;
    const int traj = idx / S, seg = idx - traj * S;
    const int64_t o0 = (int64_t)j * T + traj;
    const float *pv = dth0 ? dth0 : th0, *pa = ddth0 ? ddth0 : th0;
    const float th = th0[o0];
    const float v = pv[o0] * (dth0 ? dt : 0.f);
    const float a = pa[o0] * (ddth0 ? dt * dt : 0.f);
    float w[4], c[4];
    segment_window(U + o0 * K, K, seg, th, v, a, printed != 0, w);
    window_coefficients(w, c);
    const float inv = 1.f / dt;
    float p[4], pd[4], pdd[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) sample_at(c, 0.25f * i, inv, p[i], pd[i], pdd[i]);
    const int64_t o = (int64_t)j * NS * 4 + (int64_t)idx * 4;   // = j * T * H + traj * H + seg * 4
    *reinterpret_cast<float4 *>(q + o) = make_float4(p[0], p[1], p[2], p[3]);
    if (qd) *reinterpret_cast<float4 *>(qd + o) = make_float4(pd[0], pd[1], pd[2], pd[3]);
    if (qdd) *reinterpret_cast<float4 *>(qdd + o) = make_float4(pdd[0], pdd[1], pdd[2], pdd[3]);
}

// Gradient for four samples per interval: lane (trajectory, segment) of a
// workgroup holding whole trajectories forms its segment's window gradient
// from three 16-byte loads, the workgroup stages them in LDS, and lane
// (trajectory, s) for s >= 3 sums knot s over the (at most four) segments
// that contain it -- the final control point also over its three copies --
// in a fixed order.
//
// With the row-normalized step (ROW_RMS) the K lanes of each (joint,
// trajectory) row also sum their squared gradients through LDS, every lane
// in the same order, and step by lr * g / rms(row).
template <bool ROW_RMS>
__global__ void __launch_bounds__(256) k_bspline_backward4(int32_t T, int32_t K, float dt,
                                                           const float *__restrict__ g_q,
                                                           const float *__restrict__ g_qd,
                                                           const float *__restrict__ g_qdd,
                                                           float *__restrict__ g_U, float lr,
                                                           float *__restrict__ U) {
    __shared__ float4 gw[256];
    __shared__ float g2[256];
    const int S = K + 3, tpb = 256 / S;
    const int lt = threadIdx.x / S, seg = threadIdx.x - lt * S;
    const int traj = blockIdx.x * tpb + lt;
    const int j = blockIdx.y;
    const bool act = lt < tpb && traj < T;
    float r0 = 0.f, r1 = 0.f, r2 = 0.f, r3 = 0.f;
    if (act) {
        const int64_t o = (int64_t)j * T * S * 4 + ((int64_t)traj * S + seg) * 4;
        const float inv = 1.f / dt, inv2 = inv * inv;
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 p = g_q ? *reinterpret_cast<const float4 *>(g_q + o) : z;
        const float4 v = g_qd ? *reinterpret_cast<const float4 *>(g_qd + o) : z;
        const float4 a = g_qdd ? *reinterpret_cast<const float4 *>(g_qdd + o) : z;
        window_grad(0.00f, p.x, v.x * inv, a.x * inv2, r0, r1, r2, r3);
        window_grad(0.25f, p.y, v.y * inv, a.y * inv2, r0, r1, r2, r3);
        window_grad(0.50f, p.z, v.z * inv, a.z * inv2, r0, r1, r2, r3);
        window_grad(0.75f, p.w, v.w * inv, a.w * inv2, r0, r1, r2, r3);
    }
    gw[threadIdx.x] = make_float4(r0, r1, r2, r3);
    __syncthreads();
    const bool knot = act && seg >= 3;   // ghost knots take no gradient
    float g = 0.f;
    if (knot) {
        const float4 *row = gw + lt * S;
        // knot e = seg is slot m of segment seg - m
        g = row[seg].x + row[seg - 1].y + row[seg - 2].z + row[seg - 3].w;
        if (seg == S - 1) {
            // copies e = S .. S+2 of the final control point: slot e - s of segment s
            g += row[S - 1].y + row[S - 2].z + row[S - 3].w;   // e = S
            g += row[S - 1].z + row[S - 2].w;                  // e = S + 1
            g += row[S - 1].w;                                 // e = S + 2
        }
    }
    float step = lr;
    if (ROW_RMS) {
        g2[threadIdx.x] = g * g;
        __syncthreads();
        if (knot) {
            float ss = 0.f;
            for (int k = 0; k < K; ++k) ss += g2[lt * S + 3 + k];
            step = ss > 0.f ? lr * rsqrtf(ss / (float)K) : 0.f;
        }
    }
    if (!knot) return;
    const int64_t o = ((int64_t)j * T + traj) * K + (seg - 3);
    if (g_U) g_U[o] = g;
    if (lr != 0.f) U[o] -= step * g;
}

// The row-normalized step on a computed gradient: one lane per (joint,
// trajectory) row of K control points, U -= lr * g / rms(g) over the row
// (no step for an all-zero row).
__global__ void __launch_bounds__(256) k_bspline_row_step(int64_t rows, int32_t K, const float *__restrict__ g_U,
                                                          float lr, float *__restrict__ U) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    const float *g = g_U + r * K;
    float ss = 0.f;
    for (int k = 0; k < K; ++k) ss += g[k] * g[k];
    if (!(ss > 0.f)) return;
    const float step = lr * rsqrtf(ss / (float)K);
    float *u = U + r * K;
    for (int k = 0; k < K; ++k) u[k] -= step * g[k];
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

hipError_t launch_bspline_eval(int64_t T, int32_t d, int32_t K, int32_t n_interp, float dt, int32_t printed,
                               const float *U, const float *th0, const float *dth0, const float *ddth0, float *q,
                               float *qd, float *qdd, hipStream_t s) {
    const int64_t NB = T * (int64_t)(K + 3) * n_interp;
    if (NB == 0 || d == 0) return hipSuccess;
    if (n_interp == 4 && aligned16(q) && aligned16(qd) && aligned16(qdd)) {
        const int64_t NS = T * (int64_t)(K + 3);
        dim3 grid((unsigned)((NS + 255) / 256), (unsigned)d);
        hipLaunchKernelGGL(k_bspline_eval4, grid, dim3(256), 0, s, (int32_t)T, K, dt, printed, U, th0, dth0, ddth0, q,
                           qd, qdd);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((NB + 255) / 256), (unsigned)d);
    hipLaunchKernelGGL(k_bspline_eval, grid, dim3(256), 0, s, T, K, n_interp, dt, printed, U, th0, dth0, ddth0, q,
                       qd, qdd);
    return hipGetLastError();
}

hipError_t launch_bspline_backward(int64_t T, int32_t d, int32_t K, int32_t n_interp, float dt, const float *g_q,
                                   const float *g_qd, const float *g_qdd, float *g_U, float lr, int32_t rule,
                                   float *U, hipStream_t s) {
    if (T == 0 || d == 0) return hipSuccess;
    const bool rms = rule == WB_STEP_ROW_RMS && lr != 0.f;
    if (n_interp == 4 && K + 3 <= 256 && aligned16(g_q) && aligned16(g_qd) && aligned16(g_qdd)) {
        const int tpb = 256 / (K + 3);
        dim3 grid((unsigned)((T + tpb - 1) / tpb), (unsigned)d);
        if (rms)
            hipLaunchKernelGGL(k_bspline_backward4<true>, grid, dim3(256), 0, s, (int32_t)T, K, dt, g_q, g_qd, g_qdd,
                               g_U, lr, U);
        else
            hipLaunchKernelGGL(k_bspline_backward4<false>, grid, dim3(256), 0, s, (int32_t)T, K, dt, g_q, g_qd, g_qdd,
                               g_U, lr, U);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((T * K + 255) / 256), (unsigned)d);
    // the row-normalized step needs the whole row's gradient first: g_U, then a row pass
    hipLaunchKernelGGL(k_bspline_backward, grid, dim3(256), 0, s, T, K, n_interp, dt, g_q, g_qd, g_qdd, g_U,
                       rms ? 0.f : lr, U);
    if (rms) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t rows = (int64_t)d * T;
        hipLaunchKernelGGL(k_bspline_row_step, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, rows, K, g_U, lr,
                           U);
    }
    return hipGetLastError();
}

}  // namespace wb
