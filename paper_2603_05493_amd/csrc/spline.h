// Uniform cubic B-spline sampling shared by the B-spline kernels and the
// fused iteration's spline-sampling form (cuRoboV2 Sec. 4, Eq. 10): the
// four-knot window of a segment with the ghost knots of the initial state
// blended in, its monomial coefficients C w, the position, velocity and
// acceleration at alpha in [0, 1) of a knot interval of length dt, and the
// transpose: a sample's gradient back onto its window.
// Everything is written once here so that every caller rounds alike.
#pragma once

#include "wb_internal.h"

namespace wb {

// Knots of segment seg of one trajectory and joint, ghost knots blended in.
// Every load is issued unconditionally (indices clamped, a missing initial
// derivative read from theta0 with weight 0), so no load waits behind a
// branch.
__device__ __forceinline__ void segment_window(const float *__restrict__ Uj, int K, int seg, float th, float v,
                                               float a, bool printed, float w[4]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) w[m] = Uj[min(max(seg + m - 3, 0), K - 1)];
    // ghost knots from the initial state: the paper's printed formulas, or
    // the exact anchoring theta(0) = theta_0, theta_dot(0) = theta_dot_0,
    // theta_ddot(0) = theta_ddot_0
    const float g0 = printed ? th - a * (1.f / 6.f) : th - v + a * (1.f / 3.f);
    const float g1 = printed ? th + v + a * (1.f / 3.f) : th - a * (1.f / 6.f);
    const float g2 = printed ? th + 2.f * v + a * (11.f / 6.f) : th + v + a * (1.f / 3.f);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int e = seg + m;
        const float f0 = e == 0 ? 1.f : 0.f, f1 = e == 1 ? 1.f : 0.f, f2 = e == 2 ? 1.f : 0.f;
        w[m] = w[m] * (1.f - f0 - f1 - f2) + f0 * g0 + f1 * g1 + f2 * g2;
    }
}

// Window gradient of one sample at alpha: B(alpha)^T [gp, gv, ga] added to
// (r0, r1, r2, r3), with gv, ga already divided by dt, dt^2.
__device__ __forceinline__ void window_grad(float alpha, float gp, float gv, float ga, float &r0, float &r1,
                                            float &r2, float &r3) {
    // gradient on the monomial coefficients (alpha^3, alpha^2, alpha, 1)
    const float a2 = alpha * alpha;
    const float d3 = gp * a2 * alpha + gv * 3.f * a2 + ga * 6.f * alpha;
    const float d2 = gp * a2 + gv * 2.f * alpha + ga * 2.f;
    const float d1 = gp * alpha + gv;
    const float d0 = gp;
    // C^T: onto the window
    r0 += (-d3 + 3.f * d2 - 3.f * d1 + d0) * (1.f / 6.f);
    r1 += (3.f * d3 - 6.f * d2 + 4.f * d0) * (1.f / 6.f);
    r2 += (-3.f * d3 + 3.f * d2 + 3.f * d1 + d0) * (1.f / 6.f);
    r3 += d3 * (1.f / 6.f);
}

// Monomial coefficients (alpha^3, alpha^2, alpha, 1) of a window: C w.
__device__ __forceinline__ void window_coefficients(const float w[4], float c[4]) {
    c[0] = (-w[0] + 3.f * w[1] - 3.f * w[2] + w[3]) * (1.f / 6.f);
    c[1] = (3.f * w[0] - 6.f * w[1] + 3.f * w[2]) * (1.f / 6.f);
    c[2] = (-3.f * w[0] + 3.f * w[2]) * (1.f / 6.f);
    c[3] = (w[0] + 4.f * w[1] + w[2]) * (1.f / 6.f);
}

// Position, velocity and acceleration at alpha (inv = 1 / dt).
__device__ __forceinline__ void sample_at(const float c[4], float al, float inv, float &p, float &pd, float &pdd) {
    p = ((c[0] * al + c[1]) * al + c[2]) * al + c[3];
    pd = ((3.f * c[0] * al + 2.f * c[1]) * al + c[2]) * inv;
    pdd = (6.f * c[0] * al + 2.f * c[1]) * (inv * inv);
}

}  // namespace wb
