// Group-of-lanes tree operations shared by the kernels that give each state
// a group of G lanes (G = 16, 32 or 64) with lane i holding link perm[i] in
// depth-first pre-order (the subtree of lane i is the lane range
// [i, sub_end_i]): path sums by pointer jumping over the parent lanes,
// subtree sums as differences of a group scan, world-frame inertia
// products, and the per-lane forward kinematics.
#pragma once

#include "lanes.h"
#include "spatial.h"

namespace wb {

// ------------------------------------------------------------ group shuffles
__device__ __forceinline__ SV shfl_sv(SV x, int src, int G) {
    return sv(v3(__shfl(x.w.x, src, G), __shfl(x.w.y, src, G), __shfl(x.w.z, src, G)),
              v3(__shfl(x.l.x, src, G), __shfl(x.l.y, src, G), __shfl(x.l.z, src, G)));
}
__device__ __forceinline__ SV zsv() { return sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f)); }

// Sum of x over the path from the root to this lane's link.  Lane 0 (the
// fixed root) and the lanes past the robot must hold zero: a chain that has
// reached the root keeps jumping to lane 0 and adds that zero, exactly, so
// no lane needs a guard (and no masked copy of x) per step.
__device__ __forceinline__ SV path_sum(SV x, int parent_lane, int glane, int steps, int G) {
    (void)glane;
    int anc = max(parent_lane, 0);
    for (int s = 0; s < steps; ++s) {
        const SV y = shfl_sv(x, anc, G);
        anc = __shfl(anc, anc, G);
        x += y;
    }
    return x;
}

// Sum of x over this lane's subtree (group lanes [glane, sub_end]): the
// difference of two values of the group's inclusive scan.  Lanes outside the
// robot must hold zero.
__device__ __forceinline__ SV subtree_sum(SV x, int glane, int sub_end, int G) {
    SV s = x;
    group_scan6(s.w.x, s.w.y, s.w.z, s.l.x, s.l.y, s.l.z, G);
    const SV hi = shfl_sv(s, sub_end, G);
    const SV lo = sv(v3(lane_prev(s.w.x), lane_prev(s.w.y), lane_prev(s.w.z)),
                     v3(lane_prev(s.l.x), lane_prev(s.l.y), lane_prev(s.l.z)));
    return glane > 0 ? hi - lo : hi;
}

// World-frame spatial inertia of a link: mass m, CoM cw and the rotational
// inertia about the CoM in world axes, Iw = R Ic R^T (xx yy zz xy xz yz).
struct WInertia {
    float m;
    V3 cw;
    float I[6];
};
__device__ __forceinline__ SV iw_apply(const WInertia &J, SV u) {
    const V3 h = J.m * (u.l + cross(u.w, J.cw));
    const V3 Iw = v3(J.I[0] * u.w.x + J.I[3] * u.w.y + J.I[4] * u.w.z,
                     J.I[3] * u.w.x + J.I[1] * u.w.y + J.I[5] * u.w.z,
                     J.I[4] * u.w.x + J.I[5] * u.w.y + J.I[2] * u.w.z);
    return sv(Iw + cross(J.cw, h), h);
}
// R Ic R^T for a symmetric Ic given as xx yy zz xy xz yz.
__device__ __forceinline__ void rotate_inertia(const M3 &R, const float *Ic, float *Iw) {
    float T[9];   // R Ic
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float r0 = R.m[3 * i], r1 = R.m[3 * i + 1], r2 = R.m[3 * i + 2];
        T[3 * i + 0] = r0 * Ic[0] + r1 * Ic[3] + r2 * Ic[4];
        T[3 * i + 1] = r0 * Ic[3] + r1 * Ic[1] + r2 * Ic[5];
        T[3 * i + 2] = r0 * Ic[4] + r1 * Ic[5] + r2 * Ic[2];
    }
    const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int e = 0; e < 6; ++e)
        Iw[e] = T[3 * ii[e]] * R.m[3 * jj[e]] + T[3 * ii[e] + 1] * R.m[3 * jj[e] + 1] +
                T[3 * ii[e] + 2] * R.m[3 * jj[e] + 2];
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Sum over the links joint `glane` drives (connectedLinks, lanes of the
// group) of their x; 0 in lanes past the last joint.
__device__ __forceinline__ float gather_joint(float x, const DevFused &fz, int glane, int G) {
    float acc = 0.f;
    for (int kk = 0; kk < fz.mc; ++kk) {
        const int l = fz.conn[kk * 64 + glane];
        const float y = __shfl(x, l >= 0 ? l : glane, G);
        if (l >= 0) acc += y;
    }
    return acc;
}

// World pose (R, p) of the lane's link: the lane's local transform (fixed
// rotation and translation, then the joint rotation by angle th), composed
// with its ancestors' by pointer jumping, T <- T_anc o T, anc <- anc(anc),
// `steps` times.  Lane 0 (the fixed root) and the lanes past the robot hold
// the identity and are their own ancestors, so a chain that has reached
// the root keeps composing with the identity, exactly.
__device__ __forceinline__ void lane_world_pose(const DevFused &fz, int gl, bool revolute, float th, int parent_lane,
                                                int G, M3 &R, V3 &p) {
    const float *lf = fz.lf;
    const int *li = fz.li;
#pragma unroll
    for (int t = 0; t < 9; ++t) R.m[t] = lf[(3 + t) * 64 + gl];
    p = v3(lf[12 * 64 + gl], lf[13 * 64 + gl], lf[14 * 64 + gl]);
    if (revolute) {
        float s, c;
        sincosf(th, &s, &c);
        const M3 Jr = axis_angle(v3(lf[0 * 64 + gl], lf[1 * 64 + gl], lf[2 * 64 + gl]), s, c);
        R = li[6 * 64 + gl] ? Jr : matmul(R, Jr);
    }
    int anc = max(parent_lane, 0);
    for (int st = 0; st < fz.jsteps; ++st) {
        M3 Ra;
#pragma unroll
        for (int t = 0; t < 9; ++t) Ra.m[t] = __shfl(R.m[t], anc, G);
        const V3 pa = v3(__shfl(p.x, anc, G), __shfl(p.y, anc, G), __shfl(p.z, anc, G));
        anc = __shfl(anc, anc, G);
        p = mul(Ra, p) + pa;
        R = matmul(Ra, R);
    }
}

}  // namespace wb
