// Storage-free per-operation kernels with one state per group of G lanes,
// lane i holding link perm[i] in depth-first pre-order as in the fused
// iteration: RNEA and its vector-Jacobian product without a cache (cuRoboV2
// Alg. 4 and the role of Alg. 5, with transforms and every forward quantity
// recomputed in the backward), and the adjoint of forward kinematics
// (Alg. 1) from sphere and pose gradients.
//
// The recursions are carried in world coordinates (Plucker vectors about
// the world origin), where they become tree sums:
//   v_k = sum over the root path of S qd,  a_k = -g + sum of (S qdd + v x S qd),
//   f_k = I_k a_k + v_k x* I_k v_k - X*_k f_ext_k,
//   F_k = sum over the subtree of f,  tau = S . F.
// Path sums use pointer jumping over the parent lanes, subtree sums the
// difference of two values of a group scan; link poses, velocities,
// accelerations and forces never leave registers, so the forward needs no
// traversal storage and the backward needs no cache.  The VJP is the exact
// reverse mode of those sums (the transpose of a path sum is a subtree sum
// and vice versa):
//   fb = pathsum(taub S);  ab = I fb;  vb = -fb x* I v - I (v x fb)
//   A = subsum(ab);  vb += (S qd) x* A;  V = subsum(vb)
//   qdd-bar = S.A,  qd-bar = S.V - S.(v x* A)
//   W = taub S x* F - fb x* I a - a x* I fb + (v x fb) x* I v + v x* I (v x fb)
//       + qdd S x* A - qd S x* (v x* A) + qd S x* V + fb x* f_w
//   q-bar = S . subsum(W),  f_ext-bar = -X*^T fb
// (rotating joint i moves every world axis, inertia and external force of
// its subtree).  Mimic joints: link l turns by m_l q_j + o_l; lane j of the
// group gathers joint j's torque (and adjoints) from the links it drives,
// and returns m_l tau-bar_j to each of them.
#include "tree.h"

namespace wb {

// nb: states; B: row length of every [k][B] array (the ABI's ld >= nb);
// G: lanes per state, a compile-time constant (one kernel per lane count).
template <bool BACKWARD, int G>
__global__ void __launch_bounds__(256) k_rnea_lanes(DevRobot rb, DevFused fz, int64_t nb, int64_t B,
                                                    const float *__restrict__ q, const float *__restrict__ qd,
                                                    const float *__restrict__ qdd, const float *__restrict__ f_ext,
                                                    float *__restrict__ tau, const float *__restrict__ g_tau,
                                                    float *__restrict__ g_q, float *__restrict__ g_qd,
                                                    float *__restrict__ g_qdd, float *__restrict__ g_fext) {
    const int lane = threadIdx.x & 63;
    const int per_wave = 64 / G, grp = lane / G, gl = lane - grp * G;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t s = wave * per_wave + grp;
    if (wave * per_wave >= nb) return;   // the whole wavefront is past the batch
    const bool valid = s < nb;
    const int64_t b = valid ? s : nb - 1;   // groups past the end compute on a valid state, store nothing
    const int *li = fz.li;
    const float *lf = fz.lf;
    const bool act = gl < rb.L;
    const int parent_lane = li[1 * 64 + gl];
    const bool revolute = li[5 * 64 + gl] != 0;
    const int jidx = li[3 * 64 + gl];
    const int link = li[0 * 64 + gl];
    const int sub_end = li[2 * 64 + gl];
    const bool mim = fz.mimic != 0;
    float th = 0.f, thd = 0.f, thdd = 0.f, mult = 1.f;
    if (revolute) {
        const int64_t o = (int64_t)jidx * B + b;
        th = q[o];
        thd = qd[o];
        thdd = qdd[o];
        if (mim) {
            mult = lf[29 * 64 + gl];
            th = mult * th + lf[30 * 64 + gl];
            thd *= mult;
            thdd *= mult;
        }
    }
    M3 R;
    V3 p;
    lane_world_pose(fz, gl, revolute, th, parent_lane, G, R, p);
    SV S = zsv();
    if (revolute) {
        const V3 sw = mul(R, v3(lf[0 * 64 + gl], lf[1 * 64 + gl], lf[2 * 64 + gl]));
        S = sv(sw, cross(p, sw));
    }
    WInertia J;
    J.m = lf[15 * 64 + gl];
    J.cw = mul(R, v3(lf[16 * 64 + gl], lf[17 * 64 + gl], lf[18 * 64 + gl])) + p;
    {
        float Ic[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) Ic[t] = lf[(19 + t) * 64 + gl];
        rotate_inertia(R, Ic, J.I);
    }
    // external force in world coordinates, f_w = X* f_ext (moment about the world origin)
    SV fe = zsv();
    if (f_ext && act) {
        const float *fx = f_ext + (int64_t)(link * 6) * B + b;
        const V3 Rf = mul(R, v3(fx[3 * B], fx[4 * B], fx[5 * B]));
        fe = sv(mul(R, v3(fx[0], fx[B], fx[2 * B])) + cross(p, Rf), Rf);
    }
    const SV Sqd = thd * S;
    const SV v = path_sum(Sqd, parent_lane, gl, fz.jsteps, G);
    SV a = path_sum(thdd * S + crm(v, Sqd), parent_lane, gl, fz.jsteps, G);
    if (act) a += sv(v3(0.f, 0.f, 0.f), v3(-rb.gx, -rb.gy, -rb.gz));
    const SV Ia = iw_apply(J, a), Iv = iw_apply(J, v);
    SV F = Ia + crf(v, Iv) - fe;
    if (!act) F = zsv();
    F = subtree_sum(F, gl, sub_end, G);
    const bool jlane = mim ? gl < rb.n : revolute;
    const int64_t jrow = (int64_t)(mim ? gl : jidx) * B + b;
    if (!BACKWARD) {
        float t = revolute ? dot(S, F) : 0.f;
        if (mim) t = gather_joint(mult * t, fz, gl, G);
        if (valid && jlane) tau[jrow] = t;
        return;
    }
    // tau-bar of the lane's link: m_l tau-bar_j with mimic joints
    float taub = jlane ? g_tau[jrow] : 0.f;
    if (mim) {
        const float tj = __shfl(taub, revolute ? jidx : gl, G);
        taub = revolute ? mult * tj : 0.f;
    }
    SV W = taub * crf(S, F);
    const SV fb = path_sum(taub * S, parent_lane, gl, fz.jsteps, G);
    SV ab = iw_apply(J, fb);
    W = W - (crf(fb, Ia) + crf(a, ab)) + crf(fb, fe);
    const SV vxfb = crm(v, fb);
    const SV Ivxfb = iw_apply(J, vxfb);
    SV vb = zsv() - (crf(fb, Iv) + Ivxfb);
    W += crf(vxfb, Iv) + crf(v, Ivxfb);
    if (!act) ab = zsv();
    const SV Acc = subtree_sum(ab, gl, sub_end, G);
    vb += crf(Sqd, Acc);
    if (!act) vb = zsv();
    const SV vxA = crf(v, Acc);
    float thdd_b = dot(S, Acc);
    W += thdd * crf(S, Acc) - thd * crf(S, vxA);
    const SV V = subtree_sum(vb, gl, sub_end, G);
    float thd_b = dot(S, V) - dot(S, vxA);
    W += thd * crf(S, V);
    if (!act) W = zsv();
    const SV Ws = subtree_sum(W, gl, sub_end, G);
    float th_b = dot(S, Ws);
    if (mim) {
        th_b = gather_joint(mult * th_b, fz, gl, G);
        thd_b = gather_joint(mult * thd_b, fz, gl, G);
        thdd_b = gather_joint(mult * thdd_b, fz, gl, G);
    }
    if (!valid) return;
    if (g_fext && act) {
        // -X*^T fb: moment part -R^T fb_w, force part -R^T (fb_l + fb_w x p)
        const V3 gn = mulT(R, fb.w), gf = mulT(R, fb.l + cross(fb.w, p));
        float *gx = g_fext + (int64_t)(link * 6) * B + b;
        gx[0] = -gn.x; gx[B] = -gn.y; gx[2 * B] = -gn.z;
        gx[3 * B] = -gf.x; gx[4 * B] = -gf.y; gx[5 * B] = -gf.z;
    }
    if (jlane) {
        g_q[jrow] = th_b;
        g_qd[jrow] = thd_b;
        g_qdd[jrow] = thdd_b;
    }
}

// Adjoint of forward kinematics (Alg. 1) from gradients on sphere centres
// g_sph[S][3][B] and/or link poses g_pose[L][12][B], one state per group of
// lanes: the lane of link l forms the wrench its gradients exert about the
// world origin, W_l = sum over its spheres of [c x g; g] plus, for a pose
// gradient (G on R, g_p on p), [sum_c r_c x G_c + p x g_p; g_p]; the
// subtree sum of W, projected on the joint's world axis S = [s; p x s],
// is the joint's gradient (a rotation about s moves every point and frame
// of the subtree).  Transforms are recomputed by pointer jumping; nothing is
// stored.  Mimic joints gather m_l times their links' values.
template <int G>
__global__ void __launch_bounds__(256) k_fk_backward_lanes(DevRobot rb, DevFused fz, int64_t nb, int64_t B,
                                                           const float *__restrict__ q,
                                                           const float *__restrict__ g_pose,
                                                           const float *__restrict__ g_sph,
                                                           float *__restrict__ g_q) {
    const int lane = threadIdx.x & 63;
    const int per_wave = 64 / G, grp = lane / G, gl = lane - grp * G;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t s = wave * per_wave + grp;
    if (wave * per_wave >= nb) return;
    const bool valid = s < nb;
    const int64_t b = valid ? s : nb - 1;
    const int *li = fz.li;
    const float *lf = fz.lf;
    const bool act = gl < rb.L;
    const int parent_lane = li[1 * 64 + gl];
    const bool revolute = li[5 * 64 + gl] != 0;
    const int jidx = li[3 * 64 + gl];
    const int link = li[0 * 64 + gl];
    const int sub_end = li[2 * 64 + gl];
    const bool mim = fz.mimic != 0;
    float th = 0.f, mult = 1.f;
    if (revolute) {
        th = q[(int64_t)jidx * B + b];
        if (mim) {
            mult = lf[29 * 64 + gl];
            th = mult * th + lf[30 * 64 + gl];
        }
    }
    M3 R;
    V3 p;
    lane_world_pose(fz, gl, revolute, th, parent_lane, G, R, p);
    SV W = zsv();
    if (act) {
        if (g_sph) {
            const int first = rb.li[link].sph_first, cnt = rb.li[link].sph_count;
            for (int j = 0; j < cnt; ++j) {
                const float4 c4 = rb.sph[first + j];
                const V3 c = mul(R, v3(c4.x, c4.y, c4.z)) + p;
                const float *gp = g_sph + (int64_t)(first + j) * 3 * B + b;
                const V3 g = v3(gp[0], gp[B], gp[2 * B]);
                W += sv(cross(c, g), g);
            }
        }
        if (g_pose) {
            const float *gp = g_pose + (int64_t)link * 12 * B + b;
            M3 Gm;
#pragma unroll
            for (int t = 0; t < 9; ++t) Gm.m[t] = gp[t * B];
            const V3 gt = v3(gp[9 * B], gp[10 * B], gp[11 * B]);
            V3 m = cross(p, gt);
#pragma unroll
            for (int c = 0; c < 3; ++c) m += cross(col(R, c), col(Gm, c));
            W += sv(m, gt);
        }
    }
    const SV Ws = subtree_sum(W, gl, sub_end, G);
    float th_b = 0.f;
    if (revolute) {
        const V3 sw = mul(R, v3(lf[0 * 64 + gl], lf[1 * 64 + gl], lf[2 * 64 + gl]));
        th_b = dot(sv(sw, cross(p, sw)), Ws);
    }
    if (mim) th_b = gather_joint(mult * th_b, fz, gl, G);
    const bool jlane = mim ? gl < rb.n : revolute;
    if (valid && jlane) g_q[(int64_t)(mim ? gl : jidx) * B + b] = th_b;
}

static int lanes_for(int L) { return L <= 16 ? 16 : (L <= 32 ? 32 : 64); }

hipError_t launch_fk_backward_lanes(const DevRobot &rb, const DevFused &fz, int64_t B, int64_t ld, const float *q,
                                    const float *g_pose, const float *g_sph, float *g_q, hipStream_t s) {
    if (B == 0) return hipSuccess;
    const int G = lanes_for(rb.L);
    const int64_t per_wg = 4 * (64 / G);
    const dim3 grid((unsigned)((B + per_wg - 1) / per_wg));
    switch (G) {
        case 16: hipLaunchKernelGGL(k_fk_backward_lanes<16>, grid, dim3(256), 0, s, rb, fz, B, ld, q, g_pose, g_sph, g_q); break;
        case 32: hipLaunchKernelGGL(k_fk_backward_lanes<32>, grid, dim3(256), 0, s, rb, fz, B, ld, q, g_pose, g_sph, g_q); break;
        default: hipLaunchKernelGGL(k_fk_backward_lanes<64>, grid, dim3(256), 0, s, rb, fz, B, ld, q, g_pose, g_sph, g_q); break;
    }
    return hipGetLastError();
}

hipError_t launch_rnea_lanes(const DevRobot &rb, const DevFused &fz, int64_t B, int64_t ld, const float *q,
                             const float *qd, const float *qdd, const float *f_ext, float *tau, hipStream_t s) {
    if (B == 0) return hipSuccess;
    const int G = lanes_for(rb.L);
    const int64_t per_wg = 4 * (64 / G);
    const dim3 grid((unsigned)((B + per_wg - 1) / per_wg));
    const float *no = nullptr;
    float *nw = nullptr;
    switch (G) {
        case 16: hipLaunchKernelGGL((k_rnea_lanes<false, 16>), grid, dim3(256), 0, s, rb, fz, B, ld, q, qd, qdd, f_ext, tau, no, nw, nw, nw, nw); break;
        case 32: hipLaunchKernelGGL((k_rnea_lanes<false, 32>), grid, dim3(256), 0, s, rb, fz, B, ld, q, qd, qdd, f_ext, tau, no, nw, nw, nw, nw); break;
        default: hipLaunchKernelGGL((k_rnea_lanes<false, 64>), grid, dim3(256), 0, s, rb, fz, B, ld, q, qd, qdd, f_ext, tau, no, nw, nw, nw, nw); break;
    }
    return hipGetLastError();
}

hipError_t launch_rnea_backward_lanes(const DevRobot &rb, const DevFused &fz, int64_t B, int64_t ld,
                                      const float *q, const float *qd, const float *qdd, const float *f_ext,
                                      const float *g_tau, float *g_q, float *g_qd, float *g_qdd, float *g_fext,
                                      hipStream_t s) {
    if (B == 0) return hipSuccess;
    const int G = lanes_for(rb.L);
    const int64_t per_wg = 4 * (64 / G);
    const dim3 grid((unsigned)((B + per_wg - 1) / per_wg));
    float *nw = nullptr;
    switch (G) {
        case 16: hipLaunchKernelGGL((k_rnea_lanes<true, 16>), grid, dim3(256), 0, s, rb, fz, B, ld, q, qd, qdd, f_ext, nw, g_tau, g_q, g_qd, g_qdd, g_fext); break;
        case 32: hipLaunchKernelGGL((k_rnea_lanes<true, 32>), grid, dim3(256), 0, s, rb, fz, B, ld, q, qd, qdd, f_ext, nw, g_tau, g_q, g_qd, g_qdd, g_fext); break;
        default: hipLaunchKernelGGL((k_rnea_lanes<true, 64>), grid, dim3(256), 0, s, rb, fz, B, ld, q, qd, qdd, f_ext, nw, g_tau, g_q, g_qd, g_qdd, g_fext); break;
    }
    return hipGetLastError();
}

}  // namespace wb
