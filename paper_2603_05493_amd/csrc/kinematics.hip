// Kinematics outputs for optimizers and solvers in one launch (cuRoboV2
// Sec. 6.1: a forward-kinematics call yields frame transforms, tool poses,
// sphere centres, centres of mass and Jacobians), and the gradient of
// tool-pose and centre-of-mass losses.
//
// Mapping: a group of G lanes (16, 32 or 64) owns one state; lane i holds
// link perm[i] in depth-first pre-order and lane j also owns Jacobian
// column j.  World poses follow by pointer jumping over the parent lanes
// as in the fused iteration; nothing but the requested outputs reaches
// memory.
//
// The Jacobians are stored state-major ([B][T][6][n] and [B][3][n]): one
// state's block is contiguous, as batched linear algebra on them (J^T J per
// state) wants, and a group writes each row as n consecutive floats, so
// cache lines are written whole.  The other outputs keep the [k][B] layout.
//
// Jacobian of tool t (Alg. 2).  Column lane j walks connectedLinks[j] (the
// links whose angle joint j sets, several for a mimic joint) and fetches
// each one's world axis s and origin o from that link's lane.  The coarse
// filter is affects[j, e] (a bit mask per tool, built on the host); the
// fine filter keeps a link l only when it lies on the chain of the tool's
// link e, which in depth-first lane order is lane(l) <= lane(e) <=
// sub_end(l).  Each kept link adds mult_l [s x (x - o); s] with x the tool
// point.
//
// Centre of mass: sum_l m_l c_l / M by a group reduction.  Its Jacobian:
// link lane l forms mult_l s_l x (C_l - M_l o_l) / M from its subtree's
// mass M_l and first moment C_l (subtree sums by the group's prefix scan),
// and column lane j gathers its connected links as above.
//
// Gradient: dL/dq_j = sum_t J_t[:, j] . [g_x; w_t] + J_com[:, j] . g_com,
// where w_t = sum_c r_c x G_c over the columns of the tool rotation and of
// its gradient (a rotation turns by [s]x R about a joint axis s).
#include "kin.h"
#include "lanes.h"
#include "spatial.h"

namespace wb {
namespace {

constexpr int KIN_WG = 256;

__device__ __forceinline__ V3 shfl3(V3 v, int src, int G) {
    return v3(__shfl(v.x, src, G), __shfl(v.y, src, G), __shfl(v.z, src, G));
}

__device__ __forceinline__ V3 scan3(V3 v, int G) {
    return v3(group_scan(v.x, G), group_scan(v.y, G), group_scan(v.z, G));
}

// Tool frames of one state (Alg. 2).  Poses lane-parallel: lane (t, c) of
// a pass, t = gl / 12 and c = gl % 12, forms element c of tool t's pose
// (R_e R_o row-major, then R_e p_o + p_e) with one 3-term dot product, so
// a 64-lane group covers five tools per pass.  Jacobian columns: every
// column lane fetches its first connected link's axis, origin, multiplier
// and subtree end once for all tools, then takes each tool point (and, for
// the gradient, the tool rotation) from the lanes that formed it.
// Forward: writes the poses and Jacobians.  BWD: returns this column's
// dL/dq_j = sum_t J_t[:, j] . [g_x; w_t].  GC: the lanes per state, known
// at compile time (16, 32 or 64; it equals k.G).
template <bool BWD, int GC>
__device__ __forceinline__ float tool_frames(const DevKin &k, int64_t B, int64_t b, bool valid, int gl, const M3 &R,
                                             V3 p, V3 s_w, float mult, int sub_end, const KinOut &o,
                                             const float *__restrict__ g_tool) {
    constexpr int G = GC;
    const int n = k.n;
    const bool col_lane = gl < n;
    const int lk0 = k.conn[gl];
    const int src0 = lk0 >= 0 ? lk0 : gl;
    const V3 s0 = shfl3(s_w, src0, G), o0 = shfl3(p, src0, G);
    const float m0 = __shfl(mult, src0, G);
    const int lend0 = __shfl(sub_end, src0, G);
    const int per = G / 12;   // tools per pass (G >= 16)
    const int c = gl % 12, row = c < 9 ? c / 3 : c - 9, cj = c % 3;
    float gq = 0.f;
    for (int t0 = 0; t0 < k.n_tools; t0 += per) {
        const int tt = t0 + gl / 12;
        const bool tl = gl < per * 12 && tt < k.n_tools;
        const int tq = tl ? tt : t0;
        const int e = k.tool_lane[tq];
        const float *off = k.tool_off + 12 * tq;
        const V3 re = v3(__shfl(R.m[3 * 0 + 0], e, G), __shfl(R.m[3 * 0 + 1], e, G), __shfl(R.m[3 * 0 + 2], e, G));
        const V3 r1 = v3(__shfl(R.m[3 * 1 + 0], e, G), __shfl(R.m[3 * 1 + 1], e, G), __shfl(R.m[3 * 1 + 2], e, G));
        const V3 r2 = v3(__shfl(R.m[3 * 2 + 0], e, G), __shfl(R.m[3 * 2 + 1], e, G), __shfl(R.m[3 * 2 + 2], e, G));
        const V3 pe = shfl3(p, e, G);
        const V3 rr = row == 0 ? re : (row == 1 ? r1 : r2);
        const V3 oc = c < 9 ? v3(off[cj], off[3 + cj], off[6 + cj]) : v3(off[9], off[10], off[11]);
        const float val = dot(rr, oc) + (c < 9 ? 0.f : (row == 0 ? pe.x : (row == 1 ? pe.y : pe.z)));
        if (!BWD && o.tool_pose && valid && tl) o.tool_pose[((int64_t)tt * 12 + c) * B + b] = val;
        if (!BWD && !o.jac) continue;
        const int t1 = min(t0 + per, k.n_tools);
        for (int t = t0; t < t1; ++t) {
            const int xb = (t - t0) * 12;
            const V3 x = v3(__shfl(val, xb + 9, G), __shfl(val, xb + 10, G), __shfl(val, xb + 11, G));
            const int et = k.tool_lane[t];
            const bool aff = col_lane && ((k.tool_aff[t] >> gl) & 1ull);
            V3 jl = v3(0.f, 0.f, 0.f), ja = v3(0.f, 0.f, 0.f);
            if (aff && lk0 >= 0 && lk0 <= et && et <= lend0) {
                jl = m0 * cross(s0, x - o0);
                ja = m0 * s0;
            }
            for (int kk = 1; kk < k.mc; ++kk) {   // further links of a mimic joint
                const int lk = k.conn[kk * 64 + gl];
                const int src = lk >= 0 ? lk : gl;
                const V3 sk = shfl3(s_w, src, G), ok = shfl3(p, src, G);
                const float mk = __shfl(mult, src, G);
                const int lend = __shfl(sub_end, src, G);
                if (aff && lk >= 0 && lk <= et && et <= lend) {
                    jl += mk * cross(sk, x - ok);
                    ja += mk * sk;
                }
            }
            if (!BWD) {
                if (valid && col_lane) {   // state-major: each row is n consecutive floats
                    float *d = o.jac + ((int64_t)b * k.n_tools + t) * 6 * n + gl;
                    d[0] = jl.x;
                    d[n] = jl.y;
                    d[2 * n] = jl.z;
                    d[3 * n] = ja.x;
                    d[4 * n] = ja.y;
                    d[5 * n] = ja.z;
                }
            } else {
                // a rotation turns by [s]x R about a joint axis s: w = sum_c r_c x G_c
                M3 Rt;
#pragma unroll
                for (int i = 0; i < 9; ++i) Rt.m[i] = __shfl(val, xb + i, G);
                const float *gt = g_tool + (int64_t)t * 12 * B + b;
                M3 GR;
#pragma unroll
                for (int i = 0; i < 9; ++i) GR.m[i] = gt[i * B];
                const V3 gx = v3(gt[9 * B], gt[10 * B], gt[11 * B]);
                V3 w = v3(0.f, 0.f, 0.f);
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) w += cross(col(Rt, cc), col(GR, cc));
                gq += dot(jl, gx) + dot(ja, w);
            }
        }
    }
    return gq;
}

template <bool BWD, int GC>
__device__ __forceinline__ void kin_state(const DevKin &k, int64_t B, int64_t b, bool valid, int gl,
                                          const float *__restrict__ q, const KinOut &o, const KinGrad &g) {
    constexpr int G = GC;
    const int *li = k.li;
    const float *lf = k.lf;
    const bool act = gl < k.L;
    const int parent_lane = li[1 * 64 + gl];
    const int sub_end = li[2 * 64 + gl];
    const bool rev = li[4 * 64 + gl] != 0;
    const float mult = lf[15 * 64 + gl];
    const V3 ax = v3(lf[0 * 64 + gl], lf[1 * 64 + gl], lf[2 * 64 + gl]);
    // ---- forward kinematics: local transform, then pointer jumping
    M3 R;
#pragma unroll
    for (int t = 0; t < 9; ++t) R.m[t] = lf[(3 + t) * 64 + gl];
    V3 p = v3(lf[12 * 64 + gl], lf[13 * 64 + gl], lf[14 * 64 + gl]);
    if (rev) {
        const float th = mult * q[(int64_t)li[3 * 64 + gl] * B + b] + lf[16 * 64 + gl];
        float sn, cs;
        sincosf(th, &sn, &cs);
        const M3 Jr = axis_angle(ax, sn, cs);
        R = li[5 * 64 + gl] ? Jr : matmul(R, Jr);
    }
    {
        // Lane 0 is the fixed root at the world frame (identity pose), as is
        // every lane past the robot: a finished chain keeps composing with
        // that identity, which changes nothing exactly, so no step needs a
        // guard; two steps per trip let the pose alternate between register
        // sets instead of being copied back.
        int anc = max(parent_lane, 0);
        auto jump = [&]() {
            M3 Ra;
#pragma unroll
            for (int t = 0; t < 9; ++t) Ra.m[t] = __shfl(R.m[t], anc, G);
            const V3 pa = shfl3(p, anc, G);
            anc = __shfl(anc, anc, G);
            p = mul(Ra, p) + pa;
            R = matmul(Ra, R);
        };
        int st = 0;
        for (; st + 1 < k.jsteps; st += 2) {
            jump();
            jump();
        }
        if (st < k.jsteps) jump();
    }
    if (!BWD && valid && act) {
        const int link = li[0 * 64 + gl];
        if (o.link_pose) {
            float *d = o.link_pose + (int64_t)link * 12 * B + b;
#pragma unroll
            for (int t = 0; t < 9; ++t) d[t * B] = R.m[t];
            d[9 * B] = p.x;
            d[10 * B] = p.y;
            d[11 * B] = p.z;
        }
        if (o.spheres) {
            const int first = li[6 * 64 + gl], cnt = li[7 * 64 + gl];
            for (int j = 0; j < cnt; ++j) {
                const float4 c4 = k.sph[first + j];
                const V3 c = mul(R, v3(c4.x, c4.y, c4.z)) + p;
                float *d = o.spheres + (int64_t)(first + j) * 3 * B + b;
                d[0] = c.x;
                d[B] = c.y;
                d[2 * B] = c.z;
            }
        }
    }
    const V3 s_w = mul(R, ax);   // world joint axis; the joint's world origin is p
    const int n = k.n;
    const bool col_lane = gl < n;
    float gq = 0.f;
    // ---- centre of mass and its Jacobian
    const bool want_com = BWD ? g.g_com != nullptr : (o.com != nullptr || o.com_jac != nullptr);
    if (want_com) {
        const float m = lf[17 * 64 + gl];
        const V3 mc = m * (mul(R, v3(lf[18 * 64 + gl], lf[19 * 64 + gl], lf[20 * 64 + gl])) + p);
        if (!BWD && o.com) {
            const V3 tot = v3(group_reduce_sum(mc.x, G), group_reduce_sum(mc.y, G), group_reduce_sum(mc.z, G));
            if (valid && gl < 3) o.com[(int64_t)gl * B + b] = (gl == 0 ? tot.x : gl == 1 ? tot.y : tot.z) * k.inv_mass;
        }
        if (BWD || o.com_jac) {
            const V3 sc = scan3(mc, G);
            const float sm = group_scan(m, G);
            const V3 hc = shfl3(sc, sub_end, G);
            const float hm = __shfl(sm, sub_end, G);
            const V3 lc = v3(lane_prev(sc.x), lane_prev(sc.y), lane_prev(sc.z));
            const float lm = lane_prev(sm);
            const V3 Csub = gl > 0 ? hc - lc : hc;
            const float Msub = gl > 0 ? hm - lm : hm;
            const V3 cj = rev ? (mult * k.inv_mass) * cross(s_w, Csub - Msub * p) : v3(0.f, 0.f, 0.f);
            V3 col = v3(0.f, 0.f, 0.f);
            for (int kk = 0; kk < k.mc; ++kk) {
                const int lk = k.conn[kk * 64 + gl];
                const V3 y = shfl3(cj, lk >= 0 ? lk : gl, G);
                if (lk >= 0) col += y;
            }
            if (!BWD) {
                if (valid && col_lane) {   // state-major: the state's 3 x n block is contiguous
                    float *d = o.com_jac + (int64_t)b * 3 * n + gl;
                    d[0] = col.x;
                    d[n] = col.y;
                    d[2 * n] = col.z;
                }
            } else {
                const V3 gc = v3(g.g_com[b], g.g_com[B + b], g.g_com[2 * B + b]);
                gq += dot(col, gc);
            }
        }
    }
    // ---- tool frames: poses and Jacobians, or their gradient
    if (BWD ? g.g_tool != nullptr : (o.tool_pose != nullptr || o.jac != nullptr))
        gq += tool_frames<BWD, GC>(k, B, b, valid, gl, R, p, s_w, mult, sub_end, o, g.g_tool);
    if (BWD && valid && col_lane) g.g_q[(int64_t)gl * B + b] = gq;
}

// Each workgroup takes `spb` consecutive states (a multiple of its 256 / G
// groups), so the rows of every [k][B] output are written in runs of
// consecutive states by one workgroup.
// nb: states; B: row length of the [k][B] arrays (>= nb).
template <bool BWD, int GC>
__global__ void __launch_bounds__(KIN_WG, 5) k_kinematics(DevKin k, int64_t nb_states, int64_t B,
                                                       const float *__restrict__ q, KinOut o, KinGrad g,
                                                       int32_t spb) {
    constexpr int G = GC;
    const int gl = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int gpw = KIN_WG / G;
    // Workgroups are dealt round-robin to the 8 XCDs, each with its own L2:
    // renumber them so that every XCD takes one contiguous range of runs
    // and the cache lines its runs share are fetched and written once.
    const unsigned nb = gridDim.x;
    const unsigned bid = (nb & 7u) == 0 ? (blockIdx.x & 7u) * (nb >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    const int64_t base = (int64_t)bid * spb;
    for (int it = 0; it < spb / gpw; ++it) {
        const int64_t b0 = base + (int64_t)it * gpw;
        if (b0 >= nb_states) break;   // uniform over the workgroup
        const int64_t br = b0 + grp;
        const bool valid = br < nb_states;
        kin_state<BWD, GC>(k, B, valid ? br : nb_states - 1, valid, gl, q, o, g);
    }
}

// Runs of up to 32 consecutive states (128-byte rows of the [k][B]
// outputs), shortened until the grid has 2048 workgroups: each state is a
// chain of dependent cross-lane steps, so latency hiding wants many
// resident wavefronts.
int32_t states_per_block(const DevKin &k, int64_t B) {
    const int gpw = KIN_WG / k.G;
    int32_t spb = gpw > 32 ? gpw : 32;
    while (spb > gpw && (B + spb - 1) / spb < 2048) spb /= 2;
    return spb;
}

}  // namespace

hipError_t launch_kinematics(const DevKin &k, int64_t B, int64_t ld, const float *q, const KinOut &o,
                             hipStream_t s) {
    if (B == 0) return hipSuccess;
    const int32_t spb = states_per_block(k, B);
    const dim3 grid((unsigned)((B + spb - 1) / spb));
    switch (k.G) {   // one kernel per lane count: the group width is a compile-time constant
        case 16: hipLaunchKernelGGL((k_kinematics<false, 16>), grid, dim3(KIN_WG), 0, s, k, B, ld, q, o, KinGrad{}, spb); break;
        case 32: hipLaunchKernelGGL((k_kinematics<false, 32>), grid, dim3(KIN_WG), 0, s, k, B, ld, q, o, KinGrad{}, spb); break;
        case 64: hipLaunchKernelGGL((k_kinematics<false, 64>), grid, dim3(KIN_WG), 0, s, k, B, ld, q, o, KinGrad{}, spb); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_kinematics_backward(const DevKin &k, int64_t B, const float *q, const KinGrad &g,
                                      hipStream_t s) {
    if (B == 0) return hipSuccess;
    const int32_t spb = states_per_block(k, B);
    const dim3 grid((unsigned)((B + spb - 1) / spb));
    switch (k.G) {
        case 16: hipLaunchKernelGGL((k_kinematics<true, 16>), grid, dim3(KIN_WG), 0, s, k, B, B, q, KinOut{}, g, spb); break;
        case 32: hipLaunchKernelGGL((k_kinematics<true, 32>), grid, dim3(KIN_WG), 0, s, k, B, B, q, KinOut{}, g, spb); break;
        case 64: hipLaunchKernelGGL((k_kinematics<true, 64>), grid, dim3(KIN_WG), 0, s, k, B, B, q, KinOut{}, g, spb); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wb
