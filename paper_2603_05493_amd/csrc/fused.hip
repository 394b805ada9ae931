// One trajectory-optimizer iteration of the whole-body hot path in a single
// kernel: forward kinematics, self-collision, RNEA, cost head, every adjoint
// and the gradient step (cuRoboV2 Sec. 3 loop steps 2, 3, 5 and 6 for the
// whole-body terms; Sec. 6.1-6.3).  Two kernels share the per-state
// pipeline: one robot (k_fused_step) and an uneven batch of robots in one
// persistent launch (k_plan_step).
//
// Mapping: a group of G lanes (G = 16, 32 or 64; 64/G states per wavefront)
// owns one state; lane i of the group holds link perm[i] in depth-first
// pre-order, so the subtree of lane i is the lane range [i, sub_end_i].
// Nothing intermediate leaves the chip: link poses and spatial quantities
// live in registers, sphere centres and link bounding spheres (transformed
// from their link-frame tables) in the group's LDS.
//
// Forward kinematics: each lane forms its local transform (fixed (R, p) then
// the joint rotation) and the world pose follows by pointer jumping over the
// parent links: T <- T_anc o T, anc <- anc(anc), ceil(log2(depth+1)) steps.
//
// Dynamics are carried in world coordinates (Plucker vectors about the world
// origin), where the RNEA recursions of Alg. 4 lose their per-link
// transforms and become tree prefix sums:
//   v_k = sum over the root path of S_j qd_j                  (path sum)
//   a_k = -g + sum over the root path of (S_j qdd_j + v_j x S_j qd_j)
//   f_k = I_k a_k + v_k x* I_k v_k                            (per link)
//   F_k = sum over the subtree of f_j,  tau_k = S_k . F_k      (subtree sum)
// with S_k the joint's world axis and I_k its world inertia.  Path sums use
// pointer jumping; subtree sums use an inclusive scan in DFS order and the
// difference of two scan values.
//
// The VJP is the exact reverse mode of those sums (the transpose of a path
// sum is a subtree sum and vice versa):
//   fb = pathsum(taub S);  ab = I fb;  vb = -fb x* I v - I (v x fb)
//   A = subsum(ab);  vb += (S qd) x* A;  V = subsum(vb)
//   qdd-bar = S.A,  qd-bar = S.V - S.(v x* A)
//   Sb = taub F + qdd A - qd (v x* A) + qd V                  (adjoint of S)
//   W = S x* Sb - fb x* I a - a x* I fb + (v x fb) x* I v + v x* I (v x fb)
//       + [c x g; g] for the hinge gradient g at each argmax sphere centre c
//   q-bar = S . subsum(W)
// since rotating joint i moves every world axis and inertia in its subtree
// (dS = dq S_i x S, dI = dq (S_i x* I - I S_i x)).
//
// The EXT variant adds two features, each switched on at run time:
// * external link forces: f_ext is given in link coordinates and turns with
//   its link, f_w = X* f_ext; it enters the force line as
//   f = I a + v x* I v - f_w, adds fb x* f_w to W (the rotation of f_w with
//   the joints above it), and its gradient is f_ext-bar = -X*^T fb;
// * mimic joints (Alg. 4's m_k and joint map): link l turns by
//   theta_l = m_l q_j + o_l, so its rates are m_l qd_j and m_l qdd_j; joint j's
//   torque is sum over its links of m_l S_l . F_l.  Lane j of the group owns
//   joint j: it gathers the torque from the links' lanes (connectedLinks),
//   runs the cost head, and its tau-bar returns to each link as m_l tau-bar_j;
//   the per-link adjoints (q-bar, qd-bar, qdd-bar) come back the same way,
//   each scaled by m_l, and lane j writes joint j's outputs and step.
#include "spline.h"
#include "sweep.h"
#include "tree.h"

namespace wb {

// The whole iteration for one state per group of G lanes.  Every lane of
// the wavefront calls this (group-local shuffles need all lanes); `valid`
// is false for groups past the end of the batch, which compute on a copy of
// a valid state and store nothing.  The lane's link constants are read from
// the lane tables at the point of use in every state (they stay in the L1
// cache), so that no register holds them across the sweep.
// SPL >= 1: the lane's joint position, velocity and acceleration are the
// spline sample of state b (trajectory b / H, segment, quarter of the
// interval) formed from the control points, with the arithmetic of the
// B-spline kernels; the state arrays are not read and the state step is off.
// SPL == 2: the sample's gradient also goes back onto its four-knot window
// and is added to this group's partial sums gpart[d][K + 6] in LDS (one
// group at a time per partial, states in a fixed order: deterministic).
// With SPL the state is sample t of trajectory traj (b = traj * H + t).
template <int NMAX, bool FULL, bool EXT, int SPL>
__device__ __forceinline__ void iterate_state(const DevRobot &rb, const uint16_t *tab, const DevFused &fz,
                                              const TreeIO &io, const SplineIn &sp, const StepScalars &k,
                                              float4 *P, float4 *Bd, uint16_t *list, float *gpart, int G, int grp,
                                              int glane, int64_t B, int64_t b, bool valid, int traj, int t) {
    int gl = glane;
    asm volatile("" : "+v"(gl));   // keeps the table reads inside the state loop
    const int *li = fz.li;
    const float *lf = fz.lf;
    const bool act = glane < rb.L;
    const int parent_lane = li[1 * 64 + gl];
    const bool revolute = li[5 * 64 + gl] != 0;
    const int64_t jo = (int64_t)li[3 * 64 + gl] * B + b;
    const bool mim = EXT && fz.mimic;
    float th = 0.f, thd = 0.f, thdd = 0.f, mult = 1.f;
    if (SPL > 0 && revolute) {
        const int64_t o0 = (int64_t)li[3 * 64 + gl] * sp.T + traj;
        const float t0 = sp.th0[o0];
        const float v0 = sp.dth0 ? sp.dth0[o0] * sp.dt : 0.f;
        const float a0 = sp.ddth0 ? sp.ddth0[o0] * (sp.dt * sp.dt) : 0.f;
        float w[4], c[4];
        segment_window(sp.U + o0 * sp.K, sp.K, t >> 2, t0, v0, a0, sp.printed != 0, w);
        window_coefficients(w, c);
        sample_at(c, 0.25f * (t & 3), 1.f / sp.dt, th, thd, thdd);
    } else if (revolute) {
        th = io.q[jo];
        thd = io.qd[jo];
        thdd = io.qdd[jo];
        if (mim) {
            mult = lf[29 * 64 + gl];
            th = mult * th + lf[30 * 64 + gl];
            thd *= mult;
            thdd *= mult;
        }
    }
    // ---- forward kinematics
    M3 R;
#pragma unroll
    for (int t = 0; t < 9; ++t) R.m[t] = lf[(3 + t) * 64 + gl];
    V3 p = v3(lf[12 * 64 + gl], lf[13 * 64 + gl], lf[14 * 64 + gl]);
    if (revolute) {
        float s, c;
        sincosf(th, &s, &c);
        const M3 Jr = axis_angle(v3(lf[0 * 64 + gl], lf[1 * 64 + gl], lf[2 * 64 + gl]), s, c);
        R = li[6 * 64 + gl] ? Jr : matmul(R, Jr);
    }
    {
        // Lane 0 is the fixed root, whose pose is the world frame (identity),
        // as is every lane past the robot: a chain that has reached the root
        // keeps composing with that identity, which changes nothing exactly,
        // so every lane takes every step without a guard.
        int anc = max(parent_lane, 0);
        auto jump = [&]() {
            M3 Ra;
#pragma unroll
            for (int t = 0; t < 9; ++t) Ra.m[t] = __shfl(R.m[t], anc, G);
            const V3 pa = v3(__shfl(p.x, anc, G), __shfl(p.y, anc, G), __shfl(p.z, anc, G));
            anc = __shfl(anc, anc, G);
            p = mul(Ra, p) + pa;
            R = matmul(Ra, R);
        };
        // two steps per trip: the pose alternates between two register sets
        // instead of being copied back after every step
        int st = 0;
        for (; st + 1 < fz.jsteps; st += 2) {
            jump();
            jump();
        }
        if (st < fz.jsteps) jump();
    }
    // ---- sphere centres and the link's bounding sphere into the group's LDS
    const int link = li[0 * 64 + gl];
    {
        const int nsph = li[4 * 64 + gl];
        wave_sync();
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
            if (j < nsph) {
                const float4 loc = fz.lsph[j * 64 + gl];
                const V3 c = mul(R, v3(loc.x, loc.y, loc.z)) + p;
                P[link * NMAX + j] = make_float4(c.x, c.y, c.z, loc.w);
            }
        if (nsph > 0) {
            const V3 c = mul(R, v3(lf[25 * 64 + gl], lf[26 * 64 + gl], lf[27 * 64 + gl])) + p;
            Bd[link] = make_float4(c.x, c.y, c.z, lf[28 * 64 + gl]);
        }
        wave_sync();
    }
    // ---- self-collision
    float M;
    int key;
    unsigned cnt;
    // the group's row ring follows its list
    sweep_state<NMAX, FULL>(rb, tab, P, Bd, list, reinterpret_cast<uint32_t *>(list + rb.list_cap), glane, G, grp, M,
                            key, cnt);
    const float hmarg = M + k.margin;
    const bool hinge_on = key != INT_MAX && hmarg > 0.f && k.hinge_weight != 0.f;
    // W: adjoint of the lane's joint rotation, before the subtree sum.  The
    // hinge force is formed without branches: a state without it reads the
    // pair (0, 0) and selects zero.  A checked pair joins two different
    // links, so a lane takes at most one of the two sphere forces.
    SV W = zsv();
    if (rb.S > 0) {
        const int hk = hinge_on ? key : 0;
        const int s = (int)((unsigned)hk / (unsigned)rb.S), t = hk - s * rb.S;
        const float4 cs = P[rb.sph_slot[s]], ct = P[rb.sph_slot[t]];
        const V3 d = v3(cs.x - ct.x, cs.y - ct.y, cs.z - ct.z);
        const float d2 = dot(d, d);
        // 1/n as the reciprocal of the rounded root (n >= 2^-75 for any d2 > 0)
        const bool on = hinge_on && d2 > 0.f;
        const V3 g = on ? (k.hinge_weight * __builtin_amdgcn_rcpf(sqrtf(d2))) * d : v3(0.f, 0.f, 0.f);
        const bool on_s = act && link == rb.sph_link[s], on_t = act && link == rb.sph_link[t];
        const V3 c = on_s ? v3(cs.x, cs.y, cs.z) : v3(ct.x, ct.y, ct.z);
        const V3 f = on_s ? -g : g;   // gradient on c_t is g, on c_s -g
        if (on_s || on_t) W = sv(cross(c, f), f);
    }
    // ---- world axis and inertia
    SV S = zsv();
    if (revolute) {
        const V3 sw = mul(R, v3(lf[0 * 64 + gl], lf[1 * 64 + gl], lf[2 * 64 + gl]));
        S = sv(sw, cross(p, sw));
    }
    WInertia J;
    {
        J.m = lf[15 * 64 + gl];
        J.cw = mul(R, v3(lf[16 * 64 + gl], lf[17 * 64 + gl], lf[18 * 64 + gl])) + p;
        float Ic[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) Ic[t] = lf[(19 + t) * 64 + gl];
        rotate_inertia(R, Ic, J.I);
    }
    const int sub_end = li[2 * 64 + gl];
    // ---- external force in world coordinates, f_w = X* f_ext (moment about the world origin)
    SV fe = zsv();
    if (EXT && io.f_ext && act) {
        const float *fx = io.f_ext + (int64_t)(link * 6) * B + b;
        const V3 Rf = mul(R, v3(fx[3 * B], fx[4 * B], fx[5 * B]));
        fe = sv(mul(R, v3(fx[0], fx[B], fx[2 * B])) + cross(p, Rf), Rf);
    }
    // ---- RNEA forward.  A lane past the robot is a massless link without a
    // joint whose parent is the fixed root (zero velocity and acceleration),
    // so every force and adjoint it forms below is exactly zero and the
    // subtree scans take it unguarded.
    const SV Sqd = thd * S;
    const SV v = path_sum(Sqd, parent_lane, glane, fz.jsteps, G);
    SV a = path_sum(thdd * S + crm(v, Sqd), parent_lane, glane, fz.jsteps, G);
    if (act) a += sv(v3(0.f, 0.f, 0.f), v3(-rb.gx, -rb.gy, -rb.gz));
    const SV Ia = iw_apply(J, a), Iv = iw_apply(J, v);
    SV F = Ia + crf(v, Iv);
    if (EXT) F = F - fe;
    F = subtree_sum(F, glane, sub_end, G);
    float tau = revolute ? dot(S, F) : 0.f;
    // with mimic joints, joint lane j (j < n) holds joint j from here to the cost head
    const bool jlane = mim ? gl < rb.n : revolute;
    const int64_t jrow = mim ? (int64_t)gl * B + b : jo;
    if (mim) tau = gather_joint(mult * tau, fz, gl, G);
    // ---- cost head
    float tcost = 0.f, taub = 0.f;
    if (jlane) {
        if (io.w) {
            const float wj = io.w[jrow];
            tcost = wj * tau;
            taub = wj;
        } else {
            tcost = k.torque_weight * tau * tau;
            taub = k.torque_weight * (2.f * tau);   // the same product as 2 tw tau (x2 is exact), nothing loop-invariant to keep
        }
    }
    tcost = group_reduce_sum(tcost, G);
    if (mim) {   // tau-bar back to the links: m_l tau-bar_j
        const float tj = __shfl(taub, revolute ? li[3 * 64 + gl] : gl, G);
        taub = revolute ? mult * tj : 0.f;
    }
    // ---- VJP, with the terms of W added as soon as their factors exist;
    // the terms crf(S, .) are linear in their second argument, so they are
    // gathered in X and crossed with S once at the end
    SV X = taub * F;
    const SV fb = path_sum(taub * S, parent_lane, glane, fz.jsteps, G);
    if (EXT && io.g_fext && act && valid) {
        // the external-force gradient needs only fb, so it leaves here and the
        // link's pose is dead for the rest of the adjoint: -X*^T fb, moment
        // part -R^T fb_w, force part -R^T (fb_l + fb_w x p)
        const V3 gn = mulT(R, fb.w), gf = mulT(R, fb.l + cross(fb.w, p));
        float *gx = io.g_fext + (int64_t)(link * 6) * B + b;
        gx[0] = -gn.x; gx[B] = -gn.y; gx[2 * B] = -gn.z;
        gx[3 * B] = -gf.x; gx[4 * B] = -gf.y; gx[5 * B] = -gf.z;
    }
    SV ab = iw_apply(J, fb);
    W = W - (crf(fb, Ia) + crf(a, ab));
    if (EXT) W += crf(fb, fe);
    const SV vxfb = crm(v, fb);
    const SV Ivxfb = iw_apply(J, vxfb);
    SV vb = zsv() - (crf(fb, Iv) + Ivxfb);
    W += crf(vxfb, Iv) + crf(v, Ivxfb);
    const SV Acc = subtree_sum(ab, glane, sub_end, G);
    vb += thd * crf(S, Acc);   // crf(S qd, Acc)
    const SV vxA = crf(v, Acc);
    const float thdd_b = dot(S, Acc);
    X += thdd * Acc - thd * vxA;
    const SV V = subtree_sum(vb, glane, sub_end, G);
    const float thd_b = dot(S, V) - dot(S, vxA);
    X += thd * V;
    W += crf(S, X);
    const SV Ws = subtree_sum(W, glane, sub_end, G);
    float th_b = dot(S, Ws);
    float thd_o = thd_b, thdd_o = thdd_b;
    if (mim) {   // per-link adjoints to joints: sum of m_l x (link adjoint)
        th_b = gather_joint(mult * th_b, fz, gl, G);
        thd_o = gather_joint(mult * thd_b, fz, gl, G);
        thdd_o = gather_joint(mult * thdd_b, fz, gl, G);
    }
    // ---- outputs and the gradient step
    if (!valid) return;
    if (SPL == 2 && revolute) {   // the sample's gradient onto its window of extended knots
        const int seg = t >> 2;
        const float inv = 1.f / sp.dt;
        float r0 = 0.f, r1 = 0.f, r2 = 0.f, r3 = 0.f;
        window_grad(0.25f * (t & 3), th_b, thd_b * inv, thdd_b * (inv * inv), r0, r1, r2, r3);
        float *row = gpart + li[3 * 64 + gl] * (sp.K + 6) + seg;
        row[0] += r0;
        row[1] += r1;
        row[2] += r2;
        row[3] += r3;
    }
    if (jlane) {
        if (io.tau) io.tau[jrow] = tau;
        if (io.g_q) io.g_q[jrow] = th_b;
        if (io.g_qd) io.g_qd[jrow] = thd_o;
        if (io.g_qdd) io.g_qdd[jrow] = thdd_o;
        if (SPL == 0 && k.lr != 0.f) {
            if (mim) {   // the joint's own values (a link lane holds m_l q + o_l)
                io.q[jrow] -= k.lr * th_b;
                io.qd[jrow] -= k.lr * thd_o;
                io.qdd[jrow] -= k.lr * thdd_o;
            } else {
                io.q[jo] = th - k.lr * th_b;
                io.qd[jo] = thd - k.lr * thd_b;
                io.qdd[jo] = thdd - k.lr * thdd_b;
            }
        }
    }
    if (glane == 0) {
        if (io.cost) io.cost[b] = tcost + k.hinge_weight * fmaxf(hmarg, 0.f);
        if (io.max_pen) io.max_pen[b] = M;
        if (io.argmax) io.argmax[b] = pair_index(rb, key);
        if (io.n_coll) io.n_coll[b] = (int32_t)cnt;
    }
}

// Process `count` states starting at b0 of one robot with the 4 waves of
// this workgroup, 64/G states per wavefront at a time; tab is the robot's
// block table staged in LDS.  GSEL: 64 builds only the one-state-per-
// wavefront path (G must be 64), 0 only the path for G = 16 or 32, -1 both
// (a plan mixes trees of every G).  A kernel holding one path keeps far
// fewer values live across the state loop (the two paths' scalars spilled
// to VGPR lanes and were re-read per state).
template <int NMAX, bool EXT, int SPL, int GSEL>
__device__ __forceinline__ void run_states(const DevRobot &rb, const uint16_t *tab, const DevFused &fz, const TreeIO &io,
                                           const SplineIn &sp, const StepScalars &k, float4 *lds_wave,
                                           float *gparts, int G, int64_t B, int64_t b0, int count, int traj) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int per_wave = 64 / G, grp = lane / G, glane = lane - grp * G;
    const int SL = (rb.L + 1) * NMAX;
    float4 *P = lds_wave + grp * (int)(group_lds_bytes(rb.L, NMAX, rb.list_cap) / 16);
    float4 *Bd = P + SL;
    uint16_t *list = reinterpret_cast<uint16_t *>(Bd + rb.L + 1);
    wave_sync();
    for (int i = glane; i < SL; i += G) P[i] = make_float4(0.f, 0.f, 0.f, rb.slot_r[i]);
    // links without spheres (and the padding link L) keep an empty bounding sphere
    for (int i = glane; i <= rb.L; i += G) Bd[i] = make_float4(0.f, 0.f, 0.f, -1e30f);
    for (int base = wave * per_wave; base < count; base += 4 * per_wave) {
        const int s = base + grp;
        const bool valid = s < count;
        const int64_t b = b0 + (valid ? s : base);
        float *gpart = SPL == 2 ? gparts + (wave * per_wave + grp) * rb.n * (sp.K + 6) : nullptr;
        // SPL == 2: the workgroup's trajectory, sample s; SPL == 1: chunks
        // span trajectories (the spline form keeps B below 2^31)
        int tr = traj, t = valid ? s : base;
        if (SPL == 1) {
            const int bi = (int)b;
            tr = bi / sp.H;
            t = bi - tr * sp.H;
        }
        if (GSEL == 64 || (GSEL < 0 && G == 64))
            iterate_state<NMAX, true, EXT, SPL>(rb, tab, fz, io, sp, k, P, Bd, list, gpart, 64, 0, glane, B, b, valid,
                                                tr, t);
        else
            iterate_state<NMAX, false, EXT, SPL>(rb, tab, fz, io, sp, k, P, Bd, list, gpart, G, grp, glane, B, b,
                                                 valid, tr, t);
    }
}

// The robot's block table into LDS as 16-bit link pairs (a << 8) | b (the
// fused kernels take at most 64 links); padding entries become (L, L).
__device__ __forceinline__ void stage_table(const DevRobot &rb, uint16_t *tab) {
    for (int i = threadIdx.x; i < rb.n_blocks_pad; i += 256) {
        const int ab = rb.blocks[i];
        tab[i] = (uint16_t)PairCode<uint16_t>::make(ab >> 16, ab & 0xffff);
    }
}

// The control-point gradient of the workgroup's trajectory (SPL == 2): the
// groups' partial sums over the extended knots, added in a fixed order; knot
// e = k + 3 is control point k, and the three copies of the final control
// point add into it; then the step, plain or row-normalized (the row's sum
// of squares taken by every lane of the row in the same order).
__device__ __forceinline__ void spline_reduce_step(const SplineIn &sp, const float *gparts, float *gsum, int d,
                                                   int nparts, int traj) {
    const int KE = sp.K + 6;
    for (int i = threadIdx.x; i < d * sp.K; i += 256) {
        const int j = i / sp.K, kk = i - j * sp.K;
        float g = 0.f;
        for (int p = 0; p < nparts; ++p) {
            const float *row = gparts + (p * d + j) * KE;
            g += row[kk + 3];
            if (kk == sp.K - 1) g += row[sp.K + 3] + row[sp.K + 4] + row[sp.K + 5];
        }
        gsum[i] = g;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < d * sp.K; i += 256) {
        const int j = i / sp.K, kk = i - j * sp.K;
        const float g = gsum[i];
        const int64_t o = ((int64_t)j * sp.T + traj) * sp.K + kk;
        if (sp.g_U) sp.g_U[o] = g;
        if (sp.lr != 0.f) {
            float step = sp.lr;
            if (sp.rule == WB_STEP_ROW_RMS) {
                float ss = 0.f;
                for (int m = 0; m < sp.K; ++m) ss += gsum[j * sp.K + m] * gsum[j * sp.K + m];
                step = ss > 0.f ? sp.lr * rsqrtf(ss / (float)sp.K) : 0.f;
            }
            sp.U[o] -= step * g;
        }
    }
}

// Waves per SIMD the register budget is set for: 4 (128 VGPRs) for the lean
// iteration; 3 for EXT, the variant with external link forces and mimic
// joints, which holds the forces, the joint-to-link map and their adjoints
// as well (at 128 VGPRs it spilled ~48 registers); 2 for 12 sphere slots
// per link, where the group regions (about 55 KB per workgroup) leave room
// for two workgroups per CU anyway.
template <int NMAX, bool EXT>
constexpr int fused_waves() { return NMAX > 8 ? 2 : (EXT ? 3 : 4); }

template <int NMAX, bool EXT, int SPL, int GSEL>
__global__ void __launch_bounds__(256, (fused_waves<NMAX, EXT>())) k_fused_step(FusedArgs A) {
    extern __shared__ float4 lds[];
    const int wave = threadIdx.x >> 6;
    const int G = GSEL == 64 ? 64 : A.lanes_per_state;
    const int SLW = (64 / G) * (int)(group_lds_bytes(A.rb.L, NMAX, A.rb.list_cap) / 16);
    // XCD-aware chunk order: consecutive chunks stay on one XCD's L2.
    const int nwg = gridDim.x, x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int qd8 = nwg >> 3, rd8 = nwg & 7;
    const int chunk = x * qd8 + min(x, rd8) + y;
    const int64_t b0 = (int64_t)chunk * A.chunk;
    const int64_t rem = A.B - b0;
    const int count = rem < A.chunk ? (int)rem : A.chunk;
    uint16_t *tab = reinterpret_cast<uint16_t *>(lds + 4 * SLW);
    // the control-point partial sums follow the block table (n_blocks_pad is a multiple of 128)
    float *gparts = reinterpret_cast<float *>(tab + A.rb.n_blocks_pad);
    const int nparts = 256 / G, d = A.rb.n;
    stage_table(A.rb, tab);
    if (SPL == 2)
        for (int i = threadIdx.x; i < nparts * d * (A.sp.K + 6); i += 256) gparts[i] = 0.f;
    __syncthreads();
    // with SPL == 2 each workgroup owns one trajectory (chunk == H)
    const int traj = SPL == 2 ? chunk : 0;
    run_states<NMAX, EXT, SPL, GSEL>(A.rb, tab, A.fz, A.io, A.sp, A.k, lds + wave * SLW, gparts, G, A.io.ld, b0, count,
                               traj);
    if (SPL == 2) {
        __syncthreads();
        spline_reduce_step(A.sp, gparts, gparts + nparts * d * (A.sp.K + 6), d, nparts, traj);
    }
}

// A plan tree's descriptors, read from device memory, with every table
// pointer re-derived as a global one (see as_global).
__device__ __forceinline__ PlanTree load_tree(const PlanTree *t) {
    PlanTree T = ldu(t);
    DevRobot &r = T.rb;
    r.lf = as_global(r.lf);
    r.li = as_global(r.li);
    r.sph = as_global(r.sph);
    r.sph_link = as_global(r.sph_link);
    r.sph_slot = as_global(r.sph_slot);
    r.slot_r = as_global(r.slot_r);
    r.blocks = as_global(r.blocks);
    r.pair_off = as_global(r.pair_off);
    r.pair_cnt = as_global(r.pair_cnt);
    r.pair_s = as_global(r.pair_s);
    r.pair_t = as_global(r.pair_t);
    DevFused &z = T.fz;
    z.li = as_global(z.li);
    z.lf = as_global(z.lf);
    z.lsph = as_global(z.lsph);
    z.conn = as_global(z.conn);
    return T;
}

// Persistent launch over an uneven batch of robots: workgroup w processes
// the items [item_start[w], item_start[w+1]) of the plan's work list, each a
// contiguous range of states of one robot.  EXT as for k_fused_step, chosen
// when any tree has mimic joints or external forces.
template <int NMAX, bool EXT>
__global__ void __launch_bounds__(256) k_plan_step(PlanArgs A) {
    extern __shared__ float4 lds[];
    const int wave = threadIdx.x >> 6;
    const int w = blockIdx.x;
    uint16_t *tab = reinterpret_cast<uint16_t *>(lds + 4 * A.wave_stride);
    int staged = -1;   // tree whose block table is in LDS
    for (int it = A.item_start[w]; it < A.item_start[w + 1]; ++it) {
        const PlanItem item = A.items[it];
        const PlanTree T = load_tree(A.trees + item.tree);
        const int G = T.lanes_per_state;
        if (item.tree != staged) {
            __syncthreads();   // every wave is done with the previous table
            stage_table(T.rb, tab);
            __syncthreads();
            staged = item.tree;
        }
        // a fixed region per wave, sized for the plan's largest tree
        run_states<NMAX, EXT, 0, -1>(T.rb, tab, T.fz, A.io[item.tree], SplineIn{}, A.k, lds + wave * A.wave_stride,
                                 nullptr, G, A.io[item.tree].ld,
                              item.b0, item.count, 0);
    }
}

template <int NMAX, int GSEL>
static hipError_t launch_fused_g(const FusedArgs &a, size_t lds, unsigned nwg, hipStream_t s) {
    const bool reduce = a.sp.U && (a.sp.g_U || a.sp.lr != 0.f);
    if (reduce) {
        lds += spline_lds_bytes(a.lanes_per_state, a.rb.n, a.sp.K);
        hipLaunchKernelGGL((k_fused_step<NMAX, false, 2, GSEL>), dim3(nwg), dim3(256), lds, s, a);
    } else if (a.sp.U)
        hipLaunchKernelGGL((k_fused_step<NMAX, false, 1, GSEL>), dim3(nwg), dim3(256), lds, s, a);
    else if (a.io.f_ext || a.io.g_fext || a.fz.mimic)
        hipLaunchKernelGGL((k_fused_step<NMAX, true, 0, GSEL>), dim3(nwg), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((k_fused_step<NMAX, false, 0, GSEL>), dim3(nwg), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <int NMAX>
static hipError_t launch_fused_t(const FusedArgs &a, hipStream_t s) {
    const size_t lds = fused_lds_bytes(a.rb.L, NMAX, a.rb.list_cap, a.lanes_per_state, a.rb.n_blocks_pad);
    const unsigned nwg = (unsigned)((a.B + a.chunk - 1) / a.chunk);
    return a.lanes_per_state == 64 ? launch_fused_g<NMAX, 64>(a, lds, nwg, s) : launch_fused_g<NMAX, 0>(a, lds, nwg, s);
}

hipError_t launch_fused(const FusedArgs &a, hipStream_t s) {
    if (a.B == 0) return hipSuccess;
    switch (a.rb.nmax) {
        case 1: return launch_fused_t<1>(a, s);
        case 2: return launch_fused_t<2>(a, s);
        case 3: return launch_fused_t<3>(a, s);
        case 4: return launch_fused_t<4>(a, s);
        case 5: return launch_fused_t<5>(a, s);
        case 6: return launch_fused_t<6>(a, s);
        case 7: return launch_fused_t<7>(a, s);
        case 8: return launch_fused_t<8>(a, s);
        case 12: return launch_fused_t<12>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int NMAX>
static hipError_t launch_plan_t(const PlanArgs &a, int n_wg, size_t lds, bool ext, hipStream_t s) {
    if (ext) hipLaunchKernelGGL((k_plan_step<NMAX, true>), dim3(n_wg), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((k_plan_step<NMAX, false>), dim3(n_wg), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <int NMAX>
static int plan_workgroups_per_cu_t(bool ext, size_t lds) {
    int n = 0;
    const hipError_t e = ext ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plan_step<NMAX, true>, 256, lds)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_plan_step<NMAX, false>, 256, lds);
    return e == hipSuccess && n > 0 ? n : 1;
}

int plan_workgroups_per_cu(int nmax, bool ext, size_t lds) {
    switch (nmax) {
        case 1: return plan_workgroups_per_cu_t<1>(ext, lds);
        case 2: return plan_workgroups_per_cu_t<2>(ext, lds);
        case 3: return plan_workgroups_per_cu_t<3>(ext, lds);
        case 4: return plan_workgroups_per_cu_t<4>(ext, lds);
        case 5: return plan_workgroups_per_cu_t<5>(ext, lds);
        case 6: return plan_workgroups_per_cu_t<6>(ext, lds);
        case 7: return plan_workgroups_per_cu_t<7>(ext, lds);
        case 8: return plan_workgroups_per_cu_t<8>(ext, lds);
        case 12: return plan_workgroups_per_cu_t<12>(ext, lds);
        default: return 1;
    }
}

hipError_t launch_plan(const PlanArgs &a, int nmax, int n_wg, size_t lds, bool ext, hipStream_t s) {
    if (n_wg == 0) return hipSuccess;
    switch (nmax) {
        case 1: return launch_plan_t<1>(a, n_wg, lds, ext, s);
        case 2: return launch_plan_t<2>(a, n_wg, lds, ext, s);
        case 3: return launch_plan_t<3>(a, n_wg, lds, ext, s);
        case 4: return launch_plan_t<4>(a, n_wg, lds, ext, s);
        case 5: return launch_plan_t<5>(a, n_wg, lds, ext, s);
        case 6: return launch_plan_t<6>(a, n_wg, lds, ext, s);
        case 7: return launch_plan_t<7>(a, n_wg, lds, ext, s);
        case 8: return launch_plan_t<8>(a, n_wg, lds, ext, s);
        case 12: return launch_plan_t<12>(a, n_wg, lds, ext, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace wb
