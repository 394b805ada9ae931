// One trajectory-optimizer iteration of the whole-body hot path in a single
// kernel: forward kinematics, self-collision, RNEA, cost head, every adjoint
// and the gradient step (cuRoboV2 Sec. 3 loop steps 2, 3, 5 and 6 for the
// whole-body terms; Sec. 6.1-6.3).
//
// Mapping: one wavefront per state, lane i = link perm[i] in depth-first
// pre-order (so the subtree of lane i is the lane range [i, sub_end_i]).
// Nothing intermediate leaves the chip: link poses and spatial quantities
// live in registers, sphere centres in the wave's LDS slots.
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
// pointer jumping; subtree sums use an inclusive wave scan in DFS order and
// the difference of two scan values.
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
#include "sweep.h"

namespace wb {

__device__ __forceinline__ SV shfl_sv(SV x, int src) {
    return sv(v3(__shfl(x.w.x, src, 64), __shfl(x.w.y, src, 64), __shfl(x.w.z, src, 64)),
              v3(__shfl(x.l.x, src, 64), __shfl(x.l.y, src, 64), __shfl(x.l.z, src, 64)));
}
__device__ __forceinline__ SV shfl_up_sv(SV x, int d) {
    return sv(v3(__shfl_up(x.w.x, d, 64), __shfl_up(x.w.y, d, 64), __shfl_up(x.w.z, d, 64)),
              v3(__shfl_up(x.l.x, d, 64), __shfl_up(x.l.y, d, 64), __shfl_up(x.l.z, d, 64)));
}
__device__ __forceinline__ SV zsv() { return sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f)); }

// Sum of x over the path from the root to this lane's link.
__device__ __forceinline__ SV path_sum(SV x, int parent_lane, int lane, int steps) {
    int anc = parent_lane;
    for (int s = 0; s < steps; ++s) {
        const int src = anc < 0 ? lane : anc;
        const SV y = shfl_sv(x, src);
        const int aa = __shfl(anc, src, 64);
        if (anc >= 0) {
            x += y;
            anc = aa;
        }
    }
    return x;
}

// Sum of x over this lane's subtree (lanes [lane, sub_end]); lanes outside
// the robot must hold zero.
__device__ __forceinline__ SV subtree_sum(SV x, int lane, int sub_end) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const SV t = shfl_up_sv(x, d);
        if (lane >= d) x += t;
    }
    const SV hi = shfl_sv(x, sub_end);
    const SV lo = shfl_sv(x, lane > 0 ? lane - 1 : 0);
    return lane > 0 ? hi - lo : hi;
}

// World-frame spatial inertia product: CoM cw (world), mass m, rotational
// inertia Ic about the CoM in link axes with world rotation R.
struct WInertia {
    float m;
    V3 cw;
    M3 R;
    float I[6];
};
__device__ __forceinline__ SV iw_apply(const WInertia &J, SV u) {
    const V3 h = J.m * (u.l + cross(u.w, J.cw));
    const V3 wl = mulT(J.R, u.w);
    const V3 Iw = v3(J.I[0] * wl.x + J.I[3] * wl.y + J.I[4] * wl.z,
                     J.I[3] * wl.x + J.I[1] * wl.y + J.I[5] * wl.z,
                     J.I[4] * wl.x + J.I[5] * wl.y + J.I[2] * wl.z);
    return sv(mul(J.R, Iw) + cross(J.cw, h), h);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int NMAX>
__global__ void __launch_bounds__(256) k_fused_step(FusedArgs A) {
    extern __shared__ float4 lds[];
    const DevRobot &rb = A.rb;
    const DevFused &fz = A.fz;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int SL = (rb.L + 1) * NMAX;
    float4 *P = lds + wave * SL;
    for (int i = lane; i < SL; i += 64) P[i] = make_float4(0.f, 0.f, 0.f, rb.slot_r[i]);

    // Per-lane link constants (loaded once per wave).
    const bool act = lane < rb.L;
    const int link = act ? fz.li[0 * 64 + lane] : 0;
    const int parent_lane = act ? fz.li[1 * 64 + lane] : -1;
    const int sub_end = act ? fz.li[2 * 64 + lane] : lane;
    const int jidx = act ? fz.li[3 * 64 + lane] : -1;
    const int nsph = act ? fz.li[4 * 64 + lane] : 0;
    const bool revolute = act && fz.li[5 * 64 + lane] != 0;
    const bool fr_ident = !act || fz.li[6 * 64 + lane] != 0;
    const float *lf = fz.lf;
    V3 axis = v3(0.f, 0.f, 1.f), fp = v3(0.f, 0.f, 0.f), com = v3(0.f, 0.f, 0.f);
    M3 fR;
#pragma unroll
    for (int t = 0; t < 9; ++t) fR.m[t] = (t % 4 == 0) ? 1.f : 0.f;
    WInertia J;
    J.m = 0.f;
#pragma unroll
    for (int t = 0; t < 6; ++t) J.I[t] = 0.f;
    float4 loc[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) loc[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (act) {
        axis = v3(lf[0 * 64 + lane], lf[1 * 64 + lane], lf[2 * 64 + lane]);
#pragma unroll
        for (int t = 0; t < 9; ++t) fR.m[t] = lf[(3 + t) * 64 + lane];
        fp = v3(lf[12 * 64 + lane], lf[13 * 64 + lane], lf[14 * 64 + lane]);
        J.m = lf[15 * 64 + lane];
        com = v3(lf[16 * 64 + lane], lf[17 * 64 + lane], lf[18 * 64 + lane]);
#pragma unroll
        for (int t = 0; t < 6; ++t) J.I[t] = lf[(19 + t) * 64 + lane];
#pragma unroll
        for (int j = 0; j < NMAX; ++j) loc[j] = fz.lsph[j * 64 + lane];
    }
    const SV a0 = sv(v3(0.f, 0.f, 0.f), v3(-rb.gx, -rb.gy, -rb.gz));

    // XCD-aware chunk order: consecutive chunks stay on one XCD's L2.
    const int nwg = gridDim.x, x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int qd8 = nwg >> 3, rd8 = nwg & 7;
    const int chunk = x * qd8 + min(x, rd8) + y;
    const int64_t b0 = (int64_t)chunk * A.chunk;

    for (int k = wave; k < A.chunk; k += 4) {
        const int64_t b = b0 + k;
        if (b >= A.B) break;
        const int64_t jo = (int64_t)jidx * A.B + b;
        float th = 0.f, thd = 0.f, thdd = 0.f;
        if (revolute) {
            th = A.q[jo];
            thd = A.qd[jo];
            thdd = A.qdd[jo];
        }
        // ---- forward kinematics
        M3 R = fR;
        V3 p = fp;
        if (revolute) {
            float s, c;
            sincosf(th, &s, &c);
            const M3 Jr = axis_angle(axis, s, c);
            R = fr_ident ? Jr : matmul(fR, Jr);
        }
        {
            int anc = parent_lane;
            for (int st = 0; st < A.jsteps; ++st) {
                const int src = anc < 0 ? lane : anc;
                M3 Ra;
#pragma unroll
                for (int t = 0; t < 9; ++t) Ra.m[t] = __shfl(R.m[t], src, 64);
                const V3 pa = v3(__shfl(p.x, src, 64), __shfl(p.y, src, 64), __shfl(p.z, src, 64));
                const int aa = __shfl(anc, src, 64);
                if (anc >= 0) {
                    p = mul(Ra, p) + pa;
                    R = matmul(Ra, R);
                    anc = aa;
                }
            }
        }
        // ---- sphere centres into the wave's LDS slots
        wave_sync();
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
            if (j < nsph) {
                const V3 c = mul(R, v3(loc[j].x, loc[j].y, loc[j].z)) + p;
                P[link * NMAX + j] = make_float4(c.x, c.y, c.z, loc[j].w);
            }
        wave_sync();
        // ---- self-collision
        float M;
        int key;
        unsigned cnt;
        sweep_state<NMAX>(rb, P, lane, M, key, cnt);
        const float hmarg = M + A.margin;
        const bool hinge_on = key != INT_MAX && hmarg > 0.f && A.hinge_weight != 0.f;
        SV W = zsv();
        if (hinge_on) {
            const int s = key / rb.S, t = key - s * rb.S;
            const float4 cs = P[rb.sph_slot[s]], ct = P[rb.sph_slot[t]];
            const V3 d = v3(cs.x - ct.x, cs.y - ct.y, cs.z - ct.z);
            const float n = sqrtf(dot(d, d));
            if (n > 0.f) {
                const V3 g = (A.hinge_weight / n) * d;   // gradient on c_t; -g on c_s
                if (act && link == rb.sph_link[s]) {
                    const V3 c = v3(cs.x, cs.y, cs.z);
                    W += sv(cross(c, -g), -g);
                }
                if (act && link == rb.sph_link[t]) {
                    const V3 c = v3(ct.x, ct.y, ct.z);
                    W += sv(cross(c, g), g);
                }
            }
        }
        // ---- world axes and inertias
        SV S = zsv();
        if (revolute) {
            const V3 sw = mul(R, axis);
            S = sv(sw, cross(p, sw));
        }
        J.R = R;
        J.cw = mul(R, com) + p;
        // ---- RNEA forward
        const SV Sqd = thd * S;
        const SV v = path_sum(Sqd, parent_lane, lane, A.jsteps);
        const SV cterm = thdd * S + crm(v, Sqd);
        SV a = path_sum(cterm, parent_lane, lane, A.jsteps);
        if (act) a += a0;
        const SV Ia = iw_apply(J, a), Iv = iw_apply(J, v);
        SV f = Ia + crf(v, Iv);
        if (!act) f = zsv();
        const SV F = subtree_sum(f, lane, sub_end);
        const float tau = revolute ? dot(S, F) : 0.f;
        // ---- cost head
        float wj = 0.f, tcost = 0.f, taub = 0.f;
        if (revolute) {
            if (A.w) {
                wj = A.w[jo];
                tcost = wj * tau;
                taub = wj;
            } else {
                tcost = A.torque_weight * tau * tau;
                taub = 2.f * A.torque_weight * tau;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tcost += __shfl_xor(tcost, o, 64);
        // ---- VJP
        const SV fb = path_sum(taub * S, parent_lane, lane, A.jsteps);
        const SV ab = iw_apply(J, fb);
        const SV vxfb = crm(v, fb);
        const SV Ivxfb = iw_apply(J, vxfb);
        SV vb = zsv() - (crf(fb, Iv) + Ivxfb);
        SV ab_act = act ? ab : zsv();
        const SV Acc = subtree_sum(ab_act, lane, sub_end);
        vb += crf(Sqd, Acc);
        if (!act) vb = zsv();
        const SV vxA = crf(v, Acc);
        const float thdd_b = dot(S, Acc);
        const SV V = subtree_sum(vb, lane, sub_end);
        const float thd_b = dot(S, V) - dot(S, vxA);
        const SV Sb = taub * F + thdd * Acc - thd * vxA + thd * V;
        W += crf(S, Sb) - crf(fb, Ia) - crf(a, ab) + crf(vxfb, Iv) + crf(v, Ivxfb);
        if (!act) W = zsv();
        const SV Ws = subtree_sum(W, lane, sub_end);
        const float th_b = dot(S, Ws);
        // ---- outputs and the gradient step
        if (revolute) {
            if (A.tau) A.tau[jo] = tau;
            if (A.g_q) A.g_q[jo] = th_b;
            if (A.g_qd) A.g_qd[jo] = thd_b;
            if (A.g_qdd) A.g_qdd[jo] = thdd_b;
            if (A.lr != 0.f) {
                A.q[jo] = th - A.lr * th_b;
                A.qd[jo] = thd - A.lr * thd_b;
                A.qdd[jo] = thdd - A.lr * thdd_b;
            }
        }
        if (lane == 0) {
            if (A.cost) A.cost[b] = tcost + A.hinge_weight * fmaxf(hmarg, 0.f);
            if (A.max_pen) A.max_pen[b] = M;
            if (A.argmax) A.argmax[b] = pair_index(rb, key);
            if (A.n_coll) A.n_coll[b] = (int32_t)cnt;
        }
    }
}

template <int NMAX>
static hipError_t launch_fused_t(const FusedArgs &a, hipStream_t s) {
    const size_t lds = (size_t)4 * (a.rb.L + 1) * NMAX * sizeof(float4);
    const unsigned nwg = (unsigned)((a.B + a.chunk - 1) / a.chunk);
    hipLaunchKernelGGL(k_fused_step<NMAX>, dim3(nwg), dim3(256), lds, s, a);
    return hipGetLastError();
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
        default: return hipErrorInvalidValue;
    }
}

}  // namespace wb
