// Recursive Newton-Euler inverse dynamics and its vector-Jacobian product,
// one state per lane (cuRoboV2 Sec. 6.3, Alg. 4 and the role of Alg. 5).
//
// The per-link sweeps follow Alg. 4 in link coordinates with the compact
// transform (R, p) and compact inertia (m, c, Ic).  Links are visited in
// index order (parents first) instead of level by level: with one state per
// lane there is no intra-state parallelism to exploit, and index order keeps
// the parent's values in registers whenever the parent is the previous link
// (a "carry"), touching the cache only at branch points.
//
// Cache layout [L][18][B]: v (6), a (6), accumulated force F (6) per link;
// link 0 (the fixed base, v = 0, a = -g) is not stored.  External link
// forces f_ext [L][6][B] (link coordinates, moment then force about the link
// origin) enter Alg. 4 as f_k = I a + v x* I v - f_ext_k, so the cached F
// includes them and the backward needs only their adjoint, -F-bar_k.
//
// The backward is the exact reverse mode of the forward sweep (with
// dX/dtheta = -crm(S) X):
//   sweep A, base -> tips:  Fb_k = S m taub + X Fb_p,  thb += (X Fb_p).crf(S) F_k
//   sweep B, tips -> base:  ab_k = I Fb_k + sum_children X_c^T ab_c,
//                           vb_k = -crf(Fb) I v - I crm(v) Fb + crf(S thd) ab_k
//                                  + sum_children X_c^T vb_c,
//                           qdd-bar = S.ab, qd-bar = S.vb - S.(crf(v) ab),
//                           thb -= ab.crm(S) X a_p + vb.crm(S) X v_p.
// The crf(S thd) ab term is the velocity dependence of the Coriolis term of
// the acceleration recursion; it belongs to the exact VJP.
#include "spatial.h"

namespace wb {

__device__ __forceinline__ SV ld_sv(const float *__restrict__ base, int64_t B) {
    return sv(v3(base[0], base[B], base[2 * B]), v3(base[3 * B], base[4 * B], base[5 * B]));
}
__device__ __forceinline__ void st_sv(float *__restrict__ base, int64_t B, SV x) {
    base[0] = x.w.x; base[B] = x.w.y; base[2 * B] = x.w.z;
    base[3 * B] = x.l.x; base[4 * B] = x.l.y; base[5 * B] = x.l.z;
}
__device__ __forceinline__ void add_sv(float *__restrict__ base, int64_t B, SV x) {
    base[0] += x.w.x; base[B] += x.w.y; base[2 * B] += x.w.z;
    base[3 * B] += x.l.x; base[4 * B] += x.l.y; base[5 * B] += x.l.z;
}

struct JointIn {
    float th, thd, thdd;
};

__device__ __forceinline__ JointIn joint_in(const LinkF &f, const LinkI &i, const float *__restrict__ q,
                                            const float *__restrict__ qd, const float *__restrict__ qdd,
                                            int64_t B, int64_t b) {
    JointIn r{0.f, 0.f, 0.f};
    if (i.revolute) {
        const int64_t o = (int64_t)i.jidx * B + b;
        r.th = f.mult * q[o] + f.offset;
        r.thd = f.mult * qd[o];
        r.thdd = f.mult * qdd[o];
    }
    return r;
}

// nb: states; B: row length of every [k][B] array (the ABI's ld >= nb).
__global__ void __launch_bounds__(256) k_rnea(DevRobot rb, int64_t nb, int64_t B, const float *__restrict__ q,
                                              const float *__restrict__ qd, const float *__restrict__ qdd,
                                              const float *__restrict__ f_ext, float *__restrict__ tau,
                                              float *__restrict__ cache) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int L = rb.L;
    const SV a0 = sv(v3(0.f, 0.f, 0.f), v3(-rb.gx, -rb.gy, -rb.gz));
    const SV zero = sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f));
    float *cb = cache + b;
    if (!rb.simple_joints)
        for (int j = 0; j < rb.n; ++j) tau[(int64_t)j * B + b] = 0.0f;
    // Pass 1 (base -> tips): velocities, accelerations, link forces.
    SV v = zero, a = a0;
    for (int k = 1; k < L; ++k) {
        const LinkI li = ldu(rb.li + k);
        const LinkF lf = ldu(rb.lf + k);
        const int p = li.parent;
        SV vp = v, ap = a;
        if (p == 0) {
            vp = zero;
            ap = a0;
        } else if (p != k - 1) {
            vp = ld_sv(cb + (int64_t)(p * 18) * B, B);
            ap = ld_sv(cb + (int64_t)(p * 18 + 6) * B, B);
        }
        const JointIn J = joint_in(lf, li, q, qd, qdd, B, b);
        const M3 R = local_rotation(lf, li, J.th);
        const V3 r = v3(lf.fp[0], lf.fp[1], lf.fp[2]);
        const V3 s = v3(lf.axis[0], lf.axis[1], lf.axis[2]);
        const SV Sqd = sv(J.thd * s, v3(0.f, 0.f, 0.f));
        v = X_apply(R, r, vp) + Sqd;
        a = X_apply(R, r, ap) + sv(J.thdd * s, v3(0.f, 0.f, 0.f)) + crm(v, Sqd);
        SV f = I_apply(lf, a) + crf(v, I_apply(lf, v));
        if (f_ext) f = f - ld_sv(f_ext + (int64_t)(k * 6) * B + b, B);
        float *ck = cb + (int64_t)(k * 18) * B;
        st_sv(ck, B, v);
        st_sv(ck + 6 * B, B, a);
        st_sv(ck + 12 * B, B, f);
    }
    // Pass 3 (tips -> base): accumulate forces into parents, project on joints.
    SV carry = zero;
    bool have_carry = false;
    for (int k = L - 1; k >= 1; --k) {
        const LinkI li = ldu(rb.li + k);
        const LinkF lf = ldu(rb.lf + k);
        float *cF = cb + (int64_t)(k * 18 + 12) * B;
        SV F = ld_sv(cF, B);
        if (have_carry) {
            F += carry;
            st_sv(cF, B, F);
        }
        const JointIn J = joint_in(lf, li, q, qd, qdd, B, b);
        if (li.revolute) {
            const float t = lf.mult * (lf.axis[0] * F.w.x + lf.axis[1] * F.w.y + lf.axis[2] * F.w.z);
            float *tj = tau + (int64_t)li.jidx * B + b;
            if (rb.simple_joints) *tj = t;
            else *tj += t;
        }
        const int p = li.parent;
        have_carry = false;
        if (p >= 1) {
            const M3 R = local_rotation(lf, li, J.th);
            const SV fp = XT_apply(R, v3(lf.fp[0], lf.fp[1], lf.fp[2]), F);
            if (p == k - 1) {
                carry = fp;
                have_carry = true;
            } else {
                add_sv(cb + (int64_t)(p * 18 + 12) * B, B, fp);
            }
        }
    }
}

// ws layout per state: [L][18]: Fb (6), ab (6), vb (6).
__global__ void __launch_bounds__(256) k_rnea_backward(DevRobot rb, int64_t nb, int64_t B, const float *__restrict__ q,
                                                       const float *__restrict__ qd,
                                                       const float *__restrict__ qdd,
                                                       const float *__restrict__ cache,
                                                       const float *__restrict__ g_tau,
                                                       float *__restrict__ g_q, float *__restrict__ g_qd,
                                                       float *__restrict__ g_qdd, float *__restrict__ g_fext,
                                                       float *__restrict__ ws) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int L = rb.L;
    const SV a0 = sv(v3(0.f, 0.f, 0.f), v3(-rb.gx, -rb.gy, -rb.gz));
    const SV zero = sv(v3(0.f, 0.f, 0.f), v3(0.f, 0.f, 0.f));
    const float *cb = cache + b;
    float *wb_ = ws + b;
    if (!rb.simple_joints)
        for (int j = 0; j < rb.n; ++j) {
            g_q[(int64_t)j * B + b] = 0.0f;
            g_qd[(int64_t)j * B + b] = 0.0f;
            g_qdd[(int64_t)j * B + b] = 0.0f;
        }
    // Sweep A (base -> tips): adjoint of the force accumulation.
    SV Fb = zero;
    if (g_fext) st_sv(g_fext + b, B, zero);   // the base's force reaches no joint
    for (int k = 1; k < L; ++k) {
        const LinkI li = ldu(rb.li + k);
        const LinkF lf = ldu(rb.lf + k);
        const int p = li.parent;
        SV Fbp = Fb;
        if (p == 0) Fbp = zero;
        else if (p != k - 1) Fbp = ld_sv(wb_ + (int64_t)(p * 18) * B, B);
        const JointIn J = joint_in(lf, li, q, qd, qdd, B, b);
        const M3 R = local_rotation(lf, li, J.th);
        const V3 s = v3(lf.axis[0], lf.axis[1], lf.axis[2]);
        const SV XFp = X_apply(R, v3(lf.fp[0], lf.fp[1], lf.fp[2]), Fbp);
        const float tb = li.revolute ? lf.mult * g_tau[(int64_t)li.jidx * B + b] : 0.0f;
        Fb = sv(tb * s, v3(0.f, 0.f, 0.f)) + XFp;
        float *wk = wb_ + (int64_t)(k * 18) * B;
        st_sv(wk, B, Fb);
        if (g_fext) st_sv(g_fext + (int64_t)(k * 6) * B + b, B, zero - Fb);
        if (li.far_child) {
            st_sv(wk + 6 * B, B, zero);
            st_sv(wk + 12 * B, B, zero);
        }
        if (li.revolute) {
            const SV F = ld_sv(cb + (int64_t)(k * 18 + 12) * B, B);
            const float thb = lf.mult * (dot(XFp.w, cross(s, F.w)) + dot(XFp.l, cross(s, F.l)));
            float *gq = g_q + (int64_t)li.jidx * B + b;
            if (rb.simple_joints) *gq = thb;
            else *gq += thb;
        }
    }
    // Sweep B (tips -> base): adjoint of the velocity/acceleration recursion.
    SV ca = zero, cv = zero;
    bool have_carry = false;
    for (int k = L - 1; k >= 1; --k) {
        const LinkI li = ldu(rb.li + k);
        const LinkF lf = ldu(rb.lf + k);
        const int p = li.parent;
        const float *wk = wb_ + (int64_t)(k * 18) * B;
        const float *ck = cb + (int64_t)(k * 18) * B;
        const SV Fbk = ld_sv(wk, B);
        const SV vk = ld_sv(ck, B);
        SV ab = I_apply(lf, Fbk);
        SV vb = zero - (crf(Fbk, I_apply(lf, vk)) + I_apply(lf, crm(vk, Fbk)));
        if (have_carry) {
            ab += ca;
            vb += cv;
        }
        if (li.far_child) {
            ab += ld_sv(wk + 6 * B, B);
            vb += ld_sv(wk + 12 * B, B);
        }
        const JointIn J = joint_in(lf, li, q, qd, qdd, B, b);
        const V3 s = v3(lf.axis[0], lf.axis[1], lf.axis[2]);
        const SV Sqd = sv(J.thd * s, v3(0.f, 0.f, 0.f));
        vb += crf(Sqd, ab);
        const M3 R = local_rotation(lf, li, J.th);
        const V3 r = v3(lf.fp[0], lf.fp[1], lf.fp[2]);
        if (li.revolute) {
            SV vp = zero, ap = a0;
            if (p != 0) {
                vp = ld_sv(cb + (int64_t)(p * 18) * B, B);
                ap = ld_sv(cb + (int64_t)(p * 18 + 6) * B, B);
            }
            const SV Xa = X_apply(R, r, ap), Xv = X_apply(R, r, vp);
            const float thdd_b = dot(s, ab.w);
            const float thd_b = dot(s, vb.w) - dot(s, crf(vk, ab).w);
            const float th_b = -(dot(ab.w, cross(s, Xa.w)) + dot(ab.l, cross(s, Xa.l)) +
                                 dot(vb.w, cross(s, Xv.w)) + dot(vb.l, cross(s, Xv.l)));
            const int64_t o = (int64_t)li.jidx * B + b;
            if (rb.simple_joints) {
                g_qdd[o] = thdd_b;
                g_qd[o] = thd_b;
            } else {
                g_qdd[o] += lf.mult * thdd_b;
                g_qd[o] += lf.mult * thd_b;
            }
            g_q[o] += lf.mult * th_b;
        }
        have_carry = false;
        if (p >= 1) {
            const SV pa = XT_apply(R, r, ab), pv = XT_apply(R, r, vb);
            if (p == k - 1) {
                ca = pa;
                cv = pv;
                have_carry = true;
            } else {
                float *wp = wb_ + (int64_t)(p * 18) * B;
                add_sv(wp + 6 * B, B, pa);
                add_sv(wp + 12 * B, B, pv);
            }
        }
    }
}

hipError_t launch_rnea(const DevRobot &rb, int64_t B, int64_t ld, const float *q, const float *qd,
                       const float *qdd, const float *f_ext, float *tau, float *cache, hipStream_t s) {
    if (B == 0) return hipSuccess;
    dim3 grid((unsigned)((B + 255) / 256));
    hipLaunchKernelGGL(k_rnea, grid, dim3(256), 0, s, rb, B, ld, q, qd, qdd, f_ext, tau, cache);
    return hipGetLastError();
}

hipError_t launch_rnea_backward(const DevRobot &rb, int64_t B, int64_t ld, const float *q, const float *qd,
                                const float *qdd, const float *cache, const float *g_tau,
                                float *g_q, float *g_qd, float *g_qdd, float *g_fext, float *ws, hipStream_t s) {
    if (B == 0) return hipSuccess;
    dim3 grid((unsigned)((B + 255) / 256));
    hipLaunchKernelGGL(k_rnea_backward, grid, dim3(256), 0, s, rb, B, ld, q, qd, qdd, cache, g_tau, g_q,
                       g_qd, g_qdd, g_fext, ws);
    return hipGetLastError();
}

}  // namespace wb
