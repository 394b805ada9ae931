// Forward kinematics and its adjoint, one state per lane.
//
// Forward (cuRoboV2 Sec. 6.1): links are visited in index order (parents
// first); the running pose stays in registers while the next link is the
// current one's child and is re-read from the pose array otherwise (or,
// without one, recomposed from q along the parent's chain), so a serial
// chain never reloads.  Sphere centres are R c_local + p.
//
// Backward (the gradient of Alg. 1): instead of walking every link's
// ancestor chain, each link accumulates the force F = sum of point-gradient
// vectors and the moment M about its own origin of everything below it
// (spheres, pose gradients, children); the joint gradient is then
// s_world . M, which equals the ancestor-chain sum of Alg. 1 link by link.
// Subtree totals move to the parent as F_p += F, M_p += M + (o - o_p) x F.
#include "spatial.h"

namespace wb {

__device__ __forceinline__ void store_pose(float *__restrict__ pose, int k, int64_t B, int64_t b,
                                           const M3 &R, V3 p) {
    float *o = pose + (int64_t)k * 12 * B + b;
#pragma unroll
    for (int t = 0; t < 9; ++t) o[t * B] = R.m[t];
    o[9 * B] = p.x;
    o[10 * B] = p.y;
    o[11 * B] = p.z;
}

__device__ __forceinline__ void load_pose(const float *__restrict__ pose, int k, int64_t B, int64_t b,
                                          M3 &R, V3 &p) {
    const float *o = pose + (int64_t)k * 12 * B + b;
#pragma unroll
    for (int t = 0; t < 9; ++t) R.m[t] = o[t * B];
    p = v3(o[9 * B], o[10 * B], o[11 * B]);
}

__device__ __forceinline__ float joint_angle(const DevRobot &rb, const LinkF &f, const LinkI &i,
                                             const float *__restrict__ q, int64_t B, int64_t b) {
    return i.revolute ? f.mult * q[(int64_t)i.jidx * B + b] + f.offset : 0.0f;
}

// World pose of link k from q alone: the local transforms of its chain,
// each ancestor's pre-multiplied onto the product of the links below it
// (T_x o T = (R_x R, R_x p + p_x)), so no stored pose is read.
__device__ __forceinline__ void chain_pose(const DevRobot &rb, int k, const float *__restrict__ q, int64_t B,
                                           int64_t b, M3 &R, V3 &p) {
#pragma unroll
    for (int t = 0; t < 9; ++t) R.m[t] = (t % 4 == 0) ? 1.0f : 0.0f;
    p = v3(0.f, 0.f, 0.f);
    for (int x = k; x > 0;) {
        const LinkI li = ldu(rb.li + x);
        const LinkF lf = ldu(rb.lf + x);
        const M3 Rl = local_rotation(lf, li, joint_angle(rb, lf, li, q, B, b));
        p = mul(Rl, p) + v3(lf.fp[0], lf.fp[1], lf.fp[2]);
        R = matmul(Rl, R);
        x = li.parent;
    }
}

// Full FK for one state; writes poses (if given) and sphere centres (if
// given).  The running pose is carried while the next link is the current
// one's child; at a branch the parent's pose is re-read from the pose array,
// or recomposed along its chain when no pose array is given.
__device__ __forceinline__ void fk_state(const DevRobot &rb, int64_t B, int64_t b,
                                         const float *__restrict__ q, float *__restrict__ pose,
                                         float *__restrict__ sph) {
    M3 R;
#pragma unroll
    for (int t = 0; t < 9; ++t) R.m[t] = (t % 4 == 0) ? 1.0f : 0.0f;
    V3 p = v3(0.f, 0.f, 0.f);
    for (int k = 0; k < rb.L; ++k) {
        const LinkI li = ldu(rb.li + k);
        if (k > 0) {
            const LinkF lf = ldu(rb.lf + k);
            if (li.parent != k - 1) {
                if (pose) load_pose(pose, li.parent, B, b, R, p);
                else chain_pose(rb, li.parent, q, B, b, R, p);
            }
            M3 Rl = local_rotation(lf, li, joint_angle(rb, lf, li, q, B, b));
            p = mul(R, v3(lf.fp[0], lf.fp[1], lf.fp[2])) + p;
            R = matmul(R, Rl);
        }
        if (pose) store_pose(pose, k, B, b, R, p);
        if (sph) {
            for (int s = li.sph_first; s < li.sph_first + li.sph_count; ++s) {
                const float4 c4 = ldu(rb.sph + s);
                V3 c = mul(R, v3(c4.x, c4.y, c4.z)) + p;
                float *o = sph + (int64_t)s * 3 * B + b;
                o[0] = c.x;
                o[B] = c.y;
                o[2 * B] = c.z;
            }
        }
    }
}

// In the kernels below nb is the number of states and B the row length of
// every [k][B] array (the ABI's leading dimension ld >= nb).
__global__ void __launch_bounds__(256) k_fk(DevRobot rb, int64_t nb, int64_t B, const float *__restrict__ q,
                                            float *__restrict__ pose, float *__restrict__ sph) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    fk_state(rb, B, b, q, pose, sph);
}

// ws layout per state: [0, 12L) recomputed poses (when pose == nullptr),
// [12L, 18L) per-link accumulators (F, M) for links with a non-adjacent child.
__global__ void __launch_bounds__(256) k_fk_backward(DevRobot rb, int64_t nb, int64_t B, const float *__restrict__ q,
                                                     const float *__restrict__ pose_in,
                                                     const float *__restrict__ g_pose,
                                                     const float *__restrict__ g_sph,
                                                     float *__restrict__ g_q, float *__restrict__ ws) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int L = rb.L;
    const float *pose = pose_in;
    if (!pose) {
        fk_state(rb, B, b, q, ws, nullptr);
        pose = ws;
    }
    float *acc = ws + (int64_t)12 * L * B;
    if (!rb.simple_joints)
        for (int j = 0; j < rb.n; ++j) g_q[(int64_t)j * B + b] = 0.0f;
    for (int k = 1; k < L; ++k) {
        const LinkI li = ldu(rb.li + k);
        if (li.far_child) {  // zero the accumulator a non-adjacent child adds into
            float *a = acc + (int64_t)k * 6 * B + b;
#pragma unroll
            for (int t = 0; t < 6; ++t) a[t * B] = 0.0f;
        }
    }
    V3 cF = v3(0.f, 0.f, 0.f), cM = v3(0.f, 0.f, 0.f);  // carry from child k+1
    for (int k = L - 1; k >= 1; --k) {
        const LinkI li = ldu(rb.li + k);
        const LinkF lf = ldu(rb.lf + k);
        M3 R;
        V3 o;
        load_pose(pose, k, B, b, R, o);
        V3 F = cF, M = cM;
        if (li.far_child) {
            const float *a = acc + (int64_t)k * 6 * B + b;
            F += v3(a[0], a[B], a[2 * B]);
            M += v3(a[3 * B], a[4 * B], a[5 * B]);
        }
        if (g_sph) {
            for (int s = li.sph_first; s < li.sph_first + li.sph_count; ++s) {
                const float4 c4 = ldu(rb.sph + s);
                const float *g = g_sph + (int64_t)s * 3 * B + b;
                V3 gv = v3(g[0], g[B], g[2 * B]);
                V3 r = mul(R, v3(c4.x, c4.y, c4.z));
                F += gv;
                M += cross(r, gv);
            }
        }
        if (g_pose) {
            const float *g = g_pose + (int64_t)k * 12 * B + b;
            M3 G;
#pragma unroll
            for (int t = 0; t < 9; ++t) G.m[t] = g[t * B];
#pragma unroll
            for (int j = 0; j < 3; ++j) M += cross(col(R, j), col(G, j));
            F += v3(g[9 * B], g[10 * B], g[11 * B]);
        }
        if (li.revolute) {
            V3 sw = mul(R, v3(lf.axis[0], lf.axis[1], lf.axis[2]));
            float th = lf.mult * dot(sw, M);
            float *gq = g_q + (int64_t)li.jidx * B + b;
            if (rb.simple_joints) *gq = th;
            else *gq += th;
        }
        const int p = li.parent;
        cF = v3(0.f, 0.f, 0.f);
        cM = v3(0.f, 0.f, 0.f);
        if (p >= 1) {
            const float *op = pose + ((int64_t)p * 12 + 9) * B + b;
            V3 Mp = M + cross(o - v3(op[0], op[B], op[2 * B]), F);
            if (p == k - 1) {
                cF = F;
                cM = Mp;
            } else {
                float *a = acc + (int64_t)p * 6 * B + b;
                a[0] += F.x; a[B] += F.y; a[2 * B] += F.z;
                a[3 * B] += Mp.x; a[4 * B] += Mp.y; a[5 * B] += Mp.z;
            }
        }
    }
}

hipError_t launch_fk(const DevRobot &rb, int64_t B, int64_t ld, const float *q, float *pose, float *spheres,
                     hipStream_t s) {
    if (B == 0) return hipSuccess;
    dim3 grid((unsigned)((B + 255) / 256));
    hipLaunchKernelGGL(k_fk, grid, dim3(256), 0, s, rb, B, ld, q, pose, spheres);
    return hipGetLastError();
}

hipError_t launch_fk_backward(const DevRobot &rb, int64_t B, int64_t ld, const float *q, const float *pose,
                              const float *g_pose, const float *g_sph, float *g_q, float *ws,
                              hipStream_t s) {
    if (B == 0) return hipSuccess;
    dim3 grid((unsigned)((B + 255) / 256));
    hipLaunchKernelGGL(k_fk_backward, grid, dim3(256), 0, s, rb, B, ld, q, pose, g_pose, g_sph, g_q, ws);
    return hipGetLastError();
}

}  // namespace wb
