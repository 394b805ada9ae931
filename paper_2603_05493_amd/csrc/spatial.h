// FP32 device helpers: 3-vectors, rotations and Featherstone spatial algebra
// in the compact forms of cuRoboV2 Sec. 6.3 ("Compact spatial
// representations"): a transform is a rotation R plus a translation p, an
// inertia is (m, c, Ic), and every product is written out analytically.
#pragma once

#include <hip/hip_runtime.h>
#include "wb_internal.h"

namespace wb {

// A pointer read from memory as raw bits (as ldu below does) carries no
// address space, so accesses through it compile to flat instructions, which
// wait on the LDS and the vector-memory counters alike.  Re-deriving it from
// its integer value as a global pointer lets the compiler emit global ones.
template <typename T>
__device__ __forceinline__ T *as_global(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

// Uniform (same address in every lane) descriptor read through the scalar cache.
template <typename T>
__device__ __forceinline__ T ldu(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "uniform loads move whole dwords");
    typedef const __attribute__((address_space(4))) uint32_t *cptr;
    T out;
    cptr src = (cptr)(p);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return out;
}

struct V3 {
    float x, y, z;
};

__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ V3 operator-(V3 a) { return v3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ V3 &operator+=(V3 &a, V3 b) { a = a + b; return a; }
__device__ __forceinline__ V3 &operator-=(V3 &a, V3 b) { a = a - b; return a; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Row-major 3x3.
struct M3 {
    float m[9];
};
__device__ __forceinline__ V3 mul(const M3 &R, V3 v) {
    return v3(R.m[0] * v.x + R.m[1] * v.y + R.m[2] * v.z, R.m[3] * v.x + R.m[4] * v.y + R.m[5] * v.z,
              R.m[6] * v.x + R.m[7] * v.y + R.m[8] * v.z);
}
__device__ __forceinline__ V3 mulT(const M3 &R, V3 v) {
    return v3(R.m[0] * v.x + R.m[3] * v.y + R.m[6] * v.z, R.m[1] * v.x + R.m[4] * v.y + R.m[7] * v.z,
              R.m[2] * v.x + R.m[5] * v.y + R.m[8] * v.z);
}
__device__ __forceinline__ M3 matmul(const M3 &A, const M3 &B) {
    M3 C;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C.m[3 * i + j] = A.m[3 * i] * B.m[j] + A.m[3 * i + 1] * B.m[3 + j] + A.m[3 * i + 2] * B.m[6 + j];
    return C;
}
__device__ __forceinline__ V3 col(const M3 &R, int j) { return v3(R.m[j], R.m[3 + j], R.m[6 + j]); }

// Axis-angle rotation for a unit axis a: c I + s [a]x + (1 - c) a a^T.
__device__ __forceinline__ M3 axis_angle(V3 a, float s, float c) {
    float C = 1.0f - c;
    float xC = a.x * C, yC = a.y * C, zC = a.z * C;
    float xs = a.x * s, ys = a.y * s, zs = a.z * s;
    M3 R;
    R.m[0] = c + a.x * xC;  R.m[1] = a.x * yC - zs; R.m[2] = a.x * zC + ys;
    R.m[3] = a.y * xC + zs; R.m[4] = c + a.y * yC;  R.m[5] = a.y * zC - xs;
    R.m[6] = a.z * xC - ys; R.m[7] = a.z * yC + xs; R.m[8] = c + a.z * zC;
    return R;
}

// Local rotation of link k: fixed_R * Rot(axis, theta) (Rot = I for fixed links).
__device__ __forceinline__ M3 local_rotation(const LinkF &f, const LinkI &i, float theta) {
    M3 R;
    if (i.revolute) {
        float s, c;
        sincosf(theta, &s, &c);
        M3 J = axis_angle(v3(f.axis[0], f.axis[1], f.axis[2]), s, c);
        if (i.fR_identity) return J;
        M3 F;
#pragma unroll
        for (int t = 0; t < 9; ++t) F.m[t] = f.fR[t];
        return matmul(F, J);
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) R.m[t] = f.fR[t];
    return R;
}

// Spatial vector [angular; linear].
struct SV {
    V3 w, l;
};
__device__ __forceinline__ SV sv(V3 w, V3 l) { return SV{w, l}; }
__device__ __forceinline__ SV operator+(SV a, SV b) { return sv(a.w + b.w, a.l + b.l); }
__device__ __forceinline__ SV operator-(SV a, SV b) { return sv(a.w - b.w, a.l - b.l); }
__device__ __forceinline__ SV operator*(float s, SV a) { return sv(s * a.w, s * a.l); }
__device__ __forceinline__ SV &operator+=(SV &a, SV b) { a = a + b; return a; }
__device__ __forceinline__ float dot(SV a, SV b) { return dot(a.w, b.w) + dot(a.l, b.l); }

// Parent->child motion transform with E = R^T, r = p: [R^T w; R^T (v - p x w)].
__device__ __forceinline__ SV X_apply(const M3 &R, V3 p, SV u) {
    return sv(mulT(R, u.w), mulT(R, u.l - cross(p, u.w)));
}
// Its transpose, child->parent for forces: [R n + p x (R f); R f].
__device__ __forceinline__ SV XT_apply(const M3 &R, V3 p, SV f) {
    V3 Rf = mul(R, f.l);
    return sv(mul(R, f.w) + cross(p, Rf), Rf);
}
// Motion cross product v x u.
__device__ __forceinline__ SV crm(SV v, SV u) { return sv(cross(v.w, u.w), cross(v.w, u.l) + cross(v.l, u.w)); }
// Force cross product v x* f.
__device__ __forceinline__ SV crf(SV v, SV f) { return sv(cross(v.w, f.w) + cross(v.l, f.l), cross(v.w, f.l)); }

// Spatial inertia product from (m, c, Ic): [Ic w + c x h; h], h = m (v + w x c).
__device__ __forceinline__ SV I_apply(const LinkF &f, SV u) {
    V3 c = v3(f.com[0], f.com[1], f.com[2]);
    V3 h = f.mass * (u.l + cross(u.w, c));
    V3 Iw = v3(f.I[0] * u.w.x + f.I[3] * u.w.y + f.I[4] * u.w.z,
               f.I[3] * u.w.x + f.I[1] * u.w.y + f.I[5] * u.w.z,
               f.I[4] * u.w.x + f.I[5] * u.w.y + f.I[2] * u.w.z);
    return sv(Iw + cross(c, h), h);
}

// Strided [k][B] access helpers.
__device__ __forceinline__ float ld(const float *__restrict__ a, int64_t k, int64_t B, int64_t b) {
    return a[k * B + b];
}
__device__ __forceinline__ void st(float *__restrict__ a, int64_t k, int64_t B, int64_t b, float v) {
    a[k * B + b] = v;
}

}  // namespace wb
