// Exact Euclidean distance transform of a site grid (cuRoboV2 Sec. 5,
// "Stage 2: Distance Propagation"): the nearest site of every voxel by
// three separable axis passes, the PBA+ decomposition of the paper, with
// Maurer's dominance test deciding the lower envelope of the distance
// parabolas along a line.  Integer arithmetic throughout, so the result is
// exact.
//
// Grid [nz][ny][nx], x fastest.  A site is stored packed as
// x | y << 10 | z << 20 (coordinates below 1024), NONE (-1) when there is
// none.  Five launches, fixed for a grid size (graph-capturable, no atomics):
//   1. along z, thread per (x, y): a forward flood keeps the last site seen,
//      a backward flood the next one; the closer wins -> A [nz][ny][nx];
//   2. along y, thread per (x, z): the lower envelope of the parabolas
//      (y - y')^2 + (z - z*)^2 of the column sites, built as a stack in place
//      in the line of A (entry k lands at position k <= the position being
//      read), with its size in kY;
//   3. along y, thread per (x, z, segment of SEG voxels): a binary search
//      finds the envelope entry that owns the segment's first voxel, then a
//      walk assigns the segment -> Bt [nz][nx][ny] (transposed, so the x pass
//      reads along its lines' contiguous axis);
//   4. along x, thread per (y, z): the envelope of (x - x')^2 + h, h the
//      squared y, z offsets of the plane's nearest site, in place in Bt, kX;
//   5. along x, thread per (y, z, segment): as 3 -> nearest site and
//      voxel_size * sqrt(d2) in [nz][ny][nx].
// Lanes run along a contiguous axis for every line read: x in passes 1-3,
// y in passes 4-5.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wb_internal.h"

namespace wb {
namespace {

constexpr int32_t EDT_NONE = -1;
constexpr int EDT_SEG = 32;      // voxels per thread in the assignment passes
constexpr int EDT_CHUNK = 8;     // loads issued ahead in the sequential passes

__device__ __forceinline__ int32_t pack(int x, int y, int z) { return x | (y << 10) | (z << 20); }
__device__ __forceinline__ int cx(int32_t c) { return c & 1023; }
__device__ __forceinline__ int cy(int32_t c) { return (c >> 10) & 1023; }
__device__ __forceinline__ int cz(int32_t c) { return c >> 20; }

// Position along the line and the squared offset across it, for a line of
// the y pass (fixed x, z) or of the x pass (fixed y, z).
template <int AX>
__device__ __forceinline__ int pos(int32_t c) { return AX == 1 ? cy(c) : cx(c); }
template <int AX>
__device__ __forceinline__ int height(int32_t c, int qy, int qz) {
    const int dz = qz - cz(c);
    if (AX == 1) return dz * dz;
    const int dy = qy - cy(c);
    return dy * dy + dz * dz;
}

// Maurer's test: with positions ua < ub < uc, b never attains the minimum of
// the three parabolas (t - u)^2 + h when the a/b crossing is not left of
// the b/c crossing.
__device__ __forceinline__ bool dominated(int ua, int ha, int ub, int hb, int uc, int hc) {
    const int64_t ab = (int64_t)(ub * ub + hb - ua * ua - ha) * (uc - ub);
    const int64_t bc = (int64_t)(uc * uc + hc - ub * ub - hb) * (ub - ua);
    return ab >= bc;
}

struct LineGeom {
    int64_t base, stride;   // element i of the line is at base + i * stride
    int n;                  // line length
    int qy, qz;             // fixed coordinates of the line (qy unused in the y pass)
};

template <int AX>
__device__ __forceinline__ LineGeom line_of(int64_t t, int nx, int ny, int nz) {
    LineGeom g;
    if (AX == 1) {   // line (x, z) of A, along y
        const int x = (int)(t % nx), z = (int)(t / nx);
        g.base = (int64_t)z * ny * nx + x;
        g.stride = nx;
        g.n = ny;
        g.qy = 0;
        g.qz = z;
    } else {         // line (y, z) of Bt, along x
        const int y = (int)(t % ny), z = (int)(t / ny);
        g.base = (int64_t)z * nx * ny + y;
        g.stride = ny;
        g.n = nx;
        g.qy = y;
        g.qz = z;
    }
    return g;
}

// ---- pass 1: nearest site along z
__global__ void __launch_bounds__(256) k_edt_z(const uint8_t *__restrict__ sites, int32_t *__restrict__ A, int nx,
                                               int ny, int nz) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)nx * ny) return;
    const int x = (int)(t % nx), y = (int)(t / nx);
    const int64_t plane = (int64_t)nx * ny;
    int last = EDT_NONE;
    for (int z0 = 0; z0 < nz; z0 += EDT_CHUNK) {
        uint8_t m[EDT_CHUNK];
#pragma unroll
        for (int j = 0; j < EDT_CHUNK; ++j) m[j] = z0 + j < nz ? sites[(z0 + j) * plane + t] : 0;
#pragma unroll
        for (int j = 0; j < EDT_CHUNK; ++j)
            if (z0 + j < nz) {
                if (m[j]) last = z0 + j;
                A[(z0 + j) * plane + t] = last;
            }
    }
    int next = EDT_NONE;
    for (int z1 = nz; z1 > 0; z1 -= EDT_CHUNK) {
        int32_t f[EDT_CHUNK];
#pragma unroll
        for (int j = 0; j < EDT_CHUNK; ++j) f[j] = z1 - 1 - j >= 0 ? A[(z1 - 1 - j) * plane + t] : EDT_NONE;
#pragma unroll
        for (int j = 0; j < EDT_CHUNK; ++j) {
            const int z = z1 - 1 - j;
            if (z < 0) continue;
            if (f[j] == z) next = z;
            const int prev = f[j];
            const int best = prev < 0 ? next : (next < 0 ? prev : (z - prev <= next - z ? prev : next));
            A[z * plane + t] = best < 0 ? EDT_NONE : pack(x, y, best);
        }
    }
}

// ---- passes 2 and 4: the lower envelope of a line, in place
template <int AX>
__global__ void __launch_bounds__(256) k_edt_envelope(int32_t *__restrict__ buf, int32_t *__restrict__ kcount,
                                                      int nx, int ny, int nz) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t lines = AX == 1 ? (int64_t)nx * nz : (int64_t)ny * nz;
    if (t >= lines) return;
    const LineGeom g = line_of<AX>(t, nx, ny, nz);
    int k = 0;
    // the two top entries of the stack: position and height
    int u1 = 0, h1 = 0, u2 = 0, h2 = 0;
    for (int i0 = 0; i0 < g.n; i0 += EDT_CHUNK) {
        int32_t c[EDT_CHUNK];
#pragma unroll
        for (int j = 0; j < EDT_CHUNK; ++j) c[j] = i0 + j < g.n ? buf[g.base + (i0 + j) * g.stride] : EDT_NONE;
#pragma unroll
        for (int j = 0; j < EDT_CHUNK; ++j) {
            if (c[j] < 0) continue;
            const int uc = pos<AX>(c[j]), hc = height<AX>(c[j], g.qy, g.qz);
            while (k >= 2 && dominated(u1, h1, u2, h2, uc, hc)) {
                --k;
                u2 = u1;
                h2 = h1;
                if (k >= 2) {
                    const int32_t e = buf[g.base + (int64_t)(k - 2) * g.stride];
                    u1 = pos<AX>(e);
                    h1 = height<AX>(e, g.qy, g.qz);
                }
            }
            buf[g.base + (int64_t)k * g.stride] = c[j];   // k <= i0 + j: that input is consumed
            ++k;
            u1 = u2;
            h1 = h2;
            u2 = uc;
            h2 = hc;
        }
    }
    kcount[t] = k;
}

// ---- passes 3 and 5: assign every voxel of a segment its envelope entry
template <int AX>
__global__ void __launch_bounds__(256) k_edt_assign(const int32_t *__restrict__ buf, const int32_t *__restrict__ kcount,
                                                    int32_t *__restrict__ out, float *__restrict__ dist,
                                                    float voxel_size, int nx, int ny, int nz) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int n = AX == 1 ? ny : nx;            // line length
    const int m = AX == 1 ? nx : ny;            // lines per z slice, consecutive in t
    const int nseg = (n + EDT_SEG - 1) / EDT_SEG;
    if (t >= (int64_t)m * nseg * nz) return;
    const int a = (int)(t % m);
    const int64_t r = t / m;
    const int seg = (int)(r % nseg), z = (int)(r / nseg);
    const int64_t line = (int64_t)z * m + a;
    const LineGeom g = line_of<AX>(line, nx, ny, nz);
    const int k = kcount[line];
    const int t0 = seg * EDT_SEG, t1 = min(t0 + EDT_SEG, n);
    // outputs: Bt [z][x][y] for the y pass, [z][y][x] for the x pass; both contiguous along t
    const int64_t obase = AX == 1 ? ((int64_t)z * nx + a) * ny : ((int64_t)z * ny + a) * nx;
    if (k == 0) {
        for (int s = t0; s < t1; ++s) {
            out[obase + s] = EDT_NONE;
            if (AX == 0 && dist) dist[obase + s] = INFINITY;
        }
        return;
    }
    auto entry = [&](int i) { return buf[g.base + (int64_t)i * g.stride]; };
    auto f = [&](int32_t c, int s) {
        const int d = s - pos<AX>(c);
        return d * d + height<AX>(c, g.qy, g.qz);
    };
    // first entry i with f(i + 1, t0) > f(i, t0): the owner of t0
    int lo = 0, hi = k - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (f(entry(mid + 1), t0) <= f(entry(mid), t0)) lo = mid + 1;
        else hi = mid;
    }
    int ptr = lo;
    int32_t cur = entry(ptr);
    int32_t nxt = ptr + 1 < k ? entry(ptr + 1) : cur;
    for (int s = t0; s < t1; ++s) {
        while (ptr + 1 < k && f(nxt, s) <= f(cur, s)) {
            ++ptr;
            cur = nxt;
            nxt = ptr + 1 < k ? entry(ptr + 1) : cur;
        }
        out[obase + s] = cur;
        if (AX == 0 && dist) dist[obase + s] = voxel_size * sqrtf((float)f(cur, s));
    }
}

}  // namespace

hipError_t launch_edt(int nx, int ny, int nz, const uint8_t *sites, float voxel_size, int32_t *nearest, float *dist,
                      int32_t *A, int32_t *Bt, int32_t *kY, int32_t *kX, hipStream_t s) {
    const int64_t cols = (int64_t)nx * ny, ly = (int64_t)nx * nz, lx = (int64_t)ny * nz;
    const int64_t ay = ly * ((ny + EDT_SEG - 1) / EDT_SEG), ax = lx * ((nx + EDT_SEG - 1) / EDT_SEG);
    auto blocks = [](int64_t n) { return dim3((unsigned)((n + 255) / 256)); };
    hipLaunchKernelGGL(k_edt_z, blocks(cols), dim3(256), 0, s, sites, A, nx, ny, nz);
    hipLaunchKernelGGL(k_edt_envelope<1>, blocks(ly), dim3(256), 0, s, A, kY, nx, ny, nz);
    hipLaunchKernelGGL(k_edt_assign<1>, blocks(ay), dim3(256), 0, s, A, kY, Bt, (float *)nullptr, voxel_size, nx, ny,
                       nz);
    hipLaunchKernelGGL(k_edt_envelope<0>, blocks(lx), dim3(256), 0, s, Bt, kX, nx, ny, nz);
    hipLaunchKernelGGL(k_edt_assign<0>, blocks(ax), dim3(256), 0, s, Bt, kX, nearest, dist, voxel_size, nx, ny, nz);
    return hipGetLastError();
}

}  // namespace wb
