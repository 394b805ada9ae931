// Exact Euclidean distance transform of a site grid (cuRoboV2 Sec. 5,
// "Stage 2: Distance Propagation"): the nearest site of every voxel by
// three separable axis passes, the PBA+ decomposition of the paper, with
// Maurer's dominance test deciding the lower envelope of the distance
// parabolas along a line.  Integer arithmetic throughout, so the result is
// exact.
//
// Grid [nz][ny][nx], x fastest.  A site is stored packed as
// x | y << 10 | z << 20 (coordinates below 1024), NONE (-1) when there is
// none.  The axes are taken in the order x, y, z so that every pass keeps
// its lanes along x, the contiguous axis: loads and stores are coalesced
// and no transpose is needed.  Three launches, fixed for a grid size
// (graph-capturable, no atomics):
//   1. along x, one wavefront per row (y, z): the nearest site of the row,
//      from a forward and a backward flood, each an inclusive max-scan over
//      the wavefront (DPP; the backward one toward lower lanes) carried
//      across chunks -> A (rows of a multiple of 4 voxels: 4 voxels per
//      lane, in registers, one read and one write of the row);
//   2. along y, a workgroup per tile of lines (x0 .. x0+TL-1, z) held in
//      LDS: the lower envelope of the parabolas (y - y')^2 + (x - x*)^2 of
//      the row sites, built band by band and merged at the band junctions
//      as in PBA+, then every voxel assigned its envelope entry -> B;
//   3. along z, the same on tiles (x0 .. x0+TL-1, y) with the parabolas
//      (z - z')^2 + (x - x*)^2 + (y - y*)^2 -> the nearest site and
//      voxel_size * sqrt(d2).
// Each pass reads its input grid once and writes its output once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "edt.h"

namespace wb {
namespace {

constexpr int32_t EDT_NONE = -1;
constexpr int EDT_BIG = 1 << 20; // above any coordinate

__device__ __forceinline__ int32_t pack(int x, int y, int z) { return x | (y << 10) | (z << 20); }
__device__ __forceinline__ int cx(int32_t c) { return c & 1023; }
__device__ __forceinline__ int cy(int32_t c) { return (c >> 10) & 1023; }
__device__ __forceinline__ int cz(int32_t c) { return c >> 20; }

// Inclusive max-scan over the 64 lanes of a wavefront, for values >= 0 (0 is
// the identity): row_shr 1, 2, 4, 8 inside each row of 16, then row_bcast15
// and row_bcast31 carry the row maxima upward.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_up(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ int wave_max_scan(int v) {
    v = max(v, dpp_up<0x111>(v));
    v = max(v, dpp_up<0x112>(v));
    v = max(v, dpp_up<0x114>(v));
    v = max(v, dpp_up<0x118>(v));
    v = max(v, dpp_up<0x142, 0xa>(v));
    v = max(v, dpp_up<0x143, 0xc>(v));
    return v;
}
// Inclusive max-scan toward lower lanes (lane i: max over lanes >= i):
// row_shl 1, 2, 4, 8 inside each row, then the maxima of the rows above,
// read from the first lane of each row.
__device__ __forceinline__ int wave_max_suffix_scan(int v, int lane) {
    v = max(v, dpp_up<0x101>(v));
    v = max(v, dpp_up<0x102>(v));
    v = max(v, dpp_up<0x104>(v));
    v = max(v, dpp_up<0x108>(v));
    const int r1 = __builtin_amdgcn_readlane(v, 16), r2 = __builtin_amdgcn_readlane(v, 32),
              r3 = __builtin_amdgcn_readlane(v, 48);
    const int row = lane >> 4;
    if (row < 3) v = max(v, r3);
    if (row < 2) v = max(v, r2);
    if (row < 1) v = max(v, r1);
    return v;
}

// ---- pass 1: nearest site along x, one wavefront per row (y, z)
__global__ void __launch_bounds__(256) k_edt_x(const uint8_t *__restrict__ sites, int32_t *__restrict__ A, int nx,
                                               int ny, int nz) {
    const int64_t w = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= (int64_t)ny * nz) return;   // uniform over the wavefront
    const int y = (int)(w % ny), z = (int)(w / ny);
    const int64_t base = w * nx;
    // forward: 1 + the last site at or before x (0: none)
    int carry = 0;
    for (int x0 = 0; x0 < nx; x0 += 64) {
        const int x = x0 + lane;
        const int s = x < nx && sites[base + x] ? x + 1 : 0;
        const int v = max(wave_max_scan(s), carry);
        carry = __builtin_amdgcn_readlane(v, 63);
        if (x < nx) A[base + x] = v - 1;
    }
    // backward: BIG - the next site at or after x (0: none); each lane reads
    // back only what it stored itself
    carry = 0;
    for (int x0 = ((nx - 1) >> 6) << 6; x0 >= 0; x0 -= 64) {
        const int x = x0 + lane;
        const int s = x < nx && sites[base + x] ? EDT_BIG - x : 0;
        const int v = max(wave_max_suffix_scan(s, lane), carry);
        carry = __builtin_amdgcn_readlane(v, 0);
        if (x < nx) {
            const int prev = A[base + x], next = v > 0 ? EDT_BIG - v : EDT_NONE;
            const int best = prev < 0 ? next : (next < 0 ? prev : (x - prev <= next - x ? prev : next));
            A[base + x] = best < 0 ? EDT_NONE : pack(best, y, z);
        }
    }
}

// Pass 1 for rows whose length is a multiple of 4 (up to 1024): lane i of
// the row's wavefront holds voxels 4i .. 4i + 3 of each 256-voxel chunk in
// registers, read as one 4-byte word per chunk.  Both floods run on those
// registers (a 4-voxel scan inside the lane, a wavefront scan of the lane
// totals, a carry across chunks), and each chunk's result leaves as one
// 16-byte store per lane: the site row is read once and A written once.
template <int NC>
__global__ void __launch_bounds__(256) k_edt_x4(const uint8_t *__restrict__ sites, int32_t *__restrict__ A, int nx,
                                                int ny, int nz) {
    const int64_t w = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= (int64_t)ny * nz) return;   // uniform over the wavefront
    const int y = (int)(w % ny), z = (int)(w / ny);
    const int n4 = nx >> 2;
    const uint32_t *row = reinterpret_cast<const uint32_t *>(sites + w * nx);
    int4 *out = reinterpret_cast<int4 *>(A + w * nx);
    uint32_t sb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int i = c * 64 + lane;
        sb[c] = i < n4 ? row[i] : 0u;
    }
    // forward: 1 + the last site at or before x (0: none)
    int prev[NC][4];
    int carry = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int x0 = (c * 64 + lane) * 4;
        int v = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v = (sb[c] >> (8 * j)) & 0xffu ? x0 + j + 1 : v;
            prev[c][j] = v;
        }
        const int incl = wave_max_scan(v);
        const int up = __shfl_up(incl, 1, 64);
        const int excl = max(lane > 0 ? up : 0, carry);
#pragma unroll
        for (int j = 0; j < 4; ++j) prev[c][j] = max(prev[c][j], excl);
        carry = max(carry, __builtin_amdgcn_readlane(incl, 63));
    }
    // backward: BIG - the next site at or after x (0: none), then the nearer
    carry = 0;
#pragma unroll
    for (int c = NC - 1; c >= 0; --c) {
        const int x0 = (c * 64 + lane) * 4;
        int nxt[4];
        int v = 0;
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            v = (sb[c] >> (8 * j)) & 0xffu ? EDT_BIG - (x0 + j) : v;
            nxt[j] = v;
        }
        const int incl = wave_max_suffix_scan(v, lane);
        const int down = __shfl_down(incl, 1, 64);
        const int excl = max(lane < 63 ? down : 0, carry);
        carry = max(carry, __builtin_amdgcn_readlane(incl, 0));
        int r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = x0 + j;
            const int pv = prev[c][j] - 1;
            const int nv = max(nxt[j], excl);
            const int nx_ = nv > 0 ? EDT_BIG - nv : EDT_NONE;
            const int best = pv < 0 ? nx_ : (nx_ < 0 ? pv : (x - pv <= nx_ - x ? pv : nx_));
            r[j] = best < 0 ? EDT_NONE : pack(best, y, z);
        }
        const int i = c * 64 + lane;
        if (i < n4) out[i] = make_int4(r[0], r[1], r[2], r[3]);
    }
}

// Positions along the line and squared cross offsets: AX == 1 runs along y
// (a line (x, z); the candidate is the row's nearest site (x*, y', z)),
// AX == 2 along z (a line (x, y); the candidate is the plane's nearest site
// (x*, y*, z')).
template <int AX>
__device__ __forceinline__ int pos(int32_t c) { return AX == 1 ? cy(c) : cz(c); }
template <int AX>
__device__ __forceinline__ int height(int32_t c, int qx, int qy) {
    const int dx = qx - cx(c);
    if (AX == 1) return dx * dx;
    const int dy = qy - cy(c);
    return dx * dx + dy * dy;
}

// A candidate at line position u with squared cross offset h is kept as
// (u, g = u^2 + h).  Maurer's test: with positions ua < ub < uc, b never
// attains the minimum of the three parabolas (t - u)^2 + h when the a/b
// crossing is not left of the b/c crossing.
__device__ __forceinline__ bool dominated(int ua, int ga, int ub, int gb, int uc, int gc) {
    return (int64_t)(gb - ga) * (uc - ub) >= (int64_t)(gc - gb) * (ub - ua);
}

// ---- passes 2 and 3: one workgroup per tile of TL lines (consecutive x)
// at a fixed z (AX == 1) or y (AX == 2), the tile resident in LDS as
// ent[p * TL + l] (position p, line l).  Phases, after PBA+'s banding:
//   bands:  thread (l, b) stacks the envelope of band b of line l in place
//           from the band's first position (256 / TL bands per line);
//   trim:   thread (l, b) merges the envelopes of bands b - 1 and b alone,
//           then of what is left of bands b - 2 and b.  An entry off such a
//           pair's envelope is off the line's envelope too, so the trimmed
//           prefix of band b and suffix of the other band go; every
//           junction of a round is trimmed at once;
//   merge:  thread l merges the trimmed bands left to right.  Only the
//           junctions change, so each band keeps a range [lo, hi) of its
//           stack: popping the envelope's last entry shortens its band's
//           range, dropping a band's first entry raises lo; nothing moves;
//   pack:   thread (l, b) moves band b's surviving range down, so the
//           line's envelope ends up packed at positions [0, K);
//   assign: thread (l, s) takes segment s of line l: a binary search finds
//           the envelope entry owning the segment's first voxel, a walk the
//           rest, and the segment is written to the next pass's grid (and
//           the distances after the last pass).
template <int AX, int TL>
__global__ void __launch_bounds__(256) k_edt_tile(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                  float *__restrict__ dist, float voxel_size, int nx, int ny,
                                                  int nz) {
    extern __shared__ int32_t ent[];
    constexpr int NB = 256 / TL;   // bands (and assignment segments) per line
    __shared__ int32_t bcnt[256], blo[256], bhi[256], boff[256], ksz[TL];
    const int n = AX == 1 ? ny : nz;
    const int ntx = (nx + TL - 1) / TL;
    const int x0 = (int)(blockIdx.x % ntx) * TL;
    const int o = (int)(blockIdx.x / ntx);   // z for AX == 1, y for AX == 2
    // element p of line x: AX == 1 (x, p, o), AX == 2 (x, o, p)
    auto gidx = [&](int p, int x) -> uint32_t {
        return AX == 1 ? ((uint32_t)o * ny + p) * nx + x : ((uint32_t)p * ny + o) * nx + x;
    };
    // the tile into LDS, eight loads in flight per thread
    for (int i0 = threadIdx.x; i0 < n * TL; i0 += 256 * 8) {
        int32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = i0 + 256 * j;
            const int p = i / TL, x = x0 + (i - p * TL);
            v[j] = i < n * TL && x < nx ? in[gidx(p, x)] : EDT_NONE;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (i0 + 256 * j < n * TL) ent[i0 + 256 * j] = v[j];
    }
    __syncthreads();
    const int l = threadIdx.x % TL, sidx = threadIdx.x / TL;
    const int qx = x0 + l, qy = o;
    const int bw = (n + NB - 1) / NB;
    // ---- bands
    {
        const int p0 = sidx * bw, p1 = min(p0 + bw, n);
        int k = 0, u1 = 0, g1 = 0, u2 = 0, g2 = 0;
        for (int p = p0; p < p1; ++p) {
            const int32_t c = ent[p * TL + l];
            if (c < 0) continue;
            const int gc = p * p + height<AX>(c, qx, qy);   // a candidate sits at its own position
            while (k >= 2 && dominated(u2, g2, u1, g1, p, gc)) {
                --k;
                u1 = u2;
                g1 = g2;
                if (k >= 2) {
                    const int32_t e = ent[(p0 + k - 2) * TL + l];
                    u2 = pos<AX>(e);
                    g2 = u2 * u2 + height<AX>(e, qx, qy);
                }
            }
            ent[(p0 + k) * TL + l] = c;   // p0 + k <= p: that input is consumed
            ++k;
            u2 = u1;
            g2 = g1;
            u1 = p;
            g1 = gc;
        }
        bcnt[sidx * TL + l] = k;
    }
    __syncthreads();
    auto ug = [&](int b, int i, int &u, int &gg) {   // entry i of band b's stack
        const int32_t c = ent[(b * bw + i) * TL + l];
        u = pos<AX>(c);
        gg = u * u + height<AX>(c, qx, qy);
    };
    // Trim the junction of band ba's range [la, ha) and band bb's range
    // [lb, hb) (ba < bb) from those two ranges alone: the new end of ba's
    // range and the new start of bb's.
    auto trim = [&](int ba, int la, int ha, int bb, int lb, int hb, int &nha, int &nlb) {
        int lo = lb, hi = ha;
        if (ha > la && hb > lb) {
            int u1, g1, u2 = 0, g2 = 0;   // last and second-to-last kept entries of band ba
            ug(ba, hi - 1, u1, g1);
            if (hi - la >= 2) ug(ba, hi - 2, u2, g2);
            while (lo < hb) {
                int uc, gc;
                ug(bb, lo, uc, gc);
                while (hi - la >= 2 && dominated(u2, g2, u1, g1, uc, gc)) {
                    --hi;
                    u1 = u2;
                    g1 = g2;
                    if (hi - la >= 2) ug(ba, hi - 2, u2, g2);
                }
                if (lo + 1 < hb) {
                    int un, gn;
                    ug(bb, lo + 1, un, gn);
                    if (dominated(u1, g1, uc, gc, un, gn)) {
                        ++lo;
                        continue;
                    }
                }
                break;
            }
        }
        nha = hi;
        nlb = lo;
    };
    // ---- trim, round 1: bands b - 1 and b, from the two stacks alone
    {
        const int b = sidx;
        int hi = b > 0 ? bcnt[(b - 1) * TL + l] : 0, lo = 0;
        const int cb = bcnt[b * TL + l];
        if (b > 0) trim(b - 1, 0, hi, b, 0, cb, hi, lo);
        blo[b * TL + l] = lo;
        if (b > 0) bhi[(b - 1) * TL + l] = hi;
        if (b == NB - 1) bhi[b * TL + l] = cb;
    }
    __syncthreads();
    // ---- trim, round 2: bands b - 2 and b, from their trimmed ranges (each
    // range end has one writer; every thread reads its ranges first)
    {
        const int b = sidx;
        int la = 0, ha = 0, lb = 0, hb = 0;
        if (b >= 2) {
            la = blo[(b - 2) * TL + l];
            ha = bhi[(b - 2) * TL + l];
            lb = blo[b * TL + l];
            hb = bhi[b * TL + l];
        }
        __syncthreads();
        if (b >= 2) {
            int nha, nlb;
            trim(b - 2, la, ha, b, lb, hb, nha, nlb);
            bhi[(b - 2) * TL + l] = nha;
            blo[b * TL + l] = nlb;
        }
    }
    __syncthreads();
    // ---- merge: the junctions of the trimmed ranges only
    if (threadIdx.x < TL) {
        // the envelope's last (b1, i1) and second-to-last (b2, i2) entries
        int K = 0, b1 = 0, i1 = 0, u1 = 0, g1 = 0, b2 = 0, i2 = 0, u2 = 0, g2 = 0;
        for (int b = 0; b < NB; ++b) {
            int lo = blo[b * TL + l];
            const int cb = max(bhi[b * TL + l], lo);
            while (lo < cb) {
                int uc, gc;
                ug(b, lo, uc, gc);
                while (K >= 2 && dominated(u2, g2, u1, g1, uc, gc)) {
                    bhi[b1 * TL + l] = i1;   // the last entry of band b1's range goes
                    --K;
                    b1 = b2;
                    i1 = i2;
                    u1 = u2;
                    g1 = g2;
                    if (K >= 2) {   // the entry before (b1, i1), in b1 or the last non-empty band before it
                        if (i1 > blo[b1 * TL + l]) {
                            b2 = b1;
                            i2 = i1 - 1;
                        } else {
                            int bb = b1 - 1;
                            while (blo[bb * TL + l] >= bhi[bb * TL + l]) --bb;
                            b2 = bb;
                            i2 = bhi[bb * TL + l] - 1;
                        }
                        ug(b2, i2, u2, g2);
                    }
                }
                if (K >= 1 && lo + 1 < cb) {
                    int un, gn;
                    ug(b, lo + 1, un, gn);
                    if (dominated(u1, g1, uc, gc, un, gn)) {
                        ++lo;
                        continue;
                    }
                }
                break;
            }
            blo[b * TL + l] = lo;
            bhi[b * TL + l] = cb;
            const int m = cb - lo;
            if (m >= 2) {
                b2 = b;
                i2 = cb - 2;
                ug(b, i2, u2, g2);
                b1 = b;
                i1 = cb - 1;
                ug(b, i1, u1, g1);
            } else if (m == 1) {
                b2 = b1;
                i2 = i1;
                u2 = u1;
                g2 = g1;
                b1 = b;
                i1 = lo;
                ug(b, lo, u1, g1);
            }
            K += m;
        }
        int off = 0;
        for (int b = 0; b < NB; ++b) {
            boff[b * TL + l] = off;
            off += max(bhi[b * TL + l] - blo[b * TL + l], 0);
        }
        ksz[l] = off;
    }
    __syncthreads();
    // ---- pack: thread (l, b) moves band b's range to its place in the
    // packed envelope [0, K) through registers (a range holds at most
    // bw <= 32 entries), so no thread overwrites a range still being read.
    {
        const int lo = blo[sidx * TL + l], cnt = bhi[sidx * TL + l] - lo, dst = boff[sidx * TL + l];
        const int src = sidx * bw + lo;
        int32_t v[32];
#pragma unroll
        for (int j = 0; j < 32; ++j)
            if (j < cnt) v[j] = ent[(src + j) * TL + l];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 32; ++j)
            if (j < cnt) ent[(dst + j) * TL + l] = v[j];
    }
    __syncthreads();
    // ---- assign
    const int x = x0 + l;
    if (x >= nx) return;
    const int K = ksz[l];
    const int t0 = sidx * bw, t1 = min(t0 + bw, n);
    if (t0 >= t1) return;
    if (K == 0) {
        for (int s = t0; s < t1; ++s) {
            out[gidx(s, x)] = EDT_NONE;
            if (dist) dist[gidx(s, x)] = INFINITY;
        }
        return;
    }
    auto entry = [&](int i) { return ent[i * TL + l]; };
    auto f = [&](int32_t c, int s) {
        const int d = s - pos<AX>(c);
        return d * d + height<AX>(c, qx, qy);
    };
    int lo = 0, hi = K - 1;   // the first entry i with f(i + 1, t0) > f(i, t0) owns t0
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (f(entry(mid + 1), t0) <= f(entry(mid), t0)) lo = mid + 1;
        else hi = mid;
    }
    int ptr = lo;
    int32_t cur = entry(ptr);
    int32_t nxt = ptr + 1 < K ? entry(ptr + 1) : cur;
    for (int s = t0; s < t1; ++s) {
        while (ptr + 1 < K && f(nxt, s) <= f(cur, s)) {
            ++ptr;
            cur = nxt;
            nxt = ptr + 1 < K ? entry(ptr + 1) : cur;
        }
        out[gidx(s, x)] = cur;
        if (dist) dist[gidx(s, x)] = voxel_size * sqrtf((float)f(cur, s));
    }
}

// Tiles of TL lines with TL * n * 4 bytes of LDS at most 32 KB: 32 lines
// up to n = 256, 16 up to 512, 8 up to 1024.
template <int AX>
bool tile_pass(const int32_t *in, int32_t *out, float *dist, float voxel_size, int nx, int ny, int nz, hipStream_t s) {
    const int n = AX == 1 ? ny : nz, o_n = AX == 1 ? nz : ny;
    const int tl = n <= 256 ? 32 : (n <= 512 ? 16 : 8);
    const dim3 grid((unsigned)(((nx + tl - 1) / tl) * (int64_t)o_n));
    const size_t lds = (size_t)n * tl * 4;
    switch (tl) {
        case 32: hipLaunchKernelGGL((k_edt_tile<AX, 32>), grid, dim3(256), lds, s, in, out, dist, voxel_size, nx, ny, nz); break;
        case 16: hipLaunchKernelGGL((k_edt_tile<AX, 16>), grid, dim3(256), lds, s, in, out, dist, voxel_size, nx, ny, nz); break;
        case 8: hipLaunchKernelGGL((k_edt_tile<AX, 8>), grid, dim3(256), lds, s, in, out, dist, voxel_size, nx, ny, nz); break;
        default: return false;
    }
    return true;
}

}  // namespace

hipError_t launch_edt(int nx, int ny, int nz, const uint8_t *sites, float voxel_size, int32_t *nearest, float *dist,
                      int32_t *A, int32_t *B, hipStream_t s) {
    const int64_t rows = (int64_t)ny * nz;
    const dim3 xgrid((unsigned)((rows * 64 + 255) / 256));
    // the 4-voxel form needs rows of whole 4-byte words and 16-byte aligned rows of A
    if (nx % 4 != 0 || reinterpret_cast<uintptr_t>(sites) % 4 != 0 || reinterpret_cast<uintptr_t>(A) % 16 != 0)
        hipLaunchKernelGGL(k_edt_x, xgrid, dim3(256), 0, s, sites, A, nx, ny, nz);
    else if (nx <= 256)
        hipLaunchKernelGGL(k_edt_x4<1>, xgrid, dim3(256), 0, s, sites, A, nx, ny, nz);
    else if (nx <= 512)
        hipLaunchKernelGGL(k_edt_x4<2>, xgrid, dim3(256), 0, s, sites, A, nx, ny, nz);
    else if (nx <= 768)
        hipLaunchKernelGGL(k_edt_x4<3>, xgrid, dim3(256), 0, s, sites, A, nx, ny, nz);
    else
        hipLaunchKernelGGL(k_edt_x4<4>, xgrid, dim3(256), 0, s, sites, A, nx, ny, nz);
    if (!tile_pass<1>(A, B, nullptr, voxel_size, nx, ny, nz, s)) return hipErrorInvalidValue;
    if (!tile_pass<2>(B, nearest, dist, voxel_size, nx, ny, nz, s)) return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace wb
