// The self-collision pair sweep of one state by one wavefront (cuRoboV2
// Sec. 6.2, the "map" over pair blocks and the "reduce" to the most
// penetrating pair), shared by the standalone and the fused kernels.
//
// The checked pair set is a union of dense link blocks: every allowed link
// pair (a < b) contributes all spheres of a times all spheres of b.  The
// state's sphere centres sit in LDS, padded to NMAX slots per link (empty
// slots carry radius -1e30, so they can neither be the maximum nor count as
// a collision), plus one all-empty row that the block list is padded with to
// a multiple of 64.  Each lane owns whole link blocks: it loads the
// NMAX + NMAX centres of its block into registers once and evaluates
// NMAX * NMAX pairs, so the control flow of the sweep is uniform.
//
// Reduce: the pair count accumulates on the scalar unit from a ballot of
// pen > 0 per pair; the maximum is a per-lane running max per block plus a
// wave shuffle reduction.  The lowest pair index attaining the maximum is
// recovered exactly: each lane remembers the block where its running max was
// set and whether another of its blocks tied it; lanes holding the wave
// maximum re-evaluate that block (or, after a tie, all their blocks) with the
// same arithmetic and report the lowest (s, t) whose penetration equals it.
#pragma once

#include <climits>
#include "spatial.h"

namespace wb {

// Penetration depth of one sphere pair; .w is the radius.  Written with
// explicit fused multiply-adds so every evaluation rounds identically.
__device__ __forceinline__ float pair_pen(float4 A, float4 Bv) {
    const float dx = A.x - Bv.x, dy = A.y - Bv.y, dz = A.z - Bv.z;
    const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    return (A.w + Bv.w) - __builtin_amdgcn_sqrtf(d2);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

template <int NMAX>
__device__ __forceinline__ int block_min_key(const DevRobot &rb, const float4 *P, int blk, float M) {
    const int ab = rb.blocks[blk];
    const int a = ab >> 16, bb = ab & 0xffff;
    if (a >= rb.L) return INT_MAX;
    const int fa = rb.li[a].sph_first, fb = rb.li[bb].sph_first;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
        const float4 A = P[a * NMAX + i];
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
            if (pair_pen(A, P[bb * NMAX + j]) == M) return (fa + i) * rb.S + (fb + j);
    }
    return INT_MAX;
}


// Sweep one state's checked pairs.  P points at the state's padded sphere
// slots in LDS ((L+1)*NMAX float4, .w = radius).  Called by all 64 lanes of
// the wavefront; every lane returns the state's maximum penetration M, the
// sphere key s*S + t of the lowest pair attaining it (INT_MAX if none) and
// the count of pairs with positive penetration.
template <int NMAX>
__device__ __forceinline__ void sweep_state(const DevRobot &rb, const float4 *P, int lane, float &M_out,
                                            int &key_out, unsigned &cnt_out) {
    float best = -INFINITY;
    int best_blk = -1;
    bool tie = false;
    unsigned cnt = 0;
    for (int base = 0; base < rb.n_blocks_pad; base += 64) {
        const int blk = base + lane;
        const int ab = rb.blocks[blk];
        const int a = ab >> 16, bb = ab & 0xffff;
        float4 A[NMAX], Bv[NMAX];
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            A[i] = P[a * NMAX + i];
            Bv[i] = P[bb * NMAX + i];
        }
        float m = -INFINITY;
#pragma unroll
        for (int i = 0; i < NMAX; ++i)
#pragma unroll
            for (int j = 0; j < NMAX; ++j) {
                const float pen = pair_pen(A[i], Bv[j]);
                m = fmaxf(m, pen);
                cnt += (unsigned)__popcll(__ballot(pen > 0.0f));
            }
        if (m > best) {
            best = m;
            best_blk = blk;
            tie = false;
        } else if (m == best) {
            tie = true;
        }
    }
    const float M = wave_max(best);
    int key = INT_MAX;
    if (best == M && M > -INFINITY) {
        if (!tie) {
            key = block_min_key<NMAX>(rb, P, best_blk, M);
        } else {
            for (int blk = lane; blk < rb.n_blocks_pad; blk += 64)
                key = min(key, block_min_key<NMAX>(rb, P, blk, M));
        }
    }
    M_out = M;
    key_out = wave_min(key);
    cnt_out = cnt;
}

// The same sweep by a group of G < 64 lanes (64/G states per wavefront).
// Blocks are dealt to the group's lanes; the pair count is a per-lane
// counter summed over the group at the end.
template <int NMAX>
__device__ __forceinline__ void sweep_group(const DevRobot &rb, const float4 *P, int glane, int G, float &M_out,
                                            int &key_out, unsigned &cnt_out) {
    float best = -INFINITY;
    int best_blk = -1;
    bool tie = false;
    unsigned cnt = 0;
    const int nb = (rb.n_blocks + G - 1) / G * G;
    for (int base = 0; base < nb; base += G) {
        const int blk = base + glane;
        const int ab = rb.blocks[blk];
        const int a = ab >> 16, bb = ab & 0xffff;
        float4 A[NMAX], Bv[NMAX];
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            A[i] = P[a * NMAX + i];
            Bv[i] = P[bb * NMAX + i];
        }
        float m = -INFINITY;
#pragma unroll
        for (int i = 0; i < NMAX; ++i)
#pragma unroll
            for (int j = 0; j < NMAX; ++j) {
                const float pen = pair_pen(A[i], Bv[j]);
                m = fmaxf(m, pen);
                cnt += pen > 0.0f ? 1u : 0u;
            }
        if (m > best) {
            best = m;
            best_blk = blk;
            tie = false;
        } else if (m == best) {
            tie = true;
        }
    }
    float M = best;
    for (int o = G >> 1; o > 0; o >>= 1) M = fmaxf(M, __shfl_xor(M, o, G));
    int key = INT_MAX;
    if (best == M && M > -INFINITY) {
        if (!tie) {
            key = block_min_key<NMAX>(rb, P, best_blk, M);
        } else {
            for (int blk = glane; blk < nb; blk += G) key = min(key, block_min_key<NMAX>(rb, P, blk, M));
        }
    }
    for (int o = G >> 1; o > 0; o >>= 1) {
        key = min(key, __shfl_xor(key, o, G));
        cnt += __shfl_xor(cnt, o, G);
    }
    M_out = M;
    key_out = key;
    cnt_out = cnt;
}

// Pair index (lexicographic in (s, t)) of a sphere key s*S + t.
__device__ __forceinline__ int32_t pair_index(const DevRobot &rb, int key) {
    if (key == INT_MAX) return -1;
    const int s = key / rb.S, t = key - s * rb.S;
    const int a = rb.sph_link[s], bt = rb.sph_link[t];
    return rb.pair_off[s] + rb.pair_cnt[a * rb.L + bt] + (t - rb.li[bt].sph_first);
}

}  // namespace wb
