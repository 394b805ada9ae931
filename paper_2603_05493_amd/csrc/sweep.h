// The self-collision pair sweep of one state by a group of G lanes of a
// wavefront (cuRoboV2 Sec. 6.2: the "map" over pair blocks and the "reduce"
// to the most penetrating pair), shared by the standalone and fused kernels.
//
// The checked pair set is a union of dense link blocks: every allowed link
// pair (a < b) contributes all spheres of a times all spheres of b.  The
// state's sphere centres sit in LDS, padded to NMAX slots per link (empty
// slots carry radius -1e30, so they can neither be the maximum nor count as
// a collision), plus one all-empty row for padding blocks.  A lane owns a
// whole link block: it loads the NMAX + NMAX centres into registers once and
// evaluates NMAX * NMAX pairs.
//
// Broad phase (exact): each link gets a bounding sphere (centroid C_a of its
// sphere centres, reach R_a = max |c - C_a| + r), and no pair of block (a, b)
// can penetrate more than bound = R_a + R_b - |C_a - C_b|.  A seed, the
// exact maximum of the block with the largest bound, is a lower bound of the
// state's maximum M.  Blocks with bound < min(seed, 0) - eps therefore hold
// no pair that is the maximum, ties it, or collides; they are skipped.  eps
// covers the FP32 rounding of both the bound and the pair penetrations (all
// computed from the same FP32 centres), so the result is identical to the
// full sweep.  Survivors are compacted into an LDS list per chunk of blocks
// so the pair loop stays lane-dense.
//
// Reduce: the pair count is a scalar ballot popcount per pair (one state per
// wavefront) or a per-lane counter summed over the group; the maximum is a
// per-lane running max per block plus a group shuffle reduction.  The lowest
// pair index attaining the maximum is recovered exactly: lanes holding the
// maximum re-evaluate the block where their running max was set with the
// same arithmetic and report the lowest (s, t) whose penetration equals it;
// if any lane saw two of its blocks tie the maximum, the group rescans every
// block instead.
#pragma once

#include <climits>
#include "spatial.h"

namespace wb {

constexpr int SWEEP_CHUNK = 256;   // blocks per compaction chunk (list entries per group)

// Penetration depth of one sphere pair; .w is the radius.  Written with
// explicit fused multiply-adds so every evaluation rounds identically.
__device__ __forceinline__ float pair_pen(float4 A, float4 Bv) {
    const float dx = A.x - Bv.x, dy = A.y - Bv.y, dz = A.z - Bv.z;
    const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    return (A.w + Bv.w) - __builtin_amdgcn_sqrtf(d2);
}

__device__ __forceinline__ float group_max(float v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, G));
    return v;
}
__device__ __forceinline__ int group_min(int v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, G));
    return v;
}
__device__ __forceinline__ unsigned group_sum(unsigned v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

__device__ __forceinline__ float block_bound(const float4 *Bd, int ab) {
    const float4 A = Bd[ab >> 16], Bv = Bd[ab & 0xffff];
    const float dx = A.x - Bv.x, dy = A.y - Bv.y, dz = A.z - Bv.z;
    return (A.w + Bv.w) - __builtin_amdgcn_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
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

// Bounding sphere of every link's (non-empty) sphere slots, into Bd[0..L).
template <int NMAX>
__device__ __forceinline__ void link_bounds(const DevRobot &rb, const float4 *P, float4 *Bd, int glane, int G) {
    for (int a = glane; a < rb.L; a += G) {
        float cx = 0.f, cy = 0.f, cz = 0.f, n = 0.f;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            const float4 s = P[a * NMAX + i];
            if (s.w > -1e29f) {
                cx += s.x;
                cy += s.y;
                cz += s.z;
                n += 1.f;
            }
        }
        float R = -1e30f;
        if (n > 0.f) {
            const float inv = 1.f / n;
            cx *= inv;
            cy *= inv;
            cz *= inv;
#pragma unroll
            for (int i = 0; i < NMAX; ++i) {
                const float4 s = P[a * NMAX + i];
                if (s.w > -1e29f) {
                    const float dx = s.x - cx, dy = s.y - cy, dz = s.z - cz;
                    R = fmaxf(R, __builtin_amdgcn_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz))) + s.w);
                }
            }
        }
        Bd[a] = make_float4(cx, cy, cz, R);
    }
}

// Sweep one state.  P: the state's (L+1)*NMAX sphere slots; Bd: its link
// bounding spheres (link_bounds); list: SWEEP_CHUNK ints of LDS scratch for
// this group.  Every lane of the group returns the maximum penetration M,
// the sphere key s*S + t of the lowest pair attaining it (INT_MAX if none)
// and the number of pairs with positive penetration.  FULL: G == 64.
template <int NMAX, bool FULL>
__device__ __forceinline__ void sweep_state(const DevRobot &rb, const float4 *P, const float4 *Bd, int *list,
                                            int glane, int G, int grp, float &M_out, int &key_out,
                                            unsigned &cnt_out) {
    const int nb = (rb.n_blocks + G - 1) / G * G;
    const uint64_t gmask = FULL ? ~0ull : ((1ull << G) - 1ull);
    const int gshift = FULL ? 0 : grp * G;
    // extent of the robot in this state, for the rounding margin
    float ext = 0.f;
    for (int a = glane; a < rb.L; a += G) {
        const float4 c = Bd[a];
        if (c.w > -1e29f) ext = fmaxf(ext, sqrtf(c.x * c.x + c.y * c.y + c.z * c.z) + c.w);
    }
    const float eps = 4e-6f * (1.f + group_max(ext, G));
    // seed: exact maximum of the block with the largest bound
    float bmax = -INFINITY;
    int bblk = INT_MAX;
    for (int base = 0; base < nb; base += G) {
        const int blk = base + glane;
        if (blk < rb.n_blocks) {
            const float bd = block_bound(Bd, rb.blocks[blk]);
            if (bd > bmax) {
                bmax = bd;
                bblk = blk;
            }
        }
    }
    const float gbmax = group_max(bmax, G);
    const int cand = group_min(bmax == gbmax ? bblk : INT_MAX, G);
    float seed = -INFINITY;
    if (cand != INT_MAX) {
        const int ab = rb.blocks[cand];
        const int a = ab >> 16, bb = ab & 0xffff;
        for (int j = glane; j < NMAX * NMAX; j += G) {
            const int i = j / NMAX, k = j - i * NMAX;
            seed = fmaxf(seed, pair_pen(P[a * NMAX + i], P[bb * NMAX + k]));
        }
    }
    const float theta = fminf(group_max(seed, G), 0.f) - eps;

    float best = -INFINITY;
    int best_blk = -1;
    bool tie = false;
    unsigned cnt = 0;
    for (int c0 = 0; c0 < nb; c0 += SWEEP_CHUNK) {
        const int cend = min(c0 + SWEEP_CHUNK, nb);
        int nl = 0;
        for (int base = c0; base < cend; base += G) {
            const int blk = base + glane;
            const bool surv = blk < rb.n_blocks && block_bound(Bd, rb.blocks[blk]) >= theta;
            const uint64_t m = (__ballot(surv) >> gshift) & gmask;
            if (surv) list[nl + __popcll(m & ((1ull << glane) - 1ull))] = blk;
            nl += __popcll(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int j = 0; j < nl; j += G) {
            const int idx = j + glane;
            const int blk = idx < nl ? list[idx] : -1;
            const int ab = blk >= 0 ? rb.blocks[blk] : ((rb.L << 16) | rb.L);
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
                for (int k = 0; k < NMAX; ++k) {
                    const float pen = pair_pen(A[i], Bv[k]);
                    m = fmaxf(m, pen);
                    if (FULL) cnt += (unsigned)__popcll(__ballot(pen > 0.0f));
                    else cnt += pen > 0.0f ? 1u : 0u;
                }
            if (m > best) {
                best = m;
                best_blk = blk;
                tie = false;
            } else if (m == best) {
                tie = true;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    const float M = group_max(best, G);
    int key = INT_MAX;
    const bool holder = best == M && M > -INFINITY && best_blk >= 0;
    const int rescan = group_min((holder && tie) ? 0 : 1, G) == 0;
    if (rescan) {
        for (int blk = glane; blk < nb; blk += G) key = min(key, block_min_key<NMAX>(rb, P, blk, M));
    } else if (holder) {
        key = block_min_key<NMAX>(rb, P, best_blk, M);
    }
    M_out = M;
    key_out = group_min(key, G);
    cnt_out = FULL ? cnt : group_sum(cnt, G);
}

// Pair index (lexicographic in (s, t)) of a sphere key s*S + t.
__device__ __forceinline__ int32_t pair_index(const DevRobot &rb, int key) {
    if (key == INT_MAX) return -1;
    const int s = key / rb.S, t = key - s * rb.S;
    const int a = rb.sph_link[s], bt = rb.sph_link[t];
    return rb.pair_off[s] + rb.pair_cnt[a * rb.L + bt] + (t - rb.li[bt].sph_first);
}

}  // namespace wb
