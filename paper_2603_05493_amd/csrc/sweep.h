// The self-collision pair sweep of one state by a group of G lanes of a
// wavefront (cuRoboV2 Sec. 6.2: the "map" over pair blocks and the "reduce"
// to the most penetrating pair), shared by the standalone and fused kernels.
//
// The checked pair set is a union of dense link blocks: every allowed link
// pair (a < b) contributes all spheres of a times all spheres of b.  The
// state's sphere centres sit in LDS, padded to NMAX slots per link (empty
// slots carry radius -1e30, so they can neither be the maximum nor count as
// a collision), plus one all-empty row for padding.
//
// Broad phase (exact): each link gets a bounding sphere (centroid C_a of its
// sphere centres, reach R_a = max |c - C_a| + r), and no pair of block (a, b)
// can penetrate more than bound = R_a + R_b - |C_a - C_b|.  eps covers the
// FP32 rounding of both the bound and the pair penetrations (all computed
// from the same FP32 centres), so a block whose computed bound is below t -
// eps holds no pair whose computed penetration reaches t.
//   Pass 1 sweeps the blocks that may reach -eps, tested without a square
//   root as |C_a - C_b|^2 <= (R_a + R_b + eps)^2.  If their maximum M0 is
//   >= 0, every skipped pair penetrates less than 0 <= M0: none is the
//   maximum, ties it, or collides, and the result is that of the full sweep.
//   Otherwise (no collision) a lower bound of M -- M0, or the exact maximum
//   of the block with the largest bound when pass 1 found nothing -- sets
//   t1, and pass 2 sweeps the blocks that pass 1 skipped and whose bound is
//   >= t1 - eps (the two passes partition the blocks exactly).
// The surviving link pairs of each pass are compacted into the group's LDS
// list (ballot + popcount), and the pair loop runs over rows -- (link pair,
// sphere slot of the first link) against the NMAX slots of the second link
// -- so that the lanes stay dense whatever the number of survivors.
// Row test (the same broad phase one level down, in the per-group sweeps):
// no pair of a row penetrates more than r_A + R_b - |c_A - C_b|, sphere A of
// the first link against the second link's bounding sphere, so a row is
// evaluated only where that bound may reach the pass's threshold.  Passing
// rows are queued in a 128-entry LDS ring per group (ballot + popcount) and
// evaluated G at a time, so the lanes stay dense.  Pass 2 then takes every
// block whose bound reaches t1 - eps and, in it, the rows pass 1 did not
// evaluate whose row bound reaches t1 - eps: the rows of the two passes
// partition the rows of the table exactly, with the same eps argument.  Robots
// with more blocks than the list holds are swept in chunks.  The block
// table is read from LDS where the caller has staged it; it is padded to a
// multiple of 128 entries with the empty pair (L, L), whose bounding sphere
// Bd[L] has radius -1e30, so the pass-1 loop needs no range tests.  Table and
// list entries are link pairs packed as (a << SH) | b in an entry type E:
// 32-bit with SH = 16, or 16-bit with SH = 8 for robots of at most 255 links.
//
// Reduce: the pair count is a scalar ballot popcount per pair (one state per
// wavefront) or a per-lane counter summed over the group; the maximum is a
// per-lane running max plus a group reduction.  The lowest pair index
// attaining the maximum is recovered exactly: lanes holding the maximum
// re-evaluate the row where their running max was set with the same
// arithmetic and report the lowest (s, t) whose penetration equals it; if
// any lane saw two of its rows tie the maximum, the group rescans every
// block instead.
#pragma once

#include <climits>
#include "lanes.h"
#include "spatial.h"

namespace wb {

// Penetration depth of one sphere pair; .w is the radius.  Written with
// explicit fused multiply-adds so every evaluation rounds identically.
__device__ __forceinline__ float pair_pen(float4 A, float4 Bv) {
    const float dx = A.x - Bv.x, dy = A.y - Bv.y, dz = A.z - Bv.z;
    const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    return (A.w + Bv.w) - __builtin_amdgcn_sqrtf(d2);
}

template <typename E>
struct PairCode {
    static constexpr int SH = sizeof(E) == 2 ? 8 : 16;
    static __device__ __forceinline__ int a(int ab) { return ab >> SH; }
    static __device__ __forceinline__ int b(int ab) { return ab & ((1 << SH) - 1); }
    static __device__ __forceinline__ int make(int a, int b) { return (a << SH) | b; }
};

__device__ __forceinline__ float block_bound(const float4 *Bd, int a, int b) {
    const float4 A = Bd[a], Bv = Bd[b];
    const float dx = A.x - Bv.x, dy = A.y - Bv.y, dz = A.z - Bv.z;
    return (A.w + Bv.w) - __builtin_amdgcn_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
}

// Lowest sphere key s*S + t in row i of link pair (a, bb) whose penetration
// equals M.
template <int NMAX>
__device__ __forceinline__ int row_min_key(const DevRobot &rb, const float4 *P, int a, int bb, int i, float M) {
    if (a >= rb.L) return INT_MAX;
    const float4 A = P[a * NMAX + i];
    const int s = rb.li[a].sph_first + i, fb = rb.li[bb].sph_first;
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
        if (pair_pen(A, P[bb * NMAX + j]) == M) return s * rb.S + (fb + j);
    return INT_MAX;
}

template <int NMAX>
__device__ __forceinline__ int block_min_key(const DevRobot &rb, const float4 *P, int a, int bb, float M) {
    int key = INT_MAX;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) key = min(key, row_min_key<NMAX>(rb, P, a, bb, i, M));
    return key;
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

// Pass-1 test: block (a, b) may hold a pair whose penetration reaches -eps,
// |C_a - C_b| <= R_a + R_b + eps, as one compare without a square root:
// d2 <= s |s| is false for every s < 0 (d2 >= 0), so the empty pair (L, L)
// never passes.
__device__ __forceinline__ bool may_reach(const float4 *Bd, int a, int b, float eps) {
    const float4 A = Bd[a], Bv = Bd[b];
    const float dx = A.x - Bv.x, dy = A.y - Bv.y, dz = A.z - Bv.z;
    const float s = (A.w + Bv.w) + eps;
    const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    return d2 <= s * fabsf(s);
}

// Appends to list[0, nl) the link pairs of blocks [c0, cend) that pass the
// pass-1 test (PASS1) or, for pass 2, fail it with bound >= lo; returns nl.
// cend - c0 is a multiple of 2G and every entry below cend is a table entry.
// MODE 1: the pass-1 test; 2: blocks that fail it with bound >= lo (pass 2
// of the row-by-row sweep); 3: every block with bound >= lo (pass 2 of the
// row-culled sweep, which filters the rows itself).
template <int MODE, typename E>
__device__ __forceinline__ int compact_blocks(const E *tab, const float4 *Bd, E *list, int c0, int cend, float eps,
                                              float lo, int glane, int G, int gshift, uint64_t gmask) {
    typedef PairCode<E> PC;
    const uint64_t below = (1ull << glane) - 1ull;
    int nl = 0;
    for (int base = c0; base < cend; base += 2 * G) {
        const int k0 = base + glane, k1 = k0 + G;
        const int ab0 = tab[k0], ab1 = tab[k1];
        bool s0, s1;
        if (MODE == 3) {
            s0 = block_bound(Bd, PC::a(ab0), PC::b(ab0)) >= lo;
            s1 = block_bound(Bd, PC::a(ab1), PC::b(ab1)) >= lo;
        } else {
            s0 = may_reach(Bd, PC::a(ab0), PC::b(ab0), eps);
            s1 = may_reach(Bd, PC::a(ab1), PC::b(ab1), eps);
            if (MODE == 2) {
                s0 = !s0 && block_bound(Bd, PC::a(ab0), PC::b(ab0)) >= lo;
                s1 = !s1 && block_bound(Bd, PC::a(ab1), PC::b(ab1)) >= lo;
            }
        }
        const uint64_t m0 = (__ballot(s0) >> gshift) & gmask;
        const uint64_t m1 = (__ballot(s1) >> gshift) & gmask;
        const int n0 = __popcll(m0);
        if (s0) list[nl + __popcll(m0 & below)] = (E)ab0;
        if (s1) list[nl + n0 + __popcll(m1 & below)] = (E)ab1;
        nl += n0 + __popcll(m1);
    }
    return nl;
}

// Pair loop over the rows of list[0, nl): running maximum, the row where it
// was set (link pair * NMAX + slot), whether it was met twice, and the count.
template <int NMAX, bool FULL, typename E>
__device__ __forceinline__ void sweep_rows(const DevRobot &rb, const float4 *P, const E *list, int nl, int glane,
                                           int G, float &best, int &best_code, bool &tie, unsigned &cnt) {
    typedef PairCode<E> PC;
    const int items = nl * NMAX;
    for (int j0 = 0; j0 < items; j0 += G) {
        const int it = j0 + glane;
        const bool ok = it < items;
        const int e = it / NMAX, row = it - e * NMAX;
        const int ab = ok ? (int)list[e] : PC::make(rb.L, rb.L);
        const int a = PC::a(ab), bb = PC::b(ab);
        const float4 A = P[a * NMAX + row];
        float m = -INFINITY;
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
            const float pen = pair_pen(A, P[bb * NMAX + k]);
            m = fmaxf(m, pen);
            if (FULL) cnt += (unsigned)__popcll(__ballot(pen > 0.0f));
            else cnt += pen > 0.0f ? 1u : 0u;
        }
        if (m > best) {
            best = m;
            best_code = ok ? ab * NMAX + row : -1;
            tie = false;
        } else if (m == best) {
            tie = true;
        }
    }
}

// Row test: sphere slot A against link bound Bb may hold a pair reaching
// -eps (squared, as may_reach; an empty slot never passes), and the row
// bound itself.
__device__ __forceinline__ bool row_may_reach(float4 A, float4 Bb, float eps) {
    const float dx = A.x - Bb.x, dy = A.y - Bb.y, dz = A.z - Bb.z;
    const float s = (A.w + Bb.w) + eps;
    const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    return d2 <= s * fabsf(s);
}
__device__ __forceinline__ float row_bound(float4 A, float4 Bb) {
    const float dx = A.x - Bb.x, dy = A.y - Bb.y, dz = A.z - Bb.z;
    return (A.w + Bb.w) - __builtin_amdgcn_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
}

constexpr int ROW_RING = SWEEP_ROW_RING;   // queued rows per group (a power of two, >= 2 G - 1)

// Evaluates the n queued rows at ring[head, head + n) (mod ROW_RING), one
// per lane; a row code is (slot of A) << 16 | (first slot of the second
// link), and best_code keeps the code of the row that set the running max.
template <int NMAX, bool FULL>
__device__ __forceinline__ void eval_rows(const float4 *P, const uint32_t *ring, int head, int n, int glane,
                                          float &best, int &best_code, bool &tie, unsigned &cnt) {
    if (glane < n) {
        const uint32_t code = ring[(head + glane) & (ROW_RING - 1)];
        const float4 A = P[code >> 16];
        const float4 *Bp = P + (code & 0xffffu);
        float m = -INFINITY;
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
            const float pen = pair_pen(A, Bp[k]);
            m = fmaxf(m, pen);
            if (FULL) cnt += (unsigned)__popcll(__ballot(pen > 0.0f));
            else cnt += pen > 0.0f ? 1u : 0u;
        }
        if (m > best) {
            best = m;
            best_code = (int)code;
            tie = false;
        } else if (m == best) {
            tie = true;
        }
    }
}

// The rows of list[0, nl) that pass the row test (pass 1: may reach -eps;
// PASS2: row bound >= lo and not evaluated by pass 1), queued in the ring
// and evaluated G at a time: running maximum, its row code, ties, count.
template <int NMAX, bool FULL, bool PASS2, typename E>
__device__ __forceinline__ void sweep_rows_culled(const float4 *P, const float4 *Bd, const E *list, int nl,
                                                  uint32_t *ring, float eps, float lo, int glane, int G, int gshift,
                                                  uint64_t gmask, float &best, int &best_code, bool &tie,
                                                  unsigned &cnt) {
    typedef PairCode<E> PC;
    const uint64_t below = (1ull << glane) - 1ull;
    const int items = nl * NMAX;
    int head = 0, pending = 0;   // the same in every lane of the group
    for (int j0 = 0; j0 < items; j0 += G) {
        const int it = j0 + glane;
        bool pass = false;
        uint32_t code = 0;
        if (it < items) {
            const int e = it / NMAX, row = it - e * NMAX;
            const int ab = list[e];
            const int a = PC::a(ab), bb = PC::b(ab);
            const float4 A = P[a * NMAX + row], Bb = Bd[bb];
            const bool may = row_may_reach(A, Bb, eps);
            pass = PASS2 ? (row_bound(A, Bb) >= lo && !(may && may_reach(Bd, a, bb, eps))) : may;
            code = ((uint32_t)(a * NMAX + row) << 16) | (uint32_t)(bb * NMAX);
        }
        const uint64_t m = (__ballot(pass) >> gshift) & gmask;
        if (pass) ring[(head + pending + __popcll(m & below)) & (ROW_RING - 1)] = code;
        pending += __popcll(m);
        if (pending >= G) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            eval_rows<NMAX, FULL>(P, ring, head, G, glane, best, best_code, tie, cnt);
            head = (head + G) & (ROW_RING - 1);
            pending -= G;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (pending > 0) eval_rows<NMAX, FULL>(P, ring, head, pending, glane, best, best_code, tie, cnt);
}

// Sweep one state.  tab: the robot's block table (rb.blocks, or an LDS copy
// in the entry type E); P: the state's (L+1)*NMAX sphere slots; Bd: its link
// bounding spheres; list: rb.list_cap entries of LDS scratch for this group.
// Every lane of the group returns the maximum penetration M, the sphere key
// s*S + t of the lowest pair attaining it (INT_MAX if none) and the number
// of pairs with positive penetration.  FULL: G == 64.  ring: ROW_RING words
// of LDS scratch for this group (the row-culled sweep).
template <int NMAX, bool FULL, typename E>
__device__ __forceinline__ void sweep_state(const DevRobot &rb, const E *tab, const float4 *P, const float4 *Bd,
                                            E *list, uint32_t *ring, int glane, int G, int grp, float &M_out,
                                            int &key_out, unsigned &cnt_out) {
    typedef PairCode<E> PC;
    const int n = rb.n_blocks;
    const int nb = (n + 2 * G - 1) / (2 * G) * (2 * G);   // <= n_blocks_pad, a multiple of 128
    const int cap = rb.list_cap;                          // a multiple of 128
    const uint64_t gmask = FULL ? ~0ull : ((1ull << G) - 1ull);
    const int gshift = FULL ? 0 : grp * G;
    // extent of the robot in this state, for the rounding margin
    float ext = 0.f;
    for (int a = glane; a < rb.L; a += G) {
        const float4 c = Bd[a];
        if (c.w > -1e29f)
            ext = fmaxf(ext, __builtin_amdgcn_sqrtf(__builtin_fmaf(c.x, c.x, __builtin_fmaf(c.y, c.y, c.z * c.z))) + c.w);
    }
    const float eps = 4e-6f * (1.f + group_reduce_max(ext, G));

    float best = -INFINITY;
    int best_code = -1;
    bool tie = false;
    unsigned cnt = 0;
    // pass 1: blocks that may hold a collision
    for (int c0 = 0; c0 < nb; c0 += cap) {
        const int nl = compact_blocks<1>(tab, Bd, list, c0, min(c0 + cap, nb), eps, 0.f, glane, G, gshift, gmask);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        sweep_rows_culled<NMAX, FULL, false>(P, Bd, list, nl, ring, eps, 0.f, glane, G, gshift, gmask, best,
                                             best_code, tie, cnt);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    float M = group_reduce_max(best, G);
    if (!(M >= 0.f) && n > 0) {
        // pass 2 (no collision): a lower bound of M, then the skipped blocks that can reach it
        float lb = M;
        if (lb == -INFINITY) {
            float bmax = -INFINITY;
            int bblk = INT_MAX;
            for (int k = glane; k < n; k += G) {
                const int ab = tab[k];
                const float d = block_bound(Bd, PC::a(ab), PC::b(ab));
                if (d > bmax) {
                    bmax = d;
                    bblk = k;
                }
            }
            const float gbmax = group_reduce_max(bmax, G);
            const int cand = group_reduce_min(bmax == gbmax ? bblk : INT_MAX, G);
            float seed = -INFINITY;
            if (cand != INT_MAX) {   // no candidate only when every bound is NaN
                const int ab = tab[cand];
                const int a = PC::a(ab), bb = PC::b(ab);
                for (int j = glane; j < NMAX * NMAX; j += G) {
                    const int i = j / NMAX, k = j - i * NMAX;
                    seed = fmaxf(seed, pair_pen(P[a * NMAX + i], P[bb * NMAX + k]));
                }
            }
            lb = group_reduce_max(seed, G);
        }
        const float theta1 = lb - eps;
        for (int c0 = 0; c0 < nb; c0 += cap) {
            const int nl = compact_blocks<3>(tab, Bd, list, c0, min(c0 + cap, nb), eps, theta1, glane, G, gshift,
                                             gmask);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            sweep_rows_culled<NMAX, FULL, true>(P, Bd, list, nl, ring, eps, theta1, glane, G, gshift, gmask, best,
                                                best_code, tie, cnt);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        M = group_reduce_max(best, G);
    }
    int key = INT_MAX;
    const bool holder = best == M && M > -INFINITY && best_code >= 0;
    const bool rescan = group_reduce_min((holder && tie) ? 0 : 1, G) == 0;
    if (rescan) {
        for (int blk = glane; blk < n; blk += G) {
            const int ab = tab[blk];
            key = min(key, block_min_key<NMAX>(rb, P, PC::a(ab), PC::b(ab), M));
        }
    } else if (holder) {   // the row code: slot of A (link a, row i) and the first slot of link bb
        const int sa = best_code >> 16, a = sa / NMAX;
        key = row_min_key<NMAX>(rb, P, a, (best_code & 0xffff) / NMAX, sa - a * NMAX, M);
    }
    M_out = M;
    key_out = group_reduce_min(key, G);
    cnt_out = FULL ? cnt : group_reduce_sum_u(cnt, G);
}

// Sweep one state with the four wavefronts of a workgroup (the map of the
// paper's two-stage self-collision split over wavefronts, then a second
// reduce through LDS): the block table's 128-entry chunks are dealt
// round-robin to the wavefronts (chunk c to wavefront c % 4); each compacts
// and sweeps its chunks as sweep_state does with G = 64 (one chunk at a
// time, so its list holds 128 entries), and the workgroup combines the
// wavefronts' maxima, counts and argmax keys.  Pass 2, the seed block and
// the tie rescan follow the single-wavefront rules with workgroup-wide
// values, so the result is the full sweep's.  red: 8 words of LDS.  Every
// thread of the workgroup must call this (it synchronizes the workgroup).
__device__ __forceinline__ float wg_max4(float v, float *red, int wave, int lane) {
    if (lane == 0) red[wave] = v;
    __syncthreads();
    const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    return m;
}
__device__ __forceinline__ int wg_min4(int v, int *red, int wave, int lane) {
    if (lane == 0) red[wave] = v;
    __syncthreads();
    const int m = min(min(red[0], red[1]), min(red[2], red[3]));
    __syncthreads();
    return m;
}

template <int NMAX, typename E>
__device__ __forceinline__ void sweep_state_wg(const DevRobot &rb, const E *tab, const float4 *P, const float4 *Bd,
                                               E *list, float *red, int wave, int lane, float &M_out, int &key_out,
                                               unsigned &cnt_out) {
    typedef PairCode<E> PC;
    const int n = rb.n_blocks;
    const int nb = (n + 127) / 128 * 128;   // <= n_blocks_pad
    int *redi = reinterpret_cast<int *>(red);
    float ext = 0.f;
    for (int a = lane; a < rb.L; a += 64) {
        const float4 c = Bd[a];
        if (c.w > -1e29f)
            ext = fmaxf(ext, __builtin_amdgcn_sqrtf(__builtin_fmaf(c.x, c.x, __builtin_fmaf(c.y, c.y, c.z * c.z))) + c.w);
    }
    const float eps = 4e-6f * (1.f + group_reduce_max(ext, 64));

    float best = -INFINITY;
    int best_code = -1;
    bool tie = false;
    unsigned cnt = 0;
    for (int c0 = wave * 128; c0 < nb; c0 += 4 * 128) {
        const int nl = compact_blocks<1>(tab, Bd, list, c0, c0 + 128, eps, 0.f, lane, 64, 0, ~0ull);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        sweep_rows<NMAX, true>(rb, P, list, nl, lane, 64, best, best_code, tie, cnt);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    float M = wg_max4(group_reduce_max(best, 64), red, wave, lane);
    if (!(M >= 0.f) && n > 0) {
        float lb = M;
        if (lb == -INFINITY) {
            // the block with the largest bound over the whole table (lowest index among equals)
            float bmax = -INFINITY;
            int bblk = INT_MAX;
            for (int c0 = wave * 128; c0 < nb; c0 += 4 * 128)
                for (int k = c0 + lane; k < min(c0 + 128, n); k += 64) {
                    const int ab = tab[k];
                    const float d = block_bound(Bd, PC::a(ab), PC::b(ab));
                    if (d > bmax) {
                        bmax = d;
                        bblk = k;
                    }
                }
            const float gbmax = wg_max4(group_reduce_max(bmax, 64), red, wave, lane);
            const int cand = wg_min4(group_reduce_min(bmax == gbmax ? bblk : INT_MAX, 64), redi, wave, lane);
            float seed = -INFINITY;
            if (cand != INT_MAX) {
                const int ab = tab[cand];
                const int a = PC::a(ab), bb = PC::b(ab);
                for (int j = lane; j < NMAX * NMAX; j += 64) {
                    const int i = j / NMAX, k = j - i * NMAX;
                    seed = fmaxf(seed, pair_pen(P[a * NMAX + i], P[bb * NMAX + k]));
                }
            }
            lb = group_reduce_max(seed, 64);   // the same in every wavefront
        }
        const float theta1 = lb - eps;
        for (int c0 = wave * 128; c0 < nb; c0 += 4 * 128) {
            const int nl = compact_blocks<2>(tab, Bd, list, c0, c0 + 128, eps, theta1, lane, 64, 0, ~0ull);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            sweep_rows<NMAX, true>(rb, P, list, nl, lane, 64, best, best_code, tie, cnt);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        M = wg_max4(group_reduce_max(best, 64), red, wave, lane);
    }
    int key = INT_MAX;
    const bool holder = best == M && M > -INFINITY && best_code >= 0;
    const bool rescan = wg_min4(group_reduce_min((holder && tie) ? 0 : 1, 64), redi, wave, lane) == 0;
    if (rescan) {
        for (int c0 = wave * 128; c0 < nb; c0 += 4 * 128)
            for (int blk = c0 + lane; blk < min(c0 + 128, n); blk += 64) {
                const int ab = tab[blk];
                key = min(key, block_min_key<NMAX>(rb, P, PC::a(ab), PC::b(ab), M));
            }
    } else if (holder) {
        const int ab = best_code / NMAX;
        key = row_min_key<NMAX>(rb, P, PC::a(ab), PC::b(ab), best_code - ab * NMAX, M);
    }
    M_out = M;
    key_out = wg_min4(group_reduce_min(key, 64), redi, wave, lane);
    // counts: the wavefronts' (uniform) counts summed in a fixed order
    if (lane == 0) redi[4 + wave] = (int)cnt;
    __syncthreads();
    cnt_out = (unsigned)redi[4] + (unsigned)redi[5] + (unsigned)redi[6] + (unsigned)redi[7];
    __syncthreads();
}

// Pair index (lexicographic in (s, t)) of a sphere key s*S + t.
__device__ __forceinline__ int32_t pair_index(const DevRobot &rb, int key) {
    if (key == INT_MAX) return -1;
    const int s = (int)((unsigned)key / (unsigned)rb.S), t = key - s * rb.S;
    const int a = rb.sph_link[s], bt = rb.sph_link[t];
    return rb.pair_off[s] + rb.pair_cnt[a * rb.L + bt] + (t - rb.li[bt].sph_first);
}

}  // namespace wb
