// Self-collision map-reduce (cuRoboV2 Sec. 6.2), one wavefront per state.
//
// The checked pair set is a union of dense link blocks: every allowed link
// pair (a < b) contributes all spheres of a times all spheres of b.  Each
// workgroup stages the sphere centres of a tile of states in LDS, padded to
// nmax slots per link (empty slots carry radius -1e30, so they can neither be
// the maximum nor count as a collision), plus one all-empty row that the
// block list is padded with to a multiple of 64.  Each lane of the state's
// wave then owns whole link blocks: it loads the nmax + nmax centres of its
// block into registers once and evaluates nmax * nmax pairs (the "map"), so
// the control flow of the sweep is uniform across the wave.
//
// Reduce: the pair count accumulates on the scalar unit from a ballot of
// pen > 0 per pair; the maximum is a per-lane running max per block plus a
// wave shuffle reduction.  The lowest pair index attaining the maximum is
// recovered exactly: each lane remembers the block where its running max was
// set and whether another of its blocks tied it; lanes holding the wave
// maximum re-evaluate that block (or, after a tie, all their blocks) with the
// same arithmetic and report the lowest (s, t) whose penetration equals it.
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

template <int NMAX>
__global__ void __launch_bounds__(256) k_self_collision(DevRobot rb, int64_t B, int TS,
                                                        const float *__restrict__ sph,
                                                        float *__restrict__ max_pen,
                                                        int32_t *__restrict__ argmax,
                                                        int32_t *__restrict__ n_coll) {
    extern __shared__ float4 lds[];
    const int SL = (rb.L + 1) * NMAX;
    const int64_t b0 = (int64_t)blockIdx.x * TS;
    const int tid = threadIdx.x;
    for (int i = tid; i < TS * SL; i += 256) lds[i] = make_float4(0.f, 0.f, 0.f, rb.slot_r[i % SL]);
    __syncthreads();
    const int n3 = rb.S * 3;
    for (int i = tid; i < n3 * TS; i += 256) {
        const int st = i % TS, sc = i / TS;
        const int64_t b = b0 + st;
        if (b < B) {
            const int s = sc / 3, c = sc - 3 * s;
            reinterpret_cast<float *>(&lds[st * SL + rb.sph_slot[s]])[c] = sph[(int64_t)sc * B + b];
        }
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    for (int st = wave; st < TS; st += 4) {
        const int64_t b = b0 + st;
        if (b >= B) break;
        const float4 *P = lds + st * SL;
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
        key = wave_min(key);
        if (lane == 0) {
            int32_t idx = -1;
            if (key != INT_MAX) {
                const int s = key / rb.S, t = key - s * rb.S;
                const int a = rb.sph_link[s], bt = rb.sph_link[t];
                idx = rb.pair_off[s] + rb.pair_cnt[a * rb.L + bt] + (t - rb.li[bt].sph_first);
            }
            if (max_pen) max_pen[b] = M;
            if (argmax) argmax[b] = idx;
            if (n_coll) n_coll[b] = (int32_t)cnt;
        }
    }
}

int self_collision_tile(int L, int nmax) {
    const int bytes_per_state = (L + 1) * nmax * (int)sizeof(float4);
    int ts = 65536 / bytes_per_state;
    if (ts > 16) ts = 16;
    if (ts >= 4) ts &= ~3;
    if (ts < 1) ts = 1;
    return ts;
}

template <int NMAX>
static hipError_t launch_sc(const DevRobot &rb, int64_t B, const float *sph, float *mp, int32_t *am,
                            int32_t *nc, hipStream_t s) {
    const int TS = self_collision_tile(rb.L, NMAX);
    const size_t lds = (size_t)TS * (rb.L + 1) * NMAX * sizeof(float4);
    dim3 grid((unsigned)((B + TS - 1) / TS));
    hipLaunchKernelGGL(k_self_collision<NMAX>, grid, dim3(256), lds, s, rb, B, TS, sph, mp, am, nc);
    return hipGetLastError();
}

hipError_t launch_self_collision(const DevRobot &rb, int64_t B, const float *spheres,
                                 float *max_pen, int32_t *argmax, int32_t *n_coll, hipStream_t s) {
    if (B == 0) return hipSuccess;
    switch (rb.nmax) {
        case 1: return launch_sc<1>(rb, B, spheres, max_pen, argmax, n_coll, s);
        case 2: return launch_sc<2>(rb, B, spheres, max_pen, argmax, n_coll, s);
        case 3: return launch_sc<3>(rb, B, spheres, max_pen, argmax, n_coll, s);
        case 4: return launch_sc<4>(rb, B, spheres, max_pen, argmax, n_coll, s);
        case 5: return launch_sc<5>(rb, B, spheres, max_pen, argmax, n_coll, s);
        case 6: return launch_sc<6>(rb, B, spheres, max_pen, argmax, n_coll, s);
        case 7: return launch_sc<7>(rb, B, spheres, max_pen, argmax, n_coll, s);
        case 8: return launch_sc<8>(rb, B, spheres, max_pen, argmax, n_coll, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace wb
