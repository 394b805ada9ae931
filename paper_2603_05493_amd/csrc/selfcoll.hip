// Standalone self-collision kernel (cuRoboV2 Sec. 6.2): stages the sphere
// centres of a tile of states in LDS and sweeps each state with one
// wavefront (sweep.h).
#include <algorithm>
#include "sweep.h"

namespace wb {

// LDS: TS states x [(L+1)*NMAX slots | (L+1) link bounds], then 4 lists of
// rb.list_cap ints and 4 row rings of SWEEP_ROW_RING words (one of each per
// wavefront), then (TAB_LDS) the block table.
// nb: states; B: row length of the sphere array (the ABI's ld >= nb).
template <int NMAX, bool TAB_LDS>
__global__ void __launch_bounds__(256) k_self_collision(DevRobot rb, int64_t nb, int64_t B, int TS,
                                                        const float *__restrict__ sph,
                                                        float *__restrict__ max_pen,
                                                        int32_t *__restrict__ argmax,
                                                        int32_t *__restrict__ n_coll) {
    extern __shared__ float4 lds[];
    const int SL = (rb.L + 1) * NMAX;
    const int SLB = SL + rb.L + 1;
    const int64_t b0 = (int64_t)blockIdx.x * TS;
    const int tid = threadIdx.x;
    int *lists = reinterpret_cast<int *>(lds + TS * SLB);
    uint32_t *rings = reinterpret_cast<uint32_t *>(lists + 4 * rb.list_cap);
    const int *tab = rb.blocks;
    if (TAB_LDS) {
        int *t = reinterpret_cast<int *>(rings + 4 * SWEEP_ROW_RING);
        for (int i = tid; i < rb.n_blocks_pad; i += 256) t[i] = rb.blocks[i];
        tab = t;
    }
    for (int i = tid; i < TS * SLB; i += 256) {
        const int st = i / SLB, o = i - st * SLB;
        lds[i] = make_float4(0.f, 0.f, 0.f, o < SL ? rb.slot_r[o] : -1e30f);
    }
    __syncthreads();
    const int n3 = rb.S * 3;
    for (int i = tid; i < n3 * TS; i += 256) {
        const int st = i % TS, sc = i / TS;
        const int64_t b = b0 + st;
        if (b < nb) {
            const int s = sc / 3, c = sc - 3 * s;
            reinterpret_cast<float *>(&lds[st * SLB + rb.sph_slot[s]])[c] = sph[(int64_t)sc * B + b];
        }
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    int *list = lists + wave * rb.list_cap;
    for (int st = wave; st < TS; st += 4) {
        const int64_t b = b0 + st;
        if (b >= nb) break;
        float4 *P = lds + st * SLB;
        float4 *Bd = P + SL;
        link_bounds<NMAX>(rb, P, Bd, lane, 64);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        float M;
        int key;
        unsigned cnt;
        sweep_state<NMAX, true>(rb, tab, P, Bd, list, rings + wave * SWEEP_ROW_RING, lane, 64, 0, M, key, cnt);
        if (lane == 0) {
            if (max_pen) max_pen[b] = M;
            if (argmax) argmax[b] = pair_index(rb, key);
            if (n_coll) n_coll[b] = (int32_t)cnt;
        }
    }
}

// One state per workgroup, its pairs split over the four wavefronts and
// reduced through LDS (sweep_state_wg): for batches too small to fill the
// chip with one state per wavefront, and for robots with many pairs.
// LDS: [(L+1)*NMAX slots | L+1 link bounds] (float4), then 4 lists of 128
// entries, the block table (int32) and 8 words for the reductions.
template <int NMAX>
__global__ void __launch_bounds__(256) k_self_collision_wg(DevRobot rb, int64_t nb, int64_t B,
                                                           const float *__restrict__ sph,
                                                           float *__restrict__ max_pen,
                                                           int32_t *__restrict__ argmax,
                                                           int32_t *__restrict__ n_coll) {
    extern __shared__ float4 lds[];
    const int SL = (rb.L + 1) * NMAX;
    float4 *P = lds;
    float4 *Bd = P + SL;
    int *lists = reinterpret_cast<int *>(Bd + rb.L + 1);
    int *tab = lists + 4 * 128;
    float *red = reinterpret_cast<float *>(tab + rb.n_blocks_pad);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < rb.n_blocks_pad; i += 256) tab[i] = rb.blocks[i];
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        for (int i = tid; i < SL; i += 256) P[i] = make_float4(0.f, 0.f, 0.f, rb.slot_r[i]);
        if (tid == 0) Bd[rb.L] = make_float4(0.f, 0.f, 0.f, -1e30f);
        __syncthreads();
        for (int i = tid; i < rb.S * 3; i += 256) {
            const int sph_i = i / 3, c = i - 3 * sph_i;
            reinterpret_cast<float *>(&P[rb.sph_slot[sph_i]])[c] = sph[(int64_t)i * B + b];
        }
        __syncthreads();
        link_bounds<NMAX>(rb, P, Bd, tid, 256);
        __syncthreads();
        float M;
        int key;
        unsigned cnt;
        sweep_state_wg<NMAX>(rb, tab, P, Bd, lists + wave * 128, red, wave, lane, M, key, cnt);
        if (tid == 0) {
            if (max_pen) max_pen[b] = M;
            if (argmax) argmax[b] = pair_index(rb, key);
            if (n_coll) n_coll[b] = (int32_t)cnt;
        }
        __syncthreads();   // the slots are rewritten for the next state
    }
}

size_t self_collision_wg_lds(int L, int nmax, int n_blocks_pad) {
    return state_lds_bytes(L, nmax) + (size_t)4 * 128 * 4 + (size_t)n_blocks_pad * 4 + 8 * 4;
}

// States per workgroup that fit the LDS limit next to `fixed` bytes.
static int sc_tile(size_t per_state, size_t fixed) {
    int ts = (int)((LDS_LIMIT - fixed) / per_state);
    if (ts > 16) ts = 16;
    if (ts >= 4) ts &= ~3;
    if (ts < 1) ts = 1;
    return ts;
}

// LDS of the four wavefronts' lists and row rings.
static size_t sc_lists_bytes(int list_cap) { return (size_t)16 * list_cap + (size_t)16 * SWEEP_ROW_RING; }

int self_collision_tile(int L, int nmax, int list_cap) {
    return sc_tile(state_lds_bytes(L, nmax), sc_lists_bytes(list_cap));
}

// The block table goes to LDS when one state, the four lists and the table
// fit; otherwise the lists shrink to fit beside one state and the table is
// read from device memory.
template <int NMAX>
static hipError_t launch_sc(const DevRobot &rb0, int64_t B, int64_t ld, const float *sph, float *mp, int32_t *am,
                            int32_t *nc, hipStream_t s) {
    DevRobot rb = rb0;
    const size_t per_state = state_lds_bytes(rb.L, NMAX);
    const size_t tab = (size_t)rb.n_blocks_pad * 4;
    dim3 block(256);
    if (per_state + sc_lists_bytes(rb.list_cap) + tab <= LDS_LIMIT) {
        const int TS = sc_tile(per_state, sc_lists_bytes(rb.list_cap) + tab);
        const size_t lds = (size_t)TS * per_state + sc_lists_bytes(rb.list_cap) + tab;
        dim3 grid((unsigned)((B + TS - 1) / TS));
        hipLaunchKernelGGL((k_self_collision<NMAX, true>), grid, block, lds, s, rb, B, ld, TS, sph, mp, am, nc);
    } else {
        const int room = (int)((LDS_LIMIT - per_state - (size_t)16 * SWEEP_ROW_RING) / 16) / 128 * 128;
        if (room < rb.list_cap) rb.list_cap = room;
        const int TS = self_collision_tile(rb.L, NMAX, rb.list_cap);
        const size_t lds = (size_t)TS * per_state + sc_lists_bytes(rb.list_cap);
        dim3 grid((unsigned)((B + TS - 1) / TS));
        hipLaunchKernelGGL((k_self_collision<NMAX, false>), grid, block, lds, s, rb, B, ld, TS, sph, mp, am, nc);
    }
    return hipGetLastError();
}

template <int NMAX>
static hipError_t launch_sc_wg(const DevRobot &rb, int64_t B, int64_t ld, const float *sph, float *mp, int32_t *am,
                               int32_t *nc, hipStream_t s) {
    const size_t lds = self_collision_wg_lds(rb.L, NMAX, rb.n_blocks_pad);
    const unsigned grid = (unsigned)std::min<int64_t>(B, 1 << 20);
    hipLaunchKernelGGL((k_self_collision_wg<NMAX>), dim3(grid), dim3(256), lds, s, rb, B, ld, sph, mp, am, nc);
    return hipGetLastError();
}

template <int NMAX>
static hipError_t launch_sc_any(const DevRobot &rb, int64_t B, int64_t ld, const float *sph, float *mp, int32_t *am,
                                int32_t *nc, bool split, hipStream_t s) {
    return split ? launch_sc_wg<NMAX>(rb, B, ld, sph, mp, am, nc, s) : launch_sc<NMAX>(rb, B, ld, sph, mp, am, nc, s);
}

hipError_t launch_self_collision(const DevRobot &rb, int64_t B, int64_t ld, const float *spheres,
                                 float *max_pen, int32_t *argmax, int32_t *n_coll, bool split, hipStream_t s) {
    if (B == 0) return hipSuccess;
    switch (rb.nmax) {
        case 1: return launch_sc_any<1>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 2: return launch_sc_any<2>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 3: return launch_sc_any<3>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 4: return launch_sc_any<4>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 5: return launch_sc_any<5>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 6: return launch_sc_any<6>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 7: return launch_sc_any<7>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 8: return launch_sc_any<8>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 12: return launch_sc_any<12>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 16: return launch_sc_any<16>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 24: return launch_sc_any<24>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 32: return launch_sc_any<32>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 48: return launch_sc_any<48>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        case 64: return launch_sc_any<64>(rb, B, ld, spheres, max_pen, argmax, n_coll, split, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace wb
