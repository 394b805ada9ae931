// Standalone self-collision kernel (cuRoboV2 Sec. 6.2): stages the sphere
// centres of a tile of states in LDS and sweeps each state with one
// wavefront (sweep.h).
#include "sweep.h"

namespace wb {

// LDS: TS states x [(L+1)*NMAX slots | (L+1) link bounds], then 4 lists of
// rb.list_cap ints (one per wavefront), then (TAB_LDS) the block table.
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
    const int *tab = rb.blocks;
    if (TAB_LDS) {
        int *t = lists + 4 * rb.list_cap;
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
        sweep_state<NMAX, true>(rb, tab, P, Bd, list, lane, 64, 0, M, key, cnt);
        if (lane == 0) {
            if (max_pen) max_pen[b] = M;
            if (argmax) argmax[b] = pair_index(rb, key);
            if (n_coll) n_coll[b] = (int32_t)cnt;
        }
    }
}

// States per workgroup that fit the LDS limit next to `fixed` bytes.
static int sc_tile(size_t per_state, size_t fixed) {
    int ts = (int)((LDS_LIMIT - fixed) / per_state);
    if (ts > 16) ts = 16;
    if (ts >= 4) ts &= ~3;
    if (ts < 1) ts = 1;
    return ts;
}

int self_collision_tile(int L, int nmax, int list_cap) {
    return sc_tile(state_lds_bytes(L, nmax), (size_t)16 * list_cap);
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
    if (per_state + (size_t)16 * rb.list_cap + tab <= LDS_LIMIT) {
        const int TS = sc_tile(per_state, (size_t)16 * rb.list_cap + tab);
        const size_t lds = (size_t)TS * per_state + (size_t)16 * rb.list_cap + tab;
        dim3 grid((unsigned)((B + TS - 1) / TS));
        hipLaunchKernelGGL((k_self_collision<NMAX, true>), grid, block, lds, s, rb, B, ld, TS, sph, mp, am, nc);
    } else {
        const int room = (int)((LDS_LIMIT - per_state) / 16) / 128 * 128;
        if (room < rb.list_cap) rb.list_cap = room;
        const int TS = self_collision_tile(rb.L, NMAX, rb.list_cap);
        const size_t lds = (size_t)TS * per_state + (size_t)16 * rb.list_cap;
        dim3 grid((unsigned)((B + TS - 1) / TS));
        hipLaunchKernelGGL((k_self_collision<NMAX, false>), grid, block, lds, s, rb, B, ld, TS, sph, mp, am, nc);
    }
    return hipGetLastError();
}

hipError_t launch_self_collision(const DevRobot &rb, int64_t B, int64_t ld, const float *spheres,
                                 float *max_pen, int32_t *argmax, int32_t *n_coll, hipStream_t s) {
    if (B == 0) return hipSuccess;
    switch (rb.nmax) {
        case 1: return launch_sc<1>(rb, B, ld, spheres, max_pen, argmax, n_coll, s);
        case 2: return launch_sc<2>(rb, B, ld, spheres, max_pen, argmax, n_coll, s);
        case 3: return launch_sc<3>(rb, B, ld, spheres, max_pen, argmax, n_coll, s);
        case 4: return launch_sc<4>(rb, B, ld, spheres, max_pen, argmax, n_coll, s);
        case 5: return launch_sc<5>(rb, B, ld, spheres, max_pen, argmax, n_coll, s);
        case 6: return launch_sc<6>(rb, B, ld, spheres, max_pen, argmax, n_coll, s);
        case 7: return launch_sc<7>(rb, B, ld, spheres, max_pen, argmax, n_coll, s);
        case 8: return launch_sc<8>(rb, B, ld, spheres, max_pen, argmax, n_coll, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace wb
