// Cross-lane primitives for aligned groups of G = 16, 32 or 64 lanes of a
// wave64, built from DPP row operations (a few cycles, no LDS), the gfx950
// permlane16/32 swaps, and one ds_bpermute where an arbitrary gather is
// needed.
//
//   group_scan      inclusive prefix sum over the group (Hillis-Steele with
//                   row_shr 1, 2, 4, 8 inside each 16-lane row, then
//                   row_bcast:15 and row_bcast:31 to carry row totals);
//                   group_scan4/6 the same for four or six values at once
//   group_reduce_*  butterfly reduction, result in every lane of the group
//                   (quad_perm xor 1, xor 2, row_half_mirror, row_mirror,
//                   then the permlane swaps across rows and halves)
//   lane_prev       value of the previous lane of the wave (wave_shr:1)
#pragma once

#include <hip/hip_runtime.h>

namespace wb {

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
    // lanes whose source is outside the row, or whose row is masked off,
    // receive 0 (the "old" operand)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK,
                                                                 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

constexpr int DPP_QUAD_XOR1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int DPP_ROW_SHR = 0x110;        // + n: row_shr:n
constexpr int DPP_WAVE_SHR1 = 0x138;
constexpr int DPP_ROW_MIRROR = 0x140;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_BCAST15 = 0x142;
constexpr int DPP_ROW_BCAST31 = 0x143;

__device__ __forceinline__ float group_scan(float x, int G) {
    x += dpp_f<DPP_ROW_SHR + 1>(x);
    x += dpp_f<DPP_ROW_SHR + 2>(x);
    x += dpp_f<DPP_ROW_SHR + 4>(x);
    x += dpp_f<DPP_ROW_SHR + 8>(x);
    if (G >= 32) x += dpp_f<DPP_ROW_BCAST15, 0xa>(x);   // rows 1 and 3 add the previous row's total
    if (G >= 64) x += dpp_f<DPP_ROW_BCAST31, 0xc>(x);   // rows 2 and 3 add the first half's total
    return x;
}

// Inclusive prefix sums over the group of four or six values at once (a
// point and a mass; the six components of a spatial vector), each
// Hillis-Steele step an in-place DPP add.  The row_bcast steps write only the
// rows named by the row mask, and the rows left out keep their value, which
// is the sum wanted there; written as builtins, such a step costs three
// instructions (the compiler does not fold a masked DPP move into a float
// add).  The chains are interleaved, so each DPP read of a value comes four
// or six instructions after its last write.  The compiler's hazard checks
// do not look into inline asm: the block opens with the 5 wait states a DPP
// read needs after a VALU write of EXEC (2 after one of its source) and
// closes with the 2 that a DPP read of its results needs.  The blocks are
// volatile, so they stay where they are written: their results depend on
// other lanes' values and on EXEC.
#define WB_DPP4(op)                                  \
    "v_add_f32_dpp %0, %0, %0 " op "\n\t"             \
    "v_add_f32_dpp %1, %1, %1 " op "\n\t"             \
    "v_add_f32_dpp %2, %2, %2 " op "\n\t"             \
    "v_add_f32_dpp %3, %3, %3 " op "\n\t"
#define WB_DPP6(op)                                  \
    WB_DPP4(op)                                      \
    "v_add_f32_dpp %4, %4, %4 " op "\n\t"             \
    "v_add_f32_dpp %5, %5, %5 " op "\n\t"
#define WB_SHR(n) "row_shr:" #n " row_mask:0xf bank_mask:0xf bound_ctrl:1"
#define WB_BC15 "row_bcast:15 row_mask:0xa bank_mask:0xf"
#define WB_BC31 "row_bcast:31 row_mask:0xc bank_mask:0xf"
#define WB_SCAN(D, G, ...)                                                                                \
    do {                                                                                                 \
        if (G >= 64)                                                                                     \
            asm volatile("s_nop 4\n\t" D(WB_SHR(1)) D(WB_SHR(2)) D(WB_SHR(4)) D(WB_SHR(8)) D(WB_BC15) D(WB_BC31)     \
                "s_nop 1"                                                                                \
                : __VA_ARGS__);                                                                 \
        else if (G >= 32)                                                                                \
            asm volatile("s_nop 4\n\t" D(WB_SHR(1)) D(WB_SHR(2)) D(WB_SHR(4)) D(WB_SHR(8)) D(WB_BC15)       \
                             "s_nop 1"                                                                   \
                         : __VA_ARGS__);                                                                 \
        else                                                                                             \
            asm volatile("s_nop 4\n\t" D(WB_SHR(1)) D(WB_SHR(2)) D(WB_SHR(4)) D(WB_SHR(8)) "s_nop 1"     \
                         : __VA_ARGS__);                                                                 \
    } while (0)
__device__ __forceinline__ void group_scan4(float &a, float &b, float &c, float &d, int G) {
    WB_SCAN(WB_DPP4, G, "+v"(a), "+v"(b), "+v"(c), "+v"(d));
}
__device__ __forceinline__ void group_scan6(float &a, float &b, float &c, float &d, float &e, float &f, int G) {
    WB_SCAN(WB_DPP6, G, "+v"(a), "+v"(b), "+v"(c), "+v"(d), "+v"(e), "+v"(f));
}
#undef WB_SCAN
#undef WB_DPP4
#undef WB_DPP6
#undef WB_SHR
#undef WB_BC15
#undef WB_BC31

// Value held by lane - 1 of the wave (0 in lane 0: with bound_ctrl set, a
// lane whose source is outside the wave reads 0, so no "old" value is kept).
__device__ __forceinline__ float lane_prev(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), DPP_WAVE_SHR1, 0xf,
                                                                 0xf, true));
}

// The other row of each row pair (0<->1, 2<->3) and the other half of the wave.
__device__ __forceinline__ void swap16(unsigned v, unsigned &a, unsigned &b) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void swap32(unsigned v, unsigned &a, unsigned &b) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    a = r[0];
    b = r[1];
}

// Reductions: after swapN, the two returned values are the lane's own row
// (half) and the partner's, in an order that depends on the lane, so the
// operator is applied to both.
__device__ __forceinline__ float group_reduce_max(float x, int G) {
    x = fmaxf(x, dpp_f<DPP_QUAD_XOR1>(x));
    x = fmaxf(x, dpp_f<DPP_QUAD_XOR2>(x));
    x = fmaxf(x, dpp_f<DPP_ROW_HALF_MIRROR>(x));
    x = fmaxf(x, dpp_f<DPP_ROW_MIRROR>(x));
    unsigned a, b;
    if (G >= 32) {
        swap16(__builtin_bit_cast(unsigned, x), a, b);
        x = fmaxf(__builtin_bit_cast(float, a), __builtin_bit_cast(float, b));
    }
    if (G >= 64) {
        swap32(__builtin_bit_cast(unsigned, x), a, b);
        x = fmaxf(__builtin_bit_cast(float, a), __builtin_bit_cast(float, b));
    }
    return x;
}
__device__ __forceinline__ float group_reduce_sum(float x, int G) {
    x += dpp_f<DPP_QUAD_XOR1>(x);
    x += dpp_f<DPP_QUAD_XOR2>(x);
    x += dpp_f<DPP_ROW_HALF_MIRROR>(x);
    x += dpp_f<DPP_ROW_MIRROR>(x);
    unsigned a, b;
    if (G >= 32) {
        swap16(__builtin_bit_cast(unsigned, x), a, b);
        x = __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
    }
    if (G >= 64) {
        swap32(__builtin_bit_cast(unsigned, x), a, b);
        x = __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
    }
    return x;
}
__device__ __forceinline__ int group_reduce_min(int x, int G) {
    x = min(x, dpp_i<DPP_QUAD_XOR1>(x));
    x = min(x, dpp_i<DPP_QUAD_XOR2>(x));
    x = min(x, dpp_i<DPP_ROW_HALF_MIRROR>(x));
    x = min(x, dpp_i<DPP_ROW_MIRROR>(x));
    unsigned a, b;
    if (G >= 32) {
        swap16((unsigned)x, a, b);
        x = min((int)a, (int)b);
    }
    if (G >= 64) {
        swap32((unsigned)x, a, b);
        x = min((int)a, (int)b);
    }
    return x;
}
__device__ __forceinline__ unsigned group_reduce_sum_u(unsigned x, int G) {
    x += (unsigned)dpp_i<DPP_QUAD_XOR1>((int)x);
    x += (unsigned)dpp_i<DPP_QUAD_XOR2>((int)x);
    x += (unsigned)dpp_i<DPP_ROW_HALF_MIRROR>((int)x);
    x += (unsigned)dpp_i<DPP_ROW_MIRROR>((int)x);
    unsigned a, b;
    if (G >= 32) {
        swap16(x, a, b);
        x = a + b;
    }
    if (G >= 64) {
        swap32(x, a, b);
        x = a + b;
    }
    return x;
}

}  // namespace wb
