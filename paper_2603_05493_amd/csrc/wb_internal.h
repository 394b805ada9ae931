// Internal structures shared by the host code and the HIP kernels of libwb.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include "wb.h"

namespace wb {

// Per-link float record, 32 floats (128 bytes) so a uniform link index turns
// into one scalar-cache fetch in lane-per-state kernels.
struct LinkF {
    float axis[3];     // 0
    float fR[9];       // 3   row-major fixed rotation
    float fp[3];       // 12  fixed translation (child joint origin in parent frame)
    float mult;        // 15
    float offset;      // 16
    float mass;        // 17
    float com[3];      // 18
    float I[6];        // 21  xx yy zz xy xz yz about the CoM, link axes
    float pad[5];      // 27
};
static_assert(sizeof(LinkF) == 128, "LinkF layout");

// Per-link integer record.
struct LinkI {
    int32_t parent;
    int32_t revolute;  // 1 if the link has a revolute joint
    int32_t jidx;      // actuated joint, -1 if fixed
    int32_t sph_first;
    int32_t sph_count;
    int32_t depth;
    int32_t fR_identity;  // fixed rotation is exactly the identity
    int32_t far_child;    // has a child other than link k+1
};
static_assert(sizeof(LinkI) == 32, "LinkI layout");

// Device view of a robot, passed by value to kernels.
struct DevRobot {
    int32_t L, n, S, nmax;        // nmax: sphere slots per link (max spheres on a link)
    int32_t n_blocks, n_blocks_pad, max_depth, simple_joints;  // simple: one link per actuated joint, mult 1, offset 0
    int64_t n_pairs;
    float gx, gy, gz;
    int32_t list_cap;             // ints of the per-group LDS list of the pair sweep (multiple of 128)
    const LinkF *__restrict__ lf;         // [L]
    const LinkI *__restrict__ li;         // [L]
    const float4 *__restrict__ sph;       // [S] local centre + radius
    const int32_t *__restrict__ sph_link; // [S]
    const int32_t *__restrict__ sph_slot; // [S] padded slot a*nmax + (s - first sphere of a)
    const float *__restrict__ slot_r;     // [(L+1)*nmax] radius of slot (a,i), -1e30 for empty slots
    const int32_t *__restrict__ blocks;   // [n_blocks_pad] packed (a<<16)|b, padded to a multiple of 128 with (L<<16)|L
    const int32_t *__restrict__ pair_off; // [S] index of sphere s's first pair
    const int32_t *__restrict__ pair_cnt; // [L*L] pairs of a sphere on link a with links a<b'<b
    const int32_t *__restrict__ pair_s;   // [P]
    const int32_t *__restrict__ pair_t;   // [P]
};

// Per-lane tables of the fused kernel: lane i holds link perm[i] in
// depth-first pre-order.  Structure of arrays, 64 entries per field.
//   li[f*64 + i]: f = 0 link, 1 parent lane (-1 root), 2 last lane of the
//                 subtree, 3 joint index (-1 fixed), 4 sphere count,
//                 5 revolute, 6 fixed rotation is the identity
//   lf[f*64 + i]: f = 0..2 axis, 3..11 fixed R, 12..14 fixed p, 15 mass,
//                 16..18 CoM, 19..24 inertia (xx yy zz xy xz yz),
//                 25..27 centre and 28 radius of the link's bounding sphere in
//                 link coordinates (-1e30 without spheres), 29 joint
//                 multiplier, 30 joint offset
//   lsph[j*64 + i]: local centre and radius of the link's j-th sphere
//   conn[k*64 + j]: lane of the k-th link that joint j drives, -1 past the
//                 end of the list (read only when mimic is set)
// Lanes past the last link hold an empty link: link -1, parent -1, subtree
// end i, no joint, no spheres, identity fixed rotation, zero mass.
struct DevFused {
    int32_t supported;   // L <= 64 and the sweep tables fit the LDS budget
    int32_t jsteps;      // pointer-jumping steps, ceil(log2(max_depth + 1))
    int32_t mimic;       // some joint drives several links, or a multiplier != 1 or offset != 0
    int32_t mc;          // longest connectedLinks list
    const int32_t *__restrict__ li;
    const float *__restrict__ lf;
    const float4 *__restrict__ lsph;
    const int32_t *__restrict__ conn;
};

// Device pointers of one robot's batch in a fused iteration.
struct TreeIO {
    float *q, *qd, *qdd;          // [n][B], updated in place when lr != 0
    const float *w;               // [n][B] or null
    float *tau, *cost, *max_pen;  // optional outputs
    int32_t *argmax, *n_coll;
    float *g_q, *g_qd, *g_qdd;
    const float *f_ext;           // [L][6][B] external link forces (link coordinates) or null
    float *g_fext;                // [L][6][B] their gradient or null
    int64_t ld;                   // row length B of the [k][B] arrays (>= the states)
};

// Scalars of the cost head and the step.
struct StepScalars {
    float torque_weight, margin, hinge_weight, lr;
};

// The spline-sampling form of the fused iteration: its states are the
// samples of uniform cubic B-splines (four per knot interval), formed in the
// kernel from the control points instead of read from q, qd, qdd.
struct SplineIn {
    float *U;                              // [d][T][K] control points, or null (states from io.q, qd, qdd)
    const float *th0, *dth0, *ddth0;       // [d][T] initial states (dth0, ddth0 may be null: at rest)
    int32_t T, K, H, printed;              // trajectories, control points, samples per trajectory, ghost reading
    float dt;
    // the control-point gradient reduced in the kernel (each workgroup owns
    // whole trajectories), then the step: g_U [d][T][K] (may be null), lr,
    // step rule (WB_STEP_*)
    float *g_U;
    float lr;
    int32_t rule;
};

// Arguments of the single-robot fused kernel (by value).
struct FusedArgs {
    DevRobot rb;
    DevFused fz;
    TreeIO io;
    SplineIn sp;
    StepScalars k;
    int64_t B;                // states (the arrays' row length is io.ld)
    int32_t chunk;            // states per workgroup
    int32_t lanes_per_state;  // G: 16, 32 or 64
};

// One robot of an uneven batch, and one unit of work of the persistent launch.
struct PlanTree {
    DevRobot rb;              // tables re-derived for the plan's slots per link
    DevFused fz;
    int64_t B;                // states (the arrays' row length is the run's io.ld)
    int32_t lanes_per_state;
    int32_t pad;
};
struct PlanItem {
    int64_t b0;
    int32_t tree, count;
};

#define WB_PLAN_MAX_TREES 16
struct PlanArgs {
    const PlanTree *trees;
    const PlanItem *items;        // grouped by workgroup
    const int32_t *item_start;    // [n_wg + 1]
    int32_t wave_stride;          // float4s of LDS per wave (the largest over the plan's trees);
                                  // the block table follows the four waves' regions
    StepScalars k;
    TreeIO io[WB_PLAN_MAX_TREES];
};

hipError_t launch_fused(const FusedArgs &a, hipStream_t s);
hipError_t launch_plan(const PlanArgs &a, int nmax, int n_wg, size_t lds, bool ext, hipStream_t s);
// Workgroups of the plan kernel (variant nmax, ext, `lds` bytes of dynamic
// LDS) that one compute unit keeps resident; at least 1.
int plan_workgroups_per_cu(int nmax, bool ext, size_t lds);

// Kernel launchers (each defined next to its kernels).
hipError_t launch_fk(const DevRobot &rb, int64_t B, int64_t ld, const float *q, float *pose, float *spheres,
                     hipStream_t s);
hipError_t launch_fk_backward(const DevRobot &rb, int64_t B, int64_t ld, const float *q, const float *pose,
                              const float *g_pose, const float *g_sph, float *g_q, float *ws,
                              hipStream_t s);
hipError_t launch_rnea(const DevRobot &rb, int64_t B, int64_t ld, const float *q, const float *qd,
                       const float *qdd, const float *f_ext, float *tau, float *cache, hipStream_t s);
hipError_t launch_rnea_backward(const DevRobot &rb, int64_t B, int64_t ld, const float *q, const float *qd,
                                const float *qdd, const float *cache, const float *g_tau,
                                float *g_q, float *g_qd, float *g_qdd, float *g_fext, float *ws, hipStream_t s);
// Group-per-state RNEA and VJP without a cache (tree_kernels.hip); robots of
// at most 64 links.
hipError_t launch_rnea_lanes(const DevRobot &rb, const DevFused &fz, int64_t B, int64_t ld, const float *q,
                             const float *qd, const float *qdd, const float *f_ext, float *tau, hipStream_t s);
hipError_t launch_rnea_backward_lanes(const DevRobot &rb, const DevFused &fz, int64_t B, int64_t ld,
                                      const float *q, const float *qd, const float *qdd, const float *f_ext,
                                      const float *g_tau, float *g_q, float *g_qd, float *g_qdd, float *g_fext,
                                      hipStream_t s);
// split: one state per workgroup with its pairs over the four wavefronts
// (else one state per wavefront).
// Group-per-state FK adjoint from sphere and/or pose gradients (dense
// arrays, robots of at most 64 links).
hipError_t launch_fk_backward_lanes(const DevRobot &rb, const DevFused &fz, int64_t B, int64_t ld, const float *q,
                                    const float *g_pose, const float *g_sph, float *g_q, hipStream_t s);
hipError_t launch_self_collision(const DevRobot &rb, int64_t B, int64_t ld, const float *spheres,
                                 float *max_pen, int32_t *argmax, int32_t *n_coll, bool split, hipStream_t s);
size_t self_collision_wg_lds(int L, int nmax, int n_blocks_pad);
hipError_t launch_self_collision_backward(const DevRobot &rb, int64_t B, int64_t ld, const float *spheres,
                                          const int32_t *argmax, const float *max_pen,
                                          float margin, const float *g_cost, float *g_sph,
                                          hipStream_t s);
hipError_t launch_cost_head(int64_t B, int64_t ld, int32_t n, const float *tau, const float *w, float tw,
                            const float *max_pen, float margin, float hw, float *cost,
                            float *g_tau, float *g_maxpen, hipStream_t s);
hipError_t launch_sgd_step(int64_t B, int64_t ld, int32_t n, float lr, float *q, float *qd, float *qdd,
                           const float *g_q, const float *g_q2, const float *g_qd,
                           const float *g_qdd, hipStream_t s);

hipError_t launch_bspline_eval(int64_t T, int32_t d, int32_t K, int32_t n_interp, float dt, int32_t printed,
                               const float *U, const float *th0, const float *dth0, const float *ddth0, float *q,
                               float *qd, float *qdd, hipStream_t s);
hipError_t launch_bspline_backward(int64_t T, int32_t d, int32_t K, int32_t n_interp, float dt, const float *g_q,
                                   const float *g_qd, const float *g_qdd, float *g_U, float lr, int32_t rule,
                                   float *U, hipStream_t s);

// LDS of one state's sweep: (L+1)*nmax sphere slots and L+1 link bounding
// spheres (float4 each); plus, per sweeping group, a list of list_cap
// surviving link pairs (16-bit entries in the fused kernels, 32-bit in the
// standalone self-collision kernel) and a ring of SWEEP_ROW_RING row codes.
constexpr int SWEEP_LIST_MAX = 2048;
inline int sweep_list_cap(int n_blocks) {
    int c = (n_blocks + 127) / 128 * 128;
    return c < 128 ? 128 : (c > SWEEP_LIST_MAX ? SWEEP_LIST_MAX : c);
}
__host__ __device__ inline size_t state_lds_bytes(int L, int nmax) { return (size_t)(L + 1) * (nmax + 1) * 16; }
// Rows queued per sweeping group by the row-culled sweep (32-bit codes).
constexpr int SWEEP_ROW_RING = 128;
__host__ __device__ inline size_t group_lds_bytes(int L, int nmax, int list_cap) {
    return state_lds_bytes(L, nmax) + (size_t)list_cap * 2 + (size_t)SWEEP_ROW_RING * 4;
}
// LDS copy of the block table in the fused kernels (n_blocks_pad 16-bit
// entries, a multiple of 128).
__host__ __device__ inline size_t tab_lds_bytes(int n_blocks_pad) { return (size_t)n_blocks_pad * 2; }
// LDS of a 256-lane workgroup of the fused kernels with G lanes per state:
// four wavefronts' group regions, then the block table.
inline size_t fused_lds_bytes(int L, int nmax, int list_cap, int G, int n_blocks_pad) {
    return (size_t)4 * (64 / G) * group_lds_bytes(L, nmax, list_cap) + tab_lds_bytes(n_blocks_pad);
}
// LDS of the in-kernel control-point gradient beyond the fused kernel's:
// one partial sum per group of lanes (4 * 64 / G of them) over the
// d x (K + 6) extended knots, then the d x K reduced gradient.
inline size_t spline_lds_bytes(int G, int d, int K) {
    return ((size_t)(256 / G) * (K + 6) + (size_t)K) * d * 4;
}
constexpr size_t LDS_LIMIT = 65536;
// Sphere slots per link the fused kernels are instantiated for: 1 to 8, and
// 12 (links of up to 12 spheres are padded to 12 slots).
constexpr int FUSED_MAX_SLOTS = 12;

// States per workgroup of the self-collision kernel (LDS tile).
int self_collision_tile(int L, int nmax, int list_cap);

// Workspace floats per state needed by the backward kernels.
inline int64_t workspace_floats_per_state(int L) { return (int64_t)L * 18 + 8; }

}  // namespace wb
