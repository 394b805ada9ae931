// Device view and launchers of the kinematics-outputs kernel: link poses,
// sphere centres, tool poses, the centre of mass, the tool-frame Jacobians
// of Alg. 2, the Jacobian of the centre of mass, and the gradient of
// tool-pose and centre-of-mass losses (cuRoboV2 Sec. 6.1).
#pragma once

#include "wb_internal.h"

namespace wb {

// Lane tables: lane i of a group holds link perm[i] in depth-first
// pre-order, so the subtree of lane i is the lane range [i, sub_end_i];
// lane j also owns Jacobian column j.  Structure of arrays, 64 per field.
//   li[f*64 + i]: f = 0 link (-1 past the robot), 1 parent lane (-1 root),
//                 2 last lane of the subtree, 3 joint index (-1 fixed),
//                 4 revolute, 5 fixed rotation is the identity,
//                 6 first sphere, 7 sphere count
//   lf[f*64 + i]: f = 0..2 axis, 3..11 fixed R (row-major), 12..14 fixed p,
//                 15 joint multiplier, 16 joint offset, 17 mass, 18..20 CoM
//   conn[k*64 + j]: lane of the k-th link whose angle joint j sets
//                 (connectedLinks[j]), -1 past the end of the list
// Lanes past the robot hold a massless link with no joint, no parent and an
// identity fixed transform.
struct DevKin {
    int32_t L, n, G, jsteps, mc;      // G lanes per state; mc: longest connectedLinks list
    float inv_mass;                   // 1 / total mass, 0 for a massless robot
    const int32_t *__restrict__ li;
    const float *__restrict__ lf;
    const int32_t *__restrict__ conn;
    const float4 *__restrict__ sph;   // [S] local centre and radius
    int32_t n_tools;
    const int32_t *__restrict__ tool_lane;   // [n_tools] lane of the tool's link
    const float *__restrict__ tool_off;      // [n_tools][12] offset R (row-major) then p
    const uint64_t *__restrict__ tool_aff;   // [n_tools] bit j set: joint j affects the tool's link
};

// Outputs of the forward call (each null to skip).
struct KinOut {
    float *link_pose;   // [L][12][B]
    float *spheres;     // [S][3][B]
    float *tool_pose;   // [T][12][B]
    float *com;         // [3][B]
    float *jac;         // [B][T][6][n] (state-major)
    float *com_jac;     // [B][3][n] (state-major)
};

// Inputs and output of the backward call.
struct KinGrad {
    const float *g_tool;   // [T][12][B] or null
    const float *g_com;    // [3][B] or null
    float *g_q;            // [n][B], overwritten
};

// ld: row length of the [k][B] arrays (the state-major Jacobians are dense).
hipError_t launch_kinematics(const DevKin &k, int64_t B, int64_t ld, const float *q, const KinOut &o,
                             hipStream_t s);
hipError_t launch_kinematics_backward(const DevKin &k, int64_t B, const float *q, const KinGrad &g,
                                      hipStream_t s);

}  // namespace wb
