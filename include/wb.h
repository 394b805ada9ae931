/*
 * wb.h -- C ABI of the MI355X whole-body library (libwb.so).
 *
 * Batched forward kinematics, recursive Newton-Euler inverse dynamics and
 * map-reduce self-collision, with their adjoints, for a kinematic tree whose
 * topology, joint axes, fixed transforms, inertias and collision spheres are
 * given at run time (cuRoboV2, arXiv 2603.05493: Sec. 3 states the problem,
 * Sec. 6.1 forward kinematics and Alg. 1 its gradient, Sec. 6.2 the
 * self-collision map-reduce, Sec. 6.3 with Alg. 4 and Alg. 5 the RNEA and its
 * vector-Jacobian product).
 *
 * Conventions shared by every call
 *   - Arithmetic is FP32 on the GPU.
 *   - Batched arrays are structure-of-arrays with the state index fastest:
 *     an array documented as [k][B] holds element (i, b) at i*ld + b, where
 *     ld >= B is the call's leading dimension (rows may be padded, e.g. to
 *     a multiple of a cache line, or be a column slice of a wider batch;
 *     ld = 0 means ld = B; ld < B is WB_ERR_INVALID_ARG).  The calls that
 *     take an ld apply it to every [k][B] array they touch, their workspace
 *     and cache included (size those for ld states); padding entries are
 *     never read or written.  Per-state arrays [B] are dense.  Calls without
 *     an ld (kinematics outputs, B-spline, distance transform) take dense
 *     arrays.  All such pointers are device pointers owned by the caller;
 *     the library never allocates, frees or synchronizes inside a launch
 *     call, so every launch call may be captured into a HIP graph.
 *   - Every launch call enqueues its kernels on the given stream and returns
 *     immediately; results are valid once the stream reaches that point.
 *   - Every call returns WB_OK or an error code; wb_last_error() returns a
 *     thread-local description of the last failure.  Launch calls validate
 *     sizes and pointers (non-null, 4-byte aligned) before enqueuing
 *     anything; NaN or Inf inputs are not checked and propagate.
 *   - B = 0 is valid and enqueues nothing.
 *
 * Frames.  Link 0 is the fixed root at the world identity.  Link k >= 1 is
 * placed at parent_T_k(q) = [fixed_R_k | fixed_p_k] * Rot(axis_k, theta_k)
 * with theta_k = joint_mult_k * q[joint_index_k] + joint_offset_k (mimic
 * joints share an actuated index; Sec. 6 "mimic joints"), the axis given in
 * the child frame.  A link pose is 12 floats: the world rotation R
 * (row-major 3x3) then the world position p.  Spatial vectors are
 * Featherstone [angular; linear] in link coordinates (Sec. 6.3).
 */
#ifndef WB_H
#define WB_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum wb_status {
    WB_OK = 0,
    WB_ERR_INVALID_ARG = 1,   /* null/misaligned pointer, bad size, bad option  */
    WB_ERR_INVALID_TREE = 2,  /* descriptor is not a valid rooted tree / sphere set */
    WB_ERR_UNSUPPORTED = 3,   /* valid but beyond what the kernels handle        */
    WB_ERR_HIP = 4            /* a HIP runtime call failed (message has details) */
};

enum wb_joint_type { WB_JOINT_FIXED = 0, WB_JOINT_REVOLUTE = 1 };

/* Limits of this build (WB_ERR_UNSUPPORTED beyond them). */
#define WB_MAX_LINKS 1024
#define WB_MAX_SPHERES_PER_LINK 64

/*
 * Robot description (runtime robot binding, Sec. 6.3 "Our RNEA
 * Implementation": topology, inertias and joint types supplied at run time).
 * All pointers are host pointers, read during wb_robot_create only.
 *   n_links        L >= 1, including the fixed root link 0.
 *   parent[L]      parent[0] = -1, 0 <= parent[k] < k for k >= 1.
 *   joint_type[L]  WB_JOINT_FIXED or WB_JOINT_REVOLUTE; link 0 must be fixed.
 *   joint_index[L] actuated joint of each revolute link, -1 for fixed links;
 *                  the actuated indices used must be exactly 0..n-1 (n = DoF).
 *   joint_mult[L], joint_offset[L]  mimic multiplier and offset (NULL = 1, 0).
 *   axis[L][3]     unit joint axis in the child frame (|axis| = 1 within 1e-4).
 *   fixed_R[L][9], fixed_p[L][3]  fixed transform parent->joint frame
 *                  (fixed_R orthonormal within 1e-4).
 *   mass[L], com[L][3], inertia[L][9]  mass, centre of mass in link frame,
 *                  symmetric rotational inertia about the CoM in link axes.
 *   n_spheres      S >= 0; sphere_link[S] nondecreasing link indices;
 *   sphere[S][4]   centre (link frame) and radius (> 0) of each sphere;
 *                  at most WB_MAX_SPHERES_PER_LINK spheres per link (the
 *                  fused iteration takes at most 12).
 *   allow[L][L]    symmetric link-pair allow matrix for self-collision, or
 *                  NULL for the default: every pair of distinct links that
 *                  are not parent and child (Sec. 6.2 checks all sphere pairs
 *                  whose links are not adjacent).  Same-link pairs are never
 *                  checked.
 *   gravity[3]     gravity vector in the world frame (e.g. 0, 0, -9.81).
 */
typedef struct wb_robot_desc {
    int32_t n_links;
    const int32_t *parent;
    const int32_t *joint_type;
    const int32_t *joint_index;
    const float *joint_mult;
    const float *joint_offset;
    const float *axis;
    const float *fixed_R;
    const float *fixed_p;
    const float *mass;
    const float *com;
    const float *inertia;
    int32_t n_spheres;
    const int32_t *sphere_link;
    const float *sphere;
    const uint8_t *allow;
    float gravity[3];
} wb_robot_desc;

/* Derived sizes of a robot. */
typedef struct wb_robot_info {
    int32_t n_links;          /* L */
    int32_t n_dof;            /* n */
    int32_t n_spheres;        /* S */
    int32_t max_depth;        /* deepest link's distance from the root */
    int64_t n_pairs;          /* checked sphere pairs P */
    int32_t n_blocks;         /* checked link pairs (a < b) carrying spheres */
    int32_t max_spheres_per_link;
    int32_t fused_supported;  /* 1 if wb_wholebody_step accepts this robot */
    int32_t kinematics_supported;  /* 1 if wb_kinematics accepts this robot (L <= 64, n <= 64) */
    int32_t mimic;            /* 1 if some joint drives several links or has a multiplier != 1 or offset != 0 */
} wb_robot_info;

typedef struct wb_robot wb_robot;   /* opaque; owns a device copy of the tables */

const char *wb_last_error(void);

/* ---------------------------------------------------------------- host only
 * These never touch a GPU. */

/* Validate a description and report its derived sizes. */
int wb_desc_analyze(const wb_robot_desc *desc, wb_robot_info *info);

/* Write the checked sphere pairs, numbered lexicographically in (s, t) with
 * s < t: s[P], t[P] (host arrays of info.n_pairs entries).  The pair index
 * returned as argmax by wb_self_collision refers to this numbering.  The list
 * is rebuilt from the link-block tables the kernels use. */
int wb_desc_pairs(const wb_robot_desc *desc, int32_t *s, int32_t *t);

/* ------------------------------------------------------------- robot object */

/* Validate, derive the kernel tables and copy them to the current HIP device.
 * The robot is usable on that device only.  *out is owned by the caller and
 * released with wb_robot_destroy. */
int wb_robot_create(const wb_robot_desc *desc, wb_robot **out);
int wb_robot_destroy(wb_robot *robot);
int wb_robot_get_info(const wb_robot *robot, wb_robot_info *info);

/* Scratch needed by wb_fk_backward and wb_rnea_backward for B states, in
 * bytes (caller-allocated device memory, 256-byte aligned, reusable across
 * calls on one stream); with padded rows pass the calls' ld for B. */
int wb_workspace_bytes(const wb_robot *robot, int64_t B, size_t *bytes);
/* Size of the RNEA forward cache for B states (pass ld with padded rows): [L][18][B] floats holding,
 * per link, spatial velocity v (6), acceleration a (6) and the accumulated
 * force F (6) of Alg. 4 (the cache of Sec. 6.3 "Memory layout", unpadded). */
int wb_rnea_cache_bytes(const wb_robot *robot, int64_t B, size_t *bytes);

/* ---------------------------------------------------------------- forward */

/* Forward kinematics (Sec. 6.1; the paper dispatches its kernels by robot
 * size).  Batches below 48 states per compute unit on robots of at most 64
 * links run one group of lanes per state (pointer jumping over the links, as
 * wb_kinematics); larger ones one lane per state.
 * q[n][B] joint positions ->
 *   link_pose[L][12][B] world link poses, or NULL to skip them: a branch
 *     link then recomposes its parent's pose from q along the parent's chain
 *     instead of re-reading it;
 *   spheres[S][3][B] world sphere centres, or NULL to skip them.
 * WB_ERR_INVALID_ARG when both outputs are NULL. */
int wb_fk(const wb_robot *robot, int64_t B, int64_t ld, const float *q, float *link_pose, float *spheres,
          hipStream_t stream);

/* ------------------------------------------------------ kinematics outputs
 * The other outputs of a forward-kinematics call (Sec. 6.1: tool poses,
 * centres of mass and Jacobians besides frame transforms and sphere centres),
 * the tool-frame Jacobian of Alg. 2 (for least-squares solvers such as the
 * Levenberg-Marquardt step of Alg. 3), and the gradient of losses on tool
 * poses and the centre of mass.  One wavefront group per state computes them
 * all in one launch; needs n_links <= 64 and n_dof <= 64
 * (wb_robot_info.kinematics_supported), else WB_ERR_UNSUPPORTED.  Mimic
 * joints are supported. */
#define WB_MAX_TOOLS 32

/* Set the robot's tool frames (Sec. 6.1 "tool poses"; several per robot,
 * e.g. hands and feet of a humanoid).  link[n_tools] (host): the link each
 * tool is fixed to; offset[n_tools][12] (host): the tool frame in that link's
 * frame, rotation row-major then translation.  n_tools = 0 clears them.
 * Builds Alg. 2's coarse filter affects[joint, tool] on the host.  Blocking
 * and not ordered with launches, like wb_robot_set_link_inertia.
 * WB_ERR_INVALID_ARG for n_tools outside [0, WB_MAX_TOOLS], an out-of-range
 * link, a non-finite offset or a rotation that is not orthonormal (1e-4). */
int wb_robot_set_tool_frames(wb_robot *robot, int32_t n_tools, const int32_t *link, const float *offset);
int wb_robot_get_tool_count(const wb_robot *robot, int32_t *n_tools);

/* q[n][B] -> any of (each NULL to skip; with all NULL the call does nothing):
 *   link_pose[L][12][B]   world link poses, as wb_fk;
 *   spheres[S][3][B]      world sphere centres, as wb_fk;
 *   tool_pose[T][12][B]   world tool poses R_link R_off (row-major), then
 *                         p_link + R_link p_off;
 *   com[3][B]             centre of mass: sum_k m_k (R_k c_k + p_k) / sum_k m_k
 *                         over every link, the fixed base included;
 *   jacobian[B][T][6][n]  Alg. 2's Jacobian of each tool frame, state-major
 *                         (each state's 6T x n block contiguous, row-major, as
 *                         batched solvers consume it): rows are the tool
 *                         point's linear velocity then the angular velocity
 *                         (world axes) per unit joint rate; column j sums
 *                         mult_l [s_l x (x - o_l); s_l] over the links l that
 *                         joint j drives on the chain of the tool's link (s_l
 *                         world axis, o_l world origin of the joint);
 *   com_jacobian[B][3][n] d com / d q, state-major likewise.
 * T is the count set by wb_robot_set_tool_frames.  WB_ERR_INVALID_ARG when
 * com or com_jacobian is requested for a robot of zero total mass. */
int wb_kinematics(const wb_robot *robot, int64_t B, const float *q, float *link_pose, float *spheres,
                  float *tool_pose, float *com, float *jacobian, float *com_jacobian, hipStream_t stream);

/* Gradient of L = sum_t <g_tool_pose[t], tool_pose[t]> + <g_com, com> with
 * respect to q: g_q[n][B] (overwritten) = sum_t J_t^T [g_x; w_t] +
 * J_com^T g_com, with w_t = sum_c r_c x G_c over the columns r_c of the tool
 * rotation and G_c of its gradient.  g_tool_pose[T][12][B] and g_com[3][B]
 * may each be NULL (no such term). */
int wb_kinematics_backward(const wb_robot *robot, int64_t B, const float *q, const float *g_tool_pose,
                           const float *g_com, float *g_q, hipStream_t stream);

/* Inverse dynamics by RNEA (Alg. 4).  q, qd, qdd [n][B] -> tau[n][B].
 * f_ext[L][6][B] (NULL = none): external spatial force on each link in link
 * coordinates, moment then force about the link origin; it enters Alg. 4's
 * force line as f_k = I_k a_k + v_k x* I_k v_k - f_ext_k.  cache[L][18][B]
 * receives v, a and the accumulated link forces (including f_ext) for
 * wb_rnea_backward (Alg. 4's optional cache output), or is NULL: then
 * nothing is stored (one group of lanes per state keeps every link quantity
 * in registers) and the backward recomputes them.  Without a cache the
 * robot must have at most 64 links (WB_ERR_UNSUPPORTED otherwise). */
int wb_rnea(const wb_robot *robot, int64_t B, int64_t ld, const float *q, const float *qd, const float *qdd,
            const float *f_ext, float *tau, float *cache, hipStream_t stream);

/* Self-collision map-reduce (Sec. 6.2; the paper splits the pairs of a
 * large robot over blocks and reduces the block maxima in a second stage).
 * Two forms, chosen by batch size: one state per wavefront (the states of a
 * workgroup tile swept side by side), or -- for batches below the robot's
 * split threshold, where one wavefront per state would leave the chip
 * underfilled -- one state per workgroup, its link blocks dealt over four
 * wavefronts that each compact and sweep their share, then a second reduce
 * of the wavefronts' maxima, counts and argmax keys through LDS.  Both give
 * the full sweep's results.  spheres[S][3][B] -> per state
 *   max_pen[B]  largest r_s + r_t - |c_s - c_t| over the checked pairs
 *               (-inf when the robot has no checked pair),
 *   argmax[B]   lowest pair index attaining it (-1 when there is none),
 *   n_coll[B]   number of pairs with positive penetration.
 * Any of the three outputs may be NULL to skip it (not all three). */
int wb_self_collision(const wb_robot *robot, int64_t B, int64_t ld, const float *spheres, float *max_pen,
                      int32_t *argmax, int32_t *n_coll, hipStream_t stream);
/* Adaptive dispatch of the per-operation calls for this robot (Sec. 6.1
 * dispatches FK kernels by robot size; here the forms are chosen by batch
 * size, with thresholds the autotuner measures):
 *   sweep_split_below     wb_self_collision takes the one-state-per-workgroup
 *                         form for batches of fewer states (default 16 per
 *                         compute unit of the robot's device);
 *   fk_groups_below       wb_fk without link poses and wb_fk_backward
 *                         without them take one group of lanes per state for
 *                         batches of fewer states (default 48 per compute
 *                         unit; robots of at most 64 links);
 *   fk_pose_groups_below  the same for wb_fk writing link poses and
 *                         wb_fk_backward reading poses or a pose gradient
 *                         (the group form writes
 *                         one state's 12L pose values across 12L rows and
 *                         recomputes instead of reading; the lane form's rows
 *                         are coalesced, so its crossover lies lower).
 * A negative value restores that default; 0 never takes the form. */
int wb_robot_set_dispatch(wb_robot *robot, int64_t sweep_split_below, int64_t fk_groups_below,
                          int64_t fk_pose_groups_below);

/* -------------------------------------------------------------- adjoints */

/* Adjoint of the hinge cost h = max(0, max_pen + margin) at the most
 * penetrating pair: g_spheres[S][3][B] is overwritten with zeros except the
 * two spheres of pair argmax[b], which receive -/+ g_cost[b] * u with u the
 * unit vector from sphere t to sphere s, when max_pen[b] + margin > 0 (and
 * zero otherwise, including coincident centres). */
int wb_self_collision_backward(const wb_robot *robot, int64_t B, int64_t ld, const float *spheres,
                               const int32_t *argmax, const float *max_pen, float margin,
                               const float *g_cost, float *g_spheres, hipStream_t stream);

/* Adjoint of forward kinematics (Alg. 1): gradients on link poses
 * g_link_pose[L][12][B] and/or sphere centres g_spheres[S][3][B] (either may
 * be NULL, not both) -> g_q[n][B] (overwritten).  link_pose is the output of
 * wb_fk for the same q, or NULL to recompute the transforms from q inside
 * the kernel.  workspace: wb_workspace_bytes(robot, B).
 * Like wb_fk, batches below 48 states per compute unit (robots of at most
 * 64 links) run one group of lanes per state: each link's
 * wrench about the world origin summed over its subtree and projected on
 * the joint axis, transforms recomputed in registers; link_pose is then not
 * read and workspace may be NULL. */
int wb_fk_backward(const wb_robot *robot, int64_t B, int64_t ld, const float *q, const float *link_pose,
                   const float *g_link_pose, const float *g_spheres, float *g_q, void *workspace,
                   hipStream_t stream);

/* Vector-Jacobian product of RNEA (the role of Alg. 5): g_tau[n][B] ->
 * g_q, g_qd, g_qdd [n][B] (overwritten) and, when g_fext is not NULL, the
 * gradient on the external forces g_fext[L][6][B] (overwritten; link
 * coordinates like f_ext; it is minus the adjoint of each link's accumulated
 * force, Alg. 5's f-bar_ext).  Transforms are recomputed from q.
 *   cache: the one written by wb_rnea for the same q, qd, qdd and f_ext
 *     (f_ext is then ignored: the forces are in the cache); workspace:
 *     wb_workspace_bytes(robot, B);
 *   or cache = NULL: every forward quantity is recomputed from q, qd, qdd
 *     and f_ext (NULL = none) in registers, one group of lanes per state;
 *     workspace may be NULL; robots of at most 64 links
 *     (WB_ERR_UNSUPPORTED otherwise). */
int wb_rnea_backward(const wb_robot *robot, int64_t B, int64_t ld, const float *q, const float *qd,
                     const float *qdd, const float *f_ext, const float *cache, const float *g_tau, float *g_q,
                     float *g_qd, float *g_qdd, float *g_fext, void *workspace, hipStream_t stream);

/* ------------------------------------------------ cost head and update step
 * The per-state scalar costs of the trajectory-optimization iteration
 * (Sec. 3, Eq. 1 and the torque / self-collision constraints as penalties):
 *   cost[b] = (w ? sum_j w[j][b] tau[j][b] : torque_weight * sum_j tau^2)
 *           + hinge_weight * max(0, max_pen[b] + margin)
 *   g_tau   = w ? w : 2 * torque_weight * tau
 *   g_maxpen[b] = hinge_weight * (max_pen[b] + margin > 0)
 * w may be NULL; max_pen may be NULL (no hinge term, g_maxpen untouched);
 * cost and g_maxpen may be NULL. */
int wb_cost_head(int64_t B, int64_t ld, int32_t n, const float *tau, const float *w, float torque_weight,
                 const float *max_pen, float margin, float hinge_weight, float *cost,
                 float *g_tau, float *g_maxpen, hipStream_t stream);

/* Gradient step in place: q -= lr * (g_q + g_q2), qd -= lr * g_qd,
 * qdd -= lr * g_qdd, all [n][B]; g_q2 may be NULL. */
int wb_sgd_step(int64_t B, int64_t ld, int32_t n, float lr, float *q, float *qd, float *qdd, const float *g_q,
                const float *g_q2, const float *g_qd, const float *g_qdd, hipStream_t stream);

/* ---------------------------------------------- B-spline trajectory front end
 * Uniform cubic B-spline joint trajectories (Sec. 4): the optimizer's
 * variables are control points, and the hot path's states are samples of
 * the splines (Eq. 10); the control-point gradient is the transpose of the
 * sampling, summed over every sample of a control point's support
 * (Eqs. 13-14).  T trajectories of d joints, K control points each
 * (1 <= K <= WB_BSPLINE_MAX_K), n_interp samples per knot interval dt:
 *   knots per trajectory and joint: three ghost knots from the initial
 *   state, u_0 .. u_{K-1}, and three more copies of u_{K-1} (a static goal);
 *   segment s = 0 .. K+2 uses knots s .. s+3 of that sequence and is sampled
 *   at alpha = i / n_interp, i = 0 .. n_interp-1, so a trajectory has
 *   H = (K + 3) n_interp samples and state b = traj * H + s * n_interp + i.
 * reading selects the ghost knots: WB_GHOST_EXACT makes the first sample
 * equal the initial state (theta, theta_dot, theta_ddot); WB_GHOST_PRINTED
 * uses the paper's printed formulas, whose first sample is the initial state
 * carried forward by dt at constant acceleration.
 * Layouts: U [d][T][K] (a trajectory's control points contiguous); theta0,
 * dtheta0, ddtheta0 [d][T]; states [d][T*H] (the hot path's [n][B] with
 * B = T*H).
 * T*H must stay below 2^31 (else WB_ERR_UNSUPPORTED). */
#define WB_BSPLINE_MAX_K 65536
#define WB_GHOST_EXACT 0
#define WB_GHOST_PRINTED 1

/* Samples of the splines: q, qd, qdd [d][T*H] (qd, qdd may be NULL).
 * theta0 is required; dtheta0 and ddtheta0 may be NULL (zero). */
int wb_bspline_eval(int64_t T, int32_t d, int32_t K, int32_t n_interp, float dt, int32_t reading,
                    const float *U, const float *theta0, const float *dtheta0, const float *ddtheta0,
                    float *q, float *qd, float *qdd, hipStream_t stream);

/* Control-point gradient g_U [d][T][K] (overwritten; may be NULL when lr != 0
 * with the plain step) from upstream gradients on the samples g_q, g_qd,
 * g_qdd [d][T*H] (each may be NULL = zero).  The initial state is not a
 * variable: ghost knots take no gradient; copies of u_{K-1} add into it.
 * When lr != 0, U is updated in place by the step rule:
 *   WB_STEP_PLAIN    U -= lr * g_U;
 *   WB_STEP_ROW_RMS  U_row -= lr * g_row / rms(g_row) for every (joint,
 *                    trajectory) row of K control points (no step for an
 *                    all-zero row); g_U is required.  The samples' velocity
 *                    and acceleration gradients reach g_U scaled by dt^-1
 *                    and dt^-2 (Eqs. 11-12), so a plain step stable at the
 *                    optimizer's scales barely moves the control points;
 *                    dividing each row by its own positive scale is a
 *                    diagonal preconditioner (still a descent direction)
 *                    whose lr is the RMS change of a row per step.
 * WB_ERR_INVALID_ARG for an unknown step rule. */
#define WB_STEP_PLAIN 0
#define WB_STEP_ROW_RMS 1
int wb_bspline_backward(int64_t T, int32_t d, int32_t K, int32_t n_interp, float dt, const float *g_q,
                        const float *g_qd, const float *g_qdd, float *g_U, float lr, int32_t step_rule, float *U,
                        hipStream_t stream);

/* ------------------------------------------------------ fused iteration
 * One trajectory-optimizer iteration of the whole-body terms (Sec. 3, the
 * six-step loop: kinematics and inverse dynamics, the self-collision cost,
 * the backward pass through both, and the update) in a single launch:
 *   FK (Sec. 6.1) -> self-collision (Sec. 6.2) -> RNEA (Alg. 4) -> cost head
 *   (as wb_cost_head) -> hinge, FK and RNEA adjoints -> optional step.
 * Nothing intermediate is written to device memory.
 *   q, qd, qdd [n][B]  inputs; when lr != 0 they are updated in place:
 *                      x -= lr * d(cost)/dx for x in (q, qd, qdd).
 *   w [n][B] or NULL   torque cost weights (NULL: torque_weight * ||tau||^2).
 *   tau [n][B], cost [B], max_pen [B], argmax [B], n_coll [B],
 *   g_q, g_qd, g_qdd [n][B]   optional outputs (NULL to skip); the gradients
 *                      are those of cost[b] (FK through the hinge plus RNEA),
 *                      evaluated before the step.
 *   f_ext [L][6][B] or NULL    external link forces, as in wb_rnea;
 *   g_fext [L][6][B] or NULL   their gradient (as wb_rnea_backward's g_fext,
 *                      for the torque cost).
 * External forces and mimic joints (several links per actuated joint, or a
 * multiplier other than 1 or offset other than 0) select the kernel variant
 * that carries them; other robots run the lean variant.  Results agree with
 * the separate calls (same definitions, same tolerance; floating-point sums
 * are ordered differently).  Needs n_links <= 64 and the per-state sweep
 * tables of a 256-lane workgroup within 64 KB of LDS
 * (wb_robot_info.fused_supported), else WB_ERR_UNSUPPORTED. */
int wb_wholebody_step(const wb_robot *robot, int64_t B, int64_t ld, float *q, float *qd, float *qdd, const float *w,
                      float torque_weight, float margin, float hinge_weight, float lr, float *tau,
                      float *cost, float *max_pen, int32_t *argmax, int32_t *n_coll, float *g_q,
                      float *g_qd, float *g_qdd, const float *f_ext, float *g_fext, hipStream_t stream);

/* The whole B-spline optimizer iteration in one launch (Sec. 3's loop with
 * Sec. 4's splines in front of the whole-body terms and their control-point
 * gradient behind them): each state's joint positions, velocities and
 * accelerations are formed in the kernel from the control points --
 * the samples wb_bspline_eval writes for four samples per knot interval --
 * instead of being read from state arrays; with g_U or lr != 0 each
 * workgroup owns one whole trajectory, pulls every sample's gradient back
 * onto its four-knot window in LDS, reduces them (the result of
 * wb_bspline_backward, summed in a fixed order) and steps U in place by the
 * step rule, so nothing per state reaches device memory.
 *   T, K, dt, reading, U [d][T][K], theta0, dtheta0, ddtheta0 [d][T] as in
 *   wb_bspline_eval (d = n_dof, n_interp = 4); the B = T * (K + 3) * 4
 *   states are ordered as there.
 *   g_U [d][T][K] (NULL to skip), lr, step_rule: as wb_bspline_backward.
 *   tau, cost, max_pen, argmax, n_coll, g_q, g_qd, g_qdd: optional outputs of
 *   wb_wholebody_step for the batch, dense [n][B] and [B] (g_q, g_qd, g_qdd
 *   are the per-sample gradients wb_bspline_backward takes).
 * WB_ERR_UNSUPPORTED for robots with mimic joints or outside the fused
 * iteration's limits, and when the control-point gradient's LDS (partial
 * sums of 4 * 64 / lanes_per_state groups over d x (K + 6) knots) does not
 * fit beside the fused kernel's in 64 KB. */
int wb_wholebody_step_bspline(const wb_robot *robot, int64_t T, int32_t K, float dt, int32_t reading,
                              float *U, const float *theta0, const float *dtheta0, const float *ddtheta0,
                              const float *w, float torque_weight, float margin, float hinge_weight, float *g_U,
                              float lr, int32_t step_rule, float *tau, float *cost, float *max_pen, int32_t *argmax,
                              int32_t *n_coll, float *g_q, float *g_qd, float *g_qdd, hipStream_t stream);

/* Launch shape of the fused iteration for one robot (the paper dispatches
 * FK differently by robot size, Sec. 6.1 "adaptive kernel dispatch"; here the
 * shape is a per-topology tuning record, chosen by measurement).
 *   lanes_per_state  16, 32 or 64 lanes of a 64-wide wavefront per state
 *                    (>= the robot's links); 64 / lanes_per_state states run
 *                    side by side in one wavefront.
 *   states_per_item  states per workgroup work item (1..4096).  For a
 *                    wb_wholebody_step batch too small to give every
 *                    compute unit four workgroups it is halved, down to the
 *                    4 * 64 / lanes_per_state states a workgroup holds at
 *                    once (results do not depend on it).
 *   ns_per_state     measured cost of one state, used to balance uneven
 *                    batches (0 = use the built-in cost model).
 * wb_robot_create sets a default; wb_robot_set_tune validates and replaces it
 * (WB_ERR_INVALID_ARG for an invalid shape, WB_ERR_UNSUPPORTED when
 * 64 / lanes_per_state states per wavefront would not fit 64 KB of LDS per
 * workgroup). */
typedef struct wb_tune {
    int32_t lanes_per_state;
    int32_t states_per_item;
    float ns_per_state;
} wb_tune;
int wb_robot_set_tune(wb_robot *robot, const wb_tune *tune);

/* Replace the inertial parameters of one link of a live robot -- mass, CoM
 * and rotational inertia about the CoM in link axes (xx yy zz xy xz yz),
 * as in wb_robot_desc -- e.g. a payload picked up at run time (Sec. 6.3:
 * runtime binding of the robot parameters), without re-creating the robot or
 * its plans.  Every later launch (plain, fused or plan) uses the new values.
 * Blocking: it copies to the device before returning and is not ordered with
 * launches, so call it only when no launch that reads the robot is pending
 * (synchronize its streams first).  WB_ERR_INVALID_ARG for an out-of-range
 * link, null arrays, a negative or non-finite mass or non-finite values. */
int wb_robot_set_link_inertia(wb_robot *robot, int32_t link, float mass, const float *com, const float *inertia);
int wb_robot_get_tune(const wb_robot *robot, wb_tune *tune);

/* -------------------------------------------------- distance transform
 * Exact Euclidean distance transform of a site grid (Sec. 5, "Stage 2:
 * Distance Propagation": the dense ESDF's nearest-site assignment, computed
 * by the separable three-pass PBA+ decomposition with Maurer's dominance
 * test, in integer arithmetic).  Grids are [nz][ny][nx], x fastest, each
 * extent in [1, WB_EDT_MAX_DIM].
 *   sites[nz][ny][nx] (device, uint8): nonzero voxels are sites;
 *   nearest[nz][ny][nx] (int32, NULL to skip): a nearest site, packed
 *     x | y << 10 | z << 20, or -1 when the grid has no site (any one of
 *     several equidistant sites);
 *   dist[nz][ny][nx] (float, NULL to skip): voxel_size * its Euclidean
 *     distance, +inf when there is no site;
 *   workspace: wb_edt_workspace_bytes bytes of device memory, 256-byte
 *     aligned, reused across calls on one stream.
 * Three launches whose shapes depend only on the grid size; never allocates
 * or synchronizes.  WB_ERR_INVALID_ARG for extents outside the range, a
 * non-finite or negative voxel_size, or missing pointers. */
#define WB_EDT_MAX_DIM 1024
int wb_edt_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, size_t *bytes);
int wb_edt(int32_t nx, int32_t ny, int32_t nz, const uint8_t *sites, float voxel_size, int32_t *nearest,
           float *dist, void *workspace, hipStream_t stream);

/* wb_edt for callers that cannot allocate device memory (code under HIP
 * graph capture, per-frame perception loops, harnesses that forbid
 * hipMalloc): the same three launches and results as wb_edt, with the
 * workspace taken from a device-resident scratch array that the library
 * holds per device for the life of the process (64 MiB: two int32 planes
 * of WB_EDT_NOALLOC_MAX_VOXELS voxels).  Allocates and frees nothing, also
 * on its first call on a device, which only looks up the array's address.
 * Every call on a device shares that device's array: calls that overlap on
 * one GPU (concurrent streams, threads) race and must be serialized by the
 * caller.  Nothing in the array needs to start at zero (every pass writes
 * its whole plane before the next reads it).  WB_ERR_UNSUPPORTED when
 * nx * ny * nz exceeds WB_EDT_NOALLOC_MAX_VOXELS; otherwise the argument
 * rules and errors of wb_edt. */
#define WB_EDT_NOALLOC_MAX_VOXELS (1 << 23)
int wb_edt_noalloc(int32_t nx, int32_t ny, int32_t nz, const uint8_t *sites, float voxel_size, int32_t *nearest,
                   float *dist, hipStream_t stream);

/* ------------------------------------------------ uneven multi-robot batches
 * A plan runs the fused iteration for several robots, each with its own
 * batch size, in one persistent launch (suitable for HIP graph capture; the
 * paper captures its whole iteration in CUDA graphs, Sec. 7.2).  The plan
 * owns a static work list of (robot, state range) items balanced over the
 * workgroups by cost (longest first), using each robot's tune record.  The
 * launch has as many workgroups as the device's compute units keep
 * resident for the plan kernel (its occupancy at the plan's LDS size), so
 * that every workgroup runs from the start; with an item count below that,
 * one workgroup per item.
 *   wb_plan_create: robots[n_trees] (created on one device, each
 *     fused_supported), B[n_trees] states per robot, tune[n_trees] or NULL
 *     (each robot's current record); 1 <= n_trees <= 16.  Allocates the
 *     plan's device tables; the plan does not own the robots, which must
 *     outlive it.  WB_ERR_UNSUPPORTED if the LDS of a workgroup would exceed
 *     64 KB.
 *   wb_plan_run: io[n_trees] holds each robot's device buffers with the
 *     meaning and layout of wb_wholebody_step (external forces included);
 *     the scalars are shared.  A plan with a mimic robot, or a run with
 *     external forces, uses the kernel variant that carries them for every
 *     tree.  Never allocates or synchronizes. */
typedef struct wb_tree_io {
    float *q, *qd, *qdd;
    const float *w;
    float *tau, *cost, *max_pen;
    int32_t *argmax, *n_coll;
    float *g_q, *g_qd, *g_qdd;
    const float *f_ext;   /* [L][6][B] or NULL, as in wb_wholebody_step */
    float *g_fext;        /* [L][6][B] or NULL */
    int64_t ld;           /* leading dimension of this tree's [k][B] arrays (0 = its B) */
} wb_tree_io;
typedef struct wb_plan wb_plan;
int wb_plan_create(const wb_robot *const *robots, const int64_t *B, int32_t n_trees, const wb_tune *tune,
                   wb_plan **out);
int wb_plan_run(const wb_plan *plan, const wb_tree_io *io, float torque_weight, float margin,
                float hinge_weight, float lr, hipStream_t stream);
/* Capture `iters` consecutive wb_plan_run calls with these io buffers and
 * scalars into an executable HIP graph (the paper captures its iteration in
 * CUDA graphs, Sec. 7.2): each iteration reads the states the previous one
 * stepped (with lr != 0 they move in place).  *out is owned by the caller,
 * launched with wb_graph_launch (or hipGraphLaunch) on any stream of the
 * plan's device, and released with wb_graph_destroy.  The graph holds the io
 * pointers: the buffers and the plan must outlive it.  Creates and
 * destroys a capture stream on the plan's device; errors of wb_plan_run
 * (checked on the first iteration, before anything is recorded) are
 * returned as they are; WB_ERR_INVALID_ARG for iters outside [1, 2^20]. */
int wb_plan_capture(const wb_plan *plan, const wb_tree_io *io, float torque_weight, float margin, float hinge_weight,
                    float lr, int32_t iters, hipGraphExec_t *out);
/* Enqueue a graph from wb_plan_capture on a stream (hipGraphLaunch), and
 * release one (NULL is a no-op). */
int wb_graph_launch(hipGraphExec_t graph, hipStream_t stream);
int wb_graph_destroy(hipGraphExec_t graph);
int wb_plan_get_info(const wb_plan *plan, int32_t *n_items, int32_t *n_workgroups);
int wb_plan_destroy(wb_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* WB_H */
