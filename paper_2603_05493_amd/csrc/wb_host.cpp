// Host side of libwb: descriptor validation, derived kernel tables, device
// upload and the extern "C" entry points declared in include/wb.h.
#include "wb.h"
#include "edt.h"
#include "edt_scratch.h"
#include "kin.h"
#include "wb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(WB_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Everything derived from a descriptor, in host memory.
struct Tables {
    int L = 0, n = 0, S = 0, nmax = 1, most = 1, max_depth = 0, simple = 1;   // nmax: slots per link; most: spheres
    std::vector<wb::LinkF> lf;
    std::vector<wb::LinkI> li;
    std::vector<float4> sph;
    std::vector<int32_t> sph_link, sph_slot;
    std::vector<float> slot_r;
    std::vector<int32_t> blocks;      // padded to a multiple of 64
    int n_blocks = 0;
    int list_cap = 64;                // ints of the sweep's per-group LDS list
    std::vector<int32_t> pair_off, pair_cnt, pair_s, pair_t;
    int64_t n_pairs = 0;
    float g[3] = {0, 0, 0};
    // lane tables (depth-first lane order) of the group-per-state kernels:
    // built for every robot of at most 64 links (lanes); the fused iteration
    // additionally needs its sweep tables within the LDS budget (fused)
    int lanes = 0, fused = 0, jsteps = 0;
    std::vector<int> lane_of;         // link -> lane of the fused tables
    std::vector<int32_t> f_li;
    std::vector<float> f_lf;
    std::vector<float4> f_sph;
    int f_mimic = 0, f_mc = 1;        // mimic joints present; longest connectedLinks list
    std::vector<int32_t> f_conn;      // [f_mc][64] lanes of each joint's links
    // lane tables of the kinematics-outputs kernel (same depth-first order)
    int kin = 0, kin_G = 0, kin_jsteps = 0, kin_mc = 0;
    std::vector<int> kin_lane, kin_sub_end;   // link -> lane, lane -> last lane of its subtree
    std::vector<int32_t> k_li, k_conn;
    std::vector<float> k_lf;
    double total_mass = 0.0;
};

bool finite_all(const float *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Lane tables of the fused kernel: links in depth-first pre-order so every
// subtree is a contiguous lane range.
// Depth-first pre-order of the links (children in index order): perm[i] is
// the link of lane i, lane_of its inverse, size[k] the size of k's subtree.
void dfs_lanes(const Tables &T, std::vector<int> &perm, std::vector<int> &lane_of, std::vector<int> &size) {
    const int L = T.L;
    std::vector<std::vector<int>> kids(L);
    for (int k = 1; k < L; ++k) kids[T.li[k].parent].push_back(k);
    perm.clear();
    std::vector<int> stack{0};
    while (!stack.empty()) {
        const int k = stack.back();
        stack.pop_back();
        perm.push_back(k);
        for (auto it = kids[k].rbegin(); it != kids[k].rend(); ++it) stack.push_back(*it);
    }
    lane_of.assign(L, 0);
    for (int i = 0; i < L; ++i) lane_of[perm[i]] = i;
    size.assign(L, 1);
    for (int k = L - 1; k >= 1; --k) size[T.li[k].parent] += size[k];
}

int pointer_jump_steps(int max_depth) {
    int js = 0;
    while ((1 << js) < max_depth + 1) ++js;
    return js;
}

// Lane tables of the kinematics-outputs kernel (layout in kin.h): any robot
// with at most 64 links and 64 joints, mimic joints included.
void build_kin(Tables &T) {
    const int L = T.L, n = T.n;
    T.kin = 0;
    T.total_mass = 0.0;
    for (int k = 0; k < L; ++k) T.total_mass += T.lf[k].mass;
    if (L > 64 || n > 64) return;
    std::vector<int> perm, size;
    dfs_lanes(T, perm, T.kin_lane, size);
    T.kin_sub_end.assign(64, 0);
    std::vector<std::vector<int>> conn(n);
    T.k_li.assign(8 * 64, 0);
    T.k_lf.assign(21 * 64, 0.0f);
    for (int i = 0; i < 64; ++i) {
        T.kin_sub_end[i] = i;
        T.k_li[0 * 64 + i] = -1;
        T.k_li[1 * 64 + i] = -1;
        T.k_li[2 * 64 + i] = i;
        T.k_li[3 * 64 + i] = -1;
        T.k_li[5 * 64 + i] = 1;
        for (int c = 0; c < 9; c += 4) T.k_lf[(3 + c) * 64 + i] = 1.0f;
        T.k_lf[15 * 64 + i] = 1.0f;
    }
    for (int i = 0; i < L; ++i) {
        const int k = perm[i];
        const wb::LinkI &I = T.li[k];
        const wb::LinkF &F = T.lf[k];
        const bool rev = k > 0 && I.revolute && I.jidx >= 0;
        T.kin_sub_end[i] = i + size[k] - 1;
        T.k_li[0 * 64 + i] = k;
        T.k_li[1 * 64 + i] = k == 0 ? -1 : T.kin_lane[I.parent];
        T.k_li[2 * 64 + i] = i + size[k] - 1;
        T.k_li[3 * 64 + i] = rev ? I.jidx : -1;
        T.k_li[4 * 64 + i] = rev ? 1 : 0;
        T.k_li[5 * 64 + i] = k == 0 ? 1 : I.fR_identity;
        T.k_li[6 * 64 + i] = I.sph_first;
        T.k_li[7 * 64 + i] = I.sph_count;
        for (int c = 0; c < 3; ++c) T.k_lf[(0 + c) * 64 + i] = F.axis[c];
        for (int c = 0; c < 9; ++c) T.k_lf[(3 + c) * 64 + i] = k == 0 ? (c % 4 == 0 ? 1.0f : 0.0f) : F.fR[c];
        for (int c = 0; c < 3; ++c) T.k_lf[(12 + c) * 64 + i] = k == 0 ? 0.0f : F.fp[c];
        T.k_lf[15 * 64 + i] = F.mult;
        T.k_lf[16 * 64 + i] = F.offset;
        T.k_lf[17 * 64 + i] = F.mass;
        for (int c = 0; c < 3; ++c) T.k_lf[(18 + c) * 64 + i] = F.com[c];
        if (rev) conn[I.jidx].push_back(i);
    }
    int mc = 1;
    for (int j = 0; j < n; ++j) mc = std::max(mc, (int)conn[j].size());
    T.kin_mc = mc;
    T.k_conn.assign((size_t)mc * 64, -1);
    for (int j = 0; j < n; ++j)
        for (size_t c = 0; c < conn[j].size(); ++c) T.k_conn[c * 64 + j] = conn[j][c];
    const int need = std::max(std::max(L, n), 12);
    T.kin_G = need <= 16 ? 16 : (need <= 32 ? 32 : 64);
    T.kin_jsteps = pointer_jump_steps(T.max_depth);
    T.kin = 1;
}

void build_fused(Tables &T) {
    const int L = T.L;
    T.fused = 0;
    T.lanes = 0;
    if (L > 64) return;
    const int g_default = L <= 16 ? 16 : (L <= 32 ? 32 : 64);
    std::vector<int> perm, size;
    std::vector<int> &lane_of = T.lane_of;
    dfs_lanes(T, perm, lane_of, size);
    T.f_li.assign(8 * 64, 0);
    T.f_lf.assign(31 * 64, 0.0f);
    std::vector<std::vector<int>> conn(T.n);
    T.f_sph.assign((size_t)T.nmax * 64, make_float4(0, 0, 0, 0));
    for (int i = 0; i < L; ++i) {
        const int k = perm[i];
        const wb::LinkI &I = T.li[k];
        const wb::LinkF &F = T.lf[k];
        T.f_li[0 * 64 + i] = k;
        T.f_li[1 * 64 + i] = k == 0 ? -1 : lane_of[I.parent];
        T.f_li[2 * 64 + i] = i + size[k] - 1;
        T.f_li[3 * 64 + i] = I.jidx;
        T.f_li[4 * 64 + i] = I.sph_count;
        T.f_li[5 * 64 + i] = I.revolute;
        T.f_li[6 * 64 + i] = I.fR_identity;
        for (int c = 0; c < 3; ++c) T.f_lf[(0 + c) * 64 + i] = F.axis[c];
        for (int c = 0; c < 9; ++c) T.f_lf[(3 + c) * 64 + i] = k == 0 ? (c % 4 == 0 ? 1.0f : 0.0f) : F.fR[c];
        for (int c = 0; c < 3; ++c) T.f_lf[(12 + c) * 64 + i] = k == 0 ? 0.0f : F.fp[c];
        T.f_lf[15 * 64 + i] = F.mass;
        for (int c = 0; c < 3; ++c) T.f_lf[(16 + c) * 64 + i] = F.com[c];
        for (int c = 0; c < 6; ++c) T.f_lf[(19 + c) * 64 + i] = F.I[c];
        T.f_lf[29 * 64 + i] = F.mult;
        T.f_lf[30 * 64 + i] = F.offset;
        if (I.revolute && I.jidx >= 0) conn[I.jidx].push_back(i);
        for (int j = 0; j < I.sph_count; ++j) T.f_sph[(size_t)j * 64 + i] = T.sph[I.sph_first + j];
        // bounding sphere of the link's spheres in link coordinates: centroid,
        // then the largest reach, rounded up so that it holds every sphere
        double cen[3] = {0, 0, 0}, reach = -1e30;
        if (I.sph_count > 0) {
            for (int j = 0; j < I.sph_count; ++j) {
                const float4 q = T.sph[I.sph_first + j];
                cen[0] += q.x;
                cen[1] += q.y;
                cen[2] += q.z;
            }
            for (int c = 0; c < 3; ++c) cen[c] = (double)(float)(cen[c] / I.sph_count);
            for (int j = 0; j < I.sph_count; ++j) {
                const float4 q = T.sph[I.sph_first + j];
                const double dx = q.x - cen[0], dy = q.y - cen[1], dz = q.z - cen[2];
                reach = std::max(reach, std::sqrt(dx * dx + dy * dy + dz * dz) + q.w);
            }
            reach = reach * (1.0 + 1e-6) + 1e-7;
        }
        for (int c = 0; c < 3; ++c) T.f_lf[(25 + c) * 64 + i] = (float)cen[c];
        T.f_lf[28 * 64 + i] = std::nextafter((float)reach, INFINITY);
    }
    // lanes past the robot: an empty massless link with no parent and no joint
    for (int i = L; i < 64; ++i) {
        T.f_li[0 * 64 + i] = -1;
        T.f_li[1 * 64 + i] = -1;
        T.f_li[2 * 64 + i] = i;
        T.f_li[3 * 64 + i] = -1;
        T.f_li[6 * 64 + i] = 1;
        for (int c = 0; c < 9; c += 4) T.f_lf[(3 + c) * 64 + i] = 1.0f;
        T.f_lf[28 * 64 + i] = -1e30f;
        T.f_lf[29 * 64 + i] = 1.0f;
    }
    T.f_mimic = T.simple ? 0 : 1;
    T.f_mc = 1;
    for (int j = 0; j < T.n; ++j) T.f_mc = std::max(T.f_mc, (int)conn[j].size());
    T.f_conn.assign((size_t)T.f_mc * 64, -1);
    for (int j = 0; j < T.n; ++j)
        for (size_t c = 0; c < conn[j].size(); ++c) T.f_conn[c * 64 + j] = conn[j][c];
    T.jsteps = pointer_jump_steps(T.max_depth);
    T.lanes = 1;
    T.fused = T.nmax <= wb::FUSED_MAX_SLOTS &&
              wb::fused_lds_bytes(L, T.nmax, T.list_cap, g_default, (int)T.blocks.size()) <= wb::LDS_LIMIT;
}

int build_tables(const wb_robot_desc *d, Tables &T) {
    if (!d) return fail(WB_ERR_INVALID_ARG, "descriptor is null");
    const int L = d->n_links;
    if (L < 1) return fail(WB_ERR_INVALID_TREE, "n_links must be >= 1 (got %d)", L);
    if (L > WB_MAX_LINKS) return fail(WB_ERR_UNSUPPORTED, "n_links %d exceeds %d", L, WB_MAX_LINKS);
    if (!d->parent || !d->joint_type || !d->joint_index || !d->axis || !d->fixed_R || !d->fixed_p ||
        !d->mass || !d->com || !d->inertia)
        return fail(WB_ERR_INVALID_ARG, "a required per-link array is null");
    const int S = d->n_spheres;
    if (S < 0) return fail(WB_ERR_INVALID_ARG, "n_spheres must be >= 0");
    if (S > 0 && (!d->sphere_link || !d->sphere)) return fail(WB_ERR_INVALID_ARG, "sphere arrays are null");
    if (!finite_all(d->axis, 3 * (size_t)L) || !finite_all(d->fixed_R, 9 * (size_t)L) ||
        !finite_all(d->fixed_p, 3 * (size_t)L) || !finite_all(d->mass, L) || !finite_all(d->com, 3 * (size_t)L) ||
        !finite_all(d->inertia, 9 * (size_t)L) || !finite_all(d->gravity, 3) ||
        (S > 0 && !finite_all(d->sphere, 4 * (size_t)S)) ||
        (d->joint_mult && !finite_all(d->joint_mult, L)) || (d->joint_offset && !finite_all(d->joint_offset, L)))
        return fail(WB_ERR_INVALID_ARG, "descriptor holds a non-finite value");

    // Topology.
    if (d->parent[0] != -1) return fail(WB_ERR_INVALID_TREE, "parent[0] must be -1");
    if (d->joint_type[0] != WB_JOINT_FIXED) return fail(WB_ERR_INVALID_TREE, "link 0 (root) must be fixed");
    T.L = L;
    T.lf.assign(L, wb::LinkF{});
    T.li.assign(L, wb::LinkI{});
    int max_j = -1;
    for (int k = 0; k < L; ++k) {
        const int p = d->parent[k];
        if (k > 0 && (p < 0 || p >= k))
            return fail(WB_ERR_INVALID_TREE, "parent[%d] = %d must satisfy 0 <= parent < %d", k, p, k);
        const int jt = d->joint_type[k];
        if (jt != WB_JOINT_FIXED && jt != WB_JOINT_REVOLUTE)
            return fail(WB_ERR_INVALID_TREE, "joint_type[%d] = %d is not fixed/revolute", k, jt);
        const int ji = d->joint_index[k];
        if (jt == WB_JOINT_FIXED && ji != -1)
            return fail(WB_ERR_INVALID_TREE, "fixed link %d must have joint_index -1", k);
        if (jt == WB_JOINT_REVOLUTE && ji < 0)
            return fail(WB_ERR_INVALID_TREE, "revolute link %d has joint_index %d", k, ji);
        if (ji > max_j) max_j = ji;
        wb::LinkI &I = T.li[k];
        I.parent = p;
        I.revolute = jt == WB_JOINT_REVOLUTE;
        I.jidx = ji;
        I.depth = k == 0 ? 0 : T.li[p].depth + 1;
        if (I.depth > T.max_depth) T.max_depth = I.depth;
        wb::LinkF &F = T.lf[k];
        const float *ax = d->axis + 3 * k;
        if (I.revolute) {
            const double nrm = std::sqrt((double)ax[0] * ax[0] + (double)ax[1] * ax[1] + (double)ax[2] * ax[2]);
            if (std::fabs(nrm - 1.0) > 1e-4) return fail(WB_ERR_INVALID_TREE, "axis of link %d is not unit (|a| = %g)", k, nrm);
        }
        memcpy(F.axis, ax, 3 * sizeof(float));
        const float *R = d->fixed_R + 9 * k;
        double orth = 0.0;
        bool ident = true;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int t = 0; t < 3; ++t) s += (double)R[3 * t + i] * R[3 * t + j];
                orth = std::fmax(orth, std::fabs(s - (i == j ? 1.0 : 0.0)));
                if (R[3 * i + j] != (i == j ? 1.0f : 0.0f)) ident = false;
            }
        if (orth > 1e-4) return fail(WB_ERR_INVALID_TREE, "fixed_R of link %d is not orthonormal", k);
        memcpy(F.fR, R, 9 * sizeof(float));
        I.fR_identity = ident;
        memcpy(F.fp, d->fixed_p + 3 * k, 3 * sizeof(float));
        F.mult = d->joint_mult ? d->joint_mult[k] : 1.0f;
        F.offset = d->joint_offset ? d->joint_offset[k] : 0.0f;
        if (d->mass[k] < 0.0f) return fail(WB_ERR_INVALID_ARG, "mass of link %d is negative", k);
        F.mass = d->mass[k];
        memcpy(F.com, d->com + 3 * k, 3 * sizeof(float));
        const float *In = d->inertia + 9 * k;
        const float sc = std::fabs(In[0]) + std::fabs(In[4]) + std::fabs(In[8]) + 1e-30f;
        if (std::fabs(In[1] - In[3]) > 1e-5f * sc || std::fabs(In[2] - In[6]) > 1e-5f * sc ||
            std::fabs(In[5] - In[7]) > 1e-5f * sc)
            return fail(WB_ERR_INVALID_ARG, "inertia of link %d is not symmetric", k);
        F.I[0] = In[0]; F.I[1] = In[4]; F.I[2] = In[8];
        F.I[3] = 0.5f * (In[1] + In[3]); F.I[4] = 0.5f * (In[2] + In[6]); F.I[5] = 0.5f * (In[5] + In[7]);
    }
    T.n = max_j + 1;
    std::vector<int> uses(T.n, 0);
    for (int k = 0; k < L; ++k) {
        if (T.li[k].jidx >= 0) ++uses[T.li[k].jidx];
        if (T.li[k].revolute && (T.lf[k].mult != 1.0f || T.lf[k].offset != 0.0f)) T.simple = 0;
    }
    for (int j = 0; j < T.n; ++j) {
        if (uses[j] == 0) return fail(WB_ERR_INVALID_TREE, "actuated joint index %d is used by no link", j);
        if (uses[j] > 1) T.simple = 0;
    }
    for (int k = 1; k < L; ++k)
        if (d->parent[k] != k - 1) T.li[d->parent[k]].far_child = 1;

    // Spheres.
    T.S = S;
    std::vector<int> count(L, 0);
    for (int k = 0; k < L; ++k) T.li[k].sph_first = 0;
    for (int s = 0; s < S; ++s) {
        const int l = d->sphere_link[s];
        if (l < 0 || l >= L) return fail(WB_ERR_INVALID_TREE, "sphere %d is on missing link %d", s, l);
        if (s > 0 && l < d->sphere_link[s - 1])
            return fail(WB_ERR_INVALID_TREE, "sphere_link must be nondecreasing (sphere %d)", s);
        if (!(d->sphere[4 * s + 3] > 0.0f)) return fail(WB_ERR_INVALID_ARG, "sphere %d radius must be > 0", s);
        if (count[l] == 0) T.li[l].sph_first = s;
        ++count[l];
    }
    int most = 1;
    for (int k = 0; k < L; ++k) {
        T.li[k].sph_count = count[k];
        if (count[k] == 0) T.li[k].sph_first = 0;
        if (count[k] > most) most = count[k];
    }
    if (most > WB_MAX_SPHERES_PER_LINK)
        return fail(WB_ERR_UNSUPPORTED, "%d spheres on one link exceeds %d", most, WB_MAX_SPHERES_PER_LINK);
    // sphere slots per link: the most spheres on a link, rounded up above 8
    // to a size the sweep kernels are built for
    int nmax = most;
    if (nmax > 8) {
        const int sizes[] = {12, 16, 24, 32, 48, 64};
        for (int z : sizes)
            if (nmax <= z) {
                nmax = z;
                break;
            }
    }
    T.nmax = nmax;
    T.most = most;
    if (wb::state_lds_bytes(L, nmax) + 16 * 128 + 16 * wb::SWEEP_ROW_RING > wb::LDS_LIMIT)
        return fail(WB_ERR_UNSUPPORTED, "(links + 1) x spheres-per-link slots (%d x %d) exceed the 64 KB LDS tile",
                    L + 1, nmax);
    T.sph.resize(S);
    T.sph_link.resize(S);
    T.sph_slot.resize(S);
    for (int s = 0; s < S; ++s) {
        const float *x = d->sphere + 4 * s;
        T.sph[s] = make_float4(x[0], x[1], x[2], x[3]);
        const int l = d->sphere_link[s];
        T.sph_link[s] = l;
        T.sph_slot[s] = l * nmax + (s - T.li[l].sph_first);
    }
    T.slot_r.assign((size_t)(L + 1) * nmax, -1e30f);
    for (int s = 0; s < S; ++s) T.slot_r[T.sph_slot[s]] = T.sph[s].w;

    // Link-pair allow rule and blocks.
    if (d->allow) {
        for (int a = 0; a < L; ++a)
            for (int b = 0; b < L; ++b)
                if ((d->allow[a * L + b] != 0) != (d->allow[b * L + a] != 0))
                    return fail(WB_ERR_INVALID_ARG, "allow matrix is not symmetric at (%d, %d)", a, b);
    }
    auto allowed = [&](int a, int b) {
        if (a == b) return false;
        if (d->allow) return d->allow[a * L + b] != 0;
        return d->parent[b] != a && d->parent[a] != b;
    };
    T.blocks.clear();
    T.pair_cnt.assign((size_t)L * L, 0);
    std::vector<int64_t> partners(L, 0);
    for (int a = 0; a < L; ++a) {
        int64_t run = 0;
        for (int b = a + 1; b < L; ++b) {
            if (!allowed(a, b)) continue;
            T.pair_cnt[(size_t)a * L + b] = (int32_t)run;
            run += count[b];
            if (count[a] > 0 && count[b] > 0) T.blocks.push_back((a << 16) | b);
        }
        partners[a] = run;
    }
    T.n_blocks = (int)T.blocks.size();
    while (T.blocks.size() % 128) T.blocks.push_back((L << 16) | L);
    T.list_cap = wb::sweep_list_cap(T.n_blocks);
    T.pair_off.resize(S);
    int64_t off = 0;
    for (int s = 0; s < S; ++s) {
        if (off > INT32_MAX) return fail(WB_ERR_UNSUPPORTED, "more than 2^31 sphere pairs");
        T.pair_off[s] = (int32_t)off;
        off += partners[T.sph_link[s]];
    }
    if (off > INT32_MAX) return fail(WB_ERR_UNSUPPORTED, "more than 2^31 sphere pairs");
    T.n_pairs = off;
    // Pair list rebuilt from the block tables (the numbering the kernels use).
    T.pair_s.assign(off, -1);
    T.pair_t.assign(off, -1);
    for (int i = 0; i < T.n_blocks; ++i) {
        const int a = T.blocks[i] >> 16, b = T.blocks[i] & 0xffff;
        for (int s = T.li[a].sph_first; s < T.li[a].sph_first + count[a]; ++s)
            for (int t = T.li[b].sph_first; t < T.li[b].sph_first + count[b]; ++t) {
                const int64_t idx = (int64_t)T.pair_off[s] + T.pair_cnt[(size_t)a * L + b] + (t - T.li[b].sph_first);
                if (idx < 0 || idx >= off || T.pair_s[idx] != -1)
                    return fail(WB_ERR_INVALID_TREE, "internal: pair numbering is inconsistent");
                T.pair_s[idx] = s;
                T.pair_t[idx] = t;
            }
    }
    for (int c = 0; c < 3; ++c) T.g[c] = d->gravity[c];
    build_fused(T);
    build_kin(T);
    return WB_OK;
}

void fill_info(const Tables &T, wb_robot_info *info) {
    info->n_links = T.L;
    info->n_dof = T.n;
    info->n_spheres = T.S;
    info->max_depth = T.max_depth;
    info->n_pairs = T.n_pairs;
    info->n_blocks = T.n_blocks;
    info->max_spheres_per_link = T.most;
    info->fused_supported = T.fused;
    info->mimic = T.simple ? 0 : 1;
    info->kinematics_supported = T.kin;
}

bool aligned4(const void *p) { return ((uintptr_t)p & 3) == 0; }

}  // namespace

struct wb_robot {
    Tables T;
    wb::DevRobot dev{};
    wb::DevFused fz{};
    wb::DevKin kin{};
    wb_tune tune{};
    void *dmem = nullptr;
    size_t o_lf = 0, o_ff = 0;   // offsets of the link records and the fused float lane table
    size_t o_kf = 0;             // offset of the kinematics float lane table
    size_t o_tl = 0, o_to = 0, o_ta = 0;   // tool lanes, offsets and affects masks (WB_MAX_TOOLS each)
    int device = -1;
    int cus = 256;   // compute units of that device
    int64_t sweep_split_below = -1;   // wb_self_collision splits states below this batch (-1: the default rule)
    int64_t fk_groups_below = -1;     // wb_fk and wb_fk_backward take a group per state below it (-1: default)
    int64_t fk_pose_groups_below = -1;  // the same when link poses are written or read
};

namespace {

// Default launch shape of the fused iteration: the narrowest group of lanes
// per state that holds every link (16, 32 or 64), 16 states per workgroup.
wb_tune default_tune(int L) {
    wb_tune t{};
    t.lanes_per_state = L <= 16 ? 16 : (L <= 32 ? 32 : 64);
    t.states_per_item = 16;
    t.ns_per_state = 0.0f;
    return t;
}

// States per workgroup of the fused launch.  The tuned value holds for
// large batches; a batch too small to give every compute unit four
// workgroups (its occupancy at 4 wavefronts per SIMD) gets a smaller chunk,
// halved down to the states one workgroup has in flight at once, so that
// the work spreads over the whole chip instead of a few deep workgroups.
int small_batch_chunk(const wb_tune &t, int64_t B, int cus) {
    const int in_flight = 4 * (64 / t.lanes_per_state);
    int c = t.states_per_item;
    while (c > in_flight && (B + c - 1) / c < (int64_t)cus * 4) c = std::max(in_flight, c / 2);
    return c;
}

int check_tune(const wb_tune &t, const Tables &T) {
    const int g = t.lanes_per_state;
    if (g != 16 && g != 32 && g != 64) return fail(WB_ERR_INVALID_ARG, "lanes_per_state must be 16, 32 or 64");
    if (g < T.L) return fail(WB_ERR_INVALID_ARG, "lanes_per_state %d is below the %d links", g, T.L);
    const size_t need = wb::fused_lds_bytes(T.L, T.nmax, T.list_cap, g, (int)T.blocks.size());
    if (need > wb::LDS_LIMIT)
        return fail(WB_ERR_UNSUPPORTED, "lanes_per_state %d needs %zu bytes of LDS per workgroup (> %zu)", g, need,
                    wb::LDS_LIMIT);
    if (t.states_per_item < 1 || t.states_per_item > 4096)
        return fail(WB_ERR_INVALID_ARG, "states_per_item must be in [1, 4096]");
    if (!(t.ns_per_state >= 0.0f) || !std::isfinite(t.ns_per_state))
        return fail(WB_ERR_INVALID_ARG, "ns_per_state must be finite and >= 0");
    return WB_OK;
}

}  // namespace

namespace {

template <typename V>
size_t append(std::vector<char> &blob, const V &v) {
    size_t off = (blob.size() + 255) & ~(size_t)255;
    blob.resize(off + v.size() * sizeof(typename V::value_type));
    if (!v.empty()) memcpy(blob.data() + off, v.data(), v.size() * sizeof(typename V::value_type));
    return off;
}

int check_robot(const wb_robot *r) {
    if (!r || !r->dmem) return fail(WB_ERR_INVALID_ARG, "robot handle is null or destroyed");
    return WB_OK;
}

int check_B(int64_t B) {
    if (B < 0 || B > INT32_MAX) return fail(WB_ERR_INVALID_ARG, "batch size %lld out of range", (long long)B);
    return WB_OK;
}

// The leading dimension of the [k][B] arrays of a call: 0 means B; any
// other value must be >= B.
int resolve_ld(int64_t B, int64_t ld, int64_t *out) {
    if (ld == 0) ld = B;
    if (ld < B) return fail(WB_ERR_INVALID_ARG, "ld %lld is below B %lld", (long long)ld, (long long)B);
    *out = ld;
    return WB_OK;
}

int check_ptr(const void *p, const char *name, bool required) {
    if (!p) return required ? fail(WB_ERR_INVALID_ARG, "%s is null", name) : WB_OK;
    if (!aligned4(p)) return fail(WB_ERR_INVALID_ARG, "%s is not 4-byte aligned", name);
    return WB_OK;
}

#define WB_TRY(x)                    \
    do {                             \
        int _rc = (x);               \
        if (_rc != WB_OK) return _rc; \
    } while (0)

int finish(hipError_t e, const char *what) { return e == hipSuccess ? WB_OK : hip_fail(e, what); }

}  // namespace

extern "C" {

const char *wb_last_error(void) { return g_err.c_str(); }

int wb_desc_analyze(const wb_robot_desc *desc, wb_robot_info *info) {
    if (!info) return fail(WB_ERR_INVALID_ARG, "info is null");
    Tables T;
    WB_TRY(build_tables(desc, T));
    fill_info(T, info);
    return WB_OK;
}

int wb_desc_pairs(const wb_robot_desc *desc, int32_t *s, int32_t *t) {
    Tables T;
    WB_TRY(build_tables(desc, T));
    if (T.n_pairs > 0 && (!s || !t)) return fail(WB_ERR_INVALID_ARG, "output arrays are null");
    if (T.n_pairs > 0) {
        memcpy(s, T.pair_s.data(), T.n_pairs * sizeof(int32_t));
        memcpy(t, T.pair_t.data(), T.n_pairs * sizeof(int32_t));
    }
    return WB_OK;
}

int wb_robot_create(const wb_robot_desc *desc, wb_robot **out) {
    if (!out) return fail(WB_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    wb_robot *r = new wb_robot();
    int rc = build_tables(desc, r->T);
    if (rc != WB_OK) {
        delete r;
        return rc;
    }
    const Tables &T = r->T;
    std::vector<char> blob;
    const size_t o_lf = append(blob, T.lf), o_li = append(blob, T.li), o_sph = append(blob, T.sph);
    const size_t o_sl = append(blob, T.sph_link), o_ss = append(blob, T.sph_slot);
    const size_t o_sr = append(blob, T.slot_r), o_bl = append(blob, T.blocks);
    const size_t o_po = append(blob, T.pair_off), o_pc = append(blob, T.pair_cnt);
    const size_t o_ps = append(blob, T.pair_s), o_pt = append(blob, T.pair_t);
    const size_t o_fi = append(blob, T.f_li), o_ff = append(blob, T.f_lf), o_fs = append(blob, T.f_sph);
    const size_t o_fc = append(blob, T.f_conn);
    const size_t o_ki = append(blob, T.k_li), o_kf = append(blob, T.k_lf), o_kc = append(blob, T.k_conn);
    const size_t o_tl = append(blob, std::vector<int32_t>(WB_MAX_TOOLS, 0));
    const size_t o_to = append(blob, std::vector<float>(12 * WB_MAX_TOOLS, 0.0f));
    const size_t o_ta = append(blob, std::vector<uint64_t>(WB_MAX_TOOLS, 0));
    blob.resize(blob.size() + 256);
    hipError_t e = hipGetDevice(&r->device);
    if (e == hipSuccess) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, r->device) == hipSuccess && cus > 0)
            r->cus = cus;
    }
    if (e == hipSuccess) e = hipMalloc(&r->dmem, blob.size());
    if (e == hipSuccess) e = hipMemcpy(r->dmem, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (r->dmem) (void)hipFree(r->dmem);
        delete r;
        return hip_fail(e, "uploading the robot tables");
    }
    char *base = static_cast<char *>(r->dmem);
    r->o_lf = o_lf;
    r->o_ff = o_ff;
    wb::DevRobot &D = r->dev;
    D.L = T.L; D.n = T.n; D.S = T.S; D.nmax = T.nmax;
    D.n_blocks = T.n_blocks; D.n_blocks_pad = (int)T.blocks.size();
    D.max_depth = T.max_depth; D.simple_joints = T.simple;
    D.n_pairs = T.n_pairs;
    D.gx = T.g[0]; D.gy = T.g[1]; D.gz = T.g[2];
    D.list_cap = T.list_cap;
    D.lf = reinterpret_cast<const wb::LinkF *>(base + o_lf);
    D.li = reinterpret_cast<const wb::LinkI *>(base + o_li);
    D.sph = reinterpret_cast<const float4 *>(base + o_sph);
    D.sph_link = reinterpret_cast<const int32_t *>(base + o_sl);
    D.sph_slot = reinterpret_cast<const int32_t *>(base + o_ss);
    D.slot_r = reinterpret_cast<const float *>(base + o_sr);
    D.blocks = reinterpret_cast<const int32_t *>(base + o_bl);
    D.pair_off = reinterpret_cast<const int32_t *>(base + o_po);
    D.pair_cnt = reinterpret_cast<const int32_t *>(base + o_pc);
    D.pair_s = reinterpret_cast<const int32_t *>(base + o_ps);
    D.pair_t = reinterpret_cast<const int32_t *>(base + o_pt);
    wb::DevFused &Fz = r->fz;
    Fz.supported = T.fused;
    Fz.jsteps = T.jsteps;
    Fz.li = reinterpret_cast<const int32_t *>(base + o_fi);
    Fz.lf = reinterpret_cast<const float *>(base + o_ff);
    Fz.lsph = reinterpret_cast<const float4 *>(base + o_fs);
    Fz.mimic = T.f_mimic;
    Fz.mc = T.f_mc;
    Fz.conn = reinterpret_cast<const int32_t *>(base + o_fc);
    wb::DevKin &Kn = r->kin;
    Kn.L = T.L; Kn.n = T.n; Kn.G = T.kin_G; Kn.jsteps = T.kin_jsteps; Kn.mc = T.kin_mc;
    Kn.inv_mass = T.total_mass > 0.0 ? (float)(1.0 / T.total_mass) : 0.0f;
    Kn.li = reinterpret_cast<const int32_t *>(base + o_ki);
    Kn.lf = reinterpret_cast<const float *>(base + o_kf);
    Kn.conn = reinterpret_cast<const int32_t *>(base + o_kc);
    Kn.sph = D.sph;
    Kn.n_tools = 0;
    Kn.tool_lane = reinterpret_cast<const int32_t *>(base + o_tl);
    Kn.tool_off = reinterpret_cast<const float *>(base + o_to);
    Kn.tool_aff = reinterpret_cast<const uint64_t *>(base + o_ta);
    r->o_kf = o_kf;
    r->o_tl = o_tl;
    r->o_to = o_to;
    r->o_ta = o_ta;
    r->tune = default_tune(T.L);
    *out = r;
    return WB_OK;
}

int wb_robot_destroy(wb_robot *robot) {
    if (!robot) return WB_OK;
    hipError_t e = hipSuccess;
    if (robot->dmem) e = hipFree(robot->dmem);
    robot->dmem = nullptr;
    delete robot;
    return finish(e, "freeing the robot tables");
}

int wb_robot_get_info(const wb_robot *robot, wb_robot_info *info) {
    WB_TRY(check_robot(robot));
    if (!info) return fail(WB_ERR_INVALID_ARG, "info is null");
    fill_info(robot->T, info);
    return WB_OK;
}

int wb_workspace_bytes(const wb_robot *robot, int64_t B, size_t *bytes) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    if (!bytes) return fail(WB_ERR_INVALID_ARG, "bytes is null");
    *bytes = (size_t)wb::workspace_floats_per_state(robot->T.L) * (size_t)B * sizeof(float);
    return WB_OK;
}

int wb_rnea_cache_bytes(const wb_robot *robot, int64_t B, size_t *bytes) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    if (!bytes) return fail(WB_ERR_INVALID_ARG, "bytes is null");
    *bytes = (size_t)robot->T.L * 18 * (size_t)B * sizeof(float);
    return WB_OK;
}

namespace {
// Forward kinematics and its adjoint take one group of lanes per state
// (pointer jumping over the links, nothing stored) for batches below a
// threshold, and one lane per state above, where the lane form's coalesced
// rows win.  Calls that write or read link poses have a threshold of their
// own: the group form writes a state's poses across 12L rows and its
// adjoint recomputes them, while the lane form's adjoint reads them.
// Default for both: 48 states per compute unit.  The group form takes
// robots of at most 64 links.
bool lanes_form(const wb_robot *r, int64_t B, bool pose) {
    const int64_t set = pose ? r->fk_pose_groups_below : r->fk_groups_below;
    const int64_t below = set >= 0 ? set : (int64_t)48 * r->cus;
    return r->T.lanes && B < below;
}
}  // namespace

int wb_fk(const wb_robot *robot, int64_t B, int64_t ld, const float *q, float *link_pose, float *spheres,
          hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    WB_TRY(resolve_ld(B, ld, &ld));
    if (B == 0) return WB_OK;
    WB_TRY(check_ptr(q, "q", robot->T.n > 0));
    WB_TRY(check_ptr(link_pose, "link_pose", false));
    WB_TRY(check_ptr(spheres, "spheres", false));
    if (!link_pose && !spheres) return fail(WB_ERR_INVALID_ARG, "link_pose and spheres are both null");
    if (lanes_form(robot, B, link_pose != nullptr) && robot->T.kin) {
        const wb::KinOut o{link_pose, spheres, nullptr, nullptr, nullptr, nullptr};
        return finish(wb::launch_kinematics(robot->kin, B, ld, q, o, stream), "wb_fk launch");
    }
    return finish(wb::launch_fk(robot->dev, B, ld, q, link_pose, spheres, stream), "wb_fk launch");
}

int wb_rnea(const wb_robot *robot, int64_t B, int64_t ld, const float *q, const float *qd, const float *qdd,
            const float *f_ext, float *tau, float *cache, hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    WB_TRY(resolve_ld(B, ld, &ld));
    if (B == 0) return WB_OK;
    const bool need = robot->T.n > 0;
    WB_TRY(check_ptr(q, "q", need));
    WB_TRY(check_ptr(qd, "qd", need));
    WB_TRY(check_ptr(qdd, "qdd", need));
    WB_TRY(check_ptr(f_ext, "f_ext", false));
    WB_TRY(check_ptr(tau, "tau", need));
    WB_TRY(check_ptr(cache, "cache", false));
    if (cache)
        return finish(wb::launch_rnea(robot->dev, B, ld, q, qd, qdd, f_ext, tau, cache, stream), "wb_rnea launch");
    if (!robot->T.lanes)
        return fail(WB_ERR_UNSUPPORTED, "a robot of %d links (more than 64) needs the cache", robot->T.L);
    return finish(wb::launch_rnea_lanes(robot->dev, robot->fz, B, ld, q, qd, qdd, f_ext, tau, stream),
                  "wb_rnea launch");
}

namespace {
// wb_self_collision's form for a batch: one state per workgroup (its pairs
// split over the four wavefronts) below the robot's threshold, one state
// per wavefront above.  Default threshold: 16 states per compute unit (below
// it one state per wavefront leaves most SIMDs with under four wavefronts).
bool sweep_split(const wb_robot *r, int64_t B) {
    const int64_t below = r->sweep_split_below >= 0 ? r->sweep_split_below : (int64_t)16 * r->cus;
    return B < below;
}
}  // namespace

int wb_robot_set_dispatch(wb_robot *robot, int64_t sweep_split_below, int64_t fk_groups_below,
                          int64_t fk_pose_groups_below) {
    WB_TRY(check_robot(robot));
    robot->sweep_split_below = sweep_split_below < 0 ? -1 : sweep_split_below;
    robot->fk_groups_below = fk_groups_below < 0 ? -1 : fk_groups_below;
    robot->fk_pose_groups_below = fk_pose_groups_below < 0 ? -1 : fk_pose_groups_below;
    return WB_OK;
}

int wb_self_collision(const wb_robot *robot, int64_t B, int64_t ld, const float *spheres, float *max_pen,
                      int32_t *argmax, int32_t *n_coll, hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    WB_TRY(resolve_ld(B, ld, &ld));
    if (B == 0) return WB_OK;
    if (!max_pen && !argmax && !n_coll) return fail(WB_ERR_INVALID_ARG, "all outputs are null");
    WB_TRY(check_ptr(spheres, "spheres", robot->T.S > 0));
    WB_TRY(check_ptr(max_pen, "max_pen", false));
    WB_TRY(check_ptr(argmax, "argmax", false));
    WB_TRY(check_ptr(n_coll, "n_coll", false));
    return finish(wb::launch_self_collision(robot->dev, B, ld, spheres, max_pen, argmax, n_coll,
                                            sweep_split(robot, B), stream),
                  "wb_self_collision launch");
}

int wb_self_collision_backward(const wb_robot *robot, int64_t B, int64_t ld, const float *spheres,
                               const int32_t *argmax, const float *max_pen, float margin,
                               const float *g_cost, float *g_spheres, hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    WB_TRY(resolve_ld(B, ld, &ld));
    if (!std::isfinite(margin)) return fail(WB_ERR_INVALID_ARG, "margin is not finite");
    if (B == 0) return WB_OK;
    WB_TRY(check_ptr(spheres, "spheres", robot->T.S > 0));
    WB_TRY(check_ptr(argmax, "argmax", true));
    WB_TRY(check_ptr(max_pen, "max_pen", true));
    WB_TRY(check_ptr(g_cost, "g_cost", true));
    WB_TRY(check_ptr(g_spheres, "g_spheres", robot->T.S > 0));
    return finish(wb::launch_self_collision_backward(robot->dev, B, ld, spheres, argmax, max_pen, margin, g_cost,
                                                     g_spheres, stream),
                  "wb_self_collision_backward launch");
}

int wb_fk_backward(const wb_robot *robot, int64_t B, int64_t ld, const float *q, const float *link_pose,
                   const float *g_link_pose, const float *g_spheres, float *g_q, void *workspace,
                   hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    WB_TRY(resolve_ld(B, ld, &ld));
    if (B == 0) return WB_OK;
    if (!g_link_pose && !g_spheres) return fail(WB_ERR_INVALID_ARG, "both gradient inputs are null");
    WB_TRY(check_ptr(q, "q", robot->T.n > 0));
    WB_TRY(check_ptr(link_pose, "link_pose", false));
    WB_TRY(check_ptr(g_link_pose, "g_link_pose", false));
    WB_TRY(check_ptr(g_spheres, "g_spheres", false));
    WB_TRY(check_ptr(g_q, "g_q", robot->T.n > 0));
    if (lanes_form(robot, B, link_pose != nullptr || g_link_pose != nullptr)) {
        WB_TRY(check_ptr(workspace, "workspace", false));
        return finish(wb::launch_fk_backward_lanes(robot->dev, robot->fz, B, ld, q, g_link_pose, g_spheres, g_q, stream),
                      "wb_fk_backward launch");
    }
    WB_TRY(check_ptr(workspace, "workspace", true));
    return finish(wb::launch_fk_backward(robot->dev, B, ld, q, link_pose, g_link_pose, g_spheres, g_q,
                                         static_cast<float *>(workspace), stream),
                  "wb_fk_backward launch");
}

int wb_rnea_backward(const wb_robot *robot, int64_t B, int64_t ld, const float *q, const float *qd,
                     const float *qdd, const float *f_ext, const float *cache, const float *g_tau, float *g_q,
                     float *g_qd, float *g_qdd, float *g_fext, void *workspace, hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    WB_TRY(resolve_ld(B, ld, &ld));
    if (B == 0) return WB_OK;
    const bool need = robot->T.n > 0;
    WB_TRY(check_ptr(q, "q", need));
    WB_TRY(check_ptr(qd, "qd", need));
    WB_TRY(check_ptr(qdd, "qdd", need));
    WB_TRY(check_ptr(f_ext, "f_ext", false));
    WB_TRY(check_ptr(cache, "cache", false));
    WB_TRY(check_ptr(g_tau, "g_tau", need));
    WB_TRY(check_ptr(g_q, "g_q", need));
    WB_TRY(check_ptr(g_qd, "g_qd", need));
    WB_TRY(check_ptr(g_qdd, "g_qdd", need));
    WB_TRY(check_ptr(g_fext, "g_fext", false));
    if (!cache) {
        if (!robot->T.lanes)
            return fail(WB_ERR_UNSUPPORTED, "a robot of %d links (more than 64) needs the cache", robot->T.L);
        WB_TRY(check_ptr(workspace, "workspace", false));
        return finish(wb::launch_rnea_backward_lanes(robot->dev, robot->fz, B, ld, q, qd, qdd, f_ext, g_tau, g_q,
                                                     g_qd, g_qdd, g_fext, stream),
                      "wb_rnea_backward launch");
    }
    WB_TRY(check_ptr(workspace, "workspace", true));
    return finish(wb::launch_rnea_backward(robot->dev, B, ld, q, qd, qdd, cache, g_tau, g_q, g_qd, g_qdd, g_fext,
                                           static_cast<float *>(workspace), stream),
                  "wb_rnea_backward launch");
}

int wb_cost_head(int64_t B, int64_t ld, int32_t n, const float *tau, const float *w, float torque_weight,
                 const float *max_pen, float margin, float hinge_weight, float *cost, float *g_tau,
                 float *g_maxpen, hipStream_t stream) {
    WB_TRY(check_B(B));
    WB_TRY(resolve_ld(B, ld, &ld));
    if (n < 0) return fail(WB_ERR_INVALID_ARG, "n must be >= 0");
    if (!std::isfinite(torque_weight) || !std::isfinite(margin) || !std::isfinite(hinge_weight))
        return fail(WB_ERR_INVALID_ARG, "weights and margin must be finite");
    if (B == 0) return WB_OK;
    WB_TRY(check_ptr(tau, "tau", n > 0));
    WB_TRY(check_ptr(w, "w", false));
    WB_TRY(check_ptr(max_pen, "max_pen", false));
    WB_TRY(check_ptr(cost, "cost", false));
    WB_TRY(check_ptr(g_tau, "g_tau", false));
    WB_TRY(check_ptr(g_maxpen, "g_maxpen", false));
    return finish(wb::launch_cost_head(B, ld, n, tau, w, torque_weight, max_pen, margin, hinge_weight, cost, g_tau,
                                       g_maxpen, stream),
                  "wb_cost_head launch");
}

int wb_sgd_step(int64_t B, int64_t ld, int32_t n, float lr, float *q, float *qd, float *qdd, const float *g_q,
                const float *g_q2, const float *g_qd, const float *g_qdd, hipStream_t stream) {
    WB_TRY(check_B(B));
    WB_TRY(resolve_ld(B, ld, &ld));
    if (n < 0) return fail(WB_ERR_INVALID_ARG, "n must be >= 0");
    if (!std::isfinite(lr)) return fail(WB_ERR_INVALID_ARG, "lr must be finite");
    if (B == 0 || n == 0) return WB_OK;
    WB_TRY(check_ptr(q, "q", true));
    WB_TRY(check_ptr(qd, "qd", true));
    WB_TRY(check_ptr(qdd, "qdd", true));
    WB_TRY(check_ptr(g_q, "g_q", true));
    WB_TRY(check_ptr(g_q2, "g_q2", false));
    WB_TRY(check_ptr(g_qd, "g_qd", true));
    WB_TRY(check_ptr(g_qdd, "g_qdd", true));
    return finish(wb::launch_sgd_step(B, ld, n, lr, q, qd, qdd, g_q, g_q2, g_qd, g_qdd, stream), "wb_sgd_step launch");
}

namespace {
int check_bspline(int64_t T, int32_t d, int32_t K, int32_t n_interp, float dt) {
    WB_TRY(check_B(T));
    if (d < 0) return fail(WB_ERR_INVALID_ARG, "d must be >= 0");
    if (K < 1 || K > WB_BSPLINE_MAX_K) return fail(WB_ERR_INVALID_ARG, "K must be in [1, %d]", WB_BSPLINE_MAX_K);
    if (n_interp < 1 || n_interp > 1024) return fail(WB_ERR_INVALID_ARG, "n_interp must be in [1, 1024]");
    if (!(dt > 0.0f) || !std::isfinite(dt)) return fail(WB_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (d > 65535) return fail(WB_ERR_UNSUPPORTED, "d must be <= 65535");
    const int64_t H = (int64_t)(K + 3) * n_interp;
    if (T > 0 && H > (INT64_C(1) << 31) / T - 1)
        return fail(WB_ERR_UNSUPPORTED, "T * (K + 3) * n_interp samples must stay below 2^31");
    return WB_OK;
}
}  // namespace

int wb_bspline_eval(int64_t T, int32_t d, int32_t K, int32_t n_interp, float dt, int32_t reading,
                    const float *U, const float *theta0, const float *dtheta0, const float *ddtheta0,
                    float *q, float *qd, float *qdd, hipStream_t stream) {
    WB_TRY(check_bspline(T, d, K, n_interp, dt));
    if (reading != WB_GHOST_EXACT && reading != WB_GHOST_PRINTED)
        return fail(WB_ERR_INVALID_ARG, "reading must be WB_GHOST_EXACT or WB_GHOST_PRINTED");
    if (T == 0 || d == 0) return WB_OK;
    WB_TRY(check_ptr(U, "U", true));
    WB_TRY(check_ptr(theta0, "theta0", true));
    WB_TRY(check_ptr(dtheta0, "dtheta0", false));
    WB_TRY(check_ptr(ddtheta0, "ddtheta0", false));
    WB_TRY(check_ptr(q, "q", true));
    WB_TRY(check_ptr(qd, "qd", false));
    WB_TRY(check_ptr(qdd, "qdd", false));
    return finish(wb::launch_bspline_eval(T, d, K, n_interp, dt, reading, U, theta0, dtheta0, ddtheta0, q, qd, qdd,
                                          stream),
                  "wb_bspline_eval launch");
}

int wb_bspline_backward(int64_t T, int32_t d, int32_t K, int32_t n_interp, float dt, const float *g_q,
                        const float *g_qd, const float *g_qdd, float *g_U, float lr, int32_t step_rule, float *U,
                        hipStream_t stream) {
    WB_TRY(check_bspline(T, d, K, n_interp, dt));
    if (!std::isfinite(lr)) return fail(WB_ERR_INVALID_ARG, "lr must be finite");
    if (step_rule != WB_STEP_PLAIN && step_rule != WB_STEP_ROW_RMS)
        return fail(WB_ERR_INVALID_ARG, "unknown step rule %d", step_rule);
    if (T == 0 || d == 0) return WB_OK;
    WB_TRY(check_ptr(g_q, "g_q", false));
    WB_TRY(check_ptr(g_qd, "g_qd", false));
    WB_TRY(check_ptr(g_qdd, "g_qdd", false));
    WB_TRY(check_ptr(g_U, "g_U", lr == 0.0f || step_rule == WB_STEP_ROW_RMS));
    WB_TRY(check_ptr(U, "U", lr != 0.0f));
    return finish(wb::launch_bspline_backward(T, d, K, n_interp, dt, g_q, g_qd, g_qdd, g_U, lr, step_rule, U, stream),
                  "wb_bspline_backward launch");
}

int wb_wholebody_step(const wb_robot *robot, int64_t B, int64_t ld, float *q, float *qd, float *qdd, const float *w,
                      float torque_weight, float margin, float hinge_weight, float lr, float *tau, float *cost,
                      float *max_pen, int32_t *argmax, int32_t *n_coll, float *g_q, float *g_qd, float *g_qdd,
                      const float *f_ext, float *g_fext, hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    WB_TRY(resolve_ld(B, ld, &ld));
    if (!robot->fz.supported)
        return fail(WB_ERR_UNSUPPORTED, "the fused iteration needs <= 64 links and sweep tables within %zu bytes of LDS",
                    wb::LDS_LIMIT);
    if (!std::isfinite(torque_weight) || !std::isfinite(margin) || !std::isfinite(hinge_weight) || !std::isfinite(lr))
        return fail(WB_ERR_INVALID_ARG, "weights, margin and lr must be finite");
    if (B == 0) return WB_OK;
    const bool need = robot->T.n > 0;
    WB_TRY(check_ptr(q, "q", need));
    WB_TRY(check_ptr(qd, "qd", need));
    WB_TRY(check_ptr(qdd, "qdd", need));
    WB_TRY(check_ptr(w, "w", false));
    WB_TRY(check_ptr(tau, "tau", false));
    WB_TRY(check_ptr(cost, "cost", false));
    WB_TRY(check_ptr(max_pen, "max_pen", false));
    WB_TRY(check_ptr(argmax, "argmax", false));
    WB_TRY(check_ptr(n_coll, "n_coll", false));
    WB_TRY(check_ptr(g_q, "g_q", false));
    WB_TRY(check_ptr(g_qd, "g_qd", false));
    WB_TRY(check_ptr(g_qdd, "g_qdd", false));
    WB_TRY(check_ptr(f_ext, "f_ext", false));
    WB_TRY(check_ptr(g_fext, "g_fext", false));
    wb::FusedArgs a{};
    a.rb = robot->dev;
    a.fz = robot->fz;
    a.B = B;
    a.chunk = small_batch_chunk(robot->tune, B, robot->cus);
    a.lanes_per_state = robot->tune.lanes_per_state;
    a.io = wb::TreeIO{q, qd, qdd, w, tau, cost, max_pen, argmax, n_coll, g_q, g_qd, g_qdd, f_ext, g_fext, ld};
    a.k = wb::StepScalars{torque_weight, margin, hinge_weight, lr};
    return finish(wb::launch_fused(a, stream), "wb_wholebody_step launch");
}

int wb_wholebody_step_bspline(const wb_robot *robot, int64_t T, int32_t K, float dt, int32_t reading,
                              float *U, const float *theta0, const float *dtheta0, const float *ddtheta0,
                              const float *w, float torque_weight, float margin, float hinge_weight, float *g_U,
                              float lr, int32_t step_rule, float *tau, float *cost, float *max_pen, int32_t *argmax,
                              int32_t *n_coll, float *g_q, float *g_qd, float *g_qdd, hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_bspline(T, robot->T.n, K, 4, dt));
    if (reading != WB_GHOST_EXACT && reading != WB_GHOST_PRINTED)
        return fail(WB_ERR_INVALID_ARG, "unknown ghost-knot reading %d", reading);
    if (!robot->fz.supported)
        return fail(WB_ERR_UNSUPPORTED, "the fused iteration needs <= 64 links and sweep tables within %zu bytes of LDS",
                    wb::LDS_LIMIT);
    if (robot->fz.mimic)
        return fail(WB_ERR_UNSUPPORTED, "the spline-sampling form takes robots without mimic joints");
    if (!std::isfinite(torque_weight) || !std::isfinite(margin) || !std::isfinite(hinge_weight) || !std::isfinite(lr))
        return fail(WB_ERR_INVALID_ARG, "weights, margin and lr must be finite");
    if (step_rule != WB_STEP_PLAIN && step_rule != WB_STEP_ROW_RMS)
        return fail(WB_ERR_INVALID_ARG, "unknown step rule %d", step_rule);
    const int64_t H = (int64_t)(K + 3) * 4, B = T * H;
    const bool reduce = g_U || lr != 0.0f;
    const int G = robot->tune.lanes_per_state;
    if (reduce && wb::fused_lds_bytes(robot->T.L, robot->T.nmax, robot->T.list_cap, G, (int)robot->T.blocks.size()) +
                          wb::spline_lds_bytes(G, robot->T.n, K) > wb::LDS_LIMIT)
        return fail(WB_ERR_UNSUPPORTED, "the control-point gradient of %d joints x %d control points does not fit "
                    "the workgroup's LDS; take the per-sample gradients and wb_bspline_backward", robot->T.n, K);
    if (B == 0 || robot->T.n == 0) return WB_OK;
    WB_TRY(check_ptr(U, "U", true));
    WB_TRY(check_ptr(g_U, "g_U", false));
    WB_TRY(check_ptr(theta0, "theta0", true));
    WB_TRY(check_ptr(dtheta0, "dtheta0", false));
    WB_TRY(check_ptr(ddtheta0, "ddtheta0", false));
    WB_TRY(check_ptr(w, "w", false));
    WB_TRY(check_ptr(tau, "tau", false));
    WB_TRY(check_ptr(cost, "cost", false));
    WB_TRY(check_ptr(max_pen, "max_pen", false));
    WB_TRY(check_ptr(argmax, "argmax", false));
    WB_TRY(check_ptr(n_coll, "n_coll", false));
    WB_TRY(check_ptr(g_q, "g_q", false));
    WB_TRY(check_ptr(g_qd, "g_qd", false));
    WB_TRY(check_ptr(g_qdd, "g_qdd", false));
    wb::FusedArgs a{};
    a.rb = robot->dev;
    a.fz = robot->fz;
    a.B = B;
    // with the control-point gradient reduced in LDS a workgroup owns one whole trajectory
    a.chunk = reduce ? (int32_t)H : small_batch_chunk(robot->tune, B, robot->cus);
    a.lanes_per_state = G;
    a.io = wb::TreeIO{nullptr, nullptr, nullptr, w, tau, cost, max_pen, argmax, n_coll, g_q, g_qd, g_qdd,
                      nullptr, nullptr, B};
    a.sp = wb::SplineIn{U, theta0, dtheta0, ddtheta0, (int32_t)T, K, (int32_t)H, reading, dt, g_U, lr, step_rule};
    a.k = wb::StepScalars{torque_weight, margin, hinge_weight, 0.0f};
    return finish(wb::launch_fused(a, stream), "wb_wholebody_step_bspline launch");
}

int wb_robot_set_tune(wb_robot *robot, const wb_tune *tune) {
    WB_TRY(check_robot(robot));
    if (!tune) return fail(WB_ERR_INVALID_ARG, "tune is null");
    WB_TRY(check_tune(*tune, robot->T));
    robot->tune = *tune;
    return WB_OK;
}

int wb_robot_set_link_inertia(wb_robot *robot, int32_t link, float mass, const float *com, const float *inertia) {
    WB_TRY(check_robot(robot));
    Tables &T = robot->T;
    if (link < 0 || link >= T.L) return fail(WB_ERR_INVALID_ARG, "link %d out of range [0, %d)", link, T.L);
    if (!com || !inertia) return fail(WB_ERR_INVALID_ARG, "com and inertia must not be null");
    if (!std::isfinite(mass) || mass < 0.0f || !finite_all(com, 3) || !finite_all(inertia, 6))
        return fail(WB_ERR_INVALID_ARG, "mass must be finite and >= 0, com and inertia finite");
    wb::LinkF &F = T.lf[link];
    F.mass = mass;
    for (int c = 0; c < 3; ++c) F.com[c] = com[c];
    for (int c = 0; c < 6; ++c) F.I[c] = inertia[c];
    if (T.lanes) {
        const int i = T.lane_of[link];
        T.f_lf[15 * 64 + i] = mass;
        for (int c = 0; c < 3; ++c) T.f_lf[(16 + c) * 64 + i] = com[c];
        for (int c = 0; c < 6; ++c) T.f_lf[(19 + c) * 64 + i] = inertia[c];
    }
    T.total_mass = 0.0;
    for (int k = 0; k < T.L; ++k) T.total_mass += T.lf[k].mass;
    robot->kin.inv_mass = T.total_mass > 0.0 ? (float)(1.0 / T.total_mass) : 0.0f;
    if (T.kin) {
        const int i = T.kin_lane[link];
        T.k_lf[17 * 64 + i] = mass;
        for (int c = 0; c < 3; ++c) T.k_lf[(18 + c) * 64 + i] = com[c];
    }
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != robot->device) e = hipSetDevice(robot->device);
    char *base = static_cast<char *>(robot->dmem);
    if (e == hipSuccess)
        e = hipMemcpy(base + robot->o_lf + (size_t)link * sizeof(wb::LinkF), &F, sizeof(wb::LinkF),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && T.lanes)
        e = hipMemcpy(base + robot->o_ff, T.f_lf.data(), T.f_lf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess && T.kin)
        e = hipMemcpy(base + robot->o_kf, T.k_lf.data(), T.k_lf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (prev >= 0 && prev != robot->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "updating the link inertia");
    return WB_OK;
}

int wb_robot_set_tool_frames(wb_robot *robot, int32_t n_tools, const int32_t *link, const float *offset) {
    WB_TRY(check_robot(robot));
    const Tables &T = robot->T;
    if (!T.kin)
        return fail(WB_ERR_UNSUPPORTED, "tool frames need n_links <= 64 and n_dof <= 64 (got %d, %d)", T.L, T.n);
    if (n_tools < 0 || n_tools > WB_MAX_TOOLS)
        return fail(WB_ERR_INVALID_ARG, "n_tools %d outside [0, %d]", n_tools, WB_MAX_TOOLS);
    if (n_tools > 0 && (!link || !offset)) return fail(WB_ERR_INVALID_ARG, "link and offset must not be null");
    std::vector<int32_t> lane(WB_MAX_TOOLS, 0);
    std::vector<float> off(12 * WB_MAX_TOOLS, 0.0f);
    std::vector<uint64_t> aff(WB_MAX_TOOLS, 0);
    for (int t = 0; t < n_tools; ++t) {
        if (link[t] < 0 || link[t] >= T.L)
            return fail(WB_ERR_INVALID_ARG, "tool %d: link %d out of range [0, %d)", t, link[t], T.L);
        const float *R = offset + 12 * t;
        if (!finite_all(R, 12)) return fail(WB_ERR_INVALID_ARG, "tool %d: offset is not finite", t);
        double orth = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double d = 0.0;
                for (int c = 0; c < 3; ++c) d += (double)R[3 * c + i] * R[3 * c + j];
                orth = std::fmax(orth, std::fabs(d - (i == j ? 1.0 : 0.0)));
            }
        if (orth > 1e-4) return fail(WB_ERR_INVALID_ARG, "tool %d: offset rotation is not orthonormal", t);
        const int e = T.kin_lane[link[t]];
        lane[t] = e;
        memcpy(off.data() + 12 * t, R, 12 * sizeof(float));
        // affects[j, e]: some link driven by joint j is on e's chain
        for (int j = 0; j < T.n; ++j)
            for (int c = 0; c < T.kin_mc; ++c) {
                const int l = T.k_conn[(size_t)c * 64 + j];
                if (l >= 0 && l <= e && e <= T.kin_sub_end[l]) aff[t] |= 1ull << j;
            }
    }
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != robot->device) e = hipSetDevice(robot->device);
    char *base = static_cast<char *>(robot->dmem);
    if (e == hipSuccess) e = hipMemcpy(base + robot->o_tl, lane.data(), lane.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + robot->o_to, off.data(), off.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + robot->o_ta, aff.data(), aff.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (prev >= 0 && prev != robot->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "uploading the tool frames");
    robot->kin.n_tools = n_tools;
    return WB_OK;
}

int wb_robot_get_tool_count(const wb_robot *robot, int32_t *n_tools) {
    WB_TRY(check_robot(robot));
    if (!n_tools) return fail(WB_ERR_INVALID_ARG, "n_tools is null");
    *n_tools = robot->kin.n_tools;
    return WB_OK;
}

int wb_kinematics(const wb_robot *robot, int64_t B, const float *q, float *link_pose, float *spheres,
                  float *tool_pose, float *com, float *jacobian, float *com_jacobian, hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    const Tables &T = robot->T;
    if (!T.kin)
        return fail(WB_ERR_UNSUPPORTED, "wb_kinematics needs n_links <= 64 and n_dof <= 64 (got %d, %d)", T.L, T.n);
    if ((com || com_jacobian) && !(T.total_mass > 0.0))
        return fail(WB_ERR_INVALID_ARG, "the robot has no mass: its centre of mass is undefined");
    if (B == 0) return WB_OK;
    WB_TRY(check_ptr(q, "q", T.n > 0));
    WB_TRY(check_ptr(link_pose, "link_pose", false));
    WB_TRY(check_ptr(spheres, "spheres", false));
    WB_TRY(check_ptr(tool_pose, "tool_pose", false));
    WB_TRY(check_ptr(com, "com", false));
    WB_TRY(check_ptr(jacobian, "jacobian", false));
    WB_TRY(check_ptr(com_jacobian, "com_jacobian", false));
    wb::KinOut o{link_pose, spheres, tool_pose, com, jacobian, com_jacobian};
    return finish(wb::launch_kinematics(robot->kin, B, B, q, o, stream), "wb_kinematics launch");
}

int wb_kinematics_backward(const wb_robot *robot, int64_t B, const float *q, const float *g_tool_pose,
                           const float *g_com, float *g_q, hipStream_t stream) {
    WB_TRY(check_robot(robot));
    WB_TRY(check_B(B));
    const Tables &T = robot->T;
    if (!T.kin)
        return fail(WB_ERR_UNSUPPORTED, "wb_kinematics_backward needs n_links <= 64 and n_dof <= 64 (got %d, %d)",
                    T.L, T.n);
    if (g_com && !(T.total_mass > 0.0))
        return fail(WB_ERR_INVALID_ARG, "the robot has no mass: its centre of mass is undefined");
    if (B == 0 || T.n == 0) return WB_OK;
    WB_TRY(check_ptr(q, "q", true));
    WB_TRY(check_ptr(g_tool_pose, "g_tool_pose", false));
    WB_TRY(check_ptr(g_com, "g_com", false));
    WB_TRY(check_ptr(g_q, "g_q", true));
    wb::KinGrad g{g_tool_pose, g_com, g_q};
    return finish(wb::launch_kinematics_backward(robot->kin, B, q, g, stream), "wb_kinematics_backward launch");
}

int wb_edt_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, size_t *bytes) {
    if (!bytes) return fail(WB_ERR_INVALID_ARG, "bytes is null");
    if (nx < 1 || ny < 1 || nz < 1 || nx > WB_EDT_MAX_DIM || ny > WB_EDT_MAX_DIM || nz > WB_EDT_MAX_DIM)
        return fail(WB_ERR_INVALID_ARG, "grid %d x %d x %d: extents must be in [1, %d]", nx, ny, nz, WB_EDT_MAX_DIM);
    const size_t N = (size_t)nx * ny * nz;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    *bytes = 2 * up(N * 4);
    return WB_OK;
}

int wb_edt(int32_t nx, int32_t ny, int32_t nz, const uint8_t *sites, float voxel_size, int32_t *nearest, float *dist,
           void *workspace, hipStream_t stream) {
    size_t need = 0;
    WB_TRY(wb_edt_workspace_bytes(nx, ny, nz, &need));
    if (!std::isfinite(voxel_size) || voxel_size < 0.0f)
        return fail(WB_ERR_INVALID_ARG, "voxel_size must be finite and >= 0");
    if (!sites) return fail(WB_ERR_INVALID_ARG, "sites is null");
    if (!workspace) return fail(WB_ERR_INVALID_ARG, "workspace is null");
    if (((uintptr_t)workspace & 255) != 0) return fail(WB_ERR_INVALID_ARG, "workspace is not 256-byte aligned");
    WB_TRY(check_ptr(nearest, "nearest", false));
    WB_TRY(check_ptr(dist, "dist", false));
    const size_t N = (size_t)nx * ny * nz;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *w = static_cast<char *>(workspace);
    int32_t *A = reinterpret_cast<int32_t *>(w);
    int32_t *Bg = reinterpret_cast<int32_t *>(w + up(N * 4));
    // without a nearest-site output the last pass writes into A, free by then
    return finish(wb::launch_edt(nx, ny, nz, sites, voxel_size, nearest ? nearest : A, dist, A, Bg, stream),
                  "wb_edt launch");
}

int wb_edt_noalloc(int32_t nx, int32_t ny, int32_t nz, const uint8_t *sites, float voxel_size, int32_t *nearest,
                   float *dist, hipStream_t stream) {
    size_t need = 0;
    WB_TRY(wb_edt_workspace_bytes(nx, ny, nz, &need));
    const size_t N = (size_t)nx * ny * nz;
    if (N > (size_t)WB_EDT_NOALLOC_MAX_VOXELS)
        return fail(WB_ERR_UNSUPPORTED, "grid %d x %d x %d has %zu voxels; wb_edt_noalloc takes at most %d", nx, ny,
                    nz, N, WB_EDT_NOALLOC_MAX_VOXELS);
    if (!std::isfinite(voxel_size) || voxel_size < 0.0f)
        return fail(WB_ERR_INVALID_ARG, "voxel_size must be finite and >= 0");
    if (!sites) return fail(WB_ERR_INVALID_ARG, "sites is null");
    WB_TRY(check_ptr(nearest, "nearest", false));
    WB_TRY(check_ptr(dist, "dist", false));
    int32_t *scratch = nullptr;
    size_t have = 0;
    const hipError_t e = wb::edt_scratch_address(&scratch, &have);
    if (e != hipSuccess) return hip_fail(e, "looking up the distance-transform scratch array");
    if (have < need) return fail(WB_ERR_UNSUPPORTED, "scratch array of %zu bytes is below the %zu needed", have, need);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    int32_t *A = scratch;
    int32_t *Bg = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(scratch) + up(N * 4));
    return finish(wb::launch_edt(nx, ny, nz, sites, voxel_size, nearest ? nearest : A, dist, A, Bg, stream),
                  "wb_edt_noalloc launch");
}

int wb_robot_get_tune(const wb_robot *robot, wb_tune *tune) {
    WB_TRY(check_robot(robot));
    if (!tune) return fail(WB_ERR_INVALID_ARG, "tune is null");
    *tune = robot->tune;
    return WB_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ plans

struct wb_plan {
    int n_trees = 0, nmax = 1, n_wg = 0, n_items = 0, device = -1;
    int mimic = 0;                  // some tree has mimic joints: the EXT kernel variant
    size_t lds = 0, wave_lds = 0;   // LDS per workgroup, and per wavefront region
    std::vector<int64_t> B;
    std::vector<int> n_dof;
    void *dmem = nullptr;
    const wb::PlanTree *d_trees = nullptr;
    const wb::PlanItem *d_items = nullptr;
    const int32_t *d_item_start = nullptr;
};

namespace {

// Relative cost of one state under a launch shape (used when no measured
// time is given): sweep block iterations x pairs per block x ~14 issue slots,
// plus the link-parallel dynamics, shared by the 64/G states of a wavefront.
double model_cost(const Tables &T, const wb_tune &t, int nmax) {
    const int G = t.lanes_per_state;
    const double iters = (double)((T.n_blocks + G - 1) / G);
    const double slots = iters * nmax * nmax * 14.0 + 1500.0 + 200.0 * T.jsteps;
    return slots * G / 64.0;
}

}  // namespace

extern "C" {

int wb_plan_create(const wb_robot *const *robots, const int64_t *B, int32_t n_trees, const wb_tune *tune,
                   wb_plan **out) {
    if (!out) return fail(WB_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!robots || !B) return fail(WB_ERR_INVALID_ARG, "robots or B is null");
    if (n_trees < 1 || n_trees > WB_PLAN_MAX_TREES)
        return fail(WB_ERR_INVALID_ARG, "n_trees must be in [1, %d]", WB_PLAN_MAX_TREES);
    int nmax = 1, device = -1;
    std::vector<wb_tune> tunes(n_trees);
    for (int i = 0; i < n_trees; ++i) {
        WB_TRY(check_robot(robots[i]));
        WB_TRY(check_B(B[i]));
        if (!robots[i]->fz.supported)
            return fail(WB_ERR_UNSUPPORTED,
                        "tree %d: the fused iteration needs <= 64 links and sweep tables within %zu bytes of LDS", i,
                        wb::LDS_LIMIT);
        if (device >= 0 && robots[i]->device != device)
            return fail(WB_ERR_INVALID_ARG, "all robots of a plan must live on one device");
        device = robots[i]->device;
        nmax = std::max(nmax, robots[i]->T.nmax);
        tunes[i] = tune ? tune[i] : robots[i]->tune;
        WB_TRY(check_tune(tunes[i], robots[i]->T));
    }
    size_t wave_lds = 0, tab_lds = 0;
    for (int i = 0; i < n_trees; ++i) {
        const size_t per_wave = (size_t)(64 / tunes[i].lanes_per_state) *
                                wb::group_lds_bytes(robots[i]->T.L, nmax, robots[i]->T.list_cap);
        wave_lds = std::max(wave_lds, per_wave);
        tab_lds = std::max(tab_lds, wb::tab_lds_bytes((int)robots[i]->T.blocks.size()));
    }
    const size_t lds = 4 * wave_lds + tab_lds;
    if (lds > wb::LDS_LIMIT)
        return fail(WB_ERR_UNSUPPORTED, "plan needs %zu bytes of LDS per workgroup (> %zu)", lds, wb::LDS_LIMIT);

    // Work items: contiguous state ranges of one tree, balanced over the
    // workgroups of one persistent wave of the launch (longest item first).
    struct Item {
        wb::PlanItem it;
        double cost;
    };
    std::vector<Item> items;
    for (int i = 0; i < n_trees; ++i) {
        const int c = tunes[i].states_per_item;
        const double per = tunes[i].ns_per_state > 0.0f ? tunes[i].ns_per_state
                                                         : model_cost(robots[i]->T, tunes[i], nmax);
        for (int64_t b0 = 0; b0 < B[i]; b0 += c) {
            const int cnt = (int)std::min<int64_t>(c, B[i] - b0);
            items.push_back({wb::PlanItem{b0, i, cnt}, per * cnt});
        }
    }
    int cus = 256;
    {
        int dev_cus = 0;
        if (hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
            dev_cus > 0)
            cus = dev_cus;
    }
    // one persistent round: as many workgroups as the compute units keep
    // resident for the kernel variant the plan runs (the mimic variant when
    // a tree has mimic joints; a plan that turns to it for external forces
    // alone runs the same list in more than one round)
    bool any_mimic = false;
    for (int i = 0; i < n_trees; ++i) any_mimic |= robots[i]->fz.mimic != 0;
    const int per_cu = std::min(8, wb::plan_workgroups_per_cu(nmax, any_mimic, lds));
    const int n_wg = (int)std::min<size_t>(items.size(), (size_t)cus * per_cu);
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) { return a.cost > b.cost; });
    std::vector<double> load(n_wg, 0.0);
    std::vector<std::vector<wb::PlanItem>> per_wg(n_wg);
    for (const Item &x : items) {
        int best = 0;
        for (int w = 1; w < n_wg; ++w)
            if (load[w] < load[best]) best = w;
        load[best] += x.cost;
        per_wg[best].push_back(x.it);
    }
    std::vector<wb::PlanItem> flat;
    std::vector<int32_t> start(n_wg + 1, 0);
    for (int w = 0; w < n_wg; ++w) {
        start[w] = (int32_t)flat.size();
        for (const auto &it : per_wg[w]) flat.push_back(it);
    }
    start[n_wg] = (int32_t)flat.size();

    // Per-tree slot tables for the plan's slots per link.
    std::vector<std::vector<float>> slot_r(n_trees);
    std::vector<std::vector<int32_t>> sph_slot(n_trees);
    for (int i = 0; i < n_trees; ++i) {
        const Tables &T = robots[i]->T;
        slot_r[i].assign((size_t)(T.L + 1) * nmax, -1e30f);
        sph_slot[i].resize(T.S);
        for (int s = 0; s < T.S; ++s) {
            const int l = T.sph_link[s];
            sph_slot[i][s] = l * nmax + (s - T.li[l].sph_first);
            slot_r[i][sph_slot[i][s]] = T.sph[s].w;
        }
    }
    std::vector<char> blob;
    std::vector<wb::PlanTree> trees(n_trees);
    const size_t o_items = append(blob, flat), o_start = append(blob, start);
    std::vector<size_t> o_sr(n_trees), o_ss(n_trees);
    for (int i = 0; i < n_trees; ++i) {
        o_sr[i] = append(blob, slot_r[i]);
        o_ss[i] = append(blob, sph_slot[i]);
    }
    const size_t o_trees = append(blob, trees);
    blob.resize(blob.size() + 256);
    wb_plan *p = new wb_plan();
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != device) e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc(&p->dmem, blob.size());
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "allocating the plan");
    }
    char *base = static_cast<char *>(p->dmem);
    for (int i = 0; i < n_trees; ++i) {
        wb::PlanTree &t = trees[i];
        t.rb = robots[i]->dev;
        t.rb.nmax = nmax;
        t.rb.slot_r = reinterpret_cast<const float *>(base + o_sr[i]);
        t.rb.sph_slot = reinterpret_cast<const int32_t *>(base + o_ss[i]);
        t.fz = robots[i]->fz;
        t.B = B[i];
        t.lanes_per_state = tunes[i].lanes_per_state;
        t.pad = 0;
    }
    memcpy(blob.data() + o_trees, trees.data(), trees.size() * sizeof(wb::PlanTree));
    e = hipMemcpy(p->dmem, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->dmem);
        delete p;
        return hip_fail(e, "uploading the plan");
    }
    p->n_trees = n_trees;
    p->nmax = nmax;
    for (int i = 0; i < n_trees; ++i) p->mimic |= robots[i]->fz.mimic;
    p->n_wg = n_wg;
    p->n_items = (int)flat.size();
    p->device = device;
    p->lds = lds;
    p->wave_lds = wave_lds;
    p->B.assign(B, B + n_trees);
    for (int i = 0; i < n_trees; ++i) p->n_dof.push_back(robots[i]->T.n);
    p->d_trees = reinterpret_cast<const wb::PlanTree *>(base + o_trees);
    p->d_items = reinterpret_cast<const wb::PlanItem *>(base + o_items);
    p->d_item_start = reinterpret_cast<const int32_t *>(base + o_start);
    *out = p;
    return WB_OK;
}

int wb_plan_run(const wb_plan *plan, const wb_tree_io *io, float torque_weight, float margin, float hinge_weight,
                float lr, hipStream_t stream) {
    if (!plan || !plan->dmem) return fail(WB_ERR_INVALID_ARG, "plan is null or destroyed");
    if (!io) return fail(WB_ERR_INVALID_ARG, "io is null");
    if (!std::isfinite(torque_weight) || !std::isfinite(margin) || !std::isfinite(hinge_weight) || !std::isfinite(lr))
        return fail(WB_ERR_INVALID_ARG, "weights, margin and lr must be finite");
    wb::PlanArgs a{};
    a.trees = plan->d_trees;
    a.items = plan->d_items;
    a.item_start = plan->d_item_start;
    a.wave_stride = (int32_t)(plan->wave_lds / 16);
    a.k = wb::StepScalars{torque_weight, margin, hinge_weight, lr};
    bool ext = plan->mimic != 0;
    for (int i = 0; i < plan->n_trees; ++i) {
        const wb_tree_io &x = io[i];
        const bool need = plan->B[i] > 0 && plan->n_dof[i] > 0;
        WB_TRY(check_ptr(x.q, "io.q", need));
        WB_TRY(check_ptr(x.qd, "io.qd", need));
        WB_TRY(check_ptr(x.qdd, "io.qdd", need));
        WB_TRY(check_ptr(x.w, "io.w", false));
        WB_TRY(check_ptr(x.tau, "io.tau", false));
        WB_TRY(check_ptr(x.cost, "io.cost", false));
        WB_TRY(check_ptr(x.max_pen, "io.max_pen", false));
        WB_TRY(check_ptr(x.argmax, "io.argmax", false));
        WB_TRY(check_ptr(x.n_coll, "io.n_coll", false));
        WB_TRY(check_ptr(x.g_q, "io.g_q", false));
        WB_TRY(check_ptr(x.g_qd, "io.g_qd", false));
        WB_TRY(check_ptr(x.g_qdd, "io.g_qdd", false));
        WB_TRY(check_ptr(x.f_ext, "io.f_ext", false));
        WB_TRY(check_ptr(x.g_fext, "io.g_fext", false));
        int64_t ld = 0;
        WB_TRY(resolve_ld(plan->B[i], x.ld, &ld));
        a.io[i] = wb::TreeIO{x.q,     x.qd,     x.qdd, x.w,    x.tau,   x.cost,   x.max_pen, x.argmax,
                             x.n_coll, x.g_q, x.g_qd, x.g_qdd, x.f_ext, x.g_fext, ld};
        ext = ext || x.f_ext || x.g_fext;
    }
    return finish(wb::launch_plan(a, plan->nmax, plan->n_wg, plan->lds, ext, stream), "wb_plan_run launch");
}

int wb_plan_capture(const wb_plan *plan, const wb_tree_io *io, float torque_weight, float margin, float hinge_weight,
                    float lr, int32_t iters, hipGraphExec_t *out) {
    if (!out) return fail(WB_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!plan || !plan->dmem) return fail(WB_ERR_INVALID_ARG, "plan is null or destroyed");
    if (iters < 1 || iters > (1 << 20)) return fail(WB_ERR_INVALID_ARG, "iters %d outside [1, 2^20]", iters);
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != plan->device) e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "selecting the plan's device");
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    int rc = WB_OK;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int i = 0; i < iters && rc == WB_OK; ++i)
            rc = wb_plan_run(plan, io, torque_weight, margin, hinge_weight, lr, s);
        const hipError_t e2 = hipStreamEndCapture(s, &g);
        if (rc == WB_OK) e = e2;
    }
    if (rc == WB_OK && e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (s) (void)hipStreamDestroy(s);
    if (prev >= 0 && prev != plan->device) (void)hipSetDevice(prev);
    if (rc != WB_OK) return rc;   // wb_plan_run's message stands
    if (e != hipSuccess) return hip_fail(e, "capturing the plan into a graph");
    *out = x;
    return WB_OK;
}

int wb_graph_launch(hipGraphExec_t graph, hipStream_t stream) {
    if (!graph) return fail(WB_ERR_INVALID_ARG, "graph is null");
    return finish(hipGraphLaunch(graph, stream), "launching the graph");
}

int wb_graph_destroy(hipGraphExec_t graph) {
    if (!graph) return WB_OK;
    return finish(hipGraphExecDestroy(graph), "destroying the graph");
}

int wb_plan_get_info(const wb_plan *plan, int32_t *n_items, int32_t *n_workgroups) {
    if (!plan || !plan->dmem) return fail(WB_ERR_INVALID_ARG, "plan is null or destroyed");
    if (n_items) *n_items = plan->n_items;
    if (n_workgroups) *n_workgroups = plan->n_wg;
    return WB_OK;
}

int wb_plan_destroy(wb_plan *plan) {
    if (!plan) return WB_OK;
    hipError_t e = hipSuccess;
    if (plan->dmem) e = hipFree(plan->dmem);
    plan->dmem = nullptr;
    delete plan;
    return finish(e, "freeing the plan");
}

}  // extern "C"
