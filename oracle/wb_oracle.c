/*
 * wb_oracle.c -- plain, slow, FP64 CPU oracle for the batched whole-body
 * computation of cuRoboV2 (arXiv 2603.05493): forward kinematics to link
 * poses and collision-sphere centres, recursive Newton-Euler inverse
 * dynamics, all-pairs self-collision, and the adjoints of each.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP library; it is written directly from the
 * paper's definitions, one state at a time, with OpenMP over states.
 *
 * Conventions (the paper leaves these implicit; the readings are listed in
 * the design notes):
 *   - Link 0 is the fixed root at the world identity.  Link k >= 1 sits at
 *     parentT_k(q) = [fixed_R_k | fixed_p_k] * Rot(axis_k, theta_k), with
 *     theta_k = mult_k * q[jidx_k] + off_k (mimic joints, Sec. 6.3) and the
 *     axis in the child frame.  Rot is Rodrigues' formula.
 *   - Spatial vectors are Featherstone [angular; linear] in link coordinates
 *     (Sec. 6.3, Fig. "RNEA Forward and Backward Kernels").  The compact
 *     parent-to-child transform is X*[w;v] = [E w; E (v - r x w)] with
 *     E = (fixed_R * Rot)^T and r = fixed_p (the identity given in Sec. 6.3,
 *     "Compact spatial representations").
 *   - Inertia: mass m, CoM c and rotational inertia Ic about the CoM in link
 *     axes; I*[w;v] = [Ic w + c x h; h], h = m (v + w x c).
 *   - The base acceleration is minus gravity (fictitious-acceleration
 *     treatment of the root line of Alg. 4).
 *   - Self-collision pairs are sphere pairs (s,t), s < t, on different links
 *     that are not parent and child (or as given by an explicit link-pair
 *     allow matrix), numbered lexicographically in (s,t).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int L, n, S;
    const int *parent;     /* [L] */
    const int *jtype;      /* [L] 0 fixed, 1 revolute */
    const int *jidx;       /* [L] actuated joint index or -1 */
    const double *jmult;   /* [L] */
    const double *joff;    /* [L] */
    const double *axis;    /* [L][3] */
    const double *fR;      /* [L][9] row-major */
    const double *fp;      /* [L][3] */
    const double *mass;    /* [L] */
    const double *com;     /* [L][3] */
    const double *inertia; /* [L][9] */
    const int *sph_link;   /* [S] */
    const double *sph_pos; /* [S][3] */
    const double *sph_r;   /* [S] */
    const double *gravity; /* [3] */
    const unsigned char *allow; /* [L][L] or NULL */
} orc_robot;

/* ------------------------------------------------------------ 3-vectors */

static void cross3(const double a[3], const double b[3], double o[3]) {
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
/* o = M a (M row-major 3x3) */
static void matvec(const double M[9], const double a[3], double o[3]) {
    double x = M[0] * a[0] + M[1] * a[1] + M[2] * a[2];
    double y = M[3] * a[0] + M[4] * a[1] + M[5] * a[2];
    double z = M[6] * a[0] + M[7] * a[1] + M[8] * a[2];
    o[0] = x; o[1] = y; o[2] = z;
}
/* o = M^T a */
static void matTvec(const double M[9], const double a[3], double o[3]) {
    double x = M[0] * a[0] + M[3] * a[1] + M[6] * a[2];
    double y = M[1] * a[0] + M[4] * a[1] + M[7] * a[2];
    double z = M[2] * a[0] + M[5] * a[1] + M[8] * a[2];
    o[0] = x; o[1] = y; o[2] = z;
}
/* O = A B */
static void matmul(const double A[9], const double B[9], double O[9]) {
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    memcpy(O, T, sizeof T);
}

/* Rodrigues' formula: R = I + sin(th) K + (1 - cos(th)) K K, K = [s]x. */
static void rodrigues(const double s[3], double th, double R[9]) {
    double K[9] = {0, -s[2], s[1], s[2], 0, -s[0], -s[1], s[0], 0};
    double K2[9];
    matmul(K, K, K2);
    double sn = sin(th), vc = 1.0 - cos(th);
    for (int i = 0; i < 9; ++i) R[i] = K[i] * sn + K2[i] * vc;
    R[0] += 1.0; R[4] += 1.0; R[8] += 1.0;
}

/* ------------------------------------------------------- joint helpers */

static double theta_of(const orc_robot *rb, int k, const double *q) {
    if (rb->jtype[k] != 1 || rb->jidx[k] < 0) return 0.0;
    return rb->jmult[k] * q[rb->jidx[k]] + rb->joff[k];
}
static double rate_of(const orc_robot *rb, int k, const double *qd) {
    if (rb->jtype[k] != 1 || rb->jidx[k] < 0) return 0.0;
    return rb->jmult[k] * qd[rb->jidx[k]];
}

/* Local rotation fixed_R * Rot(axis, theta) of link k. */
static void local_rotation(const orc_robot *rb, int k, const double *q, double Rl[9]) {
    double Rj[9];
    if (rb->jtype[k] == 1) rodrigues(rb->axis + 3 * k, theta_of(rb, k, q), Rj);
    else { memset(Rj, 0, sizeof Rj); Rj[0] = Rj[4] = Rj[8] = 1.0; }
    matmul(rb->fR + 9 * k, Rj, Rl);
}

/* ------------------------------------------------------ spatial algebra
 * Featherstone spatial algebra (Sec. 6.3): vectors are [ang(3); lin(3)]. */

/* out = X u with X the parent->child transform (E = Rl^T, r = fixed_p). */
static void X_apply(const double Rl[9], const double r[3], const double u[6], double out[6]) {
    double t[3], rxw[3];
    cross3(r, u, rxw);
    t[0] = u[3] - rxw[0]; t[1] = u[4] - rxw[1]; t[2] = u[5] - rxw[2];
    double o[6];
    matTvec(Rl, u, o);
    matTvec(Rl, t, o + 3);
    memcpy(out, o, sizeof o);
}
/* out = X^T f: [E^T n + r x (E^T f); E^T f]. */
static void XT_apply(const double Rl[9], const double r[3], const double f[6], double out[6]) {
    double n[3], ff[3], rf[3];
    matvec(Rl, f, n);
    matvec(Rl, f + 3, ff);
    cross3(r, ff, rf);
    out[0] = n[0] + rf[0]; out[1] = n[1] + rf[1]; out[2] = n[2] + rf[2];
    out[3] = ff[0]; out[4] = ff[1]; out[5] = ff[2];
}
/* motion cross product: crm(v) u = [w x uw; w x ul + vl x uw] */
static void crm(const double v[6], const double u[6], double o[6]) {
    double a[3], b[3], c[3];
    cross3(v, u, a);
    cross3(v, u + 3, b);
    cross3(v + 3, u, c);
    o[0] = a[0]; o[1] = a[1]; o[2] = a[2];
    o[3] = b[0] + c[0]; o[4] = b[1] + c[1]; o[5] = b[2] + c[2];
}
/* force cross product: crf(v) f = [w x fn + vl x ff; w x ff] */
static void crf(const double v[6], const double f[6], double o[6]) {
    double a[3], b[3], c[3];
    cross3(v, f, a);
    cross3(v + 3, f + 3, b);
    cross3(v, f + 3, c);
    o[0] = a[0] + b[0]; o[1] = a[1] + b[1]; o[2] = a[2] + b[2];
    o[3] = c[0]; o[4] = c[1]; o[5] = c[2];
}
/* spatial inertia product from (m, c, Ic). */
static void I_apply(const orc_robot *rb, int k, const double u[6], double o[6]) {
    const double m = rb->mass[k];
    const double *c = rb->com + 3 * k;
    double wxc[3], h[3], Icw[3], cxh[3];
    cross3(u, c, wxc);
    h[0] = m * (u[3] + wxc[0]); h[1] = m * (u[4] + wxc[1]); h[2] = m * (u[5] + wxc[2]);
    matvec(rb->inertia + 9 * k, u, Icw);
    cross3(c, h, cxh);
    o[0] = Icw[0] + cxh[0]; o[1] = Icw[1] + cxh[1]; o[2] = Icw[2] + cxh[2];
    o[3] = h[0]; o[4] = h[1]; o[5] = h[2];
}
static void motion_subspace(const orc_robot *rb, int k, double S[6]) {
    memset(S, 0, 6 * sizeof(double));
    if (rb->jtype[k] == 1) { S[0] = rb->axis[3 * k]; S[1] = rb->axis[3 * k + 1]; S[2] = rb->axis[3 * k + 2]; }
}
static double dot6(const double a[6], const double b[6]) {
    double s = 0.0;
    for (int i = 0; i < 6; ++i) s += a[i] * b[i];
    return s;
}

static int max_depth(const orc_robot *rb, int *depth) {
    int md = 0;
    depth[0] = 0;
    for (int k = 1; k < rb->L; ++k) {
        depth[k] = depth[rb->parent[k]] + 1;
        if (depth[k] > md) md = depth[k];
    }
    return md;
}

/* ------------------------------------------------------------------ FK
 * Forward kinematics (Sec. 6.1, "Forward Kinematics"): world pose of every
 * link by composing parent pose and local transform, then sphere centres
 * c = R_link * c_local + p_link.  R [B][L][9], p [B][L][3], c [B][S][3];
 * any output may be NULL. */
static void fk_one(const orc_robot *rb, const double *q, double *Rw, double *pw) {
    memset(Rw, 0, 9 * sizeof(double));
    Rw[0] = Rw[4] = Rw[8] = 1.0;
    pw[0] = pw[1] = pw[2] = 0.0;
    for (int k = 1; k < rb->L; ++k) {
        int p = rb->parent[k];
        double Rl[9], t[3];
        local_rotation(rb, k, q, Rl);
        matmul(Rw + 9 * p, Rl, Rw + 9 * k);
        matvec(Rw + 9 * p, rb->fp + 3 * k, t);
        pw[3 * k] = t[0] + pw[3 * p];
        pw[3 * k + 1] = t[1] + pw[3 * p + 1];
        pw[3 * k + 2] = t[2] + pw[3 * p + 2];
    }
}

void orc_fk(const orc_robot *rb, int B, const double *q, double *R, double *p, double *c) {
    const int L = rb->L, S = rb->S, n = rb->n;
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b) {
        double *Rw = (double *)malloc(sizeof(double) * 12 * L);
        double *pw = Rw + 9 * L;
        fk_one(rb, q + (size_t)b * n, Rw, pw);
        if (R) memcpy(R + (size_t)b * L * 9, Rw, sizeof(double) * 9 * L);
        if (p) memcpy(p + (size_t)b * L * 3, pw, sizeof(double) * 3 * L);
        if (c) {
            for (int s = 0; s < S; ++s) {
                int l = rb->sph_link[s];
                double t[3];
                matvec(Rw + 9 * l, rb->sph_pos + 3 * s, t);
                double *cs = c + ((size_t)b * S + s) * 3;
                cs[0] = t[0] + pw[3 * l];
                cs[1] = t[1] + pw[3 * l + 1];
                cs[2] = t[2] + pw[3 * l + 2];
            }
        }
        free(Rw);
    }
}

/* ---------------------------------------------------------- FK backward
 * Joint gradients from link-pose and sphere-centre gradients (Alg. 1,
 * "Backprop with Topology Cache"): every link with a gradient walks its
 * ancestor chain and adds, for each ancestor joint k, the projection of its
 * gradient on the motion that joint induces: for a point x,
 * dx/dtheta_k = s_k x (x - o_k), and for a rotation, dR/dtheta_k = [s_k]x R,
 * with s_k the joint's world axis and o_k its world origin.  gR [B][L][9],
 * gp [B][L][3], gc [B][S][3] (each may be NULL); gq [B][n] is overwritten. */
void orc_fk_backward(const orc_robot *rb, int B, const double *q, const double *gR,
                     const double *gp, const double *gc, double *gq) {
    const int L = rb->L, S = rb->S, n = rb->n;
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b) {
        double *Rw = (double *)malloc(sizeof(double) * 16 * L);
        double *pw = Rw + 9 * L;
        double *th = pw + 3 * L;        /* theta-bar per link */
        fk_one(rb, q + (size_t)b * n, Rw, pw);
        for (int k = 0; k < L; ++k) th[k] = 0.0;
        if (gc) {
            for (int s = 0; s < S; ++s) {
                const double *g = gc + ((size_t)b * S + s) * 3;
                int l = rb->sph_link[s];
                double x[3];
                matvec(Rw + 9 * l, rb->sph_pos + 3 * s, x);
                x[0] += pw[3 * l]; x[1] += pw[3 * l + 1]; x[2] += pw[3 * l + 2];
                for (int k = l; k > 0; k = rb->parent[k]) {
                    if (rb->jtype[k] != 1) continue;
                    double sw[3], d[3], m[3];
                    matvec(Rw + 9 * k, rb->axis + 3 * k, sw);
                    d[0] = x[0] - pw[3 * k]; d[1] = x[1] - pw[3 * k + 1]; d[2] = x[2] - pw[3 * k + 2];
                    cross3(sw, d, m);
                    th[k] += dot3(g, m);
                }
            }
        }
        if (gR || gp) {
            for (int l = 0; l < L; ++l) {
                for (int k = l; k > 0; k = rb->parent[k]) {
                    if (rb->jtype[k] != 1) continue;
                    double sw[3];
                    matvec(Rw + 9 * k, rb->axis + 3 * k, sw);
                    if (gR) {
                        /* sum_ij gR_ij ([s]x R)_ij */
                        const double *G = gR + ((size_t)b * L + l) * 9;
                        const double *Rl = Rw + 9 * l;
                        double acc = 0.0;
                        for (int j = 0; j < 3; ++j) {
                            double col[3] = {Rl[j], Rl[3 + j], Rl[6 + j]}, sc[3];
                            cross3(sw, col, sc);
                            acc += G[j] * sc[0] + G[3 + j] * sc[1] + G[6 + j] * sc[2];
                        }
                        th[k] += acc;
                    }
                    if (gp) {
                        const double *g = gp + ((size_t)b * L + l) * 3;
                        double d[3], m[3];
                        d[0] = pw[3 * l] - pw[3 * k]; d[1] = pw[3 * l + 1] - pw[3 * k + 1];
                        d[2] = pw[3 * l + 2] - pw[3 * k + 2];
                        cross3(sw, d, m);
                        th[k] += dot3(g, m);
                    }
                }
            }
        }
        double *gqb = gq + (size_t)b * n;
        for (int j = 0; j < n; ++j) gqb[j] = 0.0;
        for (int k = 1; k < L; ++k)
            if (rb->jtype[k] == 1 && rb->jidx[k] >= 0) gqb[rb->jidx[k]] += rb->jmult[k] * th[k];
        free(Rw);
    }
}

/* ------------------------------------------------------------------ RNEA
 * Inverse dynamics by Alg. 4 ("RNEA Forward"): a base-to-tips level sweep
 * for velocities and accelerations, a per-link force pass, and a
 * tips-to-base level sweep accumulating forces into joint torques.  fext is
 * [B][L][6] in link coordinates or NULL.  Optionally returns the per-link
 * v, a and accumulated force F of every link (each [L][6]) for one state. */
static void rnea_one(const orc_robot *rb, const int *depth, int md, const double *q,
                     const double *qd, const double *qdd, const double *fext, double *tau,
                     double *v, double *a, double *F) {
    const int L = rb->L;
    for (int i = 0; i < 6; ++i) { v[i] = 0.0; a[i] = 0.0; }
    a[3] = -rb->gravity[0]; a[4] = -rb->gravity[1]; a[5] = -rb->gravity[2];
    /* Pass 1: base -> tips, by level. */
    for (int lev = 1; lev <= md; ++lev) {
        for (int k = 1; k < L; ++k) {
            if (depth[k] != lev) continue;
            int p = rb->parent[k];
            double Rl[9], S[6], Sqd[6], t[6], c[6];
            local_rotation(rb, k, q, Rl);
            motion_subspace(rb, k, S);
            double thd = rate_of(rb, k, qd), thdd = rate_of(rb, k, qdd);
            for (int i = 0; i < 6; ++i) Sqd[i] = S[i] * thd;
            X_apply(Rl, rb->fp + 3 * k, v + 6 * p, t);
            for (int i = 0; i < 6; ++i) v[6 * k + i] = t[i] + Sqd[i];
            X_apply(Rl, rb->fp + 3 * k, a + 6 * p, t);
            crm(v + 6 * k, Sqd, c);
            for (int i = 0; i < 6; ++i) a[6 * k + i] = t[i] + S[i] * thdd + c[i];
        }
    }
    /* Pass 2: forces. */
    for (int k = 0; k < L; ++k) {
        double Ia[6], Iv[6], vxIv[6];
        I_apply(rb, k, a + 6 * k, Ia);
        I_apply(rb, k, v + 6 * k, Iv);
        crf(v + 6 * k, Iv, vxIv);
        for (int i = 0; i < 6; ++i) F[6 * k + i] = Ia[i] + vxIv[i] - (fext ? fext[6 * k + i] : 0.0);
    }
    /* Pass 3: tips -> base, by level. */
    for (int j = 0; j < rb->n; ++j) tau[j] = 0.0;
    for (int lev = md; lev >= 1; --lev) {
        for (int k = L - 1; k >= 1; --k) {
            if (depth[k] != lev) continue;
            int p = rb->parent[k];
            double S[6], Rl[9], t[6];
            motion_subspace(rb, k, S);
            if (rb->jtype[k] == 1 && rb->jidx[k] >= 0)
                tau[rb->jidx[k]] += rb->jmult[k] * dot6(S, F + 6 * k);
            local_rotation(rb, k, q, Rl);
            XT_apply(Rl, rb->fp + 3 * k, F + 6 * k, t);
            for (int i = 0; i < 6; ++i) F[6 * p + i] += t[i];
        }
    }
}

void orc_rnea(const orc_robot *rb, int B, const double *q, const double *qd, const double *qdd,
              const double *fext, double *tau) {
    const int L = rb->L, n = rb->n;
    int *depth = (int *)malloc(sizeof(int) * L);
    int md = max_depth(rb, depth);
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b) {
        double *w = (double *)malloc(sizeof(double) * 18 * L);
        rnea_one(rb, depth, md, q + (size_t)b * n, qd + (size_t)b * n, qdd + (size_t)b * n,
                 fext ? fext + (size_t)b * L * 6 : NULL, tau + (size_t)b * n, w, w + 6 * L, w + 12 * L);
        free(w);
    }
    free(depth);
}

/* ------------------------------------------------------------- RNEA VJP
 * Vector-Jacobian product of Alg. 4 (the role of Alg. 5, "RNEA Backward
 * (VJP)"): given tau-bar, returns q-bar, qd-bar, qdd-bar (overwritten) and
 * optionally fext-bar = -F-bar.  Derived as the exact reverse mode of the
 * forward sweep above, with dX/dtheta = -crm(S) X:
 *   pass 1 (base -> tips): Fb_k = m S taub_j + X Fb_p;
 *                          thb_k += (X Fb_p)^T crf(S) F_k;
 *   pass 3 (tips -> base): ab_k += I Fb_k;
 *                          vb_k += -crf(Fb_k) I v_k - I crm(v_k) Fb_k
 *                                  + crf(S thd_k) ab_k;
 *                          thdd-bar = S^T ab_k;
 *                          thd-bar  = S^T vb_k - S^T crf(v_k) ab_k;
 *                          thb_k   -= ab_k^T crm(S) X a_p + vb_k^T crm(S) X v_p;
 *                          ab_p += X^T ab_k;  vb_p += X^T vb_k.
 * The term crf(S thd_k) ab_k (velocity dependence of the Coriolis term in the
 * acceleration recursion) is part of the exact reverse mode even though the
 * printed listing does not show it; finite differences confirm it.  The
 * root link is the fixed base, so every jointed link receives all terms. */
void orc_rnea_vjp(const orc_robot *rb, int B, const double *q, const double *qd,
                  const double *qdd, const double *fext, const double *gtau, double *gq,
                  double *gqd, double *gqdd, double *gfext) {
    const int L = rb->L, n = rb->n;
    int *depth = (int *)malloc(sizeof(int) * L);
    int md = max_depth(rb, depth);
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b) {
        const double *qb = q + (size_t)b * n, *qdb = qd + (size_t)b * n, *qddb = qdd + (size_t)b * n;
        const double *tb = gtau + (size_t)b * n;
        double *w = (double *)malloc(sizeof(double) * (36 * L + 3 * L + n));
        double *v = w, *a = w + 6 * L, *F = w + 12 * L;
        double *Fb = w + 18 * L, *ab = w + 24 * L, *vb = w + 30 * L;
        double *thb = w + 36 * L, *thdb = thb + L, *thddb = thdb + L, *tau = thddb + L;
        rnea_one(rb, depth, md, qb, qdb, qddb, fext ? fext + (size_t)b * L * 6 : NULL, tau, v, a, F);
        for (int i = 0; i < 18 * L; ++i) Fb[i] = 0.0;
        for (int k = 0; k < L; ++k) thb[k] = thdb[k] = thddb[k] = 0.0;
        /* pass 1: adjoint of the tips->base accumulation, base -> tips */
        for (int lev = 1; lev <= md; ++lev) {
            for (int k = 1; k < L; ++k) {
                if (depth[k] != lev) continue;
                int p = rb->parent[k];
                double S[6], Rl[9], XFp[6], cF[6];
                motion_subspace(rb, k, S);
                local_rotation(rb, k, qb, Rl);
                double tbk = (rb->jtype[k] == 1 && rb->jidx[k] >= 0) ? rb->jmult[k] * tb[rb->jidx[k]] : 0.0;
                X_apply(Rl, rb->fp + 3 * k, Fb + 6 * p, XFp);
                for (int i = 0; i < 6; ++i) Fb[6 * k + i] = S[i] * tbk + XFp[i];
                crf(S, F + 6 * k, cF);
                thb[k] += dot6(XFp, cF);
            }
        }
        if (gfext) {
            double *g = gfext + (size_t)b * L * 6;
            for (int i = 0; i < 6 * L; ++i) g[i] = -Fb[i];
        }
        /* pass 3: adjoint of the base->tips sweep and the force pass, tips -> base */
        for (int lev = md; lev >= 1; --lev) {
            for (int k = L - 1; k >= 1; --k) {
                if (depth[k] != lev) continue;
                int p = rb->parent[k];
                double S[6], Rl[9], t[6], u[6], Iv[6], cv[6], Sqd[6];
                motion_subspace(rb, k, S);
                local_rotation(rb, k, qb, Rl);
                double thd = rate_of(rb, k, qdb);
                I_apply(rb, k, Fb + 6 * k, t);
                for (int i = 0; i < 6; ++i) ab[6 * k + i] += t[i];
                I_apply(rb, k, v + 6 * k, Iv);
                crf(Fb + 6 * k, Iv, t);
                crm(v + 6 * k, Fb + 6 * k, cv);
                I_apply(rb, k, cv, u);
                for (int i = 0; i < 6; ++i) vb[6 * k + i] -= t[i] + u[i];
                for (int i = 0; i < 6; ++i) Sqd[i] = S[i] * thd;
                crf(Sqd, ab + 6 * k, t);
                for (int i = 0; i < 6; ++i) vb[6 * k + i] += t[i];
                thddb[k] += dot6(S, ab + 6 * k);
                crf(v + 6 * k, ab + 6 * k, t);
                thdb[k] += dot6(S, vb + 6 * k) - dot6(S, t);
                X_apply(Rl, rb->fp + 3 * k, a + 6 * p, t);
                crm(S, t, u);
                thb[k] -= dot6(ab + 6 * k, u);
                X_apply(Rl, rb->fp + 3 * k, v + 6 * p, t);
                crm(S, t, u);
                thb[k] -= dot6(vb + 6 * k, u);
                XT_apply(Rl, rb->fp + 3 * k, ab + 6 * k, t);
                for (int i = 0; i < 6; ++i) ab[6 * p + i] += t[i];
                XT_apply(Rl, rb->fp + 3 * k, vb + 6 * k, t);
                for (int i = 0; i < 6; ++i) vb[6 * p + i] += t[i];
            }
        }
        double *gqb = gq + (size_t)b * n, *gqdb = gqd + (size_t)b * n, *gqddb = gqdd + (size_t)b * n;
        for (int j = 0; j < n; ++j) gqb[j] = gqdb[j] = gqddb[j] = 0.0;
        for (int k = 1; k < L; ++k) {
            if (rb->jtype[k] != 1 || rb->jidx[k] < 0) continue;
            int j = rb->jidx[k];
            double m = rb->jmult[k];
            gqb[j] += m * thb[k];
            gqdb[j] += m * thdb[k];
            gqddb[j] += m * thddb[k];
        }
        free(w);
    }
    free(depth);
}

/* ------------------------------------------------------- self-collision
 * All-pairs sphere self-collision (Sec. 6.2, "Self-Collision via
 * Map-Reduce"), by brute-force enumeration.  Pair (s,t), s < t, is checked
 * when the two spheres sit on different links that are not parent and
 * child (or, with an explicit matrix, when allow[a][b] is set).  pen =
 * r_s + r_t - |c_s - c_t|; the result per state is the largest pen, the
 * lowest pair index attaining it, and the number of pairs with pen > 0. */
static int link_pair_allowed(const orc_robot *rb, int a, int b) {
    if (a == b) return 0;
    if (rb->allow) return rb->allow[a * rb->L + b] != 0;
    return rb->parent[b] != a && rb->parent[a] != b;
}

int orc_pairs(const orc_robot *rb, int *ps, int *pt) {
    int P = 0;
    for (int s = 0; s < rb->S; ++s)
        for (int t = s + 1; t < rb->S; ++t)
            if (link_pair_allowed(rb, rb->sph_link[s], rb->sph_link[t])) {
                if (ps) { ps[P] = s; pt[P] = t; }
                ++P;
            }
    return P;
}

void orc_self_collision_pens(const orc_robot *rb, int B, const double *c, double *pen) {
    const int S = rb->S;
    int P = orc_pairs(rb, NULL, NULL);
    int *ps = (int *)malloc(sizeof(int) * (P + 1)), *pt = (int *)malloc(sizeof(int) * (P + 1));
    orc_pairs(rb, ps, pt);
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b) {
        const double *cb = c + (size_t)b * S * 3;
        for (int i = 0; i < P; ++i) {
            const double *x = cb + 3 * ps[i], *y = cb + 3 * pt[i];
            double d = sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) +
                            (x[2] - y[2]) * (x[2] - y[2]));
            pen[(size_t)b * P + i] = rb->sph_r[ps[i]] + rb->sph_r[pt[i]] - d;
        }
    }
    free(ps); free(pt);
}

void orc_self_collision(const orc_robot *rb, int B, const double *c, double *maxpen,
                        int *argmax, int *ncoll) {
    const int S = rb->S;
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b) {
        const double *cb = c + (size_t)b * S * 3;
        double best = -INFINITY;
        int arg = -1, cnt = 0, idx = 0;
        for (int s = 0; s < S; ++s) {
            for (int t = s + 1; t < S; ++t) {
                if (!link_pair_allowed(rb, rb->sph_link[s], rb->sph_link[t])) continue;
                const double *x = cb + 3 * s, *y = cb + 3 * t;
                double d = sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) +
                                (x[2] - y[2]) * (x[2] - y[2]));
                double pen = rb->sph_r[s] + rb->sph_r[t] - d;
                if (pen > best) { best = pen; arg = idx; }
                if (pen > 0.0) ++cnt;
                ++idx;
            }
        }
        maxpen[b] = best;
        argmax[b] = arg;
        ncoll[b] = cnt;
    }
}

/* Hinge cost h = max(0, maxpen + margin) and its subgradient at the most
 * penetrating pair (zero where h = 0 or the pair's spheres coincide):
 * d maxpen / d c_s = -(c_s - c_t)/|c_s - c_t|, d/d c_t = +(c_s - c_t)/|.|.
 * gc [B][S][3] is overwritten; gcost [B] is the upstream gradient on h. */
void orc_self_collision_backward(const orc_robot *rb, int B, const double *c,
                                 const int *argmax, const double *maxpen, double margin,
                                 const double *gcost, double *gc) {
    const int S = rb->S;
    int P = orc_pairs(rb, NULL, NULL);
    int *ps = (int *)malloc(sizeof(int) * (P + 1)), *pt = (int *)malloc(sizeof(int) * (P + 1));
    orc_pairs(rb, ps, pt);
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b) {
        double *g = gc + (size_t)b * S * 3;
        for (int i = 0; i < 3 * S; ++i) g[i] = 0.0;
        int p = argmax[b];
        if (p < 0 || !(maxpen[b] + margin > 0.0)) continue;
        const double *cb = c + (size_t)b * S * 3;
        int s = ps[p], t = pt[p];
        double d3[3] = {cb[3 * s] - cb[3 * t], cb[3 * s + 1] - cb[3 * t + 1], cb[3 * s + 2] - cb[3 * t + 2]};
        double d = sqrt(dot3(d3, d3));
        if (!(d > 0.0)) continue;
        for (int i = 0; i < 3; ++i) {
            g[3 * s + i] += -gcost[b] * d3[i] / d;
            g[3 * t + i] += gcost[b] * d3[i] / d;
        }
    }
    free(ps); free(pt);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the OpenMP loops above (timing only; results do not depend on it). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
