/* FP64 CPU oracle of the SPaSM data-parallel hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use this file.
 * It is written for clarity, not speed: every cost term is evaluated pair by pair,
 * and every gradient is assembled with textbook geometric Jacobians
 *     d p / d q_j = z_{j-1} x (p - o_{j-1}),   d u / d q_j = z_{j-1} x u
 * for points p and directions u attached to the links (j <= link index).
 *
 * Paper references (Chen, Iyer, Kingston, "Differentiable Particle Optimization for
 * Fast Sequential Manipulation", arXiv 2510.07674):
 *   Sec. III            problem: penetration penalties, everything is spheres
 *   Alg. 1              sample -> cost -> argsort/top-M -> linear descent with
 *                       eta = eta_init (1 - k/K_lin) -> quadratic refinement at alpha
 *                       -> satisfying particles -> best
 *   Sec. III-A          pose clamping into the problem bounding box; linear vs
 *                       quadratic cost formulations
 *   Sec. III-B          lift by IK, intermediate waypoints, linear interpolation,
 *                       gradient descent over the whole trajectory
 *   Appendix B          tower costs C_placement = w_stable C_stable + w_height C_height
 *                       + w_coll C_coll; C_trajopt = C_placement + w_start C_start
 *                       + w_arm C_arm + w_block C_block
 * Readings of points the paper leaves open are listed where they are used.
 *
 * Parity unpinned: the paper allows any parallel IK and any sampled intermediate
 * waypoint, so two choices here are this implementation's own and nothing in the paper
 * fixes them -- the multi-start lift's rule (among converged starts the one least deep in
 * the clutter, ik_multistart) and the seeding's best-of-candidates rule for the
 * intermediate waypoint (or_traj_init).  Tests check them only against restatements of
 * the same rules; the GPU follows the same rules.
 *
 * Diagnostics (or_traj_residuals, or_traj_slot_residuals, or_box_clearance) take the
 * violation apart by kind or measure a plan's clearance from boxes; they serve the scene
 * builder and failure analysis, not parity.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NJ 7
#define OR_PI 3.14159265358979323846
#define STREAM_SAMPLE 1u
#define STREAM_IK 2u
#define STREAM_MID 3u

/* ------------------------------------------------------------------------------------
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11).  Uniforms use the top 24 bits: u = (x >> 40) * 2^-24.
 * ------------------------------------------------------------------------------------ */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void uniforms4(uint64_t seed, uint64_t a, uint64_t b, uint64_t c, uint64_t stream,
                      double u[4])
{
    uint64_t ctr[4] = {a, b, c, stream}, key[2] = {seed, 0}, o[4];
    or_philox4x64_10(ctr, key, o);
    for (int i = 0; i < 4; ++i) u[i] = (double)(o[i] >> 40) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------------------
 * Small vector helpers and rigid frames (R row-major 3x3, p translation).
 * ------------------------------------------------------------------------------------ */
typedef struct { double R[9], p[3]; } frame;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static void col(const frame *F, int c, double *v) { v[0] = F->R[c]; v[1] = F->R[3 + c]; v[2] = F->R[6 + c]; }
static void apply(const frame *F, const double *x, double *y)
{
    for (int i = 0; i < 3; ++i) y[i] = F->R[3 * i] * x[0] + F->R[3 * i + 1] * x[1] + F->R[3 * i + 2] * x[2] + F->p[i];
}
static void compose(const frame *A, const frame *B, frame *C)
{
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            C->R[3 * i + j] = A->R[3 * i] * B->R[j] + A->R[3 * i + 1] * B->R[3 + j] + A->R[3 * i + 2] * B->R[6 + j];
        C->p[i] = A->R[3 * i] * B->p[0] + A->R[3 * i + 1] * B->p[1] + A->R[3 * i + 2] * B->p[2] + A->p[i];
    }
}
static double sgn(double x) { return x >= 0.0 ? 1.0 : -1.0; }
static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }
static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* ------------------------------------------------------------------------------------
 * Forward kinematics (Appendix B uses fk(q); the chain is given by classic DH parameters):
 *   A_k(theta) = Rz(theta) Tz(d_k) Tx(a_k) Rx(alpha_k),  T_0 = I,  T_k = T_{k-1} A_k(q_k),
 *   T_E = T_7 Tz(tool_d).
 * frames[0..7] are T_0..T_7 and frames[8] is T_E.
 * ------------------------------------------------------------------------------------ */
static void fk_frames(const or_problem *pb, const double *q, frame F[9])
{
    memset(&F[0], 0, sizeof(frame));
    F[0].R[0] = F[0].R[4] = F[0].R[8] = 1.0;
    for (int k = 1; k <= NJ; ++k) {
        double a = pb->dh[3 * (k - 1)], d = pb->dh[3 * (k - 1) + 1], al = pb->dh[3 * (k - 1) + 2];
        double ct = cos(q[k - 1]), st = sin(q[k - 1]), ca = cos(al), sa = sin(al);
        frame A = {{ct, -st * ca, st * sa, st, ct * ca, -ct * sa, 0.0, sa, ca}, {a * ct, a * st, d}};
        compose(&F[k - 1], &A, &F[k]);
    }
    frame T = {{1, 0, 0, 0, 1, 0, 0, 0, 1}, {0, 0, pb->tool_d}};
    compose(&F[7], &T, &F[8]);
}

void or_fk(const or_problem *pb, const double *q, double *frames)
{
    frame F[9];
    fk_frames(pb, q, F);
    for (int k = 0; k < 9; ++k) {
        memcpy(frames + 12 * k, F[k].R, 9 * sizeof(double));
        memcpy(frames + 12 * k + 9, F[k].p, 3 * sizeof(double));
    }
}

/* dC/dq += (dC/dp) . (z_{j-1} x (p - o_{j-1})) for a point on link L (1..7) */
static void jac_point(const frame F[9], int L, const double *p, const double *gp, double *gq)
{
    for (int j = 1; j <= L; ++j) {
        double z[3], r[3], t[3];
        col(&F[j - 1], 2, z);
        for (int i = 0; i < 3; ++i) r[i] = p[i] - F[j - 1].p[i];
        cross3(z, r, t);
        gq[j - 1] += dot3(gp, t);
    }
}

/* dC/dq += (dC/du) . (z_{j-1} x u) for a direction on link L */
static void jac_dir(const frame F[9], int L, const double *u, const double *gu, double *gq)
{
    for (int j = 1; j <= L; ++j) {
        double z[3], t[3];
        col(&F[j - 1], 2, z);
        cross3(z, u, t);
        gq[j - 1] += dot3(gu, t);
    }
}

/* ------------------------------------------------------------------------------------
 * Signed distance to an axis-aligned box (closest-point form, e.g. Ericson, Real-Time
 * Collision Detection, Sec. 5.1.3):  u = |p - c| - e,
 *   outside: sdf = |max(u, 0)|, grad = sgn(p - c) * max(u, 0) / |max(u, 0)|
 *   inside : sdf = max_i u_i,   grad = sgn(p_k - c_k) e_k with k the first argmax.
 * feat (optional) is the gap between the two largest u when inside (where the
 * gradient switches faces), +inf outside.
 * ------------------------------------------------------------------------------------ */
static double box_sdf_ex(const double *p, const double *box, double *g, double *feat)
{
    double d[3], u[3], qq = 0.0;
    int out = 0;
    for (int i = 0; i < 3; ++i) {
        d[i] = p[i] - box[i];
        u[i] = fabs(d[i]) - box[3 + i];
        if (u[i] > 0.0) {
            qq += u[i] * u[i];
            out = 1;
        }
    }
    if (out) {
        double n = sqrt(qq);
        for (int i = 0; i < 3; ++i) g[i] = (u[i] > 0.0 ? u[i] / n : 0.0) * sgn(d[i]);
        if (feat) *feat = INFINITY;
        return n;
    }
    int k = 0;
    for (int i = 1; i < 3; ++i)
        if (u[i] > u[k]) k = i;
    double second = -INFINITY;
    for (int i = 0; i < 3; ++i)
        if (i != k && u[i] > second) second = u[i];
    for (int i = 0; i < 3; ++i) g[i] = 0.0;
    g[k] = sgn(d[k]);
    if (feat) *feat = u[k] - second;
    return u[k];
}

double or_box_sdf(const double *p, const double *box, double *grad)
{
    return box_sdf_ex(p, box, grad, NULL);
}

/* Box of half edge `half` with pose (x, y, z, yaw): sdf(Rz(-yaw)(p - t)).
 * gp = d sdf / dp, gpose = d sdf / d(x, y, z, yaw). */
static double obb_sdf_ex(const double *p, const double *pose, double half, double *gp,
                         double *gpose, double *feat)
{
    double c = cos(pose[3]), s = sin(pose[3]);
    double dx = p[0] - pose[0], dy = p[1] - pose[1], dz = p[2] - pose[2];
    double pl[3] = {c * dx + s * dy, -s * dx + c * dy, dz};
    double box0[6] = {0, 0, 0, half, half, half}, gl[3];
    double sdf = box_sdf_ex(pl, box0, gl, feat);
    gp[0] = c * gl[0] - s * gl[1];
    gp[1] = s * gl[0] + c * gl[1];
    gp[2] = gl[2];
    if (gpose) {
        gpose[0] = -gp[0];
        gpose[1] = -gp[1];
        gpose[2] = -gp[2];
        /* d pl / d yaw = (pl_y, -pl_x, 0) */
        gpose[3] = gl[0] * pl[1] - gl[1] * pl[0];
    }
    return sdf;
}

double or_obb_sdf(const double *p, const double *pose, double half, double *gp, double *gpose)
{
    return obb_sdf_ex(p, pose, half, gp, gpose, NULL);
}

/* Phase shaping (Sec. III-A): the linear phase uses residuals as they are, the quadratic
 * phase squares them.  Terms that are squared by definition are not reshaped. */
static double phi(int phase, double d) { return phase == OR_QUAD ? d * d : d; }
static double dphi(int phase, double d) { return phase == OR_QUAD ? 2.0 * d : 1.0; }

/* Kink margin of one sphere-box pair: distance of the pair from any point where its
 * penalty gradient jumps (activation r = sdf; face switches inside; edge/corner
 * transition at the surface). */
static double pair_kink(double r, double sdf, double feat)
{
    double m = fabs(r - sdf);
    if (r - sdf > 0.0) m = dmin(m, dmin(fabs(sdf), feat));
    return m;
}

/* Motion segments of a particle: transit and transfer per block, or the one motion of a
 * point-to-point problem (mode 3). */
static int n_seg(const or_problem *pb) { return pb->mode == 3 ? 1 : 2 * pb->B; }

static double zstar(const or_problem *pb, int i)
{
    if (pb->mode == 2) return 0.5 * pb->h; /* packing: every piece rests on the table */
    return pb->mode == 0 ? (i + 0.5) * pb->h : pb->goal[4 * i + 2];
}

/* Block collision spheres (a cube as spheres, Sec. III): 8 spheres at (+-h/4)^3 in the
 * block frame, radius h/4 - block_margin so that stacked blocks do not touch. */
static void block_sphere(double h, int k, double *sb)
{
    double qd = 0.25 * h;
    sb[0] = (k & 1) ? qd : -qd;
    sb[1] = (k & 2) ? qd : -qd;
    sb[2] = (k & 4) ? qd : -qd;
}

/* ------------------------------------------------------------------------------------
 * Packing geometry (Appendix A, Tetris problem).  A piece is a union of square cells of
 * edge h that share the piece's yaw; penetration depths are those of the squares.
 * ------------------------------------------------------------------------------------ */

/* Penetration depth of two squares of half edge s (centres ca, cb, yaws tha, thb) by the
 * separating axis theorem: along each of the four edge normals n (ua, va of square a, ub,
 * vb of square b) the two projections overlap by
 *     s (|ua.n| + |va.n|) + s (|ub.n| + |vb.n|) - |(ca - cb).n|,
 * and the depth (minimum translation distance) is the smallest of the four, or 0 when one
 * of them is <= 0 (a separating axis).  g, when not NULL, receives
 * d depth / d (ca_x, ca_y, tha, cb_x, cb_y, thb) for the axis of the smallest overlap
 * (the first of ua, va, ub, vb on ties) and, in g[6], the distance of the configuration
 * from a gradient switch: the gap to the second-smallest overlap, the depth itself,
 * the projection of ca - cb on the chosen axis, and |cos|, |sin| of the relative yaw. */
double or_square_pen(const double *ca, double tha, const double *cb, double thb, double s, double *g)
{
    const double ua[2] = {cos(tha), sin(tha)}, va[2] = {-sin(tha), cos(tha)};
    const double ub[2] = {cos(thb), sin(thb)}, vb[2] = {-sin(thb), cos(thb)};
    const double d[2] = {ca[0] - cb[0], ca[1] - cb[1]};
    const double *axis[4] = {ua, va, ub, vb};
    /* derivative of each axis by tha and by thb: ua' = va, va' = -ua (same for b) */
    const double zero[2] = {0.0, 0.0}, mua[2] = {-ua[0], -ua[1]}, mub[2] = {-ub[0], -ub[1]};
    const double *dax[4] = {va, mua, zero, zero}, *dbx[4] = {zero, zero, vb, mub};
    double ov[4], gov[4][6];
    for (int k = 0; k < 4; ++k) {
        const double *n = axis[k], *na = dax[k], *nb = dbx[k];
        double pu = ua[0] * n[0] + ua[1] * n[1], pv = va[0] * n[0] + va[1] * n[1];
        double qu = ub[0] * n[0] + ub[1] * n[1], qv = vb[0] * n[0] + vb[1] * n[1];
        double dist = d[0] * n[0] + d[1] * n[1];
        ov[k] = s * (fabs(pu) + fabs(pv) + fabs(qu) + fabs(qv)) - fabs(dist);
        /* derivatives of the projections by tha and thb */
        double pu_a = va[0] * n[0] + va[1] * n[1] + ua[0] * na[0] + ua[1] * na[1];
        double pv_a = -(ua[0] * n[0] + ua[1] * n[1]) + va[0] * na[0] + va[1] * na[1];
        double qu_a = ub[0] * na[0] + ub[1] * na[1], qv_a = vb[0] * na[0] + vb[1] * na[1];
        double pu_b = ua[0] * nb[0] + ua[1] * nb[1], pv_b = va[0] * nb[0] + va[1] * nb[1];
        double qu_b = vb[0] * n[0] + vb[1] * n[1] + ub[0] * nb[0] + ub[1] * nb[1];
        double qv_b = -(ub[0] * n[0] + ub[1] * n[1]) + vb[0] * nb[0] + vb[1] * nb[1];
        double sd = sgn(dist);
        gov[k][0] = -sd * n[0];
        gov[k][1] = -sd * n[1];
        gov[k][2] = s * (sgn(pu) * pu_a + sgn(pv) * pv_a + sgn(qu) * qu_a + sgn(qv) * qv_a) -
                    sd * (d[0] * na[0] + d[1] * na[1]);
        gov[k][3] = sd * n[0];
        gov[k][4] = sd * n[1];
        gov[k][5] = s * (sgn(pu) * pu_b + sgn(pv) * pv_b + sgn(qu) * qu_b + sgn(qv) * qv_b) -
                    sd * (d[0] * nb[0] + d[1] * nb[1]);
    }
    int best = 0;
    for (int k = 1; k < 4; ++k)
        if (ov[k] < ov[best]) best = k;
    double pen = ov[best] > 0.0 ? ov[best] : 0.0;
    if (g) {
        for (int c = 0; c < 6; ++c) g[c] = pen > 0.0 ? gov[best][c] : 0.0;
        double gap = INFINITY;
        for (int k = 0; k < 4; ++k)
            if (k != best) gap = dmin(gap, ov[k] - ov[best]);
        double dist = d[0] * axis[best][0] + d[1] * axis[best][1];
        double cr = ua[0] * ub[0] + ua[1] * ub[1], sr = ua[0] * ub[1] - ua[1] * ub[0];
        double kink = fabs(ov[best]);
        if (ov[best] > 0.0) kink = dmin(kink, dmin(gap, dmin(fabs(dist), dmin(fabs(cr), fabs(sr)))));
        g[6] = kink;
    }
    return pen;
}

/* Depth of a square (centre c, yaw th, half edge s) past a wall line with inward unit
 * normal m at offset b (the interior is m.p >= b): b - (m.c - s (|ua.m| + |va.m|)).
 * gc, gth: derivatives by c and th; kink: distance from a gradient switch. */
static double wall_depth(const double *c, double th, double s, const double *m, double b, double *gc, double *gth,
                         double *kink)
{
    const double ua[2] = {cos(th), sin(th)}, va[2] = {-sin(th), cos(th)};
    double pu = ua[0] * m[0] + ua[1] * m[1], pv = va[0] * m[0] + va[1] * m[1];
    double dep = b - (c[0] * m[0] + c[1] * m[1]) + s * (fabs(pu) + fabs(pv));
    gc[0] = -m[0];
    gc[1] = -m[1];
    *gth = s * (sgn(pu) * pv - sgn(pv) * pu);
    *kink = fabs(dep);
    if (dep > 0.0) *kink = dmin(*kink, dmin(fabs(pu), fabs(pv)));
    return dep;
}

/* Packing placement cost of one particle (Appendix A):
 *   C = sum_{i<j} Pen(piece i, piece j) + sum_i sum_{walls} Pen(piece i, wall) + height term
 * Pen(piece, piece) = sum over the cell pairs of phi(square depth); Pen(piece, wall) = sum
 * over the cells of phi(depth past the wall); the walls are the four sides of the
 * placement region.  The 3-dof state keeps z at h/2, so the height term is zero; the
 * 4-dof state adds w_height (z - h/2)^2 as for towers (the paper's |z - z*| read as the
 * same squared residual).  Every term is weighted by w_coll. */
static void pack_one(const or_problem *pb, int dim, int phase, const double *x, double *cost_out,
                     double *viol_out, double *g, double *kink_out)
{
    const int B = pb->B;
    const double s = 0.5 * pb->h, w_height = pb->w[1], w_coll = pb->w[2];
    const double *T = pb->table;
    const double wall_m[4][2] = {{1.0, 0.0}, {-1.0, 0.0}, {0.0, 1.0}, {0.0, -1.0}};
    const double wall_b[4] = {T[0], -T[1], T[2], -T[3]};
    double P[B][4], gP[B][4];
    for (int i = 0; i < B; ++i) {
        P[i][0] = x[i * dim + 0];
        P[i][1] = x[i * dim + 1];
        P[i][2] = dim == 4 ? x[i * dim + 2] : zstar(pb, i);
        P[i][3] = x[i * dim + dim - 1];
        for (int c = 0; c < 4; ++c) gP[i][c] = 0.0;
    }
    double cost = 0.0, viol = 0.0, kink = INFINITY;
    /* cell centre of cell k of piece i and its derivative by the piece yaw */
    double C[B][8][2], dC[B][8][2];
    for (int i = 0; i < B; ++i) {
        double c = cos(P[i][3]), sn = sin(P[i][3]);
        for (int k = 0; k < pb->pack_cells[i]; ++k) {
            const double *o = pb->pack_off + (i * 8 + k) * 2;
            C[i][k][0] = P[i][0] + c * o[0] - sn * o[1];
            C[i][k][1] = P[i][1] + sn * o[0] + c * o[1];
            dC[i][k][0] = -sn * o[0] - c * o[1];
            dC[i][k][1] = c * o[0] - sn * o[1];
        }
    }
    for (int i = 0; i < B; ++i) {
        for (int k = 0; k < pb->pack_cells[i]; ++k) {
            for (int wl = 0; wl < 4; ++wl) {
                double gc[2], gth, kk;
                double dep = wall_depth(C[i][k], P[i][3], s, wall_m[wl], wall_b[wl], gc, &gth, &kk);
                kink = dmin(kink, kk);
                if (dep > 0.0) {
                    cost += w_coll * phi(phase, dep);
                    viol = dmax(viol, dep);
                    double sc = w_coll * dphi(phase, dep);
                    gP[i][0] += sc * gc[0];
                    gP[i][1] += sc * gc[1];
                    gP[i][3] += sc * (gc[0] * dC[i][k][0] + gc[1] * dC[i][k][1] + gth);
                }
            }
            for (int j = i + 1; j < B; ++j)
                for (int m = 0; m < pb->pack_cells[j]; ++m) {
                    double gs[7];
                    double pen = or_square_pen(C[i][k], P[i][3], C[j][m], P[j][3], s, gs);
                    kink = dmin(kink, gs[6]);
                    if (pen > 0.0) {
                        cost += w_coll * phi(phase, pen);
                        viol = dmax(viol, pen);
                        double sc = w_coll * dphi(phase, pen);
                        gP[i][0] += sc * gs[0];
                        gP[i][1] += sc * gs[1];
                        gP[i][3] += sc * (gs[0] * dC[i][k][0] + gs[1] * dC[i][k][1] + gs[2]);
                        gP[j][0] += sc * gs[3];
                        gP[j][1] += sc * gs[4];
                        gP[j][3] += sc * (gs[3] * dC[j][m][0] + gs[4] * dC[j][m][1] + gs[5]);
                    }
                }
        }
    }
    for (int i = 0; i < B; ++i) {
        double e = P[i][2] - zstar(pb, i);
        cost += w_height * e * e;
        viol = dmax(viol, fabs(e));
        gP[i][2] += 2.0 * w_height * e;
    }
    *cost_out = cost;
    *viol_out = viol;
    if (kink_out) *kink_out = kink;
    if (g)
        for (int i = 0; i < B; ++i) {
            g[i * dim + 0] = gP[i][0];
            g[i * dim + 1] = gP[i][1];
            if (dim == 4) g[i * dim + 2] = gP[i][2];
            g[i * dim + dim - 1] = gP[i][3];
        }
}

/* ------------------------------------------------------------------------------------
 * Tower placement cost of one particle (Appendix B):
 *   C_coll   = sum_{i<j} Pen(B_i, B_j) + sum_{i,o} Pen(B_i, o)
 *              + sum_{i<j} Pen(B_i, block j at its initial pose)   [block i is placed
 *                while the later blocks j are still where they started]
 *   C_stable = sum_{i=1}^{B-1} Dist(CoM(blocks above i), Footprint(block i))
 *   C_height = sum_i (z_i - z_i*)^2,  z_i* = (i + 1/2) h  (0-based i: block centre)
 * Pen(A, box) = sum over spheres s of A of max(0, r_s - sdf_box(c_s)).
 * Dist = 2-D distance from the centre of mass (equal masses) of the blocks above to the
 * h x h footprint square of block i (0 inside).  Fixed-goal problems have no stability
 * term.  dim 3: x, y, yaw (z at its slot); dim 4: x, y, z, yaw.
 * ------------------------------------------------------------------------------------ */
static void place_one(const or_problem *pb, int dim, int phase, const double *x, double *cost_out,
                      double *viol_out, double *g, double *kink_out)
{
    const int B = pb->B;
    const double h = pb->h, rb = 0.25 * h - pb->block_margin;
    const double w_stable = pb->w[0], w_height = pb->w[1], w_coll = pb->w[2];
    double P[B][4], gP[B][4];
    for (int i = 0; i < B; ++i) {
        P[i][0] = x[i * dim + 0];
        P[i][1] = x[i * dim + 1];
        P[i][2] = dim == 4 ? x[i * dim + 2] : zstar(pb, i);
        P[i][3] = x[i * dim + dim - 1];
        for (int c = 0; c < 4; ++c) gP[i][c] = 0.0;
    }
    double cost = 0.0, viol = 0.0, kink = INFINITY;

    for (int i = 0; i < B; ++i) {
        double ci = cos(P[i][3]), si = sin(P[i][3]);
        for (int k = 0; k < 8; ++k) {
            double sb[3], c[3], dcdy[3];
            block_sphere(h, k, sb);
            c[0] = P[i][0] + ci * sb[0] - si * sb[1];
            c[1] = P[i][1] + si * sb[0] + ci * sb[1];
            c[2] = P[i][2] + sb[2];
            dcdy[0] = -si * sb[0] - ci * sb[1];
            dcdy[1] = ci * sb[0] - si * sb[1];
            dcdy[2] = 0.0;
            /* every target this sphere is tested against: obstacles, placed blocks j>i,
             * and the initial poses of blocks j>i */
            int ntarget = pb->O + 2 * (B - 1 - i);
            for (int t = 0; t < ntarget; ++t) {
                double gp[3], gpo[4], feat, sdf;
                int movable = -1;
                if (t < pb->O) {
                    sdf = box_sdf_ex(c, pb->boxes + 6 * t, gp, &feat);
                } else if (t < pb->O + (B - 1 - i)) {
                    int j = i + 1 + (t - pb->O);
                    sdf = obb_sdf_ex(c, P[j], 0.5 * h, gp, gpo, &feat);
                    movable = j;
                } else {
                    int j = i + 1 + (t - pb->O - (B - 1 - i));
                    sdf = obb_sdf_ex(c, pb->block_init + 4 * j, 0.5 * h, gp, gpo, &feat);
                }
                double delta = rb - sdf;
                kink = dmin(kink, pair_kink(rb, sdf, feat));
                if (delta > 0.0) {
                    cost += w_coll * phi(phase, delta);
                    viol = dmax(viol, delta);
                    double s = -w_coll * dphi(phase, delta);  /* d cost / d sdf */
                    for (int a = 0; a < 3; ++a) gP[i][a] += s * gp[a];
                    gP[i][3] += s * dot3(gp, dcdy);
                    if (movable >= 0)
                        for (int a = 0; a < 4; ++a) gP[movable][a] += s * gpo[a];
                }
            }
        }
    }

    if (pb->mode == 0) {
        for (int i = 0; i + 1 < B; ++i) {
            double mx = 0.0, my = 0.0;
            int n = B - 1 - i;
            for (int j = i + 1; j < B; ++j) {
                mx += P[j][0];
                my += P[j][1];
            }
            mx /= n;
            my /= n;
            double c = cos(P[i][3]), s = sin(P[i][3]);
            double ex = mx - P[i][0], ey = my - P[i][1];
            double v[2] = {c * ex + s * ey, -s * ex + c * ey};
            double a[2] = {dmax(fabs(v[0]) - 0.5 * h, 0.0), dmax(fabs(v[1]) - 0.5 * h, 0.0)};
            double D = sqrt(a[0] * a[0] + a[1] * a[1]);
            kink = dmin(kink, dmin(fabs(fabs(v[0]) - 0.5 * h), fabs(fabs(v[1]) - 0.5 * h)));
            viol = dmax(viol, D);
            cost += w_stable * phi(phase, D);
            if (D > 0.0) {
                double gw = w_stable * dphi(phase, D);
                double dv[2] = {sgn(v[0]) * a[0] / D, sgn(v[1]) * a[1] / D};
                /* v = Rz(-yaw)(m - t): dD/dm = Rz(yaw) dD/dv, dD/dt = -dD/dm,
                 * d v / d yaw = (v_y, -v_x) */
                double dm[2] = {c * dv[0] - s * dv[1], s * dv[0] + c * dv[1]};
                for (int j = i + 1; j < B; ++j) {
                    gP[j][0] += gw * dm[0] / n;
                    gP[j][1] += gw * dm[1] / n;
                }
                gP[i][0] -= gw * dm[0];
                gP[i][1] -= gw * dm[1];
                gP[i][3] += gw * (dv[0] * v[1] - dv[1] * v[0]);
            }
        }
    }

    for (int i = 0; i < B; ++i) {
        double e = P[i][2] - zstar(pb, i);
        cost += w_height * e * e;
        viol = dmax(viol, fabs(e));
        gP[i][2] += 2.0 * w_height * e;
    }

    *cost_out = cost;
    *viol_out = viol;
    if (kink_out) *kink_out = kink;
    if (g) {
        for (int i = 0; i < B; ++i) {
            g[i * dim + 0] = gP[i][0];
            g[i * dim + 1] = gP[i][1];
            if (dim == 4) g[i * dim + 2] = gP[i][2];
            g[i * dim + dim - 1] = gP[i][3];
        }
    }
}

void or_place_cost(const or_problem *pb, int dim, int phase, int N, const double *x, double *cost,
                   double *viol, double *grad, double *kink)
{
    const int B = pb->B;
#pragma omp parallel for schedule(dynamic, 4)
    for (int n = 0; n < N; ++n)
        (pb->mode == 2 ? pack_one : place_one)(pb, dim, phase, x + (size_t)n * B * dim, cost + n, viol + n,
                                               grad ? grad + (size_t)n * B * dim : NULL, kink ? kink + n : NULL);
}

/* ------------------------------------------------------------------------------------
 * Stage-2 cost of one waypoint slot (s, w) of one particle (Appendix B, C_trajopt):
 * s = 2b is the transit to block b, s = 2b+1 carries block b to its placement.
 *   arm spheres vs every box obstacle                                  (C_arm)
 *   arm spheres vs the blocks as they stand at that moment: blocks b' < b at their
 *     placed poses (optimised), b' > b at their initial poses, block b at its initial
 *     pose during the transit except at the grasp waypoint, and not during its own
 *     transfer (it is in the hand)                                     (arm-block)
 *   held block spheres vs obstacles and the other blocks, interior transfer waypoints
 *     w in [1, W-2]                                                    (C_block)
 *   grasp alignment at the first transfer waypoint: block frame T_E G^-1 against the
 *     initial pose, position and tilt of the block z axis (roll/pitch) (C_start)
 *   tie at the last transfer waypoint: block frame against the placement variable,
 *     position, x axis (yaw) and z axis                                 (C_tie)
 *   joint-limit hinges                                                  (C_lim)
 * ------------------------------------------------------------------------------------ */
/* residual categories of the violation (or_traj_residuals) */
enum { CAT_ARM_BOX, CAT_ARM_BLOCK, CAT_HELD_BOX, CAT_HELD_BLOCK, CAT_GRASP, CAT_TIE, CAT_LIMIT, CAT_PLACE, N_CAT };

typedef struct {
    double cost, viol, kink, pose_kink;
    double cat[N_CAT];
} slot_out;

static void note(slot_out *so, int cat, double r)
{
    so->viol = dmax(so->viol, r);
    so->cat[cat] = dmax(so->cat[cat], r);
}

static void sphere_vs_targets(const or_problem *pb, int phase, double wgt, const frame F[9], int L,
                              const double *c, double r, int b, int tau, int w, int W,
                              int arm, const double *pose, double *gq, double *gpose, slot_out *so)
{
    const int B = pb->B;
    const double h = pb->h;
    for (int o = 0; o < pb->O; ++o) {
        double g[3], feat;
        double sdf = box_sdf_ex(c, pb->boxes + 6 * o, g, &feat);
        double delta = r - sdf;
        so->kink = dmin(so->kink, pair_kink(r, sdf, feat));
        if (delta > 0.0) {
            so->cost += wgt * phi(phase, delta);
            note(so, arm ? CAT_ARM_BOX : CAT_HELD_BOX, delta);
            double s = -wgt * dphi(phase, delta), gc[3] = {s * g[0], s * g[1], s * g[2]};
            jac_point(F, L, c, gc, gq);
        }
    }
    /* a point-to-point problem has no blocks to collide with */
    for (int bb = 0; bb < (pb->mode == 3 ? 0 : B); ++bb) {
        const double *bp;
        int movable = 0;
        if (bb < b) {
            bp = pose + 4 * bb;
            movable = 1;
        } else if (bb > b) {
            bp = pb->block_init + 4 * bb;
        } else {
            if (arm && tau == 0 && w < W - 1)
                bp = pb->block_init + 4 * bb;
            else
                continue;
        }
        double gp[3], gpo[4], feat;
        double sdf = obb_sdf_ex(c, bp, 0.5 * h, gp, gpo, &feat);
        double delta = r - sdf;
        double km = pair_kink(r, sdf, feat);
        so->kink = dmin(so->kink, km);
        if (movable) so->pose_kink = dmin(so->pose_kink, km);
        if (delta > 0.0) {
            so->cost += wgt * phi(phase, delta);
            note(so, arm ? CAT_ARM_BLOCK : CAT_HELD_BLOCK, delta);
            double s = -wgt * dphi(phase, delta), gc[3] = {s * gp[0], s * gp[1], s * gp[2]};
            jac_point(F, L, c, gc, gq);
            if (movable)
                for (int a = 0; a < 4; ++a) gpose[4 * bb + a] += s * gpo[a];
        }
    }
}

static void traj_slot(const or_problem *pb, int phase, int W, int s, int w, const double *q,
                      const double *pose, const double *lam, double *e_out, double *gq, double *gpose,
                      slot_out *so)
{
    const int b = s / 2, tau = s % 2;
    const double h = pb->h;
    const double w_start = pb->w[3], w_tie = pb->w[4], w_arm = pb->w[5], w_block = pb->w[6],
                 w_lim = pb->w[7];
    frame F[9];
    fk_frames(pb, q, F);

    for (int i = 0; i < pb->S; ++i) {
        int L = pb->sph_link[i];
        double c[3];
        apply(&F[L], pb->sph_c + 3 * i, c);
        sphere_vs_targets(pb, phase, w_arm, F, L, c, pb->sph_r[i], b, tau, w, W, 1, pose, gq,
                          gpose, so);
    }

    /* block frame from the end effector: T_B = T_E G^-1 */
    const double *G = pb->grasp;
    frame Gi;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Gi.R[3 * i + j] = G[4 * j + i];
    for (int i = 0; i < 3; ++i) Gi.p[i] = -(Gi.R[3 * i] * G[3] + Gi.R[3 * i + 1] * G[7] + Gi.R[3 * i + 2] * G[11]);
    frame TB;
    compose(&F[8], &Gi, &TB);

    if (tau == 1 && w >= 1 && w <= W - 2) {
        double rb = 0.25 * h - pb->block_margin;
        for (int k = 0; k < 8; ++k) {
            double sb[3], c[3];
            block_sphere(h, k, sb);
            apply(&TB, sb, c);
            sphere_vs_targets(pb, phase, w_block, F, 7, c, rb, b, tau, w, W, 0, pose, gq, gpose, so);
        }
    }

    if (tau == 1 && w == 0) {
        const double *I = pb->block_init + 4 * b;
        double rp[3], u[3], rz[3];
        for (int i = 0; i < 3; ++i) rp[i] = TB.p[i] - I[i];
        col(&TB, 2, u);
        rz[0] = u[0];
        rz[1] = u[1];
        rz[2] = u[2] - 1.0;
        double c2 = dot3(rp, rp) + dot3(rz, rz);
        so->cost += w_start * c2;
        note(so, CAT_GRASP, sqrt(c2));
        double gp[3], gu[3];
        for (int i = 0; i < 3; ++i) {
            gp[i] = 2.0 * w_start * rp[i];
            gu[i] = 2.0 * w_start * rz[i];
        }
        /* equality residual e = (rp, rz) of block b, components 0..5; multiplier term
         * lambda . e of the augmented Lagrangian */
        if (e_out)
            for (int i = 0; i < 3; ++i) {
                e_out[15 * b + i] = rp[i];
                e_out[15 * b + 3 + i] = rz[i];
            }
        if (lam) {
            const double *l = lam + 15 * b;
            so->cost += dot3(l, rp) + dot3(l + 3, rz);
            for (int i = 0; i < 3; ++i) {
                gp[i] += l[i];
                gu[i] += l[3 + i];
            }
        }
        jac_point(F, 7, TB.p, gp, gq);
        jac_dir(F, 7, u, gu, gq);
    }

    if (tau == 1 && w == W - 1) {
        const double *P = pose + 4 * b;
        double cps = cos(P[3]), sps = sin(P[3]);
        double rp[3], ux[3], uz[3], rx[3], rz[3];
        for (int i = 0; i < 3; ++i) rp[i] = TB.p[i] - P[i];
        col(&TB, 0, ux);
        col(&TB, 2, uz);
        rx[0] = ux[0] - cps;
        rx[1] = ux[1] - sps;
        rx[2] = ux[2];
        rz[0] = uz[0];
        rz[1] = uz[1];
        rz[2] = uz[2] - 1.0;
        double c2 = dot3(rp, rp) + dot3(rx, rx) + dot3(rz, rz);
        so->cost += w_tie * c2;
        note(so, CAT_TIE, sqrt(c2));
        double gp[3], gx[3], gz[3];
        for (int i = 0; i < 3; ++i) {
            gp[i] = 2.0 * w_tie * rp[i];
            gx[i] = 2.0 * w_tie * rx[i];
            gz[i] = 2.0 * w_tie * rz[i];
        }
        /* equality residual (rp, rx, rz) of block b, components 6..14 */
        if (e_out)
            for (int i = 0; i < 3; ++i) {
                e_out[15 * b + 6 + i] = rp[i];
                e_out[15 * b + 9 + i] = rx[i];
                e_out[15 * b + 12 + i] = rz[i];
            }
        if (lam) {
            const double *l = lam + 15 * b + 6;
            so->cost += dot3(l, rp) + dot3(l + 3, rx) + dot3(l + 6, rz);
            for (int i = 0; i < 3; ++i) {
                gp[i] += l[i];
                gx[i] += l[3 + i];
                gz[i] += l[6 + i];
            }
        }
        jac_point(F, 7, TB.p, gp, gq);
        jac_dir(F, 7, ux, gx, gq);
        jac_dir(F, 7, uz, gz, gq);
        for (int i = 0; i < 3; ++i) gpose[4 * b + i] -= gp[i];
        gpose[4 * b + 3] -= gx[0] * (-sps) + gx[1] * cps;
    }

    for (int j = 0; j < NJ; ++j) {
        /* not a kink for parity: with FP32-exact limits and inputs both precisions take
         * the same hinge decision */
        double eh = q[j] - pb->hi[j], el = pb->lo[j] - q[j];
        if (eh > 0.0) {
            so->cost += w_lim * phi(phase, eh);
            note(so, CAT_LIMIT, eh);
            gq[j] += w_lim * dphi(phase, eh);
        }
        if (el > 0.0) {
            so->cost += w_lim * phi(phase, el);
            note(so, CAT_LIMIT, el);
            gq[j] -= w_lim * dphi(phase, el);
        }
    }
}

/* Whole stage-2 cost of a batch of particles: every slot, the smoothness objective
 * (squared configuration-space steps inside each segment; the objective of Sec. III is
 * configuration-space distance) and the placement cost of the pose variables. */
void or_traj_cost(const or_problem *pb, int phase, int P, int W, const double *q, const double *pose,
                  double *cost, double *viol, double *gq, double *gpose, double *slot_kink,
                  double *pose_kink)
{
    or_traj_cost_al(pb, phase, P, W, q, pose, NULL, NULL, cost, viol, gq, gpose, slot_kink, pose_kink);
}

/* The stage-2 cost with the augmented Lagrangian's multiplier terms: lam [P][B][15]
 * (nullable) adds lambda . e for each block's equality residual e (grasp alignment rp,
 * rz: components 0..5; tie rp, rx, rz: 6..14); e_out [P][B][15] (nullable) receives e. */
static void traj_cost_impl(const or_problem *pb, int phase, int P, int W, const double *q, const double *pose,
                           const double *lam, double *e_out, double *cost, double *viol, double *gq, double *gpose,
                           double *slot_kink, double *pose_kink, double *cat_out, double *slot_cat_out);

void or_traj_cost_al(const or_problem *pb, int phase, int P, int W, const double *q, const double *pose,
                     const double *lam, double *e_out, double *cost, double *viol, double *gq, double *gpose,
                     double *slot_kink, double *pose_kink)
{
    traj_cost_impl(pb, phase, P, W, q, pose, lam, e_out, cost, viol, gq, gpose, slot_kink, pose_kink, NULL, NULL);
}

/* Diagnostics: per particle, the largest residual of each kind that makes up the
 * violation -- arm spheres in a box, arm spheres in a block, held block in a box, held
 * block in another block, grasp, tie, joint limit, placement cost of the pose variables
 * (block-block / block-box penetration, stability, height) -- as cat [P][8]; their
 * maximum is the violation. */
void or_traj_residuals(const or_problem *pb, int P, int W, const double *q, const double *pose, double *cat)
{
    double *c = malloc(sizeof(double) * (size_t)P), *v = malloc(sizeof(double) * (size_t)P);
    traj_cost_impl(pb, OR_QUAD, P, W, q, pose, NULL, NULL, c, v, NULL, NULL, NULL, NULL, cat, NULL);
    free(v);
    free(c);
}

/* The same breakdown per waypoint slot: slot_cat [P][NS][W][8] (the placement entry, a
 * property of the pose variables, is left zero here). */
void or_traj_slot_residuals(const or_problem *pb, int P, int W, const double *q, const double *pose,
                            double *slot_cat)
{
    double *c = malloc(sizeof(double) * (size_t)P), *v = malloc(sizeof(double) * (size_t)P);
    traj_cost_impl(pb, OR_QUAD, P, W, q, pose, NULL, NULL, c, v, NULL, NULL, NULL, NULL, NULL, slot_cat);
    free(v);
    free(c);
}

/* Clearance of a single-particle plan from candidate boxes (test infrastructure for
 * building scenes around a known plan): for each box k of boxes [n][6] (centre, half
 * extents), the smallest sdf_box(c) - r over every robot sphere at every waypoint slot,
 * the held block's spheres at the interior waypoints of each transfer segment, and the
 * block spheres of every block at its initial pose and at its placement pose[b]. */
static double box_dist(const double *p, const double *box)
{
    double g[3];
    return box_sdf_ex(p, box, g, NULL);
}

void or_box_clearance(const or_problem *pb, int W, const double *q, const double *pose, int n,
                      const double *boxes, double *out)
{
    const int B = pb->B, NS = n_seg(pb);
    const double h = pb->h, rb = 0.25 * h - pb->block_margin;
    for (int k = 0; k < n; ++k) out[k] = INFINITY;
    const double *G = pb->grasp;
    frame Gi;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Gi.R[3 * i + j] = G[4 * j + i];
    for (int i = 0; i < 3; ++i) Gi.p[i] = -(Gi.R[3 * i] * G[3] + Gi.R[3 * i + 1] * G[7] + Gi.R[3 * i + 2] * G[11]);
    for (int s = 0; s < NS; ++s)
        for (int w = 0; w < W; ++w) {
            frame F[9], TB;
            fk_frames(pb, q + ((size_t)s * W + w) * NJ, F);
            for (int i = 0; i < pb->S; ++i) {
                double c[3];
                apply(&F[pb->sph_link[i]], pb->sph_c + 3 * i, c);
                for (int k = 0; k < n; ++k) out[k] = dmin(out[k], box_dist(c, boxes + 6 * k) - pb->sph_r[i]);
            }
            if (s % 2 == 1 && w >= 1 && w <= W - 2) {
                compose(&F[8], &Gi, &TB);
                for (int m = 0; m < 8; ++m) {
                    double sb[3], c[3];
                    block_sphere(h, m, sb);
                    apply(&TB, sb, c);
                    for (int k = 0; k < n; ++k) out[k] = dmin(out[k], box_dist(c, boxes + 6 * k) - rb);
                }
            }
        }
    for (int b = 0; b < (pb->mode == 3 ? 0 : B); ++b)
        for (int which = 0; which < 2; ++which) {
            const double *P = which ? pose + 4 * b : pb->block_init + 4 * b;
            const double cy = cos(P[3]), sy = sin(P[3]);
            for (int m = 0; m < 8; ++m) {
                double sb[3], c[3];
                block_sphere(h, m, sb);
                c[0] = P[0] + cy * sb[0] - sy * sb[1];
                c[1] = P[1] + sy * sb[0] + cy * sb[1];
                c[2] = P[2] + sb[2];
                for (int k = 0; k < n; ++k) out[k] = dmin(out[k], box_dist(c, boxes + 6 * k) - rb);
            }
        }
}

static void traj_cost_impl(const or_problem *pb, int phase, int P, int W, const double *q, const double *pose,
                           const double *lam, double *e_out, double *cost, double *viol, double *gq, double *gpose,
                           double *slot_kink, double *pose_kink, double *cat_out, double *slot_cat_out)
{
    const int B = pb->B, NS = n_seg(pb);
    const size_t qstride = (size_t)NS * W * NJ;
    const double w_smooth = pb->w[8];
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < P; ++p) {
        const double *qp = q + p * qstride;
        const double *pp = pose + (size_t)p * B * 4;
        double *gqp = gq ? gq + p * qstride : NULL;
        double gpo[4 * B];
        double scratch[NJ];
        for (int i = 0; i < 4 * B; ++i) gpo[i] = 0.0;
        if (gqp)
            for (size_t i = 0; i < qstride; ++i) gqp[i] = 0.0;
        double c = 0.0, v = 0.0, pk = INFINITY, cat[N_CAT] = {0.0};
        for (int s = 0; s < NS; ++s) {
            for (int w = 0; w < W; ++w) {
                slot_out so = {0.0, 0.0, INFINITY, INFINITY, {0.0}};
                double *g = gqp ? gqp + ((size_t)s * W + w) * NJ : scratch;
                if (!gqp)
                    for (int j = 0; j < NJ; ++j) scratch[j] = 0.0;
                traj_slot(pb, phase, W, s, w, qp + ((size_t)s * W + w) * NJ, pp,
                          lam ? lam + (size_t)p * B * 15 : NULL, e_out ? e_out + (size_t)p * B * 15 : NULL, g,
                          gpo, &so);
                c += so.cost;
                v = dmax(v, so.viol);
                for (int k = 0; k < N_CAT; ++k) cat[k] = dmax(cat[k], so.cat[k]);
                if (slot_cat_out)
                    for (int k = 0; k < N_CAT; ++k)
                        slot_cat_out[(((size_t)p * NS + s) * W + w) * N_CAT + k] = so.cat[k];
                pk = dmin(pk, so.pose_kink);
                if (slot_kink) slot_kink[((size_t)p * NS + s) * W + w] = so.kink;
            }
            for (int w = 0; w + 1 < W; ++w) {
                const double *a = qp + ((size_t)s * W + w) * NJ, *bq = a + NJ;
                for (int j = 0; j < NJ; ++j) {
                    double d = bq[j] - a[j];
                    c += w_smooth * d * d;
                    if (gqp) {
                        gqp[((size_t)s * W + w) * NJ + j] -= 2.0 * w_smooth * d;
                        gqp[((size_t)s * W + w + 1) * NJ + j] += 2.0 * w_smooth * d;
                    }
                }
            }
        }
        double pc = 0.0, pv = 0.0, pkk = INFINITY, gpl[4 * B];
        for (int i = 0; i < 4 * B; ++i) gpl[i] = 0.0;
        if (pb->mode != 3) /* placement variables exist only with blocks to place */
            place_one(pb, 4, phase, pp, &pc, &pv, gpl, &pkk);
        c += pc;
        v = dmax(v, pv);
        cat[CAT_PLACE] = pv;
        if (cat_out)
            for (int k = 0; k < N_CAT; ++k) cat_out[(size_t)p * N_CAT + k] = cat[k];
        pk = dmin(pk, pkk);
        for (int i = 0; i < 4 * B; ++i) gpo[i] += gpl[i];
        cost[p] = c;
        viol[p] = v;
        if (gpose)
            for (int i = 0; i < 4 * B; ++i) gpose[(size_t)p * 4 * B + i] = gpo[i];
        if (pose_kink) pose_kink[p] = pk;
    }
}

/* ------------------------------------------------------------------------------------
 * Updates.  Alg. 1: eta_k = eta_init (1 - k / K_lin) for k = 1..K_lin on the linear
 * cost, then a fixed alpha on the quadratic cost.
 * ------------------------------------------------------------------------------------ */
void or_schedule(int k, int k_lin, double eta, double alpha, int *phase, double *lr)
{
    if (k <= k_lin) {
        *phase = OR_LIN;
        *lr = eta * (1.0 - (double)k / (double)k_lin);
    } else {
        *phase = OR_QUAD;
        *lr = alpha;
    }
}

/* Stage-1 descent step with the block positions clamped into the table (Sec. III-A). */
void or_gd_step(const or_problem *pb, int N, double *x, const double *g, double lr)
{
    const double h = pb->h;
    const double xl = pb->table[0] + 0.5 * h, xh = pb->table[1] - 0.5 * h;
    const double yl = pb->table[2] + 0.5 * h, yh = pb->table[3] - 0.5 * h;
    for (size_t n = 0; n < (size_t)N * pb->B; ++n) {
        double *s = x + 3 * n;
        const double *gs = g + 3 * n;
        s[0] = clampd(s[0] - lr * gs[0], xl, xh);
        s[1] = clampd(s[1] - lr * gs[1], yl, yh);
        s[2] = s[2] - lr * gs[2];
    }
}

static void adam1(double *x, double *m, double *v, double g, double lr, int t, double b1, double b2,
                  double eps)
{
    *m = b1 * *m + (1.0 - b1) * g;
    *v = b2 * *v + (1.0 - b2) * g * g;
    double mh = *m / (1.0 - pow(b1, t)), vh = *v / (1.0 - pow(b2, t));
    *x -= lr * mh / (sqrt(vh) + eps);
}

/* Stage-2 Adam step (Sec. III-B descends the whole trajectory; Adam with the torch
 * defaults).  Consecutive segments share their boundary configuration: the copies
 * q[s][W-1] and q[s+1][0] both receive the sum of their gradients, so with equal
 * moments they stay equal.  The first configuration of the first segment is the robot's
 * start (q_home, as seeded) and is not a variable; a single motion also keeps its goal.
 * Pose variables are only optimised for towers (fixed goals are given). */
void or_traj_adam_step(const or_problem *pb, int P, int W, double *q, double *pose, double *mq,
                       double *vq, double *mp, double *vp, const double *gq, const double *gpose,
                       double lr, int t, double b1, double b2, double eps)
{
    const int B = pb->B, NS = n_seg(pb);
    const size_t qstride = (size_t)NS * W * NJ;
    for (int p = 0; p < P; ++p) {
        for (int s = 0; s < NS; ++s) {
            for (int w = 0; w < W; ++w) {
                if (s == 0 && w == 0) continue;                  /* the start stays at q_home */
                if (pb->mode == 3 && w == W - 1) continue;       /* the goal of a single motion */
                for (int j = 0; j < NJ; ++j) {
                    size_t i = p * qstride + ((size_t)s * W + w) * NJ + j;
                    double g = gq[i];
                    if (w == W - 1 && s + 1 < NS) g = gq[i] + gq[p * qstride + ((size_t)(s + 1) * W) * NJ + j];
                    if (w == 0 && s > 0) g = gq[p * qstride + ((size_t)(s - 1) * W + W - 1) * NJ + j] + gq[i];
                    adam1(q + i, mq + i, vq + i, g, lr, t, b1, b2, eps);
                }
            }
        }
        if (pb->mode == 0)
            for (int i = 0; i < 4 * B; ++i) {
                size_t k = (size_t)p * 4 * B + i;
                adam1(pose + k, mp + k, vp + k, gpose[k], lr, t, b1, b2, eps);
            }
    }
}

/* ------------------------------------------------------------------------------------
 * Sampling (Alg. 1 SampleUniform): x, y uniform over the table shrunk by h/2, yaw
 * uniform in [-pi, pi).  Counter (particle, block, round, stream 1), key (seed, 0).
 * ------------------------------------------------------------------------------------ */
void or_sample(const or_problem *pb, int N, uint64_t seed, int round, double *x)
{
    const double h = pb->h;
    const double xl = pb->table[0] + 0.5 * h, xh = pb->table[1] - 0.5 * h;
    const double yl = pb->table[2] + 0.5 * h, yh = pb->table[3] - 0.5 * h;
    for (int n = 0; n < N; ++n)
        for (int i = 0; i < pb->B; ++i) {
            double u[4];
            uniforms4(seed, (uint64_t)n, (uint64_t)i, (uint64_t)round, STREAM_SAMPLE, u);
            double *s = x + ((size_t)n * pb->B + i) * 3;
            s[0] = xl + (xh - xl) * u[0];
            s[1] = yl + (yh - yl) * u[1];
            s[2] = -OR_PI + 2.0 * OR_PI * u[2];
            if (pb->sample_yaw_steps > 0) {
                /* yaw on n directions: the integer j = floor(n u) from the 24-bit draw */
                const int n_dir = pb->sample_yaw_steps;
                const int64_t k24 = (int64_t)(u[2] * 16777216.0);
                const int64_t j = (n_dir * k24) >> 24;
                s[2] = -OR_PI + 2.0 * OR_PI / n_dir * (double)j;
            }
        }
}

/* Alg. 1 ArgSort: ascending, equal keys in index order. */
static const double *g_sort_key;
static int cmp_idx(const void *a, const void *b)
{
    int i = *(const int32_t *)a, j = *(const int32_t *)b;
    if (g_sort_key[i] < g_sort_key[j]) return -1;
    if (g_sort_key[i] > g_sort_key[j]) return 1;
    return (i > j) - (i < j);
}
void or_argsort(int n, const double *key, int32_t *idx)
{
    for (int i = 0; i < n; ++i) idx[i] = i;
    g_sort_key = key;
    qsort(idx, (size_t)n, sizeof(int32_t), cmp_idx);
}

/* Satisfying particles first (violation below eps), each group by cost then index
 * (Alg. 1 GetSatisfyingParticles, re-evaluated cost, ArgSort). */
static const double *g_ord_cost, *g_ord_viol;
static double g_ord_eps;
static int cmp_ord(const void *a, const void *b)
{
    int i = *(const int32_t *)a, j = *(const int32_t *)b;
    int ui = !(g_ord_viol[i] < g_ord_eps), uj = !(g_ord_viol[j] < g_ord_eps);
    if (ui != uj) return ui - uj;
    if (g_ord_cost[i] < g_ord_cost[j]) return -1;
    if (g_ord_cost[i] > g_ord_cost[j]) return 1;
    return (i > j) - (i < j);
}
void or_order(int n, const double *cost, const double *viol, double eps, int32_t *order, int32_t *n_sat)
{
    int c = 0;
    for (int i = 0; i < n; ++i) {
        order[i] = i;
        c += viol[i] < eps;
    }
    g_ord_cost = cost;
    g_ord_viol = viol;
    g_ord_eps = eps;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_ord);
    *n_sat = c;
}

/* ------------------------------------------------------------------------------------
 * Lift (Sec. III-B): the paper uses analytic Franka IK and allows any parallel IK.  Here:
 * damped least squares, dq = J^T (J J^T + lambda^2 I)^-1 e, clamped to the limits, on the
 * block frame T_E G^-1.  kind 0 (grasp): block origin to the target position and block z
 * axis up (yaw free); kind 1 (place): full pose (x, y, z, yaw).
 * ------------------------------------------------------------------------------------ */
static void solve6(double A[6][6], double *b)
{
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        for (int r = c + 1; r < 6; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < 6; ++k) {
                double t = A[c][k];
                A[c][k] = A[piv][k];
                A[piv][k] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < 6; ++r) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < 6; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int c = 5; c >= 0; --c) {
        double s = b[c];
        for (int k = c + 1; k < 6; ++k) s -= A[c][k] * b[k];
        b[c] = s / A[c][c];
    }
}

/* IK error of the block frame T_B = T_E G^-1 at q: position error, then the
 * orientation error (kind 0: z axis against e_z; kind 1: half the sum of the axis cross
 * products against Rz(yaw)).  J (optional) receives the 6x7 geometric Jacobian of T_B. */
static void ik_error(const or_problem *pb, int kind, const double *target, const double *q, double e[6],
                     double J[6][NJ])
{
    const double *G = pb->grasp;
    frame Gi, F[9], TB;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Gi.R[3 * i + j] = G[4 * j + i];
    for (int i = 0; i < 3; ++i) Gi.p[i] = -(Gi.R[3 * i] * G[3] + Gi.R[3 * i + 1] * G[7] + Gi.R[3 * i + 2] * G[11]);
    fk_frames(pb, q, F);
    compose(&F[8], &Gi, &TB);
    for (int i = 0; i < 3; ++i) e[i] = target[i] - TB.p[i];
    double ew[3] = {0, 0, 0};
    if (kind == 0) {
        double u[3], ez[3] = {0, 0, 1};
        col(&TB, 2, u);
        cross3(u, ez, ew);
    } else {
        double c = cos(target[3]), s = sin(target[3]);
        double Rt[3][3] = {{c, -s, 0}, {s, c, 0}, {0, 0, 1}};
        for (int a = 0; a < 3; ++a) {
            double u[3], v[3] = {Rt[0][a], Rt[1][a], Rt[2][a]}, t[3];
            col(&TB, a, u);
            cross3(u, v, t);
            for (int i = 0; i < 3; ++i) ew[i] += 0.5 * t[i];
        }
    }
    e[3] = ew[0];
    e[4] = ew[1];
    e[5] = ew[2];
    if (!J) return;
    for (int j = 1; j <= NJ; ++j) {
        double z[3], r[3], t[3];
        col(&F[j - 1], 2, z);
        for (int i = 0; i < 3; ++i) r[i] = TB.p[i] - F[j - 1].p[i];
        cross3(z, r, t);
        for (int i = 0; i < 3; ++i) {
            J[i][j - 1] = t[i];
            J[3 + i][j - 1] = z[i];
        }
    }
}

double or_ik_error(const or_problem *pb, int kind, const double *target, const double *q)
{
    double e[6];
    ik_error(pb, kind, target, q, e, NULL);
    double s = 0.0;
    for (int i = 0; i < 6; ++i) s += e[i] * e[i];
    return sqrt(s);
}

void or_ik_iterate(const or_problem *pb, int kind, const double *target, double *q, int iters, double lambda)
{
    for (int it = 0; it < iters; ++it) {
        double e[6], J[6][NJ], A[6][6];
        ik_error(pb, kind, target, q, e, J);
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) {
                double s = 0.0;
                for (int k = 0; k < NJ; ++k) s += J[r][k] * J[c][k];
                A[r][c] = s + (r == c ? lambda * lambda : 0.0);
            }
        solve6(A, e);
        for (int k = 0; k < NJ; ++k) {
            double d = 0.0;
            for (int r = 0; r < 6; ++r) d += J[r][k] * e[r];
            q[k] = clampd(q[k] + d, pb->lo[k], pb->hi[k]);
        }
    }
}

/* How deep the arm stands in the clutter at q, for block b in situation `kind`: the sum
 * over robot spheres of max(0, r - sdf) against every box and every block visible there
 * (as in the stage-2 cost): blocks below b at their placements pose[bb], blocks above b at
 * their initial poses, and block b itself at its placement after the place (kind 1), at
 * its initial pose inside its transit (kind 2), not at the grasp (kind 0) nor while held
 * (kind 3). */
double or_arm_clutter(const or_problem *pb, const double *q, const double *pose, int b, int kind)
{
    frame F[9];
    fk_frames(pb, q, F);
    const double half = 0.5 * pb->h;
    double pen = 0.0;
    for (int i = 0; i < pb->S; ++i) {
        double c[3], g[3], gpo[4];
        apply(&F[pb->sph_link[i]], pb->sph_c + 3 * i, c);
        const double r = pb->sph_r[i];
        for (int o = 0; o < pb->O; ++o) {
            const double d = r - box_sdf_ex(c, pb->boxes + 6 * o, g, NULL);
            if (d > 0.0) pen += d;
        }
        for (int bb = 0; bb < (pb->mode == 3 ? 0 : pb->B); ++bb) { /* no blocks in mode 3 */
            const double *bp;
            if (bb < b || (bb == b && kind == 1))
                bp = pose + 4 * bb;
            else if (bb > b || (bb == b && kind == 2))
                bp = pb->block_init + 4 * bb;
            else
                continue;
            const double d = r - obb_sdf_ex(c, bp, half, g, gpo, NULL);
            if (d > 0.0) pen += d;
        }
    }
    return pen;
}

/* One multi-start solve: start 0 is q0, start r >= 1 is uniform over the joint limits
 * (counter (particle, sub, r, stream 2) and (particle, sub + 1, r, stream 2)).  Among
 * the starts whose final error is below OR_IK_ACCEPT the result is the one standing
 * least deep in the obstacles (the first on ties); when no start converges, the one with
 * the smallest error (the first on ties). */
#define OR_IK_ACCEPT 1e-4
static void ik_multistart(const or_problem *pb, int kind, const double *target, const double *q0, uint64_t seed,
                          int p, int sub, int restarts, int iters, double lambda, const double *pose, int b,
                          double *q_out)
{
    double best_err = INFINITY, best_pen = INFINITY;
    int have_acc = 0;
    for (int r = 0; r < restarts; ++r) {
        double q[NJ];
        if (r == 0) {
            for (int j = 0; j < NJ; ++j) q[j] = q0[j];
        } else {
            double u[8];
            uniforms4(seed, (uint64_t)p, (uint64_t)sub, (uint64_t)r, STREAM_IK, u);
            uniforms4(seed, (uint64_t)p, (uint64_t)(sub + 1), (uint64_t)r, STREAM_IK, u + 4);
            for (int j = 0; j < NJ; ++j) q[j] = pb->lo[j] + (pb->hi[j] - pb->lo[j]) * u[j];
        }
        or_ik_iterate(pb, kind, target, q, iters, lambda);
        const double err = or_ik_error(pb, kind, target, q);
        if (err < OR_IK_ACCEPT) {
            const double pen = or_arm_clutter(pb, q, pose, b, kind);
            if (!have_acc || pen < best_pen) {
                have_acc = 1;
                best_pen = pen;
                for (int j = 0; j < NJ; ++j) q_out[j] = q[j];
            }
        } else if (!have_acc && err < best_err) {
            best_err = err;
            for (int j = 0; j < NJ; ++j) q_out[j] = q[j];
        }
    }
}

/* Per particle and block (Sec. III-B lift): the grasp at block_init[b] from q_home +
 * noise U[-1,1]^7 (counter (particle, 2b + chunk, 0, stream 2)) and restarts drawn at
 * sub-index 2b; then the placement at pose[p][b] from the grasp solution, restarts at
 * sub-index 2B + 2b. */
void or_ik_lift(const or_problem *pb, int P, const double *pose, uint64_t seed, int iters, double lambda,
                double noise, int restarts, double *q_grasp, double *q_place)
{
    const int B = pb->B;
#pragma omp parallel for schedule(dynamic, 4)
    for (int p = 0; p < P; ++p)
        for (int b = 0; b < B; ++b) {
            double u[8], q0[NJ];
            uniforms4(seed, (uint64_t)p, (uint64_t)(2 * b), 0, STREAM_IK, u);
            uniforms4(seed, (uint64_t)p, (uint64_t)(2 * b + 1), 0, STREAM_IK, u + 4);
            for (int j = 0; j < NJ; ++j)
                q0[j] = clampd(pb->q_home[j] + noise * (2.0 * u[j] - 1.0), pb->lo[j], pb->hi[j]);
            double *g = q_grasp + ((size_t)p * B + b) * NJ;
            const double *pp = pose + (size_t)p * B * 4;
            ik_multistart(pb, 0, pb->block_init + 4 * b, q0, seed, p, 2 * b, restarts, iters, lambda, pp, b, g);
            double *pl = q_place + ((size_t)p * B + b) * NJ;
            ik_multistart(pb, 1, pp + 4 * b, g, seed, p, 2 * B + 2 * b, restarts, iters, lambda, pp, b, pl);
        }
}

/* Trajectory seeds (Sec. III-B): one intermediate waypoint between each segment's start
 * and goal, at index m = (W-1)/2, and straight lines start -> intermediate -> goal.  The
 * intermediate waypoint is the best of `candidates` draws of the endpoints' midpoint plus
 * uniform noise (see below).  The first segment starts at q_home.  Segment ends are
 * copied exactly so that the shared boundary configurations are equal. */
void or_traj_init(const or_problem *pb, int P, int W, const double *q_grasp, const double *q_place,
                  const double *pose, uint64_t seed, double noise, int candidates, double *q)
{
    const int B = pb->B, NS = n_seg(pb), m = (W - 1) / 2;
    double qh[NJ], qgoal[NJ];
    for (int j = 0; j < NJ; ++j) qh[j] = clampd(pb->q_home[j], pb->lo[j], pb->hi[j]);
    if (pb->mode == 3)
        for (int j = 0; j < NJ; ++j) qgoal[j] = clampd(pb->p2p_goal[j], pb->lo[j], pb->hi[j]);
    for (int p = 0; p < P; ++p)
        for (int s = 0; s < NS; ++s) {
            int b = s / 2;
            const double *qa, *qb;
            if (pb->mode == 3) { /* the one motion: start to goal */
                qa = qh;
                qb = qgoal;
            } else if (s % 2 == 0) {
                qa = b == 0 ? qh : q_place + ((size_t)p * B + b - 1) * NJ;
                qb = q_grasp + ((size_t)p * B + b) * NJ;
            } else {
                qa = q_grasp + ((size_t)p * B + b) * NJ;
                qb = q_place + ((size_t)p * B + b) * NJ;
            }
            /* candidate c: midpoint + noise from counter (particle, 2s + chunk, c, stream 3);
             * keep the one whose seed path stands least deep in the obstacles at the
             * intermediate waypoint and the two quarter points (first on ties) */
            double qm[NJ], best = INFINITY;
            for (int c = 0; c < candidates; ++c) {
                double u[8], qc[NJ], h1[NJ], h2[NJ];
                uniforms4(seed, (uint64_t)p, (uint64_t)(2 * s), (uint64_t)c, STREAM_MID, u);
                uniforms4(seed, (uint64_t)p, (uint64_t)(2 * s + 1), (uint64_t)c, STREAM_MID, u + 4);
                for (int j = 0; j < NJ; ++j) {
                    qc[j] = clampd(0.5 * (qa[j] + qb[j]) + noise * (2.0 * u[j] - 1.0), pb->lo[j], pb->hi[j]);
                    h1[j] = 0.5 * (qa[j] + qc[j]);
                    h2[j] = 0.5 * (qc[j] + qb[j]);
                }
                const double *pp = pose ? pose + (size_t)p * B * 4 : NULL;
                const int kind = 2 + s % 2;  /* transit or transfer interior */
                const double sc = candidates > 1 ? or_arm_clutter(pb, qc, pp, b, kind) +
                                                       or_arm_clutter(pb, h1, pp, b, kind) +
                                                       or_arm_clutter(pb, h2, pp, b, kind)
                                                 : 0.0;
                if (c == 0 || sc < best) {
                    best = sc;
                    for (int j = 0; j < NJ; ++j) qm[j] = qc[j];
                }
            }
            for (int w = 0; w < W; ++w) {
                double *d = q + (((size_t)p * NS + s) * W + w) * NJ;
                for (int j = 0; j < NJ; ++j) {
                    if (w == 0)
                        d[j] = qa[j];
                    else if (w == W - 1)
                        d[j] = qb[j];
                    else if (w == m)
                        d[j] = qm[j];
                    else if (w < m)
                        d[j] = qa[j] + ((double)w / m) * (qm[j] - qa[j]);
                    else
                        d[j] = qm[j] + ((double)(w - m) / (W - 1 - m)) * (qb[j] - qm[j]);
                }
            }
        }
}

/* ------------------------------------------------------------------------------------
 * Stage 1 (Alg. 1 lines 1-14) and stage 2 (Sec. III-B) drivers.
 * ------------------------------------------------------------------------------------ */
void or_stage1(const or_problem *pb, int N, int M, uint64_t seed, int round, int k_lin, int k_quad,
               double eta, double alpha, double *x_out, double *cost_out, double *viol_out)
{
    const int B = pb->B;
    double *x = malloc(sizeof(double) * (size_t)N * B * 3);
    double *c = malloc(sizeof(double) * (size_t)N), *v = malloc(sizeof(double) * (size_t)N);
    int32_t *idx = malloc(sizeof(int32_t) * (size_t)N);
    or_sample(pb, N, seed, round, x);
    or_place_cost(pb, 3, OR_LIN, N, x, c, v, NULL, NULL);
    or_argsort(N, c, idx);
    for (int i = 0; i < M; ++i) memcpy(x_out + (size_t)i * B * 3, x + (size_t)idx[i] * B * 3, sizeof(double) * B * 3);
    double *g = malloc(sizeof(double) * (size_t)M * B * 3);
    for (int k = 1; k <= k_lin + k_quad; ++k) {
        int phase;
        double lr;
        or_schedule(k, k_lin, eta, alpha, &phase, &lr);
        or_place_cost(pb, 3, phase, M, x_out, cost_out, viol_out, g, NULL);
        or_gd_step(pb, M, x_out, g, lr);
    }
    or_place_cost(pb, 3, OR_QUAD, M, x_out, cost_out, viol_out, NULL, NULL);
    free(g);
    free(idx);
    free(v);
    free(c);
    free(x);
}

/* Augmented-Lagrangian multiplier step: lambda <- lambda + rho * 2 w * e for the grasp
 * (w_start, components 0..5) and tie (w_tie, 6..14) residuals of every block; the penalty
 * w |e|^2 is the (mu / 2) |e|^2 of the method of multipliers with mu = 2 w. */
void or_al_update(const or_problem *pb, int P, const double *e, double rho, double *lam)
{
    const double w_start = pb->w[3], w_tie = pb->w[4];
    for (size_t i = 0; i < (size_t)P * pb->B * 15; ++i)
        lam[i] += rho * 2.0 * ((i % 15) < 6 ? w_start : w_tie) * e[i];
}

void or_stage2(const or_problem *pb, int P, int W, int K, int k_lin, double eta, double alpha, double b1,
               double b2, double eps, double *q, double *pose)
{
    or_stage2_al(pb, P, W, K, k_lin, eta, alpha, b1, b2, eps, 0, 0.0, q, pose, NULL);
}

/* Stage 2 with the augmented-Lagrangian outer loop (Sec. III-B): after the evaluation of
 * every al_every-th iteration the multipliers take the step above with that evaluation's
 * residuals (al_every = 0: the plain penalty method; lam may be NULL then). */
void or_stage2_al(const or_problem *pb, int P, int W, int K, int k_lin, double eta, double alpha, double b1,
                  double b2, double eps, int al_every, double al_rho, double *q, double *pose, double *lam)
{
    const int B = pb->B;
    const size_t nq = (size_t)P * n_seg(pb) * W * NJ, np = (size_t)P * B * 4;
    double *mq = calloc(nq, sizeof(double)), *vq = calloc(nq, sizeof(double));
    double *mp = calloc(np, sizeof(double)), *vp = calloc(np, sizeof(double));
    double *gq = malloc(nq * sizeof(double)), *gp = malloc(np * sizeof(double));
    double *c = malloc((size_t)P * sizeof(double)), *v = malloc((size_t)P * sizeof(double));
    double *e = calloc((size_t)P * B * 15, sizeof(double));
    for (int k = 1; k <= K; ++k) {
        int phase;
        double lr;
        or_schedule(k, k_lin, eta, alpha, &phase, &lr);
        or_traj_cost_al(pb, phase, P, W, q, pose, al_every > 0 ? lam : NULL, al_every > 0 ? e : NULL, c, v, gq,
                        gp, NULL, NULL);
        or_traj_adam_step(pb, P, W, q, pose, mq, vq, mp, vp, gq, gp, lr, k, b1, b2, eps);
        if (al_every > 0 && k % al_every == 0) or_al_update(pb, P, e, al_rho, lam);
    }
    free(e);
    free(v);
    free(c);
    free(gp);
    free(gq);
    free(vp);
    free(mp);
    free(vq);
    free(mq);
}
