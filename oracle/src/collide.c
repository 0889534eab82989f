/*
 * Oracle collision geometry, candidate pairs and narrowphase (FP64).
 *
 * The paper's collision cost (Eq. collision_cost) needs the signed
 * distances d_k between the manipulators and the environment (and between
 * the two manipulators); its world model (MuJoCo) also produces contacts.
 * Geometry readings: arm links 1..6 are capsules (segment from joint i to
 * joint i+1), link 7 carries a spherical pad at its tip, the free object is
 * a sphere (the ball) or a box (the tray, the cube; object.c), obstacles are
 * static axis-aligned boxes, the table is the plane z = 0.  Every pair
 * yields at most one contact (a box object on the table up to four):
 * signed distance phi, unit normal n pointing from geom B to geom A, and
 * point p midway between the two closest surface points.
 *
 * Canonical pair order (also the contact order and the order in which the
 * contact cap truncates):
 *   1 ball-table; 2 ball-pads; 3 ball-arm links 1..6; 4 ball-boxes;
 *   5 arm geoms 2..7 - table; 6 arm geoms - boxes; 7 arm1 geoms - arm2 geoms.
 * Same-arm pairs, base link - table and static-static pairs are excluded.
 * The collision-cost pairs are groups 6 and 7 (arm-ball and table pairs are
 * excluded from the cost because the grasp needs contact).
 * TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

enum { SH_SPHERE = 0, SH_CAPSULE = 1, SH_PLANE = 2, SH_BOX = 3, SH_OBOX = 4 };

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double clamp01(double t) { return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t); }

int or_num_pairs(const OScene *s) { return 1 + 2 + 12 + s->n_box + 12 + 14 * s->n_box + 49; }
int or_num_cost_pairs(const OScene *s) { return 14 * s->n_box + 49; }
int or_cost_pair_index(const OScene *s, int i) { return 27 + s->n_box + i; }

void or_pair(const OScene *s, int idx, int *ga, int *gb)
{
    int nb = s->n_box;
    if (idx == 0) { *ga = OG_BALL; *gb = OG_TABLE; return; }
    idx -= 1;
    if (idx < 2) { *ga = OG_BALL; *gb = OG_ARM + 7 * idx + 6; return; }
    idx -= 2;
    if (idx < 12) { *ga = OG_BALL; *gb = OG_ARM + 7 * (idx / 6) + (idx % 6); return; }
    idx -= 12;
    if (idx < nb) { *ga = OG_BALL; *gb = OG_BOX + idx; return; }
    idx -= nb;
    if (idx < 12) { *ga = OG_ARM + 7 * (idx / 6) + 1 + (idx % 6); *gb = OG_TABLE; return; }
    idx -= 12;
    if (idx < 14 * nb) { *ga = OG_ARM + idx / nb; *gb = OG_BOX + idx % nb; return; }
    idx -= 14 * nb;
    *ga = OG_ARM + idx / 7;
    *gb = OG_ARM + 7 + idx % 7;
}

/* pball points at the object's state: centre, then quaternion */
void or_geom_shape(const OScene *s, const OArmKin kin[2], const double *pball, int gid, int *type, double P0[3],
                   double P1[3], double *r)
{
    if (gid == OG_BALL && s->obj_box) {
        *type = SH_OBOX;
        memcpy(P0, pball, 3 * sizeof(double));
        memcpy(P1, s->obj_h, 3 * sizeof(double));
        *r = 0.0;
    } else if (gid == OG_BALL) {
        *type = SH_SPHERE;
        memcpy(P0, pball, 3 * sizeof(double));
        memcpy(P1, pball, 3 * sizeof(double));
        *r = s->ball_r;
    } else if (gid == OG_TABLE) {
        *type = SH_PLANE;
        P0[0] = P0[1] = P0[2] = 0.0;
        P1[0] = P1[1] = P1[2] = 0.0;
        *r = 0.0;
    } else if (gid >= OG_BOX) {
        int b = gid - OG_BOX;
        *type = SH_BOX;
        memcpy(P0, s->box_c[b], 3 * sizeof(double));
        memcpy(P1, s->box_h[b], 3 * sizeof(double));
        *r = 0.0;
    } else {
        int arm = (gid - OG_ARM) / 7, g = (gid - OG_ARM) % 7;
        if (g < 6) {
            *type = SH_CAPSULE;
            memcpy(P0, kin[arm].o[g], 3 * sizeof(double));
            memcpy(P1, kin[arm].o[g + 1], 3 * sizeof(double));
            *r = s->link_rad[g];
        } else {
            *type = SH_SPHERE;
            memcpy(P0, kin[arm].o[7], 3 * sizeof(double));
            memcpy(P1, kin[arm].o[7], 3 * sizeof(double));
            *r = s->pad_rad;
        }
    }
}

void or_aabb(const OScene *s, const OArmKin kin[2], const double *pball, int gid, double lo[3], double hi[3])
{
    int type;
    double P0[3], P1[3], r;
    or_geom_shape(s, kin, pball, gid, &type, P0, P1, &r);
    double R[3][3];
    if (type == SH_OBOX) or_quat_to_R(pball + 3, R);
    for (int i = 0; i < 3; ++i) {
        if (type == SH_PLANE) {
            lo[i] = -INFINITY;
            hi[i] = (i == 2) ? 0.0 : INFINITY;
        } else if (type == SH_OBOX) {
            double e = fabs(R[i][0]) * P1[0] + fabs(R[i][1]) * P1[1] + fabs(R[i][2]) * P1[2];
            lo[i] = P0[i] - e;
            hi[i] = P0[i] + e;
        } else if (type == SH_BOX) {
            lo[i] = P0[i] - P1[i];
            hi[i] = P0[i] + P1[i];
        } else {
            lo[i] = fmin(P0[i], P1[i]) - r;
            hi[i] = fmax(P0[i], P1[i]) + r;
        }
    }
}

/* contact between two spheres with centres xa, xb */
static void sphere_sphere(const double xa[3], double ra, const double xb[3], double rb, double *phi, double n[3],
                          double p[3])
{
    double d[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
    double dist = sqrt(dot3(d, d));
    if (dist > 1e-9) {
        for (int i = 0; i < 3; ++i) n[i] = d[i] / dist;
    } else {
        n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
    }
    *phi = dist - ra - rb;
    for (int i = 0; i < 3; ++i) p[i] = 0.5 * ((xa[i] - ra * n[i]) + (xb[i] + rb * n[i]));
}

/* sphere (centre x, radius r) against the plane z = 0 */
static void sphere_plane(const double x[3], double r, double *phi, double n[3], double p[3])
{
    n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
    *phi = x[2] - r;
    p[0] = x[0]; p[1] = x[1]; p[2] = 0.5 * (x[2] - r);
}

/* sphere against an axis-aligned box (centre c, half extents hh) */
static void sphere_box(const double x[3], double r, const double c[3], const double hh[3], double *phi, double n[3],
                       double p[3])
{
    double l[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    int outside = 0;
    for (int i = 0; i < 3; ++i)
        if (fabs(l[i]) > hh[i]) outside = 1;
    double q[3];
    if (outside) {
        for (int i = 0; i < 3; ++i) q[i] = l[i] < -hh[i] ? -hh[i] : (l[i] > hh[i] ? hh[i] : l[i]);
        double d[3] = {l[0] - q[0], l[1] - q[1], l[2] - q[2]};
        double dist = sqrt(dot3(d, d));
        for (int i = 0; i < 3; ++i) n[i] = d[i] / dist;
        *phi = dist - r;
    } else {
        /* inside: leave through the face of least penetration (lowest axis on ties) */
        int best = 0;
        double be = fabs(l[0]) - hh[0];
        for (int i = 1; i < 3; ++i) {
            double e = fabs(l[i]) - hh[i];
            if (e > be) { be = e; best = i; }
        }
        double sg = l[best] >= 0.0 ? 1.0 : -1.0;
        n[0] = n[1] = n[2] = 0.0;
        n[best] = sg;
        memcpy(q, l, sizeof(q));
        q[best] = sg * hh[best];
        *phi = be - r;
    }
    for (int i = 0; i < 3; ++i) p[i] = 0.5 * ((x[i] - r * n[i]) + (c[i] + q[i]));
}

/* closest point parameter on segment P0 + t (P1 - P0) to point x */
static double seg_point_t(const double P0[3], const double P1[3], const double x[3])
{
    double D[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
    double w[3] = {x[0] - P0[0], x[1] - P0[1], x[2] - P0[2]};
    double dd = dot3(D, D);
    if (dd <= 0.0) return 0.0;
    return clamp01(dot3(w, D) / dd);
}

/* closest points between two segments, by enumerating the interior
 * stationary point and the four edges of the parameter square */
static void seg_seg(const double P0[3], const double P1[3], const double Q0[3], const double Q1[3], double *so,
                    double *to)
{
    double D1[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
    double D2[3] = {Q1[0] - Q0[0], Q1[1] - Q0[1], Q1[2] - Q0[2]};
    double r[3] = {P0[0] - Q0[0], P0[1] - Q0[1], P0[2] - Q0[2]};
    double a = dot3(D1, D1), b = dot3(D1, D2), e = dot3(D2, D2), c = dot3(D1, r), f = dot3(D2, r);
    double cs[5], ct[5];
    int nc = 0;
    double den = a * e - b * b;
    if (den > 0.0) {
        double s = (b * f - c * e) / den, t = (a * f - b * c) / den;
        if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) { cs[nc] = s; ct[nc] = t; ++nc; }
    }
    cs[nc] = 0.0; ct[nc] = clamp01(f / e); ++nc;
    cs[nc] = 1.0; ct[nc] = clamp01((f + b) / e); ++nc;
    ct[nc] = 0.0; cs[nc] = clamp01(-c / a); ++nc;
    ct[nc] = 1.0; cs[nc] = clamp01((b - c) / a); ++nc;
    double best = INFINITY;
    for (int i = 0; i < nc; ++i) {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = r[k] + cs[i] * D1[k] - ct[i] * D2[k];
        double v = dot3(d, d);
        if (v < best) { best = v; *so = cs[i]; *to = ct[i]; }
    }
}

/* signed distance from point l (box frame) to the box with half extents hh */
static double box_sd(const double l[3], const double hh[3])
{
    double out2 = 0.0, mx = -INFINITY;
    for (int i = 0; i < 3; ++i) {
        double e = fabs(l[i]) - hh[i];
        if (e > 0.0) out2 += e * e;
        if (e > mx) mx = e;
    }
    return out2 > 0.0 ? sqrt(out2) : mx;
}

/* t* = minimiser over [0,1] of the (convex) signed distance from the
 * segment A + t (B - A) to the box; the midpoint of the minimising interval
 * when it is not a single point.  Exact: the minimiser of a convex
 * piecewise function lies at an end, a breakpoint or a stationary point of
 * a smooth piece, so every such candidate is evaluated. */
double or_seg_box_tstar(const double A[3], const double B[3], const double c[3], const double hh[3])
{
    double a[3] = {A[0] - c[0], A[1] - c[1], A[2] - c[2]};
    double D[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double cand[64];
    int nc = 0;
    cand[nc++] = 0.0;
    cand[nc++] = 1.0;
    for (int i = 0; i < 3; ++i) {
        if (D[i] != 0.0) {
            cand[nc++] = (hh[i] - a[i]) / D[i];
            cand[nc++] = (-hh[i] - a[i]) / D[i];
            cand[nc++] = -a[i] / D[i];
        }
    }
    /* stationary points of the outside squared distance, every active set
     * and sign pattern: state 0 = axis inside its slab, 1 = above, 2 = below */
    for (int pat = 0; pat < 27; ++pat) {
        int st[3] = {pat % 3, (pat / 3) % 3, pat / 9};
        double num = 0.0, dd = 0.0;
        for (int i = 0; i < 3; ++i) {
            if (st[i] == 0) continue;
            double sg = st[i] == 1 ? 1.0 : -1.0;
            num += sg * D[i] * hh[i] - D[i] * a[i];
            dd += D[i] * D[i];
        }
        if (dd > 0.0) cand[nc++] = num / dd;
    }
    /* crossings of the six linear pieces s (a_i + t D_i) - h_i (inside) */
    for (int p = 0; p < 6; ++p)
        for (int q = p + 1; q < 6; ++q) {
            int i = p / 2, j = q / 2;
            double si = (p % 2) ? -1.0 : 1.0, sj = (q % 2) ? -1.0 : 1.0;
            double den = si * D[i] - sj * D[j];
            if (den != 0.0) cand[nc++] = (hh[i] - hh[j] - si * a[i] + sj * a[j]) / den;
        }
    double gmin = INFINITY;
    double val[64];
    for (int i = 0; i < nc; ++i) {
        if (!(cand[i] >= 0.0 && cand[i] <= 1.0)) { val[i] = INFINITY; continue; }
        double l[3] = {a[0] + cand[i] * D[0], a[1] + cand[i] * D[1], a[2] + cand[i] * D[2]};
        val[i] = box_sd(l, hh);
        if (val[i] < gmin) gmin = val[i];
    }
    double tlo = INFINITY, thi = -INFINITY;
    for (int i = 0; i < nc; ++i)
        if (val[i] <= gmin) {
            if (cand[i] < tlo) tlo = cand[i];
            if (cand[i] > thi) thi = cand[i];
        }
    return 0.5 * (tlo + thi);
}

/* narrowphase between two shapes; A is a sphere or capsule */
static void narrow_shapes(int ta, const double A0[3], const double A1[3], double ra, int tb, const double B0[3],
                          const double B1[3], double rb, double *phi, double n[3], double p[3])
{
    if (tb == SH_PLANE) {
        const double *x = A0;
        if (ta == SH_CAPSULE && A1[2] < A0[2]) x = A1; /* deepest end (A0 on ties) */
        sphere_plane(x, ra, phi, n, p);
        return;
    }
    if (tb == SH_BOX) {
        double x[3];
        if (ta == SH_CAPSULE) {
            double t = or_seg_box_tstar(A0, A1, B0, B1);
            for (int i = 0; i < 3; ++i) x[i] = A0[i] + t * (A1[i] - A0[i]);
        } else {
            memcpy(x, A0, sizeof(x));
        }
        sphere_box(x, ra, B0, B1, phi, n, p);
        return;
    }
    /* sphere/capsule against sphere/capsule: closest core points */
    double xa[3], xb[3];
    if (ta == SH_CAPSULE && tb == SH_CAPSULE) {
        double sp, tq;
        seg_seg(A0, A1, B0, B1, &sp, &tq);
        for (int i = 0; i < 3; ++i) {
            xa[i] = A0[i] + sp * (A1[i] - A0[i]);
            xb[i] = B0[i] + tq * (B1[i] - B0[i]);
        }
    } else if (ta == SH_CAPSULE) {
        double t = seg_point_t(A0, A1, B0);
        for (int i = 0; i < 3; ++i) { xa[i] = A0[i] + t * (A1[i] - A0[i]); xb[i] = B0[i]; }
    } else if (tb == SH_CAPSULE) {
        double t = seg_point_t(B0, B1, A0);
        for (int i = 0; i < 3; ++i) { xb[i] = B0[i] + t * (B1[i] - B0[i]); xa[i] = A0[i]; }
    } else {
        memcpy(xa, A0, sizeof(xa));
        memcpy(xb, B0, sizeof(xb));
    }
    sphere_sphere(xa, ra, xb, rb, phi, n, p);
}

void or_narrow_prim(int ta, const double A0[3], const double A1[3], double ra, int tb, const double B0[3],
                    const double B1[3], double rb, double *phi, double n[3], double p[3])
{
    narrow_shapes(ta, A0, A1, ra, tb, B0, B1, rb, phi, n, p);
}

/* narrowphase for pair (ga, gb); returns 1 and fills (phi, n, p) (a box
 * object on the table: its deepest vertex) */
int or_narrow(const OScene *s, const OArmKin kin[2], const double *pball, int ga, int gb, double *phi, double n[3],
              double p[3])
{
    int ta, tb;
    double A0[3], A1[3], B0[3], B1[3], ra, rb;
    or_geom_shape(s, kin, pball, ga, &ta, A0, A1, &ra);
    or_geom_shape(s, kin, pball, gb, &tb, B0, B1, &rb);
    if (ta == SH_OBOX)
        or_obj_narrow(s, pball, tb, B0, B1, rb, phi, n, p);
    else
        narrow_shapes(ta, A0, A1, ra, tb, B0, B1, rb, phi, n, p);
    return 1;
}

/* primitive-level narrowphase for tests: types 0 sphere, 1 capsule,
 * 2 plane z = 0, 3 box (B0 = centre, B1 = half extents) */
void oracle_prim(int ta, const double *A0, const double *A1, double ra, int tb, const double *B0, const double *B1,
                 double rb, double *out /* phi, n[3], p[3] */)
{
    narrow_shapes(ta, A0, A1, ra, tb, B0, B1, rb, &out[0], out + 1, out + 4);
}

/* every pair in canonical order, keep the first `cap` with phi < 0 */
int or_contacts(const OScene *s, const OArmKin kin[2], const double *pball, OContact *out, int cap)
{
    int np = or_num_pairs(s), nc = 0;
    for (int i = 0; i < np && nc < cap; ++i) {
        int ga, gb;
        double phi, n[3], p[3];
        or_pair(s, i, &ga, &gb);
        if (ga == OG_BALL && gb == OG_TABLE && s->obj_box) {
            /* a box object on the table: every vertex below it, in vertex order, four at most */
            double ph[8], nn[8][3], pp[8][3];
            or_obj_table(s, pball, ph, nn, pp);
            int taken = 0;
            for (int k = 0; k < 8 && nc < cap && taken < 4; ++k)
                if (ph[k] < 0.0) {
                    out[nc].pair = i;
                    out[nc].ga = ga;
                    out[nc].gb = gb;
                    out[nc].phi = ph[k];
                    memcpy(out[nc].n, nn[k], sizeof(nn[k]));
                    memcpy(out[nc].p, pp[k], sizeof(pp[k]));
                    ++nc;
                    ++taken;
                }
            continue;
        }
        or_narrow(s, kin, pball, ga, gb, &phi, n, p);
        if (phi < 0.0) {
            out[nc].pair = i;
            out[nc].ga = ga;
            out[nc].gb = gb;
            out[nc].phi = phi;
            memcpy(out[nc].n, n, sizeof(n));
            memcpy(out[nc].p, p, sizeof(p));
            ++nc;
        }
    }
    return nc;
}

/* ---- exported for tests ---- */
int oracle_num_pairs(const OScene *s) { return or_num_pairs(s); }

void oracle_pairs(const OScene *s, int *ga, int *gb)
{
    int np = or_num_pairs(s);
    for (int i = 0; i < np; ++i) or_pair(s, i, &ga[i], &gb[i]);
}

/* narrowphase of every pair at state x: phi[np], n[np*3], p[np*3] */
void oracle_narrow_all(const OScene *s, const double *x, double *phi, double *n, double *p)
{
    OArmKin kin[2];
    or_fk(s, 0, x, &kin[0]);
    or_fk(s, 1, x + 7, &kin[1]);
    int np = or_num_pairs(s);
    for (int i = 0; i < np; ++i) {
        int ga, gb;
        or_pair(s, i, &ga, &gb);
        or_narrow(s, kin, x + 42, ga, gb, &phi[i], n + 3 * i, p + 3 * i);
    }
}

/* AABBs of every geom at state x: lo/hi [ngeom*3], geoms 0..(16+n_box-1) */
void oracle_aabbs(const OScene *s, const double *x, double *lo, double *hi)
{
    OArmKin kin[2];
    or_fk(s, 0, x, &kin[0]);
    or_fk(s, 1, x + 7, &kin[1]);
    int ng = OG_BOX + s->n_box;
    for (int g = 0; g < ng; ++g) or_aabb(s, kin, x + 42, g, lo + 3 * g, hi + 3 * g);
}

/* brute-force broadphase: for every candidate pair, do the closed AABBs
 * of its two geoms overlap (after inflating geom A's box by `margin`)? */
void oracle_broadphase(const OScene *s, const float *lo, const float *hi, float margin, int *flags)
{
    int np = or_num_pairs(s);
    for (int i = 0; i < np; ++i) {
        int ga, gb;
        or_pair(s, i, &ga, &gb);
        int ok = 1;
        for (int k = 0; k < 3; ++k) {
            double la = (double)lo[3 * ga + k] - (double)margin, ha = (double)hi[3 * ga + k] + (double)margin;
            double lb = lo[3 * gb + k], hb = hi[3 * gb + k];
            if (!(la <= hb && lb <= ha)) ok = 0;
        }
        flags[i] = ok;
    }
}

double oracle_seg_box_tstar(const double *A, const double *B, const double *c, const double *hh)
{
    return or_seg_box_tstar(A, B, c, hh);
}

void oracle_contacts(const OScene *s, const double *x, int cap, int *n, int *pair, double *phi, double *nrm,
                     double *p)
{
    OArmKin kin[2];
    OContact con[OR_MAXCON];
    or_fk(s, 0, x, &kin[0]);
    or_fk(s, 1, x + 7, &kin[1]);
    if (cap > OR_MAXCON) cap = OR_MAXCON;
    int nc = or_contacts(s, kin, x + 42, con, cap);
    *n = nc;
    for (int i = 0; i < nc; ++i) {
        pair[i] = con[i].pair;
        phi[i] = con[i].phi;
        memcpy(nrm + 3 * i, con[i].n, 3 * sizeof(double));
        memcpy(p + 3 * i, con[i].p, 3 * sizeof(double));
    }
}
