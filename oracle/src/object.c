/*
 * Oracle geometry of the free object when it is a solid box (FP64): the tray
 * of the tray-moving task (Sec. IV-A) and the cube of the hand-over task
 * (Sec. IV-C); both are free bodies moved only through contact with the
 * end-effectors.  Readings (the paper's world model is MuJoCo and fixes
 * none of this):
 *   * pose: centre p and unit quaternion q = (w, x, y, z), R(q) its rotation;
 *     vertex k (0..7) is p + R (s_x hx, s_y hy, s_z hz) with s_x = +1 when
 *     bit 0 of k is set, else -1 (bits 1, 2 for y, z);
 *   * box - table: every vertex below the plane z = 0 is a contact (phi = its
 *     height, n = +z, p midway between the vertex and the plane), in vertex
 *     order, at most four per substep;
 *   * box - sphere and box - capsule: the sphere / capsule pair against a box,
 *     computed in the box's frame (the capsule core point that minimises the
 *     box's signed distance, as for the static boxes), with the normal turned
 *     to point from the other geom towards the object;
 *   * box - static box: separating axes (the three face normals of each box
 *     and their nine cross products, in that order, cross products shorter
 *     than 1e-9 skipped): phi is the largest separation over the axes (the
 *     penetration depth when they overlap, a lower bound of the distance when
 *     apart), n that axis (the first on ties) turned towards the object, p
 *     midway between the object's support vertex along -n and the static
 *     box's support vertex along n (lowest vertex index on ties).
 * TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

/* exported from collide.c: the pairwise narrowphase of two primitives */
void or_narrow_prim(int ta, const double A0[3], const double A1[3], double ra, int tb, const double B0[3],
                    const double B1[3], double rb, double *phi, double n[3], double p[3]);

enum { SH_SPHERE = 0, SH_CAPSULE = 1, SH_PLANE = 2, SH_BOX = 3 };

void or_quat_to_R(const double q[4], double R[3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

/* rotation matrix -> unit quaternion (Shepperd's method: the largest of
 * w^2, x^2, y^2, z^2 is taken from the diagonal first) */
void or_R_to_quat(const double R[3][3], double q[4])
{
    double tr = R[0][0] + R[1][1] + R[2][2];
    double c[4] = {tr, R[0][0], R[1][1], R[2][2]};
    int k = 0;
    for (int i = 1; i < 4; ++i)
        if (c[i] > c[k]) k = i;
    if (k == 0) {
        double w = 0.5 * sqrt(1.0 + tr);
        q[0] = w;
        q[1] = (R[2][1] - R[1][2]) / (4 * w);
        q[2] = (R[0][2] - R[2][0]) / (4 * w);
        q[3] = (R[1][0] - R[0][1]) / (4 * w);
    } else if (k == 1) {
        double x = 0.5 * sqrt(1.0 + 2 * R[0][0] - tr);
        q[1] = x;
        q[0] = (R[2][1] - R[1][2]) / (4 * x);
        q[2] = (R[0][1] + R[1][0]) / (4 * x);
        q[3] = (R[0][2] + R[2][0]) / (4 * x);
    } else if (k == 2) {
        double y = 0.5 * sqrt(1.0 + 2 * R[1][1] - tr);
        q[2] = y;
        q[0] = (R[0][2] - R[2][0]) / (4 * y);
        q[1] = (R[0][1] + R[1][0]) / (4 * y);
        q[3] = (R[1][2] + R[2][1]) / (4 * y);
    } else {
        double z = 0.5 * sqrt(1.0 + 2 * R[2][2] - tr);
        q[3] = z;
        q[0] = (R[1][0] - R[0][1]) / (4 * z);
        q[1] = (R[0][2] + R[2][0]) / (4 * z);
        q[2] = (R[1][2] + R[2][1]) / (4 * z);
    }
}

/* geodesic distance of two unit quaternions: 2 acos |<q, Q>| (Sec. IV) */
double or_quat_angle(const double q[4], const double Q[4])
{
    double d = fabs(q[0] * Q[0] + q[1] * Q[1] + q[2] * Q[2] + q[3] * Q[3]);
    if (d > 1.0) d = 1.0;
    return 2.0 * acos(d);
}

static void vertex(const double c[3], const double R[3][3], const double h[3], int k, double v[3])
{
    double l[3] = {(k & 1) ? h[0] : -h[0], (k & 2) ? h[1] : -h[1], (k & 4) ? h[2] : -h[2]};
    for (int i = 0; i < 3; ++i) v[i] = c[i] + R[i][0] * l[0] + R[i][1] * l[1] + R[i][2] * l[2];
}

/* the eight vertex contacts with the table (phi = height; the caller keeps
 * the ones below it); returns 8 */
int or_obj_table(const OScene *s, const double *xo, double phi[8], double n[8][3], double p[8][3])
{
    double R[3][3];
    or_quat_to_R(xo + 3, R);
    for (int k = 0; k < 8; ++k) {
        double v[3];
        vertex(xo, R, s->obj_h, k, v);
        phi[k] = v[2];
        n[k][0] = 0.0; n[k][1] = 0.0; n[k][2] = 1.0;
        p[k][0] = v[0]; p[k][1] = v[1]; p[k][2] = 0.5 * v[2];
    }
    return 8;
}

static void to_frame(const double c[3], const double R[3][3], const double x[3], double l[3])
{
    double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    for (int i = 0; i < 3; ++i) l[i] = R[0][i] * d[0] + R[1][i] * d[1] + R[2][i] * d[2];
}

static void from_frame(const double c[3], const double R[3][3], const double l[3], double x[3])
{
    for (int i = 0; i < 3; ++i) x[i] = c[i] + R[i][0] * l[0] + R[i][1] * l[1] + R[i][2] * l[2];
}

/* support vertex of a box (centre c, rotation R, half extents h) along d */
static void support(const double c[3], const double R[3][3], const double h[3], const double d[3], double v[3])
{
    double best = -INFINITY;
    for (int k = 0; k < 8; ++k) {
        double w[3];
        vertex(c, R, h, k, w);
        double e = w[0] * d[0] + w[1] * d[1] + w[2] * d[2];
        if (e > best) {
            best = e;
            memcpy(v, w, sizeof(w));
        }
    }
}

/* the object (geom A) against geom B of type tb: sphere / capsule (B0, B1,
 * rb), the plane (deepest vertex) or a static axis-aligned box (B0 centre,
 * B1 half extents) */
void or_obj_narrow(const OScene *s, const double *xo, int tb, const double B0[3], const double B1[3], double rb,
                   double *phi, double n[3], double p[3])
{
    double R[3][3];
    or_quat_to_R(xo + 3, R);
    const double *c = xo;
    if (tb == SH_PLANE) {
        double ph[8], nn[8][3], pp[8][3];
        or_obj_table(s, xo, ph, nn, pp);
        int k = 0;
        for (int i = 1; i < 8; ++i)
            if (ph[i] < ph[k]) k = i;
        *phi = ph[k];
        memcpy(n, nn[k], 3 * sizeof(double));
        memcpy(p, pp[k], 3 * sizeof(double));
        return;
    }
    if (tb == SH_SPHERE || tb == SH_CAPSULE) {
        double l0[3], l1[3], zero[3] = {0, 0, 0}, nl[3], pl[3];
        to_frame(c, R, B0, l0);
        to_frame(c, R, B1, l1);
        or_narrow_prim(tb, l0, l1, rb, SH_BOX, zero, s->obj_h, 0.0, phi, nl, pl);
        /* nl points from the box towards the other geom: turn it around */
        for (int i = 0; i < 3; ++i) n[i] = -(R[i][0] * nl[0] + R[i][1] * nl[1] + R[i][2] * nl[2]);
        from_frame(c, R, pl, p);
        return;
    }
    /* static axis-aligned box: separating axes */
    double I3[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double axes[15][3];
    int na = 0;
    for (int i = 0; i < 3; ++i) {
        for (int r = 0; r < 3; ++r) axes[na][r] = R[r][i];
        ++na;
    }
    for (int j = 0; j < 3; ++j) {
        for (int r = 0; r < 3; ++r) axes[na][r] = I3[r][j];
        ++na;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a[3] = {R[0][i], R[1][i], R[2][i]}, e[3] = {I3[0][j], I3[1][j], I3[2][j]};
            double x[3] = {a[1] * e[2] - a[2] * e[1], a[2] * e[0] - a[0] * e[2], a[0] * e[1] - a[1] * e[0]};
            double len = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            if (len < 1e-9) continue;
            for (int r = 0; r < 3; ++r) axes[na][r] = x[r] / len;
            ++na;
        }
    double d[3] = {c[0] - B0[0], c[1] - B0[1], c[2] - B0[2]};
    double best = -INFINITY, bn[3] = {0, 0, 1};
    for (int k = 0; k < na; ++k) {
        const double *L = axes[k];
        double ra = 0.0, rbx = 0.0;
        for (int i = 0; i < 3; ++i) {
            ra += s->obj_h[i] * fabs(R[0][i] * L[0] + R[1][i] * L[1] + R[2][i] * L[2]);
            rbx += B1[i] * fabs(L[i]);
        }
        double dl = d[0] * L[0] + d[1] * L[1] + d[2] * L[2];
        double sep = fabs(dl) - ra - rbx;
        if (sep > best) {
            best = sep;
            double sg = dl >= 0.0 ? 1.0 : -1.0;
            for (int r = 0; r < 3; ++r) bn[r] = sg * L[r];
        }
    }
    *phi = best;
    memcpy(n, bn, sizeof(bn));
    double mn[3] = {-bn[0], -bn[1], -bn[2]}, va[3], vb[3];
    support(c, R, s->obj_h, mn, va);
    support(B0, I3, B1, bn, vb);
    for (int i = 0; i < 3; ++i) p[i] = 0.5 * (va[i] + vb[i]);
}

/* ---- exported for tests ---- */
void oracle_obj_prim(const OScene *s, const double *xo, int tb, const double *B0, const double *B1, double rb,
                     double *out /* phi, n[3], p[3] */)
{
    or_obj_narrow(s, xo, tb, B0, B1, rb, &out[0], out + 1, out + 4);
}

void oracle_quat_R(const double *q, double *R, double *q_back)
{
    double M[3][3];
    or_quat_to_R(q, M);
    memcpy(R, M, sizeof(M));
    or_R_to_quat(M, q_back);
}
