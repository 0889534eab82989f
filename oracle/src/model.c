/*
 * Oracle rigid-body model of the two arms: link inertias, forward
 * kinematics, joint-space mass matrix and inverse dynamics, in FP64.
 *
 * The paper's world model f (Eq. state_evol) is MuJoCo; the arms and their
 * inertias are readings: each link is a solid capsule of uniform density,
 * joint i+1 sits at the end of link i along its local z axis, and the
 * joints rotate about the local axes given in the scene.  The forward
 * kinematics places the end-effector pads used by the task costs
 * (Sec. IV-A, end-effector poses e_{i,k} are part of x_k).
 * TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

/* Solid capsule (cylinder of length L plus two hemispherical caps, radius
 * r) of density rho: mass, transverse and axial inertia about its centre. */
static void capsule_inertia(double rho, double L, double r, double *m, double *Ix, double *Iz)
{
    double mc = rho * M_PI * r * r * L;
    double ms = rho * 4.0 / 3.0 * M_PI * r * r * r;
    *m = mc + ms;
    *Iz = mc * r * r / 2.0 + ms * 2.0 * r * r / 5.0;
    /* each cap: mass ms/2, centroid 3r/8 from its flat face; inertia about a
     * diameter of the flat face is (2/5)(ms/2)r^2; move to the centroid, then
     * to the capsule centre at distance L/2 + 3r/8. */
    double cap_c = 2.0 / 5.0 * (ms / 2.0) * r * r - (ms / 2.0) * (3.0 * r / 8.0) * (3.0 * r / 8.0);
    double dist = L / 2.0 + 3.0 * r / 8.0;
    double caps = 2.0 * (cap_c + (ms / 2.0) * dist * dist);
    *Ix = mc * (3.0 * r * r + L * L) / 12.0 + caps;
}

void or_model(const OScene *s, OModel *md)
{
    for (int a = 0; a < 2; ++a)
        for (int i = 0; i < OR_NJ; ++i)
            capsule_inertia(s->density[a][i], s->link_len[i], s->link_rad[i], &md->m[a][i], &md->Ix[a][i],
                            &md->Iz[a][i]);
    md->ball_I = 0.4 * s->ball_m * s->ball_r * s->ball_r;
    if (s->obj_box) {
        /* solid box: m (b^2 + c^2) / 12 with full sides b = 2 h_y, c = 2 h_z, ... */
        const double *hh = s->obj_h;
        md->obj_I[0] = s->ball_m * (hh[1] * hh[1] + hh[2] * hh[2]) / 3.0;
        md->obj_I[1] = s->ball_m * (hh[0] * hh[0] + hh[2] * hh[2]) / 3.0;
        md->obj_I[2] = s->ball_m * (hh[0] * hh[0] + hh[1] * hh[1]) / 3.0;
    } else {
        md->obj_I[0] = md->obj_I[1] = md->obj_I[2] = md->ball_I;
    }
    md->eps = s->eps_frac * s->ball_r;
    double rr = s->ball_r + s->pad_rad;
    md->l_ball = 2.0 * sqrt(rr * rr - md->eps * md->eps);
}

static void mat_mul3(const double A[3][3], const double B[3][3], double C[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += A[i][k] * B[k][j];
            C[i][j] = acc;
        }
}

/* rotation by angle t about coordinate axis ax */
static void axis_rot(int ax, double t, double R[3][3])
{
    double c = cos(t), s = sin(t);
    memset(R, 0, 9 * sizeof(double));
    R[ax][ax] = 1.0;
    int i = (ax + 1) % 3, j = (ax + 2) % 3;
    R[i][i] = c; R[i][j] = -s;
    R[j][i] = s; R[j][j] = c;
}

void or_fk(const OScene *s, int arm, const double *q7, OArmKin *k)
{
    double R[3][3] = {{s->base_cs[arm][0], -s->base_cs[arm][1], 0.0},
                      {s->base_cs[arm][1], s->base_cs[arm][0], 0.0},
                      {0.0, 0.0, 1.0}};
    double o[3] = {s->base_pos[arm][0], s->base_pos[arm][1], s->base_pos[arm][2]};
    for (int i = 0; i < OR_NJ; ++i) {
        int ax = s->axes[i];
        /* the joint axis is the same before and after rotating about it */
        for (int r = 0; r < 3; ++r) k->a[i][r] = R[r][ax];
        for (int r = 0; r < 3; ++r) k->o[i][r] = o[r];
        double Rj[3][3], Rn[3][3];
        axis_rot(ax, q7[i], Rj);
        mat_mul3(R, Rj, Rn);
        memcpy(R, Rn, sizeof(R));
        memcpy(k->R[i], R, sizeof(R));
        for (int r = 0; r < 3; ++r) {
            k->c[i][r] = o[r] + 0.5 * s->link_len[i] * R[r][2];
            o[r] = o[r] + s->link_len[i] * R[r][2];
        }
    }
    for (int r = 0; r < 3; ++r) k->o[OR_NJ][r] = o[r];
}

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* world-frame rotational inertia of link i about its COM (axisymmetric
 * about the link's local z axis) */
static void link_inertia_world(const OModel *md, int arm, int i, const OArmKin *k, double I[3][3])
{
    double z[3] = {k->R[i][0][2], k->R[i][1][2], k->R[i][2][2]};
    double ix = md->Ix[arm][i], iz = md->Iz[arm][i];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) I[r][c] = ix * ((r == c) ? 1.0 : 0.0) + (iz - ix) * z[r] * z[c];
}

/* M = sum_i (m_i Jv_i^T Jv_i + Jw_i^T I_i Jw_i): the kinetic-energy
 * definition of the joint-space inertia, written out link by link. */
void or_mass_matrix(const OScene *s, const OModel *md, int arm, const OArmKin *k, double M[OR_NJ][OR_NJ])
{
    (void)s;
    memset(M, 0, sizeof(double) * OR_NJ * OR_NJ);
    for (int i = 0; i < OR_NJ; ++i) {
        double Jv[3][OR_NJ], Jw[3][OR_NJ];
        memset(Jv, 0, sizeof(Jv));
        memset(Jw, 0, sizeof(Jw));
        for (int j = 0; j <= i; ++j) {
            double d[3] = {k->c[i][0] - k->o[j][0], k->c[i][1] - k->o[j][1], k->c[i][2] - k->o[j][2]};
            double v[3];
            cross(k->a[j], d, v);
            for (int r = 0; r < 3; ++r) { Jv[r][j] = v[r]; Jw[r][j] = k->a[j][r]; }
        }
        double I[3][3];
        link_inertia_world(md, arm, i, k, I);
        double m = md->m[arm][i];
        for (int p = 0; p < OR_NJ; ++p)
            for (int q = 0; q < OR_NJ; ++q) {
                double acc = 0.0;
                for (int r = 0; r < 3; ++r) acc += m * Jv[r][p] * Jv[r][q];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) acc += Jw[r][p] * I[r][c] * Jw[c][q];
                M[p][q] += acc;
            }
    }
}

/* Recursive Newton-Euler inverse dynamics in the world frame (Featherstone,
 * Rigid Body Dynamics Algorithms, 2008, ch. 5, written with 3-vectors).
 * Returns tau = M(q) qdd + c(q, qd) [+ gravity torques if gravity != 0]. */
void or_rnea(const OScene *s, const OModel *md, int arm, const OArmKin *k, const double *qd,
             const double *qdd, int gravity, double *tau)
{
    double w[OR_NJ][3], al[OR_NJ][3], ao[OR_NJ][3], ac[OR_NJ][3];
    double wprev[3] = {0, 0, 0}, alprev[3] = {0, 0, 0};
    /* base acceleration: gravity enters as an upward acceleration of the base */
    double aoprev[3] = {0, 0, gravity ? s->g : 0.0};
    for (int i = 0; i < OR_NJ; ++i) {
        double t[3];
        if (i == 0) {
            for (int r = 0; r < 3; ++r) ao[i][r] = aoprev[r];
        } else {
            double d[3] = {k->o[i][0] - k->o[i - 1][0], k->o[i][1] - k->o[i - 1][1], k->o[i][2] - k->o[i - 1][2]};
            double t1[3], t2[3], t3[3];
            cross(alprev, d, t1);
            cross(wprev, d, t2);
            cross(wprev, t2, t3);
            for (int r = 0; r < 3; ++r) ao[i][r] = aoprev[r] + t1[r] + t3[r];
        }
        cross(wprev, k->a[i], t);
        for (int r = 0; r < 3; ++r) {
            w[i][r] = wprev[r] + qd[i] * k->a[i][r];
            al[i][r] = alprev[r] + qdd[i] * k->a[i][r] + qd[i] * t[r];
        }
        double dc[3] = {k->c[i][0] - k->o[i][0], k->c[i][1] - k->o[i][1], k->c[i][2] - k->o[i][2]};
        double t1[3], t2[3], t3[3];
        cross(al[i], dc, t1);
        cross(w[i], dc, t2);
        cross(w[i], t2, t3);
        for (int r = 0; r < 3; ++r) ac[i][r] = ao[i][r] + t1[r] + t3[r];
        for (int r = 0; r < 3; ++r) { wprev[r] = w[i][r]; alprev[r] = al[i][r]; aoprev[r] = ao[i][r]; }
    }
    double F[3] = {0, 0, 0}, N[3] = {0, 0, 0};
    for (int i = OR_NJ - 1; i >= 0; --i) {
        double I[3][3];
        link_inertia_world(md, arm, i, k, I);
        double m = md->m[arm][i];
        double Ia[3], Iw[3], wIw[3];
        for (int r = 0; r < 3; ++r) {
            Ia[r] = I[r][0] * al[i][0] + I[r][1] * al[i][1] + I[r][2] * al[i][2];
            Iw[r] = I[r][0] * w[i][0] + I[r][1] * w[i][1] + I[r][2] * w[i][2];
        }
        cross(w[i], Iw, wIw);
        double fi[3] = {m * ac[i][0], m * ac[i][1], m * ac[i][2]};
        double dc[3] = {k->c[i][0] - k->o[i][0], k->c[i][1] - k->o[i][1], k->c[i][2] - k->o[i][2]};
        double dn[3] = {k->o[i + 1][0] - k->o[i][0], k->o[i + 1][1] - k->o[i][1], k->o[i + 1][2] - k->o[i][2]};
        double m1[3], m2[3];
        cross(dc, fi, m1);
        cross(dn, F, m2); /* F, N still hold the child's values here */
        double Nn[3];
        for (int r = 0; r < 3; ++r) Nn[r] = Ia[r] + wIw[r] + m1[r] + N[r] + m2[r];
        for (int r = 0; r < 3; ++r) { F[r] = fi[r] + F[r]; N[r] = Nn[r]; }
        tau[i] = k->a[i][0] * N[0] + k->a[i][1] * N[1] + k->a[i][2] * N[2];
    }
}

/* dense Cholesky A = L L^T (row-major n x n); returns 0 if a pivot <= 0 */
int or_cholesky(int n, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * n * n);
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return 0;
        L[j * n + j] = sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = v / L[j * n + j];
        }
    }
    return 1;
}

void or_chol_solve(int n, const double *L, const double *b, double *x)
{
    double y[64];
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
        y[i] = v / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * x[k];
        x[i] = v / L[i * n + i];
    }
}

/* exported for tests */
void oracle_fk(const OScene *s, int arm, const double *q7, double *R /*7*9*/, double *o /*8*3*/,
               double *a /*7*3*/, double *c /*7*3*/)
{
    OArmKin k;
    or_fk(s, arm, q7, &k);
    memcpy(R, k.R, sizeof(k.R));
    memcpy(o, k.o, sizeof(k.o));
    memcpy(a, k.a, sizeof(k.a));
    memcpy(c, k.c, sizeof(k.c));
}

void oracle_model(const OScene *s, double *m /*2*7*/, double *Ix, double *Iz, double *extra /*3*/)
{
    OModel md;
    or_model(s, &md);
    memcpy(m, md.m, sizeof(md.m));
    memcpy(Ix, md.Ix, sizeof(md.Ix));
    memcpy(Iz, md.Iz, sizeof(md.Iz));
    extra[0] = md.ball_I; extra[1] = md.eps; extra[2] = md.l_ball;
}

void oracle_mass_matrix(const OScene *s, int arm, const double *q7, double *M)
{
    OModel md;
    OArmKin k;
    or_model(s, &md);
    or_fk(s, arm, q7, &k);
    or_mass_matrix(s, &md, arm, &k, (double(*)[OR_NJ])M);
}

void oracle_rnea(const OScene *s, int arm, const double *q7, const double *qd, const double *qdd, int gravity,
                 double *tau)
{
    OModel md;
    OArmKin k;
    or_model(s, &md);
    or_fk(s, arm, q7, &k);
    or_rnea(s, &md, arm, &k, qd, qdd, gravity, tau);
}

int oracle_cholesky(int n, const double *A, double *L) { return or_cholesky(n, A, L); }
