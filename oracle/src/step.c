/*
 * Oracle physics substep (FP64): the world model f of Eq. state_evol.
 *
 * The paper only says that f is a MuJoCo physics engine stepped at 0.1 s
 * (Sec. V-A); the joint-velocity command of Eq. cost drives the arms.  The
 * substep below is the reading used throughout:
 *   1. PD target: q_des += h u;
 *   2. actuator torque tau = clamp(Kp (q_des - q) + Kd (u - qd), +-tau_max);
 *   3. free velocity from (M + diag(armature + h (Kd + b))) (qd_f - qd)
 *      = h (tau - b qd - c(q, qd)), with c from inverse dynamics (no arm
 *      gravity when gravity compensation is on); the object falls freely
 *      and, when it is a box, its angular velocity takes the explicit
 *      gyroscopic step w_f = w - h W (w x I_w w), I_w = R I R^T, W = I_w^-1;
 *   4. contacts at the current positions, four pyramid-edge rows each
 *      (n +- mu t1, n +- mu t2), solved by projected Gauss-Seidel on the
 *      explicitly assembled soft LCP (A + R) f + b >= 0, f >= 0,
 *      A = J Mt^-1 J^T, R_e = eps_r A_ee, b = J qd_f - kappa max(-phi, 0)/h,
 *      f = 0 at the start, n_pgs sweeps in row order;
 *   5. qd+ = qd_f + Mt^-1 J^T f, then semi-implicit Euler:
 *      q += h qd+, p_ball += h v+, r <- normalize(exp(h w+/2) (x) r).
 * TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Orthonormal tangents of a unit normal (Duff, Burgess, Christensen, Hery,
 * Kensler, Liani, Villemin, "Building an orthonormal basis, revisited",
 * JCGT 6(1), 2017). */
void or_tangents(const double n[3], double t1[3], double t2[3])
{
    double sg = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sg + n[2]);
    double b = n[0] * n[1] * a;
    t1[0] = 1.0 + sg * n[0] * n[0] * a; t1[1] = sg * b; t1[2] = -sg * n[0];
    t2[0] = b; t2[1] = sg + n[1] * n[1] * a; t2[2] = -n[1];
}

/* 3 x 20 point Jacobian of the point p attached to geom gid */
void or_point_jac(const OScene *s, const OArmKin kin[2], const double *pball, int gid, const double p[3],
                      double J[3][OR_NDOF], double sign)
{
    (void)s;
    if (gid == OG_BALL) {
        double r[3] = {p[0] - pball[0], p[1] - pball[1], p[2] - pball[2]};
        /* v_p = v + w x r = v - [r]x w */
        double Rx[3][3] = {{0, -r[2], r[1]}, {r[2], 0, -r[0]}, {-r[1], r[0], 0}};
        for (int i = 0; i < 3; ++i) {
            J[i][14 + i] += sign;
            for (int j = 0; j < 3; ++j) J[i][17 + j] += -sign * Rx[i][j];
        }
    } else if (gid >= OG_ARM && gid < OG_BOX) {
        int arm = (gid - OG_ARM) / 7, g = (gid - OG_ARM) % 7;
        int link = g; /* capsules g = 0..5 on links 0..5, pad (g = 6) on link 6 */
        for (int j = 0; j <= link; ++j) {
            double d[3] = {p[0] - kin[arm].o[j][0], p[1] - kin[arm].o[j][1], p[2] - kin[arm].o[j][2]};
            double v[3];
            cross(kin[arm].a[j], d, v);
            for (int i = 0; i < 3; ++i) J[i][7 * arm + j] += sign * v[i];
        }
    }
    /* table and boxes are static */
}

/* world-frame inverse inertia W = R diag(1/I) R^T and inertia I_w = R diag(I) R^T
 * of the object at quaternion q */
static void obj_inertia_world(const OModel *md, const double *q, double W[3][3], double Iw[3][3])
{
    double R[3][3];
    or_quat_to_R(q, R);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double w = 0.0, v = 0.0;
            for (int k = 0; k < 3; ++k) {
                w += R[i][k] * R[j][k] / md->obj_I[k];
                v += R[i][k] * R[j][k] * md->obj_I[k];
            }
            W[i][j] = w;
            Iw[i][j] = v;
        }
}

/* x_out = Mt^-1 y for the block-diagonal Mt (two arm factors + object);
 * W: the box object's world inverse inertia (unused for the ball) */
static void mt_solve(const double Larm[2][OR_NJ * OR_NJ], const OScene *s, const OModel *md, const double W[3][3],
                     const double *y, double *xo)
{
    or_chol_solve(OR_NJ, Larm[0], y, xo);
    or_chol_solve(OR_NJ, Larm[1], y + 7, xo + 7);
    for (int i = 0; i < 3; ++i) xo[14 + i] = y[14 + i] / s->ball_m;
    if (s->obj_box) {
        for (int i = 0; i < 3; ++i) xo[17 + i] = W[i][0] * y[17] + W[i][1] * y[18] + W[i][2] * y[19];
    } else {
        for (int i = 0; i < 3; ++i) xo[17 + i] = y[17 + i] / md->ball_I;
    }
}

/* the object's free angular velocity: w, minus the explicit gyroscopic step
 * h W (w x I_w w) for a box */
static void obj_free_w(const OScene *s, const double W[3][3], const double Iw[3][3], const double *w, double *wf)
{
    for (int i = 0; i < 3; ++i) wf[i] = w[i];
    if (!s->obj_box) return;
    double L[3], g[3];
    for (int i = 0; i < 3; ++i) L[i] = Iw[i][0] * w[0] + Iw[i][1] * w[1] + Iw[i][2] * w[2];
    cross(w, L, g);
    for (int i = 0; i < 3; ++i) wf[i] -= s->h * (W[i][0] * g[0] + W[i][1] * g[1] + W[i][2] * g[2]);
}

void or_substep(const OScene *s, const OModel *md, const double *x, const double *u, double *xn, int *ncon_out)
{
    const double h = s->h;
    const double *q = x, *qd = x + 14, *qdes = x + 28, *pb = x + 42, *quat = x + 45, *vb = x + 49, *wb = x + 52;
    double qdes_n[14];
    for (int i = 0; i < 14; ++i) qdes_n[i] = qdes[i] + h * u[i];

    OArmKin kin[2];
    or_fk(s, 0, q, &kin[0]);
    or_fk(s, 1, q + 7, &kin[1]);

    double Larm[2][OR_NJ * OR_NJ];
    double vfree[OR_NDOF];
    for (int a = 0; a < 2; ++a) {
        double M[OR_NJ][OR_NJ], c[OR_NJ], zero[OR_NJ] = {0};
        or_mass_matrix(s, md, a, &kin[a], M);
        or_rnea(s, md, a, &kin[a], qd + 7 * a, zero, s->gravcomp ? 0 : 1, c);
        double rhs[OR_NJ];
        for (int i = 0; i < OR_NJ; ++i) {
            int d = 7 * a + i;
            double tau = s->kp * (qdes_n[d] - q[d]) + s->kd * (u[d] - qd[d]);
            if (tau > s->tau_max) tau = s->tau_max;
            if (tau < -s->tau_max) tau = -s->tau_max;
            rhs[i] = h * (tau - s->damp * qd[d] - c[i]);
            M[i][i] += s->armature + h * (s->kd + s->damp);
        }
        if (!or_cholesky(OR_NJ, &M[0][0], Larm[a])) {
            /* non-SPD inertia: poison the state */
            for (int i = 0; i < OR_NX; ++i) xn[i] = NAN;
            if (ncon_out) *ncon_out = 0;
            return;
        }
        double dq[OR_NJ];
        or_chol_solve(OR_NJ, Larm[a], rhs, dq);
        for (int i = 0; i < OR_NJ; ++i) vfree[7 * a + i] = qd[7 * a + i] + dq[i];
    }
    double W[3][3], Iw[3][3];
    obj_inertia_world(md, quat, W, Iw);
    for (int i = 0; i < 3; ++i) vfree[14 + i] = vb[i];
    vfree[16] -= h * s->g;
    obj_free_w(s, W, Iw, wb, vfree + 17);

    OContact con[OR_MAXCON];
    int nc = or_contacts(s, kin, pb, con, s->n_cmax < OR_MAXCON ? s->n_cmax : OR_MAXCON);
    if (ncon_out) *ncon_out = nc;
    double vplus[OR_NDOF];
    memcpy(vplus, vfree, sizeof(vplus));
    if (nc > 0) {
        int m = 4 * nc;
        static __thread double J[4 * OR_MAXCON][OR_NDOF], MiJT[4 * OR_MAXCON][OR_NDOF];
        static __thread double A[4 * OR_MAXCON][4 * OR_MAXCON];
        double b[4 * OR_MAXCON], Rr[4 * OR_MAXCON], f[4 * OR_MAXCON];
        for (int c = 0; c < nc; ++c) {
            double Jp[3][OR_NDOF];
            memset(Jp, 0, sizeof(Jp));
            or_point_jac(s, kin, pb, con[c].ga, con[c].p, Jp, 1.0);
            or_point_jac(s, kin, pb, con[c].gb, con[c].p, Jp, -1.0);
            double t1[3], t2[3];
            or_tangents(con[c].n, t1, t2);
            double e[4][3];
            for (int i = 0; i < 3; ++i) {
                e[0][i] = con[c].n[i] + s->mu * t1[i];
                e[1][i] = con[c].n[i] - s->mu * t1[i];
                e[2][i] = con[c].n[i] + s->mu * t2[i];
                e[3][i] = con[c].n[i] - s->mu * t2[i];
            }
            double pen = con[c].phi < 0.0 ? -con[c].phi : 0.0;
            for (int r = 0; r < 4; ++r) {
                int row = 4 * c + r;
                for (int d = 0; d < OR_NDOF; ++d)
                    J[row][d] = e[r][0] * Jp[0][d] + e[r][1] * Jp[1][d] + e[r][2] * Jp[2][d];
                double jv = 0.0;
                for (int d = 0; d < OR_NDOF; ++d) jv += J[row][d] * vfree[d];
                b[row] = jv - s->kappa * pen / h;
            }
        }
        for (int r = 0; r < m; ++r)
            mt_solve((const double(*)[OR_NJ * OR_NJ])Larm, s, md, (const double(*)[3])W, J[r], MiJT[r]);
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < m; ++c) {
                double acc = 0.0;
                for (int d = 0; d < OR_NDOF; ++d) acc += J[r][d] * MiJT[c][d];
                A[r][c] = acc;
            }
        for (int r = 0; r < m; ++r) { Rr[r] = s->eps_r * A[r][r]; f[r] = 0.0; }
        for (int sweep = 0; sweep < s->n_pgs; ++sweep) {
            for (int r = 0; r < m; ++r) {
                double res = b[r] + Rr[r] * f[r];
                for (int c = 0; c < m; ++c) res += A[r][c] * f[c];
                double fn = f[r] - res / (A[r][r] + Rr[r]);
                f[r] = fn > 0.0 ? fn : 0.0;
            }
        }
        for (int r = 0; r < m; ++r)
            for (int d = 0; d < OR_NDOF; ++d) vplus[d] += MiJT[r][d] * f[r];
    }

    /* semi-implicit Euler */
    for (int i = 0; i < 14; ++i) {
        xn[i] = q[i] + h * vplus[i];
        xn[14 + i] = vplus[i];
        xn[28 + i] = qdes_n[i];
    }
    for (int i = 0; i < 3; ++i) {
        xn[42 + i] = pb[i] + h * vplus[14 + i];
        xn[49 + i] = vplus[14 + i];
        xn[52 + i] = vplus[17 + i];
    }
    /* quaternion (w, x, y, z), world-frame angular velocity: exp map */
    double th[3] = {h * vplus[17], h * vplus[18], h * vplus[19]};
    double ang = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    double dq[4];
    if (ang < 1e-8) {
        dq[0] = 1.0; dq[1] = 0.5 * th[0]; dq[2] = 0.5 * th[1]; dq[3] = 0.5 * th[2];
    } else {
        double sh = sin(0.5 * ang) / ang;
        dq[0] = cos(0.5 * ang); dq[1] = sh * th[0]; dq[2] = sh * th[1]; dq[3] = sh * th[2];
    }
    /* dq (x) quat */
    double w1 = dq[0], w2 = quat[0];
    const double *v1 = dq + 1, *v2 = quat + 1;
    double cr[3];
    cross(v1, v2, cr);
    double qn[4];
    qn[0] = w1 * w2 - (v1[0] * v2[0] + v1[1] * v2[1] + v1[2] * v2[2]);
    for (int i = 0; i < 3; ++i) qn[1 + i] = w1 * v2[i] + w2 * v1[i] + cr[i];
    double nq = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int i = 0; i < 4; ++i) xn[45 + i] = qn[i] / nq;
}

/* ---- exported for tests ---- */
void oracle_substep(const OScene *s, const double *x, const double *u, double *xn, int *ncon)
{
    OModel md;
    or_model(s, &md);
    or_substep(s, &md, x, u, xn, ncon);
}

void oracle_tangents(const double *n, double *t1, double *t2) { or_tangents(n, t1, t2); }

/* dense LCP pieces at state x for inspection: returns m (rows); fills
 * A[m*m], b[m], f[m] after n_pgs sweeps (caps at 64 rows) */
int oracle_lcp(const OScene *s, const double *x, const double *u, double *Aout, double *bout, double *fout,
               double *vfree_out)
{
    OModel md;
    or_model(s, &md);
    const double h = s->h;
    const double *q = x, *qd = x + 14, *qdes = x + 28, *pb = x + 42, *vb = x + 49, *wb = x + 52;
    OArmKin kin[2];
    or_fk(s, 0, q, &kin[0]);
    or_fk(s, 1, q + 7, &kin[1]);
    double Larm[2][OR_NJ * OR_NJ], vfree[OR_NDOF];
    for (int a = 0; a < 2; ++a) {
        double M[OR_NJ][OR_NJ], c[OR_NJ], zero[OR_NJ] = {0}, rhs[OR_NJ], dq[OR_NJ];
        or_mass_matrix(s, &md, a, &kin[a], M);
        or_rnea(s, &md, a, &kin[a], qd + 7 * a, zero, s->gravcomp ? 0 : 1, c);
        for (int i = 0; i < OR_NJ; ++i) {
            int d = 7 * a + i;
            double tau = s->kp * (qdes[d] + h * u[d] - q[d]) + s->kd * (u[d] - qd[d]);
            tau = tau > s->tau_max ? s->tau_max : (tau < -s->tau_max ? -s->tau_max : tau);
            rhs[i] = h * (tau - s->damp * qd[d] - c[i]);
            M[i][i] += s->armature + h * (s->kd + s->damp);
        }
        or_cholesky(OR_NJ, &M[0][0], Larm[a]);
        or_chol_solve(OR_NJ, Larm[a], rhs, dq);
        for (int i = 0; i < OR_NJ; ++i) vfree[7 * a + i] = qd[7 * a + i] + dq[i];
    }
    double W[3][3], Iw[3][3];
    obj_inertia_world(&md, x + 45, W, Iw);
    for (int i = 0; i < 3; ++i) vfree[14 + i] = vb[i];
    vfree[16] -= h * s->g;
    obj_free_w(s, W, Iw, wb, vfree + 17);
    memcpy(vfree_out, vfree, sizeof(vfree));
    OContact con[16];
    int nc = or_contacts(s, kin, pb, con, 16 < s->n_cmax ? 16 : s->n_cmax);
    int m = 4 * nc;
    static double J[64][OR_NDOF], MiJT[64][OR_NDOF];
    for (int c = 0; c < nc; ++c) {
        double Jp[3][OR_NDOF];
        memset(Jp, 0, sizeof(Jp));
        or_point_jac(s, kin, pb, con[c].ga, con[c].p, Jp, 1.0);
        or_point_jac(s, kin, pb, con[c].gb, con[c].p, Jp, -1.0);
        double t1[3], t2[3], e[4][3];
        or_tangents(con[c].n, t1, t2);
        for (int i = 0; i < 3; ++i) {
            e[0][i] = con[c].n[i] + s->mu * t1[i];
            e[1][i] = con[c].n[i] - s->mu * t1[i];
            e[2][i] = con[c].n[i] + s->mu * t2[i];
            e[3][i] = con[c].n[i] - s->mu * t2[i];
        }
        for (int r = 0; r < 4; ++r) {
            double jv = 0.0;
            for (int d = 0; d < OR_NDOF; ++d) {
                J[4 * c + r][d] = e[r][0] * Jp[0][d] + e[r][1] * Jp[1][d] + e[r][2] * Jp[2][d];
                jv += J[4 * c + r][d] * vfree[d];
            }
            bout[4 * c + r] = jv - s->kappa * (con[c].phi < 0 ? -con[c].phi : 0.0) / h;
        }
    }
    for (int r = 0; r < m; ++r)
        mt_solve((const double(*)[OR_NJ * OR_NJ])Larm, s, &md, (const double(*)[3])W, J[r], MiJT[r]);
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) {
            double acc = 0.0;
            for (int d = 0; d < OR_NDOF; ++d) acc += J[r][d] * MiJT[c][d];
            Aout[r * m + c] = acc;
        }
    for (int r = 0; r < m; ++r) fout[r] = 0.0;
    for (int sweep = 0; sweep < s->n_pgs; ++sweep)
        for (int r = 0; r < m; ++r) {
            double R = s->eps_r * Aout[r * m + r];
            double res = bout[r] + R * fout[r];
            for (int c = 0; c < m; ++c) res += Aout[r * m + c] * fout[c];
            double fn = fout[r] - res / (Aout[r * m + r] + R);
            fout[r] = fn > 0.0 ? fn : 0.0;
        }
    return m;
}

/* 3 x 20 Jacobian (row-major) of a point p rigidly attached to geom gid at
 * state x: its world velocity is J qd (arm joints, ball v, ball w). */
void oracle_point_jac(const OScene *s, const double *x, int gid, const double *p, double *Jout)
{
    OArmKin kin[2];
    or_fk(s, 0, x, &kin[0]);
    or_fk(s, 1, x + 7, &kin[1]);
    double J[3][OR_NDOF];
    memset(J, 0, sizeof(J));
    or_point_jac(s, kin, x + 42, gid, p, J, 1.0);
    memcpy(Jout, J, sizeof(J));
}
