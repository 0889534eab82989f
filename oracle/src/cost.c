/*
 * Oracle task cost and rollout (FP64).
 *
 * Ball lifting and transport (Sec. IV-B), single phase, at the H
 * post-step states k = 0..H-1 of a rollout:
 *   goal       ||p_ball,k - p_goal||                 (object-to-target cost,
 *              with the simulated ball position in place of the
 *              end-effector proxy c_k + (0,0,eps))
 *   eef-obj    ||c_k - (p_ball,k - (0,0,eps))||        (Eq. ball_alignment_cost)
 *   distance   (||p1,k - p2,k|| - l_ball)^2            (Eq. end_effector_distance_cost)
 *   planar     ||p1yz,k - p2yz,k||                     (Eq. planar_alignment_cost)
 *   smooth     ||u_k - u_{k-1}||^2, k >= 1             (not in the paper; the
 *              paper gets smoothness from its QP projection)
 *   collision  sum_{k<=H-2} max(-d_{k+1} + (1-gamma) d_k, 0)
 *              + sum_{k<=H-1} 1{d_k < 0}, elementwise over the distance
 *              vector and summed                     (Eq. collision_cost)
 * with c_k the pad midpoint, eps = eps_frac * r_ball and
 * l_ball = 2 sqrt((r_ball + r_pad)^2 - eps^2).  The distance vector holds
 * the signed distances of the arm-box and arm-arm pairs, saturated at m_c
 * (saturation leaves the cost unchanged where it matters: a pair farther
 * than m_c at both steps contributes nothing).
 *
 * The further terms of the paper's task costs (evaluated when s->ext), with
 * p_i, q_i the pad position and frame orientation of arm i (the end-effector
 * pose e_{i,k}), theta the 14 joint angles, and q_obj the object's
 * orientation; each term's weight (and, per task phase, its target) is set
 * by the caller, so the tray total of Sec. IV-A, the ball total of
 * Sec. IV-B and the hand-over total of Sec. IV-C are weightings of them:
 *   7  joint deviation  ||theta_k - theta_home||            (Eq. home_cost)
 *   8  vertical         |p_z,1 - p_z,2|                     (Eq. vertical_alignment_cost,
 *                                                            summed over k)
 *   9  relative velocity sqrt(sum_k ((p1 - p2) . (p1' - p2'))^2)  (Eq. rel_vel_cost)
 *   10, 11 position     ||p_i,k - a_i||                     (Eq. tray_grasp_pos_cost with
 *                                                            weight 1/2 each; hand-over pick /
 *                                                            place position costs)
 *   12, 13 x position   |p_i,k,x - x_i|                     (hand-over pass cost)
 *   14, 15 orientation  2 acos |<q_i,k, Q_i>|               (Eqs. tray_grasp_ori_cost,
 *                                                            tray_move_ori_cost, the ball's
 *                                                            C_r, hand-over phase terms)
 *   16 object orientation 2 acos |<q_obj,k, Q_obj>|          (Eq. tray_ori_cost)
 * The object-position term of the tray (Eq. tray_position_cost) is term 0
 * with the goal as its target; the end-effector distance term 2 takes
 * l_target (l_tray) in place of l_ball when given.  The pad velocity p_i'
 * is the point Jacobian of the pad centre times the joint velocities.
 * TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

void or_stage_terms(const OScene *s, const OModel *md, const double *x, double terms[4])
{
    OArmKin k0, k1;
    or_fk(s, 0, x, &k0);
    or_fk(s, 1, x + 7, &k1);
    const double *p1 = k0.o[7], *p2 = k1.o[7], *pb = x + 42;
    double dg[3], de[3], d12[3];
    for (int i = 0; i < 3; ++i) {
        dg[i] = pb[i] - s->goal[i];
        double c = 0.5 * (p1[i] + p2[i]);
        de[i] = c - (pb[i] - (i == 2 ? md->eps : 0.0));
        d12[i] = p1[i] - p2[i];
    }
    terms[0] = sqrt(dg[0] * dg[0] + dg[1] * dg[1] + dg[2] * dg[2]);
    terms[1] = sqrt(de[0] * de[0] + de[1] * de[1] + de[2] * de[2]);
    double l = sqrt(d12[0] * d12[0] + d12[1] * d12[1] + d12[2] * d12[2]) - (s->l_target > 0 ? s->l_target : md->l_ball);
    terms[2] = l * l;
    terms[3] = sqrt(d12[1] * d12[1] + d12[2] * d12[2]);
}

/* saturated signed distances of the cost pairs at state x */
void or_cost_dist(const OScene *s, const double *x, double *d)
{
    OArmKin kin[2];
    or_fk(s, 0, x, &kin[0]);
    or_fk(s, 1, x + 7, &kin[1]);
    int nb = or_num_cost_pairs(s);
    for (int i = 0; i < nb; ++i) {
        int ga, gb;
        double phi, n[3], p[3];
        or_pair(s, or_cost_pair_index(s, i), &ga, &gb);
        or_narrow(s, kin, x + 42, ga, gb, &phi, n, p);
        d[i] = phi < s->m_c ? phi : s->m_c;
    }
}

/* Eq. collision_cost, one step: barrier max(-d_k + (1 - gamma) d_{k-1}, 0)
 * (when a previous step exists) and indicator 1{d_k < 0}, elementwise and
 * summed over the distance vector. */
static void collision_terms(const double *dprev, const double *dcur, int nd, double gamma, double *barrier,
                            double *indicator)
{
    for (int i = 0; i < nd; ++i) {
        if (dprev) {
            double gk = -dcur[i] + (1.0 - gamma) * dprev[i];
            if (gk > 0.0) *barrier += gk;
        }
        if (dcur[i] < 0.0) *indicator += 1.0;
    }
}

/* terms 7..16 at state x (term 9 as its squared summand, before the root) */
static void ext_terms(const OScene *s, const double *x, double t[10])
{
    OArmKin kin[2];
    or_fk(s, 0, x, &kin[0]);
    or_fk(s, 1, x + 7, &kin[1]);
    double home = 0.0;
    for (int i = 0; i < 14; ++i) home += (x[i] - s->q_home[i]) * (x[i] - s->q_home[i]);
    t[0] = sqrt(home);
    const double *p1 = kin[0].o[7], *p2 = kin[1].o[7];
    t[1] = fabs(p1[2] - p2[2]);
    double v[2][3];
    for (int a = 0; a < 2; ++a) {
        double J[3][OR_NDOF];
        memset(J, 0, sizeof(J));
        or_point_jac(s, kin, x + 42, OG_ARM + 7 * a + 6, kin[a].o[7], J, 1.0);
        for (int r = 0; r < 3; ++r) {
            v[a][r] = 0.0;
            for (int j = 0; j < 14; ++j) v[a][r] += J[r][j] * x[14 + j];
        }
    }
    double rv = 0.0;
    for (int r = 0; r < 3; ++r) rv += (p1[r] - p2[r]) * (v[0][r] - v[1][r]);
    t[2] = rv * rv;
    for (int a = 0; a < 2; ++a) {
        const double *p = kin[a].o[7];
        double d[3] = {p[0] - s->apos[a][0], p[1] - s->apos[a][1], p[2] - s->apos[a][2]};
        t[3 + a] = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        t[5 + a] = fabs(p[0] - s->ax_t[a]);
        double q[4];
        or_R_to_quat(kin[a].R[6], q);
        t[7 + a] = or_quat_angle(q, s->arot[a]);
    }
    t[9] = or_quat_angle(x + 45, s->orot);
}

/* Roll one control sequence U[H][14] out from x0; returns the total cost.
 * traj (optional) receives the H post-step states; terms_out (optional)
 * receives the OR_NTERMS unweighted sums [goal, eef-obj, dist, planar,
 * smooth, barrier, indicator, then terms 7..16 above (zero unless s->ext)]. */
double or_rollout(const OScene *s, const OModel *md, const double *x0, const double *U, int H, double *traj,
                  double *terms_out)
{
    double x[OR_NX], xn[OR_NX];
    memcpy(x, x0, sizeof(x));
    int nd = or_num_cost_pairs(s);
    double *dprev = (double *)malloc(sizeof(double) * (nd > 0 ? nd : 1));
    double *dcur = (double *)malloc(sizeof(double) * (nd > 0 ? nd : 1));
    double acc[OR_NTERMS];
    for (int i = 0; i < OR_NTERMS; ++i) acc[i] = 0.0;
    for (int k = 0; k < H; ++k) {
        const double *u = U + 14 * k;
        for (int sub = 0; sub < s->n_sub; ++sub) {
            or_substep(s, md, x, u, xn, NULL);
            memcpy(x, xn, sizeof(x));
        }
        if (traj) memcpy(traj + (long)k * OR_NX, x, sizeof(x));
        double t[4];
        or_stage_terms(s, md, x, t);
        for (int i = 0; i < 4; ++i) acc[i] += t[i];
        if (k >= 1) {
            double sm = 0.0;
            for (int i = 0; i < 14; ++i) {
                double dd = u[i] - U[14 * (k - 1) + i];
                sm += dd * dd;
            }
            acc[4] += sm;
        }
        or_cost_dist(s, x, dcur);
        collision_terms(k >= 1 ? dprev : NULL, dcur, nd, s->gamma, &acc[5], &acc[6]);
        if (s->ext) {
            double e[10];
            ext_terms(s, x, e);
            for (int i = 0; i < 10; ++i) acc[7 + i] += e[i];
        }
        double *tmp = dprev; dprev = dcur; dcur = tmp;
    }
    free(dprev);
    free(dcur);
    acc[9] = sqrt(acc[9]);
    if (terms_out) memcpy(terms_out, acc, sizeof(acc));
    double c = s->w_goal * acc[0] + s->w_eo * acc[1] + s->w_l * acc[2] + s->w_yz * acc[3] + s->w_s * acc[4] +
               s->w_c * (acc[5] + acc[6]);
    if (s->ext)
        c += s->w_home * acc[7] + s->w_vert * acc[8] + s->w_relv * acc[9] + s->w_apos[0] * acc[10] +
             s->w_apos[1] * acc[11] + s->w_ax[0] * acc[12] + s->w_ax[1] * acc[13] + s->w_arot[0] * acc[14] +
             s->w_arot[1] * acc[15] + s->w_orot * acc[16];
    if (!isfinite(c)) return INFINITY;
    for (int i = 0; i < OR_NX; ++i)
        if (!isfinite(x[i])) return INFINITY;
    return c;
}

/* ---- exported for tests ---- */
double oracle_rollout(const OScene *s, const double *x0, const double *U, int H, double *traj, double *terms)
{
    OModel md;
    or_model(s, &md);
    return or_rollout(s, &md, x0, U, H, traj, terms);
}

void oracle_stage_terms(const OScene *s, const double *x, double *terms)
{
    OModel md;
    or_model(s, &md);
    or_stage_terms(s, &md, x, terms);
}

void oracle_cost_dist(const OScene *s, const double *x, double *d) { or_cost_dist(s, x, d); }

int oracle_num_cost_pairs(const OScene *s) { return or_num_cost_pairs(s); }

/* batch of rollouts, parallel over samples */
void oracle_rollout_batch(const OScene *s, const double *x0, const double *U, int n, int H, double *costs,
                          double *final_states, int nthreads)
{
    OModel md;
    or_model(s, &md);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int j = 0; j < n; ++j) {
        double *traj = final_states ? (double *)malloc(sizeof(double) * OR_NX * (size_t)H) : NULL;
        costs[j] = or_rollout(s, &md, x0, U + (long)j * H * 14, H, traj, NULL);
        if (final_states) {
            memcpy(final_states + (long)j * OR_NX, traj + (long)(H - 1) * OR_NX, sizeof(double) * OR_NX);
            free(traj);
        }
    }
}

/* collision cost of a scripted distance sequence d[H][B] */
void oracle_collision_cost(const double *d, int H, int B, double gamma, double *out /* barrier, indicator */)
{
    out[0] = 0.0;
    out[1] = 0.0;
    for (int k = 0; k < H; ++k)
        collision_terms(k >= 1 ? d + (long)(k - 1) * B : NULL, d + (long)k * B, B, gamma, &out[0], &out[1]);
}

/* terms 7..16 at state x, term 9 as its squared summand (tests) */
void oracle_ext_terms(const OScene *s, const double *x, double *t) { ext_terms(s, x, t); }
