/*
 * FP64 CPU oracle for the bimanual MPPI hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct reference of what the GPU path computes:
 * Gaussian sampling of joint-velocity sequences (Alg. 1, sampling step),
 * projection onto the velocity box (Eqs. proj_cost/proj_bounds with only
 * velocity bounds), rollouts through a rigid-body world (Eq. state_evol),
 * the ball-task cost (Sec. IV-B) and the MPPI update (Eqs. mean_update,
 * s_formula).  The paper delegates the world model to MuJoCo; every physics
 * constant and rule here is a stated reading (see the module docstring of
 * the Python wrapper for the list).  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code with the HIP library.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#define OR_NJ 7
#define OR_NDOF 20       /* arm0 7 | arm1 7 | ball v(3) w(3) */
#define OR_MAXBOX 16
#define OR_MAXCON 64
#define OR_NX 55

/* scene: plain data, marshalled by the Python wrapper */
typedef struct {
    double base_pos[2][3];
    double base_cs[2][2];
    int axes[OR_NJ];
    double link_len[OR_NJ], link_rad[OR_NJ], density[2][OR_NJ];
    double pad_rad;
    double ball_r, ball_m, ball_p0[3];
    int n_box;
    double box_c[OR_MAXBOX][3], box_h[OR_MAXBOX][3];
    double goal[3];
    double h;
    int n_sub;
    double kp, kd, damp, armature, tau_max;
    int gravcomp;
    double g;
    double mu, kappa, eps_r;
    int n_pgs, n_cmax;
    double u_max;
    double w_goal, w_eo, w_l, w_yz, w_s, w_c, gamma, m_c, eps_frac;
    /* free object: 0 a sphere of radius ball_r, 1 a solid box of half extents
     * obj_h (the tray of Sec. IV-A, the cube of Sec. IV-C); mass ball_m */
    int obj_box;
    double obj_h[3];
    /* the further cost terms of Sec. IV (terms 7..16 of or_rollout), evaluated
     * when ext != 0: weights and targets */
    int ext;
    double l_target;          /* end-effector distance target; <= 0: l_ball */
    double q_home[14];
    double w_home, w_vert, w_relv, w_orot;
    double w_apos[2], w_ax[2], w_arot[2];
    double apos[2][3];        /* per-arm end-effector position targets */
    double ax_t[2];           /* per-arm x targets (hand-over pass) */
    double arot[2][4];        /* per-arm end-effector orientation targets (w, x, y, z) */
    double orot[4];           /* object orientation target */
} OScene;

#define OR_NTERMS 17

/* derived model quantities */
typedef struct {
    double m[2][OR_NJ], Ix[2][OR_NJ], Iz[2][OR_NJ];
    double ball_I;
    double obj_I[3];  /* principal inertias of the object about its centre (body frame) */
    double eps, l_ball;
} OModel;

/* kinematics of one arm in the world frame */
typedef struct {
    double R[OR_NJ][3][3]; /* link frames */
    double o[OR_NJ + 1][3]; /* joint origins o[0..6], tip o[7] */
    double a[OR_NJ][3];    /* joint axes (world) */
    double c[OR_NJ][3];    /* link centres of mass */
} OArmKin;

/* one contact: geoms A (first of the pair) and B */
typedef struct {
    int pair;       /* index in the canonical pair list */
    int ga, gb;     /* global geom ids */
    double phi;     /* signed distance */
    double n[3];    /* unit normal, from B towards A */
    double p[3];    /* contact point */
} OContact;

/* global geom ids */
#define OG_BALL 0
#define OG_TABLE 1
#define OG_ARM 2      /* 2 + 7*arm + g, g = 0..5 capsules, 6 = pad sphere */
#define OG_BOX 16     /* 16 + b */

/* model.c */
void or_model(const OScene *s, OModel *md);
void or_fk(const OScene *s, int arm, const double *q7, OArmKin *k);
void or_mass_matrix(const OScene *s, const OModel *md, int arm, const OArmKin *k, double M[OR_NJ][OR_NJ]);
void or_rnea(const OScene *s, const OModel *md, int arm, const OArmKin *k, const double *qd,
             const double *qdd, int gravity, double *tau);
int or_cholesky(int n, const double *A, double *L);
void or_chol_solve(int n, const double *L, const double *b, double *x);

/* collide.c */
int or_num_pairs(const OScene *s);
void or_pair(const OScene *s, int idx, int *ga, int *gb);
int or_num_cost_pairs(const OScene *s);
int or_cost_pair_index(const OScene *s, int i);
void or_geom_shape(const OScene *s, const OArmKin kin[2], const double *pball, int gid,
                   int *type, double P0[3], double P1[3], double *r);
int or_narrow(const OScene *s, const OArmKin kin[2], const double *pball, int ga, int gb,
              double *phi, double n[3], double p[3]);
void or_aabb(const OScene *s, const OArmKin kin[2], const double *pball, int gid, double lo[3], double hi[3]);
int or_contacts(const OScene *s, const OArmKin kin[2], const double *pball, OContact *out, int cap);
double or_seg_box_tstar(const double A[3], const double B[3], const double c[3], const double hh[3]);

/* object.c */
void or_quat_to_R(const double q[4], double R[3][3]);
void or_R_to_quat(const double R[3][3], double q[4]);
double or_quat_angle(const double q[4], const double Q[4]);
int or_obj_table(const OScene *s, const double *xo, double phi[8], double n[8][3], double p[8][3]);
void or_obj_narrow(const OScene *s, const double *xo, int tb, const double B0[3], const double B1[3], double rb,
                   double *phi, double n[3], double p[3]);

/* step.c */
void or_point_jac(const OScene *s, const OArmKin kin[2], const double *pball, int gid, const double p[3],
                  double J[3][OR_NDOF], double sign);
void or_substep(const OScene *s, const OModel *md, const double *x, const double *u, double *xn,
                int *ncon_out);
void or_tangents(const double n[3], double t1[3], double t2[3]);

/* cost.c */
void or_stage_terms(const OScene *s, const OModel *md, const double *x, double terms[4]);
void or_cost_dist(const OScene *s, const double *x, double *d);
double or_rollout(const OScene *s, const OModel *md, const double *x0, const double *U, int H,
                  double *traj, double *terms_out);

/* philox.c */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_normals14(uint64_t seed, uint32_t j, uint32_t k, uint32_t m, double z[14]);

#endif
