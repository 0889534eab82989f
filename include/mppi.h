/*
 * mppi.h -- C ABI of the MI355X (gfx950) MPPI rollout library.
 *
 * The library computes the data-parallel hot path of the sampling-based
 * bimanual planner of Hurova, Dan, Kruusamae and Singh, "Sampling-Based
 * Optimization with Parallelized Physics Simulator for Bimanual
 * Manipulation" (arXiv 2511.21264): K joint-velocity sequences are drawn
 * from N(nu, Sigma) and projected onto the velocity box (Alg. 1, sampling
 * and QP steps; Eqs. proj_cost/proj_bounds), rolled out through a
 * rigid-body world (Eq. state_evol; two 7-joint arms, a free ball, static
 * boxes, a table plane), scored by the ball-task cost (Sec. IV-B, with the
 * collision cost of Eq. collision_cost), and folded into the exponentially
 * weighted mean update (Eqs. mean_update, s_formula).
 *
 * Conventions shared by every call:
 *   * Return value: MPPI_OK (0) or a negative MPPI_E_* code; the message of
 *     the last failure on the calling thread is mppi_last_error().
 *   * Ownership: the caller owns every array.  With MPPI_DEVICE_PTRS in the
 *     flags, array arguments are device pointers on the context's device;
 *     otherwise they are host pointers and the library stages them.
 *     Scene handles own a device copy of the scene model; contexts own
 *     scratch buffers, which grow on demand.
 *   * Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls
 *     enqueue on it; with host pointers they also synchronize it before
 *     returning.  Device-pointer calls return once enqueued, except that
 *     mppi_plan synchronizes when `stats` is non-NULL (to fill it) or when
 *     MPPI_SYNC is set.  Calls on one context share its scratch buffers and
 *     run in call order whatever streams they name: a call on a stream other
 *     than the previous call's first makes its stream wait for the work the
 *     previous call enqueued (an event, no host synchronisation).
 *   * State layout (MPPI_NX = 55 floats): q[14], qd[14], q_des[14] (PD
 *     target), ball p[3], ball quaternion (w, x, y, z)[4], ball v[3], ball
 *     angular velocity (world frame)[3].  Joint order: arm 1 joints 1..7,
 *     arm 2 joints 1..7.  Controls are 14 joint velocities.
 *   * Calls on one context are not thread-safe; use one context per thread.
 */
#ifndef MPPI_H
#define MPPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPPI_OK 0
#define MPPI_E_INVAL (-1)    /* bad argument: NULL, K < 1, H < 1, lambda <= 0, sigma < 0, non-finite input */
#define MPPI_E_NOMEM (-2)    /* device allocation failed */
#define MPPI_E_MODEL (-3)    /* bad scene: non-positive mass/density/size, too many boxes */
#define MPPI_E_DIVERGED (-4) /* every sample non-finite in some iteration; U_new := nominal_U */
#define MPPI_E_DEVICE (-5)   /* a HIP runtime call failed */
#define MPPI_E_BUSY (-6)     /* admission refused (serving) */

#define MPPI_NU 14
#define MPPI_NX 55
#define MPPI_MAX_BOXES 16
#define MPPI_MAX_CONTACTS 8
#define MPPI_MAX_PAIRS (76 + 15 * MPPI_MAX_BOXES)
#define MPPI_MAX_K (1 << 20)
#define MPPI_MAX_H 4096
#define MPPI_NTERMS 17  /* cost terms per sample (see mppi_scene_desc and mppi_simulate) */

/* flags */
#define MPPI_DEVICE_PTRS 1u     /* array arguments are device pointers */
#define MPPI_SIGMA_PER_STEP 2u  /* sigma holds H x 14 values instead of 14 */
#define MPPI_SYNC 4u            /* synchronize the stream before returning */
#define MPPI_TIME_KERNELS 8u    /* time every rollout launch with HIP events (fills stats->rollout_ms) */
#define MPPI_TRAJ 16u           /* mppi_simulate: write every post-step state, not only the last */
#define MPPI_MAP_LANE 32u       /* rollout mapping: one lane per sample (throughput at large K) */
#define MPPI_MAP_TEAM 64u       /* rollout mapping: 16 lanes per sample, 4 samples per wave */
#define MPPI_MAP_WAVE 256u      /* rollout mapping: one wave per sample (short steps at small K);
                                   results equal MPPI_MAP_TEAM's bit for bit */
#define MPPI_MAP_SPLIT 2048u    /* rollout mapping: two waves per sample, dynamics and contact sweep /
                                   cost concurrently (shortest steps at small K); results equal
                                   MPPI_MAP_WAVE's bit for bit */
                                /* none of the four: the mapping mppi_autotune measured for K's size
                                   class on this context, else chosen from K (two waves per sample up
                                   to 1024 samples, one wave up to 2048, a team below 65536, one lane
                                   from there on).  In packed batches and served requests each request
                                   keeps the family of the mapping it would get alone (lane, or
                                   team/wave/split, which agree bit for bit), so its results do not
                                   depend on what it is batched with.  Scenes with a box object or the
                                   further cost terms run the same flags in their task forms (lane, or
                                   wave/split; MPPI_MAP_TEAM is refused; unpinned, one lane per sample
                                   from 16384 samples on) */
#define MPPI_FP32_WEIGHTS 512u  /* mppi_plan, mppi_update: the weights of Eq. s_formula, their sums and the
                                   weighted mean of Eq. mean_update in FP32 instead of FP64 (precision
                                   study; the default keeps them in FP64) */
#define MPPI_GRAPH 1024u        /* mppi_plan: run the plan's launch sequence (nu = nominal, then M x
                                   rollout, statistics, update) as a HIP graph captured on first use and
                                   replayed while shapes, scalars and device buffers stay the same (a
                                   small per-context cache); MPPI_TIME_KERNELS is then ignored */

#define MPPI_PER_STEP 4096u     /* mppi_plan and its variants: the plain form -- one rollout launch per
                                   control step (one sample per lane; state, previous control, cost
                                   sums and distance history carried in device memory between the
                                   launches), no graph; results equal MPPI_MAP_LANE's */

/* Global geom ids (pair tables and AABB arrays use them): 0 ball,
 * 1 table, 2 + 7*arm + g (g = 0..5 capsule of link g+1, g = 6 pad sphere on
 * link 7), 16 + b box b. */
#define MPPI_GEOM_BALL 0
#define MPPI_GEOM_TABLE 1
#define MPPI_GEOM_ARM 2
#define MPPI_GEOM_BOX 16

typedef struct mppi_ctx mppi_ctx;
typedef struct mppi_scene mppi_scene;

/* Scene description: plain data, copied by mppi_scene_create.
 * Arms: joint i+1 sits link_len[i] along link i's local z axis; joint i
 * rotates about local axis axes[i] (0 x, 1 y, 2 z); links 1..6 collide as
 * capsules of radius link_rad[i], link 7 as a pad sphere of radius pad_rad at
 * its tip; each link's inertia is a solid capsule of density[arm][i].  Arm
 * bases at base_pos with yaw given as (cos, sin), a unit pair (within 1e-6,
 * else MPPI_E_MODEL).  Ball: solid sphere.
 * Boxes: static, axis-aligned (centre, half extents).  Table: plane z = 0.
 * Physics (the paper fixes none of it; these are the world-model readings):
 * substep h, n_sub substeps per control step; PD actuators (kp, kd, clamp
 * tau_max) on an integrated position target, joint damping `damp`, rotor
 * `armature`; gravcomp = 1 removes gravity from the arms; contacts with
 * friction mu (4-edge pyramid), Baumgarte rate kappa, regularisation eps_r,
 * n_pgs Gauss-Seidel sweeps, at most n_cmax (<= MPPI_MAX_CONTACTS)
 * contacts.  Controls are clamped to |u| <= u_max.  Cost weights: goal
 * distance, end-effector-to-ball alignment, end-effector distance, planar
 * alignment, smoothness, collision; gamma of the barrier; m_c distance
 * saturation; eps = eps_frac * ball_r vertical grasp offset.
 * The free object: obj_box = 0 the ball (sphere of radius ball_r), 1 a solid
 * box of half extents obj_h (the tray of Sec. IV-A, the cube of Sec. IV-C;
 * mass ball_m; on the table up to four vertex contacts, against pads and
 * links computed in its frame, against static boxes by separating axes).
 * ext = 1 adds the further task-cost terms of Sec. IV (terms 7..16 of
 * mppi_simulate) with their weights and targets: joint deviation from
 * q_home (Eq. home_cost), vertical alignment (Eq. vertical_alignment_cost),
 * relative velocity (Eq. rel_vel_cost), per-arm end-effector position
 * targets apos (Eqs. tray_grasp_pos_cost, the hand-over's pick and place
 * costs), per-arm x targets ax_t (the hand-over's pass cost), per-arm
 * end-effector orientation targets arot (Eqs. tray_grasp_ori_cost,
 * tray_move_ori_cost, the ball's C_r, the hand-over's phase terms), the
 * object orientation target orot (Eq. tray_ori_cost); quaternions (w, x,
 * y, z), normalised here.  l_target > 0 replaces the ball's grasp width in
 * the end-effector distance term (l_tray).  The paper's task totals are
 * weightings of the 17 terms; the caller sets the phase's weights (w_pick /
 * w_move, the hand-over's per-arm phase weights) by choosing the scene.
 * Scenes with obj_box or ext run one lane, one wave or two waves per sample
 * (the last two bit for bit alike); a pinned MPPI_MAP_TEAM (four samples a
 * wave) is rejected with MPPI_E_INVAL. */
typedef struct mppi_scene_desc {
    double base_pos[2][3];
    double base_cs[2][2];
    int axes[7];
    double link_len[7], link_rad[7], density[2][7];
    double pad_rad;
    double ball_r, ball_m;
    int n_box;
    double box_c[MPPI_MAX_BOXES][3], box_h[MPPI_MAX_BOXES][3];
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
    int obj_box;
    double obj_h[3];
    int ext;
    double l_target;
    double q_home[14];
    double w_home, w_vert, w_relv, w_orot;
    double w_apos[2], w_ax[2], w_arot[2];
    double apos[2][3];
    double ax_t[2];
    double arot[2][4];
    double orot[4];
} mppi_scene_desc;

/* Plan options.  M iterations of Alg. 1; seed of the Philox stream; eta
 * learning rate of Eq. mean_update (1 = plain MPPI); n_elite elite-set size
 * (<= 0 or >= K: every sample). */
typedef struct mppi_opts {
    int M;
    uint64_t seed;
    double eta;
    int n_elite;
    unsigned flags;
} mppi_opts;

/* Statistics of a plan (filled after the stream completes). */
typedef struct mppi_stats {
    double ess;            /* effective sample size (sum w)^2 / sum w^2, last iteration */
    double c_min;          /* lowest finite cost, last iteration */
    int best;              /* sample index of c_min */
    int n_nonfinite;       /* samples with a non-finite cost, last iteration */
    int diverged;          /* 1 if some iteration had no finite sample */
    int iterations;
    double cmin_iter[64];  /* c_min per iteration (first 64) */
    double contacts;       /* total contacts over all substeps, all iterations */
    double np_tests;       /* narrowphase evaluations (contacts + cost distances) */
    double box_tests;      /* capsule-box evaluations among them */
    double overflow;       /* substeps whose contact list hit n_cmax */
    float rollout_ms;      /* summed rollout kernel time (MPPI_TIME_KERNELS) */
    int rollout_launches;
} mppi_stats;

/* Create a context on HIP device `device` (or -1 = current device).
 * Destroy the servers and scenes made on a context before the context:
 * their handles refer to it and are invalid once it is gone. */
int mppi_ctx_create(int device, mppi_ctx **out);
void mppi_ctx_destroy(mppi_ctx *ctx);
const char *mppi_last_error(void);

/* Validate `desc` and upload the derived model (link masses and inertias,
 * candidate-pair table in canonical order) to the context's device.
 * Errors: MPPI_E_INVAL (NULL), MPPI_E_MODEL (bad values), MPPI_E_NOMEM. */
int mppi_scene_create(mppi_ctx *ctx, const mppi_scene_desc *desc, mppi_scene **out);
void mppi_scene_destroy(mppi_scene *scene);
/* Number of candidate pairs and of collision-cost pairs of a scene. */
int mppi_scene_num_pairs(const mppi_scene *scene, int *n_pairs, int *n_cost_pairs);

/* One MPPI plan (Alg. 1, M iterations from the same x0).
 *   x0[MPPI_NX]: start state; nominal_U[H][14]: initial mean nu_0 (warm start);
 *   K samples, horizon H; lambda: temperature (beta of Eq. s_formula);
 *   sigma[14] (or [H][14] with MPPI_SIGMA_PER_STEP): per-joint standard
 *   deviation of the diagonal covariance;
 *   U_new[H][14]: receives nu_M; costs[K]: the last iteration's costs
 *   (+INF for non-finite rollouts); stats: optional.
 * Errors: MPPI_E_INVAL, MPPI_E_NOMEM, MPPI_E_DEVICE, MPPI_E_DIVERGED (only
 * reported when the call synchronizes; U_new then holds nominal_U). */
int mppi_plan(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
              double lambda, const float *sigma, const mppi_opts *opts, float *U_new, float *costs,
              mppi_stats *stats, void *stream);

/* Bytes of the static device array that serves as mppi_plan_noalloc's
 * working memory (one copy per GPU, held until the process ends). */
#define MPPI_NOALLOC_SCRATCH_BYTES (8u << 20)

/* mppi_plan for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc.  The
 * same plan as mppi_plan (same kernels, bit-identical U_new, costs and
 * stats), but its working memory -- the mean, weights, statistics record,
 * per-sample counters, the collision-distance history and, when costs is
 * NULL, the costs -- lives in a file-scope device array of
 * MPPI_NOALLOC_SCRATCH_BYTES per GPU, whose address the library looks up
 * once per device when a context is created.  It calls no hipMalloc,
 * hipFree or other allocating routine.
 *   Arguments as mppi_plan; every array is a device pointer (MPPI_DEVICE_PTRS
 *   must be set); MPPI_GRAPH and MPPI_TIME_KERNELS are rejected.
 *   Size limit: 256-byte aligned pieces of sizeof(stats record) + 56 H +
 *   K (8 + 16 + 4 n_cost + 4) bytes must fit (n_cost = 49 + 14 boxes:
 *   about K <= 21000 at H = 64 with 3 boxes, K <= 7400 with 16 boxes);
 *   larger calls return MPPI_E_INVAL with the sizes in the message.
 *   The array is shared by every call on that GPU and keeps the last call's
 *   contents (the statistics record is cleared by a kernel at the start of
 *   each call): calls on one context run in call order (see Streams above),
 *   but calls from different contexts or threads that overlap on one GPU
 *   race on it.
 * Errors: as mppi_plan (MPPI_E_DIVERGED only when the call synchronizes,
 * i.e. with stats or MPPI_SYNC). */
int mppi_plan_noalloc(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                      double lambda, const float *sigma, const mppi_opts *opts, float *U_new, float *costs,
                      mppi_stats *stats, void *stream);

/* One request of a packed batch. */
typedef struct mppi_request {
    const mppi_scene *scene;  /* scene of this request (same context) */
    const float *x0;          /* [MPPI_NX] */
    const float *nominal_U;   /* [H][14] */
    int K, H;
    double lambda;
    const float *sigma;       /* [14], or [H][14] with MPPI_SIGMA_PER_STEP in opts.flags */
    mppi_opts opts;           /* M, seed, eta, n_elite; of the flags only MPPI_SIGMA_PER_STEP is read */
    float *U_new;             /* [H][14] out */
    float *costs;             /* [K] out, nullable */
    mppi_stats *stats;        /* out, nullable */
    int status;               /* out: MPPI_OK or MPPI_E_DIVERGED */
} mppi_request;

/* Uneven batch: n independent plans (different scenes, K, H, M) packed so
 * that each MPPI iteration is one rollout launch over every request's
 * samples, one statistics launch and one update launch (requests with fewer
 * iterations drop out of later launches).  `flags`: MPPI_DEVICE_PTRS (every
 * array of every request is a device pointer), MPPI_MAP_LANE/_TEAM/_WAVE
 * (one mapping for the whole batch; chosen from the total sample count
 * otherwise), MPPI_TIME_KERNELS (each request's stats->rollout_ms receives the
 * batch's summed rollout time).  Results of a request equal its results
 * planned alone with the same mapping, bit for bit.  Synchronizes `stream`
 * before returning.  Returns MPPI_OK when the batch ran (per-request status
 * reports divergence), or MPPI_E_INVAL / MPPI_E_NOMEM / MPPI_E_DEVICE. */
int mppi_plan_batch(mppi_ctx *ctx, int n, mppi_request *reqs, unsigned flags, void *stream);

/* Roll out explicit control sequences (Alg. 1 rollout and cost steps).
 *   X0: [n][MPPI_NX] start states (one per sample), or one state shared by
 *   all samples when x0_shared != 0; U[n][H][14] controls (used as given,
 *   not clamped); n_sub: substeps per control step (<= 0: the scene's);
 *   costs[n] (nullable); terms[n][MPPI_NTERMS] (nullable): unweighted sums
 *   of the cost terms (goal, eef-obj, distance, planar, smooth, barrier,
 *   indicator, then with ext: joint deviation, vertical alignment, relative
 *   velocity (the root of its summed squares), position of arm 1 / arm 2, x
 *   of arm 1 / arm 2, orientation of arm 1 / arm 2, object orientation; zero
 *   without ext);
 *   X_out: [n][MPPI_NX] final states, or [n][H][MPPI_NX] with MPPI_TRAJ
 *   (nullable). */
int mppi_simulate(mppi_ctx *ctx, const mppi_scene *scene, const float *X0, int x0_shared, const float *U, int n,
                  int H, int n_sub, float *costs, float *terms, float *X_out, unsigned flags, void *stream);

/* The sampled, projected controls of iteration m:
 *   U[K][H][14] = clamp(nu + sigma * z, +-u_max) with z the Philox normals
 *   (z_out[K][H][14] nullable); words_out[K][H][16] (nullable) receives the
 *   raw Philox4x32-10 words of counters (j, k, q, m), q = 0..3, key = seed. */
int mppi_sample(mppi_ctx *ctx, const mppi_scene *scene, const float *nu, const float *sigma, uint64_t seed, int m,
                int K, int H, float *U, float *z_out, uint32_t *words_out, unsigned flags, void *stream);

/* The update of Eq. mean_update from given costs: the samples of iteration m
 * are regenerated from (nu_in, sigma, seed); nu_out[H][14] (float) and
 * nu_out64 (nullable, double) receive (1 - eta) nu + eta sum_j w_j u_j with
 * w_j from Eq. s_formula over the n_elite lowest finite costs; weights[K]
 * (nullable, double) the normalized weights.  Returns MPPI_E_DIVERGED (and
 * nu_out = nu_in) when no cost is finite. */
int mppi_update(mppi_ctx *ctx, const mppi_scene *scene, const float *costs, const float *nu_in,
                const float *sigma, uint64_t seed, int m, int K, int H, double lambda, double eta, int n_elite,
                float *nu_out, double *nu_out64, double *weights, mppi_stats *stats, unsigned flags,
                void *stream);

/* ------------------------------------------------------------ QP smoothing
 * Alg. 1's sampling step followed by its QP based smoothing: every sampled
 * sequence is projected onto the bounds of Eq. proj_bounds on the joint
 * trajectory and its first three derivatives, with the objective of Eq.
 * proj_cost.  Each joint is one QP over the horizon in the H control-step
 * velocities v_0..v_{H-1} (dt = n_sub * h):
 *   r = 0: q_des0 + dt (v_0 + .. + v_k) in [pos_lo, pos_hi], q_des0 the
 *          commanded joint position of the start state;
 *   r = 1: |v_k| <= u_max (the scene's velocity box);
 *   r = 2: |v_k - v_{k-1}| <= acc_max dt, k >= 1;
 *   r = 3: |v_k - 2 v_{k-1} + v_{k-2}| <= jerk_max dt^2, k >= 2.
 * Solver: `iters` iterations of ADMM with penalty rho and over-relaxation
 * alpha on the stacked operator [I; D1; D2; prefix sums], started from
 * z = clip(A v~), w = 0; the result is clipped to the velocity box (r = 1
 * holds exactly, the other bounds to the solver's accuracy).  H <= 128. */
typedef struct mppi_qp {
    double pos_lo[14], pos_hi[14]; /* commanded-position bounds per joint (rad) */
    double acc_max;                /* rad/s^2 */
    double jerk_max;               /* rad/s^3 */
    double rho;                    /* ADMM penalty, > 0 */
    double alpha;                  /* over-relaxation, in (0, 2) */
    int iters;                     /* ADMM iterations, 1..10000 */
} mppi_qp;

/* Project U_in[K][H][14] into U_out[K][H][14] (the same array is allowed).
 *   X0: [K][MPPI_NX] start states (their commanded positions q_des), or one
 *   state for every sample when x0_shared != 0.  flags: MPPI_DEVICE_PTRS,
 *   MPPI_SYNC.  Errors: MPPI_E_INVAL (NULL, K < 1, H < 1 or H > 128, bad qp
 *   values), MPPI_E_NOMEM, MPPI_E_DEVICE. */
int mppi_project(mppi_ctx *ctx, const mppi_scene *scene, const float *X0, int x0_shared, const float *U_in,
                 float *U_out, int K, int H, const mppi_qp *qp, unsigned flags, void *stream);

/* mppi_plan with the QP smoothing of every sample: in each iteration the
 * samples nu + sigma * z (the Philox normals of mppi_sample, not clamped)
 * are projected as by mppi_project, rolled out as given, and the update of
 * Eq. mean_update averages the projected samples.  Arguments and errors as
 * mppi_plan, plus qp (H <= 128).  MPPI_GRAPH is ignored. */
int mppi_plan_qp(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                 double lambda, const float *sigma, const mppi_opts *opts, const mppi_qp *qp, float *U_new,
                 float *costs, mppi_stats *stats, void *stream);

/* mppi_plan that also returns the best sequence: U_best[H][14] receives the
 * lowest-cost sample of the final iteration (Alg. 1 returns it with nu_M),
 * or that iteration's mean when no sample had a finite cost.  U_best lives
 * on the same side as U_new.  Arguments, flags and errors as mppi_plan
 * (MPPI_GRAPH is ignored). */
int mppi_plan_best(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                   double lambda, const float *sigma, const mppi_opts *opts, float *U_new, float *U_best, float *costs,
                   mppi_stats *stats, void *stream);

/* ----------------------------------------------- closed-loop ball transport
 * Receding-horizon execution of the planner on the ball task (the pick and
 * move phases of Sec. IV-B; the experiments' success metric).  Replan r:
 * plan from the plant state with the phase's scene (`pick`: a scene whose
 * object-to-target weight is 0; `move`: every term), seed opts->seed + r,
 * warm-started with the previous mean shifted by n_exec control steps (the
 * last row repeated); average the first n_avg steps of the best sequence
 * and execute that command for n_exec control steps in the simulator (the
 * plant, with the physics of `move`).  After every executed step, in order:
 *   an arm-arm or arm-box pair at negative distance -> failure (collision);
 *   pick -> move once |pad midpoint - (p_ball - (0,0,eps))| < grasp_tol and
 *     | |p1 - p2| - l_ball | < width_tol;
 *   in move: the ball above lift_z marks it lifted; lifted and below drop_z
 *     -> failure (fallen); |p_ball - goal| < goal_tol -> success;
 *   simulated time >= t_max -> failure (timeout).
 * qp (nullable): every replan's samples are smoothed as by mppi_plan_qp
 * (H <= 128) before their rollouts.
 * Host arrays only (x0[MPPI_NX], sigma, x_final[MPPI_NX] nullable; u_exec
 * [max_replans][14] and x_hist[max_replans][MPPI_NX], nullable, receive each
 * replan's executed command and the state after its execution and need
 * max_replans > 0).  opts: M, seed, eta, n_elite, sigma-per-step and mapping
 * flags.  Errors: MPPI_E_INVAL, and those of mppi_plan_best and
 * mppi_simulate. */
typedef struct mppi_episode_opts {
    int n_avg;        /* leading steps of the best sequence averaged, 1..H */
    int n_exec;       /* control steps the averaged command runs, 1..H */
    int max_replans;  /* cap on replans (0: until an outcome) */
    int use_cov;      /* 1: plan with the full covariance (mppi_plan_cov), warm-started with Sigma_M shifted like
                         the mean (the freed tail: diag(sigma^2), no cross-covariance); opts->eta in (0, 1] */
    double grasp_tol, width_tol, goal_tol; /* m */
    double lift_z, drop_z;                 /* m */
    double t_max;                          /* s */
    double cov_eps;                        /* eps of the covariance update when use_cov */
} mppi_episode_opts;

typedef struct mppi_episode_result {
    int status;     /* 1 success, -1 collision, -2 timeout, -3 ball fell, 0 replan cap reached first */
    int phase;      /* 0 pick, 1 move, at the end */
    int n_replans;
    int n_steps;    /* executed control steps */
    double t_end;   /* simulated time at the end (s): the task time of a success */
    double t_switch; /* simulated time of the pick -> move switch, -1 if none */
    double t_comp_mean_ms, t_comp_std_ms, t_comp_max_ms; /* wall time per replan (synchronised plan call) */
    double goal_dist_min; /* closest approach of the ball to the goal (m) */
    double ball_final[3];
    int n_diverged; /* replans in which no sample had a finite cost */
    int pad2;
} mppi_episode_result;

int mppi_episode(mppi_ctx *ctx, const mppi_scene *pick, const mppi_scene *move, const float *x0, int K, int H,
                 double lambda, const float *sigma, const mppi_opts *opts, const mppi_episode_opts *eo,
                 const mppi_qp *qp, float *x_final, float *u_exec, float *x_hist, mppi_episode_result *res,
                 void *stream);

/* --------------------------------------------------- covariance adaptation
 * Alg. 1 samples from N(nu_m, Sigma_m) with a full covariance over the whole
 * sequence and updates it by Eq. cov_update.  A sequence is the vector of
 * its n = 14 H joint velocities in step-major order (index 14 k + d, the
 * [H][14] layout flattened); Sigma is n x n, row-major, double.
 *   samples:  u_j = clip(nu_m + L_m z_j, +-u_max), L_m the lower Cholesky
 *             factor of Sigma_m, z_j[14 k + d] the Philox normals of
 *             mppi_sample (so a diagonal Sigma gives mppi_sample's samples);
 *   update:   Sigma_{m+1} = (1 - eta) Sigma_m + eta Delta Sigma + eps I,
 *             Delta Sigma = sum_j w_j (u_j - nu_{m+1})(u_j - nu_{m+1})^T
 *             / sum_j w_j over the weights of Eq. s_formula (elite set), about
 *             the updated mean nu_{m+1}; eps >= 0 keeps Sigma positive
 *             definite when few samples carry weight (the paper adds none).
 *             With no positive weight (no finite cost) Sigma is kept.
 * n <= MPPI_COV_MAX_N. */
#define MPPI_COV_MAX_N 3584
#define MPPI_E_NOTPD (-8) /* Cholesky: a pivot is not positive (Sigma not positive definite) */

typedef struct mppi_cov {
    const double *Sigma0; /* [n][n] Sigma_0, or NULL: diag(sigma^2) from the sigma argument */
    double *Sigma_out;    /* [n][n] receives Sigma_M (nullable; may be Sigma0) */
    double eps;           /* >= 0, added to the diagonal after every update */
    float *U_best;        /* [H][14] receives the best sequence of the final iteration (nullable) */
} mppi_cov;

/* Sigma_out = (1 - eta) Sigma_in + eta Delta Sigma + eps I from the samples
 * U[K][n] (float), weights w[K] (double, >= 0, any scale: divided by their
 * sum) and nu_new[n] (double).  Only the lower triangle of Sigma_in is read;
 * Sigma_out is written whole and may be Sigma_in.  flags: MPPI_DEVICE_PTRS,
 * MPPI_SYNC.  Errors: MPPI_E_INVAL (NULL, K < 1, n < 1 or n > MPPI_COV_MAX_N,
 * eta or eps out of range, negative or non-finite weights in host arrays),
 * MPPI_E_NOMEM, MPPI_E_DEVICE. */
int mppi_cov_update(mppi_ctx *ctx, const float *U, const double *w, const double *nu_new, const double *Sigma_in,
                    double eta, double eps, double *Sigma_out, int K, int n, unsigned flags, void *stream);

/* L (n x n, double, upper triangle zeroed) with L L^T = Sigma; only the
 * lower triangle of Sigma is read and L may be Sigma.  Synchronises the
 * stream.  Errors: MPPI_E_NOTPD (the message names the first failing
 * column; L is then not a factor), MPPI_E_INVAL, MPPI_E_NOMEM,
 * MPPI_E_DEVICE. */
int mppi_cholesky(mppi_ctx *ctx, const double *Sigma, double *L, int n, unsigned flags, void *stream);

/* U[K][H][14] = clip(nu + L z_j, +-u_max) for iteration m of `seed`, with
 * L (n x n, n = 14 H, double, lower triangle read) and nu[H][14] (float);
 * the product runs in single precision.  Errors: MPPI_E_INVAL,
 * MPPI_E_NOMEM, MPPI_E_DEVICE. */
int mppi_sample_full(mppi_ctx *ctx, const float *nu, const double *L, uint64_t seed, int m, int K, int H,
                     float u_max, float *U, unsigned flags, void *stream);

/* mppi_plan with the full covariance: in each iteration Sigma_m is factored,
 * the samples clip(nu_m + L_m z_j) are drawn (and smoothed as by
 * mppi_project when qp is not NULL), rolled out and weighted; nu and Sigma
 * are updated with opts->eta (0 < eta <= 1).  cov->Sigma0 and
 * cov->Sigma_out follow MPPI_DEVICE_PTRS like the other arrays.  Arguments
 * and errors as mppi_plan, plus MPPI_E_NOTPD (some Sigma_m could not be
 * factored) and n = 14 H <= MPPI_COV_MAX_N.  MPPI_GRAPH is ignored. */
int mppi_plan_cov(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                  double lambda, const float *sigma, const mppi_opts *opts, const mppi_cov *cov, const mppi_qp *qp,
                  float *U_new, float *costs, mppi_stats *stats, void *stream);

/* ---------------------------------------------------------------- serving
 * A server replans for many robot cells at once by continuous batching:
 * a worker thread runs MPPI iterations over every active request in one
 * packed launch sequence (one rollout, one statistics and one update
 * launch per iteration, as mppi_plan_batch), admits queued requests at
 * every iteration boundary as active slots and device memory free up, and
 * retires requests as their last iteration completes.  Each request is the
 * plan of Alg. 1 with its own (scene, x0, nominal, K, H, lambda, sigma,
 * opts); with a pinned mapping (MPPI_MAP_LANE, _TEAM or _WAVE in the
 * server flags) its results equal mppi_plan of the same arguments and
 * mapping, bit for bit, whatever else is in flight.
 *
 * Cells keep a scene, the plant state and the warm-start nominal controls
 * resident on the device (the receding-horizon warm start of Sec. III-A):
 * a request for a cell may take x0 and nominal_U from it, and on
 * completion writes U_new back as the cell's nominal, shifted by `advance`
 * control steps (the tail repeats the last row), after advancing the cell's
 * state by the first `advance` steps of U_new in the same world model.
 * Requests of one cell run one after another, in submission order.
 *
 * Thread safety: mppi_submit, mppi_poll, mppi_cancel and mppi_cell_* may be
 * called from any thread; the server serialises them.  The context must not
 * be used by other calls while a server on it is alive (the server owns the
 * context's device for its worker). */
typedef struct mppi_server mppi_server;

#define MPPI_PENDING 1          /* mppi_poll: not finished yet */
#define MPPI_E_CANCELLED (-7)   /* request status after mppi_cancel or supersession */
#define MPPI_E_LATE (-9)        /* request status: shed unrun, it could not end by its deadline */

#define MPPI_SUPERSEDE 128u     /* submit: cancel this cell's requests still queued (not yet admitted) */

typedef struct mppi_server_opts {
    uint64_t mem_budget;  /* device bytes for in-flight requests (0: 1 GiB) */
    int max_active;       /* requests iterating together (0: 256; at most 4096) */
    int max_pending;      /* queued requests; mppi_submit returns MPPI_E_BUSY beyond (0: 4096) */
    unsigned flags;       /* MPPI_MAP_LANE, _TEAM, _WAVE or _SPLIT: mapping of every launch (else each
                             request keeps the family of the mapping it would get alone) */
    /* Deadlines (the control period of the replanning cells).  deadline_ms > 0:
     * every request must end within deadline_ms of its submission.  The queue
     * is then served earliest deadline first; a request is admitted only when
     * the predicted end of its M iterations (plus the packed iteration in
     * flight), at the load it would join, is within its deadline and no
     * active request predicted on time would become late (otherwise it waits
     * and nothing overtakes it); a queued request that cannot end in time even
     * alone is shed (status MPPI_E_LATE).  The prediction of one packed
     * iteration is max(floor, iter_base_ms + iter_ms_per_menv * W / 1e6), W
     * the sum of K * H over the active requests: the values given here (floor
     * 0) until 8 packed iterations have been measured, then a fit to the last
     * 64 measured (floor: the fastest; base and slope: least squares); every
     * predicted end adds a margin learned from past predictions (see
     * mppi_server_info). */
    double deadline_ms;
    double iter_base_ms;
    double iter_ms_per_menv;
} mppi_server_opts;

typedef struct mppi_ticket_info {
    int status;           /* MPPI_OK, MPPI_E_DIVERGED, MPPI_E_CANCELLED or MPPI_E_LATE */
    int iterations;       /* iterations run */
    double t_submit_ms;   /* host steady clock, ms since the server was created */
    double t_admit_ms;    /* admitted into the active set (negative if never) */
    double t_done_ms;     /* completion observed by the worker */
    double t_deadline_ms; /* t_submit_ms + deadline_ms (infinite without a deadline) */
} mppi_ticket_info;

typedef struct mppi_server_info {
    uint64_t submitted, completed, cancelled, superseded, rejected;
    uint64_t iterations;        /* packed iterations launched */
    uint64_t request_iters;     /* sum over iterations of the active requests */
    uint64_t env_steps;         /* sum of K * H over request iterations */
    uint64_t mem_high_water;    /* device bytes */
    int active, pending;
    uint64_t shed;              /* requests dropped unrun because they could not end by their deadline */
    uint64_t late;              /* requests completed after their deadline */
    double model_base_ms, model_ms_per_menv, model_floor_ms;  /* the iteration model in use */
    double model_margin_ms;     /* added to predicted ends: the 95th percentile of how late the recent
                                   completions came against their predictions (16 to 128 of them) */
} mppi_server_info;

/* Create a server on `ctx` with its own non-blocking stream and worker
 * thread; the device arena (opts->mem_budget bytes) and a pinned host
 * arena of the same bound for staging are allocated here, once.
 * Errors: MPPI_E_INVAL, MPPI_E_NOMEM, MPPI_E_DEVICE. */
int mppi_server_create(mppi_ctx *ctx, const mppi_server_opts *opts, mppi_server **out);
/* Cancel everything queued or running, join the worker, free the server. */
void mppi_server_destroy(mppi_server *srv);

/* A cell: scene (not owned; must outlive the server), horizon H, start
 * state x0[MPPI_NX] (host), initial nominal[H][14] (host, NULL = zeros).
 * Returns the cell id in *cell. */
int mppi_cell_create(mppi_server *srv, const mppi_scene *scene, int H, const float *x0, const float *nominal_U,
                     int *cell);
/* Copy a cell's resident state and nominal to host arrays (each nullable),
 * after waiting until none of its requests is queued or running. */
int mppi_cell_read(mppi_server *srv, int cell, float *x, float *nominal_U);

/* Queue one request; *ticket identifies it.
 *   cell < 0: a stand-alone request; every field of *req is used as in
 *     mppi_plan_batch (inputs copied at submission when host pointers;
 *     device pointers, with MPPI_DEVICE_PTRS in req->opts.flags, must stay
 *     valid and unchanged until the request is done).
 *   cell >= 0: req->scene is NULL or the cell's scene, req->H is 0 or the
 *     cell's H; req->x0 == NULL takes the cell's state and
 *     req->nominal_U == NULL the cell's nominal; `advance` in [0, H].
 *   Outputs (U_new, costs, stats; each nullable for cell requests) are
 *   written when the request completes and must stay valid until
 *   mppi_poll reports it done.  `flags`: MPPI_SUPERSEDE.
 * Errors: MPPI_E_INVAL, MPPI_E_BUSY (queue full or the request can never
 * fit in the memory budget). */
int mppi_submit(mppi_server *srv, const mppi_request *req, int cell, int advance, unsigned flags,
                uint64_t *ticket);
/* Wait up to timeout_ms (0: do not wait, < 0: no limit) for a request.
 * Returns MPPI_OK once it is done (info filled, ticket released),
 * MPPI_PENDING while it is not, MPPI_E_INVAL for an unknown ticket. */
int mppi_poll(mppi_server *srv, uint64_t ticket, int timeout_ms, mppi_ticket_info *info);
/* Cancel a request: a queued one is dropped at once, a running one at the
 * next iteration boundary (its outputs are not written).  Its status
 * becomes MPPI_E_CANCELLED; it must still be polled.  MPPI_E_INVAL for an
 * unknown or finished ticket. */
int mppi_cancel(mppi_server *srv, uint64_t ticket);
/* Counters of the server since creation. */
int mppi_server_query(mppi_server *srv, mppi_server_info *info);

/* Autotuner of the sample-to-lane mapping: times one rollout launch of K
 * samples over H control steps of `scene` (from state x0[MPPI_NX], mean 0,
 * sigma[14]; host arrays) with each mapping (lane, team, wave, split; best of two
 * after a warm-up launch) and records the fastest for K's size class
 * (ceil(log2 K)) in the context.  Later calls on the context that pin no
 * mapping use the recorded one for that class.  *mapping (nullable)
 * receives the MPPI_MAP_* flag chosen, ms[4] (nullable) the times of the
 * lane, team, wave and split launches.  Synchronous; uses a private stream
 * that first waits for the context's previous call (whose scratch it reuses). */
int mppi_autotune(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *sigma, int K, int H,
                  int *mapping, float *ms);

/* Broadphase of the contact pass: for every candidate pair of the scene
 * (canonical order), flags[p] = 1 when the closed AABBs of its geoms
 * overlap after growing geom A's box by `margin`.  lo/hi: [n][16 + n_box][3]
 * AABBs (geom ids above); flags: [n][n_pairs]. */
int mppi_broadphase(mppi_ctx *ctx, const mppi_scene *scene, const float *lo, const float *hi, int n, float margin,
                    int *flags, unsigned flags_in, void *stream);

/* Narrowphase of every candidate pair at states X[n][MPPI_NX]: phi[n][P],
 * normal[n][P][3] (from geom B to geom A), point[n][P][3]; and the geom
 * AABBs lo/hi[n][16 + n_box][3] (nullable).  With a box-shaped object its
 * pair with the table reports the deepest vertex (the lowest index on ties)
 * and its AABB is that of the rotated box. */
int mppi_narrowphase(mppi_ctx *ctx, const mppi_scene *scene, const float *X, int n, float *phi, float *normal,
                     float *point, float *lo, float *hi, unsigned flags, void *stream);

#ifdef __cplusplus
}
#endif
#endif
