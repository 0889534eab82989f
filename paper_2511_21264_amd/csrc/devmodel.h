// Scene model as the kernels see it: FP32 constants derived on the host from
// mppi_scene_desc (link masses and inertias, combined diagonal terms, the
// candidate-pair table in canonical order).  One copy per scene lives in
// device memory; every lane of a launch reads the same words, so the loads
// go through the scalar cache.
#pragma once
#include <stdint.h>

#include "../../include/mppi.h"

namespace mppi {

constexpr int NJ = 7;
constexpr int NU = MPPI_NU;
constexpr int NX = MPPI_NX;
constexpr int MAXBOX = MPPI_MAX_BOXES;
constexpr int MAXPAIR = MPPI_MAX_PAIRS;
constexpr int MAXCOST = 49 + 14 * MAXBOX;
constexpr int NTERMS = MPPI_NTERMS;

// state offsets
constexpr int XQ = 0, XQD = 14, XQDES = 28, XPB = 42, XQUAT = 45, XVB = 49, XWB = 52;

// geom ids
constexpr int G_BALL = MPPI_GEOM_BALL, G_TABLE = MPPI_GEOM_TABLE, G_ARM = MPPI_GEOM_ARM, G_BOX = MPPI_GEOM_BOX;

struct DevModel {
    float base_pos[2][3];
    float base_cs[2][2];
    int axes[NJ];
    float link_len[NJ], link_rad[NJ];
    float m[2][NJ], Ix[2][NJ], Iz[2][NJ];
    float pad_rad;
    float ball_r, ball_m, inv_ball_m, inv_ball_I;
    int n_box;
    float box_c[MAXBOX][3], box_h[MAXBOX][3];
    float h;
    int n_sub;
    float kp, kd, damp, tau_max, diag_add;  // diag_add = armature + h (kd + damp)
    int gravcomp;
    float g;
    float mu, kappa_h, eps_r;  // kappa_h = kappa / h
    int n_pgs, n_cmax;
    float u_max;
    float goal[3];
    float w_goal, w_eo, w_l, w_yz, w_s, w_c, one_m_gamma, m_c, eps, l_ball;
    int n_pairs, cost_first, n_cost;
    uint8_t pa[MAXPAIR], pb[MAXPAIR];
    // the free object as a box (obj_box): half extents, principal inertias
    // and their inverses (body frame); ext: the further task-cost terms;
    // task_form: either of them (the scene runs in the task forms)
    int obj_box, ext, task_form;
    float obj_h[3], obj_I[3], obj_iI[3];
    float l_cost;  // end-effector distance target of the cost (l_target or l_ball)
    float q_home[14];
    float w_home, w_vert, w_relv, w_orot;
    float w_apos[2], w_ax[2], w_arot[2];
    float apos[2][3], ax_t[2];
    float arotR[2][9];  // per-arm orientation targets as rotation matrices, row-major
    float orot[4];      // object orientation target (w, x, y, z), unit
};

}  // namespace mppi
