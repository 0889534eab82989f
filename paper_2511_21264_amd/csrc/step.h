// One physics substep of the world model f (Eq. state_evol) for one sample,
// FP32, one lane per sample.
//
//   1. PD target q_des += h u; actuator tau = clamp(Kp (q_des - q) + Kd (u - qd));
//   2. free velocity (M + diag(armature + h (Kd + b))) (qd_f - qd) = h (tau - b qd - c),
//      the ball falls freely;
//   3. contacts of the candidate pairs in canonical order (AABB cull, then
//      narrowphase), the first n_cmax with phi < 0;
//   4. projected Gauss-Seidel on the soft LCP (A + R) f + b >= 0, f >= 0 with
//      four pyramid-edge rows per contact (e = n +- mu t1, n +- mu t2),
//      n_pgs sweeps from f = 0, rows in contact order;
//   5. qd+ = qd_f + Mt^-1 J^T f, semi-implicit Euler q += h qd+, p += h v+,
//      r <- normalize(exp(h w+/2) (x) r).
// With a box-shaped object (the BOX forms) the object's inverse inertia is
// W = R diag(1/I) R^T in the world frame, its free angular velocity takes
// the explicit gyroscopic step w - h W (w x I_w w), and its contacts are the
// box's: up to four vertices below the table (vertex order), pads and links
// against the box in its own frame, static boxes by separating axes.
//
// Layout of the contact solve (impulse space).  A contact's four rows share
// its 3-row point Jacobian J_s (relative velocity of the touching points), so
// A is handled as 3x3 blocks G_st = J_s Mt^-1 J_t^T, and the solver keeps per
// contact the accumulated impulse P_s = sum_q f_q e_q.  Visiting contact s,
// its point velocity is J_s v = J_s qd_f + sum_t G_st P_t, each row's residual
// is e_q . (J_s v) + R_q f_q - kappa max(-phi, 0) / h, and a row update moves
// J_s v by G_ss e_q df: exactly the Gauss-Seidel sequence of the dense
// formulation.  Joint velocities are formed once at the end (one Cholesky
// solve of the generalized impulse).  Candidates are appended to a per-lane
// list in LDS (dynamic slot index); the solver data lives in registers in NC
// statically indexed slots.
#pragma once
#include "collision.h"

namespace mppi {

// Tangent basis of a unit normal (Duff et al., "Building an orthonormal
// basis, revisited", JCGT 2017).
__device__ __forceinline__ void tangents(V3 n, V3 &t1, V3 &t2)
{
    const float sg = n.z >= 0.f ? 1.f : -1.f;
    const float a = -frcp(sg + n.z);
    const float b = n.x * n.y * a;
    t1 = v3(1.0f + sg * n.x * n.x * a, sg * b, -sg * n.x);
    t2 = v3(b, sg + n.y * n.y * a, -n.y);
}

struct StepCounters {
    int contacts;   // contacts used
    int np_tests;   // narrowphase evaluations
    int box_tests;  // capsule-box evaluations
    int overflow;   // substeps with a full contact list
};

// Per-lane contact list in LDS, layout [slot][field][lane] (lane-contiguous:
// conflict-free).  Fields: ga, gb (as int bits), phi, n (3), p (3).
constexpr int CL_FIELDS = 9;
struct LaneList {
    float *base;  // workgroup base
    int lane;
    int width;    // lanes per workgroup
    __device__ __forceinline__ float &at(int slot, int f) const { return base[(slot * CL_FIELDS + f) * width + lane]; }
};

__device__ __forceinline__ void push_contact(const LaneList &L, int &n, int ga, int gb, const Contact3 &c)
{
    L.at(n, 0) = __int_as_float(ga);
    L.at(n, 1) = __int_as_float(gb);
    L.at(n, 2) = c.phi;
    L.at(n, 3) = c.n.x;
    L.at(n, 4) = c.n.y;
    L.at(n, 5) = c.n.z;
    L.at(n, 6) = c.p.x;
    L.at(n, 7) = c.p.y;
    L.at(n, 8) = c.p.z;
    ++n;
}

__device__ __forceinline__ void try_contact(const DevModel &md, const LaneList &L, int &n, StepCounters &cnt, int ga,
                                            int gb, const Shape &A, const Shape &B, const AABB &ba, const AABB &bb)
{
    if (n < md.n_cmax && aabb_overlap(ba, bb, 0.f)) {
        ++cnt.np_tests;
        if (B.type == SH_BOX && A.type == SH_CAPSULE) ++cnt.box_tests;
        const Contact3 c = narrow(A, B);
        if (c.phi < 0.f) push_contact(L, n, ga, gb, c);
    }
}

// pose of a box-shaped object: centre, rotation, half extents, world AABB
struct ObjPose {
    V3 c;
    Rot3 R;
    V3 h;
    AABB bb;
};

// the box object (geom A) against a pad, a link or a static box
__device__ __forceinline__ void try_obj_contact(const DevModel &md, const LaneList &L, int &n, StepCounters &cnt,
                                                int gb, const ObjPose &o, const Shape &B, const AABB &bb)
{
    if (n < md.n_cmax && aabb_overlap(o.bb, bb, 0.f)) {
        ++cnt.np_tests;
        const Contact3 c = B.type == SH_BOX ? obox_box(o.c, o.R, o.h, B.p0, B.p1) : obox_core(o.c, o.R, o.h, B);
        if (c.phi < 0.f) push_contact(L, n, G_BALL, gb, c);
    }
}

__device__ __forceinline__ Shape arm_shape(const DevModel &md, const ArmKin &k, int g)
{
    Shape s;
    if (g < 6) {
        s.type = SH_CAPSULE; s.p0 = k.o[g]; s.p1 = k.o[g + 1]; s.r = md.link_rad[g];
    } else {
        s.type = SH_SPHERE; s.p0 = k.o[NJ]; s.p1 = s.p0; s.r = md.pad_rad;
    }
    return s;
}

__device__ __forceinline__ Shape box_shape(const DevModel &md, int b)
{
    Shape s;
    s.type = SH_BOX;
    s.p0 = v3(md.box_c[b][0], md.box_c[b][1], md.box_c[b][2]);
    s.p1 = v3(md.box_h[b][0], md.box_h[b][1], md.box_h[b][2]);
    s.r = 0.f;
    return s;
}

__device__ __forceinline__ Shape table_shape()
{
    Shape s;
    s.type = SH_PLANE; s.p0 = v3(0.f, 0.f, 0.f); s.p1 = s.p0; s.r = 0.f;
    return s;
}

__device__ __forceinline__ Shape ball_shape(const DevModel &md, V3 pb)
{
    Shape s;
    s.type = SH_SPHERE; s.p0 = pb; s.p1 = pb; s.r = md.ball_r;
    return s;
}

// sweep every candidate pair in canonical order; returns the contact count.
// BOX: the object is the box of pose o (pb unused)
template <bool BOX>
__device__ inline int collect_contacts(const DevModel &md, const ArmKin kin[2], V3 pb, const ObjPose &o,
                                       const LaneList &L, StepCounters &cnt)
{
    int n = 0;
    const Shape ball = ball_shape(md, pb), table = table_shape();
    const AABB bball = shape_aabb(ball), btab = shape_aabb(table);
    Shape arm[2][7];
    AABB barm[2][7];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int g = 0; g < 7; ++g) {
            arm[a][g] = arm_shape(md, kin[a], g);
            barm[a][g] = shape_aabb(arm[a][g]);
        }
    if (BOX) {
        // 1 object-table: the vertices below the plane, four at most
        if (o.bb.lo.z < 0.f) {
            ++cnt.np_tests;
            int taken = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const V3 v = obox_vertex(o.c, o.R, o.h, k);
                if (v.z < 0.f && n < md.n_cmax && taken < 4) {
                    Contact3 c;
                    c.phi = v.z;
                    c.n = v3(0.f, 0.f, 1.f);
                    c.p = v3(v.x, v.y, 0.5f * v.z);
                    push_contact(L, n, G_BALL, G_TABLE, c);
                    ++taken;
                }
            }
        }
        // 2 object-pads, 3 object-links, 4 object-boxes
#pragma unroll
        for (int a = 0; a < 2; ++a) try_obj_contact(md, L, n, cnt, G_ARM + 7 * a + 6, o, arm[a][6], barm[a][6]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int g = 0; g < 6; ++g) try_obj_contact(md, L, n, cnt, G_ARM + 7 * a + g, o, arm[a][g], barm[a][g]);
        for (int b = 0; b < md.n_box; ++b) {
            const Shape bx = box_shape(md, b);
            try_obj_contact(md, L, n, cnt, G_BOX + b, o, bx, shape_aabb(bx));
        }
    } else {
        // 1 ball-table
        try_contact(md, L, n, cnt, G_BALL, G_TABLE, ball, table, bball, btab);
        // 2 ball-pads
#pragma unroll
        for (int a = 0; a < 2; ++a)
            try_contact(md, L, n, cnt, G_BALL, G_ARM + 7 * a + 6, ball, arm[a][6], bball, barm[a][6]);
        // 3 ball-links
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int g = 0; g < 6; ++g)
                try_contact(md, L, n, cnt, G_BALL, G_ARM + 7 * a + g, ball, arm[a][g], bball, barm[a][g]);
        // 4 ball-boxes
        for (int b = 0; b < md.n_box; ++b) {
            const Shape bx = box_shape(md, b);
            try_contact(md, L, n, cnt, G_BALL, G_BOX + b, ball, bx, bball, shape_aabb(bx));
        }
    }
    // 5 arm geoms 2..7 - table
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int g = 1; g < 7; ++g)
            try_contact(md, L, n, cnt, G_ARM + 7 * a + g, G_TABLE, arm[a][g], table, barm[a][g], btab);
    // 6 arm geoms - boxes
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int g = 0; g < 7; ++g)
            for (int b = 0; b < md.n_box; ++b) {
                const Shape bx = box_shape(md, b);
                try_contact(md, L, n, cnt, G_ARM + 7 * a + g, G_BOX + b, arm[a][g], bx, barm[a][g], shape_aabb(bx));
            }
    // 7 arm 1 - arm 2
#pragma unroll
    for (int g = 0; g < 7; ++g)
#pragma unroll
        for (int g2 = 0; g2 < 7; ++g2)
            try_contact(md, L, n, cnt, G_ARM + g, G_ARM + 7 + g2, arm[0][g], arm[1][g2], barm[0][g], barm[1][g2]);
    if (n >= md.n_cmax) ++cnt.overflow;
    cnt.contacts += n;
    return n;
}

// Per-lane spill area in LDS for data that only the (rare) arm-contact path
// re-reads: both arms' Cholesky factors and joint axes.  Layout [field][lane].
constexpr int PK_L = 0;          // 2 x 28 packed factors
constexpr int PK_A = 56;         // 2 x 7 x 3 joint axes
constexpr int PK_FIELDS = 98;
struct LanePark {
    float *base;
    int lane;
    int width;
    __device__ __forceinline__ float &at(int f) const { return base[f * width + lane]; }
};

// bodies touching at a contact, from its geom ids: arm index (-1 none) and link of each side
struct Sides {
    int armA, linkA, armB, linkB;
    bool ball;  // the ball is geom A
};

__device__ __forceinline__ Sides contact_sides(int gab)
{
    const int ga = gab & 0xff, gb = gab >> 8;
    Sides s;
    const bool aa = (ga >= G_ARM) & (ga < G_BOX), ab = (gb >= G_ARM) & (gb < G_BOX);
    s.armA = aa ? (ga - G_ARM) / 7 : -1;
    s.linkA = aa ? (ga - G_ARM) % 7 : -1;
    s.armB = ab ? (gb - G_ARM) / 7 : -1;
    s.linkB = ab ? (gb - G_ARM) % 7 : -1;
    s.ball = ga == G_BALL;
    return s;
}

// coefficient of joint j of arm a in the relative point Jacobian of a contact
__device__ __forceinline__ float jac_coef(const Sides &s, int a, int j)
{
    return (((s.armA == a) & (j <= s.linkA)) ? 1.f : 0.f) - (((s.armB == a) & (j <= s.linkB)) ? 1.f : 0.f);
}

// arm part of the 3 x 14 relative point Jacobian at p (axes from the park area)
__device__ __forceinline__ void arm_jac(const ArmKin kin[2], const LanePark &pk, const Sides &s, V3 p, V3 J[14])
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int f = PK_A + 3 * (7 * a + j);
            const V3 ax = v3(pk.at(f), pk.at(f + 1), pk.at(f + 2));
            J[7 * a + j] = jac_coef(s, a, j) * cross(ax, p - kin[a].o[j]);
        }
}

__device__ __forceinline__ void solve_parked(const LanePark &pk, int a, float x[NJ])
{
    float L[28];
#pragma unroll
    for (int i = 0; i < 28; ++i) L[i] = pk.at(PK_L + 28 * a + i);
    chol7_solve(L, x);
}

// ball part of G_st: I/m + ((r_s . r_t) I - r_t r_s^T) / I_b (3x3, row-major)
__device__ __forceinline__ void ball_block(const DevModel &md, V3 rs, V3 rt, float G[9])
{
    const float im = md.inv_ball_m, iI = md.inv_ball_I, d = dot(rs, rt);
    G[0] += im + iI * (d - rt.x * rs.x);
    G[1] += -iI * rt.x * rs.y;
    G[2] += -iI * rt.x * rs.z;
    G[3] += -iI * rt.y * rs.x;
    G[4] += im + iI * (d - rt.y * rs.y);
    G[5] += -iI * rt.y * rs.z;
    G[6] += -iI * rt.z * rs.x;
    G[7] += -iI * rt.z * rs.y;
    G[8] += im + iI * (d - rt.z * rs.z);
}

// box part of G_st: I/m - [r_s]x W [r_t]x, column j = e_j / m - r_s x (W (r_t x e_j))
// (W symmetric, row-major)
__device__ __forceinline__ V3 mul9(const float G[9], V3 v);
__device__ __forceinline__ void obj_block(const DevModel &md, const float W[9], V3 rs, V3 rt, float G[9])
{
    const float im = md.inv_ball_m;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const V3 e = v3(j == 0 ? 1.f : 0.f, j == 1 ? 1.f : 0.f, j == 2 ? 1.f : 0.f);
        const V3 col = cross(rs, mul9(W, cross(rt, e)));
        G[j] += (j == 0 ? im : 0.f) - col.x;
        G[3 + j] += (j == 1 ? im : 0.f) - col.y;
        G[6 + j] += (j == 2 ? im : 0.f) - col.z;
    }
}

__device__ __forceinline__ V3 mul9(const float G[9], V3 v)
{
    return v3(G[0] * v.x + G[1] * v.y + G[2] * v.z, G[3] * v.x + G[4] * v.y + G[5] * v.z,
              G[6] * v.x + G[7] * v.y + G[8] * v.z);
}
__device__ __forceinline__ V3 mul9t(const float G[9], V3 v)
{
    return v3(G[0] * v.x + G[3] * v.y + G[6] * v.z, G[1] * v.x + G[4] * v.y + G[7] * v.z,
              G[2] * v.x + G[5] * v.y + G[8] * v.z);
}

// register-resident solver data of up to NC contacts
template <int NC>
struct Slots {
    int gab[NC];          // geom ids ga | gb << 8
    V3 r[NC];             // contact point relative to the ball centre
    V3 b[NC];             // J_s qd_f
    V3 n[NC], t1[NC], t2[NC];
    V3 ge[NC][4];         // G_ss e_q
    float dinv[NC][4], rr[NC][4], lam[NC][4];
    float bias[NC];
    V3 P[NC];
    float G[NC][NC][9];   // G_st for s <= t
};

// BOX: the object's inverse inertia is W (world frame, row-major), else 1/I_b
template <int NC, bool BOX = false>
__device__ inline void contact_solve(const DevModel &md, const ArmKin kin[2], const LanePark &pk, V3 pb,
                                     const LaneList &LL, int nc, float v[14], V3 &vb, V3 &wb,
                                     const float *W = nullptr)
{
    Slots<NC> S;
    bool any_arm = false;
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        if (s < nc) {
            S.gab[s] = __float_as_int(LL.at(s, 0)) | (__float_as_int(LL.at(s, 1)) << 8);
            const float phi = LL.at(s, 2);
            S.n[s] = v3(LL.at(s, 3), LL.at(s, 4), LL.at(s, 5));
            S.r[s] = v3(LL.at(s, 6), LL.at(s, 7), LL.at(s, 8)) - pb;
            tangents(S.n[s], S.t1[s], S.t2[s]);
            S.bias[s] = md.kappa_h * (phi < 0.f ? -phi : 0.f);
            S.P[s] = v3(0.f, 0.f, 0.f);
            const Sides sd = contact_sides(S.gab[s]);
            any_arm |= (sd.armA >= 0) | (sd.armB >= 0);
        }
    }
    // blocks G_st (s <= t) and free point velocities b_s
#pragma unroll
    for (int t = 0; t < NC; ++t) {
        if (t < nc) {
            const Sides st = contact_sides(S.gab[t]);
            const bool arm_t = (st.armA >= 0) | (st.armB >= 0);
            V3 bt = v3(0.f, 0.f, 0.f);
            if (st.ball) bt = vb + cross(wb, S.r[t]);
#pragma unroll
            for (int s = 0; s <= t; ++s) {
                if (s < nc) {
                    float G[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    const Sides ss = contact_sides(S.gab[s]);
                    if (ss.ball & st.ball) {
                        if (BOX)
                            obj_block(md, W, S.r[s], S.r[t], G);
                        else
                            ball_block(md, S.r[s], S.r[t], G);
                    }
#pragma unroll
                    for (int i = 0; i < 9; ++i) S.G[s][t][i] = G[i];
                }
            }
            if (arm_t) {
                // Mt^-1 J_t^T, one column per Cartesian row of J_t
                float Wx[14], Wy[14], Wz[14];
                V3 Jt[14];
                arm_jac(kin, pk, st, S.r[t] + pb, Jt);
#pragma unroll
                for (int d = 0; d < 14; ++d) {
                    Wx[d] = Jt[d].x;
                    Wy[d] = Jt[d].y;
                    Wz[d] = Jt[d].z;
                    bt = fma3(v[d], Jt[d], bt);
                }
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    if ((st.armA == a) | (st.armB == a)) {
                        solve_parked(pk, a, Wx + 7 * a);
                        solve_parked(pk, a, Wy + 7 * a);
                        solve_parked(pk, a, Wz + 7 * a);
                    } else {
#pragma unroll
                        for (int j = 0; j < NJ; ++j) Wx[7 * a + j] = Wy[7 * a + j] = Wz[7 * a + j] = 0.f;
                    }
                }
#pragma unroll
                for (int s = 0; s <= t; ++s) {
                    if (s < nc) {
                        const Sides ss = contact_sides(S.gab[s]);
                        if ((ss.armA >= 0) | (ss.armB >= 0)) {
                            V3 Js[14];
                            arm_jac(kin, pk, ss, S.r[s] + pb, Js);
                            float G[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                            for (int d = 0; d < 14; ++d) {
                                G[0] += Js[d].x * Wx[d]; G[1] += Js[d].x * Wy[d]; G[2] += Js[d].x * Wz[d];
                                G[3] += Js[d].y * Wx[d]; G[4] += Js[d].y * Wy[d]; G[5] += Js[d].y * Wz[d];
                                G[6] += Js[d].z * Wx[d]; G[7] += Js[d].z * Wy[d]; G[8] += Js[d].z * Wz[d];
                            }
#pragma unroll
                            for (int i = 0; i < 9; ++i) S.G[s][t][i] += G[i];
                        }
                    }
                }
            }
            S.b[t] = bt;
        }
    }
    // row constants: edges, G_ss e_q, R_q, 1 / (A_qq + R_q)
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        if (s < nc) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const V3 t = q < 2 ? S.t1[s] : S.t2[s];
                const V3 e = fma3((q & 1) ? -md.mu : md.mu, t, S.n[s]);
                S.ge[s][q] = mul9(S.G[s][s], e);
                const float aqq = dot(e, S.ge[s][q]);
                S.rr[s][q] = md.eps_r * aqq;
                S.dinv[s][q] = frcp(aqq + S.rr[s][q]);
                S.lam[s][q] = 0.f;
            }
        }
    }
    // Gauss-Seidel sweeps
    for (int sweep = 0; sweep < md.n_pgs; ++sweep) {
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            if (s < nc) {
                V3 vel = S.b[s];
#pragma unroll
                for (int t = 0; t < NC; ++t) {
                    if (t < nc) vel = vel + (s <= t ? mul9(S.G[s][t], S.P[t]) : mul9t(S.G[t][s], S.P[t]));
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const V3 t = q < 2 ? S.t1[s] : S.t2[s];
                    const V3 e = fma3((q & 1) ? -md.mu : md.mu, t, S.n[s]);
                    const float lam = S.lam[s][q];
                    const float res = dot(e, vel) + S.rr[s][q] * lam - S.bias[s];
                    const float nl = fmaxf(lam - res * S.dinv[s][q], 0.f);
                    const float dl = nl - lam;
                    S.lam[s][q] = nl;
                    vel = fma3(dl, S.ge[s][q], vel);
                    S.P[s] = fma3(dl, e, S.P[s]);
                }
            }
        }
    }
    // apply: qd+ = qd_f + Mt^-1 sum_s J_s^T P_s
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        if (s < nc) {
            if (contact_sides(S.gab[s]).ball) {
                vb = fma3(md.inv_ball_m, S.P[s], vb);
                if (BOX)
                    wb = wb + mul9(W, cross(S.r[s], S.P[s]));
                else
                    wb = fma3(md.inv_ball_I, cross(S.r[s], S.P[s]), wb);
            }
        }
    }
    if (any_arm) {
        float gimp[14];
#pragma unroll
        for (int d = 0; d < 14; ++d) gimp[d] = 0.f;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            if (s < nc) {
                const Sides ss = contact_sides(S.gab[s]);
                if ((ss.armA >= 0) | (ss.armB >= 0)) {
                    V3 Js[14];
                    arm_jac(kin, pk, ss, S.r[s] + pb, Js);
#pragma unroll
                    for (int d = 0; d < 14; ++d) gimp[d] += dot(Js[d], S.P[s]);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            solve_parked(pk, a, gimp + 7 * a);
#pragma unroll
            for (int j = 0; j < NJ; ++j) v[7 * a + j] += gimp[7 * a + j];
        }
    }
}

// Projected Gauss-Seidel on four rows (one contact), f = 0 at the start:
// row r takes res = b_r + R_r f_r + sum_c A_rc f_c, f_r <- max(f_r - res / (A_rr + R_r), 0).
// With d_r = 1 / (A_rr + R_r) that is f_r <- max(u_r, 0) where
// u_r = -d_r (b_r + sum_{c != r} A_rc f_c) does not involve f_r, so each row is
// three multiply-adds with the scaled row C = -d_r A and a max; the value
// changed last enters last, so one multiply-add per row waits for the row
// before it.
__device__ __forceinline__ void pgs4(const float a[16], const float b[4], const float rr[4], const float dd[4],
                                     int n_pgs, float f[4])
{
    (void)rr;  // R_r sits only on the diagonal, which u_r leaves out
    float c[16], ub[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        ub[r] = -dd[r] * b[r];
#pragma unroll
        for (int k = 0; k < 4; ++k) c[4 * r + k] = -dd[r] * a[4 * r + k];
    }
    float f0 = f[0], f1 = f[1], f2 = f[2], f3 = f[3];
    for (int sweep = 0; sweep < n_pgs; ++sweep) {
        f0 = fmaxf(fmaf(c[3], f3, fmaf(c[2], f2, fmaf(c[1], f1, ub[0]))), 0.f);
        f1 = fmaxf(fmaf(c[4], f0, fmaf(c[7], f3, fmaf(c[6], f2, ub[1]))), 0.f);
        f2 = fmaxf(fmaf(c[9], f1, fmaf(c[8], f0, fmaf(c[11], f3, ub[2]))), 0.f);
        f3 = fmaxf(fmaf(c[14], f2, fmaf(c[13], f1, fmaf(c[12], f0, ub[3]))), 0.f);
    }
    f[0] = f0; f[1] = f1; f[2] = f2; f[3] = f3;
}

// One contact of the ball with a static body (table or box), the common case:
// the whole solve in registers (in the team mappings identically on every
// lane of the team).
__device__ inline void ball_contact_solve(const DevModel &md, const LaneList &LL, V3 pb, V3 &vb, V3 &wb)
{
    const V3 n = v3(LL.at(0, 3), LL.at(0, 4), LL.at(0, 5));
    const V3 r = v3(LL.at(0, 6), LL.at(0, 7), LL.at(0, 8)) - pb;
    const float phi = LL.at(0, 2);
    V3 t1, t2;
    tangents(n, t1, t2);
    V3 e[4], ge[4];
    float G[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    ball_block(md, r, r, G);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        e[q] = fma3((q & 1) ? -md.mu : md.mu, q < 2 ? t1 : t2, n);
        ge[q] = mul9(G, e[q]);
    }
    const V3 bfree = vb + cross(wb, r);
    const float bias = md.kappa_h * (phi < 0.f ? -phi : 0.f);
    float a[16], b[4], rr[4], dd[4], f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int c = 0; c < 4; ++c) a[4 * q + c] = dot(e[q], ge[c]);
        rr[q] = md.eps_r * a[5 * q];
        dd[q] = frcp(a[5 * q] + rr[q]);
        b[q] = dot(e[q], bfree) - bias;
        f[q] = 0.f;
    }
    pgs4(a, b, rr, dd, md.n_pgs, f);
    V3 P = v3(0.f, 0.f, 0.f);
#pragma unroll
    for (int q = 0; q < 4; ++q) P = fma3(f[q], e[q], P);
    vb = fma3(md.inv_ball_m, P, vb);
    wb = fma3(md.inv_ball_I, cross(r, P), wb);
}

template <int NC, bool BOX = false>
__device__ inline void substep(const DevModel &md, float x[NX], const float u[NU], const LaneList &LL,
                               const LanePark &pk, StepCounters &cnt)
{
    const float h = md.h;
#pragma unroll
    for (int i = 0; i < 14; ++i) x[XQDES + i] = fmaf(h, u[i], x[XQDES + i]);
    ArmKin kin[2];
    float v[14];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        if (a == 1) {
            // keep the two arms' dynamics sequential: their live sets would
            // otherwise be interleaved by the scheduler and double the registers
#pragma unroll
            for (int i = 7; i < 14; ++i) asm volatile("" : "+v"(x[XQ + i]) : "v"(v[6]));
        }
        fk_arm(md, a, x + XQ + 7 * a, kin[a]);
        float L[28];
        crba_arm(md, a, kin[a], L);
        chol7(L);
        float c[NJ];
        rnea_bias_arm(md, a, kin[a], x + XQD + 7 * a, md.gravcomp == 0, c);
        float rhs[NJ];
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const int d = 7 * a + i;
            const float qd = x[XQD + d];
            const float tau = clampf(md.kp * (x[XQDES + d] - x[XQ + d]) + md.kd * (u[d] - qd), -md.tau_max, md.tau_max);
            rhs[i] = h * (tau - md.damp * qd - c[i]);
        }
        chol7_solve(L, rhs);
#pragma unroll
        for (int i = 0; i < NJ; ++i) v[7 * a + i] = x[XQD + 7 * a + i] + rhs[i];
        // park the factor and the joint axes for the contact path
#pragma unroll
        for (int i = 0; i < 28; ++i) pk.at(PK_L + 28 * a + i) = L[i];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            pk.at(PK_A + 3 * (7 * a + j)) = kin[a].a[j].x;
            pk.at(PK_A + 3 * (7 * a + j) + 1) = kin[a].a[j].y;
            pk.at(PK_A + 3 * (7 * a + j) + 2) = kin[a].a[j].z;
        }
    }
    const V3 pb = v3(x[XPB], x[XPB + 1], x[XPB + 2]);
    V3 vb = v3(x[XVB], x[XVB + 1], x[XVB + 2] - h * md.g);
    V3 wb = v3(x[XWB], x[XWB + 1], x[XWB + 2]);

    if (BOX && md.obj_box) {
        ObjPose o;
        o.c = pb;
        o.R = quat_R(x[XQUAT], x[XQUAT + 1], x[XQUAT + 2], x[XQUAT + 3]);
        o.h = v3(md.obj_h[0], md.obj_h[1], md.obj_h[2]);
        o.bb = obox_aabb(o.c, o.R, o.h);
        // W = R diag(1/I) R^T; free w: w - h R diag(1/I) (w_b x (I w_b)), w_b = R^T w
        float W[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                W[3 * i + j] = o.R.m[3 * i] * o.R.m[3 * j] * md.obj_iI[0] +
                               o.R.m[3 * i + 1] * o.R.m[3 * j + 1] * md.obj_iI[1] +
                               o.R.m[3 * i + 2] * o.R.m[3 * j + 2] * md.obj_iI[2];
        const V3 wbb = mulRt(o.R, wb);
        const V3 Lb = v3(md.obj_I[0] * wbb.x, md.obj_I[1] * wbb.y, md.obj_I[2] * wbb.z);
        const V3 gb = cross(wbb, Lb);
        wb = wb - h * mulR(o.R, v3(md.obj_iI[0] * gb.x, md.obj_iI[1] * gb.y, md.obj_iI[2] * gb.z));
        const int nc = collect_contacts<true>(md, kin, pb, o, LL, cnt);
        if (nc > 0) contact_solve<NC, true>(md, kin, pk, pb, LL, nc, v, vb, wb, W);
    } else {
        ObjPose o0;
        const int nc = collect_contacts<false>(md, kin, pb, o0, LL, cnt);
        if (nc == 1 && __float_as_int(LL.at(0, 0)) == G_BALL &&
            (__float_as_int(LL.at(0, 1)) == G_TABLE || __float_as_int(LL.at(0, 1)) >= G_BOX))
            ball_contact_solve(md, LL, pb, vb, wb);
        else if (nc > 0)
            contact_solve<NC>(md, kin, pk, pb, LL, nc, v, vb, wb);
    }

#pragma unroll
    for (int i = 0; i < 14; ++i) {
        x[XQ + i] = fmaf(h, v[i], x[XQ + i]);
        x[XQD + i] = v[i];
    }
    x[XPB] = fmaf(h, vb.x, pb.x);
    x[XPB + 1] = fmaf(h, vb.y, pb.y);
    x[XPB + 2] = fmaf(h, vb.z, pb.z);
    x[XVB] = vb.x; x[XVB + 1] = vb.y; x[XVB + 2] = vb.z;
    x[XWB] = wb.x; x[XWB + 1] = wb.y; x[XWB + 2] = wb.z;
    // orientation: exp map of the world-frame rotation h w, applied on the left
    const V3 th = h * wb;
    const float ang = sqrtf(dot(th, th));
    float dw, dsc;
    half_angle_sincos(ang, dw, dsc);
    const V3 dv = dsc * th;
    const float qw = x[XQUAT];
    const V3 qv = v3(x[XQUAT + 1], x[XQUAT + 2], x[XQUAT + 3]);
    const float nw = dw * qw - dot(dv, qv);
    const V3 nv = dw * qv + qw * dv + cross(dv, qv);
    const float inv = __builtin_amdgcn_rsqf(nw * nw + dot(nv, nv));
    x[XQUAT] = nw * inv;
    x[XQUAT + 1] = nv.x * inv;
    x[XQUAT + 2] = nv.y * inv;
    x[XQUAT + 3] = nv.z * inv;
}

}  // namespace mppi
