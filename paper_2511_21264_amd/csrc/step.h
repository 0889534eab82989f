// One physics substep of the world model f (Eq. state_evol) for one sample,
// FP32, one lane per sample.
//
//   1. PD target q_des += h u; actuator tau = clamp(Kp (q_des - q) + Kd (u - qd));
//   2. free velocity (M + diag(armature + h (Kd + b))) (qd_f - qd) = h (tau - b qd - c),
//      the ball falls freely;
//   3. contacts of the candidate pairs in canonical order (AABB cull, then
//      narrowphase), the first n_cmax with phi < 0;
//   4. projected Gauss-Seidel on the soft LCP (A + R) f + b >= 0, f >= 0 with
//      four pyramid-edge rows per contact, n_pgs sweeps from f = 0.  The
//      Delassus matrix A = J Mt^-1 J^T is never formed: the solver keeps the
//      velocity v = qd_f + Mt^-1 J^T f, and row e's residual is
//      e . (J_p v) + R_e f_e - kappa max(-phi, 0) / h.  Within a contact the
//      point velocity J_p v is advanced with the 3x3 block G = J_p Mt^-1 J_p^T
//      and the impulse is applied to v once per contact, which is the same
//      Gauss-Seidel sequence as row-by-row updates of v;
//   5. semi-implicit Euler q += h qd+, p += h v+, r <- normalize(exp(h w+/2) (x) r).
#pragma once
#include "collision.h"

namespace mppi {

// Tangent basis of a unit normal (Duff et al., "Building an orthonormal
// basis, revisited", JCGT 2017).
__device__ __forceinline__ void tangents(V3 n, V3 &t1, V3 &t2)
{
    const float sg = n.z >= 0.f ? 1.f : -1.f;
    const float a = -1.0f / (sg + n.z);
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

// candidate contact from the pair sweep
template <int NC>
struct ContactList {
    int n;
    int ga[NC], gb[NC];
    float phi[NC];
    float nx[NC], ny[NC], nz[NC];
    float px[NC], py[NC], pz[NC];
};

// solver rows of one contact
template <int NC>
struct ContactRows {
    float J[NC][3][14];  // arm part of J_p = J_A(p) - J_B(p)
    float W[NC][14][3];  // Mt^-1 J^T (arm part)
    float rb[NC][3];     // ball lever arm p - c (ball is always geom A)
    float sb[NC];        // 1 if the ball takes part
    float G[NC][6];      // J_p Mt^-1 J_p^T: xx yy zz xy xz yz
    float E[NC][4][3];   // pyramid edges
    float Dinv[NC][4];   // 1 / (A_ee + R_e)
    float Rr[NC][4];     // R_e
    float bias[NC];      // kappa max(-phi, 0) / h
    float lam[NC][4];
};

template <int NC>
__device__ __forceinline__ void try_contact(const DevModel &md, ContactList<NC> &cl, StepCounters &cnt, int ga,
                                            int gb, const Shape &A, const Shape &B, const AABB &ba, const AABB &bb)
{
    if (cl.n < md.n_cmax && aabb_overlap(ba, bb, 0.f)) {
        ++cnt.np_tests;
        if (B.type == SH_BOX && A.type == SH_CAPSULE) ++cnt.box_tests;
        const Contact3 c = narrow(A, B);
        if (c.phi < 0.f) {
            const int i = cl.n;
            cl.ga[i] = ga;
            cl.gb[i] = gb;
            cl.phi[i] = c.phi;
            cl.nx[i] = c.n.x; cl.ny[i] = c.n.y; cl.nz[i] = c.n.z;
            cl.px[i] = c.p.x; cl.py[i] = c.p.y; cl.pz[i] = c.p.z;
            cl.n = i + 1;
        }
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

// sweep every candidate pair in canonical order
template <int NC>
__device__ inline void collect_contacts(const DevModel &md, const ArmKin kin[2], V3 pb, ContactList<NC> &cl,
                                        StepCounters &cnt)
{
    cl.n = 0;
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
    // 1 ball-table
    try_contact(md, cl, cnt, G_BALL, G_TABLE, ball, table, bball, btab);
    // 2 ball-pads
#pragma unroll
    for (int a = 0; a < 2; ++a) try_contact(md, cl, cnt, G_BALL, G_ARM + 7 * a + 6, ball, arm[a][6], bball, barm[a][6]);
    // 3 ball-links
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int g = 0; g < 6; ++g) try_contact(md, cl, cnt, G_BALL, G_ARM + 7 * a + g, ball, arm[a][g], bball, barm[a][g]);
    // 4 ball-boxes
    for (int b = 0; b < md.n_box; ++b) {
        const Shape bx = box_shape(md, b);
        try_contact(md, cl, cnt, G_BALL, G_BOX + b, ball, bx, bball, shape_aabb(bx));
    }
    // 5 arm geoms 2..7 - table
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int g = 1; g < 7; ++g) try_contact(md, cl, cnt, G_ARM + 7 * a + g, G_TABLE, arm[a][g], table, barm[a][g], btab);
    // 6 arm geoms - boxes
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int g = 0; g < 7; ++g)
            for (int b = 0; b < md.n_box; ++b) {
                const Shape bx = box_shape(md, b);
                try_contact(md, cl, cnt, G_ARM + 7 * a + g, G_BOX + b, arm[a][g], bx, barm[a][g], shape_aabb(bx));
            }
    // 7 arm 1 - arm 2
#pragma unroll
    for (int g = 0; g < 7; ++g)
#pragma unroll
        for (int g2 = 0; g2 < 7; ++g2)
            try_contact(md, cl, cnt, G_ARM + g, G_ARM + 7 + g2, arm[0][g], arm[1][g2], barm[0][g], barm[1][g2]);
    if (cl.n >= md.n_cmax) ++cnt.overflow;
    cnt.contacts += cl.n;
}

// build the solver rows of contact c
template <int NC>
__device__ inline void build_rows(const DevModel &md, const ArmKin kin[2], const float L[2][28], V3 pb,
                                  const ContactList<NC> &cl, int c, ContactRows<NC> &cr)
{
    const int ga = cl.ga[c], gb = cl.gb[c];
    const V3 n = v3(cl.nx[c], cl.ny[c], cl.nz[c]);
    const V3 p = v3(cl.px[c], cl.py[c], cl.pz[c]);
    // body of each side: arm index (-1 none) and link
    const bool a_is_arm = (ga >= G_ARM) & (ga < G_BOX);
    const bool b_is_arm = (gb >= G_ARM) & (gb < G_BOX);
    const int armA = a_is_arm ? (ga - G_ARM) / 7 : -1, linkA = a_is_arm ? (ga - G_ARM) % 7 : -1;
    const int armB = b_is_arm ? (gb - G_ARM) / 7 : -1, linkB = b_is_arm ? (gb - G_ARM) % 7 : -1;
    float J[3][14];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const float coef = (((armA == a) & (j <= linkA)) ? 1.f : 0.f) - (((armB == a) & (j <= linkB)) ? 1.f : 0.f);
            const V3 col = coef * cross(kin[a].a[j], p - kin[a].o[j]);
            J[0][7 * a + j] = col.x;
            J[1][7 * a + j] = col.y;
            J[2][7 * a + j] = col.z;
        }
    float W[14][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        float x0[NJ], x1[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) { x0[j] = J[r][j]; x1[j] = J[r][7 + j]; }
        chol7_solve(L[0], x0);
        chol7_solve(L[1], x1);
#pragma unroll
        for (int j = 0; j < NJ; ++j) { W[j][r] = x0[j]; W[7 + j][r] = x1[j]; }
    }
    float G[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < 14; ++d) {
        G[0] += J[0][d] * W[d][0];
        G[1] += J[1][d] * W[d][1];
        G[2] += J[2][d] * W[d][2];
        G[3] += J[0][d] * W[d][1];
        G[4] += J[0][d] * W[d][2];
        G[5] += J[1][d] * W[d][2];
    }
    const float sb = ga == G_BALL ? 1.f : 0.f;
    const V3 r = p - pb;
    {
        // ball block: P/m + (|r|^2 P - r (r.P)) / I
        const float im = md.inv_ball_m * sb, iI = md.inv_ball_I * sb, rr = dot(r, r);
        G[0] += im + iI * (rr - r.x * r.x);
        G[1] += im + iI * (rr - r.y * r.y);
        G[2] += im + iI * (rr - r.z * r.z);
        G[3] -= iI * r.x * r.y;
        G[4] -= iI * r.x * r.z;
        G[5] -= iI * r.y * r.z;
    }
    V3 t1, t2;
    tangents(n, t1, t2);
    const V3 e[4] = {fma3(md.mu, t1, n), fma3(-md.mu, t1, n), fma3(md.mu, t2, n), fma3(-md.mu, t2, n)};
    const S3 Gs = {G[0], G[1], G[2], G[3], G[4], G[5]};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float aee = dot(e[q], mul(Gs, e[q]));
        const float R = md.eps_r * aee;
        cr.Dinv[c][q] = 1.0f / (aee + R);
        cr.Rr[c][q] = R;
        cr.E[c][q][0] = e[q].x; cr.E[c][q][1] = e[q].y; cr.E[c][q][2] = e[q].z;
        cr.lam[c][q] = 0.f;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int d = 0; d < 14; ++d) cr.J[c][i][d] = J[i][d];
#pragma unroll
    for (int d = 0; d < 14; ++d)
#pragma unroll
        for (int i = 0; i < 3; ++i) cr.W[c][d][i] = W[d][i];
#pragma unroll
    for (int i = 0; i < 6; ++i) cr.G[c][i] = G[i];
    cr.rb[c][0] = r.x; cr.rb[c][1] = r.y; cr.rb[c][2] = r.z;
    cr.sb[c] = sb;
    const float pen = cl.phi[c] < 0.f ? -cl.phi[c] : 0.f;
    cr.bias[c] = md.kappa_h * pen;
}

template <int NC>
__device__ inline void pgs(const DevModel &md, int nc, ContactRows<NC> &cr, float v[14], V3 &vb, V3 &wb)
{
    for (int sweep = 0; sweep < md.n_pgs; ++sweep) {
        for (int c = 0; c < nc; ++c) {
            V3 vel = v3(0.f, 0.f, 0.f);
#pragma unroll
            for (int d = 0; d < 14; ++d) {
                vel.x = fmaf(cr.J[c][0][d], v[d], vel.x);
                vel.y = fmaf(cr.J[c][1][d], v[d], vel.y);
                vel.z = fmaf(cr.J[c][2][d], v[d], vel.z);
            }
            const float sb = cr.sb[c];
            const V3 r = v3(cr.rb[c][0], cr.rb[c][1], cr.rb[c][2]);
            vel = fma3(sb, vb + cross(wb, r), vel);
            const S3 G = {cr.G[c][0], cr.G[c][1], cr.G[c][2], cr.G[c][3], cr.G[c][4], cr.G[c][5]};
            V3 P = v3(0.f, 0.f, 0.f);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const V3 e = v3(cr.E[c][q][0], cr.E[c][q][1], cr.E[c][q][2]);
                const float lam = cr.lam[c][q];
                const float res = dot(e, vel) + cr.Rr[c][q] * lam - cr.bias[c];
                const float nl = fmaxf(lam - res * cr.Dinv[c][q], 0.f);
                const float dl = nl - lam;
                cr.lam[c][q] = nl;
                vel = fma3(dl, mul(G, e), vel);
                P = fma3(dl, e, P);
            }
#pragma unroll
            for (int d = 0; d < 14; ++d)
                v[d] = fmaf(cr.W[c][d][0], P.x, fmaf(cr.W[c][d][1], P.y, fmaf(cr.W[c][d][2], P.z, v[d])));
            vb = fma3(sb * md.inv_ball_m, P, vb);
            wb = fma3(sb * md.inv_ball_I, cross(r, P), wb);
        }
    }
}

template <int NC>
__device__ inline void substep(const DevModel &md, float x[NX], const float u[NU], StepCounters &cnt)
{
    const float h = md.h;
#pragma unroll
    for (int i = 0; i < 14; ++i) x[XQDES + i] = fmaf(h, u[i], x[XQDES + i]);
    ArmKin kin[2];
    fk_arm(md, 0, x + XQ, kin[0]);
    fk_arm(md, 1, x + XQ + 7, kin[1]);
    float L[2][28];
    float v[14];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        crba_arm(md, a, kin[a], L[a]);
        chol7(L[a]);
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
        chol7_solve(L[a], rhs);
#pragma unroll
        for (int i = 0; i < NJ; ++i) v[7 * a + i] = x[XQD + 7 * a + i] + rhs[i];
    }
    const V3 pb = v3(x[XPB], x[XPB + 1], x[XPB + 2]);
    V3 vb = v3(x[XVB], x[XVB + 1], x[XVB + 2] - h * md.g);
    V3 wb = v3(x[XWB], x[XWB + 1], x[XWB + 2]);

    ContactList<NC> cl;
    collect_contacts<NC>(md, kin, pb, cl, cnt);
    if (cl.n > 0) {
        ContactRows<NC> cr;
        for (int c = 0; c < cl.n; ++c) build_rows<NC>(md, kin, L, pb, cl, c, cr);
        pgs<NC>(md, cl.n, cr, v, vb, wb);
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
    if (ang < 1e-8f) {
        dw = 1.0f;
        dsc = 0.5f;
    } else {
        float s, c;
        sincosf(0.5f * ang, &s, &c);
        dw = c;
        dsc = s / ang;
    }
    const V3 dv = dsc * th;
    const float qw = x[XQUAT];
    const V3 qv = v3(x[XQUAT + 1], x[XQUAT + 2], x[XQUAT + 3]);
    const float nw = dw * qw - dot(dv, qv);
    const V3 nv = dw * qv + qw * dv + cross(dv, qv);
    const float inv = 1.0f / sqrtf(nw * nw + dot(nv, nv));
    x[XQUAT] = nw * inv;
    x[XQUAT + 1] = nv.x * inv;
    x[XQUAT + 2] = nv.y * inv;
    x[XQUAT + 3] = nv.z * inv;
}

}  // namespace mppi
