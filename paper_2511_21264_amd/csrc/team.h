// Team-per-sample mapping of the rollout: 16 lanes of a wave64 own one sample
// (4 samples per wave).  Lane t of a team: arm = t >> 3, joint jt = t & 7
// (jt = 0..6 are the joints of that arm; lanes 7 and 15 carry no joint).
//
//   forward kinematics  segmented inclusive scan (DPP row shifts) of the
//                       joint rotations R_j = B Rot_0 ... Rot_j and of the
//                       link offsets L_j z_j;
//   joint-space inertia composite bodies as segmented suffix sums of (mass,
//                       first moment, inertia about the arm base); lane r forms
//                       row r of M from the composite of every column;
//   bias forces         Newton-Euler with prefix sums for angular velocity,
//                       angular acceleration and joint-origin acceleration and
//                       suffix sums for the propagated force and moment;
//   Cholesky / solves   replicated on the 8 lanes of an arm segment;
//   pair sweep          candidate pairs dealt 16-wide in canonical order,
//                       contacts compacted by ballot so the list keeps the
//                       canonical order (first n_cmax kept);
//   contact solve       replicated on all 16 lanes (identical data, identical
//                       arithmetic to the lane mapping);
//   collision cost      cost pairs dealt 16-wide, each lane owns the history
//                       bits of its pairs.
// Composite quantities use coordinates relative to the arm base.
#pragma once
#include "cost.h"
#include "philox.h"

namespace mppi {

constexpr int TEAM = 16;
constexpr int TEAMS_PER_WAVE = 4;

// per-team LDS block (floats): geometry, contact list, park area
constexpr int TG_PTS = 0;             // 2 arms x 8 points x 3: joint origins o_0..o_6 and tip
constexpr int TG_BALL = 48;           // ball centre
constexpr int TG_FIELDS = 52;
constexpr int team_lds_floats(int nc) { return TG_FIELDS + nc * CL_FIELDS + PK_FIELDS; }

template <int S>
__device__ __forceinline__ float dpp_shr(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + S, 0xF, 0xF, true));
}
template <int S>
__device__ __forceinline__ float dpp_shl(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + S, 0xF, 0xF, true));
}

// value of team lane src (0..15)
__device__ __forceinline__ float tbc(float v, int src) { return __shfl(v, src, TEAM); }
__device__ __forceinline__ V3 tbc3(V3 v, int src) { return v3(tbc(v.x, src), tbc(v.y, src), tbc(v.z, src)); }

// inclusive prefix sum over the 8-lane arm segment
__device__ __forceinline__ float seg_prefix(float x, int jt)
{
    float y = dpp_shr<1>(x);
    x += jt >= 1 ? y : 0.f;
    y = dpp_shr<2>(x);
    x += jt >= 2 ? y : 0.f;
    y = dpp_shr<4>(x);
    x += jt >= 4 ? y : 0.f;
    return x;
}
__device__ __forceinline__ V3 seg_prefix3(V3 v, int jt) { return v3(seg_prefix(v.x, jt), seg_prefix(v.y, jt), seg_prefix(v.z, jt)); }

// inclusive suffix sum over the 8-lane arm segment
__device__ __forceinline__ float seg_suffix(float x, int jt)
{
    float y = dpp_shl<1>(x);
    x += jt + 1 <= 7 ? y : 0.f;
    y = dpp_shl<2>(x);
    x += jt + 2 <= 7 ? y : 0.f;
    y = dpp_shl<4>(x);
    x += jt + 4 <= 7 ? y : 0.f;
    return x;
}
__device__ __forceinline__ V3 seg_suffix3(V3 v, int jt) { return v3(seg_suffix(v.x, jt), seg_suffix(v.y, jt), seg_suffix(v.z, jt)); }

// sum over the 16 lanes of a team, result in every lane
__device__ __forceinline__ float team_sum(float x)
{
    x += __shfl_xor(x, 1, TEAM);
    x += __shfl_xor(x, 2, TEAM);
    x += __shfl_xor(x, 4, TEAM);
    x += __shfl_xor(x, 8, TEAM);
    return x;
}

struct M3 {
    float m[3][3];
};
__device__ __forceinline__ M3 mmul(const M3 &A, const M3 &B)
{
    M3 C;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C.m[i][j] = A.m[i][0] * B.m[0][j] + A.m[i][1] * B.m[1][j] + A.m[i][2] * B.m[2][j];
    return C;
}
template <int S>
__device__ __forceinline__ M3 dpp_shr_m3(const M3 &A)
{
    M3 B;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) B.m[i][j] = dpp_shr<S>(A.m[i][j]);
    return B;
}

// per-lane constants of the joint a lane carries
struct JointConst {
    int ax;
    float len, m, ix, iz;
    V3 base;
    float bc, bs;  // base yaw (cos, sin)
};

// one lane's kinematic quantities of its joint
struct JointKin {
    V3 a;        // joint axis
    V3 z;        // link axis
    V3 o;        // joint origin
    V3 o1;       // next joint origin (tip for joint 7)
};

__device__ inline void team_fk(const JointConst &jc, float q, int jt, JointKin &k)
{
    const bool joint = jt < 7;
    float s, c;
    sincosf(joint ? q : 0.f, &s, &c);
    M3 R;
    // local rotation about axis ax by q (identity on non-joint lanes)
    if (jc.ax == 0) {
        R = M3{{{1.f, 0.f, 0.f}, {0.f, c, -s}, {0.f, s, c}}};
    } else if (jc.ax == 1) {
        R = M3{{{c, 0.f, s}, {0.f, 1.f, 0.f}, {-s, 0.f, c}}};
    } else {
        R = M3{{{c, -s, 0.f}, {s, c, 0.f}, {0.f, 0.f, 1.f}}};
    }
    // segmented scan of the rotation chain
    {
        const M3 P = dpp_shr_m3<1>(R);
        if (jt >= 1) R = mmul(P, R);
    }
    {
        const M3 P = dpp_shr_m3<2>(R);
        if (jt >= 2) R = mmul(P, R);
    }
    {
        const M3 P = dpp_shr_m3<4>(R);
        if (jt >= 4) R = mmul(P, R);
    }
    // base yaw
    const M3 B = M3{{{jc.bc, -jc.bs, 0.f}, {jc.bs, jc.bc, 0.f}, {0.f, 0.f, 1.f}}};
    R = mmul(B, R);
    k.z = v3(R.m[0][2], R.m[1][2], R.m[2][2]);
    k.a = jc.ax == 0 ? v3(R.m[0][0], R.m[1][0], R.m[2][0]) : (jc.ax == 1 ? v3(R.m[0][1], R.m[1][1], R.m[2][1]) : k.z);
    const V3 d = (joint ? jc.len : 0.f) * k.z;
    const V3 inc = seg_prefix3(d, jt);
    k.o1 = jc.base + inc;
    k.o = k.o1 - d;
}

// row jt of Mt = M + diag(diag_add) (full row, 7 entries) on joint lanes
__device__ inline void team_crba(const DevModel &md, const JointConst &jc, const JointKin &k, int jt, int seg,
                                 float row[NJ])
{
    const bool joint = jt < 7;
    const V3 cr = fma3(0.5f * jc.len, k.z, k.o) - jc.base;  // link centre, base-relative
    const float m = joint ? jc.m : 0.f;
    const float ix = jc.ix, dz = jc.iz - jc.ix;
    const V3 z = k.z;
    // inertia about the base of link jt: I_c + m (|c|^2 1 - c c^T)
    const float cc2 = dot(cr, cr);
    float I[6] = {ix + dz * z.x * z.x + m * (cc2 - cr.x * cr.x), ix + dz * z.y * z.y + m * (cc2 - cr.y * cr.y),
                  ix + dz * z.z * z.z + m * (cc2 - cr.z * cr.z), dz * z.x * z.y - m * cr.x * cr.y,
                  dz * z.x * z.z - m * cr.x * cr.z,           dz * z.y * z.z - m * cr.y * cr.z};
#pragma unroll
    for (int i = 0; i < 6; ++i) I[i] = joint ? I[i] : 0.f;
    // composite of links jt..6
    const float Mc = seg_suffix(m, jt);
    const V3 h = seg_suffix3(m * cr, jt);
#pragma unroll
    for (int i = 0; i < 6; ++i) I[i] = seg_suffix(I[i], jt);
    const V3 cc = (joint ? 1.0f / Mc : 0.f) * h;
    const float c2 = dot(cc, cc);
    const S3 Ic = {I[0] - Mc * (c2 - cc.x * cc.x), I[1] - Mc * (c2 - cc.y * cc.y), I[2] - Mc * (c2 - cc.z * cc.z),
                   I[3] + Mc * cc.x * cc.y,        I[4] + Mc * cc.x * cc.z,        I[5] + Mc * cc.y * cc.z};
    const V3 ob = k.o - jc.base;
    const V3 L = Mc * cross(k.a, cc - ob);
    const V3 K = mul(Ic, k.a) + cross(cc, L);
    const V3 mo = cross(k.a, ob);
    // row jt: column i >= jt from the composite of i, i < jt from symmetry
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const int src = seg + i;
        const V3 Ki = tbc3(K, src), Li = tbc3(L, src), ai = tbc3(k.a, src), mi = tbc3(mo, src);
        row[i] = i >= jt ? dot(k.a, Ki) - dot(mo, Li) : dot(ai, K) - dot(mi, L);
    }
#pragma unroll
    for (int i = 0; i < NJ; ++i)
        if (i == jt) row[i] += md.diag_add;
}

// gather the packed lower triangle of the arm's Mt on every lane of its segment
__device__ __forceinline__ void team_gather_tri(const float row[NJ], int seg, float Lp[28])
{
#pragma unroll
    for (int r = 0; r < NJ; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) Lp[tri(r, c)] = tbc(row[c], seg + r);
}

// bias torque of the lane's joint: c(q, qd) (+ gravity when gravity)
__device__ inline float team_rnea(const DevModel &md, const JointConst &jc, const JointKin &k, float qd, int jt,
                                  bool gravity)
{
    const bool joint = jt < 7;
    const float qdj = joint ? qd : 0.f;
    const V3 wa = qdj * k.a;
    const V3 w = seg_prefix3(wa, jt);
    const V3 wprev = w - wa;
    const V3 ta = qdj * cross(wprev, k.a);
    const V3 al = seg_prefix3(ta, jt);
    const V3 d = (joint ? jc.len : 0.f) * k.z;
    const V3 tt = cross(al, d) + cross(w, cross(w, d));
    const V3 g0 = v3(0.f, 0.f, gravity ? md.g : 0.f);
    const V3 ao = g0 + seg_prefix3(tt, jt) - tt;
    const V3 dc = 0.5f * d;
    const V3 ac = ao + cross(al, dc) + cross(w, cross(w, dc));
    const float m = joint ? jc.m : 0.f;
    const float ix = jc.ix, dz = jc.iz - jc.ix;
    const V3 Ia = fma3(dz * dot(k.z, al), k.z, ix * al);
    const V3 Iw = fma3(dz * dot(k.z, w), k.z, ix * w);
    const V3 f = m * ac;
    const V3 n = joint ? Ia + cross(w, Iw) : v3(0.f, 0.f, 0.f);
    const V3 cr = k.o + dc - jc.base;
    const V3 S = seg_suffix3(n + cross(cr, f), jt);
    const V3 F = seg_suffix3(f, jt);
    return dot(k.a, S - cross(k.o - jc.base, F));
}

// component jt of a 7-vector held identically by the segment
__device__ __forceinline__ float pick7(const float v[NJ], int jt)
{
    float r = v[0];
#pragma unroll
    for (int i = 1; i < NJ; ++i) r = jt == i ? v[i] : r;
    return r;
}

struct TeamState {
    float q, qd, qdes;  // own joint (joint lanes)
    V3 pb, vb, wb;      // ball (replicated)
    float quat[4];
};

__device__ __forceinline__ Shape team_geom(const float *tl, const DevModel &md, int gid)
{
    Shape s;
    if (gid == G_BALL) {
        s.type = SH_SPHERE;
        s.p0 = v3(tl[TG_BALL], tl[TG_BALL + 1], tl[TG_BALL + 2]);
        s.p1 = s.p0;
        s.r = md.ball_r;
    } else if (gid == G_TABLE) {
        s = table_shape();
    } else if (gid >= G_BOX) {
        s = box_shape(md, gid - G_BOX);
    } else {
        const int arm = (gid - G_ARM) / 7, g = (gid - G_ARM) % 7;
        const float *p = tl + TG_PTS + 24 * arm;
        if (g < 6) {
            s.type = SH_CAPSULE;
            s.p0 = v3(p[3 * g], p[3 * g + 1], p[3 * g + 2]);
            s.p1 = v3(p[3 * g + 3], p[3 * g + 4], p[3 * g + 5]);
            s.r = md.link_rad[g];
        } else {
            s.type = SH_SPHERE;
            s.p0 = v3(p[21], p[22], p[23]);
            s.p1 = s.p0;
            s.r = md.pad_rad;
        }
    }
    return s;
}

// publish the joint origins, tip and ball centre of the team to LDS
__device__ __forceinline__ void team_publish_geom(float *tl, const JointKin &k, V3 pb, int arm, int jt)
{
    if (jt < 7) {
        float *p = tl + TG_PTS + 24 * arm + 3 * jt;
        p[0] = k.o.x; p[1] = k.o.y; p[2] = k.o.z;
        if (jt == 6) { p[3] = k.o1.x; p[4] = k.o1.y; p[5] = k.o1.z; }
    } else if (arm == 0) {
        tl[TG_BALL] = pb.x; tl[TG_BALL + 1] = pb.y; tl[TG_BALL + 2] = pb.z;
    }
}

// ArmKin of both arms from the published geometry (joint axes are in the park area)
__device__ __forceinline__ void team_kin_from_lds(const float *tl, ArmKin kin[2])
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i <= NJ; ++i) {
            const float *p = tl + TG_PTS + 24 * a + 3 * i;
            kin[a].o[i] = v3(p[0], p[1], p[2]);
        }
}

// candidate pairs dealt over the team's 16 lanes in canonical order;
// contacts land in the team's LDS list in canonical order; returns the count
__device__ inline int team_collect(const DevModel &md, const float *tl, const LaneList &LL, int t, int lane_in_wave,
                                   StepCounters &cnt)
{
    int n = 0;
    const int np = md.n_pairs;
    const int team_shift = lane_in_wave & ~(TEAM - 1);
    for (int base = 0; base < np; base += TEAM) {
        const int p = base + t;
        bool hit = false;
        Contact3 c;
        int ga = 0, gb = 0;
        if (p < np && n < md.n_cmax) {
            ga = md.pa[p];
            gb = md.pb[p];
            const Shape A = team_geom(tl, md, ga), B = team_geom(tl, md, gb);
            if (aabb_overlap(shape_aabb(A), shape_aabb(B), 0.f)) {
                ++cnt.np_tests;
                if (B.type == SH_BOX && A.type == SH_CAPSULE) ++cnt.box_tests;
                c = narrow(A, B);
                hit = c.phi < 0.f;
            }
        }
        const unsigned long long wm = __ballot(hit);
        const uint32_t tm = (uint32_t)(wm >> team_shift) & 0xffffu;
        if (hit) {
            const int slot = n + __popc(tm & ((1u << t) - 1u));
            if (slot < md.n_cmax) {
                LL.at(slot, 0) = __int_as_float(ga);
                LL.at(slot, 1) = __int_as_float(gb);
                LL.at(slot, 2) = c.phi;
                LL.at(slot, 3) = c.n.x; LL.at(slot, 4) = c.n.y; LL.at(slot, 5) = c.n.z;
                LL.at(slot, 6) = c.p.x; LL.at(slot, 7) = c.p.y; LL.at(slot, 8) = c.p.z;
            }
        }
        n = min(n + __popc(tm), md.n_cmax);
    }
    return n;
}

// normal z_d of joint d for (j, k, m): the same arithmetic as normals14
__device__ __forceinline__ float normal_joint(uint32_t key0, uint32_t key1, uint32_t j, uint32_t k, uint32_t m, int d)
{
    const U4 w = philox4x32_10(U4{j, k, (uint32_t)(d >> 2), m}, key0, key1);
    const bool p = (d & 3) >> 1;
    float z0, z1;
    box_muller(p ? w.z : w.x, p ? w.w : w.y, z0, z1);
    return (d & 1) ? z1 : z0;
}

struct TeamCtx {
    int t, arm, jt, seg, lane;
    bool joint;
    float *tl;
    LaneList LL;
    LanePark pk;
};

template <int NC>
__device__ inline void team_substep(const DevModel &md, const JointConst &jc, const TeamCtx &tc, TeamState &S,
                                    float u, StepCounters &cnt)
{
    const float h = md.h;
    const int jt = tc.jt, seg = tc.seg;
    S.qdes = fmaf(h, u, S.qdes);
    JointKin k;
    team_fk(jc, S.q, jt, k);
    float row[NJ];
    team_crba(md, jc, k, jt, seg, row);
    float Lp[28];
    team_gather_tri(row, seg, Lp);
    chol7(Lp);
    const float c = team_rnea(md, jc, k, S.qd, jt, md.gravcomp == 0);
    const float tau = clampf(md.kp * (S.qdes - S.q) + md.kd * (u - S.qd), -md.tau_max, md.tau_max);
    const float rhs = h * (tau - md.damp * S.qd - c);
    float xs[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) xs[i] = tbc(rhs, seg + i);
    chol7_solve(Lp, xs);
    float v = S.qd + pick7(xs, jt);
    const V3 pb = S.pb;
    V3 vb = v3(S.vb.x, S.vb.y, S.vb.z - h * md.g);
    V3 wb = S.wb;
    // publish geometry and the contact path's factor and axes
    team_publish_geom(tc.tl, k, pb, tc.arm, jt);
    if (tc.joint) {
        const int f = PK_A + 3 * (7 * tc.arm + jt);
        tc.pk.at(f) = k.a.x;
        tc.pk.at(f + 1) = k.a.y;
        tc.pk.at(f + 2) = k.a.z;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float val = Lp[0];
#pragma unroll
            for (int e = 1; e < 28; ++e) val = (e == 4 * jt + i) ? Lp[e] : val;
            tc.pk.at(PK_L + 28 * tc.arm + 4 * jt + i) = val;
        }
    }
    __syncthreads();
    const int nc = team_collect(md, tc.tl, tc.LL, tc.t, tc.lane, cnt);
    if (tc.t == 0) {
        cnt.contacts += nc;
        if (nc >= md.n_cmax) ++cnt.overflow;
    }
    __syncthreads();
    if (nc > 0) {
        ArmKin kin[2];
        team_kin_from_lds(tc.tl, kin);
        float vall[14];
#pragma unroll
        for (int i = 0; i < 14; ++i) vall[i] = tbc(v, (i / 7) * 8 + (i % 7));
        contact_solve<NC>(md, kin, tc.pk, pb, tc.LL, nc, vall, vb, wb);
        float mine = vall[0];
#pragma unroll
        for (int i = 1; i < 14; ++i) mine = (i == 7 * tc.arm + jt) ? vall[i] : mine;
        v = tc.joint ? mine : v;
    }
    S.q = fmaf(h, v, S.q);
    S.qd = v;
    S.pb = fma3(h, vb, pb);
    S.vb = vb;
    S.wb = wb;
    const V3 th = h * wb;
    const float ang = sqrtf(dot(th, th));
    float dw, dsc;
    if (ang < 1e-8f) {
        dw = 1.0f;
        dsc = 0.5f;
    } else {
        float sn, cs;
        sincosf(0.5f * ang, &sn, &cs);
        dw = cs;
        dsc = sn / ang;
    }
    const V3 dv = dsc * th;
    const float qw = S.quat[0];
    const V3 qv = v3(S.quat[1], S.quat[2], S.quat[3]);
    const float nw = dw * qw - dot(dv, qv);
    const V3 nv = dw * qv + qw * dv + cross(dv, qv);
    const float inv = 1.0f / sqrtf(nw * nw + dot(nv, nv));
    S.quat[0] = nw * inv;
    S.quat[1] = nv.x * inv;
    S.quat[2] = nv.y * inv;
    S.quat[3] = nv.z * inv;
}

// per-control-step cost at the post-step state; lane 0 accumulates the stage
// terms, joint lanes the smoothness, every lane its share of the cost pairs
__device__ inline void team_stage_cost(const DevModel &md, const JointConst &jc, const TeamCtx &tc,
                                       const TeamState &S, float u, float uprev, bool first, uint32_t &hist,
                                       float *dist, long stride, CostAcc &acc, StepCounters &cnt)
{
    JointKin k;
    team_fk(jc, S.q, tc.jt, k);
    team_publish_geom(tc.tl, k, S.pb, tc.arm, tc.jt);
    __syncthreads();
    const float *tl = tc.tl;
    if (tc.t == 0) {
        const V3 p1 = v3(tl[TG_PTS + 21], tl[TG_PTS + 22], tl[TG_PTS + 23]);
        const V3 p2 = v3(tl[TG_PTS + 45], tl[TG_PTS + 46], tl[TG_PTS + 47]);
        const V3 pb = S.pb;
        const V3 dg = pb - v3(md.goal[0], md.goal[1], md.goal[2]);
        const V3 de = 0.5f * (p1 + p2) - v3(pb.x, pb.y, pb.z - md.eps);
        const V3 d12 = p1 - p2;
        acc.t[0] += sqrtf(dot(dg, dg));
        acc.t[1] += sqrtf(dot(de, de));
        const float l = sqrtf(dot(d12, d12)) - md.l_ball;
        acc.t[2] += l * l;
        acc.t[3] += sqrtf(d12.y * d12.y + d12.z * d12.z);
    }
    if (!first && tc.joint) {
        const float du = u - uprev;
        acc.t[4] = fmaf(du, du, acc.t[4]);
    }
    const int nd = md.n_cost, first_pair = md.n_pairs - md.n_cost;
    uint32_t nw = 0u;
    for (int i = tc.t, r = 0; i < nd; i += TEAM, ++r) {
        const int p = first_pair + i;
        const Shape A = team_geom(tl, md, md.pa[p]), B = team_geom(tl, md, md.pb[p]);
        if (aabb_overlap(shape_aabb(A), shape_aabb(B), md.m_c)) {
            ++cnt.np_tests;
            if (B.type == SH_BOX && A.type == SH_CAPSULE) ++cnt.box_tests;
            const float d = narrow(A, B).phi;
            dist_term(md, d, !first, hist, 1u << r, dist + (long)i * stride, nw, acc);
        }
    }
    hist = nw;
}

}  // namespace mppi
