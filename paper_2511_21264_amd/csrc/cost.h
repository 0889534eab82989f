// Ball-task cost of one rollout, accumulated per control step at the
// post-step state (Sec. IV-B, single phase):
//   goal      ||p_ball - p_goal||       (object-to-target cost, simulated ball)
//   eef-obj   ||c - (p_ball - (0,0,eps))||, c = pad midpoint (Eq. ball_alignment_cost)
//   distance  (||p1 - p2|| - l)^2  (Eq. end_effector_distance_cost; l the
//             scene's end-effector distance target, else l_ball)
//   planar    ||p1yz - p2yz||           (Eq. planar_alignment_cost)
//   smooth    ||u_k - u_{k-1}||^2       (smoothness term, k >= 1)
//   collision barrier max(-d_k + (1 - gamma) d_{k-1}, 0) and indicator
//             1{d_k < 0}, elementwise over the arm-box and arm-arm signed
//             distances saturated at m_c (Eq. collision_cost).
// With the further task terms of Sec. IV switched on (md.ext), ten more
// (terms 7..16, unweighted sums over the horizon):
//   home      ||q - q_home||                   (joint deviation)
//   vertical  |p1z - p2z|                      (vertical alignment)
//   relvel    sqrt(sum_k ((p1 - p2) . (v1 - v2))^2), v_a the pad velocity J_a qd
//   apos_a    ||p_a - p_a*||                   (per-arm position target)
//   ax_a      |p_a,x - x_a*|                   (per-arm x target)
//   arot_a    angle of R_a* ^T R_a             (per-arm orientation target)
//   orot      angle of conj(Q*) (x) q          (object orientation target)
//
// Saturation makes the collision term sparse: a pair at distance >= m_c now
// contributes nothing (its barrier is max(-m_c + (1 - gamma) d_{k-1}, 0) = 0),
// and pairs whose AABBs grown by m_c do not overlap take the saturated value
// without a narrowphase.  So only pairs closer than m_c need last step's
// distance: a per-lane bitmask records which pairs were closer than m_c at
// the previous step and their distances sit in a per-sample global array
// touched only for those pairs.
#pragma once
#include "step.h"

namespace mppi {

struct CostAcc {
    // goal, eef-obj, distance, planar, smooth, barrier, indicator, then the
    // further terms (relvel as its sum of squares until total_cost)
    float t[NTERMS];
};

// rotation angle of Rt^T R in [0, pi]: atan2 of the skew part's norm
// (2 sin) over the trace minus one (2 cos).  Rt row-major; R by its columns.
__device__ __forceinline__ float rot_angle(const float *Rt, V3 c0, V3 c1, V3 c2)
{
    const V3 t0 = v3(Rt[0], Rt[3], Rt[6]), t1 = v3(Rt[1], Rt[4], Rt[7]), t2 = v3(Rt[2], Rt[5], Rt[8]);
    const float tr = dot(t0, c0) + dot(t1, c1) + dot(t2, c2);
    const V3 v = v3(dot(t2, c1) - dot(t1, c2), dot(t0, c2) - dot(t2, c0), dot(t1, c0) - dot(t0, c1));
    return atan2f(sqrtf(dot(v, v)), tr - 1.0f);
}

// the further terms at the post-step state (added to t[7..16])
__device__ inline void ext_terms(const DevModel &md, const ArmKin kin[2], const float x[NX], CostAcc &acc)
{
    float home = 0.f;
#pragma unroll
    for (int i = 0; i < 14; ++i) {
        const float d = x[XQ + i] - md.q_home[i];
        home = fmaf(d, d, home);
    }
    acc.t[7] += sqrtf(home);
    const V3 p1 = kin[0].o[NJ], p2 = kin[1].o[NJ];
    acc.t[8] += fabsf(p1.z - p2.z);
    V3 vel[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        V3 va = v3(0.f, 0.f, 0.f);
#pragma unroll
        for (int j = 0; j < NJ; ++j) va = fma3(x[XQD + 7 * a + j], cross(kin[a].a[j], kin[a].o[NJ] - kin[a].o[j]), va);
        vel[a] = va;
    }
    const float rv = dot(p1 - p2, vel[0] - vel[1]);
    acc.t[9] = fmaf(rv, rv, acc.t[9]);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const V3 p = kin[a].o[NJ];
        const V3 d = p - v3(md.apos[a][0], md.apos[a][1], md.apos[a][2]);
        acc.t[10 + a] += sqrtf(dot(d, d));
        acc.t[12 + a] += fabsf(p.x - md.ax_t[a]);
        acc.t[14 + a] += rot_angle(md.arotR[a], kin[a].x7, kin[a].y7, kin[a].z[NJ - 1]);
    }
    // object: q_rel = conj(Q) (x) q, angle 2 atan2(|v_rel|, |w_rel|)
    const float qw = x[XQUAT], Qw = md.orot[0];
    const V3 qv = v3(x[XQUAT + 1], x[XQUAT + 2], x[XQUAT + 3]), Qv = v3(md.orot[1], md.orot[2], md.orot[3]);
    const float wr = fmaf(Qw, qw, dot(Qv, qv));
    const V3 vr = Qw * qv - qw * Qv - cross(Qv, qv);
    acc.t[16] += 2.0f * atan2f(sqrtf(dot(vr, vr)), fabsf(wr));
}

// weighted total of a finished rollout (takes relvel's square root)
template <bool TASK>
__device__ __forceinline__ float total_cost(const DevModel &md, CostAcc &acc)
{
    float c = md.w_goal * acc.t[0] + md.w_eo * acc.t[1] + md.w_l * acc.t[2] + md.w_yz * acc.t[3] +
              md.w_s * acc.t[4] + md.w_c * (acc.t[5] + acc.t[6]);
    if (TASK && md.ext) {
        acc.t[9] = sqrtf(acc.t[9]);
        c += md.w_home * acc.t[7] + md.w_vert * acc.t[8] + md.w_relv * acc.t[9] + md.w_apos[0] * acc.t[10] +
             md.w_apos[1] * acc.t[11] + md.w_ax[0] * acc.t[12] + md.w_ax[1] * acc.t[13] + md.w_arot[0] * acc.t[14] +
             md.w_arot[1] * acc.t[15] + md.w_orot * acc.t[16];
    }
    return c;
}

// bit set: pair closer than m_c at the previous control step
struct DistHist {
    uint32_t box[14];  // arm geom (7 * arm + g) x box bit b
    uint32_t aa[2];    // arm 1 geom x arm 2 geom, bit 7 g + g2
};

__device__ __forceinline__ void dist_term(const DevModel &md, float d, bool has_prev, uint32_t prev_word,
                                          uint32_t bit, float *slot, uint32_t &new_word, CostAcc &acc)
{
    const float dh = fminf(d, md.m_c);
    if (dh < md.m_c) {
        if (has_prev) {
            const float prev = (prev_word & bit) ? *slot : md.m_c;
            acc.t[5] += fmaxf(-dh + md.one_m_gamma * prev, 0.f);
        }
        acc.t[6] += dh < 0.f ? 1.f : 0.f;
        *slot = dh;
        new_word |= bit;
    }
}

// dist: per-sample history slots, pair-major with stride `stride` (= lanes of
// the launch).  TASK: the form that can evaluate the further terms.
template <bool TASK>
__device__ inline void stage_cost(const DevModel &md, const float x[NX], const float u[NU], const float uprev[NU],
                                  bool first, DistHist &hist, float *dist, long stride, CostAcc &acc,
                                  StepCounters &cnt)
{
    ArmKin kin[2];
    fk_arm(md, 0, x + XQ, kin[0]);
    fk_arm(md, 1, x + XQ + 7, kin[1]);
    const V3 p1 = kin[0].o[NJ], p2 = kin[1].o[NJ];
    const V3 pb = v3(x[XPB], x[XPB + 1], x[XPB + 2]);
    const V3 g = v3(md.goal[0], md.goal[1], md.goal[2]);
    const V3 dg = pb - g;
    const V3 de = 0.5f * (p1 + p2) - v3(pb.x, pb.y, pb.z - md.eps);
    const V3 d12 = p1 - p2;
    acc.t[0] += sqrtf(dot(dg, dg));
    acc.t[1] += sqrtf(dot(de, de));
    const float l = sqrtf(dot(d12, d12)) - md.l_cost;
    acc.t[2] += l * l;
    acc.t[3] += sqrtf(d12.y * d12.y + d12.z * d12.z);
    if (!first) {
        float sm = 0.f;
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            const float du = u[i] - uprev[i];
            sm = fmaf(du, du, sm);
        }
        acc.t[4] += sm;
    }
    // collision distances: arm geoms x boxes, then arm 1 x arm 2
    Shape arm[2][7];
    AABB barm[2][7];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int gg = 0; gg < 7; ++gg) {
            arm[a][gg] = arm_shape(md, kin[a], gg);
            barm[a][gg] = shape_aabb(arm[a][gg]);
        }
    const int nb = md.n_box;
    const bool has_prev = !first;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int gg = 0; gg < 7; ++gg) {
            const int row = 7 * a + gg;
            uint32_t nw = 0u;
            for (int b = 0; b < nb; ++b) {
                const Shape bx = box_shape(md, b);
                if (aabb_overlap(barm[a][gg], shape_aabb(bx), md.m_c)) {
                    ++cnt.np_tests;
                    if (gg < 6) ++cnt.box_tests;
                    const float d = narrow(arm[a][gg], bx).phi;
                    dist_term(md, d, has_prev, hist.box[row], 1u << b, dist + (long)(row * nb + b) * stride, nw, acc);
                }
            }
            hist.box[row] = nw;
        }
    const int off = 14 * nb;
    uint32_t nw0 = 0u, nw1 = 0u;
#pragma unroll
    for (int gg = 0; gg < 7; ++gg)
#pragma unroll
        for (int g2 = 0; g2 < 7; ++g2) {
            if (aabb_overlap(barm[0][gg], barm[1][g2], md.m_c)) {
                ++cnt.np_tests;
                const float d = narrow(arm[0][gg], arm[1][g2]).phi;
                const int idx = 7 * gg + g2;
                if (idx < 32)
                    dist_term(md, d, has_prev, hist.aa[0], 1u << idx, dist + (long)(off + idx) * stride, nw0, acc);
                else
                    dist_term(md, d, has_prev, hist.aa[1], 1u << (idx - 32), dist + (long)(off + idx) * stride, nw1,
                              acc);
            }
        }
    hist.aa[0] = nw0;
    hist.aa[1] = nw1;
    if (TASK && md.ext) ext_terms(md, kin, x, acc);
}

}  // namespace mppi
