// Ball-task cost of one rollout, accumulated per control step at the
// post-step state (Sec. IV-B, single phase):
//   goal      ||p_ball - p_goal||       (object-to-target cost, simulated ball)
//   eef-obj   ||c - (p_ball - (0,0,eps))||, c = pad midpoint (Eq. ball_alignment_cost)
//   distance  (||p1 - p2|| - l_ball)^2  (Eq. end_effector_distance_cost)
//   planar    ||p1yz - p2yz||           (Eq. planar_alignment_cost)
//   smooth    ||u_k - u_{k-1}||^2       (smoothness term, k >= 1)
//   collision barrier max(-d_k + (1 - gamma) d_{k-1}, 0) and indicator
//             1{d_k < 0}, elementwise over the arm-box and arm-arm signed
//             distances saturated at m_c (Eq. collision_cost).
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
    float t[7];  // goal, eef-obj, distance, planar, smooth, barrier, indicator
};

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

// dist: per-sample history slots, pair-major with stride `stride` (= lanes of the launch)
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
    const float l = sqrtf(dot(d12, d12)) - md.l_ball;
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
}

}  // namespace mppi
