// HIP kernels of the MPPI hot path for gfx950.
//
//   rollout_kernel  one lane per sample: Philox noise -> projected controls ->
//                   H control steps x n_sub physics substeps -> task cost
//                   (Alg. 1 sampling, QP, rollout and cost steps); the state
//                   stays in registers for the whole horizon, nothing but the
//                   cost (and optional diagnostics) is written.
//   stats_kernel    one workgroup: lowest finite cost, elite threshold,
//                   s_j = exp(-(c_j - c_min) / lambda) in FP64 (FP32 for the
//                   precision study), normalised
//                   weights and effective sample size (Eq. s_formula), with
//                   fixed-order tree reductions (deterministic).
//   update_kernel   one workgroup per control step: regenerates the projected
//                   samples from the Philox counters and forms
//                   (1 - eta) nu + eta sum_j w_j u_j in FP64 (Eq. mean_update).
//   sample / broadphase / narrowphase kernels expose single stages.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cost.h"
#include "kernels.h"
#include "philox.h"
#include "team.h"

namespace mppi {

// projected sample of joint d: clamp(nu + sigma z, +-u_max); one expression
// shared by the rollout and the update so both see identical bits
__device__ __forceinline__ void sample_u(const float *nu_k, const float *sig_k, float umax, uint32_t key0,
                                         uint32_t key1, uint32_t j, uint32_t k, uint32_t m, float u[NU])
{
    float z[14];
    normals14(key0, key1, j, k, m, z);
#pragma unroll
    for (int d = 0; d < NU; ++d) u[d] = clampf(fmaf(sig_k[d], z[d], nu_k[d]), -umax, umax);
}

// The model's words are re-read inside the horizon loop rather than hoisted:
// hoisted, ~100 uniform values overflow the SGPRs into VGPRs.  The pointer is
// opaque (so the reads stay where they are) and goes through the constant
// address space: the model is read-only during a launch, so uniform reads
// become scalar loads through the scalar cache instead of vector loads.
__device__ __forceinline__ const DevModel &model(const DevModel *p)
{
    const __attribute__((address_space(4))) DevModel *c = (const __attribute__((address_space(4))) DevModel *)p;
    asm volatile("" : "+s"(c));
    return *(const DevModel *)c;
}

// Scene of this workgroup: the single scene of the launch, or an entry of a
// packed table (uneven batches: block b covers block blk[2b+1] of scene blk[2b]).
__device__ __forceinline__ void block_scene(const RolloutArgs &a0, const RolloutArgs *tab, const int *blk, int m,
                                            RolloutArgs &a, int &bid)
{
    a = a0;
    bid = blockIdx.x;
    if (tab) {
        a = tab[blk[2 * blockIdx.x]];
        bid = blk[2 * blockIdx.x + 1];
        if (m >= 0) a.m = m;
    }
}

// TASK: the form for scenes with a box-shaped object or the further task
// terms (both switched per scene inside); the plain ball scene runs TASK = false
template <int NC, bool TASK>
__global__ void __launch_bounds__(64) rollout_kernel(RolloutArgs a0, const RolloutArgs *tab, const int *blk, int m)
{
    extern __shared__ float lds[];
    RolloutArgs a;
    int bid;
    block_scene(a0, tab, blk, m, a, bid);
    const int j = bid * blockDim.x + threadIdx.x;
    if (j >= a.K) return;
    const DevModel &md = *a.md;
    if (a.diverged && *a.diverged) {
        a.costs[j] = INFINITY;
        return;
    }
    const LaneList LL{lds, (int)threadIdx.x, (int)blockDim.x};
    const LanePark pk{lds + NC * CL_FIELDS * blockDim.x, (int)threadIdx.x, (int)blockDim.x};
    float x[NX];
    const float *x0 = a.x0 + (a.x0_shared ? 0 : (long)j * NX);
#pragma unroll
    for (int i = 0; i < NX; ++i) x[i] = x0[i];
    const int nsub = a.n_sub > 0 ? a.n_sub : md.n_sub;
    DistHist hist;
#pragma unroll
    for (int i = 0; i < 14; ++i) hist.box[i] = 0u;
    hist.aa[0] = hist.aa[1] = 0u;
    float *dist = a.dist + j;
    CostAcc acc;
#pragma unroll
    for (int i = 0; i < NTERMS; ++i) acc.t[i] = 0.f;
    StepCounters cnt = {0, 0, 0, 0};
    float uprev[NU];
#pragma unroll
    for (int d = 0; d < NU; ++d) uprev[d] = 0.f;
    for (int k = 0; k < a.H; ++k) {
        float u[NU];
        if (a.U) {
            const float *uk = a.U + ((long)j * a.H + k) * NU;
#pragma unroll
            for (int d = 0; d < NU; ++d) u[d] = uk[d];
        } else {
            sample_u(a.nu + k * NU, a.sigma + (a.sigma_per_step ? k * NU : 0), md.u_max, a.key0, a.key1, (uint32_t)j,
                     (uint32_t)k, (uint32_t)a.m, u);
        }
        for (int s = 0; s < nsub; ++s) substep<NC, TASK>(model(a.md), x, u, LL, pk, cnt);
        stage_cost<TASK>(model(a.md), x, u, uprev, k == 0, hist, dist, a.K, acc, cnt);
#pragma unroll
        for (int d = 0; d < NU; ++d) uprev[d] = u[d];
        if (a.xout && a.traj) {
            float *o = a.xout + ((long)j * a.H + k) * NX;
#pragma unroll
            for (int i = 0; i < NX; ++i) o[i] = x[i];
        }
    }
    const float c = total_cost<TASK>(md, acc);
    bool finite = isfinite(c);
#pragma unroll
    for (int i = 0; i < NX; ++i) finite &= isfinite(x[i]);
    a.costs[j] = finite ? c : INFINITY;
    if (a.terms) {
#pragma unroll
        for (int i = 0; i < NTERMS; ++i) a.terms[(long)j * NTERMS + i] = acc.t[i];
    }
    if (a.xout && !a.traj) {
#pragma unroll
        for (int i = 0; i < NX; ++i) a.xout[(long)j * NX + i] = x[i];
    }
    if (a.counters) {
        a.counters[4 * j + 0] = cnt.contacts;
        a.counters[4 * j + 1] = cnt.np_tests;
        a.counters[4 * j + 2] = cnt.box_tests;
        a.counters[4 * j + 3] = cnt.overflow;
    }
}

// The plain form: one launch per control step k, one sample per lane, the
// sample's state, previous control, cost accumulators, distance-history bits
// and counters kept in HBM between launches ([field][K], so a wave's loads
// and stores are coalesced).  The same device functions in the same order as
// rollout_kernel: the step-k launch loads what launch k - 1 stored.
constexpr int PS_X = 0, PS_UPREV = NX, PS_ACC = NX + NU, PS_HIST = NX + NU + NTERMS, PS_CNT = PS_HIST + 16;
static_assert(PS_CNT + 4 == PLAIN_FIELDS, "plain-form carry layout");

template <int NC, bool TASK>
__global__ void __launch_bounds__(64) rollout_step_kernel(RolloutArgs a, float *ps, int k)
{
    extern __shared__ float lds[];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.K) return;
    const DevModel &md = *a.md;
    if (a.diverged && *a.diverged) {
        if (k == a.H - 1) a.costs[j] = INFINITY;
        return;
    }
    const long K = a.K;
    const LaneList LL{lds, (int)threadIdx.x, (int)blockDim.x};
    const LanePark pk{lds + NC * CL_FIELDS * blockDim.x, (int)threadIdx.x, (int)blockDim.x};
    float x[NX], uprev[NU];
    CostAcc acc;
    DistHist hist;
    StepCounters cnt;
    if (k == 0) {
        const float *x0 = a.x0 + (a.x0_shared ? 0 : (long)j * NX);
#pragma unroll
        for (int i = 0; i < NX; ++i) x[i] = x0[i];
#pragma unroll
        for (int d = 0; d < NU; ++d) uprev[d] = 0.f;
#pragma unroll
        for (int i = 0; i < NTERMS; ++i) acc.t[i] = 0.f;
#pragma unroll
        for (int i = 0; i < 14; ++i) hist.box[i] = 0u;
        hist.aa[0] = hist.aa[1] = 0u;
        cnt = {0, 0, 0, 0};
    } else {
#pragma unroll
        for (int i = 0; i < NX; ++i) x[i] = ps[(PS_X + i) * K + j];
#pragma unroll
        for (int d = 0; d < NU; ++d) uprev[d] = ps[(PS_UPREV + d) * K + j];
#pragma unroll
        for (int i = 0; i < NTERMS; ++i) acc.t[i] = TASK || i < 7 ? ps[(PS_ACC + i) * K + j] : 0.f;
#pragma unroll
        for (int i = 0; i < 14; ++i) hist.box[i] = __float_as_uint(ps[(PS_HIST + i) * K + j]);
        hist.aa[0] = __float_as_uint(ps[(PS_HIST + 14) * K + j]);
        hist.aa[1] = __float_as_uint(ps[(PS_HIST + 15) * K + j]);
        cnt.contacts = __float_as_int(ps[(PS_CNT + 0) * K + j]);
        cnt.np_tests = __float_as_int(ps[(PS_CNT + 1) * K + j]);
        cnt.box_tests = __float_as_int(ps[(PS_CNT + 2) * K + j]);
        cnt.overflow = __float_as_int(ps[(PS_CNT + 3) * K + j]);
    }
    const int nsub = a.n_sub > 0 ? a.n_sub : md.n_sub;
    float *dist = a.dist + j;
    float u[NU];
    if (a.U) {
        const float *uk = a.U + ((long)j * a.H + k) * NU;
#pragma unroll
        for (int d = 0; d < NU; ++d) u[d] = uk[d];
    } else {
        sample_u(a.nu + k * NU, a.sigma + (a.sigma_per_step ? k * NU : 0), md.u_max, a.key0, a.key1, (uint32_t)j,
                 (uint32_t)k, (uint32_t)a.m, u);
    }
    for (int s = 0; s < nsub; ++s) substep<NC, TASK>(model(a.md), x, u, LL, pk, cnt);
    stage_cost<TASK>(model(a.md), x, u, uprev, k == 0, hist, dist, a.K, acc, cnt);
    if (a.xout && a.traj) {
        float *o = a.xout + ((long)j * a.H + k) * NX;
#pragma unroll
        for (int i = 0; i < NX; ++i) o[i] = x[i];
    }
    if (k < a.H - 1) {
#pragma unroll
        for (int i = 0; i < NX; ++i) ps[(PS_X + i) * K + j] = x[i];
#pragma unroll
        for (int d = 0; d < NU; ++d) ps[(PS_UPREV + d) * K + j] = u[d];
#pragma unroll
        for (int i = 0; i < (TASK ? NTERMS : 7); ++i) ps[(PS_ACC + i) * K + j] = acc.t[i];
#pragma unroll
        for (int i = 0; i < 14; ++i) ps[(PS_HIST + i) * K + j] = __uint_as_float(hist.box[i]);
        ps[(PS_HIST + 14) * K + j] = __uint_as_float(hist.aa[0]);
        ps[(PS_HIST + 15) * K + j] = __uint_as_float(hist.aa[1]);
        ps[(PS_CNT + 0) * K + j] = __int_as_float(cnt.contacts);
        ps[(PS_CNT + 1) * K + j] = __int_as_float(cnt.np_tests);
        ps[(PS_CNT + 2) * K + j] = __int_as_float(cnt.box_tests);
        ps[(PS_CNT + 3) * K + j] = __int_as_float(cnt.overflow);
        return;
    }
    const float c = total_cost<TASK>(md, acc);
    bool finite = isfinite(c);
#pragma unroll
    for (int i = 0; i < NX; ++i) finite &= isfinite(x[i]);
    a.costs[j] = finite ? c : INFINITY;
    if (a.terms) {
#pragma unroll
        for (int i = 0; i < NTERMS; ++i) a.terms[(long)j * NTERMS + i] = acc.t[i];
    }
    if (a.xout && !a.traj) {
#pragma unroll
        for (int i = 0; i < NX; ++i) a.xout[(long)j * NX + i] = x[i];
    }
    if (a.counters) {
        a.counters[4 * j + 0] = cnt.contacts;
        a.counters[4 * j + 1] = cnt.np_tests;
        a.counters[4 * j + 2] = cnt.box_tests;
        a.counters[4 * j + 3] = cnt.overflow;
    }
}

// Team mappings: 16 lanes per sample.  TPW = 4: four samples per 64-lane
// workgroup; TPW = 1: one sample per wave, its four 16-lane rows computing
// the same values and splitting the contact sweep 64 wide.  Teams past K
// run on a clamped sample index so that every lane reaches every barrier;
// they write nothing.
// TASK (one wave per sample only): the box object and the further terms
template <int NC, int TPW, bool TASK = false>
__global__ void __launch_bounds__(64) rollout_team_kernel(RolloutArgs a0, const RolloutArgs *tab, const int *blk, int m)
{
    extern __shared__ float lds[];
    RolloutArgs a;
    int bid;
    block_scene(a0, tab, blk, m, a, bid);
    const int lane = threadIdx.x;
    const int team = lane >> 4;
    const int slot = TPW == 1 ? 0 : team;  // sample slot of this row in the workgroup
    const bool primary = TPW != 1 || team == 0;  // the row that writes results
    TeamCtx tc;
    tc.lane = lane;
    tc.t = lane & 15;
    tc.arm = tc.t >> 3;
    tc.jt = tc.t & 7;
    tc.seg = tc.arm * 8;
    tc.joint = tc.jt < 7;
    tc.li = TPW == 1 ? lane : tc.t;
    tc.gshift = TPW == 1 ? 0 : (lane & ~15);
    tc.count = primary;
    tc.hd = lds;
    tc.tl = lds + HD_FIELDS + slot * team_lds_floats(NC);
    tc.LL = LaneList{tc.tl + TG_FIELDS, 0, 1};
    tc.pk = LanePark{tc.tl + TG_FIELDS + NC * CL_FIELDS, 0, 1};
    const int j_raw = bid * TPW + slot;
    const bool active = j_raw < a.K;
    const int j = active ? j_raw : a.K - 1;
    const DevModel &md0 = *a.md;
    const bool skip = a.diverged && *a.diverged;
    if (skip) {
        if (active && primary && tc.t == 0) a.costs[j] = INFINITY;
        return;  // uniform over the launch: every lane leaves
    }
    stage_header(lds, md0, lane, 64);
    __syncthreads();
    const int jj = tc.joint ? tc.jt : 6;
    const int d = 7 * tc.arm + jj;  // joint index of this lane
    JointConst jc;
    jc.ax = md0.axes[jj];
    jc.len = tc.joint ? md0.link_len[jj] : 0.f;
    jc.m = md0.m[tc.arm][jj];
    jc.ix = md0.Ix[tc.arm][jj];
    jc.iz = md0.Iz[tc.arm][jj];
    jc.base = v3(md0.base_pos[tc.arm][0], md0.base_pos[tc.arm][1], md0.base_pos[tc.arm][2]);
    jc.bc = md0.base_cs[tc.arm][0];
    jc.bs = md0.base_cs[tc.arm][1];
    const float *x0 = a.x0 + (a.x0_shared ? 0 : (long)j * NX);
    TeamState S;
    S.q = x0[XQ + d];
    S.qd = x0[XQD + d];
    S.qdes = x0[XQDES + d];
    S.pb = v3(x0[XPB], x0[XPB + 1], x0[XPB + 2]);
    S.vb = v3(x0[XVB], x0[XVB + 1], x0[XVB + 2]);
    S.wb = v3(x0[XWB], x0[XWB + 1], x0[XWB + 2]);
#pragma unroll
    for (int i = 0; i < 4; ++i) S.quat[i] = x0[XQUAT + i];
    const int nsub = a.n_sub > 0 ? a.n_sub : md0.n_sub;
    uint32_t hist = 0u;
    float *dist = a.dist + j;
    static_assert(!TASK || TPW == 1, "the task forms run one or two waves per sample");
    CostAcc acc;
#pragma unroll
    for (int i = 0; i < NTERMS; ++i) acc.t[i] = 0.f;
    StepCounters cnt = {0, 0, 0, 0};
    float uprev = 0.f;
    for (int k = 0; k < a.H; ++k) {
        const DevModel &md = model(a.md);
        float u = 0.f;
        if (tc.joint) {
            if (a.U) {
                u = a.U[((long)j * a.H + k) * NU + d];
            } else {
                const float z = normal_joint(a.key0, a.key1, (uint32_t)j, (uint32_t)k, (uint32_t)a.m, d);
                const float sg = a.sigma[(a.sigma_per_step ? k * NU : 0) + d];
                u = clampf(fmaf(sg, z, a.nu[k * NU + d]), -md.u_max, md.u_max);
            }
        }
        for (int s = 0; s < nsub; ++s)
            team_substep<NC, TPW == 1 ? 64 : TEAM, TPW == 1, TASK>(model(a.md), jc, tc, S, u, cnt);
        team_stage_cost<false, TASK>(model(a.md), jc, tc, S, u, uprev, k == 0, hist, dist, a.K, acc, cnt);
        uprev = u;
        if (a.xout && a.traj && active && primary) {
            float *o = a.xout + ((long)j * a.H + k) * NX;
            if (tc.joint) {
                o[XQ + d] = S.q; o[XQD + d] = S.qd; o[XQDES + d] = S.qdes;
            } else if (tc.arm == 0) {
                o[XPB] = S.pb.x; o[XPB + 1] = S.pb.y; o[XPB + 2] = S.pb.z;
#pragma unroll
                for (int i = 0; i < 4; ++i) o[XQUAT + i] = S.quat[i];
                o[XVB] = S.vb.x; o[XVB + 1] = S.vb.y; o[XVB + 2] = S.vb.z;
                o[XWB] = S.wb.x; o[XWB + 1] = S.wb.y; o[XWB + 2] = S.wb.z;
            }
        }
    }
    const DevModel &md = model(a.md);
    CostAcc tot;
#pragma unroll
    for (int i = 0; i < NTERMS; ++i) tot.t[i] = (TASK || i < 7) ? team_sum(acc.t[i]) : 0.f;
    const float c = total_cost<TASK>(md, tot);
    float bad = (isfinite(S.q) && isfinite(S.qd) && isfinite(S.qdes)) ? 0.f : 1.f;
    bad += (isfinite(S.pb.x) && isfinite(S.pb.y) && isfinite(S.pb.z) && isfinite(S.vb.x) && isfinite(S.vb.y) &&
            isfinite(S.vb.z) && isfinite(S.wb.x) && isfinite(S.wb.y) && isfinite(S.wb.z) && isfinite(S.quat[0]) &&
            isfinite(S.quat[1]) && isfinite(S.quat[2]) && isfinite(S.quat[3]))
               ? 0.f
               : 1.f;
    bad = team_sum(bad);
    const bool finite = isfinite(c) && !(bad > 0.f) && bad == bad;
    // narrowphase tests: the contact sweep spreads over the whole wave when
    // TPW = 1 (the cost pass counts on the primary row only)
    const float np = TPW == 1 ? wave_sum((float)cnt.np_tests) : team_sum((float)cnt.np_tests);
    const float nbx = TPW == 1 ? wave_sum((float)cnt.box_tests) : team_sum((float)cnt.box_tests);
    if (!active || !primary) return;
    if (tc.t == 0) {
        a.costs[j] = finite ? c : INFINITY;
        if (a.terms) {
#pragma unroll
            for (int i = 0; i < NTERMS; ++i) a.terms[(long)j * NTERMS + i] = tot.t[i];
        }
        if (a.counters) {
            a.counters[4 * j + 0] = cnt.contacts;
            a.counters[4 * j + 1] = (int)np;
            a.counters[4 * j + 2] = (int)nbx;
            a.counters[4 * j + 3] = cnt.overflow;
        }
    }
    if (a.xout && !a.traj) {
        float *o = a.xout + (long)j * NX;
        if (tc.joint) {
            o[XQ + d] = S.q; o[XQD + d] = S.qd; o[XQDES + d] = S.qdes;
        } else if (tc.arm == 0) {
            o[XPB] = S.pb.x; o[XPB + 1] = S.pb.y; o[XPB + 2] = S.pb.z;
#pragma unroll
            for (int i = 0; i < 4; ++i) o[XQUAT + i] = S.quat[i];
            o[XVB] = S.vb.x; o[XVB + 1] = S.vb.y; o[XVB + 2] = S.vb.z;
            o[XWB] = S.wb.x; o[XWB + 1] = S.wb.y; o[XWB + 2] = S.wb.z;
        }
    }
}

// Split mapping: two waves per sample.  Wave 0 (dynamics) owns the state and
// runs the inertia, factorisation, bias forces and free velocities, then the
// contact solve, the integration and the kinematics at the new positions;
// wave 1 (geometry) takes those kinematics and runs, concurrently with wave
// 0's dynamics, the geom AABBs and the contact sweep, and during wave 0's
// contact solve the cost of the previous control step.  Two workgroup
// barriers per substep hand the positions and kinematics to wave 1 (B1) and
// the contact list to wave 0 (B2); both waves run the same loop nest, so they
// meet every barrier the same number of times.  Every value equals the
// wave-per-sample mapping's bit for bit.
// state handoff: q[14], ball centre[3], contact count, finite flag; the
// task form also the object's quaternion (SA_QUAT) and qd[14] (SA_QD); the
// kinematics of the team's 16 lanes, 20 floats each (SA_KIN: a, z, o, o1,
// and the link frame's x, y)
constexpr int SA_QUAT = 19, SA_QD = 24, SA_KIN = 40, SPLIT_SA = SA_KIN + 16 * 20;

// FRAME: with the link frame's x and y axes
template <bool FRAME>
__device__ __forceinline__ void split_put_kin(float *p, const JointKin &k)
{
    float4 *o = reinterpret_cast<float4 *>(p);
    o[0] = make_float4(k.a.x, k.a.y, k.a.z, k.z.x);
    o[1] = make_float4(k.z.y, k.z.z, k.o.x, k.o.y);
    o[2] = make_float4(k.o.z, k.o1.x, k.o1.y, k.o1.z);
    if (FRAME) {
        o[3] = make_float4(k.x.x, k.x.y, k.x.z, k.y.x);
        o[4] = make_float4(k.y.y, k.y.z, 0.f, 0.f);
    }
}

template <bool FRAME>
__device__ __forceinline__ void split_get_kin(const float *p, JointKin &k)
{
    const float4 *i = reinterpret_cast<const float4 *>(p);
    const float4 a = i[0], b = i[1], c = i[2];
    k.a = v3(a.x, a.y, a.z);
    k.z = v3(a.w, b.x, b.y);
    k.o = v3(b.z, b.w, c.x);
    k.o1 = v3(c.y, c.z, c.w);
    if (FRAME) {
        const float4 d = i[3], e = i[4];
        k.x = v3(d.x, d.y, d.z);
        k.y = v3(d.w, e.x, e.y);
    }
}
template <int NC, bool TASK = false>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 2))) rollout_split_kernel(RolloutArgs a0, const RolloutArgs *tab, const int *blk,
                                                             int m)
{
    extern __shared__ float lds[];
    RolloutArgs a;
    int bid;
    block_scene(a0, tab, blk, m, a, bid);
    const int wave = threadIdx.x >> 6;
    const bool geo = wave == 1;
    // the dynamics wave carries each substep's critical path: it issues
    // ahead of the geometry waves that share its SIMD (priority 2 inside the
    // general contact solve)
    if (!geo) __builtin_amdgcn_s_setprio(1);
    const int lane = threadIdx.x & 63;
    const int row = lane >> 4;
    float *blockD = lds + HD_FIELDS, *blockG = blockD + team_lds_floats(NC);
    float *SA = blockG + team_lds_floats(NC);
    TeamCtx tc;
    tc.lane = lane;
    tc.t = lane & 15;
    tc.arm = tc.t >> 3;
    tc.jt = tc.t & 7;
    tc.seg = tc.arm * 8;
    tc.joint = tc.jt < 7;
    tc.li = lane;
    tc.gshift = 0;
    tc.count = geo && row == 0;
    tc.hd = lds;
    tc.tl = geo ? blockG : blockD;
    tc.LL = LaneList{blockG + TG_FIELDS, 0, 1};  // the contact list lives in the geometry wave's block
    tc.pk = LanePark{tc.tl + TG_FIELDS + NC * CL_FIELDS, 0, 1};
    const int j = bid;
    if (j >= a.K) return;  // uniform over the workgroup
    const DevModel &md0 = *a.md;
    const bool skip = a.diverged && *a.diverged;
    if (skip) {
        if (geo && lane == 0) a.costs[j] = INFINITY;
        return;  // uniform over the launch
    }
    stage_header(lds, md0, threadIdx.x, 128);
    __syncthreads();
    const int jj = tc.joint ? tc.jt : 6;
    const int d = 7 * tc.arm + jj;
    JointConst jc;
    jc.ax = md0.axes[jj];
    jc.len = tc.joint ? md0.link_len[jj] : 0.f;
    jc.m = md0.m[tc.arm][jj];
    jc.ix = md0.Ix[tc.arm][jj];
    jc.iz = md0.Iz[tc.arm][jj];
    jc.base = v3(md0.base_pos[tc.arm][0], md0.base_pos[tc.arm][1], md0.base_pos[tc.arm][2]);
    jc.bc = md0.base_cs[tc.arm][0];
    jc.bs = md0.base_cs[tc.arm][1];
    const float *x0 = a.x0 + (a.x0_shared ? 0 : (long)j * NX);
    TeamState S;
    S.q = x0[XQ + d];
    S.qd = x0[XQD + d];
    S.qdes = x0[XQDES + d];
    S.pb = v3(x0[XPB], x0[XPB + 1], x0[XPB + 2]);
    S.vb = v3(x0[XVB], x0[XVB + 1], x0[XVB + 2]);
    S.wb = v3(x0[XWB], x0[XWB + 1], x0[XWB + 2]);
#pragma unroll
    for (int i = 0; i < 4; ++i) S.quat[i] = x0[XQUAT + i];
    const int nsub = a.n_sub > 0 ? a.n_sub : md0.n_sub;
    uint32_t hist = 0u;
    float *dist = a.dist + j;
    CostAcc acc;
#pragma unroll
    for (int i = 0; i < NTERMS; ++i) acc.t[i] = 0.f;
    StepCounters cnt = {0, 0, 0, 0};
    float u1 = 0.f, u2 = 0.f;  // controls of the previous two steps (geometry wave's cost)
    // the kinematics at the current positions: formed by the dynamics wave
    // (at x0 here, then after each integration), published for the geometry wave
    JointKin kd;
    if (!geo) {
        team_fk<TASK>(jc, S.q, tc.jt, kd);
        if (row == 0) split_put_kin<TASK>(SA + SA_KIN + 20 * tc.t, kd);
    }
    for (int k = 0; k < a.H; ++k) {
        const DevModel &md = model(a.md);
        float u = 0.f;
        if (tc.joint) {
            if (a.U) {
                u = a.U[((long)j * a.H + k) * NU + d];
            } else {
                const float z = normal_joint(a.key0, a.key1, (uint32_t)j, (uint32_t)k, (uint32_t)a.m, d);
                const float sg = a.sigma[(a.sigma_per_step ? k * NU : 0) + d];
                u = clampf(fmaf(sg, z, a.nu[k * NU + d]), -md.u_max, md.u_max);
            }
        }
        for (int s = 0; s < nsub; ++s) {
            JointKin kk;
            float v = 0.f;
            V3 vb, wb;
            __syncthreads();  // B1: positions of this substep are in SA
            if (geo) {
                if (k > 0 || s > 0) {
                    if (tc.joint) S.q = SA[d];
                    S.pb = v3(SA[14], SA[15], SA[16]);
                    if (TASK) {
                        if (tc.joint) S.qd = SA[SA_QD + d];
#pragma unroll
                        for (int i = 0; i < 4; ++i) S.quat[i] = SA[SA_QUAT + i];
                    }
                }
                split_get_kin<TASK>(SA + SA_KIN + 20 * tc.t, kk);
                const int nc = team_contacts<64, TASK>(model(a.md), tc, kk, S.pb, cnt, S.quat);
                if (lane == 0) SA[17] = __int_as_float(nc);
            } else {
                kk = kd;
                team_dynamics<NC, true, TASK, true>(model(a.md), jc, tc, S, u, kk, v, vb, wb);
            }
            __syncthreads();  // B2: the contact list and its count are in LDS
            if (!geo) {
                const int nc = __float_as_int(SA[17]);
                team_finish<NC, true, true, TASK>(model(a.md), tc, S, kk, nc, v, vb, wb);
                team_fk<TASK>(jc, S.q, tc.jt, kd);
                if (row == 0) split_put_kin<TASK>(SA + SA_KIN + 20 * tc.t, kd);
                if (tc.joint) SA[d] = S.q;
                if (lane == 0) { SA[14] = S.pb.x; SA[15] = S.pb.y; SA[16] = S.pb.z; }
                if (TASK) {
                    if (tc.joint) SA[SA_QD + d] = S.qd;
                    if (lane == 0) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) SA[SA_QUAT + i] = S.quat[i];
                    }
                }
                if (s == nsub - 1 && a.xout && a.traj && row == 0) {
                    float *o = a.xout + ((long)j * a.H + k) * NX;
                    if (tc.joint) {
                        o[XQ + d] = S.q; o[XQD + d] = S.qd; o[XQDES + d] = S.qdes;
                    } else if (tc.arm == 0) {
                        o[XPB] = S.pb.x; o[XPB + 1] = S.pb.y; o[XPB + 2] = S.pb.z;
#pragma unroll
                        for (int i = 0; i < 4; ++i) o[XQUAT + i] = S.quat[i];
                        o[XVB] = S.vb.x; o[XVB + 1] = S.vb.y; o[XVB + 2] = S.vb.z;
                        o[XWB] = S.wb.x; o[XWB + 1] = S.wb.y; o[XWB + 2] = S.wb.z;
                    }
                }
            } else if (s == 0 && k > 0) {
                // cost of step k - 1 at its post-step state: this substep's positions,
                // whose geometry and AABBs the contact sweep has just published
                team_stage_cost<true, TASK>(model(a.md), jc, tc, S, u1, u2, k - 1 == 0, hist, dist, a.K, acc, cnt,
                                            &kk);
            }
        }
        u2 = u1;
        u1 = u;
    }
    // the final state: dynamics wave publishes it with its finiteness
    const DevModel &md = model(a.md);
    if (!geo) {
        float bad = (isfinite(S.q) && isfinite(S.qd) && isfinite(S.qdes)) ? 0.f : 1.f;
        bad += (isfinite(S.pb.x) && isfinite(S.pb.y) && isfinite(S.pb.z) && isfinite(S.vb.x) && isfinite(S.vb.y) &&
                isfinite(S.vb.z) && isfinite(S.wb.x) && isfinite(S.wb.y) && isfinite(S.wb.z) &&
                isfinite(S.quat[0]) && isfinite(S.quat[1]) && isfinite(S.quat[2]) && isfinite(S.quat[3]))
                   ? 0.f
                   : 1.f;
        bad = team_sum(bad);
        if (lane == 0) SA[18] = bad;
        if (a.xout && !a.traj && row == 0) {
            float *o = a.xout + (long)j * NX;
            if (tc.joint) {
                o[XQ + d] = S.q; o[XQD + d] = S.qd; o[XQDES + d] = S.qdes;
            } else if (tc.arm == 0) {
                o[XPB] = S.pb.x; o[XPB + 1] = S.pb.y; o[XPB + 2] = S.pb.z;
#pragma unroll
                for (int i = 0; i < 4; ++i) o[XQUAT + i] = S.quat[i];
                o[XVB] = S.vb.x; o[XVB + 1] = S.vb.y; o[XVB + 2] = S.vb.z;
                o[XWB] = S.wb.x; o[XWB + 1] = S.wb.y; o[XWB + 2] = S.wb.z;
            }
        }
    }
    __syncthreads();  // final positions and the finiteness flag are in SA
    if (!geo) return;
    if (tc.joint) S.q = SA[d];
    S.pb = v3(SA[14], SA[15], SA[16]);
    if (TASK) {
        if (tc.joint) S.qd = SA[SA_QD + d];
#pragma unroll
        for (int i = 0; i < 4; ++i) S.quat[i] = SA[SA_QUAT + i];
    }
    team_stage_cost<false, TASK>(md, jc, tc, S, u1, u2, a.H - 1 == 0, hist, dist, a.K, acc, cnt);
    CostAcc tot;
#pragma unroll
    for (int i = 0; i < NTERMS; ++i) tot.t[i] = (TASK || i < 7) ? team_sum(acc.t[i]) : 0.f;
    const float c = total_cost<TASK>(md, tot);
    const float bad = SA[18];
    const bool finite = isfinite(c) && !(bad > 0.f) && bad == bad;
    const float np = wave_sum((float)cnt.np_tests), nbx = wave_sum((float)cnt.box_tests);
    if (lane == 0) {
        a.costs[j] = finite ? c : INFINITY;
        if (a.terms) {
#pragma unroll
            for (int i = 0; i < NTERMS; ++i) a.terms[(long)j * NTERMS + i] = tot.t[i];
        }
        if (a.counters) {
            a.counters[4 * j + 0] = cnt.contacts;
            a.counters[4 * j + 1] = (int)np;
            a.counters[4 * j + 2] = (int)nbx;
            a.counters[4 * j + 3] = cnt.overflow;
        }
    }
}

int pick_mapping(int K, int requested)
{
    if (requested == MAP_LANE || requested == MAP_TEAM || requested == MAP_WAVE || requested == MAP_SPLIT ||
        requested == MAP_TASK || requested == MAP_TASK_WAVE || requested == MAP_TASK_SPLIT)
        return requested;
    // the chip holds 1024 SIMDs: up to 2 waves per SIMD two waves per sample
    // give the shortest steps (at K = 1024, H = 64: 1.90 against 2.21 ms a
    // wave per sample), up to ~2 samples per SIMD one wave per sample (at
    // 2048: 2.77 against 4.14 ms); below 64 k samples a 16-lane team per
    // sample (one lane per sample fills too few waves: at 32 k it is 1.5 x
    // slower); from 64 k on one lane per sample has the highest throughput
    if (K <= 1024) return MAP_SPLIT;
    if (K <= 2048) return MAP_WAVE;
    return K >= 65536 ? MAP_LANE : MAP_TEAM;
}

int samples_per_block(int mapping)
{
    return mapping == MAP_TEAM ? TEAMS_PER_WAVE
           : (mapping == MAP_WAVE || mapping == MAP_SPLIT || mapping == MAP_TASK_WAVE || mapping == MAP_TASK_SPLIT)
               ? 1
               : 64;
}

static void launch_rollout_impl(const RolloutArgs &a, const RolloutArgs *tab, const int *blk, int nblk, int ncmax,
                                int m, int map, hipStream_t s)
{
    const int nc = ncmax <= 4 ? 4 : 8;
    const dim3 grid(nblk), block(64);
    if (map == MAP_SPLIT || map == MAP_TASK_SPLIT) {
        const size_t lds = (size_t)(HD_FIELDS + 2 * team_lds_floats(nc) + SPLIT_SA) * sizeof(float);
        if (map == MAP_TASK_SPLIT) {
            if (nc == 4)
                hipLaunchKernelGGL((rollout_split_kernel<4, true>), grid, dim3(128), lds, s, a, tab, blk, m);
            else
                hipLaunchKernelGGL((rollout_split_kernel<8, true>), grid, dim3(128), lds, s, a, tab, blk, m);
        } else if (nc == 4) {
            hipLaunchKernelGGL(rollout_split_kernel<4>, grid, dim3(128), lds, s, a, tab, blk, m);
        } else {
            hipLaunchKernelGGL(rollout_split_kernel<8>, grid, dim3(128), lds, s, a, tab, blk, m);
        }
        return;
    }
    if (map == MAP_TASK_WAVE) {
        const size_t lds = (size_t)(HD_FIELDS + team_lds_floats(nc)) * sizeof(float);
        if (nc == 4)
            hipLaunchKernelGGL((rollout_team_kernel<4, 1, true>), grid, block, lds, s, a, tab, blk, m);
        else
            hipLaunchKernelGGL((rollout_team_kernel<8, 1, true>), grid, block, lds, s, a, tab, blk, m);
        return;
    }
    if (map == MAP_TEAM || map == MAP_WAVE) {
        const int tpw = map == MAP_TEAM ? TEAMS_PER_WAVE : 1;
        const size_t lds = (size_t)(HD_FIELDS + tpw * team_lds_floats(nc)) * sizeof(float);
        if (map == MAP_TEAM) {
            if (nc == 4)
                hipLaunchKernelGGL((rollout_team_kernel<4, TEAMS_PER_WAVE>), grid, block, lds, s, a, tab, blk, m);
            else
                hipLaunchKernelGGL((rollout_team_kernel<8, TEAMS_PER_WAVE>), grid, block, lds, s, a, tab, blk, m);
        } else {
            if (nc == 4)
                hipLaunchKernelGGL((rollout_team_kernel<4, 1>), grid, block, lds, s, a, tab, blk, m);
            else
                hipLaunchKernelGGL((rollout_team_kernel<8, 1>), grid, block, lds, s, a, tab, blk, m);
        }
        return;
    }
    const size_t lds = (size_t)(nc * CL_FIELDS + PK_FIELDS) * 64 * sizeof(float);
    if (map == MAP_TASK) {
        if (nc == 4)
            hipLaunchKernelGGL((rollout_kernel<4, true>), grid, block, lds, s, a, tab, blk, m);
        else
            hipLaunchKernelGGL((rollout_kernel<8, true>), grid, block, lds, s, a, tab, blk, m);
        return;
    }
    if (nc == 4)
        hipLaunchKernelGGL((rollout_kernel<4, false>), grid, block, lds, s, a, tab, blk, m);
    else
        hipLaunchKernelGGL((rollout_kernel<8, false>), grid, block, lds, s, a, tab, blk, m);
}

void launch_rollout(const RolloutArgs &a, int ncmax, hipStream_t s, int mapping)
{
    const int map = pick_mapping(a.K, mapping);
    const int per = samples_per_block(map);
    launch_rollout_impl(a, nullptr, nullptr, (a.K + per - 1) / per, ncmax, a.m, map, s);
}

void launch_rollout_step(const RolloutArgs &a, int ncmax, float *ps, int k, bool task, hipStream_t s)
{
    const int nc = ncmax <= 4 ? 4 : 8;
    const size_t lds = (size_t)(nc * CL_FIELDS + PK_FIELDS) * 64 * sizeof(float);
    const dim3 grid((a.K + 63) / 64), block(64);
    if (task) {
        if (nc == 4)
            hipLaunchKernelGGL((rollout_step_kernel<4, true>), grid, block, lds, s, a, ps, k);
        else
            hipLaunchKernelGGL((rollout_step_kernel<8, true>), grid, block, lds, s, a, ps, k);
    } else {
        if (nc == 4)
            hipLaunchKernelGGL((rollout_step_kernel<4, false>), grid, block, lds, s, a, ps, k);
        else
            hipLaunchKernelGGL((rollout_step_kernel<8, false>), grid, block, lds, s, a, ps, k);
    }
}

void launch_rollout_batch(const RolloutArgs *d_tab, const int *d_blk, int nblk, int ncmax, int m, int map,
                          hipStream_t s)
{
    RolloutArgs dummy = {};
    launch_rollout_impl(dummy, d_tab, d_blk, nblk, ncmax, m, map, s);
}

// ---------------------------------------------------------------------------
// statistics and weights (one workgroup of 1024 lanes)

constexpr int SB = 1024;

__device__ __forceinline__ uint32_t ordered_bits(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Sum over the 64 lanes of a wave by an xor butterfly of wavefront shuffles:
// every lane ends with the same bits (each pair of lanes adds the same two
// values, and IEEE addition commutes).
template <typename T>
__device__ __forceinline__ T wave_allsum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a workgroup of NT lanes: wave sums, then the NT / 64 of them in
// wave order (sh: NT / 64 entries); every lane returns the same value.
template <typename T, int NT = SB>
__device__ __forceinline__ T block_sum(T v, T *sh)
{
    v = wave_allsum(v);
    const int t = threadIdx.x;
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    T r = sh[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

__device__ __forceinline__ float exp_t(float x) { return expf(x); }
__device__ __forceinline__ double exp_t(double x) { return exp(x); }

// T: precision of the weights, their sums and the effective sample size
template <typename T>
__global__ void __launch_bounds__(SB) stats_kernel(StatsArgs a0, const StatsArgs *tab, int m)
{
    StatsArgs a = a0;
    if (tab) {
        a = tab[blockIdx.x];
        if (m >= 0) a.iter = m;
    }
    __shared__ double shd[SB / 64];
    __shared__ unsigned long long shu[SB / 64];
    __shared__ float shf[SB / 64];
    __shared__ int shi[SB / 64];
    const int t = threadIdx.x;
    // lowest finite cost (ties: lowest index) and finite count
    float best = INFINITY;
    int bi = 0x7fffffff, nf = 0;
    for (int j = t; j < a.K; j += SB) {
        const float c = a.costs[j];
        if (isfinite(c)) {
            ++nf;
            if (c < best || (c == best && j < bi)) { best = c; bi = j; }
        }
    }
    // (cost, index) minimum: wavefront shuffles within each wave, then the
    // waves' results in order (the selection is exact, so every lane agrees)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float c2 = __shfl_xor(best, o, 64);
        const int i2 = __shfl_xor(bi, o, 64);
        if (c2 < best || (c2 == best && i2 < bi)) { best = c2; bi = i2; }
    }
    if ((t & 63) == 0) {
        shf[t >> 6] = best;
        shi[t >> 6] = bi;
    }
    __syncthreads();
    float cmin = shf[0];
    int best_j = shi[0];
#pragma unroll
    for (int w = 1; w < SB / 64; ++w) {
        const float c2 = shf[w];
        const int i2 = shi[w];
        if (c2 < cmin || (c2 == cmin && i2 < best_j)) { cmin = c2; best_j = i2; }
    }
    __syncthreads();
    const unsigned long long nfin = block_sum<unsigned long long>((unsigned long long)nf, shu);
    // elite threshold: the n_e-th smallest key (ordered cost bits, index)
    unsigned long long thr = ~0ull;
    if (a.n_elite > 0 && (unsigned long long)a.n_elite < nfin) {
        unsigned long long lo = 0, hi = ~0ull;
        while (lo < hi) {
            const unsigned long long mid = lo + (hi - lo) / 2;
            unsigned long long cnt = 0;
            for (int j = t; j < a.K; j += SB) {
                const float c = a.costs[j];
                if (isfinite(c)) {
                    const unsigned long long key = ((unsigned long long)ordered_bits(c) << 32) | (uint32_t)j;
                    cnt += key <= mid;
                }
            }
            cnt = block_sum<unsigned long long>(cnt, shu);
            if (cnt >= (unsigned long long)a.n_elite) hi = mid; else lo = mid + 1;
        }
        thr = lo;
    }
    // weights
    T *shT = sizeof(T) == sizeof(double) ? (T *)shd : (T *)shf;
    T z = 0, z2 = 0;
    for (int j = t; j < a.K; j += SB) {
        const float c = a.costs[j];
        T s = 0;
        if (isfinite(c)) {
            const unsigned long long key = ((unsigned long long)ordered_bits(c) << 32) | (uint32_t)j;
            if (key <= thr) s = exp_t(-((T)c - (T)cmin) * (T)a.inv_lambda);
        }
        a.weights[j] = (double)s;
        z += s;
        z2 += s * s;
    }
    z = block_sum<T>(z, shT);
    z2 = block_sum<T>(z2, shT);
    const T inv = nfin > 0 ? T(1) / z : T(0);
    for (int j = t; j < a.K; j += SB) a.weights[j] = (double)((T)a.weights[j] * inv);
    // work counters
    if (a.counters) {
        for (int c = 0; c < 4; ++c) {
            unsigned long long v = 0;
            for (int j = t; j < a.K; j += SB) v += (unsigned long long)a.counters[4 * j + c];
            v = block_sum<unsigned long long>(v, shu);
            if (t == 0) a.st->counters[c] += v;
        }
    }
    if (t == 0) {
        PlanStats *st = a.st;
        st->cmin = nfin > 0 ? (double)cmin : INFINITY;
        st->best = nfin > 0 ? best_j : -1;
        st->n_finite = (int)nfin;
        st->wsum = (double)z;
        st->ess = nfin > 0 ? (double)(z * z / z2) : 0.0;
        if (a.iter < 64) st->cmin_iter[a.iter] = st->cmin;
        if (nfin == 0) st->diverged = 1;
    }
}

void launch_stats(const StatsArgs &a, hipStream_t s)
{
    if (a.fp32)
        hipLaunchKernelGGL(stats_kernel<float>, dim3(1), dim3(SB), 0, s, a, (const StatsArgs *)nullptr, a.iter);
    else
        hipLaunchKernelGGL(stats_kernel<double>, dim3(1), dim3(SB), 0, s, a, (const StatsArgs *)nullptr, a.iter);
}

void launch_stats_batch(const StatsArgs *d_tab, int n, int m, hipStream_t s)
{
    StatsArgs dummy = {};
    hipLaunchKernelGGL(stats_kernel<double>, dim3(n), dim3(SB), 0, s, dummy, d_tab, m);
}

__global__ void reset_stats_kernel(PlanStats *st0)
{
    PlanStats *st = st0 + blockIdx.x;
    const int t = threadIdx.x;
    if (t < 64) st->cmin_iter[t] = 0.0;
    if (t < 4) st->counters[t] = 0ull;
    if (t == 0) {
        st->cmin = 0.0; st->wsum = 0.0; st->ess = 0.0;
        st->best = -1; st->n_finite = 0; st->diverged = 0; st->pad = 0;
    }
}

void launch_reset_stats(PlanStats *st, hipStream_t s, int n)
{
    hipLaunchKernelGGL(reset_stats_kernel, dim3(n), dim3(64), 0, s, st);
}

// ---------------------------------------------------------------------------
// weighted mean update: one workgroup per control step

constexpr int UB = 256;

template <typename T>
__global__ void __launch_bounds__(UB) update_kernel(UpdateArgs a0, const UpdateArgs *tab, const int *blk, int m)
{
    __shared__ T red[NU][UB / 64];
    UpdateArgs a = a0;
    int k = blockIdx.x;
    if (tab) {
        a = tab[blk[2 * blockIdx.x]];
        k = blk[2 * blockIdx.x + 1];
        if (m >= 0) a.m = m;
    }
    const int t = threadIdx.x;
    const bool div = a.st->diverged != 0;
    T acc[NU];
#pragma unroll
    for (int d = 0; d < NU; ++d) acc[d] = 0;
    if (!div) {
        const float *nu_k = a.nu_in + k * NU;
        const float *sig_k = a.sigma + (a.sigma_per_step ? k * NU : 0);
        for (int j = t; j < a.K; j += UB) {
            const T w = (T)a.weights[j];
            if (w != T(0)) {
                float u[NU];
                if (a.U) {
#pragma unroll
                    for (int d = 0; d < NU; ++d) u[d] = a.U[((long)j * a.H + k) * NU + d];
                } else {
                    sample_u(nu_k, sig_k, a.u_max, a.key0, a.key1, (uint32_t)j, (uint32_t)k, (uint32_t)a.m, u);
                }
#pragma unroll
                for (int d = 0; d < NU; ++d) acc[d] = fma(w, (T)u[d], acc[d]);
            }
        }
    }
    // the sums over the samples: wavefront shuffles within each wave, then
    // the waves' sums in order
#pragma unroll
    for (int d = 0; d < NU; ++d) acc[d] = wave_allsum(acc[d]);
    if ((t & 63) == 0) {
#pragma unroll
        for (int d = 0; d < NU; ++d) red[d][t >> 6] = acc[d];
    }
    __syncthreads();
    if (t < NU) {
        T sum = red[t][0];
#pragma unroll
        for (int w = 1; w < UB / 64; ++w) sum += red[t][w];
        const T nu0 = (T)a.nu_in[k * NU + t];
        const T eta = (T)a.eta;
        const T v = div ? nu0 : (T(1) - eta) * nu0 + eta * sum;
        a.nu_out[k * NU + t] = (float)v;
        if (a.nu_out64) a.nu_out64[k * NU + t] = (double)v;
    }
}

__global__ void __launch_bounds__(64) best_kernel(BestArgs a)
{
    const int j = a.st->best;
    for (int k = threadIdx.x; k < a.H; k += 64) {
        float u[NU];
        if (j < 0) {
#pragma unroll
            for (int d = 0; d < NU; ++d) u[d] = a.nu[k * NU + d];
        } else if (a.U) {
#pragma unroll
            for (int d = 0; d < NU; ++d) u[d] = a.U[((long)j * a.H + k) * NU + d];
        } else {
            sample_u(a.nu + k * NU, a.sigma + (a.sigma_per_step ? k * NU : 0), a.u_max, a.key0, a.key1, (uint32_t)j,
                     (uint32_t)k, (uint32_t)a.m, u);
        }
#pragma unroll
        for (int d = 0; d < NU; ++d) a.out[k * NU + d] = u[d];
    }
}

void launch_best(const BestArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(best_kernel, dim3(1), dim3(64), 0, s, a);
}

void launch_update(const UpdateArgs &a, hipStream_t s)
{
    if (a.fp32)
        hipLaunchKernelGGL(update_kernel<float>, dim3(a.H), dim3(UB), 0, s, a, (const UpdateArgs *)nullptr,
                           (const int *)nullptr, a.m);
    else
        hipLaunchKernelGGL(update_kernel<double>, dim3(a.H), dim3(UB), 0, s, a, (const UpdateArgs *)nullptr,
                           (const int *)nullptr, a.m);
}

void launch_update_batch(const UpdateArgs *d_tab, const int *d_blk, int nblk, int m, hipStream_t s)
{
    UpdateArgs dummy = {};
    hipLaunchKernelGGL(update_kernel<double>, dim3(nblk), dim3(UB), 0, s, dummy, d_tab, d_blk, m);
}

// one workgroup per finishing request
__global__ void __launch_bounds__(256) finish_kernel(const FinishArgs *tab)
{
    const FinishArgs a = tab[blockIdx.x];
    const bool div = a.st->diverged != 0;
    const int n = a.H * NU;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float v = div ? a.nom[i] : a.nu[i];
        a.nu[i] = v;
        if (a.out) a.out[i] = v;
    }
    __syncthreads();
    if (!a.cell_nu) return;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int k = i / NU, d = i - k * NU;
        const int src = min(k + a.shift, a.H - 1);
        a.cell_nu[i] = a.nu[src * NU + d];
    }
}

void launch_finish_batch(const FinishArgs *d_tab, int n, hipStream_t s)
{
    hipLaunchKernelGGL(finish_kernel, dim3(n), dim3(256), 0, s, d_tab);
}

// ---------------------------------------------------------------------------
// single-stage kernels

__global__ void sample_kernel(const DevModel *md, const float *nu, const float *sigma, int sps, uint32_t k0,
                              uint32_t k1, int m, int K, int H, float *U, float *Z, uint32_t *words)
{
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long)K * H) return;
    const int j = (int)(id / H), k = (int)(id % H);
    float u[NU];
    sample_u(nu + k * NU, sigma + (sps ? k * NU : 0), md->u_max, k0, k1, (uint32_t)j, (uint32_t)k, (uint32_t)m, u);
    if (U) {
#pragma unroll
        for (int d = 0; d < NU; ++d) U[id * NU + d] = u[d];
    }
    if (Z) {
        float z[14];
        normals14(k0, k1, (uint32_t)j, (uint32_t)k, (uint32_t)m, z);
#pragma unroll
        for (int d = 0; d < NU; ++d) Z[id * NU + d] = z[d];
    }
    if (words) {
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            const U4 w = philox4x32_10(U4{(uint32_t)j, (uint32_t)k, q, (uint32_t)m}, k0, k1);
            words[id * 16 + 4 * q + 0] = w.x;
            words[id * 16 + 4 * q + 1] = w.y;
            words[id * 16 + 4 * q + 2] = w.z;
            words[id * 16 + 4 * q + 3] = w.w;
        }
    }
}

void launch_sample(const DevModel *md, const float *nu, const float *sigma, int sps, uint32_t k0, uint32_t k1, int m,
                   int K, int H, float *U, float *z, uint32_t *words, hipStream_t s)
{
    const long n = (long)K * H;
    hipLaunchKernelGGL(sample_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, md, nu, sigma, sps, k0, k1, m,
                       K, H, U, z, words);
}

__global__ void broadphase_kernel(const DevModel *md, const float *lo, const float *hi, int n, int ngeom,
                                  float margin, int *flags)
{
    const int np = md->n_pairs;
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long)n * np) return;
    const int i = (int)(id / np), p = (int)(id % np);
    const int ga = md->pa[p], gb = md->pb[p];
    const float *L = lo + (long)i * ngeom * 3, *Hh = hi + (long)i * ngeom * 3;
    AABB A, B;
    A.lo = v3(L[3 * ga], L[3 * ga + 1], L[3 * ga + 2]);
    A.hi = v3(Hh[3 * ga], Hh[3 * ga + 1], Hh[3 * ga + 2]);
    B.lo = v3(L[3 * gb], L[3 * gb + 1], L[3 * gb + 2]);
    B.hi = v3(Hh[3 * gb], Hh[3 * gb + 1], Hh[3 * gb + 2]);
    flags[id] = aabb_overlap(A, B, margin) ? 1 : 0;
}

void launch_broadphase(const DevModel *md, const float *lo, const float *hi, int n, int ngeom, float margin, int *flags,
                       hipStream_t s)
{
    const long tot = (long)n * MAXPAIR;
    hipLaunchKernelGGL(broadphase_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, md, lo, hi, n, ngeom,
                       margin, flags);
}

__global__ void narrowphase_kernel(const DevModel *md, const float *X, int n, float *phi, float *nrm, float *pt,
                                   float *lo, float *hi)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *x = X + (long)i * NX;
    ArmKin kin[2];
    fk_arm(*md, 0, x + XQ, kin[0]);
    fk_arm(*md, 1, x + XQ + 7, kin[1]);
    const V3 pb = v3(x[XPB], x[XPB + 1], x[XPB + 2]);
    const int np = md->n_pairs;
    // a box-shaped object: its pose, and its pairs through the box narrowphase
    // (against the table: the deepest vertex, the lowest index on ties)
    const bool box = md->obj_box != 0;
    const Rot3 R = quat_R(x[XQUAT], x[XQUAT + 1], x[XQUAT + 2], x[XQUAT + 3]);
    const V3 oh = v3(md->obj_h[0], md->obj_h[1], md->obj_h[2]);
    for (int p = 0; p < np; ++p) {
        const Shape A = geom_shape(*md, kin, pb, md->pa[p]);
        const Shape B = geom_shape(*md, kin, pb, md->pb[p]);
        Contact3 c;
        if (box && md->pa[p] == G_BALL && B.type == SH_PLANE) {
            V3 lowest = obox_vertex(pb, R, oh, 0);
            for (int k = 1; k < 8; ++k) {
                const V3 v = obox_vertex(pb, R, oh, k);
                if (v.z < lowest.z) lowest = v;
            }
            c.phi = lowest.z;
            c.n = v3(0.f, 0.f, 1.f);
            c.p = v3(lowest.x, lowest.y, 0.5f * lowest.z);
        } else if (box && md->pa[p] == G_BALL) {
            c = B.type == SH_BOX ? obox_box(pb, R, oh, B.p0, B.p1) : obox_core(pb, R, oh, B);
        } else {
            c = narrow(A, B);
        }
        const long o = (long)i * np + p;
        phi[o] = c.phi;
        if (nrm) { nrm[3 * o] = c.n.x; nrm[3 * o + 1] = c.n.y; nrm[3 * o + 2] = c.n.z; }
        if (pt) { pt[3 * o] = c.p.x; pt[3 * o + 1] = c.p.y; pt[3 * o + 2] = c.p.z; }
    }
    if (lo && hi) {
        const int ng = G_BOX + md->n_box;
        for (int g = 0; g < ng; ++g) {
            const AABB b = box && g == G_BALL ? obox_aabb(pb, R, oh) : shape_aabb(geom_shape(*md, kin, pb, g));
            const long o = ((long)i * ng + g) * 3;
            lo[o] = b.lo.x; lo[o + 1] = b.lo.y; lo[o + 2] = b.lo.z;
            hi[o] = b.hi.x; hi[o + 1] = b.hi.y; hi[o + 2] = b.hi.z;
        }
    }
}

void launch_narrowphase(const DevModel *md, const float *X, int n, float *phi, float *nrm, float *pt, float *lo,
                        float *hi, hipStream_t s)
{
    hipLaunchKernelGGL(narrowphase_kernel, dim3((n + 63) / 64), dim3(64), 0, s, md, X, n, phi, nrm, pt, lo, hi);
}

}  // namespace mppi
