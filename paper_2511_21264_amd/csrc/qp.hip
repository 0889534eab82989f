// QP smoothing of sampled joint-velocity sequences (Alg. 1: the projection
// of every sample after the sampling step; Eqs. proj_cost and proj_bounds
// with bounds on the joint trajectory and its first three derivatives).
//
// Each joint of each sample is a QP over the horizon in the H control-step
// velocities; the bounds are on A v with A = [I; D1; D2; L] (identity, first
// and second differences, prefix sums), all in velocity units.  The solver is
// a fixed number of over-relaxed ADMM iterations:
//     v  = P (v~ + rho A^T (z - w)),   P = (I + rho A^T A)^-1
//        (evaluated as v~ + rho P A^T (z - w - A v~))
//     a  = alpha A v + (1 - alpha) z
//     z' = clip(a + w, lo, hi);   w += a - z';   z = z'
// from z = clip(A v~), w = 0; the output is v clipped to the velocity box.
//
// Mapping: one workgroup per sample, one wave per joint (14 waves), one
// horizon step per lane for H <= 64 and two (steps k and k + 64) for
// H <= 128.  A v and A^T y are DPP whole-wave shifts and
// scans (neighbour differences, prefix and suffix sums).  The dense product
// with P, the same for every joint and sample, is one 64 x 64 by 64 x 16
// product per iteration on FP32 MFMA: the waves publish their right-hand
// sides to LDS, waves 0..4 NH - 1 each hold a 16-row block of P in registers
// for the whole kernel and multiply (16 NH steps of 16x16x4), and every wave
// reads its column of the result back.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "team.h"

namespace mppi {

namespace {

__device__ __forceinline__ float clipf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// Wave-wide shifts and scans without an LDS trip: DPP shifts within 16-lane
// rows (lanes whose source lies outside the row read 0), then the row totals
// carried across rows (DPP row broadcasts for the prefix sum, v_readlane for
// the suffix sum).  Every lane of the wave is active wherever these run.
template <int S>
__device__ __forceinline__ float shr_row(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x110 + S, 0xF, 0xF, true));
}
template <int S>
__device__ __forceinline__ float shl_row(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x100 + S, 0xF, 0xF, true));
}
// whole-wave shifts by one lane (DPP wave_shr:1 / wave_shl:1): lane k reads
// lane k - 1 / k + 1; lane 0 / 63 reads 0
__device__ __forceinline__ float wave_shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float wave_shl1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
template <int L>
__device__ __forceinline__ float lane_of(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
}

// inclusive prefix sum over the wave: scans within the rows, then the row
// totals carried by DPP row_bcast:15 (lane 15 of each row into the next row;
// rows 1 and 3 take it) and row_bcast:31 (lane 31 into rows 2 and 3); lanes
// of the rows a broadcast leaves out add 0
__device__ __forceinline__ float prefix64(float x, int)
{
    x += shr_row<1>(x);
    x += shr_row<2>(x);
    x += shr_row<4>(x);
    x += shr_row<8>(x);
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xA, 0xF, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xC, 0xF, true));
    return x;
}
// inclusive suffix sum over the wave
__device__ __forceinline__ float suffix64(float x, int k)
{
    x += shl_row<1>(x);
    x += shl_row<2>(x);
    x += shl_row<4>(x);
    x += shl_row<8>(x);
    const float t1 = lane_of<16>(x), t2 = lane_of<32>(x), t3 = lane_of<48>(x);
    const int row = k >> 4;
    const float off = row == 3 ? 0.f : (row == 2 ? t3 : (row == 1 ? t3 + t2 : (t3 + t2) + t1));
    return x + off;
}

// A v for the sequence held one element per lane (lane k: step k); rows that
// do not exist (first difference at k = 0, second at k < 2, any k >= H) are 0
__device__ __forceinline__ void apply_A(float v, int k, bool act, float &aI, float &a1, float &a2, float &aL)
{
    const float x = act ? v : 0.f;
    const float vm1 = wave_shr1(x), vm2 = wave_shr1(vm1);  // 0 before step 0
    aI = x;
    a1 = (act && k >= 1) ? x - vm1 : 0.f;
    a2 = (act && k >= 2) ? (x - 2.f * vm1) + vm2 : 0.f;
    const float p = prefix64(x, k);
    aL = act ? p : 0.f;  // lanes past the horizon hold no row (their w must stay 0)
}

// A^T y at lane k (y of absent rows are 0): y_I + (y1_k - y1_{k+1}) +
// (y2_k - 2 y2_{k+1} + y2_{k+2}) + sum_{i >= k} yL_i
__device__ __forceinline__ float apply_At(float yI, float y1, float y2, float yL, int k)
{
    // the shifts read 0 past the end of the wave
    const float y1n = wave_shl1(y1), y2n = wave_shl1(y2), y2nn = wave_shl1(y2n);
    return yI + (y1 - y1n) + ((y2 - 2.f * y2n) + y2nn) + suffix64(yL, k);
}

// Two steps per lane (64 < H <= 128): lane k holds steps k (half 0) and
// k + 64 (half 1); the halves join at the boundary through v_readlane of
// lanes 63 and 0.
__device__ __forceinline__ void apply_A2(const float v[2], int k, const bool act[2], float aI[2], float a1[2],
                                         float a2[2], float aL[2])
{
    const float x0 = act[0] ? v[0] : 0.f, x1 = act[1] ? v[1] : 0.f;
    const float e62 = lane_of<62>(x0), e63 = lane_of<63>(x0);
    const float u0 = wave_shr1(x0), w0 = wave_shr1(u0), u1 = wave_shr1(x1), w1 = wave_shr1(u1);
    const float vm1_0 = u0, vm2_0 = w0;                                  // used for k >= 1 / k >= 2
    const float vm1_1 = k >= 1 ? u1 : e63, vm2_1 = k >= 2 ? w1 : (k == 1 ? e63 : e62);
    aI[0] = x0;
    aI[1] = x1;
    a1[0] = (act[0] && k >= 1) ? x0 - vm1_0 : 0.f;
    a2[0] = (act[0] && k >= 2) ? (x0 - 2.f * vm1_0) + vm2_0 : 0.f;
    a1[1] = act[1] ? x1 - vm1_1 : 0.f;
    a2[1] = act[1] ? (x1 - 2.f * vm1_1) + vm2_1 : 0.f;
    const float p0 = prefix64(x0, k);
    const float p1 = prefix64(x1, k) + lane_of<63>(p0);
    aL[0] = act[0] ? p0 : 0.f;
    aL[1] = act[1] ? p1 : 0.f;
}

__device__ __forceinline__ void apply_At2(const float yI[2], const float y1[2], const float y2[2], const float yL[2],
                                          int k, float out[2])
{
    const float b10 = lane_of<0>(y1[1]), b20 = lane_of<0>(y2[1]), b21 = lane_of<1>(y2[1]);
    const float s1_0 = wave_shl1(y1[0]), s2_0 = wave_shl1(y2[0]), s22_0 = wave_shl1(s2_0);
    const float s1_1 = wave_shl1(y1[1]), s2_1 = wave_shl1(y2[1]), s22_1 = wave_shl1(s2_1);
    // half 0: steps k + 1, k + 2 may lie in half 1
    const float y1n0 = k + 1 < 64 ? s1_0 : b10, y2n0 = k + 1 < 64 ? s2_0 : b20;
    const float y2nn0 = k + 2 < 64 ? s22_0 : (k == 62 ? b20 : b21);
    // half 1: nothing past step 127
    const float y1n1 = s1_1, y2n1 = s2_1, y2nn1 = s22_1;  // the shifts read 0 past lane 63
    const float q1 = suffix64(yL[1], k);
    const float q0 = suffix64(yL[0], k) + lane_of<0>(q1);
    out[0] = yI[0] + (y1[0] - y1n0) + ((y2[0] - 2.f * y2n0) + y2nn0) + q0;
    out[1] = yI[1] + (y1[1] - y1n1) + ((y2[1] - 2.f * y2n1) + y2nn1) + q1;
}

}  // namespace

// NH horizon steps per lane (1: H <= 64, 2: H <= 128); waves 0 .. 4 NH - 1
// hold the 16-row blocks of P.  FULL: H = 64 NH, so every lane holds a step
// and the masks of absent steps fold away.
template <int NH, bool FULL>
__global__ void __launch_bounds__(14 * 64) project_kernel(ProjectArgs a)
{
    constexpr int QS = 64 * NH + 4;  // LDS row stride of the right-hand sides and results (floats)
    constexpr int NST = 16 * NH;     // k-steps of the product
    __shared__ __align__(16) float R[16][QS];  // right-hand sides, one row per joint (rows 14, 15: zero)
    __shared__ __align__(16) float V[16][QS];  // P times them
    const int H = a.H, S = a.S;
    const int j = blockIdx.x;
    const int d = threadIdx.x >> 6, k = threadIdx.x & 63;
    bool act[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) act[h] = FULL || k + 64 * h < H;  // FULL: H = 64 NH, every lane holds a step
    if (d < 2) {
#pragma unroll
        for (int h = 0; h < NH; ++h) R[14 + d][k + 64 * h] = 0.f;
    }
    // waves 0 .. 4 NH - 1 keep rows 16 w .. 16 w + 15 of P as MFMA A operands:
    // pa[s] = P[16 w + l % 16][4 s + l / 16]
    const int lr = k & 15, lq = k >> 4;
    float pa[NST];
#pragma unroll
    for (int st = 0; st < NST; ++st) {
        const int row = 16 * d + lr, col = 4 * st + lq;
        pa[st] = (d < 4 * NH && row < H && col < H) ? a.P[row * S + col] : 0.f;
    }
    const float *x0 = a.x0 + (a.x0_shared ? 0 : (long)j * NX);
    const float q0 = x0[XQDES + d];
    float vt[NH], loI[NH], hiI[NH], lo1[NH], hi1[NH], lo2[NH], hi2[NH], loL[NH], hiL[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const int st = k + 64 * h;  // this lane's step in half h
        vt[h] = 0.f;
        if (act[h]) {
            if (a.U_in) {
                vt[h] = a.U_in[((long)j * H + st) * NU + d];
            } else {
                const float z = normal_joint(a.key0, a.key1, (uint32_t)j, (uint32_t)st, (uint32_t)a.m, d);
                vt[h] = fmaf(a.sigma[(a.sigma_per_step ? st * NU : 0) + d], z, a.nu[st * NU + d]);
            }
        }
        // the bounds of the four rows this lane holds (absent rows: [0, 0])
        loI[h] = act[h] ? -a.u_max : 0.f;
        hiI[h] = act[h] ? a.u_max : 0.f;
        lo1[h] = (act[h] && st >= 1) ? -a.dacc : 0.f;
        hi1[h] = (act[h] && st >= 1) ? a.dacc : 0.f;
        lo2[h] = (act[h] && st >= 2) ? -a.djerk : 0.f;
        hi2[h] = (act[h] && st >= 2) ? a.djerk : 0.f;
        loL[h] = act[h] ? (a.pos_lo[d] - q0) / a.dt : 0.f;
        hiL[h] = act[h] ? (a.pos_hi[d] - q0) / a.dt : 0.f;
    }
    // A v~ is kept: the v-update is evaluated as v~ + rho P A^T (z - w - A v~),
    // the same value as P (v~ + rho A^T (z - w)) since P (I + rho A^T A) = I,
    // but without the cancellation of two large terms (the prefix-sum rows
    // of rho A^T A v~ are hundreds of times larger than v~ at H = 64)
    float tI[NH], t1[NH], t2[NH], tL[NH];
    if constexpr (NH == 1)
        apply_A(vt[0], k, act[0], tI[0], t1[0], t2[0], tL[0]);
    else
        apply_A2(vt, k, act, tI, t1, t2, tL);
    float zI[NH], z1[NH], z2[NH], zL[NH], wI[NH], w1[NH], w2[NH], wL[NH], v[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        zI[h] = clipf(tI[h], loI[h], hiI[h]);
        z1[h] = clipf(t1[h], lo1[h], hi1[h]);
        z2[h] = clipf(t2[h], lo2[h], hi2[h]);
        zL[h] = clipf(tL[h], loL[h], hiL[h]);
        wI[h] = w1[h] = w2[h] = wL[h] = 0.f;
        v[h] = vt[h];
    }
    const float rho = a.rho, alpha = a.alpha, beta = 1.f - a.alpha;
    const int nst = (H + 3) >> 2;  // k-steps of the product that touch columns < H
    for (int it = 0; it < a.iters; ++it) {
        float yI[NH], y1[NH], y2[NH], yL[NH], rhs[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            yI[h] = (zI[h] - wI[h]) - tI[h];
            y1[h] = (z1[h] - w1[h]) - t1[h];
            y2[h] = (z2[h] - w2[h]) - t2[h];
            yL[h] = (zL[h] - wL[h]) - tL[h];
        }
        if constexpr (NH == 1)
            rhs[0] = apply_At(yI[0], y1[0], y2[0], yL[0], k);
        else
            apply_At2(yI, y1, y2, yL, k, rhs);
#pragma unroll
        for (int h = 0; h < NH; ++h) R[d][k + 64 * h] = act[h] ? rho * rhs[h] : 0.f;
        __syncthreads();
        if (d < 4 * NH) {
            // V[16 d + row][joint] = sum_i P[16 d + row][i] R[joint][i]; result
            // element e of lane l is row 4 (l / 16) + e, joint l % 16
            typedef float f4 __attribute__((ext_vector_type(4)));
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            if (nst == NST) {  // full horizon: one unguarded chain
#pragma unroll
                for (int st = 0; st < NST; ++st)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[st], R[lr][4 * st + lq], acc, 0, 0, 0);
            } else {
#pragma unroll
                for (int st = 0; st < NST; ++st)
                    if (st < nst) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[st], R[lr][4 * st + lq], acc, 0, 0, 0);
            }
            *reinterpret_cast<f4 *>(&V[lr][16 * d + 4 * lq]) = acc;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < NH; ++h) v[h] = act[h] ? vt[h] + V[d][k + 64 * h] : 0.f;
        float aI[NH], a1[NH], a2[NH], aL[NH];
        if constexpr (NH == 1)
            apply_A(v[0], k, act[0], aI[0], a1[0], a2[0], aL[0]);
        else
            apply_A2(v, k, act, aI, a1, a2, aL);
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            aI[h] = fmaf(alpha, aI[h], beta * zI[h]);
            a1[h] = fmaf(alpha, a1[h], beta * z1[h]);
            a2[h] = fmaf(alpha, a2[h], beta * z2[h]);
            aL[h] = fmaf(alpha, aL[h], beta * zL[h]);
            float zn = clipf(aI[h] + wI[h], loI[h], hiI[h]);
            wI[h] += aI[h] - zn;
            zI[h] = zn;
            zn = clipf(a1[h] + w1[h], lo1[h], hi1[h]);
            w1[h] += a1[h] - zn;
            z1[h] = zn;
            zn = clipf(a2[h] + w2[h], lo2[h], hi2[h]);
            w2[h] += a2[h] - zn;
            z2[h] = zn;
            zn = clipf(aL[h] + wL[h], loL[h], hiL[h]);
            wL[h] += aL[h] - zn;
            zL[h] = zn;
        }
    }
#pragma unroll
    for (int h = 0; h < NH; ++h)
        if (act[h]) a.U_out[((long)j * H + k + 64 * h) * NU + d] = clipf(v[h], -a.u_max, a.u_max);
}

void launch_project(const ProjectArgs &a, hipStream_t s)
{
    if (a.H <= 64) {
        if (a.H == 64)
            hipLaunchKernelGGL((project_kernel<1, true>), dim3(a.K), dim3(14 * 64), 0, s, a);
        else
            hipLaunchKernelGGL((project_kernel<1, false>), dim3(a.K), dim3(14 * 64), 0, s, a);
    } else {
        if (a.H == 128)
            hipLaunchKernelGGL((project_kernel<2, true>), dim3(a.K), dim3(14 * 64), 0, s, a);
        else
            hipLaunchKernelGGL((project_kernel<2, false>), dim3(a.K), dim3(14 * 64), 0, s, a);
    }
}

}  // namespace mppi
