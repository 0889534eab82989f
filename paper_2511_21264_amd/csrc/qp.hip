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
// horizon step per lane (H <= 64).  A v and A^T y are wave-wide shuffles and
// scans (neighbour differences, prefix and suffix sums).  The dense product
// with P, the same for every joint and sample, is one 64 x 64 by 64 x 16
// product per iteration on FP32 MFMA: the waves publish their right-hand
// sides to LDS, waves 0..3 each hold a 16-row block of P in registers for
// the whole kernel and multiply (16 steps of 16x16x4), and every wave reads
// its column of the result back.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "team.h"

namespace mppi {

namespace {

__device__ __forceinline__ float clipf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// Wave-wide scans without an LDS trip: DPP shifts within 16-lane rows (lanes
// whose source lies outside the row read 0), then the row totals from
// v_readlane.  Every lane of the wave is active wherever these run.
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
template <int L>
__device__ __forceinline__ float lane_of(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
}

// inclusive prefix sum over the wave
__device__ __forceinline__ float prefix64(float x, int k)
{
    x += shr_row<1>(x);
    x += shr_row<2>(x);
    x += shr_row<4>(x);
    x += shr_row<8>(x);
    const float t0 = lane_of<15>(x), t1 = lane_of<31>(x), t2 = lane_of<47>(x);
    const int row = k >> 4;
    const float off = row == 0 ? 0.f : (row == 1 ? t0 : (row == 2 ? t0 + t1 : (t0 + t1) + t2));
    return x + off;
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
    const float vm1 = __shfl_up(x, 1), vm2 = __shfl_up(x, 2);  // masked below where they wrap
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
    // every lane takes part in each shuffle; the end of the wave is masked after
    const float t1 = __shfl_down(y1, 1), t2 = __shfl_down(y2, 1), t3 = __shfl_down(y2, 2);
    const float y1n = k + 1 < 64 ? t1 : 0.f, y2n = k + 1 < 64 ? t2 : 0.f, y2nn = k + 2 < 64 ? t3 : 0.f;
    return yI + (y1 - y1n) + ((y2 - 2.f * y2n) + y2nn) + suffix64(yL, k);
}

}  // namespace

constexpr int QS = 68;  // LDS row stride of the right-hand sides and results (floats)

__global__ void __launch_bounds__(14 * 64) project_kernel(ProjectArgs a)
{
    __shared__ __align__(16) float R[16][QS];  // right-hand sides, one row per joint (rows 14, 15: zero)
    __shared__ __align__(16) float V[16][QS];  // P times them
    const int H = a.H, S = a.S;
    const int j = blockIdx.x;
    const int d = threadIdx.x >> 6, k = threadIdx.x & 63;
    const bool act = k < H;
    if (d < 2) R[14 + d][k] = 0.f;
    // waves 0..3 keep rows 16 w .. 16 w + 15 of P as MFMA A operands:
    // pa[s] = P[16 w + l % 16][4 s + l / 16]
    const int lr = k & 15, lq = k >> 4;
    float pa[16];
#pragma unroll
    for (int st = 0; st < 16; ++st) {
        const int row = 16 * d + lr, col = 4 * st + lq;
        pa[st] = (d < 4 && row < H && col < H) ? a.P[row * S + col] : 0.f;
    }
    const float *x0 = a.x0 + (a.x0_shared ? 0 : (long)j * NX);
    const float q0 = x0[XQDES + d];
    float vt = 0.f;
    if (act) {
        if (a.U_in) {
            vt = a.U_in[((long)j * H + k) * NU + d];
        } else {
            const float z = normal_joint(a.key0, a.key1, (uint32_t)j, (uint32_t)k, (uint32_t)a.m, d);
            vt = fmaf(a.sigma[(a.sigma_per_step ? k * NU : 0) + d], z, a.nu[k * NU + d]);
        }
    }
    // the bounds of the four rows this lane holds (absent rows: [0, 0])
    const float loI = act ? -a.u_max : 0.f, hiI = act ? a.u_max : 0.f;
    const float lo1 = (act && k >= 1) ? -a.dacc : 0.f, hi1 = (act && k >= 1) ? a.dacc : 0.f;
    const float lo2 = (act && k >= 2) ? -a.djerk : 0.f, hi2 = (act && k >= 2) ? a.djerk : 0.f;
    const float loL = act ? (a.pos_lo[d] - q0) / a.dt : 0.f, hiL = act ? (a.pos_hi[d] - q0) / a.dt : 0.f;
    // A v~ is kept: the v-update is evaluated as v~ + rho P A^T (z - w - A v~),
    // the same value as P (v~ + rho A^T (z - w)) since P (I + rho A^T A) = I,
    // but without the cancellation of two large terms (the prefix-sum rows
    // of rho A^T A v~ are hundreds of times larger than v~ at H = 64)
    float tI, t1, t2, tL;
    apply_A(vt, k, act, tI, t1, t2, tL);
    float zI = clipf(tI, loI, hiI);
    float z1 = clipf(t1, lo1, hi1);
    float z2 = clipf(t2, lo2, hi2);
    float zL = clipf(tL, loL, hiL);
    float wI = 0.f, w1 = 0.f, w2 = 0.f, wL = 0.f;
    const float rho = a.rho, alpha = a.alpha, beta = 1.f - a.alpha;
    const int nst = (H + 3) >> 2;  // k-steps of the product that touch columns < H
    float v = vt;
    for (int it = 0; it < a.iters; ++it) {
        const float rhs = rho * apply_At((zI - wI) - tI, (z1 - w1) - t1, (z2 - w2) - t2, (zL - wL) - tL, k);
        R[d][k] = act ? rhs : 0.f;
        __syncthreads();
        if (d < 4) {
            // V[16 d + row][joint] = sum_i P[16 d + row][i] R[joint][i]; result
            // element e of lane l is row 4 (l / 16) + e, joint l % 16
            typedef float f4 __attribute__((ext_vector_type(4)));
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < 16; ++st)
                if (st < nst) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[st], R[lr][4 * st + lq], acc, 0, 0, 0);
            *reinterpret_cast<f4 *>(&V[lr][16 * d + 4 * lq]) = acc;
        }
        __syncthreads();
        v = act ? vt + V[d][k] : 0.f;
        float aI, a1, a2, aL;
        apply_A(v, k, act, aI, a1, a2, aL);
        aI = fmaf(alpha, aI, beta * zI);
        a1 = fmaf(alpha, a1, beta * z1);
        a2 = fmaf(alpha, a2, beta * z2);
        aL = fmaf(alpha, aL, beta * zL);
        float zn = clipf(aI + wI, loI, hiI);
        wI += aI - zn;
        zI = zn;
        zn = clipf(a1 + w1, lo1, hi1);
        w1 += a1 - zn;
        z1 = zn;
        zn = clipf(a2 + w2, lo2, hi2);
        w2 += a2 - zn;
        z2 = zn;
        zn = clipf(aL + wL, loL, hiL);
        wL += aL - zn;
        zL = zn;
    }
    if (act) a.U_out[((long)j * H + k) * NU + d] = clipf(v, -a.u_max, a.u_max);
}

void launch_project(const ProjectArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(project_kernel, dim3(a.K), dim3(14 * 64), 0, s, a);
}

}  // namespace mppi
