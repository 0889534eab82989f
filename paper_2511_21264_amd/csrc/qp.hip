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
// scans (neighbour differences, prefix and suffix sums); the dense product
// with P, which is the same for every joint and sample, reads P from LDS
// (rows padded to S floats) and the wave's right-hand side broadcast from
// LDS, four columns per load.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "team.h"

namespace mppi {

namespace {

__device__ __forceinline__ float clipf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// A v for the sequence held one element per lane (lane k: step k); rows that
// do not exist (first difference at k = 0, second at k < 2, any k >= H) are 0
__device__ __forceinline__ void apply_A(float v, int k, bool act, float &aI, float &a1, float &a2, float &aL)
{
    const float vm1 = __shfl_up(v, 1), vm2 = __shfl_up(v, 2);
    aI = act ? v : 0.f;
    a1 = (act && k >= 1) ? v - vm1 : 0.f;
    a2 = (act && k >= 2) ? (v - 2.f * vm1) + vm2 : 0.f;
    float x = act ? v : 0.f;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const float y = __shfl_up(x, s);
        if (k >= s) x += y;
    }
    aL = act ? x : 0.f;  // lanes past the horizon hold no row (their w must stay 0)
}

// A^T y at lane k (y of absent rows are 0): y_I + (y1_k - y1_{k+1}) +
// (y2_k - 2 y2_{k+1} + y2_{k+2}) + sum_{i >= k} yL_i
__device__ __forceinline__ float apply_At(float yI, float y1, float y2, float yL, int k)
{
    // every lane takes part in each shuffle; the end of the wave is masked after
    const float t1 = __shfl_down(y1, 1), t2 = __shfl_down(y2, 1), t3 = __shfl_down(y2, 2);
    const float y1n = k + 1 < 64 ? t1 : 0.f;
    const float y2n = k + 1 < 64 ? t2 : 0.f;
    const float y2nn = k + 2 < 64 ? t3 : 0.f;
    float x = yL;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const float y = __shfl_down(x, s);
        if (k + s < 64) x += y;
    }
    return yI + (y1 - y1n) + ((y2 - 2.f * y2n) + y2nn) + x;
}

}  // namespace

__global__ void __launch_bounds__(14 * 64) project_kernel(ProjectArgs a)
{
    extern __shared__ float lds[];
    const int H = a.H, S = a.S;
    float *P = lds;
    float *R = lds + H * S;  // one right-hand side per wave
    for (int i = threadIdx.x; i < H * S; i += blockDim.x) P[i] = a.P[i];
    __syncthreads();
    const int j = blockIdx.x;
    const int d = threadIdx.x >> 6, k = threadIdx.x & 63;
    float *r = R + 64 * d;
    const bool act = k < H;
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
    const int H4 = (H + 3) & ~3;
    const float *prow = P + (act ? k : 0) * S;
    float v = vt;
    for (int it = 0; it < a.iters; ++it) {
        const float rhs = rho * apply_At((zI - wI) - tI, (z1 - w1) - t1, (z2 - w2) - t2, (zL - wL) - tL, k);
        r[k] = act ? rhs : 0.f;
        wave_lds_sync();
        float acc = 0.f;
        for (int i = 0; i < H4; i += 4) {
            const float4 p4 = *reinterpret_cast<const float4 *>(prow + i);
            const float4 r4 = *reinterpret_cast<const float4 *>(r + i);
            acc = fmaf(p4.x, r4.x, acc);
            acc = fmaf(p4.y, r4.y, acc);
            acc = fmaf(p4.z, r4.z, acc);
            acc = fmaf(p4.w, r4.w, acc);
        }
        v = act ? vt + acc : 0.f;
        wave_lds_sync();  // every lane has read r before the next iteration writes it
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
    const size_t lds = (size_t)(a.H * a.S + 14 * 64) * sizeof(float);
    hipLaunchKernelGGL(project_kernel, dim3(a.K), dim3(14 * 64), lds, s, a);
}

}  // namespace mppi
