// Per-sample arm dynamics in FP32, one lane per sample: forward kinematics,
// the joint-space inertia by the composite-rigid-body method, its Cholesky
// factor and the velocity-product/gravity bias by recursive Newton-Euler.
// Everything is expressed in the world frame with 3-vectors (no 6x6 spatial
// matrices): a revolute joint r is the line (a_r, o_r), a composite body is
// (mass, centre, rotational inertia about the centre).
//   CRBA (Featherstone 2008, ch. 6): H_rj = a_r . (I^c_j a_j + (c^c_j - o_r) x
//   m^c_j (a_j x (c^c_j - o_j))) for r <= j, with I^c_j the inertia of links
//   j..7 about their joint centre c^c_j (parallel-axis combination).
//   RNEA (ch. 5) with qdd = 0 gives the bias c(q, qd) (+ gravity unless the
//   arms are gravity-compensated).
#pragma once
#include <hip/hip_runtime.h>

#include "devmodel.h"

namespace mppi {

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b)
{
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 fma3(float s, V3 a, V3 b) { return V3{fmaf(s, a.x, b.x), fmaf(s, a.y, b.y), fmaf(s, a.z, b.z)}; }

// Hardware reciprocal and square root (v_rcp_f32, v_sqrt_f32: about 1 ulp;
// a denormal argument flushes to zero) in place of the library sequences
// that rescale denormal arguments: every argument they take here is a normal
// float (masses, squared lengths of links, pivots of the contact rows) or
// sits behind a threshold well above the denormal range.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Symmetric 3x3: xx yy zz xy xz yz
struct S3 {
    float xx, yy, zz, xy, xz, yz;
};
__device__ __forceinline__ V3 mul(const S3 &I, V3 v)
{
    return V3{I.xx * v.x + I.xy * v.y + I.xz * v.z, I.xy * v.x + I.yy * v.y + I.yz * v.z,
              I.xz * v.x + I.yz * v.y + I.zz * v.z};
}
// I += m ((d.d) 1 - d d^T)  (parallel axis)
__device__ __forceinline__ void add_pa(S3 &I, float m, V3 d)
{
    const float dd = dot(d, d);
    I.xx += m * (dd - d.x * d.x);
    I.yy += m * (dd - d.y * d.y);
    I.zz += m * (dd - d.z * d.z);
    I.xy -= m * d.x * d.y;
    I.xz -= m * d.x * d.z;
    I.yz -= m * d.y * d.z;
}

// kinematics of one arm: joint origins o[0..6], tip o[7], joint axes, link z
// axes, and the x and y axes of the last link's frame (the pad's orientation)
struct ArmKin {
    V3 o[NJ + 1];
    V3 a[NJ];
    V3 z[NJ];
    V3 x7, y7;
};

// columns j1, j2 of R after a rotation by (c, s) about the third axis
template <int J1, int J2>
__device__ __forceinline__ void rot_cols(float R[3][3], float c, float s)
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float c1 = R[r][J1], c2 = R[r][J2];
        R[r][J1] = c * c1 + s * c2;
        R[r][J2] = c * c2 - s * c1;
    }
}

__device__ inline void fk_arm(const DevModel &md, int arm, const float *q, ArmKin &k)
{
    float R[3][3] = {{md.base_cs[arm][0], -md.base_cs[arm][1], 0.f},
                     {md.base_cs[arm][1], md.base_cs[arm][0], 0.f},
                     {0.f, 0.f, 1.f}};
    V3 o = v3(md.base_pos[arm][0], md.base_pos[arm][1], md.base_pos[arm][2]);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        // rotating about local axis ax mixes the other two columns of R; the
        // axis is uniform across the launch, so the branch is too
        const int ax = md.axes[i];
        k.o[i] = o;
        float s, c;
        sincosf(q[i], &s, &c);
        if (ax == 0) {
            k.a[i] = v3(R[0][0], R[1][0], R[2][0]);
            rot_cols<1, 2>(R, c, s);
        } else if (ax == 1) {
            k.a[i] = v3(R[0][1], R[1][1], R[2][1]);
            rot_cols<2, 0>(R, c, s);
        } else {
            k.a[i] = v3(R[0][2], R[1][2], R[2][2]);
            rot_cols<0, 1>(R, c, s);
        }
        k.z[i] = v3(R[0][2], R[1][2], R[2][2]);
        o = fma3(md.link_len[i], k.z[i], o);
    }
    k.o[NJ] = o;
    k.x7 = v3(R[0][0], R[1][0], R[2][0]);
    k.y7 = v3(R[0][1], R[1][1], R[2][1]);
}

// packed lower triangle index of (r, c), r >= c
__device__ __forceinline__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

// Mt = M(q) + diag(diag_add), packed lower triangle (28 floats)
__device__ inline void crba_arm(const DevModel &md, int arm, const ArmKin &k, float Mt[28])
{
    float mc = 0.f;
    V3 cc = v3(0.f, 0.f, 0.f);
    S3 Ic = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = NJ - 1; j >= 0; --j) {
        const float mi = md.m[arm][j];
        const V3 ci = fma3(0.5f * md.link_len[j], k.z[j], k.o[j]);
        const float mn = mi + mc;
        const V3 ccn = frcp(mn) * (mi * ci + mc * cc);
        // link inertia about its own centre: Ix (1 - z z^T) + Iz z z^T
        const float ix = md.Ix[arm][j], dz = md.Iz[arm][j] - ix;
        const V3 z = k.z[j];
        S3 In = {ix + dz * z.x * z.x, ix + dz * z.y * z.y, ix + dz * z.z * z.z,
                 dz * z.x * z.y,      dz * z.x * z.z,      dz * z.y * z.z};
        add_pa(In, mi, ci - ccn);
        In.xx += Ic.xx; In.yy += Ic.yy; In.zz += Ic.zz;
        In.xy += Ic.xy; In.xz += Ic.xz; In.yz += Ic.yz;
        add_pa(In, mc, cc - ccn);
        mc = mn;
        cc = ccn;
        Ic = In;
        // column j: momentum of the composite under unit rate of joint j
        const V3 L = mc * cross(k.a[j], cc - k.o[j]);
        const V3 Hc = mul(Ic, k.a[j]);
#pragma unroll
        for (int r = 0; r <= j; ++r) Mt[tri(j, r)] = dot(k.a[r], Hc + cross(cc - k.o[r], L));
        Mt[tri(j, j)] += md.diag_add;
    }
}

// cos(a / 2) and sin(a / 2) / a for a rotation angle a >= 0 (the exponential
// map of a rotation vector of length a).  Per substep a is h |w|, far below
// 1 rad: there the Taylor series (even in a, truncated after the a^8 term;
// remainder below 3e-10 for a <= 1) replaces the range-reduced library call.
__device__ __forceinline__ void half_angle_sincos(float a, float &c, float &s_over_a)
{
#pragma clang fp contract(off)
    if (a <= 1.0f) {
        const float x2 = 0.25f * a * a;  // (a / 2)^2
        c = fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 1.0f / 40320.0f, -1.0f / 720.0f), 1.0f / 24.0f), -0.5f), 1.0f);
        const float sx = fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f),
                                        -1.0f / 6.0f),
                              1.0f);  // sin(a / 2) / (a / 2)
        s_over_a = 0.5f * sx;
    } else {
        float sn, cs;
        sincosf(0.5f * a, &sn, &cs);
        c = cs;
        s_over_a = sn / a;
    }
}

// in-place Cholesky of a packed SPD 7x7 (lower); pivots stay > 0 because
// the armature is on the diagonal.  The diagonal slots receive 1 / L_jj, so
// that the solves multiply instead of dividing.
__device__ inline void chol7(float L[28])
{
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        float d = L[tri(j, j)];
#pragma unroll
        for (int k2 = 0; k2 < j; ++k2) d -= L[tri(j, k2)] * L[tri(j, k2)];
        const float inv = __builtin_amdgcn_rsqf(d);  // hardware 1 / sqrt (about 1 ulp)
        L[tri(j, j)] = inv;
#pragma unroll
        for (int i = j + 1; i < NJ; ++i) {
            float v = L[tri(i, j)];
#pragma unroll
            for (int k2 = 0; k2 < j; ++k2) v -= L[tri(i, k2)] * L[tri(j, k2)];
            L[tri(i, j)] = v * inv;
        }
    }
}

// x = (L L^T)^-1 b, in place (L from chol7: reciprocal diagonal)
__device__ inline void chol7_solve(const float L[28], float x[NJ])
{
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        float v = x[i];
#pragma unroll
        for (int k2 = 0; k2 < i; ++k2) v -= L[tri(i, k2)] * x[k2];
        x[i] = v * L[tri(i, i)];
    }
#pragma unroll
    for (int i = NJ - 1; i >= 0; --i) {
        float v = x[i];
#pragma unroll
        for (int k2 = i + 1; k2 < NJ; ++k2) v -= L[tri(k2, i)] * x[k2];
        x[i] = v * L[tri(i, i)];
    }
}

// bias torques c(q, qd) (+ gravity when gravity != 0), qdd = 0.  The forward
// pass keeps only each link's force m a_c and moment I al + w x I w about its
// centre; the backward pass accumulates them towards the base.
__device__ inline void rnea_bias_arm(const DevModel &md, int arm, const ArmKin &k, const float *qd, bool gravity,
                                     float tau[NJ])
{
    V3 f[NJ], nm[NJ];
    V3 wp = v3(0.f, 0.f, 0.f), alp = v3(0.f, 0.f, 0.f);
    V3 ao = v3(0.f, 0.f, gravity ? md.g : 0.f);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        if (i > 0) {
            const V3 d = k.o[i] - k.o[i - 1];
            ao = ao + cross(alp, d) + cross(wp, cross(wp, d));
        }
        const V3 w = fma3(qd[i], k.a[i], wp);
        const V3 al = fma3(qd[i], cross(wp, k.a[i]), alp);
        const V3 z = k.z[i];
        const V3 dc = 0.5f * md.link_len[i] * z;
        const V3 ac = ao + cross(al, dc) + cross(w, cross(w, dc));
        const float ix = md.Ix[arm][i], dz = md.Iz[arm][i] - ix;
        // I v = ix v + (iz - ix) (z . v) z
        const V3 Ia = fma3(dz * dot(z, al), z, ix * al);
        const V3 Iw = fma3(dz * dot(z, w), z, ix * w);
        f[i] = md.m[arm][i] * ac;
        nm[i] = Ia + cross(w, Iw);
        wp = w;
        alp = al;
    }
    V3 F = v3(0.f, 0.f, 0.f), N = v3(0.f, 0.f, 0.f);
#pragma unroll
    for (int i = NJ - 1; i >= 0; --i) {
        const V3 z = k.z[i];
        const V3 dc = 0.5f * md.link_len[i] * z;
        const V3 dn = md.link_len[i] * z;
        N = nm[i] + cross(dc, f[i]) + N + cross(dn, F);
        F = f[i] + F;
        tau[i] = dot(k.a[i], N);
    }
}

}  // namespace mppi
