// Collision geometry and narrowphase in FP32, one lane per sample.
//
// Geoms: the ball (sphere), the table (plane z = 0), arm link capsules
// (segment joint i -> joint i+1, links 1..6), the pad sphere at the tip of
// link 7, static axis-aligned boxes.  Every candidate pair gives one contact
// (phi, n, p): phi the signed distance, n the unit normal from geom B towards
// geom A, p midway between the two closest surface points.  The same signed
// distances feed the collision cost of Eq. collision_cost.
//   sphere/capsule vs sphere/capsule: closest points of the cores (point or
//     segment), clamped-parameter solution of the 2x2 normal equations;
//   vs plane: the core point with the lower z (first end on ties);
//   vs box: the core point minimising the box's signed distance, found on a
//     segment by bisection on the sign of the derivative (the distance is
//     convex along the segment); both ends of a flat minimising interval
//     are located and their midpoint is taken.
#pragma once
#include "dynamics.h"

namespace mppi {

enum : int { SH_SPHERE = 0, SH_CAPSULE = 1, SH_PLANE = 2, SH_BOX = 3 };

struct Shape {
    int type;
    V3 p0, p1;  // sphere: p0 centre; capsule: segment; box: p0 centre, p1 half extents
    float r;
};

__device__ __forceinline__ Shape geom_shape(const DevModel &md, const ArmKin kin[2], V3 pball, int gid)
{
    Shape s;
    if (gid == G_BALL) {
        s.type = SH_SPHERE; s.p0 = pball; s.p1 = pball; s.r = md.ball_r;
    } else if (gid == G_TABLE) {
        s.type = SH_PLANE; s.p0 = v3(0.f, 0.f, 0.f); s.p1 = s.p0; s.r = 0.f;
    } else if (gid >= G_BOX) {
        const int b = gid - G_BOX;
        s.type = SH_BOX;
        s.p0 = v3(md.box_c[b][0], md.box_c[b][1], md.box_c[b][2]);
        s.p1 = v3(md.box_h[b][0], md.box_h[b][1], md.box_h[b][2]);
        s.r = 0.f;
    } else {
        const int arm = (gid - G_ARM) / 7, g = (gid - G_ARM) % 7;
        if (g < 6) {
            s.type = SH_CAPSULE; s.p0 = kin[arm].o[g]; s.p1 = kin[arm].o[g + 1]; s.r = md.link_rad[g];
        } else {
            s.type = SH_SPHERE; s.p0 = kin[arm].o[NJ]; s.p1 = s.p0; s.r = md.pad_rad;
        }
    }
    return s;
}

struct AABB {
    V3 lo, hi;
};

__device__ __forceinline__ AABB shape_aabb(const Shape &s)
{
    AABB b;
    if (s.type == SH_PLANE) {
        b.lo = v3(-INFINITY, -INFINITY, -INFINITY);
        b.hi = v3(INFINITY, INFINITY, 0.f);
    } else if (s.type == SH_BOX) {
        b.lo = s.p0 - s.p1;
        b.hi = s.p0 + s.p1;
    } else {
        b.lo = v3(fminf(s.p0.x, s.p1.x) - s.r, fminf(s.p0.y, s.p1.y) - s.r, fminf(s.p0.z, s.p1.z) - s.r);
        b.hi = v3(fmaxf(s.p0.x, s.p1.x) + s.r, fmaxf(s.p0.y, s.p1.y) + s.r, fmaxf(s.p0.z, s.p1.z) + s.r);
    }
    return b;
}

// closed boxes overlap after growing A by margin
__device__ __forceinline__ bool aabb_overlap(const AABB &a, const AABB &b, float margin)
{
    return (a.lo.x - margin <= b.hi.x) & (b.lo.x <= a.hi.x + margin) & (a.lo.y - margin <= b.hi.y) &
           (b.lo.y <= a.hi.y + margin) & (a.lo.z - margin <= b.hi.z) & (b.lo.z <= a.hi.z + margin);
}

struct Contact3 {
    float phi;
    V3 n, p;
};

__device__ __forceinline__ Contact3 sphere_sphere(V3 xa, float ra, V3 xb, float rb)
{
    Contact3 c;
    const V3 d = xa - xb;
    const float dist = fsqrt(dot(d, d));
    c.n = dist > 1e-9f ? frcp(dist) * d : v3(0.f, 0.f, 1.f);
    c.phi = dist - ra - rb;
    c.p = 0.5f * ((xa - ra * c.n) + (xb + rb * c.n));
    return c;
}

__device__ __forceinline__ Contact3 sphere_plane(V3 x, float r)
{
    Contact3 c;
    c.n = v3(0.f, 0.f, 1.f);
    c.phi = x.z - r;
    c.p = v3(x.x, x.y, 0.5f * (x.z - r));
    return c;
}

__device__ __forceinline__ float clampf(float v, float lo, float hi) { return fminf(fmaxf(v, lo), hi); }

__device__ __forceinline__ Contact3 sphere_box(V3 x, float r, V3 c, V3 h)
{
    Contact3 out;
    const V3 l = x - c;
    const bool outside = (fabsf(l.x) > h.x) | (fabsf(l.y) > h.y) | (fabsf(l.z) > h.z);
    V3 q;
    if (outside) {
        q = v3(clampf(l.x, -h.x, h.x), clampf(l.y, -h.y, h.y), clampf(l.z, -h.z, h.z));
        const V3 d = l - q;
        const float dist = fsqrt(dot(d, d));
        out.n = frcp(dist) * d;
        out.phi = dist - r;
    } else {
        const float ex = fabsf(l.x) - h.x, ey = fabsf(l.y) - h.y, ez = fabsf(l.z) - h.z;
        int best = 0;
        float be = ex;
        if (ey > be) { be = ey; best = 1; }
        if (ez > be) { be = ez; best = 2; }
        q = l;
        if (best == 0) { const float sg = l.x >= 0.f ? 1.f : -1.f; out.n = v3(sg, 0.f, 0.f); q.x = sg * h.x; }
        else if (best == 1) { const float sg = l.y >= 0.f ? 1.f : -1.f; out.n = v3(0.f, sg, 0.f); q.y = sg * h.y; }
        else { const float sg = l.z >= 0.f ? 1.f : -1.f; out.n = v3(0.f, 0.f, sg); q.z = sg * h.z; }
        out.phi = be - r;
    }
    out.p = 0.5f * ((x - r * out.n) + (c + q));
    return out;
}

__device__ __forceinline__ float seg_point_param(V3 p0, V3 p1, V3 x)
{
    const V3 d = p1 - p0;
    const float dd = dot(d, d);
    return dd > 0.f ? clampf(dot(x - p0, d) * frcp(dd), 0.f, 1.f) : 0.f;
}

// closest points of segments P0 + s D1, Q0 + t D2
__device__ __forceinline__ void seg_seg_params(V3 p0, V3 p1, V3 q0, V3 q1, float &s, float &t)
{
    const V3 d1 = p1 - p0, d2 = q1 - q0, r = p0 - q0;
    const float a = dot(d1, d1), e = dot(d2, d2), b = dot(d1, d2), c = dot(d1, r), f = dot(d2, r);
    const float den = a * e - b * b;
    s = den > 0.f ? clampf((b * f - c * e) * frcp(den), 0.f, 1.f) : 0.f;
    t = (b * s + f) * frcp(e);
    if (t < 0.f) {
        t = 0.f;
        s = clampf(-c * frcp(a), 0.f, 1.f);
    } else if (t > 1.f) {
        t = 1.f;
        s = clampf((b - c) * frcp(a), 0.f, 1.f);
    }
}

// sign-based slope of the box signed distance along direction d at box-frame
// point l: >0 increasing, <0 decreasing, 0 flat
__device__ __forceinline__ float box_sd_slope(V3 l, V3 h, V3 d)
{
    const float ex = fabsf(l.x) - h.x, ey = fabsf(l.y) - h.y, ez = fabsf(l.z) - h.z;
    if ((ex > 0.f) | (ey > 0.f) | (ez > 0.f)) {
        // outside: (l - clamp(l)) . d
        return (ex > 0.f ? (l.x - copysignf(h.x, l.x)) * d.x : 0.f) +
               (ey > 0.f ? (l.y - copysignf(h.y, l.y)) * d.y : 0.f) +
               (ez > 0.f ? (l.z - copysignf(h.z, l.z)) * d.z : 0.f);
    }
    // inside: the face of least penetration (first axis on ties)
    float be = ex, sl = (l.x >= 0.f ? d.x : -d.x);
    if (ey > be) { be = ey; sl = (l.y >= 0.f ? d.y : -d.y); }
    if (ez > be) { sl = (l.z >= 0.f ? d.z : -d.z); }
    return sl;
}

// parameter of the segment point minimising the signed distance to the box
__device__ inline float seg_box_param(V3 a, V3 b, V3 c, V3 h)
{
    const V3 a0 = a - c, d = b - a;
    // left end of the minimising interval: first t with slope >= 0
    float lo = 0.f, hi = 1.f;
    // right end: first t with slope > 0
    float lo2 = 0.f, hi2 = 1.f;
#pragma unroll 2
    for (int it = 0; it < 26; ++it) {
        const float m1 = 0.5f * (lo + hi), m2 = 0.5f * (lo2 + hi2);
        const float s1 = box_sd_slope(fma3(m1, d, a0), h, d);
        const float s2 = box_sd_slope(fma3(m2, d, a0), h, d);
        if (s1 < 0.f) lo = m1; else hi = m1;
        if (s2 <= 0.f) lo2 = m2; else hi2 = m2;
    }
    // exact ends when the minimiser sits at t = 0 or t = 1
    const float s0 = box_sd_slope(a0, h, d), s1 = box_sd_slope(a0 + d, h, d);
    const float tl = s0 >= 0.f ? 0.f : (s1 < 0.f ? 1.f : 0.5f * (lo + hi));
    const float tr = s1 <= 0.f ? 1.f : (s0 > 0.f ? 0.f : 0.5f * (lo2 + hi2));
    return 0.5f * (tl + tr);
}

// narrowphase of shapes A (sphere or capsule) and B (any)
__device__ inline Contact3 narrow(const Shape &A, const Shape &B)
{
    if (B.type == SH_PLANE) {
        V3 x = A.p0;
        if (A.type == SH_CAPSULE && A.p1.z < A.p0.z) x = A.p1;
        return sphere_plane(x, A.r);
    }
    if (B.type == SH_BOX) {
        V3 x = A.p0;
        if (A.type == SH_CAPSULE) x = fma3(seg_box_param(A.p0, A.p1, B.p0, B.p1), A.p1 - A.p0, A.p0);
        return sphere_box(x, A.r, B.p0, B.p1);
    }
    V3 xa = A.p0, xb = B.p0;
    if (A.type == SH_CAPSULE && B.type == SH_CAPSULE) {
        float s, t;
        seg_seg_params(A.p0, A.p1, B.p0, B.p1, s, t);
        xa = fma3(s, A.p1 - A.p0, A.p0);
        xb = fma3(t, B.p1 - B.p0, B.p0);
    } else if (A.type == SH_CAPSULE) {
        xa = fma3(seg_point_param(A.p0, A.p1, B.p0), A.p1 - A.p0, A.p0);
    } else if (B.type == SH_CAPSULE) {
        xb = fma3(seg_point_param(B.p0, B.p1, A.p0), B.p1 - B.p0, B.p0);
    }
    return sphere_sphere(xa, A.r, xb, B.r);
}

// ---------------------------------------------------------------------------
// The free object as a box (the tray, the cube): centre c, rotation R (from
// its unit quaternion, row-major), half extents h.  Vertex k (0..7) sits at
// c + R (s_x h_x, s_y h_y, s_z h_z), s_x = +1 when bit 0 of k is set, else -1
// (bits 1, 2 for y, z).

struct Rot3 {
    float m[9];
};

__device__ __forceinline__ Rot3 quat_R(float w, float x, float y, float z)
{
    Rot3 R;
    R.m[0] = 1.f - 2.f * (y * y + z * z); R.m[1] = 2.f * (x * y - w * z); R.m[2] = 2.f * (x * z + w * y);
    R.m[3] = 2.f * (x * y + w * z); R.m[4] = 1.f - 2.f * (x * x + z * z); R.m[5] = 2.f * (y * z - w * x);
    R.m[6] = 2.f * (x * z - w * y); R.m[7] = 2.f * (y * z + w * x); R.m[8] = 1.f - 2.f * (x * x + y * y);
    return R;
}
__device__ __forceinline__ V3 mulR(const Rot3 &R, V3 v)
{
    return v3(R.m[0] * v.x + R.m[1] * v.y + R.m[2] * v.z, R.m[3] * v.x + R.m[4] * v.y + R.m[5] * v.z,
              R.m[6] * v.x + R.m[7] * v.y + R.m[8] * v.z);
}
__device__ __forceinline__ V3 mulRt(const Rot3 &R, V3 v)
{
    return v3(R.m[0] * v.x + R.m[3] * v.y + R.m[6] * v.z, R.m[1] * v.x + R.m[4] * v.y + R.m[7] * v.z,
              R.m[2] * v.x + R.m[5] * v.y + R.m[8] * v.z);
}
__device__ __forceinline__ V3 Rcol(const Rot3 &R, int i) { return v3(R.m[i], R.m[3 + i], R.m[6 + i]); }

__device__ __forceinline__ V3 obox_vertex(V3 c, const Rot3 &R, V3 h, int k)
{
    return c + mulR(R, v3((k & 1) ? h.x : -h.x, (k & 2) ? h.y : -h.y, (k & 4) ? h.z : -h.z));
}

__device__ __forceinline__ AABB obox_aabb(V3 c, const Rot3 &R, V3 h)
{
    const V3 e = v3(fabsf(R.m[0]) * h.x + fabsf(R.m[1]) * h.y + fabsf(R.m[2]) * h.z,
                    fabsf(R.m[3]) * h.x + fabsf(R.m[4]) * h.y + fabsf(R.m[5]) * h.z,
                    fabsf(R.m[6]) * h.x + fabsf(R.m[7]) * h.y + fabsf(R.m[8]) * h.z);
    AABB b;
    b.lo = c - e;
    b.hi = c + e;
    return b;
}

// the box object (geom A) against a sphere or capsule B: B's core taken to
// the box's frame, the static-box narrowphase there, the normal turned to
// point from B towards the object
__device__ inline Contact3 obox_core(V3 c, const Rot3 &R, V3 h, const Shape &B)
{
    Shape Bl = B;
    Bl.p0 = mulRt(R, B.p0 - c);
    Bl.p1 = mulRt(R, B.p1 - c);
    Shape bx;
    bx.type = SH_BOX;
    bx.p0 = v3(0.f, 0.f, 0.f);
    bx.p1 = h;
    bx.r = 0.f;
    const Contact3 cl = narrow(Bl, bx);
    Contact3 out;
    out.phi = cl.phi;
    out.n = -1.0f * mulR(R, cl.n);
    out.p = c + mulR(R, cl.p);
    return out;
}

// vertex of the box (c, R, h) farthest along d (the lowest index on ties)
__device__ __forceinline__ V3 obox_support(V3 c, const Rot3 &R, V3 h, V3 d)
{
    V3 best = obox_vertex(c, R, h, 0);
    float be = dot(best, d);
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        const V3 v = obox_vertex(c, R, h, k);
        const float e = dot(v, d);
        if (e > be) {
            be = e;
            best = v;
        }
    }
    return best;
}

// the box object (geom A) against a static axis-aligned box (centre cb, half
// extents hb) by separating axes: the object's face normals, the static
// box's, then their cross products (shorter than 1e-9: skipped); phi the
// largest separation, n its axis (first on ties) turned towards the object,
// p midway between the two boxes' support vertices along -n and n
__device__ inline Contact3 obox_box(V3 c, const Rot3 &R, V3 h, V3 cb, V3 hb)
{
    const V3 d = c - cb;
    float best = -INFINITY;
    V3 bn = v3(0.f, 0.f, 1.f);
    auto axis = [&](V3 L) {
        const V3 la = mulRt(R, L);
        const float ra = h.x * fabsf(la.x) + h.y * fabsf(la.y) + h.z * fabsf(la.z);
        const float rb = hb.x * fabsf(L.x) + hb.y * fabsf(L.y) + hb.z * fabsf(L.z);
        const float dl = dot(d, L);
        const float sep = fabsf(dl) - ra - rb;
        if (sep > best) {
            best = sep;
            bn = dl >= 0.f ? L : -1.0f * L;
        }
    };
#pragma unroll
    for (int i = 0; i < 3; ++i) axis(Rcol(R, i));
    axis(v3(1.f, 0.f, 0.f));
    axis(v3(0.f, 1.f, 0.f));
    axis(v3(0.f, 0.f, 1.f));
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const V3 e = v3(j == 0 ? 1.f : 0.f, j == 1 ? 1.f : 0.f, j == 2 ? 1.f : 0.f);
            const V3 x = cross(Rcol(R, i), e);
            const float len = fsqrt(dot(x, x));
            if (len >= 1e-9f) axis(frcp(len) * x);
        }
    Contact3 out;
    out.phi = best;
    out.n = bn;
    const Rot3 I3 = {{1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}};
    out.p = 0.5f * (obox_support(c, R, h, -1.0f * bn) + obox_support(cb, I3, hb, bn));
    return out;
}

}  // namespace mppi
