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
//   pair sweep          geom AABBs published once per substep; candidate
//                       pairs AABB-tested G-wide (G = 16, or 64 when one
//                       wave carries one sample) and the overlapping ones
//                       compacted by ballot into an LDS list in canonical
//                       order; narrowphase runs over that list only, and
//                       contacts are compacted the same way (first n_cmax
//                       kept);
//   contact solve       the soft LCP in row space (pyramid-edge rows, as the
//                       problem is stated): joint lane d forms its own
//                       Jacobian columns J_s[d] and, when an arm is in
//                       contact, row d of Mt^-1 from the parked factor;
//                       Delassus blocks J_s Mt^-1 J_t^T are team sums; the
//                       row matrix A = E^T G E, b, R and 1/(A_rr + R_r) sit
//                       in the team's LDS, the Gauss-Seidel sweeps run
//                       replicated from there, and the impulses return
//                       through the same columns;
//   collision cost      cost pairs dealt 16-wide, each lane owns the history
//                       bits of its pairs.
// Composite quantities use coordinates relative to the arm base.
//
// Wave-per-sample variant: the four 16-lane rows of a wave carry the same
// sample and compute identical values (one shared LDS block, identical
// writes); they only split the pair sweep, four times wider.  Every
// per-sample result equals the 4-teams-per-wave form bit for bit.
//
// TASK forms (one or two waves per sample): the free object may be a box
// (its rotation published beside its centre; its vertices against the table
// ahead of the sweep; pads, links and static boxes through the box
// narrowphase; the contact solve with its world-frame inverse inertia and
// the gyroscopic step of its free angular velocity) and the cost may carry
// the further task terms; ball scenes run the forms without these paths.
#pragma once
#include <utility>
#include "cost.h"
#include "philox.h"

namespace mppi {

constexpr int TEAM = 16;
constexpr int TEAMS_PER_WAVE = 4;

// per-team LDS block (floats): geometry, contact list, park area
constexpr int TG_PTS = 0;             // 2 arms x 8 points x 3: joint origins o_0..o_6 and tip
constexpr int TG_BALL = 48;           // ball centre
constexpr int TG_AABB = 52;           // dynamic geoms 0..15: lo[3], hi[3] (entry 1, the table, unused)
constexpr int TG_CAND = TG_AABB + 96; // candidate pair indices of the sweep
// the box object's rotation (row-major): the task forms sweep a wave wide,
// which uses no candidate list, so it shares that area (the team block's
// size sets how many workgroups fit a CU's LDS)
constexpr int TG_OBJR = TG_CAND;
constexpr int TG_FIELDS = TG_CAND + ((MPPI_MAX_PAIRS + 3) / 4) * 4;

// per-workgroup LDS header (one scene per workgroup), staged once per
// launch: candidate pairs (ga | gb << 8), box AABBs, box centres and half
// extents, link radii, pad and ball radius
constexpr int HD_PAIR = 0;
constexpr int HD_BOXAB = HD_PAIR + ((MPPI_MAX_PAIRS + 3) / 4) * 4;
constexpr int HD_BOXCH = HD_BOXAB + 6 * MPPI_MAX_BOXES;
constexpr int HD_RAD = HD_BOXCH + 6 * MPPI_MAX_BOXES;  // link_rad[0..6], pad_rad, ball_r
constexpr int HD_FIELDS = HD_RAD + 12;
// contact-solve area (after the park area; every offset a multiple of 4
// floats so rows of A load as float4): per contact 20 floats (edges
// e_q, offset r from the ball centre, bias, free velocity b_s), Delassus
// blocks G_st (NC x NC x 9), row matrix A (4NC x 4NC), b, 1/(A_rr + R_r), R,
// and the multipliers when several contacts are active
constexpr int tcs_fields(int nc) { return 20 * nc + 9 * nc * nc + 16 * nc * nc + 16 * nc; }
constexpr int PK_FIELDS4 = (PK_FIELDS + 3) / 4 * 4;  // park area rounded to 16 bytes
constexpr int team_lds_floats(int nc) { return TG_FIELDS + nc * CL_FIELDS + PK_FIELDS4 + tcs_fields(nc); }
// 16-byte alignment of the park and solve areas (float4 reads and writes)
static_assert(HD_FIELDS % 4 == 0 && TG_FIELDS % 4 == 0 && (4 * CL_FIELDS) % 4 == 0 && PK_L % 4 == 0 &&
                  team_lds_floats(4) % 4 == 0 && team_lds_floats(8) % 4 == 0,
              "team LDS blocks keep 16-byte alignment");

// DPP moves within 16-lane rows; lanes whose source falls outside the row
// read 0 (bound_ctrl)
template <int S>
__device__ __forceinline__ float dpp_shr(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x110 + S, 0xF, 0xF, true));
}
template <int S>
__device__ __forceinline__ float dpp_shl(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x100 + S, 0xF, 0xF, true));
}

// value of lane N of this lane's 16-lane row (DPP row broadcast: no LDS trip)
template <int N>
__device__ __forceinline__ float row_bcast(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + N, 0xF, 0xF, true));
}
// value of lane I of this lane's arm segment (team lane 8 * arm1 + I)
template <int I>
__device__ __forceinline__ float segb(float v, bool arm1)
{
    const float a = row_bcast<I>(v), b = row_bcast<8 + I>(v);
    return arm1 ? b : a;
}
template <int I>
__device__ __forceinline__ V3 segb3(V3 v, bool arm1)
{
    return v3(segb<I>(v.x, arm1), segb<I>(v.y, arm1), segb<I>(v.z, arm1));
}

// compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

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

// sum over the 16 lanes of a team (inclusive DPP scan of the row, then a
// broadcast of its last lane): the same value, bit for bit, in every lane
__device__ __forceinline__ float team_sum(float x)
{
    x += dpp_shr<1>(x);
    x += dpp_shr<2>(x);
    x += dpp_shr<4>(x);
    x += dpp_shr<8>(x);
    return row_bcast<15>(x);
}

// LDS writes of this wave become visible to its other lanes; no barrier,
// so it may sit under control flow that differs between the teams of a wave
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ float wave_sum(float x)
{
    x = team_sum(x);
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
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

// the box object's world-frame inverse inertia W = R diag(1/I) R^T
// (row-major) from its quaternion q
__device__ __forceinline__ void obj_world_inv_inertia(const DevModel &md, const float q[4], float W[9])
{
    const Rot3 R = quat_R(q[0], q[1], q[2], q[3]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            W[3 * i + j] = R.m[3 * i] * R.m[3 * j] * md.obj_iI[0] + R.m[3 * i + 1] * R.m[3 * j + 1] * md.obj_iI[1] +
                           R.m[3 * i + 2] * R.m[3 * j + 2] * md.obj_iI[2];
}

// the box object's free angular velocity: w - h R diag(1/I) (w_b x I w_b),
// w_b = R^T w (the explicit gyroscopic step)
__device__ __forceinline__ V3 obj_free_w(const DevModel &md, const float q[4], V3 w)
{
    const Rot3 R = quat_R(q[0], q[1], q[2], q[3]);
    const V3 wbb = mulRt(R, w);
    const V3 Lb = v3(md.obj_I[0] * wbb.x, md.obj_I[1] * wbb.y, md.obj_I[2] * wbb.z);
    const V3 gb = cross(wbb, Lb);
    return w - md.h * mulR(R, v3(md.obj_iI[0] * gb.x, md.obj_iI[1] * gb.y, md.obj_iI[2] * gb.z));
}

// one lane's kinematic quantities of its joint
struct JointKin {
    V3 a;        // joint axis
    V3 z;        // link axis
    V3 o;        // joint origin
    V3 o1;       // next joint origin (tip for joint 7)
    V3 x, y;     // link frame's x and y axes (the pad frame on the last joint's lane)
};

// FRAME: also the link frame's x and y axes (the further cost terms' pad frame)
template <bool FRAME = false>
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
    if (FRAME) {
        k.x = v3(R.m[0][0], R.m[1][0], R.m[2][0]);
        k.y = v3(R.m[0][1], R.m[1][1], R.m[2][1]);
    }
    k.a = jc.ax == 0 ? v3(R.m[0][0], R.m[1][0], R.m[2][0]) : (jc.ax == 1 ? v3(R.m[0][1], R.m[1][1], R.m[2][1]) : k.z);
    const V3 d = (joint ? jc.len : 0.f) * k.z;
    const V3 inc = seg_prefix3(d, jt);
    k.o1 = jc.base + inc;
    k.o = k.o1 - d;
}

// composite-rigid-body terms of link jt: with the composite of links jt..6
// (mass Mc, centre cc, inertia Ic about it), L = Mc a x (cc - o) and
// K = Ic a + cc x L (base-relative), and the moment arm mo = a x o
__device__ inline void team_composite(const DevModel &md, const JointConst &jc, const JointKin &k, int jt, V3 &K, V3 &L,
                                      V3 &mo)
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
    const V3 cc = (joint ? frcp(Mc) : 0.f) * h;
    const float c2 = dot(cc, cc);
    const S3 Ic = {I[0] - Mc * (c2 - cc.x * cc.x), I[1] - Mc * (c2 - cc.y * cc.y), I[2] - Mc * (c2 - cc.z * cc.z),
                   I[3] + Mc * cc.x * cc.y,        I[4] + Mc * cc.x * cc.z,        I[5] + Mc * cc.y * cc.z};
    const V3 ob = k.o - jc.base;
    L = Mc * cross(k.a, cc - ob);
    K = mul(Ic, k.a) + cross(cc, L);
    mo = cross(k.a, ob);
}

// entry (r, c), c <= r, of Mt from lane c's axis and moment arm and lane r's
// composite (K, L): a_c . K_r - mo_c . L_r (+ the diagonal term)
__device__ __forceinline__ float mass_entry(const DevModel &md, V3 ac, V3 moc, V3 K, V3 L, bool diag)
{
    float e = dot(ac, K) - dot(moc, L);
    if (diag) e += md.diag_add;
    return e;
}

// row jt of Mt = M + diag(diag_add), entries c <= jt (the rest 0), on joint lanes
__device__ inline void team_crba(const DevModel &md, const JointConst &jc, const JointKin &k, int jt, int seg,
                                 float row[NJ])
{
    V3 K, L, mo;
    team_composite(md, jc, k, jt, K, L, mo);
    // row jt, entries c <= jt (the lower triangle the factorisation reads)
    const bool arm1 = seg != 0;
    static_for<NJ>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const V3 ai = segb3<i>(k.a, arm1), mi = segb3<i>(mo, arm1);
        row[i] = i <= jt ? mass_entry(md, ai, mi, K, L, i == jt) : 0.f;
    });
}

// packed row index r of lower-triangle entry e = tri(r, c), e < 28, 4 bits each
constexpr uint64_t tri_rows(int lo)
{
    uint64_t t = 0;
    for (int r = 0, e = 0; r < 7; ++r)
        for (int c = 0; c <= r; ++c, ++e)
            if (e >= lo && e < lo + 16) t |= (uint64_t)r << (4 * (e - lo));
    return t;
}

// The arm's packed lower triangle of Mt on every lane of its segment, for a
// wave whose four 16-lane rows carry one team: each lane parks its axis,
// moment arm and composite in LDS (X, 16-byte aligned, 248 floats), lane l <
// 56 forms entry l mod 28 of arm l / 28, and every lane reads its arm's 28
// back.  The entries are those of team_crba bit for bit.
// (t: the lane's index in the team, lane: its index in the wave)
__device__ inline void team_mass_rows(const DevModel &md, const JointConst &jc, const JointKin &k, int jt, int t,
                                      int arm, int lane, float *X, float Lp[28])
{
    V3 K, L, mo;
    team_composite(md, jc, k, jt, K, L, mo);
    float4 *xl = reinterpret_cast<float4 *>(X + 12 * t);
    xl[0] = make_float4(k.a.x, k.a.y, k.a.z, mo.x);
    xl[1] = make_float4(mo.y, mo.z, K.x, K.y);
    xl[2] = make_float4(K.z, L.x, L.y, L.z);
    wave_lds_sync();
    float *T = X + 192;
    const int l = lane;
    if (l < 56) {
        const int ar = l >= 28, e = l - 28 * ar;
        constexpr uint64_t R0 = tri_rows(0), R1 = tri_rows(16);
        const int r = (int)((e < 16 ? R0 >> (4 * e) : R1 >> (4 * (e - 16))) & 15ull);
        const int c = e - r * (r + 1) / 2;
        const float *xc = X + 12 * (8 * ar + c), *xr = X + 12 * (8 * ar + r);
        T[l] = mass_entry(md, v3(xc[0], xc[1], xc[2]), v3(xc[3], xc[4], xc[5]), v3(xr[6], xr[7], xr[8]),
                          v3(xr[9], xr[10], xr[11]), r == c);
    }
    wave_lds_sync();
    const float4 *tr = reinterpret_cast<const float4 *>(T + 28 * arm);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const float4 t4 = tr[i];
        Lp[4 * i] = t4.x; Lp[4 * i + 1] = t4.y; Lp[4 * i + 2] = t4.z; Lp[4 * i + 3] = t4.w;
    }
}

// gather the packed lower triangle of the arm's Mt on every lane of its segment
__device__ __forceinline__ void team_gather_tri(const float row[NJ], int seg, float Lp[28])
{
    const bool arm1 = seg != 0;
    static_for<NJ>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
#pragma unroll
        for (int c = 0; c <= r; ++c) Lp[tri(r, c)] = segb<r>(row[c], arm1);
    });
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

// v ^ x, where the compiler no longer sees v as an element of an array: a
// chain of selects over array elements keyed on one index would otherwise
// become a dynamically indexed access, which goes through scratch memory
__device__ __forceinline__ float opaque(float v)
{
    asm("" : "+v"(v));
    return v;
}

// component jt of a 7-vector held identically by the segment
__device__ __forceinline__ float pick7(const float v[NJ], int jt)
{
    float r = v[0];
#pragma unroll
    for (int i = 1; i < NJ; ++i) r = jt == i ? opaque(v[i]) : r;
    return r;
}

struct TeamState {
    float q, qd, qdes;  // own joint (joint lanes)
    V3 pb, vb, wb;      // ball (replicated)
    float quat[4];
};

__device__ __forceinline__ Shape team_geom(const float *tl, const float *hd, int gid)
{
    Shape s;
    if (gid == G_BALL) {
        s.type = SH_SPHERE;
        s.p0 = v3(tl[TG_BALL], tl[TG_BALL + 1], tl[TG_BALL + 2]);
        s.p1 = s.p0;
        s.r = hd[HD_RAD + 8];
    } else if (gid == G_TABLE) {
        s = table_shape();
    } else if (gid >= G_BOX) {
        const float *bx = hd + HD_BOXCH + 6 * (gid - G_BOX);
        s.type = SH_BOX;
        s.p0 = v3(bx[0], bx[1], bx[2]);
        s.p1 = v3(bx[3], bx[4], bx[5]);
        s.r = 0.f;
    } else {
        const int arm = (gid - G_ARM) / 7, g = (gid - G_ARM) % 7;
        const float *p = tl + TG_PTS + 24 * arm;
        if (g < 6) {
            s.type = SH_CAPSULE;
            s.p0 = v3(p[3 * g], p[3 * g + 1], p[3 * g + 2]);
            s.p1 = v3(p[3 * g + 3], p[3 * g + 4], p[3 * g + 5]);
        } else {
            s.type = SH_SPHERE;
            s.p0 = v3(p[21], p[22], p[23]);
            s.p1 = s.p0;
        }
        s.r = hd[HD_RAD + g];  // g = 6: the pad radius
    }
    return s;
}

// stage the scene's pair table, boxes and radii in the workgroup header
__device__ inline void stage_header(float *hd, const DevModel &md, int lane, int width)
{
    for (int i = lane; i < md.n_pairs; i += width) hd[HD_PAIR + i] = __int_as_float(md.pa[i] | (md.pb[i] << 8));
    for (int b = lane; b < md.n_box; b += width) {
        float *ab = hd + HD_BOXAB + 6 * b, *ch = hd + HD_BOXCH + 6 * b;
        const Shape bx = box_shape(md, b);
        const V3 lo = bx.p0 - bx.p1, hi = bx.p0 + bx.p1;
        ab[0] = lo.x; ab[1] = lo.y; ab[2] = lo.z; ab[3] = hi.x; ab[4] = hi.y; ab[5] = hi.z;
        ch[0] = bx.p0.x; ch[1] = bx.p0.y; ch[2] = bx.p0.z; ch[3] = bx.p1.x; ch[4] = bx.p1.y; ch[5] = bx.p1.z;
    }
    if (lane < 6) hd[HD_RAD + lane] = md.link_rad[lane];
    if (lane == 6) hd[HD_RAD + 6] = md.pad_rad;
    if (lane == 7) hd[HD_RAD + 8] = md.ball_r;
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

// team_publish_geom and the AABBs of the team's geoms in one pass: lane
// (arm, jt) boxes arm geom jt (capsule jt from its own joint origin to the
// next lane's, or the pad sphere at the tip for jt = 6), arm 0's spare lane
// the ball; the values equal shape_aabb of the published shapes bit for bit,
// and one wave-local sync covers both.  TASK: a box object's rotation (from
// its quaternion q) is published too, and its AABB is the rotated box's.
template <bool TASK = false>
__device__ __forceinline__ void team_publish_geom_aabb(float *tl, const float *hd, const JointKin &k, V3 pb, int arm,
                                                       int jt, const DevModel *md = nullptr,
                                                       const float *q = nullptr)
{
    const V3 onext = v3(dpp_shl<1>(k.o.x), dpp_shl<1>(k.o.y), dpp_shl<1>(k.o.z));  // next lane's joint origin
    team_publish_geom(tl, k, pb, arm, jt);
    if (TASK && md->obj_box && jt == 7 && arm == 0) {
        const Rot3 R = quat_R(q[0], q[1], q[2], q[3]);
#pragma unroll
        for (int i = 0; i < 9; ++i) tl[TG_OBJR + i] = R.m[i];
        const AABB b = obox_aabb(pb, R, v3(md->obj_h[0], md->obj_h[1], md->obj_h[2]));
        float *o = tl + TG_AABB + 6 * G_BALL;
        o[0] = b.lo.x; o[1] = b.lo.y; o[2] = b.lo.z;
        o[3] = b.hi.x; o[4] = b.hi.y; o[5] = b.hi.z;
    } else if (jt < 7 || arm == 0) {
        Shape sh;
        int gid;
        if (jt < 6) {
            sh.type = SH_CAPSULE;
            sh.p0 = k.o;
            sh.p1 = onext;
            sh.r = hd[HD_RAD + jt];
            gid = G_ARM + 7 * arm + jt;
        } else if (jt == 6) {
            sh.type = SH_SPHERE;
            sh.p0 = k.o1;
            sh.p1 = k.o1;
            sh.r = hd[HD_RAD + 6];
            gid = G_ARM + 7 * arm + 6;
        } else {
            sh.type = SH_SPHERE;
            sh.p0 = pb;
            sh.p1 = pb;
            sh.r = hd[HD_RAD + 8];
            gid = G_BALL;
        }
        const AABB b = shape_aabb(sh);
        float *o = tl + TG_AABB + 6 * gid;
        o[0] = b.lo.x; o[1] = b.lo.y; o[2] = b.lo.z;
        o[3] = b.hi.x; o[4] = b.hi.y; o[5] = b.hi.z;
    }
    wave_lds_sync();
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

// AABB test of candidate pair p (geom A is always dynamic) after growing A
// by margin; the same comparisons as aabb_overlap on the geoms' boxes
__device__ __forceinline__ bool pair_overlap(const float *tl, const float *hd, int ga, int gb, float margin)
{
    const float *A = tl + TG_AABB + 6 * ga;
    if (gb == G_TABLE) return A[2] - margin <= 0.f;
    AABB a, b;
    a.lo = v3(A[0], A[1], A[2]);
    a.hi = v3(A[3], A[4], A[5]);
    if (gb >= G_BOX) {
        const float *B = hd + HD_BOXAB + 6 * (gb - G_BOX);
        b.lo = v3(B[0], B[1], B[2]);
        b.hi = v3(B[3], B[4], B[5]);
    } else {
        const float *B = tl + TG_AABB + 6 * gb;
        b.lo = v3(B[0], B[1], B[2]);
        b.hi = v3(B[3], B[4], B[5]);
    }
    return aabb_overlap(a, b, margin);
}

// bits of the sweeping group (G lanes starting at wave lane gshift)
template <int G>
__device__ __forceinline__ uint64_t group_bits(uint64_t wm, int gshift)
{
    return G == 64 ? wm : (wm >> gshift) & ((1ull << G) - 1ull);
}

// Contact pass of one substep: AABB pre-pass over every candidate pair,
// compaction of the overlapping ones, narrowphase over those; contacts land
// in the team's LDS list in canonical order; returns the count.  li: lane
// index within the sweeping group of G lanes.  A whole wave (G = 64) skips
// the candidate list.
template <int G, bool TASK = false>
__device__ inline int team_collect(const DevModel &md, float *tl, const float *hd, const LaneList &LL, int li,
                                   int gshift, StepCounters &cnt)
{
    static_assert(!TASK || G == 64, "the task forms sweep a wave wide");
    const int np = md.n_pairs;
    if constexpr (G == 64) {
        // one sweep a wave: each lane runs the narrowphase of its own
        // overlapping pairs right away (no candidate list), block by block in
        // pair order, and the hits are compacted into the contact list; the
        // same contacts, in the same order, as the two-pass form below
        int n = 0;
        const uint64_t below = (1ull << li) - 1ull;
        const bool box = TASK && md.obj_box;
        Rot3 R;
        V3 oc = v3(0.f, 0.f, 0.f), oh = v3(0.f, 0.f, 0.f);
        if (box) {
            // the box object: its vertices below the table first (its pair
            // with the table comes first in canonical order), in vertex
            // order, four at most
#pragma unroll
            for (int i = 0; i < 9; ++i) R.m[i] = tl[TG_OBJR + i];
            oc = v3(tl[TG_BALL], tl[TG_BALL + 1], tl[TG_BALL + 2]);
            oh = v3(md.obj_h[0], md.obj_h[1], md.obj_h[2]);
            const bool low = tl[TG_AABB + 6 * G_BALL + 2] < 0.f;
            bool vhit = false;
            V3 v = v3(0.f, 0.f, 0.f);
            if (low && li < 8) {
                v = obox_vertex(oc, R, oh, li);
                vhit = v.z < 0.f;
            }
            if (low && li == 0) ++cnt.np_tests;
            const uint64_t gm = __ballot(vhit);
            const int cap = min(4, md.n_cmax);
            if (vhit) {
                const int slot = __popcll(gm & below);
                if (slot < cap) {
                    LL.at(slot, 0) = __int_as_float(G_BALL);
                    LL.at(slot, 1) = __int_as_float(G_TABLE);
                    LL.at(slot, 2) = v.z;
                    LL.at(slot, 3) = 0.f; LL.at(slot, 4) = 0.f; LL.at(slot, 5) = 1.f;
                    LL.at(slot, 6) = v.x; LL.at(slot, 7) = v.y; LL.at(slot, 8) = 0.5f * v.z;
                }
            }
            n = min((int)__popcll(gm), cap);
        }
        auto narrow_block = [&](bool ov, int gab) {
            if (__ballot(ov) == 0ull) return;
            bool hit = false;
            Contact3 c;
            const int ga = gab & 0xff, gb = gab >> 8;
            if (ov) {
                ++cnt.np_tests;
                if (box && ga == G_BALL) {
                    const Shape B = team_geom(tl, hd, gb);
                    c = B.type == SH_BOX ? obox_box(oc, R, oh, B.p0, B.p1) : obox_core(oc, R, oh, B);
                } else {
                    const Shape A = team_geom(tl, hd, ga), B = team_geom(tl, hd, gb);
                    if (B.type == SH_BOX && A.type == SH_CAPSULE) ++cnt.box_tests;
                    c = narrow(A, B);
                }
                hit = c.phi < 0.f;
            }
            const uint64_t gm = __ballot(hit);
            if (hit) {
                const int slot = n + __popcll(gm & below);
                if (slot < md.n_cmax) {
                    LL.at(slot, 0) = __int_as_float(ga);
                    LL.at(slot, 1) = __int_as_float(gb);
                    LL.at(slot, 2) = c.phi;
                    LL.at(slot, 3) = c.n.x; LL.at(slot, 4) = c.n.y; LL.at(slot, 5) = c.n.z;
                    LL.at(slot, 6) = c.p.x; LL.at(slot, 7) = c.p.y; LL.at(slot, 8) = c.p.z;
                }
            }
            n = min(n + (int)__popcll(gm), md.n_cmax);
        };
        for (int base = 0; base < np; base += 2 * G) {
            const int p0 = base + li, p1 = p0 + G;
            int g0 = 0, g1 = 0;
            if (p0 < np) g0 = __float_as_int(hd[HD_PAIR + p0]);
            if (p1 < np) g1 = __float_as_int(hd[HD_PAIR + p1]);
            constexpr int OBJ_TABLE = G_BALL | (G_TABLE << 8);
            const bool ov0 = p0 < np && !(box && g0 == OBJ_TABLE) && pair_overlap(tl, hd, g0 & 0xff, g0 >> 8, 0.f);
            const bool ov1 = p1 < np && !(box && g1 == OBJ_TABLE) && pair_overlap(tl, hd, g1 & 0xff, g1 >> 8, 0.f);
            narrow_block(ov0, g0);
            narrow_block(ov1, g1);
        }
        return n;
    }
    int *cand = (int *)(tl + TG_CAND);  // pair words (ga | gb << 8) of the candidates
    int ncand = 0;
    // two blocks of G pairs at a time, so that their LDS reads overlap; the
    // candidates still land in pair order
    for (int base = 0; base < np; base += 2 * G) {
        const int p0 = base + li, p1 = p0 + G;
        int g0 = 0, g1 = 0;
        if (p0 < np) g0 = __float_as_int(hd[HD_PAIR + p0]);
        if (p1 < np) g1 = __float_as_int(hd[HD_PAIR + p1]);
        const bool ov0 = p0 < np && pair_overlap(tl, hd, g0 & 0xff, g0 >> 8, 0.f);
        const bool ov1 = p1 < np && pair_overlap(tl, hd, g1 & 0xff, g1 >> 8, 0.f);
        const uint64_t below = (1ull << li) - 1ull;
        const uint64_t m0 = group_bits<G>(__ballot(ov0), gshift), m1 = group_bits<G>(__ballot(ov1), gshift);
        if (ov0) cand[ncand + __popcll(m0 & below)] = g0;
        ncand += __popcll(m0);
        if (ov1) cand[ncand + __popcll(m1 & below)] = g1;
        ncand += __popcll(m1);
    }
    wave_lds_sync();
    int n = 0;
    for (int c0 = 0;; c0 += G) {
        const bool live = c0 < ncand && n < md.n_cmax;
        if (__ballot(live) == 0ull) break;
        const int i = c0 + li;
        bool hit = false;
        Contact3 c;
        int ga = 0, gb = 0;
        if (live && i < ncand) {
            const int gab = cand[i];
            ga = gab & 0xff;
            gb = gab >> 8;
            const Shape A = team_geom(tl, hd, ga), B = team_geom(tl, hd, gb);
            ++cnt.np_tests;
            if (B.type == SH_BOX && A.type == SH_CAPSULE) ++cnt.box_tests;
            c = narrow(A, B);
            hit = c.phi < 0.f;
        }
        const uint64_t gm = group_bits<G>(__ballot(hit), gshift);
        if (hit) {
            const int slot = n + __popcll(gm & ((1ull << li) - 1ull));
            if (slot < md.n_cmax) {
                LL.at(slot, 0) = __int_as_float(ga);
                LL.at(slot, 1) = __int_as_float(gb);
                LL.at(slot, 2) = c.phi;
                LL.at(slot, 3) = c.n.x; LL.at(slot, 4) = c.n.y; LL.at(slot, 5) = c.n.z;
                LL.at(slot, 6) = c.p.x; LL.at(slot, 7) = c.p.y; LL.at(slot, 8) = c.p.z;
            }
        }
        n = min(n + (int)__popcll(gm), md.n_cmax);
    }
    return n;
}

// the arm's parked factor (parked by team_dynamics)
__device__ __forceinline__ void team_parked_factor(const LanePark &pk, int arm, float Lf[28])
{
    const float4 *o = reinterpret_cast<const float4 *>(&pk.at(PK_L + 28 * arm));
#pragma unroll
    for (int e = 0; e < 7; ++e) {
        const float4 f4 = o[e];
        Lf[4 * e] = f4.x; Lf[4 * e + 1] = f4.y; Lf[4 * e + 2] = f4.z; Lf[4 * e + 3] = f4.w;
    }
}

struct TeamCtx {
    int t, arm, jt, seg, lane;
    int li, gshift;  // lane within the contact sweep's group, group offset in the wave
    bool count;      // this row counts the collision-cost narrowphase tests
    bool joint;
    float *tl;
    const float *hd;  // workgroup header (scene tables)
    LaneList LL;
    LanePark pk;
};

__device__ __forceinline__ V3 team_sum3(V3 x) { return v3(team_sum(x.x), team_sum(x.y), team_sum(x.z)); }

// Gauss-Seidel over m <= 16 rows spread over the team's lanes.  With
// d_q = 1 / (A_qq + R_q), the update of row q is f_q <- max(u_q, 0) where
// u_q = -d_q (b_q + sum_{c != q} A_qc f_c) does not depend on f_q itself.
// Lane q keeps u_q and its row of C = -d_q A with a zero diagonal; row r:
// every lane forms max(u, 0) and its change, lane r keeps it as its new f_r,
// and every lane adds C_qr times lane r's change to u_q.  One sweep is one
// asm block of five instructions a row: the lane test of the next row (VCC)
// sits between the change and its DPP broadcast, which rides on the
// multiply-add, so the two wait states that the broadcast and the VCC read
// need cost nothing.  On return f[r], r < m, holds the multipliers on every
// lane.
#define PGS_ROW(R, RN)                                                                  \
    "v_max_f32_e32 %[fn], 0, %[u]\n\t"                                                  \
    "v_sub_f32_e32 %[dl], %[fn], %[fq]\n\t"                                             \
    "v_cndmask_b32_e32 %[fq], %[fq], %[fn], vcc\n\t"                                    \
    "v_cmp_eq_u32_e32 vcc, " #RN ", %[qo]\n\t"                                          \
    "v_fmac_f32_dpp %[u], %[dl], %[c" #R "] row_newbcast:" #R " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
#define PGS_ROWS4(a, b, c, d, e) PGS_ROW(a, b) PGS_ROW(b, c) PGS_ROW(c, d) PGS_ROW(d, e)
#define PGS_HEAD "v_cmp_eq_u32_e32 vcc, 0, %[qo]\n\ts_nop 1\n\t"
#define PGS_IO [u] "+v"(u), [fq] "+v"(fq), [fn] "=&v"(fn), [dl] "=&v"(dl)
#define PGS_C4 [qo] "v"(q), [c0] "v"(c[0]), [c1] "v"(c[1]), [c2] "v"(c[2]), [c3] "v"(c[3])
#define PGS_C8 PGS_C4, [c4] "v"(c[4]), [c5] "v"(c[5]), [c6] "v"(c[6]), [c7] "v"(c[7])
#define PGS_C12 PGS_C8, [c8] "v"(c[8]), [c9] "v"(c[9]), [c10] "v"(c[10]), [c11] "v"(c[11])
#define PGS_C16 PGS_C12, [c12] "v"(c[12]), [c13] "v"(c[13]), [c14] "v"(c[14]), [c15] "v"(c[15])

template <int MW>
__device__ inline float pgs_team_rows(const float c[16], float u, int q, int n_pgs)
{
    float fq = 0.f, fn, dl;
    const int ns = __builtin_amdgcn_readfirstlane(n_pgs);  // uniform: a scalar loop
    for (int sweep = 0; sweep < ns; ++sweep) {
        if constexpr (MW == 4)
            asm volatile(PGS_HEAD PGS_ROWS4(0, 1, 2, 3, 4) : PGS_IO : PGS_C4 : "vcc");
        else if constexpr (MW == 8)
            asm volatile(PGS_HEAD PGS_ROWS4(0, 1, 2, 3, 4) PGS_ROWS4(4, 5, 6, 7, 8) : PGS_IO : PGS_C8 : "vcc");
        else if constexpr (MW == 12)
            asm volatile(PGS_HEAD PGS_ROWS4(0, 1, 2, 3, 4) PGS_ROWS4(4, 5, 6, 7, 8) PGS_ROWS4(8, 9, 10, 11, 12)
                         : PGS_IO : PGS_C12 : "vcc");
        else
            asm volatile(PGS_HEAD PGS_ROWS4(0, 1, 2, 3, 4) PGS_ROWS4(4, 5, 6, 7, 8) PGS_ROWS4(8, 9, 10, 11, 12)
                             PGS_ROWS4(12, 13, 14, 15, 16)
                         : PGS_IO : PGS_C16 : "vcc");
    }
    return fq;
}
#undef PGS_ROW
#undef PGS_ROWS4
#undef PGS_HEAD
#undef PGS_IO
#undef PGS_C4
#undef PGS_C8
#undef PGS_C12
#undef PGS_C16

__device__ inline void pgs_team(const float arow_in[16], float bq, float dq, int m, int q, int n_pgs, float f[16])
{
    // rows run up to the wave's largest m; a team with fewer rows carries
    // zeros there (its extra rows change nothing), so the sweep has no
    // per-lane branches
    const int mw = __builtin_amdgcn_readfirstlane(__ballot(m > 12) ? 16 : __ballot(m > 8) ? 12 : __ballot(m > 4) ? 8 : 4);
    const bool mine = q < m;
    const float nd = mine ? -dq : 0.f;
    float crow[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) crow[c] = (c < m && c != q) ? nd * arow_in[c] : 0.f;
    const float u = nd * bq;
    float fq;
    if (mw == 4)
        fq = pgs_team_rows<4>(crow, u, q, n_pgs);
    else if (mw == 8)
        fq = pgs_team_rows<8>(crow, u, q, n_pgs);
    else if (mw == 12)
        fq = pgs_team_rows<12>(crow, u, q, n_pgs);
    else
        fq = pgs_team_rows<16>(crow, u, q, n_pgs);
    static_for<16>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        f[r] = r < m ? row_bcast<r>(fq) : 0.f;
    });
}

// Gauss-Seidel over m <= MR rows (up to 32) for a wave that carries one team:
// the u-form of pgs_team with lane q holding row q of C = -d_q A (zero
// diagonal) and u_q; row r's change reaches every lane through a scalar
// register (v_readlane), so rows beyond one 16-lane row need no LDS trips.
// On return f[r], r < m, holds the multipliers on every lane.
template <int MR>
__device__ inline void pgs_wave(const float *A, const float *Bv, const float *Dv, int m, int n_pgs, int lane,
                                float f[MR])
{
    static_assert(MR <= 64, "one row a lane");
    const int mu = __builtin_amdgcn_readfirstlane(m), ns = __builtin_amdgcn_readfirstlane(n_pgs);
    const bool mine = lane < mu;
    const float nd = mine ? -Dv[lane] : 0.f;
    float c[MR];
#pragma unroll
    for (int cc = 0; cc < MR; ++cc) c[cc] = (mine && cc < mu && cc != lane) ? nd * A[lane * MR + cc] : 0.f;
    float u = mine ? nd * Bv[lane] : 0.f;
    float fq = 0.f;
    for (int sweep = 0; sweep < ns; ++sweep) {
        static_for<MR>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            if (r < mu) {
                const float fn = fmaxf(u, 0.f);
                const float dl = fn - fq;
                fq = lane == r ? fn : fq;
                const float sd = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dl), r));
                u = fmaf(c[r], sd, u);
            }
        });
    }
    static_for<MR>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        f[r] = r < mu ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fq), r)) : 0.f;
    });
}

// Contact solve of one team (nc >= 1 contacts in the team's list, nc uniform
// over the team).  k: this lane's joint kinematics at the contact positions;
// v: this lane's joint velocity (free on entry, post-contact on exit); vb, wb:
// the ball's free velocity and angular velocity, updated in place.
template <int NC, bool TASK = false>
__device__ inline void team_contact_solve(const DevModel &md, const TeamCtx &tc, const JointKin &k, V3 pb, int nc,
                                          float &v, V3 &vb, V3 &wb, const float *Wo = nullptr)
{
    const bool box = TASK && md.obj_box;  // Wo: the box object's world inverse inertia
    constexpr int MR = 4 * NC;
    static_assert(MR >= 16, "the lane-parallel sweeps read 16 rows of A");
    float *E = tc.tl + TG_FIELDS + NC * CL_FIELDS + PK_FIELDS4;  // 16-byte aligned
    float *Gb = E + 20 * NC;
    float *A = Gb + 9 * NC * NC;
    float *Bv = A + MR * MR;
    float *Dv = Bv + MR;
    float *Rv = Dv + MR;
    const LaneList &LL = tc.LL;
    const int m = 4 * nc;
    // contact frames: edges n +- mu t1, n +- mu t2, offset, bias (identical on every lane)
    int side_word = 0;  // bit s: contact s touches an arm; bit 8 + s: the ball is geom A
    for (int s = 0; s < nc; ++s) {
        const int ga = __float_as_int(LL.at(s, 0)), gb = __float_as_int(LL.at(s, 1));
        const Sides sd = contact_sides(ga | (gb << 8));
        side_word |= (((sd.armA >= 0) | (sd.armB >= 0)) ? 1 : 0) << s;
        side_word |= (sd.ball ? 1 : 0) << (8 + s);
        const V3 n = v3(LL.at(s, 3), LL.at(s, 4), LL.at(s, 5));
        const V3 p = v3(LL.at(s, 6), LL.at(s, 7), LL.at(s, 8));
        V3 t1, t2;
        tangents(n, t1, t2);
        float *e = E + 20 * s;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const V3 t = q < 2 ? t1 : t2;
            const V3 eq = fma3((q & 1) ? -md.mu : md.mu, t, n);
            e[3 * q] = eq.x; e[3 * q + 1] = eq.y; e[3 * q + 2] = eq.z;
        }
        const V3 r = p - pb;
        e[12] = r.x; e[13] = r.y; e[14] = r.z;
        const float phi = LL.at(s, 2);
        e[15] = md.kappa_h * (phi < 0.f ? -phi : 0.f);
    }
    const bool any_arm = (side_word & 0xff) != 0;
    // this lane's Jacobian columns and the free contact velocities b_s
    V3 Jc[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        Jc[s] = v3(0.f, 0.f, 0.f);
        if (s < nc) {
            const int ga = __float_as_int(LL.at(s, 0)), gb = __float_as_int(LL.at(s, 1));
            const Sides sd = contact_sides(ga | (gb << 8));
            const V3 p = v3(LL.at(s, 6), LL.at(s, 7), LL.at(s, 8));
            const float coef = tc.joint ? jac_coef(sd, tc.arm, tc.jt) : 0.f;
            if (coef != 0.f) Jc[s] = coef * cross(k.a, p - k.o);
            V3 b = (side_word >> s) & 1 ? team_sum3(v * Jc[s]) : v3(0.f, 0.f, 0.f);
            if ((side_word >> (8 + s)) & 1) {
                const V3 r = p - pb;
                b = b + vb + cross(wb, r);
            }
            float *e = E + 20 * s;
            e[16] = b.x; e[17] = b.y; e[18] = b.z;
        }
    }
    // row d of Mt^-1 of this lane's arm (only when an arm is in contact)
    float Minv[NJ];
#pragma unroll
    for (int e = 0; e < NJ; ++e) Minv[e] = 0.f;
    if (any_arm) {
        float Lf[28];
        team_parked_factor(tc.pk, tc.arm, Lf);
#pragma unroll
        for (int e = 0; e < NJ; ++e) Minv[e] = (tc.joint && e == tc.jt) ? 1.f : 0.f;
        chol7_solve(Lf, Minv);
        if (!tc.joint) {
#pragma unroll
            for (int e = 0; e < NJ; ++e) Minv[e] = 0.f;
        }
    }
    wave_lds_sync();
    // Delassus blocks G_st = J_s Mt^-1 J_t^T (+ the ball's), s <= t
#pragma unroll
    for (int t = 0; t < NC; ++t) {
        if (t < nc) {
            const bool arm_t = (side_word >> t) & 1, ball_t = (side_word >> (8 + t)) & 1;
            V3 W = v3(0.f, 0.f, 0.f);  // row d of Mt^-1 J_t^T
            if (arm_t) {
                static_for<NJ>([&](auto ec) {
                    constexpr int e = decltype(ec)::value;
                    W = fma3(Minv[e], segb3<e>(Jc[t], tc.arm != 0), W);
                });
            }
            const V3 rt = v3(E[20 * t + 12], E[20 * t + 13], E[20 * t + 14]);
#pragma unroll
            for (int s = 0; s <= t; ++s) {
                if (s < nc) {
                    float G[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    if (arm_t && ((side_word >> s) & 1)) {
                        const V3 J = Jc[s];
                        G[0] = team_sum(J.x * W.x); G[1] = team_sum(J.x * W.y); G[2] = team_sum(J.x * W.z);
                        G[3] = team_sum(J.y * W.x); G[4] = team_sum(J.y * W.y); G[5] = team_sum(J.y * W.z);
                        G[6] = team_sum(J.z * W.x); G[7] = team_sum(J.z * W.y); G[8] = team_sum(J.z * W.z);
                    }
                    if (ball_t && ((side_word >> (8 + s)) & 1)) {
                        const V3 rs = v3(E[20 * s + 12], E[20 * s + 13], E[20 * s + 14]);
                        if (box)
                            obj_block(md, Wo, rs, rt, G);
                        else
                            ball_block(md, rs, rt, G);
                    }
                    float *g = Gb + 9 * (s * NC + t);
#pragma unroll
                    for (int i = 0; i < 9; ++i) g[i] = G[i];
                }
            }
        }
    }
    wave_lds_sync();
    float f[MR];
#pragma unroll
    for (int r = 0; r < MR; ++r) f[r] = 0.f;
    if (nc <= 4) {
        // lane q builds row q of A = E^T G E (+ R_q on the diagonal), its b_q
        // and 1 / (A_qq + R_q) in registers; lanes q >= m carry unused rows
        const int q = tc.t, sq = q >> 2;
        const float *es = E + 20 * sq;
        const V3 eq = v3(es[3 * (q & 3)], es[3 * (q & 3) + 1], es[3 * (q & 3) + 2]);
        float arow[16];
        float aqq = 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int w = 0; w < 4; ++w) arow[4 * u + w] = 0.f;
            if (u < nc) {
                float G[9];
                const bool up = sq <= u;  // G_{sq,u} = G_{u,sq}^T below the diagonal
                const float *g = Gb + 9 * (up ? sq * NC + u : u * NC + sq);
#pragma unroll
                for (int i = 0; i < 9; ++i) G[i] = g[i];
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const float *eu = E + 20 * u + 3 * w;
                    const V3 er = v3(eu[0], eu[1], eu[2]);
                    const V3 ge = up ? mul9(G, er) : mul9t(G, er);
                    arow[4 * u + w] = dot(eq, ge);
                    aqq = (4 * u + w == q) ? arow[4 * u + w] : aqq;
                }
            }
        }
        const float rq = md.eps_r * aqq;
#pragma unroll
        for (int c = 0; c < 16; ++c) arow[c] += c == q ? rq : 0.f;
        const float dq = frcp(aqq + rq);
        const float bq = dot(eq, v3(es[16], es[17], es[18])) - es[15];
        float f16[16];
        pgs_team(arow, bq, dq, m, q, md.n_pgs, f16);
#pragma unroll
        for (int r = 0; r < 16; ++r) f[r] = f16[r];
    } else {
        // up to MPPI_MAX_CONTACTS contacts: A, b, R, 1 / (A_rr + R_r) and the
        // multipliers in the team's LDS (rows of A split over the lanes)
        for (int idx = tc.t; idx < m * m; idx += TEAM) {
            const int r = idx / m, c = idx - r * m;
            const int s = r >> 2, q = r & 3, t = c >> 2, w = c & 3;
            const float *es = E + 20 * s + 3 * q, *et = E + 20 * t + 3 * w;
            const V3 eq = v3(es[0], es[1], es[2]), er = v3(et[0], et[1], et[2]);
            float G[9];
            const float *g = Gb + 9 * (s <= t ? s * NC + t : t * NC + s);
#pragma unroll
            for (int i = 0; i < 9; ++i) G[i] = g[i];
            const V3 ge = s <= t ? mul9(G, er) : mul9t(G, er);
            A[r * MR + c] = dot(eq, ge);
        }
        wave_lds_sync();
        for (int r = tc.t; r < m; r += TEAM) {
            const int s = r >> 2, q = r & 3;
            const float *es = E + 20 * s;
            const V3 eq = v3(es[3 * q], es[3 * q + 1], es[3 * q + 2]);
            const float arr = A[r * MR + r];
            const float rr = md.eps_r * arr;
            Rv[r] = rr;
            Dv[r] = frcp(arr + rr);
            Bv[r] = dot(eq, v3(es[16], es[17], es[18])) - es[15];
        }
        wave_lds_sync();
        if (TASK) {
            // the task forms carry one team a wave: the sweep lane-parallel
            pgs_wave<MR>(A, Bv, Dv, m, md.n_pgs, tc.lane, f);
        } else {
        float *F = Rv + MR;
        for (int r = 0; r < m; ++r) F[r] = 0.f;
        for (int sweep = 0; sweep < md.n_pgs; ++sweep) {
            for (int r = 0; r < m; ++r) {
                const float fr = F[r];
                float res = fmaf(Rv[r], fr, Bv[r]);
                const float4 *ar = reinterpret_cast<const float4 *>(A + r * MR);
                const float4 *f4 = reinterpret_cast<const float4 *>(F);
                for (int t = 0; t < nc; ++t) {
                    const float4 a4 = ar[t], x4 = f4[t];
                    res = fmaf(a4.x, x4.x, res);
                    res = fmaf(a4.y, x4.y, res);
                    res = fmaf(a4.z, x4.z, res);
                    res = fmaf(a4.w, x4.w, res);
                }
                F[r] = fmaxf(fr - res * Dv[r], 0.f);
            }
        }
#pragma unroll
        for (int r = 0; r < MR; ++r)
            if (r < m) f[r] = F[r];
        }
    }
    // impulses back: ball (geom A) directly, joints through Mt^-1 J^T
    float g = 0.f;  // generalized impulse of this lane's joint
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        if (s < nc) {
            const float *es = E + 20 * s;
            V3 P = v3(0.f, 0.f, 0.f);
#pragma unroll
            for (int q = 0; q < 4; ++q) P = fma3(f[4 * s + q], v3(es[3 * q], es[3 * q + 1], es[3 * q + 2]), P);
            if ((side_word >> (8 + s)) & 1) {
                vb = fma3(md.inv_ball_m, P, vb);
                if (box)
                    wb = wb + mul9(Wo, cross(v3(es[12], es[13], es[14]), P));
                else
                    wb = fma3(md.inv_ball_I, cross(v3(es[12], es[13], es[14]), P), wb);
            }
            g += dot(Jc[s], P);
        }
    }
    if (any_arm) {
        float dv = 0.f;
        static_for<NJ>([&](auto ec) {
            constexpr int e = decltype(ec)::value;
            dv = fmaf(Minv[e], segb<e>(g, tc.arm != 0), dv);
        });
        if (tc.joint) v += dv;
    }
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


// Dynamics half of a substep (before contacts): PD target, kinematics,
// joint-space inertia and its factor (parked for the contact path), bias
// forces and the free velocities (v of this lane's joint; ball vb with
// gravity; wb).  k receives this lane's kinematics at the current positions.
// the team's contact-solve area: per-contact frames E, then Delassus blocks,
// then the row matrix A (its first 248 floats double as the mass-matrix
// exchange of team_mass_rows, which runs before any solve of the substep)
template <int NC>
__device__ __forceinline__ float *team_solve_area(float *tl) { return tl + TG_FIELDS + NC * CL_FIELDS + PK_FIELDS4; }
template <int NC>
__device__ __forceinline__ float *team_row_area(float *tl) { return team_solve_area<NC>(tl) + 20 * NC + 9 * NC * NC; }

// HAVE_K: k already holds the kinematics at S.q
template <int NC, bool ROWS = false, bool TASK = false, bool HAVE_K = false>
__device__ inline void team_dynamics(const DevModel &md, const JointConst &jc, const TeamCtx &tc, TeamState &S,
                                     float u, JointKin &k, float &v, V3 &vb, V3 &wb)
{
    static_assert(16 * NC * NC >= 248, "the row area holds the mass-matrix exchange");
    const float h = md.h;
    const int jt = tc.jt, seg = tc.seg;
    S.qdes = fmaf(h, u, S.qdes);
    if (!HAVE_K) team_fk(jc, S.q, jt, k);
    float Lp[28];
    if (ROWS) {
        team_mass_rows(md, jc, k, jt, tc.t, tc.arm, tc.lane, team_row_area<NC>(tc.tl), Lp);
    } else {
        float row[NJ];
        team_crba(md, jc, k, jt, seg, row);
        team_gather_tri(row, seg, Lp);
    }
    chol7(Lp);
    const float c = team_rnea(md, jc, k, S.qd, jt, md.gravcomp == 0);
    const float tau = clampf(md.kp * (S.qdes - S.q) + md.kd * (u - S.qd), -md.tau_max, md.tau_max);
    const float rhs = h * (tau - md.damp * S.qd - c);
    float xs[NJ];
    static_for<NJ>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        xs[i] = segb<i>(rhs, seg != 0);
    });
    chol7_solve(Lp, xs);
    v = S.qd + pick7(xs, jt);
    vb = v3(S.vb.x, S.vb.y, S.vb.z - h * md.g);
    wb = (TASK && md.obj_box) ? obj_free_w(md, S.quat, S.wb) : S.wb;
    // park the factor for the contact solve (the team keeps the joint axes in
    // registers); it is replicated on the segment: its first lane parks it
    if (jt == 0) {
        float4 *o = reinterpret_cast<float4 *>(&tc.pk.at(PK_L + 28 * tc.arm));
#pragma unroll
        for (int e = 0; e < 7; ++e) o[e] = make_float4(Lp[4 * e], Lp[4 * e + 1], Lp[4 * e + 2], Lp[4 * e + 3]);
    }
}


// Geometry half: publish the kinematics and ball centre, the geom AABBs, and
// sweep the candidate pairs into the contact list (tc.LL); returns the count.
template <int G, bool TASK = false>
__device__ inline int team_contacts(const DevModel &md, const TeamCtx &tc, const JointKin &k, V3 pb,
                                    StepCounters &cnt, const float *q = nullptr)
{
    team_publish_geom_aabb<TASK>(tc.tl, tc.hd, k, pb, tc.arm, tc.jt, &md, q);
    const int nc = team_collect<G, TASK>(md, tc.tl, tc.hd, tc.LL, tc.li, tc.gshift, cnt);
    if (tc.t == 0) {
        cnt.contacts += nc;
        if (nc >= md.n_cmax) ++cnt.overflow;
    }
    wave_lds_sync();
    return nc;
}

// Semi-implicit Euler of the ball with its post-contact velocities: centre
// by h vb, orientation by the exponential map of h wb (world frame).
__device__ __forceinline__ void integrate_ball(const DevModel &md, TeamState &S, V3 vb, V3 wb)
{
    // Every product and sum is spelt out, with contraction off, so the update
    // rounds the same wherever it is inlined (either wave of the split mapping).
#pragma clang fp contract(off)
    const float h = md.h;
    S.pb = fma3(h, vb, S.pb);
    S.vb = vb;
    S.wb = wb;
    const V3 th = h * wb;
    const float ang = sqrtf(fmaf(th.x, th.x, fmaf(th.y, th.y, th.z * th.z)));
    float dw, dsc;
    half_angle_sincos(ang, dw, dsc);
    const V3 dv = dsc * th;
    const float qw = S.quat[0];
    const V3 qv = v3(S.quat[1], S.quat[2], S.quat[3]);
    // (dw, dv) * (qw, qv): scalar part dw qw - dv.qv, vector part dw qv + qw dv + dv x qv
    const float nw = fmaf(dw, qw, -fmaf(dv.x, qv.x, fmaf(dv.y, qv.y, dv.z * qv.z)));
    const V3 nv = v3(fmaf(dw, qv.x, fmaf(qw, dv.x, fmaf(dv.y, qv.z, -(dv.z * qv.y)))),
                     fmaf(dw, qv.y, fmaf(qw, dv.y, fmaf(dv.z, qv.x, -(dv.x * qv.z)))),
                     fmaf(dw, qv.z, fmaf(qw, dv.z, fmaf(dv.x, qv.y, -(dv.y * qv.x)))));
    const float inv = __builtin_amdgcn_rsqf(fmaf(nw, nw, fmaf(nv.x, nv.x, fmaf(nv.y, nv.y, nv.z * nv.z))));
    S.quat[0] = nw * inv;
    S.quat[1] = nv.x * inv;
    S.quat[2] = nv.y * inv;
    S.quat[3] = nv.z * inv;
}

// true when the substep's only contact is the ball against the table or a
// box: the arms are untouched and the ball's solve needs no arm data
__device__ __forceinline__ bool ball_only_contact(const LaneList &LL, int nc)
{
    return nc == 1 && __float_as_int(LL.at(0, 0)) == G_BALL &&
           (__float_as_int(LL.at(0, 1)) == G_TABLE || __float_as_int(LL.at(0, 1)) >= G_BOX);
}

// element i of a register array (i uniform over a 16-lane row)
template <int N>
__device__ __forceinline__ V3 pick_v3(const V3 (&a)[N], int i)
{
    V3 r = a[0];
#pragma unroll
    for (int k = 1; k < N; ++k) r = i == k ? v3(opaque(a[k].x), opaque(a[k].y), opaque(a[k].z)) : r;
    return r;
}

// bit s of the side word from lane 16 s of a wave ballot (s < 4)
__device__ __forceinline__ int row_bits(uint64_t b)
{
    return (int)((b & 1ull) | ((b >> 15) & 2ull) | ((b >> 30) & 4ull) | ((b >> 45) & 8ull));
}

// The same solve for a wave whose four 16-lane rows all carry one team (one
// sample a wave), nc <= 4: the per-contact and per-pair work is spread over
// the rows instead of repeated on each.  Row s builds contact s's frame and
// free velocity, row t the product Mt^-1 J_t^T; the Delassus blocks (s <= t,
// t-major) go to the rows four at a time; row u builds columns 4u..4u+3 of
// every lane's row of A, which the lanes read back whole.  Every value is
// formed by the same operations as in team_contact_solve, so the two agree
// bit for bit.
template <int NC, bool TASK = false>
__device__ inline void team_contact_solve_rows(const DevModel &md, const TeamCtx &tc, const JointKin &k, V3 pb, int nc,
                                               float &v, V3 &vb, V3 &wb, const float *Wo = nullptr)
{
    const bool box = TASK && md.obj_box;  // Wo: the box object's world inverse inertia
    constexpr int MR = 4 * NC;
    static_assert(MR >= 16, "the lane-parallel sweeps read 16 rows of A");
    float *E = tc.tl + TG_FIELDS + NC * CL_FIELDS + PK_FIELDS4;  // 16-byte aligned
    float *Gb = E + 20 * NC;
    float *A = Gb + 9 * NC * NC;  // first Mt^-1 J_t^T by contact and lane, then the rows of A
    const LaneList &LL = tc.LL;
    const int m = 4 * nc;
    const int row = tc.lane >> 4;
    // contact frames: row s builds contact s
    int side_word;
    {
        const int s = row;
        bool arm_s = false, ball_s = false;
        if (s < nc) {
            const int ga = __float_as_int(LL.at(s, 0)), gb = __float_as_int(LL.at(s, 1));
            const Sides sd = contact_sides(ga | (gb << 8));
            arm_s = (sd.armA >= 0) | (sd.armB >= 0);
            ball_s = sd.ball;
            const V3 n = v3(LL.at(s, 3), LL.at(s, 4), LL.at(s, 5));
            const V3 p = v3(LL.at(s, 6), LL.at(s, 7), LL.at(s, 8));
            V3 t1, t2;
            tangents(n, t1, t2);
            float *e = E + 20 * s;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const V3 t = q < 2 ? t1 : t2;
                const V3 eq = fma3((q & 1) ? -md.mu : md.mu, t, n);
                e[3 * q] = eq.x; e[3 * q + 1] = eq.y; e[3 * q + 2] = eq.z;
            }
            const V3 r = p - pb;
            e[12] = r.x; e[13] = r.y; e[14] = r.z;
            const float phi = LL.at(s, 2);
            e[15] = md.kappa_h * (phi < 0.f ? -phi : 0.f);
        }
        side_word = row_bits(__ballot(arm_s)) | (row_bits(__ballot(ball_s)) << 8);
    }
    const bool any_arm = (side_word & 0xff) != 0;
    // this lane's Jacobian columns
    V3 Jc[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        Jc[s] = v3(0.f, 0.f, 0.f);
        if (s < nc) {
            const int ga = __float_as_int(LL.at(s, 0)), gb = __float_as_int(LL.at(s, 1));
            const Sides sd = contact_sides(ga | (gb << 8));
            const V3 p = v3(LL.at(s, 6), LL.at(s, 7), LL.at(s, 8));
            const float coef = tc.joint ? jac_coef(sd, tc.arm, tc.jt) : 0.f;
            if (coef != 0.f) Jc[s] = coef * cross(k.a, p - k.o);
        }
    }
    // free contact velocity b_s: row s
    {
        const int s = row;
        if (s < nc) {
            V3 b = (side_word >> s) & 1 ? team_sum3(v * pick_v3(Jc, s)) : v3(0.f, 0.f, 0.f);
            if ((side_word >> (8 + s)) & 1) {
                const V3 p = v3(LL.at(s, 6), LL.at(s, 7), LL.at(s, 8));
                const V3 r = p - pb;
                b = b + vb + cross(wb, r);
            }
            float *e = E + 20 * s;
            e[16] = b.x; e[17] = b.y; e[18] = b.z;
        }
    }
    // row d of Mt^-1 of this lane's arm (only when an arm is in contact)
    float Minv[NJ];
#pragma unroll
    for (int e = 0; e < NJ; ++e) Minv[e] = 0.f;
    if (any_arm) {
        float Lf[28];
        team_parked_factor(tc.pk, tc.arm, Lf);
#pragma unroll
        for (int e = 0; e < NJ; ++e) Minv[e] = (tc.joint && e == tc.jt) ? 1.f : 0.f;
        chol7_solve(Lf, Minv);
        if (!tc.joint) {
#pragma unroll
            for (int e = 0; e < NJ; ++e) Minv[e] = 0.f;
        }
    }
    // row t: row d of Mt^-1 J_t^T, parked by contact and lane
    {
        const int t = row;
        V3 W = v3(0.f, 0.f, 0.f);
        if (t < nc && ((side_word >> t) & 1)) {
            const V3 Jt = pick_v3(Jc, t);
            static_for<NJ>([&](auto ec) {
                constexpr int e = decltype(ec)::value;
                W = fma3(Minv[e], segb3<e>(Jt, tc.arm != 0), W);
            });
        }
        float *w = A + 4 * (16 * t + tc.t);
        w[0] = W.x; w[1] = W.y; w[2] = W.z;
    }
    wave_lds_sync();
    // Delassus blocks G_st = J_s Mt^-1 J_t^T (+ the ball's), s <= t: pair p
    // (t-major) on row p mod 4
    {
        constexpr uint32_t PS = 0u | (0u << 2) | (1u << 4) | (0u << 6) | (1u << 8) | (2u << 10) | (0u << 12) | (1u << 14) |
                                (2u << 16) | (3u << 18);
        constexpr uint32_t PT = 0u | (1u << 2) | (1u << 4) | (2u << 6) | (2u << 8) | (2u << 10) | (3u << 12) | (3u << 14) |
                                (3u << 16) | (3u << 18);
        const int np = nc * (nc + 1) / 2;
        for (int p0 = 0; p0 < np; p0 += 4) {
            const int p = p0 + row;
            if (p < np) {
                const int s = (PS >> (2 * p)) & 3, t = (PT >> (2 * p)) & 3;
                float G[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (((side_word >> t) & 1) && ((side_word >> s) & 1)) {
                    const float *w = A + 4 * (16 * t + tc.t);
                    const V3 W = v3(w[0], w[1], w[2]);
                    const V3 J = pick_v3(Jc, s);
                    G[0] = team_sum(J.x * W.x); G[1] = team_sum(J.x * W.y); G[2] = team_sum(J.x * W.z);
                    G[3] = team_sum(J.y * W.x); G[4] = team_sum(J.y * W.y); G[5] = team_sum(J.y * W.z);
                    G[6] = team_sum(J.z * W.x); G[7] = team_sum(J.z * W.y); G[8] = team_sum(J.z * W.z);
                }
                if (((side_word >> (8 + t)) & 1) && ((side_word >> (8 + s)) & 1)) {
                    const V3 rs = v3(E[20 * s + 12], E[20 * s + 13], E[20 * s + 14]);
                    const V3 rt = v3(E[20 * t + 12], E[20 * t + 13], E[20 * t + 14]);
                    if (box)
                        obj_block(md, Wo, rs, rt, G);
                    else
                        ball_block(md, rs, rt, G);
                }
                float *g = Gb + 9 * (s * NC + t);
#pragma unroll
                for (int i = 0; i < 9; ++i) g[i] = G[i];
            }
        }
    }
    wave_lds_sync();
    // row u: columns 4u..4u+3 of lane q's row of A = E^T G E
    const int q = tc.t, sq = q >> 2;
    const float *es = E + 20 * sq;
    const V3 eq = v3(es[3 * (q & 3)], es[3 * (q & 3) + 1], es[3 * (q & 3) + 2]);
    {
        const int u = row;
        float a4[4] = {0.f, 0.f, 0.f, 0.f};
        if (u < nc) {
            float G[9];
            const bool up = sq <= u;  // G_{sq,u} = G_{u,sq}^T below the diagonal
            const float *g = Gb + 9 * (up ? sq * NC + u : u * NC + sq);
#pragma unroll
            for (int i = 0; i < 9; ++i) G[i] = g[i];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const float *eu = E + 20 * u + 3 * w;
                const V3 er = v3(eu[0], eu[1], eu[2]);
                const V3 ge = up ? mul9(G, er) : mul9t(G, er);
                a4[w] = dot(eq, ge);
            }
        }
        *reinterpret_cast<float4 *>(A + 16 * q + 4 * u) = make_float4(a4[0], a4[1], a4[2], a4[3]);
    }
    wave_lds_sync();
    float arow[16];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float4 a4 = *reinterpret_cast<const float4 *>(A + 16 * q + 4 * c);
        arow[4 * c] = a4.x; arow[4 * c + 1] = a4.y; arow[4 * c + 2] = a4.z; arow[4 * c + 3] = a4.w;
    }
    float aqq = 0.f;
#pragma unroll
    for (int c = 0; c < 16; ++c) aqq = c == q ? arow[c] : aqq;
    const float rq = md.eps_r * aqq;
#pragma unroll
    for (int c = 0; c < 16; ++c) arow[c] += c == q ? rq : 0.f;
    const float dq = frcp(aqq + rq);
    const float bq = dot(eq, v3(es[16], es[17], es[18])) - es[15];
    float f[16];
    pgs_team(arow, bq, dq, m, q, md.n_pgs, f);
    // impulses back: ball (geom A) directly, joints through Mt^-1 J^T
    float g = 0.f;  // generalized impulse of this lane's joint
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        if (s < nc) {
            const float *e = E + 20 * s;
            V3 P = v3(0.f, 0.f, 0.f);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) P = fma3(f[4 * s + qq], v3(e[3 * qq], e[3 * qq + 1], e[3 * qq + 2]), P);
            if ((side_word >> (8 + s)) & 1) {
                vb = fma3(md.inv_ball_m, P, vb);
                if (box)
                    wb = wb + mul9(Wo, cross(v3(e[12], e[13], e[14]), P));
                else
                    wb = fma3(md.inv_ball_I, cross(v3(e[12], e[13], e[14]), P), wb);
            }
            g += dot(Jc[s], P);
        }
    }
    if (any_arm) {
        float dv = 0.f;
        static_for<NJ>([&](auto ec) {
            constexpr int e = decltype(ec)::value;
            dv = fmaf(Minv[e], segb<e>(g, tc.arm != 0), dv);
        });
        if (tc.joint) v += dv;
    }
}

// Contact solve and semi-implicit Euler: the end of a substep.  ROWS: the
// wave's four 16-lane rows carry one team, so a solve of up to four contacts
// spreads its per-contact work over them.  PRIO: the caller runs at wave
// priority 1 and the general solve at 2 (issue priority only; the results
// do not change): a launch lasts as long as its slowest samples, which are
// the ones that spend many substeps in this solve.
template <int NC, bool ROWS = false, bool PRIO = false, bool TASK = false>
__device__ inline void team_finish(const DevModel &md, const TeamCtx &tc, TeamState &S, const JointKin &k, int nc,
                                   float v, V3 vb, V3 wb)
{
    const float h = md.h;
    const bool box = TASK && md.obj_box;
    float W[9];
    if (box) obj_world_inv_inertia(md, S.quat, W);
    if (!box && ball_only_contact(tc.LL, nc)) {
        ball_contact_solve(md, tc.LL, S.pb, vb, wb);
    } else if (ROWS && nc > 0 && nc <= 4) {
        if (PRIO) __builtin_amdgcn_s_setprio(2);
        team_contact_solve_rows<NC, TASK>(md, tc, k, S.pb, nc, v, vb, wb, W);
        if (PRIO) __builtin_amdgcn_s_setprio(1);
    } else if (nc > 0)
        team_contact_solve<NC, TASK>(md, tc, k, S.pb, nc, v, vb, wb, W);
    S.q = fmaf(h, v, S.q);
    S.qd = v;
    integrate_ball(md, S, vb, wb);
}

// One physics substep of a team: dynamics, contacts, solve, integration.
template <int NC, int G, bool ROWS = false, bool TASK = false>
__device__ inline void team_substep(const DevModel &md, const JointConst &jc, const TeamCtx &tc, TeamState &S,
                                    float u, StepCounters &cnt)
{
    JointKin k;
    float v;
    V3 vb, wb;
    team_dynamics<NC, ROWS, TASK>(md, jc, tc, S, u, k, v, vb, wb);
    const int nc = team_contacts<G, TASK>(md, tc, k, S.pb, cnt, S.quat);
    team_finish<NC, ROWS, false, TASK>(md, tc, S, k, nc, v, vb, wb);
}

// per-control-step cost at the post-step state; lane 0 accumulates the stage
// terms, joint lanes the smoothness, every lane its share of the cost pairs.
// PUBLISHED: the team's geometry and AABBs in LDS already belong to this
// state (a contact sweep at the same positions wrote them).
// TASK: the further terms too (kin: this state's joint kinematics when
// PUBLISHED; a box object's AABB is published with the geometry).
template <bool PUBLISHED = false, bool TASK = false>
__device__ inline void team_stage_cost(const DevModel &md, const JointConst &jc, const TeamCtx &tc,
                                       const TeamState &S, float u, float uprev, bool first, uint32_t &hist,
                                       float *dist, long stride, CostAcc &acc, StepCounters &cnt,
                                       const JointKin *kin = nullptr)
{
    JointKin k;
    if (!PUBLISHED) {
        team_fk<TASK>(jc, S.q, tc.jt, k);
        team_publish_geom_aabb<TASK>(tc.tl, tc.hd, k, S.pb, tc.arm, tc.jt, &md, S.quat);
    } else if (TASK) {
        k = *kin;
    }
    const float *tl = tc.tl;
    if (TASK && md.ext) {
        // joint deviation (a team sum), pad velocities v_a = sum_j qd_j a_j x
        // (p_a - o_j) as segment contributions summed with arm 2's negated,
        // pad orientations from the last joint lanes' frames
        const int d = 7 * tc.arm + (tc.joint ? tc.jt : 0);
        const float hq = tc.joint ? S.q - md.q_home[d] : 0.f;
        const float home = team_sum(hq * hq);
        const V3 pa = v3(tl[TG_PTS + 24 * tc.arm + 21], tl[TG_PTS + 24 * tc.arm + 22], tl[TG_PTS + 24 * tc.arm + 23]);
        const V3 vj = (tc.joint ? (tc.arm == 0 ? S.qd : -S.qd) : 0.f) * cross(k.a, pa - k.o);
        const V3 v12 = team_sum3(vj);
        const float ang = rot_angle(md.arotR[tc.arm], k.x, k.y, k.z);
        const float ang1 = row_bcast<6>(ang), ang2 = row_bcast<14>(ang);
        if (tc.t == 0) {
            const V3 p1 = v3(tl[TG_PTS + 21], tl[TG_PTS + 22], tl[TG_PTS + 23]);
            const V3 p2 = v3(tl[TG_PTS + 45], tl[TG_PTS + 46], tl[TG_PTS + 47]);
            acc.t[7] += sqrtf(home);
            acc.t[8] += fabsf(p1.z - p2.z);
            const float rv = dot(p1 - p2, v12);
            acc.t[9] = fmaf(rv, rv, acc.t[9]);
            const V3 d1 = p1 - v3(md.apos[0][0], md.apos[0][1], md.apos[0][2]);
            const V3 d2 = p2 - v3(md.apos[1][0], md.apos[1][1], md.apos[1][2]);
            acc.t[10] += sqrtf(dot(d1, d1));
            acc.t[11] += sqrtf(dot(d2, d2));
            acc.t[12] += fabsf(p1.x - md.ax_t[0]);
            acc.t[13] += fabsf(p2.x - md.ax_t[1]);
            acc.t[14] += ang1;
            acc.t[15] += ang2;
            const float qw = S.quat[0], Qw = md.orot[0];
            const V3 qv = v3(S.quat[1], S.quat[2], S.quat[3]), Qv = v3(md.orot[1], md.orot[2], md.orot[3]);
            const float wr = fmaf(Qw, qw, dot(Qv, qv));
            const V3 vr = Qw * qv - qw * Qv - cross(Qv, qv);
            acc.t[16] += 2.0f * atan2f(sqrtf(dot(vr, vr)), fabsf(wr));
        }
    }
    if (tc.t == 0) {
        const V3 p1 = v3(tl[TG_PTS + 21], tl[TG_PTS + 22], tl[TG_PTS + 23]);
        const V3 p2 = v3(tl[TG_PTS + 45], tl[TG_PTS + 46], tl[TG_PTS + 47]);
        const V3 pb = S.pb;
        const V3 dg = pb - v3(md.goal[0], md.goal[1], md.goal[2]);
        const V3 de = 0.5f * (p1 + p2) - v3(pb.x, pb.y, pb.z - md.eps);
        const V3 d12 = p1 - p2;
        acc.t[0] += sqrtf(dot(dg, dg));
        acc.t[1] += sqrtf(dot(de, de));
        const float l = sqrtf(dot(d12, d12)) - md.l_cost;
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
        const int gab = __float_as_int(tc.hd[HD_PAIR + p]);
        const int ga = gab & 0xff, gb = gab >> 8;
        if (pair_overlap(tl, tc.hd, ga, gb, md.m_c)) {
            const Shape A = team_geom(tl, tc.hd, ga), B = team_geom(tl, tc.hd, gb);
            if (tc.count) {
                ++cnt.np_tests;
                if (B.type == SH_BOX && A.type == SH_CAPSULE) ++cnt.box_tests;
            }
            const float d = narrow(A, B).phi;
            dist_term(md, d, !first, hist, 1u << r, dist + (long)i * stride, nw, acc);
        }
    }
    hist = nw;
}

}  // namespace mppi
