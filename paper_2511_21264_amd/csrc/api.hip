// Host side of the C ABI declared in include/mppi.h: argument checks, scene
// model derivation and upload, device buffers, staging of host arrays and
// the launch sequence of a plan (M x [rollout -> stats -> update]).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mppi.h"
#include "internal.h"

using namespace mppi;
using namespace mppi_host;

namespace mppi_host {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace mppi_host

namespace {

int ensure(mppi_ctx *c, int slot, size_t bytes, void **out)
{
    Buf &b = c->buf[slot];
    if (bytes == 0) bytes = 16;
    if (b.cap < bytes) {
        // cached graphs bake in the old address: drop them with the buffer
        if (b.p) {
            (void)hipDeviceSynchronize();
            drop_graphs(c);
            (void)hipFree(b.p);
        }
        b.p = nullptr;
        b.cap = 0;
        size_t want = bytes + bytes / 4;
        if (hipMalloc(&b.p, want) != hipSuccess) {
            b.p = nullptr;
            return fail(MPPI_E_NOMEM, "device allocation of %zu bytes failed", want);
        }
        b.cap = want;
    }
    *out = b.p;
    return MPPI_OK;
}

// device view of a caller input: the pointer itself, or a staged copy
int stage_in(mppi_ctx *c, int slot, const void *src, size_t bytes, bool dev, hipStream_t s, const void **out)
{
    if (dev) {
        *out = src;
        return MPPI_OK;
    }
    void *d;
    int rc = ensure(c, slot, bytes, &d);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, s));
    *out = d;
    return MPPI_OK;
}

int out_ptr(mppi_ctx *c, int slot, void *dst, size_t bytes, bool dev, void **out)
{
    if (!dst) {
        *out = nullptr;
        return MPPI_OK;
    }
    if (dev) {
        *out = dst;
        return MPPI_OK;
    }
    return ensure(c, slot, bytes, out);
}

int copy_out(void *dst, const void *src, size_t bytes, bool dev, hipStream_t s)
{
    if (!dst || dev || !src) return MPPI_OK;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    return MPPI_OK;
}

// solid capsule: cylinder length L plus two hemispherical caps of radius r
void capsule_mass_inertia(double rho, double L, double r, double &m, double &ix, double &iz)
{
    const double pi = 3.14159265358979323846;
    const double m_cyl = rho * pi * r * r * L;
    const double m_sph = rho * (4.0 / 3.0) * pi * r * r * r;
    m = m_cyl + m_sph;
    iz = 0.5 * m_cyl * r * r + 0.4 * m_sph * r * r;
    // caps: sphere inertia about a diameter plus the shift of each half to
    // the capsule centre (centroid 3r/8 from the flat face at L/2)
    ix = m_cyl * (L * L / 12.0 + r * r / 4.0) + m_sph * (0.4 * r * r + L * L / 4.0 + 3.0 * L * r / 8.0);
}

bool finite_desc(const mppi_scene_desc *d)
{
    const double *vals[] = {&d->pad_rad, &d->ball_r, &d->ball_m, &d->h, &d->kp, &d->kd, &d->damp, &d->armature,
                            &d->tau_max, &d->g, &d->mu, &d->kappa, &d->eps_r, &d->u_max, &d->w_goal, &d->w_eo,
                            &d->w_l, &d->w_yz, &d->w_s, &d->w_c, &d->gamma, &d->m_c, &d->eps_frac};
    for (const double *v : vals)
        if (!std::isfinite(*v)) return false;
    for (int i = 0; i < 7; ++i)
        if (!std::isfinite(d->link_len[i]) || !std::isfinite(d->link_rad[i]) || !std::isfinite(d->density[0][i]) ||
            !std::isfinite(d->density[1][i]))
            return false;
    return true;
}

int build_model(const mppi_scene_desc *d, DevModel &m)
{
    if (!finite_desc(d)) return fail(MPPI_E_MODEL, "scene description has non-finite values");
    if (d->n_box < 0 || d->n_box > MPPI_MAX_BOXES) return fail(MPPI_E_MODEL, "n_box %d outside [0, %d]", d->n_box, MPPI_MAX_BOXES);
    if (!(d->h > 0) || d->n_sub < 1) return fail(MPPI_E_MODEL, "need h > 0 and n_sub >= 1");
    if (d->n_cmax < 0 || d->n_cmax > MPPI_MAX_CONTACTS) return fail(MPPI_E_MODEL, "n_cmax %d outside [0, %d]", d->n_cmax, MPPI_MAX_CONTACTS);
    if (d->n_pgs < 0) return fail(MPPI_E_MODEL, "n_pgs < 0");
    if (!(d->ball_r > 0) || !(d->ball_m > 0) || !(d->pad_rad > 0)) return fail(MPPI_E_MODEL, "ball and pad need positive size and mass");
    if (!(d->armature > 0)) return fail(MPPI_E_MODEL, "armature must be > 0 (keeps the joint-space inertia SPD)");
    if (d->kd < 0 || d->damp < 0 || d->kp < 0 || !(d->tau_max > 0)) return fail(MPPI_E_MODEL, "gains must be >= 0, tau_max > 0");
    if (!(d->u_max > 0) || d->mu < 0 || d->kappa < 0 || d->eps_r < 0) return fail(MPPI_E_MODEL, "bad contact or control bounds");
    if (!(d->m_c > 0) || !(d->gamma > 0 && d->gamma < 1)) return fail(MPPI_E_MODEL, "need m_c > 0 and 0 < gamma < 1");
    for (int a = 0; a < 2; ++a) {
        const double c = d->base_cs[a][0], s = d->base_cs[a][1];
        if (!(std::fabs(c * c + s * s - 1.0) <= 1e-6))
            return fail(MPPI_E_MODEL, "base_cs[%d] must be the (cos, sin) of a yaw", a);
    }
    std::memset(&m, 0, sizeof m);
    for (int a = 0; a < 2; ++a) {
        for (int i = 0; i < 3; ++i) m.base_pos[a][i] = (float)d->base_pos[a][i];
        m.base_cs[a][0] = (float)d->base_cs[a][0];
        m.base_cs[a][1] = (float)d->base_cs[a][1];
    }
    for (int i = 0; i < NJ; ++i) {
        if (d->axes[i] < 0 || d->axes[i] > 2) return fail(MPPI_E_MODEL, "axes[%d] must be 0, 1 or 2", i);
        if (!(d->link_len[i] > 0) || !(d->link_rad[i] > 0)) return fail(MPPI_E_MODEL, "link %d needs positive length and radius", i);
        m.axes[i] = d->axes[i];
        m.link_len[i] = (float)d->link_len[i];
        m.link_rad[i] = (float)d->link_rad[i];
        for (int a = 0; a < 2; ++a) {
            if (!(d->density[a][i] > 0)) return fail(MPPI_E_MODEL, "density[%d][%d] must be > 0", a, i);
            double mm, ix, iz;
            capsule_mass_inertia(d->density[a][i], d->link_len[i], d->link_rad[i], mm, ix, iz);
            m.m[a][i] = (float)mm;
            m.Ix[a][i] = (float)ix;
            m.Iz[a][i] = (float)iz;
        }
    }
    m.pad_rad = (float)d->pad_rad;
    m.ball_r = (float)d->ball_r;
    m.ball_m = (float)d->ball_m;
    m.inv_ball_m = (float)(1.0 / d->ball_m);
    m.inv_ball_I = (float)(1.0 / (0.4 * d->ball_m * d->ball_r * d->ball_r));
    m.n_box = d->n_box;
    for (int b = 0; b < d->n_box; ++b)
        for (int i = 0; i < 3; ++i) {
            if (!std::isfinite(d->box_c[b][i]) || !(d->box_h[b][i] > 0)) return fail(MPPI_E_MODEL, "box %d is malformed", b);
            m.box_c[b][i] = (float)d->box_c[b][i];
            m.box_h[b][i] = (float)d->box_h[b][i];
        }
    m.h = (float)d->h;
    m.n_sub = d->n_sub;
    m.kp = (float)d->kp;
    m.kd = (float)d->kd;
    m.damp = (float)d->damp;
    m.tau_max = (float)d->tau_max;
    m.diag_add = (float)(d->armature + d->h * (d->kd + d->damp));
    m.gravcomp = d->gravcomp;
    m.g = (float)d->g;
    m.mu = (float)d->mu;
    m.kappa_h = (float)(d->kappa / d->h);
    m.eps_r = (float)d->eps_r;
    m.n_pgs = d->n_pgs;
    m.n_cmax = d->n_cmax;
    m.u_max = (float)d->u_max;
    for (int i = 0; i < 3; ++i) m.goal[i] = (float)d->goal[i];
    m.w_goal = (float)d->w_goal;
    m.w_eo = (float)d->w_eo;
    m.w_l = (float)d->w_l;
    m.w_yz = (float)d->w_yz;
    m.w_s = (float)d->w_s;
    m.w_c = (float)d->w_c;
    m.one_m_gamma = (float)(1.0 - d->gamma);
    m.m_c = (float)d->m_c;
    const double eps = d->eps_frac * d->ball_r, rr = d->ball_r + d->pad_rad;
    if (!(rr > eps) || eps < 0) return fail(MPPI_E_MODEL, "grasp offset eps must lie in [0, r_ball + r_pad)");
    m.eps = (float)eps;
    m.l_ball = (float)(2.0 * std::sqrt(rr * rr - eps * eps));
    // candidate pairs in canonical order
    int n = 0;
    auto add = [&](int a, int b) {
        m.pa[n] = (uint8_t)a;
        m.pb[n] = (uint8_t)b;
        ++n;
    };
    add(G_BALL, G_TABLE);
    for (int a = 0; a < 2; ++a) add(G_BALL, G_ARM + 7 * a + 6);
    for (int a = 0; a < 2; ++a)
        for (int g = 0; g < 6; ++g) add(G_BALL, G_ARM + 7 * a + g);
    for (int b = 0; b < d->n_box; ++b) add(G_BALL, G_BOX + b);
    for (int a = 0; a < 2; ++a)
        for (int g = 1; g < 7; ++g) add(G_ARM + 7 * a + g, G_TABLE);
    m.cost_first = n + 0;  // informational: arm-box pairs start here
    for (int a = 0; a < 2; ++a)
        for (int g = 0; g < 7; ++g)
            for (int b = 0; b < d->n_box; ++b) add(G_ARM + 7 * a + g, G_BOX + b);
    for (int g = 0; g < 7; ++g)
        for (int g2 = 0; g2 < 7; ++g2) add(G_ARM + g, G_ARM + 7 + g2);
    m.n_pairs = n;
    m.n_cost = 14 * d->n_box + 49;
    // the free object and the further task-cost terms
    if (d->obj_box != 0 && d->obj_box != 1) return fail(MPPI_E_MODEL, "obj_box must be 0 (ball) or 1 (box)");
    m.obj_box = d->obj_box;
    m.ext = d->ext ? 1 : 0;
    m.task_form = m.obj_box | m.ext;
    const double inv_I_ball = 1.0 / (0.4 * d->ball_m * d->ball_r * d->ball_r);
    for (int i = 0; i < 3; ++i) {
        m.obj_I[i] = (float)(0.4 * d->ball_m * d->ball_r * d->ball_r);
        m.obj_iI[i] = (float)inv_I_ball;
    }
    if (m.obj_box) {
        for (int i = 0; i < 3; ++i)
            if (!(d->obj_h[i] > 0) || !std::isfinite(d->obj_h[i])) return fail(MPPI_E_MODEL, "obj_h must be finite and > 0");
        const double *hh = d->obj_h;
        const double I[3] = {d->ball_m * (hh[1] * hh[1] + hh[2] * hh[2]) / 3.0,
                             d->ball_m * (hh[0] * hh[0] + hh[2] * hh[2]) / 3.0,
                             d->ball_m * (hh[0] * hh[0] + hh[1] * hh[1]) / 3.0};
        for (int i = 0; i < 3; ++i) {
            m.obj_h[i] = (float)hh[i];
            m.obj_I[i] = (float)I[i];
            m.obj_iI[i] = (float)(1.0 / I[i]);
        }
    }
    if (!std::isfinite(d->l_target)) return fail(MPPI_E_MODEL, "non-finite l_target");
    m.l_cost = d->l_target > 0 ? (float)d->l_target : m.l_ball;
    const double wx[] = {d->w_home, d->w_vert, d->w_relv, d->w_orot, d->w_apos[0], d->w_apos[1], d->w_ax[0],
                         d->w_ax[1], d->w_arot[0], d->w_arot[1], d->ax_t[0], d->ax_t[1]};
    for (double v : wx)
        if (!std::isfinite(v)) return fail(MPPI_E_MODEL, "non-finite task-cost weight or target");
    for (int i = 0; i < 14; ++i) {
        if (!std::isfinite(d->q_home[i])) return fail(MPPI_E_MODEL, "non-finite q_home");
        m.q_home[i] = (float)d->q_home[i];
    }
    m.w_home = (float)d->w_home;
    m.w_vert = (float)d->w_vert;
    m.w_relv = (float)d->w_relv;
    m.w_orot = (float)d->w_orot;
    auto unit = [](const double *q, double *o) {
        const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        if (!(nq > 0) || !std::isfinite(nq)) return false;
        for (int i = 0; i < 4; ++i) o[i] = q[i] / nq;
        return true;
    };
    for (int a = 0; a < 2; ++a) {
        m.w_apos[a] = (float)d->w_apos[a];
        m.w_ax[a] = (float)d->w_ax[a];
        m.w_arot[a] = (float)d->w_arot[a];
        m.ax_t[a] = (float)d->ax_t[a];
        for (int i = 0; i < 3; ++i) {
            if (!std::isfinite(d->apos[a][i])) return fail(MPPI_E_MODEL, "non-finite apos");
            m.apos[a][i] = (float)d->apos[a][i];
        }
        double q[4];
        if (!unit(d->arot[a], q)) return fail(MPPI_E_MODEL, "arot[%d] is not a finite non-zero quaternion", a);
        const double w = q[0], x = q[1], y = q[2], z = q[3];
        const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                             2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                             2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        for (int i = 0; i < 9; ++i) m.arotR[a][i] = (float)R[i];
    }
    double qo[4];
    if (!unit(d->orot, qo)) return fail(MPPI_E_MODEL, "orot is not a finite non-zero quaternion");
    for (int i = 0; i < 4; ++i) m.orot[i] = (float)qo[i];
    return MPPI_OK;
}

}  // namespace

namespace mppi_host {

int mapping_of(unsigned flags)
{
    if (flags & MPPI_MAP_LANE) return MAP_LANE;
    if (flags & MPPI_MAP_TEAM) return MAP_TEAM;
    if (flags & MPPI_MAP_WAVE) return MAP_WAVE;
    if (flags & MPPI_MAP_SPLIT) return MAP_SPLIT;
    return MAP_AUTO;
}

int k_class(long K)
{
    int b = 0;
    while (b < 20 && (1L << b) < K) ++b;
    return b;
}

int resolve_mapping(const mppi_ctx *c, long K, unsigned flags)
{
    const int pinned = mapping_of(flags);
    if (pinned != MAP_AUTO) return pinned;
    const int Kc = (int)std::min<long>(K, MPPI_MAX_K);
    if (c && c->tuned_map[k_class(Kc)]) return c->tuned_map[k_class(Kc)];
    return pick_mapping(Kc, MAP_AUTO);
}

int family_launch_mapping(const mppi_ctx *c, int family, long total_k, unsigned flags)
{
    if (family == MAP_TASK) return MAP_TASK;  // a pin can only have been the lane mapping
    if (family == MAP_TASK_WAVE) {
        const int pinned = mapping_of(flags);
        if (pinned == MAP_SPLIT) return MAP_TASK_SPLIT;
        if (pinned == MAP_WAVE) return MAP_TASK_WAVE;
        return resolve_mapping(c, total_k, flags) == MAP_SPLIT ? MAP_TASK_SPLIT : MAP_TASK_WAVE;
    }
    const int pinned = mapping_of(flags);
    if (pinned != MAP_AUTO) return pinned;
    if (family == MAP_LANE) return MAP_LANE;
    const int m = resolve_mapping(c, total_k, flags);
    return m == MAP_LANE ? MAP_TEAM : m;  // the team family's form for the most samples
}

int set_device(mppi_ctx *c)
{
    HIPCHK(hipSetDevice(c->device));
    return MPPI_OK;
}

int scene_mapping(const mppi_ctx *c, const mppi_scene *s, long K, unsigned flags, int *map)
{
    const int pinned = mapping_of(flags);
    if (s->host.task_form) {
        // the task forms: one lane, one wave or two waves per sample
        if (pinned == MAP_TEAM)
            return fail(MPPI_E_INVAL, "scenes with a box object or the further task-cost terms run one lane, one "
                                      "wave or two waves per sample, not four samples a wave");
        // unpinned: one lane per sample from 16 k samples on (the task forms
        // have no four-samples-a-wave form: at 32 k samples one lane per
        // sample runs 1.5 x faster than a wave per sample), else the wave or
        // split form that the ball scenes get for K
        int m = pinned;
        if (m == MAP_AUTO) m = K >= 16384 ? MAP_LANE : resolve_mapping(c, K, flags);
        *map = m == MAP_LANE ? MAP_TASK : m == MAP_SPLIT ? MAP_TASK_SPLIT : MAP_TASK_WAVE;
        return MPPI_OK;
    }
    *map = resolve_mapping(c, K, flags);
    return MPPI_OK;
}

void drop_graphs(mppi_ctx *c)
{
    for (auto &g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

std::atomic<uint64_t> g_scene_gen{0};

bool all_finite(const float *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace mppi_host

namespace {

// Working memory of mppi_plan_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never names it except to look
// up its device address (kept per device in g_scratch_dev); kernels receive
// that address like any other buffer.
static __device__ __align__(256) unsigned char scratch[MPPI_NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
void *g_scratch_dev[MAX_DEVICES] = {nullptr};
std::mutex g_scratch_mu;

// with `device` current: look up the array's address on it (once per device)
int scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return fail(MPPI_E_INVAL, "device %d beyond %d", device, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return MPPI_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(MPPI_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_dev[device] = p;
    return MPPI_OK;
}

// byte offsets of mppi_plan_noalloc's buffers in the array
struct NoallocLayout {
    size_t st, nu, w, cnt, dist, costs, total;
};

NoallocLayout noalloc_layout(long K, long H, long n_cost)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    NoallocLayout L;
    size_t o = 0;
    L.st = o;
    o += al(sizeof(PlanStats));
    L.nu = o;
    o += al((size_t)H * NU * sizeof(float));
    L.w = o;
    o += al((size_t)K * sizeof(double));
    L.cnt = o;
    o += al((size_t)K * 4 * sizeof(int));
    L.dist = o;  // the collision-distance history, [n_cost][K]
    o += al((size_t)K * n_cost * sizeof(float));
    L.costs = o;
    o += al((size_t)K * sizeof(float));
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

const char *mppi_last_error(void) { return mppi_host::g_err.c_str(); }

int mppi_ctx_create(int device, mppi_ctx **out)
{
    if (!out) return fail(MPPI_E_INVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0) HIPCHK(hipGetDevice(&device));
    if (device >= n) return fail(MPPI_E_INVAL, "device %d not present (%d devices)", device, n);
    mppi_ctx *c = new mppi_ctx();
    c->device = device;
    if (hipSetDevice(device) != hipSuccess || hipMalloc((void **)&c->st, sizeof(PlanStats)) != hipSuccess ||
        hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming) != hipSuccess) {
        if (c->st) (void)hipFree(c->st);
        delete c;
        return fail(MPPI_E_NOMEM, "context allocation failed");
    }
    const int rc = scratch_init(device);  // the device is current
    if (rc) {
        mppi_ctx_destroy(c);
        return rc;
    }
    *out = c;
    return MPPI_OK;
}

void mppi_ctx_destroy(mppi_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &b : c->buf)
        if (b.p) (void)hipFree(b.p);
    if (c->st) (void)hipFree(c->st);
    for (auto e : c->ev) (void)hipEventDestroy(e);
    if (c->order_ev) (void)hipEventDestroy(c->order_ev);
    if (c->host_tab) (void)hipHostFree(c->host_tab);
    drop_graphs(c);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    delete c;
}

int mppi_scene_create(mppi_ctx *ctx, const mppi_scene_desc *desc, mppi_scene **out)
{
    if (!ctx || !desc || !out) return fail(MPPI_E_INVAL, "NULL argument");
    *out = nullptr;
    mppi_scene *s = new mppi_scene();
    s->ctx = ctx;
    s->gen = ++g_scene_gen;
    s->desc = *desc;
    int rc = build_model(desc, s->host);
    if (rc) {
        delete s;
        return rc;
    }
    if (set_device(ctx) || hipMalloc((void **)&s->dev, sizeof(DevModel)) != hipSuccess) {
        delete s;
        return fail(MPPI_E_NOMEM, "scene allocation failed");
    }
    if (hipMemcpy(s->dev, &s->host, sizeof(DevModel), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(s->dev);
        delete s;
        return fail(MPPI_E_DEVICE, "scene upload failed");
    }
    *out = s;
    return MPPI_OK;
}

void mppi_scene_destroy(mppi_scene *s)
{
    if (!s) return;
    (void)hipSetDevice(s->ctx->device);
    (void)hipDeviceSynchronize();
    // graphs of this scene's plans read its model: evict them
    auto &gs = s->ctx->graphs;
    for (size_t i = 0; i < gs.size();) {
        if (gs[i].key[0] == (uintptr_t)s->gen) {
            (void)hipGraphExecDestroy(gs[i].exec);
            (void)hipGraphDestroy(gs[i].graph);
            gs.erase(gs.begin() + i);
        } else {
            ++i;
        }
    }
    if (s->dev) (void)hipFree(s->dev);
    delete s;
}

int mppi_scene_num_pairs(const mppi_scene *s, int *n_pairs, int *n_cost)
{
    if (!s) return fail(MPPI_E_INVAL, "NULL scene");
    if (n_pairs) *n_pairs = s->host.n_pairs;
    if (n_cost) *n_cost = s->host.n_cost;
    return MPPI_OK;
}

// Checks of the QP smoothing's parameters for horizon H.
static int qp_check(const mppi_qp *qp, int H)
{
    if (!qp) return fail(MPPI_E_INVAL, "NULL qp");
    if (H > 128) return fail(MPPI_E_INVAL, "QP smoothing supports H <= 128 (H=%d)", H);
    if (!(qp->rho > 0) || !std::isfinite(qp->rho)) return fail(MPPI_E_INVAL, "qp rho must be finite and > 0");
    if (!(qp->alpha > 0 && qp->alpha < 2)) return fail(MPPI_E_INVAL, "qp alpha must lie in (0, 2)");
    if (qp->iters < 1 || qp->iters > 10000) return fail(MPPI_E_INVAL, "qp iters=%d out of range", qp->iters);
    if (!(qp->acc_max > 0) || !std::isfinite(qp->acc_max) || !(qp->jerk_max > 0) || !std::isfinite(qp->jerk_max))
        return fail(MPPI_E_INVAL, "qp acc_max and jerk_max must be finite and > 0");
    for (int d = 0; d < NU; ++d)
        if (!std::isfinite(qp->pos_lo[d]) || !std::isfinite(qp->pos_hi[d]) || !(qp->pos_lo[d] < qp->pos_hi[d]))
            return fail(MPPI_E_INVAL, "qp position bounds of joint %d must be finite with lo < hi", d);
    return MPPI_OK;
}

// (I + rho A^T A)^-1 for A = [I; D1; D2; L] on H steps, in double, stored as
// float rows of stride S (zero padded) in the context's QP slot.
static int qp_matrix(mppi_ctx *ctx, int H, double rho, hipStream_t stream, const float **out, int *S)
{
    const int st = ((H + 3) & ~3) + 4;
    void *dp;
    int rc;
    if ((rc = ensure(ctx, S_QPP, (size_t)H * st * sizeof(float), &dp))) return rc;
    if (ctx->qp_H != H || ctx->qp_rho != rho || ctx->qp_S != st) {
        std::vector<double> M((size_t)H * H, 0.0);
        auto add_row = [&](const std::vector<std::pair<int, double>> &row) {
            for (auto &a : row)
                for (auto &b : row) M[(size_t)a.first * H + b.first] += rho * a.second * b.second;
        };
        for (int k = 0; k < H; ++k) add_row({{k, 1.0}});
        for (int k = 1; k < H; ++k) add_row({{k, 1.0}, {k - 1, -1.0}});
        for (int k = 2; k < H; ++k) add_row({{k, 1.0}, {k - 1, -2.0}, {k - 2, 1.0}});
        for (int i = 0; i < H; ++i)  // prefix sums: (L^T L)_ij = H - max(i, j)
            for (int j = 0; j < H; ++j) M[(size_t)i * H + j] += rho * (double)(H - std::max(i, j));
        for (int i = 0; i < H; ++i) M[(size_t)i * H + i] += 1.0;
        // Cholesky M = C C^T, then the inverse column by column
        std::vector<double> C((size_t)H * H, 0.0);
        for (int j = 0; j < H; ++j) {
            double dsum = M[(size_t)j * H + j];
            for (int k = 0; k < j; ++k) dsum -= C[(size_t)j * H + k] * C[(size_t)j * H + k];
            if (!(dsum > 0)) return fail(MPPI_E_INVAL, "QP system not positive definite");
            const double cjj = std::sqrt(dsum);
            C[(size_t)j * H + j] = cjj;
            for (int i = j + 1; i < H; ++i) {
                double v = M[(size_t)i * H + j];
                for (int k = 0; k < j; ++k) v -= C[(size_t)i * H + k] * C[(size_t)j * H + k];
                C[(size_t)i * H + j] = v / cjj;
            }
        }
        std::vector<float> P((size_t)H * st, 0.f);
        std::vector<double> x(H);
        for (int c = 0; c < H; ++c) {
            for (int i = 0; i < H; ++i) {  // C y = e_c
                double v = i == c ? 1.0 : 0.0;
                for (int k = 0; k < i; ++k) v -= C[(size_t)i * H + k] * x[k];
                x[i] = v / C[(size_t)i * H + i];
            }
            for (int i = H - 1; i >= 0; --i) {  // C^T z = y
                double v = x[i];
                for (int k = i + 1; k < H; ++k) v -= C[(size_t)k * H + i] * x[k];
                x[i] = v / C[(size_t)i * H + i];
            }
            for (int i = 0; i < H; ++i) P[(size_t)i * st + c] = (float)x[i];
        }
        // work queued on this stream may still read the previous matrix
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(hipMemcpy(dp, P.data(), P.size() * sizeof(float), hipMemcpyHostToDevice));
        ctx->qp_H = H;
        ctx->qp_rho = rho;
        ctx->qp_S = st;
    }
    *out = (const float *)dp;
    *S = st;
    return MPPI_OK;
}

static void qp_args(ProjectArgs &pa, const mppi_scene *scene, const mppi_qp *qp, const float *P, int S, int K, int H)
{
    const double dt = scene->host.h * scene->host.n_sub;
    pa.P = P;
    pa.S = S;
    pa.K = K;
    pa.H = H;
    pa.dt = (float)dt;
    pa.u_max = scene->host.u_max;
    pa.dacc = (float)(qp->acc_max * dt);
    pa.djerk = (float)(qp->jerk_max * dt * dt);
    for (int d = 0; d < NU; ++d) {
        pa.pos_lo[d] = (float)qp->pos_lo[d];
        pa.pos_hi[d] = (float)qp->pos_hi[d];
    }
    pa.rho = (float)qp->rho;
    pa.alpha = (float)qp->alpha;
    pa.iters = qp->iters;
}

// mppi_plan, mppi_plan_qp and mppi_plan_cov (qp non-null: the samples are
// projected and stored, the rollout and the update read them; cov non-null:
// they are drawn with the factor of the full covariance, which is updated
// after the mean)
static int plan_impl(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                     double lambda, const float *sigma, const mppi_opts *opts, const mppi_qp *qp,
                     const mppi_cov *cov, float *U_new, float *costs, mppi_stats *stats, void *stream,
                     float *U_best)
{
    if (!ctx || !scene || !x0 || !nominal_U || !sigma || !opts || !U_new) return fail(MPPI_E_INVAL, "NULL argument");
    if (scene->ctx != ctx) return fail(MPPI_E_INVAL, "scene belongs to another context");
    if (K < 1 || K > MPPI_MAX_K || H < 1 || H > MPPI_MAX_H) return fail(MPPI_E_INVAL, "K=%d or H=%d out of range", K, H);
    if (!(lambda > 0) || !std::isfinite(lambda)) return fail(MPPI_E_INVAL, "lambda must be finite and > 0");
    if (opts->M < 1 || opts->M > 100000) return fail(MPPI_E_INVAL, "M=%d out of range", opts->M);
    if (!std::isfinite(opts->eta)) return fail(MPPI_E_INVAL, "eta must be finite");
    const unsigned fl = opts->flags;
    const bool dev = fl & MPPI_DEVICE_PTRS;
    const bool sps = fl & MPPI_SIGMA_PER_STEP;
    const size_t nsig = sps ? (size_t)H * NU : NU;
    if (!dev) {
        if (!all_finite(x0, NX) || !all_finite(nominal_U, (size_t)H * NU) || !all_finite(sigma, nsig))
            return fail(MPPI_E_INVAL, "non-finite input");
        for (size_t i = 0; i < nsig; ++i)
            if (sigma[i] < 0) return fail(MPPI_E_INVAL, "sigma must be >= 0");
    }
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const void *dx0, *dsig, *dnom;
    if ((rc = stage_in(ctx, S_X0, x0, NX * sizeof(float), dev, s, &dx0))) return rc;
    if ((rc = stage_in(ctx, S_SIGMA, sigma, nsig * sizeof(float), dev, s, &dsig))) return rc;
    if ((rc = stage_in(ctx, S_NOM, nominal_U, (size_t)H * NU * sizeof(float), dev, s, &dnom))) return rc;
    void *dnu, *dcost, *dw, *dcnt;
    if ((rc = ensure(ctx, S_NU, (size_t)H * NU * sizeof(float), &dnu))) return rc;
    if ((rc = ensure(ctx, S_W, (size_t)K * sizeof(double), &dw))) return rc;
    if ((rc = ensure(ctx, S_CNT, (size_t)K * 4 * sizeof(int), &dcnt))) return rc;
    void *ddist;
    if ((rc = ensure(ctx, S_DIST, (size_t)K * MAXCOST * sizeof(float), &ddist))) return rc;
    if ((rc = out_ptr(ctx, S_COSTS, costs, (size_t)K * sizeof(float), dev, &dcost))) return rc;
    if (!dcost && (rc = ensure(ctx, S_COSTS, (size_t)K * sizeof(float), &dcost))) return rc;
    const float *dP = nullptr;
    int qpS = 0;
    void *dqu = nullptr;
    if (qp) {
        if ((rc = qp_matrix(ctx, H, qp->rho, s, &dP, &qpS))) return rc;
        if ((rc = ensure(ctx, S_QPU, (size_t)K * H * NU * sizeof(float), &dqu))) return rc;
    }
    const int n = H * NU;
    void *dS = nullptr, *dA = nullptr, *dL = nullptr, *dL32 = nullptr, *dLi = nullptr, *dZ = nullptr,
         *dUc = nullptr, *dnu64 = nullptr;
    if (cov) {
        const size_t nn = (size_t)n * n;
        if ((rc = ensure(ctx, S_COVS, nn * sizeof(double), &dS)) || (rc = ensure(ctx, S_COVA, nn * sizeof(double), &dA)) ||
            (rc = ensure(ctx, S_COVL, nn * sizeof(double), &dL)) || (rc = ensure(ctx, S_COVL32, nn * sizeof(float), &dL32)) ||
            (rc = ensure(ctx, S_COVLI, 2 * 32 * 32 * sizeof(double) + 256, &dLi)) ||
            (rc = ensure(ctx, S_COVZ, (size_t)K * n * sizeof(float), &dZ)) ||
            (rc = ensure(ctx, S_COVU, (size_t)K * n * sizeof(float), &dUc)) ||
            (rc = ensure(ctx, S_NU64, (size_t)n * sizeof(double), &dnu64)))
            return rc;
        if (cov->Sigma0)
            HIPCHK(hipMemcpyAsync(dS, cov->Sigma0, nn * sizeof(double),
                                  dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        else
            launch_diag_sigma((const float *)dsig, sps, n, (double *)dS, s);
    }
    int *dflag = cov ? (int *)((char *)dLi + 2 * 32 * 32 * sizeof(double)) : nullptr;
    // the best sequence of the last iteration goes to U_best (same side as U_new)
    void *dbest = nullptr;
    if (U_best && (rc = out_ptr(ctx, S_OUT3, U_best, (size_t)H * NU * sizeof(float), dev, &dbest))) return rc;
    const bool per_step = fl & MPPI_PER_STEP;
    void *dps = nullptr;
    if (per_step && (rc = ensure(ctx, S_PLAIN, (size_t)K * PLAIN_FIELDS * sizeof(float), &dps))) return rc;
    const bool use_graph = (fl & MPPI_GRAPH) && !qp && !cov && !U_best && !per_step;
    const bool timing = (fl & MPPI_TIME_KERNELS) && !use_graph;
    const int M = opts->M;
    if (timing) {
        while ((int)ctx->ev.size() < 2 * M) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            ctx->ev.push_back(e);
        }
    }
    const uint32_t k0 = (uint32_t)(opts->seed & 0xffffffffu), k1 = (uint32_t)(opts->seed >> 32);
    const int n_elite = (opts->n_elite <= 0 || opts->n_elite >= K) ? K : opts->n_elite;
    const int f32 = (fl & MPPI_FP32_WEIGHTS) ? 1 : 0;
    int mapping;
    if ((rc = scene_mapping(ctx, scene, K, fl, &mapping))) return rc;
    if (per_step) mapping = MAP_LANE;
    // the launch sequence of the plan: nu = nominal, stats reset, M x (rollout, stats, update)
    auto enqueue = [&](hipStream_t q) -> int {
        HIPCHK(hipMemcpyAsync(dnu, dnom, (size_t)H * NU * sizeof(float), hipMemcpyDeviceToDevice, q));
        launch_reset_stats(ctx->st, q);
        for (int m = 0; m < M; ++m) {
            RolloutArgs ra = {};
            ra.md = scene->dev;
            ra.x0 = (const float *)dx0;
            ra.x0_shared = 1;
            ra.nu = (const float *)dnu;
            ra.sigma = (const float *)dsig;
            ra.sigma_per_step = sps;
            ra.U = nullptr;
            ra.key0 = k0;
            ra.key1 = k1;
            ra.m = m;
            ra.K = K;
            ra.H = H;
            ra.n_sub = 0;
            ra.costs = (float *)dcost;
            ra.counters = (int *)dcnt;
            ra.diverged = &ctx->st->diverged;
            ra.dist = (float *)ddist;
            const float *Ucur = nullptr;
            if (cov) {
                // factor Sigma_m, then draw clip(nu_m + L_m z_j) for every sample
                CholArgs ca = {(const double *)dS, (double *)dA, (double *)dL, (float *)dL32, (double *)dLi, dflag,
                               n, m == 0 ? 1 : 0};
                launch_cholesky(ca, q);
                SampleFullArgs sf = {(float *)dZ, (const float *)dL32, (const float *)dnu, (float *)dUc, K, n, k0, k1,
                                     m, scene->host.u_max};
                launch_sample_full(sf, q);
                Ucur = (const float *)dUc;
                ra.U = Ucur;
            }
            if (qp) {
                // this iteration's samples, projected, then rolled out as given
                ProjectArgs pa = {};
                qp_args(pa, scene, qp, dP, qpS, K, H);
                pa.U_out = (float *)dqu;
                pa.x0 = (const float *)dx0;
                pa.x0_shared = 1;
                pa.nu = (const float *)dnu;
                pa.sigma = (const float *)dsig;
                pa.sigma_per_step = sps;
                pa.key0 = k0;
                pa.key1 = k1;
                pa.m = m;
                pa.U_in = Ucur;
                launch_project(pa, q);
                Ucur = (const float *)dqu;
                ra.U = Ucur;
            }
            if (timing) HIPCHK(hipEventRecord(ctx->ev[2 * m], q));
            if (per_step) {
                for (int k = 0; k < H; ++k)
                    launch_rollout_step(ra, scene->host.n_cmax, (float *)dps, k, scene->host.task_form != 0, q);
            } else {
                launch_rollout(ra, scene->host.n_cmax, q, mapping);
            }
            if (timing) HIPCHK(hipEventRecord(ctx->ev[2 * m + 1], q));
            StatsArgs sa = {(const float *)dcost, K, 1.0 / lambda, n_elite, (double *)dw, ctx->st, m,
                            (const int *)dcnt, f32};
            launch_stats(sa, q);
            if (dbest && m == M - 1) {
                BestArgs ba = {ctx->st, Ucur, (const float *)dnu, (const float *)dsig, sps, scene->host.u_max, k0, k1,
                               m, H, (float *)dbest};
                launch_best(ba, q);
            }
            UpdateArgs ua = {(const double *)dw, K, H, (const float *)dnu, (const float *)dsig, sps,
                             scene->host.u_max, k0, k1, m, opts->eta, ctx->st, (float *)dnu, (double *)dnu64, f32,
                             Ucur};
            launch_update(ua, q);
            if (cov) {
                // Sigma_{m+1} about nu_{m+1}, in place
                CovArgs cv = {Ucur, (const double *)dw, (const double *)dnu64, (const double *)dS, (double *)dS, K, n,
                              opts->eta, cov->eps};
                launch_cov_update(cv, q);
            }
        }
        HIPCHK(hipGetLastError());
        return MPPI_OK;
    };
    if (!use_graph) {
        if ((rc = enqueue(s))) return rc;
    } else {
        // everything the captured nodes bake in: shapes, scalars and pointers
        double lam_bits = lambda, eta_bits = opts->eta;
        uintptr_t lb, eb;
        std::memcpy(&lb, &lam_bits, sizeof lb);
        std::memcpy(&eb, &eta_bits, sizeof eb);
        // key[0]: the scene's generation (its host scalars, such as u_max, are
        // baked into the update nodes; a later scene may reuse its address)
        const std::vector<uintptr_t> key = {(uintptr_t)scene->gen, (uintptr_t)scene->dev, (uintptr_t)K, (uintptr_t)H, (uintptr_t)M, lb, eb,
                                            (uintptr_t)opts->seed, (uintptr_t)n_elite, (uintptr_t)sps,
                                            (uintptr_t)mapping, (uintptr_t)f32, (uintptr_t)scene->host.n_cmax,
                                            (uintptr_t)dx0, (uintptr_t)dsig, (uintptr_t)dnom, (uintptr_t)dnu,
                                            (uintptr_t)dcost, (uintptr_t)dw, (uintptr_t)dcnt, (uintptr_t)ddist,
                                            (uintptr_t)ctx->st};
        PlanGraph *pg = nullptr;
        for (auto &g : ctx->graphs)
            if (g.key == key) pg = &g;
        if (!pg) {
            if (!ctx->capture) HIPCHK(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
            // the capture stream must not run ahead of work already queued on s
            HIPCHK(hipStreamSynchronize(s));
            PlanGraph g;
            g.key = key;
            HIPCHK(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
            const int rc2 = enqueue(ctx->capture);
            hipGraph_t graph = nullptr;
            const hipError_t e2 = hipStreamEndCapture(ctx->capture, &graph);
            if (rc2) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc2;
            }
            if (e2 != hipSuccess) return fail(MPPI_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e2));
            g.graph = graph;
            if (hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return fail(MPPI_E_DEVICE, "graph instantiation failed");
            }
            if (ctx->graphs.size() >= 8) {
                // evict the least recently used graph
                size_t lru = 0;
                for (size_t i = 1; i < ctx->graphs.size(); ++i)
                    if (ctx->graphs[i].last_use < ctx->graphs[lru].last_use) lru = i;
                (void)hipGraphExecDestroy(ctx->graphs[lru].exec);
                (void)hipGraphDestroy(ctx->graphs[lru].graph);
                ctx->graphs.erase(ctx->graphs.begin() + lru);
            }
            ctx->graphs.push_back(g);
            pg = &ctx->graphs.back();
        }
        pg->last_use = ++ctx->graph_clock;
        HIPCHK(hipGraphLaunch(pg->exec, s));
    }
    HIPCHK(hipGetLastError());
    // outputs
    if (dev) {
        HIPCHK(hipMemcpyAsync(U_new, dnu, (size_t)H * NU * sizeof(float), hipMemcpyDeviceToDevice, s));
    } else {
        HIPCHK(hipMemcpyAsync(U_new, dnu, (size_t)H * NU * sizeof(float), hipMemcpyDeviceToHost, s));
        if (costs) HIPCHK(hipMemcpyAsync(costs, dcost, (size_t)K * sizeof(float), hipMemcpyDeviceToHost, s));
    }
    if (dbest && (rc = copy_out(U_best, dbest, (size_t)H * NU * sizeof(float), dev, s))) return rc;
    int flag_h = n;
    if (cov) {
        if (cov->Sigma_out)
            HIPCHK(hipMemcpyAsync(cov->Sigma_out, dS, (size_t)n * n * sizeof(double),
                                  dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&flag_h, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    }
    const bool sync = !dev || stats || (fl & MPPI_SYNC) || cov;
    if (!sync) return MPPI_OK;
    PlanStats hs;
    HIPCHK(hipMemcpyAsync(&hs, ctx->st, sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flag_h < n) return fail(MPPI_E_NOTPD, "covariance not positive definite at column %d", flag_h);
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->ess = hs.ess;
        stats->c_min = hs.cmin;
        stats->best = hs.best;
        stats->n_nonfinite = K - hs.n_finite;
        stats->diverged = hs.diverged;
        stats->iterations = M;
        for (int i = 0; i < 64 && i < M; ++i) stats->cmin_iter[i] = hs.cmin_iter[i];
        stats->contacts = (double)hs.counters[0];
        stats->np_tests = (double)hs.counters[1];
        stats->box_tests = (double)hs.counters[2];
        stats->overflow = (double)hs.counters[3];
        stats->rollout_launches = M;
        if (timing) {
            float tot = 0.f;
            for (int m = 0; m < M; ++m) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, ctx->ev[2 * m], ctx->ev[2 * m + 1]));
                tot += ms;
            }
            stats->rollout_ms = tot;
        }
    }
    if (hs.diverged) {
        // every sample of some iteration was non-finite: hand back the nominal sequence
        if (dev)
            HIPCHK(hipMemcpyAsync(U_new, dnom, (size_t)H * NU * sizeof(float), hipMemcpyDeviceToDevice, s));
        else
            std::memcpy(U_new, nominal_U, (size_t)H * NU * sizeof(float));
        HIPCHK(hipStreamSynchronize(s));
        return fail(MPPI_E_DIVERGED, "every sample diverged in some iteration");
    }
    return MPPI_OK;
}

int mppi_plan(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
              double lambda, const float *sigma, const mppi_opts *opts, float *U_new, float *costs, mppi_stats *stats,
              void *stream)
{
    return plan_impl(ctx, scene, x0, nominal_U, K, H, lambda, sigma, opts, nullptr, nullptr, U_new, costs, stats,
                     stream, nullptr);
}

int mppi_plan_noalloc(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                      double lambda, const float *sigma, const mppi_opts *opts, float *U_new, float *costs,
                      mppi_stats *stats, void *stream)
{
    if (!ctx || !scene || !x0 || !nominal_U || !sigma || !opts || !U_new) return fail(MPPI_E_INVAL, "NULL argument");
    if (scene->ctx != ctx) return fail(MPPI_E_INVAL, "scene belongs to another context");
    if (K < 1 || K > MPPI_MAX_K || H < 1 || H > MPPI_MAX_H) return fail(MPPI_E_INVAL, "K=%d or H=%d out of range", K, H);
    if (!(lambda > 0) || !std::isfinite(lambda)) return fail(MPPI_E_INVAL, "lambda must be finite and > 0");
    if (opts->M < 1 || opts->M > 100000) return fail(MPPI_E_INVAL, "M=%d out of range", opts->M);
    if (!std::isfinite(opts->eta)) return fail(MPPI_E_INVAL, "eta must be finite");
    const unsigned fl = opts->flags;
    if (!(fl & MPPI_DEVICE_PTRS)) return fail(MPPI_E_INVAL, "mppi_plan_noalloc takes device pointers (MPPI_DEVICE_PTRS)");
    if (fl & (MPPI_GRAPH | MPPI_TIME_KERNELS)) return fail(MPPI_E_INVAL, "MPPI_GRAPH and MPPI_TIME_KERNELS are not supported here");
    const NoallocLayout L = noalloc_layout(K, H, scene->host.n_cost);
    if (L.total > (size_t)MPPI_NOALLOC_SCRATCH_BYTES)
        return fail(MPPI_E_INVAL, "K=%d, H=%d with %d cost pairs need %zu bytes of scratch, above MPPI_NOALLOC_SCRATCH_BYTES (%zu)",
                    K, H, scene->host.n_cost, L.total, (size_t)MPPI_NOALLOC_SCRATCH_BYTES);
    int rc = set_device(ctx);
    if (rc) return rc;
    char *base = (char *)g_scratch_dev[ctx->device];
    if (!base) return fail(MPPI_E_DEVICE, "scratch of device %d not set up", ctx->device);
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    PlanStats *st = (PlanStats *)(base + L.st);
    float *dnu = (float *)(base + L.nu);
    double *dw = (double *)(base + L.w);
    int *dcnt = (int *)(base + L.cnt);
    float *ddist = (float *)(base + L.dist);
    float *dcost = costs ? costs : (float *)(base + L.costs);
    const bool sps = fl & MPPI_SIGMA_PER_STEP;
    const uint32_t k0 = (uint32_t)(opts->seed & 0xffffffffu), k1 = (uint32_t)(opts->seed >> 32);
    const int n_elite = (opts->n_elite <= 0 || opts->n_elite >= K) ? K : opts->n_elite;
    const int f32 = (fl & MPPI_FP32_WEIGHTS) ? 1 : 0;
    int mapping;
    if ((rc = scene_mapping(ctx, scene, K, fl, &mapping))) return rc;
    // nu = nominal; the statistics record cleared by a kernel (no memset, so
    // the sequence may be captured into a graph); then M x (rollout, stats, update)
    HIPCHK(hipMemcpyAsync(dnu, nominal_U, (size_t)H * NU * sizeof(float), hipMemcpyDeviceToDevice, s));
    launch_reset_stats(st, s);
    for (int m = 0; m < opts->M; ++m) {
        RolloutArgs ra = {};
        ra.md = scene->dev;
        ra.x0 = x0;
        ra.x0_shared = 1;
        ra.nu = dnu;
        ra.sigma = sigma;
        ra.sigma_per_step = sps;
        ra.key0 = k0;
        ra.key1 = k1;
        ra.m = m;
        ra.K = K;
        ra.H = H;
        ra.costs = dcost;
        ra.counters = dcnt;
        ra.diverged = &st->diverged;
        ra.dist = ddist;
        launch_rollout(ra, scene->host.n_cmax, s, mapping);
        StatsArgs sa = {dcost, K, 1.0 / lambda, n_elite, dw, st, m, dcnt, f32};
        launch_stats(sa, s);
        UpdateArgs ua = {dw, K, H, dnu, sigma, sps, scene->host.u_max, k0, k1, m, opts->eta, st, dnu, nullptr, f32,
                         nullptr};
        launch_update(ua, s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(U_new, dnu, (size_t)H * NU * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (!stats && !(fl & MPPI_SYNC)) return MPPI_OK;
    PlanStats hs;
    HIPCHK(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->ess = hs.ess;
        stats->c_min = hs.cmin;
        stats->best = hs.best;
        stats->n_nonfinite = K - hs.n_finite;
        stats->diverged = hs.diverged;
        stats->iterations = opts->M;
        for (int i = 0; i < 64 && i < opts->M; ++i) stats->cmin_iter[i] = hs.cmin_iter[i];
        stats->contacts = (double)hs.counters[0];
        stats->np_tests = (double)hs.counters[1];
        stats->box_tests = (double)hs.counters[2];
        stats->overflow = (double)hs.counters[3];
        stats->rollout_launches = opts->M;
    }
    if (hs.diverged) {
        HIPCHK(hipMemcpyAsync(U_new, nominal_U, (size_t)H * NU * sizeof(float), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        return fail(MPPI_E_DIVERGED, "every sample diverged in some iteration");
    }
    return MPPI_OK;
}

int mppi_plan_best(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                   double lambda, const float *sigma, const mppi_opts *opts, float *U_new, float *U_best, float *costs,
                   mppi_stats *stats, void *stream)
{
    if (!U_best) return fail(MPPI_E_INVAL, "NULL argument");
    return plan_impl(ctx, scene, x0, nominal_U, K, H, lambda, sigma, opts, nullptr, nullptr, U_new, costs, stats,
                     stream, U_best);
}

int mppi_plan_qp(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                 double lambda, const float *sigma, const mppi_opts *opts, const mppi_qp *qp, float *U_new,
                 float *costs, mppi_stats *stats, void *stream)
{
    int rc;
    if ((rc = qp_check(qp, H))) return rc;
    return plan_impl(ctx, scene, x0, nominal_U, K, H, lambda, sigma, opts, qp, nullptr, U_new, costs, stats, stream,
                     nullptr);
}

static int cov_check_n(int n)
{
    if (n < 1 || n > MPPI_COV_MAX_N) return fail(MPPI_E_INVAL, "n=%d out of range (1..%d)", n, MPPI_COV_MAX_N);
    return MPPI_OK;
}

int mppi_plan_cov(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                  double lambda, const float *sigma, const mppi_opts *opts, const mppi_cov *cov, const mppi_qp *qp,
                  float *U_new, float *costs, mppi_stats *stats, void *stream)
{
    int rc;
    if (!cov || !opts) return fail(MPPI_E_INVAL, "NULL argument");
    if (H < 1 || (rc = cov_check_n(H * NU))) return H < 1 ? fail(MPPI_E_INVAL, "H=%d out of range", H) : rc;
    if (!(cov->eps >= 0) || !std::isfinite(cov->eps)) return fail(MPPI_E_INVAL, "eps must be finite and >= 0");
    if (!(opts->eta > 0 && opts->eta <= 1)) return fail(MPPI_E_INVAL, "eta must be in (0, 1] with the covariance update");
    if (qp && (rc = qp_check(qp, H))) return rc;
    if (cov->Sigma0 && !(opts->flags & MPPI_DEVICE_PTRS)) {
        const size_t nn = (size_t)H * NU * H * NU;
        for (size_t i = 0; i < nn; ++i)
            if (!std::isfinite(cov->Sigma0[i])) return fail(MPPI_E_INVAL, "non-finite Sigma0");
    }
    return plan_impl(ctx, scene, x0, nominal_U, K, H, lambda, sigma, opts, qp, cov, U_new, costs, stats, stream,
                     cov->U_best);
}

int mppi_cov_update(mppi_ctx *ctx, const float *U, const double *w, const double *nu_new, const double *Sigma_in,
                    double eta, double eps, double *Sigma_out, int K, int n, unsigned flags, void *stream)
{
    if (!ctx || !U || !w || !nu_new || !Sigma_in || !Sigma_out) return fail(MPPI_E_INVAL, "NULL argument");
    int rc;
    if ((rc = cov_check_n(n))) return rc;
    if (K < 1 || K > MPPI_MAX_K) return fail(MPPI_E_INVAL, "K=%d out of range", K);
    if (!(eta >= 0 && eta <= 1)) return fail(MPPI_E_INVAL, "eta must be in [0, 1]");
    if (!(eps >= 0) || !std::isfinite(eps)) return fail(MPPI_E_INVAL, "eps must be finite and >= 0");
    const bool dev = flags & MPPI_DEVICE_PTRS;
    const size_t nn = (size_t)n * n;
    if (!dev) {
        for (int j = 0; j < K; ++j)
            if (!(w[j] >= 0) || !std::isfinite(w[j])) return fail(MPPI_E_INVAL, "weights must be finite and >= 0");
        if (!all_finite(U, (size_t)K * n)) return fail(MPPI_E_INVAL, "non-finite samples");
    }
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const void *dU, *dw, *dnu, *dSin;
    if ((rc = stage_in(ctx, S_IN0, U, (size_t)K * n * sizeof(float), dev, s, &dU)) ||
        (rc = stage_in(ctx, S_IN1, w, (size_t)K * sizeof(double), dev, s, &dw)) ||
        (rc = stage_in(ctx, S_NU64, nu_new, (size_t)n * sizeof(double), dev, s, &dnu)) ||
        (rc = stage_in(ctx, S_COVA, Sigma_in, nn * sizeof(double), dev, s, &dSin)))
        return rc;
    void *dout;
    if ((rc = out_ptr(ctx, S_COVS, Sigma_out, nn * sizeof(double), dev, &dout))) return rc;
    CovArgs cv = {(const float *)dU, (const double *)dw, (const double *)dnu, (const double *)dSin, (double *)dout, K,
                  n, eta, eps};
    launch_cov_update(cv, s);
    HIPCHK(hipGetLastError());
    if ((rc = copy_out(Sigma_out, dout, nn * sizeof(double), dev, s))) return rc;
    if (!dev || (flags & MPPI_SYNC)) HIPCHK(hipStreamSynchronize(s));
    return MPPI_OK;
}

int mppi_cholesky(mppi_ctx *ctx, const double *Sigma, double *L, int n, unsigned flags, void *stream)
{
    if (!ctx || !Sigma || !L) return fail(MPPI_E_INVAL, "NULL argument");
    int rc;
    if ((rc = cov_check_n(n))) return rc;
    const bool dev = flags & MPPI_DEVICE_PTRS;
    const size_t nn = (size_t)n * n;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const void *dS;
    if ((rc = stage_in(ctx, S_COVS, Sigma, nn * sizeof(double), dev, s, &dS))) return rc;
    void *dA, *dLi, *dL;
    if ((rc = ensure(ctx, S_COVA, nn * sizeof(double), &dA)) ||
        (rc = ensure(ctx, S_COVLI, 2 * 32 * 32 * sizeof(double) + 256, &dLi)))
        return rc;
    if ((rc = out_ptr(ctx, S_COVL, L, nn * sizeof(double), dev, &dL))) return rc;
    int *dflag = (int *)((char *)dLi + 2 * 32 * 32 * sizeof(double));
    CholArgs ca = {(const double *)dS, (double *)dA, (double *)dL, nullptr, (double *)dLi, dflag, n, 1};
    launch_cholesky(ca, s);
    HIPCHK(hipGetLastError());
    if ((rc = copy_out(L, dL, nn * sizeof(double), dev, s))) return rc;
    int flag_h = n;
    HIPCHK(hipMemcpyAsync(&flag_h, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flag_h < n) return fail(MPPI_E_NOTPD, "matrix not positive definite at column %d", flag_h);
    return MPPI_OK;
}

int mppi_sample_full(mppi_ctx *ctx, const float *nu, const double *L, uint64_t seed, int m, int K, int H,
                     float u_max, float *U, unsigned flags, void *stream)
{
    if (!ctx || !nu || !L || !U) return fail(MPPI_E_INVAL, "NULL argument");
    int rc;
    if (H < 1) return fail(MPPI_E_INVAL, "H=%d out of range", H);
    const int n = H * NU;
    if ((rc = cov_check_n(n))) return rc;
    if (K < 1 || K > MPPI_MAX_K) return fail(MPPI_E_INVAL, "K=%d out of range", K);
    if (!(u_max > 0) || !std::isfinite(u_max)) return fail(MPPI_E_INVAL, "u_max must be finite and > 0");
    const bool dev = flags & MPPI_DEVICE_PTRS;
    const size_t nn = (size_t)n * n;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const void *dnu, *dL;
    if ((rc = stage_in(ctx, S_IN0, nu, (size_t)n * sizeof(float), dev, s, &dnu)) ||
        (rc = stage_in(ctx, S_COVL, L, nn * sizeof(double), dev, s, &dL)))
        return rc;
    void *dL32, *dZ, *dout;
    if ((rc = ensure(ctx, S_COVL32, nn * sizeof(float), &dL32)) ||
        (rc = ensure(ctx, S_COVZ, (size_t)K * n * sizeof(float), &dZ)))
        return rc;
    if ((rc = out_ptr(ctx, S_COVU, U, (size_t)K * n * sizeof(float), dev, &dout))) return rc;
    // the upper triangle of L is not read: it becomes zero in the single-precision copy
    launch_to_f32((const double *)dL, (float *)dL32, (long)nn, s);
    launch_lower_f32((float *)dL32, n, s);
    SampleFullArgs sf = {(float *)dZ, (const float *)dL32, (const float *)dnu, (float *)dout, K, n,
                         (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), m, u_max};
    launch_sample_full(sf, s);
    HIPCHK(hipGetLastError());
    if ((rc = copy_out(U, dout, (size_t)K * n * sizeof(float), dev, s))) return rc;
    if (!dev || (flags & MPPI_SYNC)) HIPCHK(hipStreamSynchronize(s));
    return MPPI_OK;
}

int mppi_project(mppi_ctx *ctx, const mppi_scene *scene, const float *X0, int x0_shared, const float *U_in,
                 float *U_out, int K, int H, const mppi_qp *qp, unsigned flags, void *stream)
{
    if (!ctx || !scene || !X0 || !U_in || !U_out) return fail(MPPI_E_INVAL, "NULL argument");
    if (scene->ctx != ctx) return fail(MPPI_E_INVAL, "scene belongs to another context");
    if (K < 1 || K > MPPI_MAX_K || H < 1) return fail(MPPI_E_INVAL, "K=%d or H=%d out of range", K, H);
    int rc;
    if ((rc = qp_check(qp, H))) return rc;
    const bool dev = flags & MPPI_DEVICE_PTRS;
    const size_t nx0 = x0_shared ? NX : (size_t)K * NX, nu_n = (size_t)K * H * NU;
    if (!dev && (!all_finite(X0, nx0) || !all_finite(U_in, nu_n))) return fail(MPPI_E_INVAL, "non-finite input");
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const float *dP;
    int S;
    if ((rc = qp_matrix(ctx, H, qp->rho, s, &dP, &S))) return rc;
    const void *dx0, *dU;
    if ((rc = stage_in(ctx, S_IN0, X0, nx0 * sizeof(float), dev, s, &dx0))) return rc;
    if ((rc = stage_in(ctx, S_IN1, U_in, nu_n * sizeof(float), dev, s, &dU))) return rc;
    void *dout;
    if ((rc = out_ptr(ctx, S_OUT0, U_out, nu_n * sizeof(float), dev, &dout))) return rc;
    ProjectArgs pa = {};
    qp_args(pa, scene, qp, dP, S, K, H);
    pa.U_in = (const float *)dU;
    pa.U_out = (float *)dout;
    pa.x0 = (const float *)dx0;
    pa.x0_shared = x0_shared ? 1 : 0;
    launch_project(pa, s);
    HIPCHK(hipGetLastError());
    if ((rc = copy_out(U_out, dout, nu_n * sizeof(float), dev, s))) return rc;
    if (!dev || (flags & MPPI_SYNC)) HIPCHK(hipStreamSynchronize(s));
    return MPPI_OK;
}

int mppi_plan_batch(mppi_ctx *ctx, int n, mppi_request *reqs, unsigned flags, void *stream)
{
    if (!ctx || !reqs || n < 1) return fail(MPPI_E_INVAL, "NULL context/requests or n < 1");
    const bool dev = flags & MPPI_DEVICE_PTRS, timing = flags & MPPI_TIME_KERNELS;
    long total_k = 0;
    int maxM = 0;
    for (int i = 0; i < n; ++i) {
        mppi_request &r = reqs[i];
        if (!r.scene || !r.x0 || !r.nominal_U || !r.sigma || !r.U_new) return fail(MPPI_E_INVAL, "request %d: NULL argument", i);
        if (r.scene->ctx != ctx) return fail(MPPI_E_INVAL, "request %d: scene of another context", i);
        int map_i;
        if (scene_mapping(ctx, r.scene, r.K, flags, &map_i)) return fail(MPPI_E_INVAL, "request %d: %s", i, mppi_last_error());
        if (r.K < 1 || r.K > MPPI_MAX_K || r.H < 1 || r.H > MPPI_MAX_H) return fail(MPPI_E_INVAL, "request %d: K or H out of range", i);
        if (!(r.lambda > 0) || !std::isfinite(r.lambda) || r.opts.M < 1 || r.opts.M > 100000 || !std::isfinite(r.opts.eta))
            return fail(MPPI_E_INVAL, "request %d: bad lambda, M or eta", i);
        const size_t nsig = (r.opts.flags & MPPI_SIGMA_PER_STEP) ? (size_t)r.H * NU : NU;
        if (!dev) {
            if (!all_finite(r.x0, NX) || !all_finite(r.nominal_U, (size_t)r.H * NU) || !all_finite(r.sigma, nsig))
                return fail(MPPI_E_INVAL, "request %d: non-finite input", i);
            for (size_t q = 0; q < nsig; ++q)
                if (r.sigma[q] < 0) return fail(MPPI_E_INVAL, "request %d: sigma < 0", i);
        }
        r.status = MPPI_OK;
        total_k += r.K;
        maxM = std::max(maxM, r.opts.M);
    }
    if (total_k > MPPI_MAX_K) return fail(MPPI_E_INVAL, "batch has more than %d samples", MPPI_MAX_K);
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    // requests in order of decreasing M: the ones still iterating form a prefix
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return reqs[a].opts.M > reqs[b].opts.M; });
    // One rollout launch per group of requests that share the family of the
    // mapping they would run alone and the contact-list instantiation (n_cmax
    // up to 4, or up to 8): each request's results then equal its plan alone
    // bit for bit, whatever it is batched with.
    std::vector<int> grp(n);
    long grp_k[NGROUP] = {};
    for (int i = 0; i < n; ++i) {
        const mppi_request &r = reqs[ord[i]];
        grp[i] = group_index(request_family(ctx, r.scene, r.K, flags), r.scene->host.n_cmax);
        grp_k[grp[i]] += r.K;
    }
    int gmap[NGROUP];
    for (int g = 0; g < NGROUP; ++g) gmap[g] = family_launch_mapping(ctx, group_family(g), grp_k[g], flags);
    // offsets of every request's slices in the packed buffers
    std::vector<size_t> o_k(n), o_h(n), o_sig(n), o_x0(n);
    size_t nk = 0, nh = 0, nsig_tot = 0;
    for (int i = 0; i < n; ++i) {
        const mppi_request &r = reqs[ord[i]];
        o_k[i] = nk;
        nk += (size_t)r.K;
        o_h[i] = nh;
        nh += (size_t)r.H * NU;
        o_sig[i] = nsig_tot;
        nsig_tot += (r.opts.flags & MPPI_SIGMA_PER_STEP) ? (size_t)r.H * NU : NU;
        o_x0[i] = (size_t)i * NX;
    }
    // block tables: the rollout blocks of each group (in request order, so the
    // requests still iterating give a prefix of every group's table), then
    // the update blocks
    std::vector<int> gblk[NGROUP], ublk, ublk_prefix(n + 1, 0);
    std::vector<std::vector<int>> blk_prefix(NGROUP, std::vector<int>(n + 1, 0));
    for (int i = 0; i < n; ++i) {
        const mppi_request &r = reqs[ord[i]];
        const int g = grp[i], per = samples_per_block(gmap[g]);
        const int nb = (r.K + per - 1) / per;
        for (int b = 0; b < nb; ++b) { gblk[g].push_back(i); gblk[g].push_back(b); }
        for (int k = 0; k < r.H; ++k) { ublk.push_back(i); ublk.push_back(k); }
        for (int q = 0; q < NGROUP; ++q) blk_prefix[q][i + 1] = (int)gblk[q].size() / 2;
        ublk_prefix[i + 1] = (int)ublk.size() / 2;
    }
    std::vector<int> blk;
    size_t goff[NGROUP];
    for (int g = 0; g < NGROUP; ++g) {
        goff[g] = blk.size();
        blk.insert(blk.end(), gblk[g].begin(), gblk[g].end());
    }
    // device buffers
    void *d_nu, *d_cost, *d_w, *d_cnt, *d_dist, *d_st, *d_in;
    if ((rc = ensure(ctx, S_BNU, nh * sizeof(float), &d_nu))) return rc;
    if ((rc = ensure(ctx, S_BCOST, nk * sizeof(float), &d_cost))) return rc;
    if ((rc = ensure(ctx, S_BW, nk * sizeof(double), &d_w))) return rc;
    if ((rc = ensure(ctx, S_BCNT, nk * 4 * sizeof(int), &d_cnt))) return rc;
    if ((rc = ensure(ctx, S_BDIST, nk * MAXCOST * sizeof(float), &d_dist))) return rc;
    if ((rc = ensure(ctx, S_BST, (size_t)n * sizeof(PlanStats), &d_st))) return rc;
    const size_t in_floats = (size_t)n * NX + nh + nsig_tot;
    if ((rc = ensure(ctx, S_BIN, in_floats * sizeof(float), &d_in))) return rc;
    float *d_x0 = (float *)d_in, *d_nom = d_x0 + (size_t)n * NX, *d_sig = d_nom + nh;
    // stage inputs into the packed buffers
    for (int i = 0; i < n; ++i) {
        const mppi_request &r = reqs[ord[i]];
        const size_t ns = (r.opts.flags & MPPI_SIGMA_PER_STEP) ? (size_t)r.H * NU : NU;
        const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        HIPCHK(hipMemcpyAsync(d_x0 + o_x0[i], r.x0, NX * sizeof(float), kind, s));
        HIPCHK(hipMemcpyAsync(d_nom + o_h[i], r.nominal_U, (size_t)r.H * NU * sizeof(float), kind, s));
        HIPCHK(hipMemcpyAsync(d_sig + o_sig[i], r.sigma, ns * sizeof(float), kind, s));
    }
    HIPCHK(hipMemcpyAsync(d_nu, d_nom, nh * sizeof(float), hipMemcpyDeviceToDevice, s));
    // argument tables (pinned staging, then one upload)
    const size_t tab_bytes = (size_t)n * (sizeof(RolloutArgs) + sizeof(StatsArgs) + sizeof(UpdateArgs)) +
                             (blk.size() + ublk.size()) * sizeof(int) + 256;
    void *d_tab;
    if ((rc = ensure(ctx, S_BTAB, tab_bytes, &d_tab))) return rc;
    HIPCHK(hipStreamSynchronize(s));  // the pinned staging area may still feed a previous upload
    if (ctx->host_tab_cap < tab_bytes) {
        if (ctx->host_tab) (void)hipHostFree(ctx->host_tab);
        ctx->host_tab = nullptr;
        ctx->host_tab_cap = 0;
        if (hipHostMalloc(&ctx->host_tab, tab_bytes * 2) != hipSuccess) return fail(MPPI_E_NOMEM, "pinned table allocation failed");
        ctx->host_tab_cap = tab_bytes * 2;
    }
    char *hbase = (char *)ctx->host_tab;
    RolloutArgs *hr = (RolloutArgs *)hbase;
    StatsArgs *hs = (StatsArgs *)(hr + n);
    UpdateArgs *hu = (UpdateArgs *)(hs + n);
    int *hblk = (int *)(hu + n);
    int *hublk = hblk + blk.size();
    PlanStats *st = (PlanStats *)d_st;
    for (int i = 0; i < n; ++i) {
        const mppi_request &r = reqs[ord[i]];
        const uint32_t k0 = (uint32_t)(r.opts.seed & 0xffffffffu), k1 = (uint32_t)(r.opts.seed >> 32);
        RolloutArgs ra = {};
        ra.md = r.scene->dev;
        ra.x0 = d_x0 + o_x0[i];
        ra.x0_shared = 1;
        ra.nu = (const float *)d_nu + o_h[i];
        ra.sigma = d_sig + o_sig[i];
        ra.sigma_per_step = (r.opts.flags & MPPI_SIGMA_PER_STEP) ? 1 : 0;
        ra.key0 = k0;
        ra.key1 = k1;
        ra.K = r.K;
        ra.H = r.H;
        ra.costs = (float *)d_cost + o_k[i];
        ra.counters = (int *)d_cnt + 4 * o_k[i];
        ra.diverged = &st[i].diverged;
        ra.dist = (float *)d_dist + MAXCOST * o_k[i];
        hr[i] = ra;
        const int ne = (r.opts.n_elite <= 0 || r.opts.n_elite >= r.K) ? r.K : r.opts.n_elite;
        hs[i] = StatsArgs{(const float *)d_cost + o_k[i], r.K, 1.0 / r.lambda, ne, (double *)d_w + o_k[i], &st[i], 0,
                          (const int *)d_cnt + 4 * o_k[i]};
        hu[i] = UpdateArgs{(const double *)d_w + o_k[i], r.K, r.H, (const float *)d_nu + o_h[i], d_sig + o_sig[i],
                           ra.sigma_per_step, r.scene->host.u_max, k0, k1, 0, r.opts.eta, &st[i],
                           (float *)d_nu + o_h[i], nullptr};
    }
    std::memcpy(hblk, blk.data(), blk.size() * sizeof(int));
    std::memcpy(hublk, ublk.data(), ublk.size() * sizeof(int));
    HIPCHK(hipMemcpyAsync(d_tab, hbase, tab_bytes - 256, hipMemcpyHostToDevice, s));
    const RolloutArgs *d_rt = (const RolloutArgs *)d_tab;
    const StatsArgs *d_sst = (const StatsArgs *)(d_rt + n);
    const UpdateArgs *d_ut = (const UpdateArgs *)(d_sst + n);
    const int *d_blk = (const int *)(d_ut + n);
    const int *d_ublk = d_blk + blk.size();
    launch_reset_stats(st, s, n);
    if (timing) {
        while ((int)ctx->ev.size() < 2 * maxM) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            ctx->ev.push_back(e);
        }
    }
    for (int m = 0; m < maxM; ++m) {
        int act = 0;
        while (act < n && reqs[ord[act]].opts.M > m) ++act;
        // stats entries carry the iteration index for the per-iteration minima
        if (timing) HIPCHK(hipEventRecord(ctx->ev[2 * m], s));
        for (int g = 0; g < NGROUP; ++g)
            if (blk_prefix[g][act] > 0)
                launch_rollout_batch(d_rt, d_blk + goff[g], blk_prefix[g][act], (g & 1) ? 8 : 4, m, gmap[g], s);
        if (timing) HIPCHK(hipEventRecord(ctx->ev[2 * m + 1], s));
        launch_stats_batch(d_sst, act, m, s);
        launch_update_batch(d_ut, d_ublk, ublk_prefix[act], m, s);
    }
    HIPCHK(hipGetLastError());
    // outputs
    std::vector<PlanStats> hst(n);
    HIPCHK(hipMemcpyAsync(hst.data(), st, (size_t)n * sizeof(PlanStats), hipMemcpyDeviceToHost, s));
    for (int i = 0; i < n; ++i) {
        mppi_request &r = reqs[ord[i]];
        const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        HIPCHK(hipMemcpyAsync(r.U_new, (const float *)d_nu + o_h[i], (size_t)r.H * NU * sizeof(float), kind, s));
        if (r.costs) HIPCHK(hipMemcpyAsync(r.costs, (const float *)d_cost + o_k[i], (size_t)r.K * sizeof(float), kind, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    float roll_ms = 0.f;
    if (timing) {
        for (int m = 0; m < maxM; ++m) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ctx->ev[2 * m], ctx->ev[2 * m + 1]));
            roll_ms += ms;
        }
    }
    for (int i = 0; i < n; ++i) {
        mppi_request &r = reqs[ord[i]];
        const PlanStats &p = hst[i];
        if (r.stats) {
            std::memset(r.stats, 0, sizeof *r.stats);
            r.stats->ess = p.ess;
            r.stats->c_min = p.cmin;
            r.stats->best = p.best;
            r.stats->n_nonfinite = r.K - p.n_finite;
            r.stats->diverged = p.diverged;
            r.stats->iterations = r.opts.M;
            for (int q = 0; q < 64 && q < r.opts.M; ++q) r.stats->cmin_iter[q] = p.cmin_iter[q];
            r.stats->contacts = (double)p.counters[0];
            r.stats->np_tests = (double)p.counters[1];
            r.stats->box_tests = (double)p.counters[2];
            r.stats->overflow = (double)p.counters[3];
            r.stats->rollout_ms = roll_ms;
            r.stats->rollout_launches = maxM;
        }
        if (p.diverged) {
            r.status = MPPI_E_DIVERGED;
            if (dev)
                HIPCHK(hipMemcpy(r.U_new, r.nominal_U, (size_t)r.H * NU * sizeof(float), hipMemcpyDeviceToDevice));
            else
                std::memcpy(r.U_new, r.nominal_U, (size_t)r.H * NU * sizeof(float));
        }
    }
    return MPPI_OK;
}

int mppi_simulate(mppi_ctx *ctx, const mppi_scene *scene, const float *X0, int x0_shared, const float *U, int n,
                  int H, int n_sub, float *costs, float *terms, float *X_out, unsigned flags, void *stream)
{
    if (!ctx || !scene || !X0 || !U) return fail(MPPI_E_INVAL, "NULL argument");
    if (n < 1 || n > MPPI_MAX_K || H < 1 || H > MPPI_MAX_H) return fail(MPPI_E_INVAL, "n=%d or H=%d out of range", n, H);
    const bool dev = flags & MPPI_DEVICE_PTRS, traj = flags & MPPI_TRAJ;
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const size_t nx0 = x0_shared ? NX : (size_t)n * NX;
    if (!dev && (!all_finite(X0, nx0) || !all_finite(U, (size_t)n * H * NU))) return fail(MPPI_E_INVAL, "non-finite input");
    const void *dx0, *dU;
    if ((rc = stage_in(ctx, S_IN0, X0, nx0 * sizeof(float), dev, s, &dx0))) return rc;
    if ((rc = stage_in(ctx, S_IN1, U, (size_t)n * H * NU * sizeof(float), dev, s, &dU))) return rc;
    void *dc, *dt, *dxo;
    const size_t nxo = traj ? (size_t)n * H * NX : (size_t)n * NX;
    if ((rc = out_ptr(ctx, S_OUT0, costs, (size_t)n * sizeof(float), dev, &dc))) return rc;
    if (!dc && (rc = ensure(ctx, S_OUT0, (size_t)n * sizeof(float), &dc))) return rc;
    if ((rc = out_ptr(ctx, S_OUT1, terms, (size_t)n * NTERMS * sizeof(float), dev, &dt))) return rc;
    if ((rc = out_ptr(ctx, S_OUT2, X_out, nxo * sizeof(float), dev, &dxo))) return rc;
    void *ddist;
    if ((rc = ensure(ctx, S_DIST, (size_t)n * MAXCOST * sizeof(float), &ddist))) return rc;
    RolloutArgs ra = {};
    ra.md = scene->dev;
    ra.dist = (float *)ddist;
    ra.x0 = (const float *)dx0;
    ra.x0_shared = x0_shared ? 1 : 0;
    ra.U = (const float *)dU;
    ra.K = n;
    ra.H = H;
    ra.n_sub = n_sub;
    ra.costs = (float *)dc;
    ra.terms = (float *)dt;
    ra.xout = (float *)dxo;
    ra.traj = traj;
    int map;
    if ((rc = scene_mapping(ctx, scene, n, flags, &map))) return rc;
    launch_rollout(ra, scene->host.n_cmax, s, map);
    HIPCHK(hipGetLastError());
    if ((rc = copy_out(costs, dc, (size_t)n * sizeof(float), dev, s))) return rc;
    if ((rc = copy_out(terms, dt, (size_t)n * NTERMS * sizeof(float), dev, s))) return rc;
    if ((rc = copy_out(X_out, dxo, nxo * sizeof(float), dev, s))) return rc;
    if (!dev || (flags & MPPI_SYNC)) HIPCHK(hipStreamSynchronize(s));
    return MPPI_OK;
}

int mppi_sample(mppi_ctx *ctx, const mppi_scene *scene, const float *nu, const float *sigma, uint64_t seed, int m,
                int K, int H, float *U, float *z_out, uint32_t *words_out, unsigned flags, void *stream)
{
    if (!ctx || !scene || !nu || !sigma) return fail(MPPI_E_INVAL, "NULL argument");
    if (K < 1 || K > MPPI_MAX_K || H < 1 || H > MPPI_MAX_H || m < 0) return fail(MPPI_E_INVAL, "K, H or m out of range");
    const bool dev = flags & MPPI_DEVICE_PTRS, sps = flags & MPPI_SIGMA_PER_STEP;
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const size_t nsig = sps ? (size_t)H * NU : NU;
    const void *dnu, *dsig;
    if ((rc = stage_in(ctx, S_IN0, nu, (size_t)H * NU * sizeof(float), dev, s, &dnu))) return rc;
    if ((rc = stage_in(ctx, S_IN1, sigma, nsig * sizeof(float), dev, s, &dsig))) return rc;
    const size_t nu_n = (size_t)K * H * NU;
    void *dU, *dz, *dw;
    if ((rc = out_ptr(ctx, S_OUT0, U, nu_n * sizeof(float), dev, &dU))) return rc;
    if ((rc = out_ptr(ctx, S_OUT1, z_out, nu_n * sizeof(float), dev, &dz))) return rc;
    if ((rc = out_ptr(ctx, S_OUT2, words_out, (size_t)K * H * 16 * sizeof(uint32_t), dev, &dw))) return rc;
    launch_sample(scene->dev, (const float *)dnu, (const float *)dsig, sps, (uint32_t)(seed & 0xffffffffu),
                  (uint32_t)(seed >> 32), m, K, H, (float *)dU, (float *)dz, (uint32_t *)dw, s);
    HIPCHK(hipGetLastError());
    if ((rc = copy_out(U, dU, nu_n * sizeof(float), dev, s))) return rc;
    if ((rc = copy_out(z_out, dz, nu_n * sizeof(float), dev, s))) return rc;
    if ((rc = copy_out(words_out, dw, (size_t)K * H * 16 * sizeof(uint32_t), dev, s))) return rc;
    if (!dev || (flags & MPPI_SYNC)) HIPCHK(hipStreamSynchronize(s));
    return MPPI_OK;
}

int mppi_update(mppi_ctx *ctx, const mppi_scene *scene, const float *costs, const float *nu_in, const float *sigma,
                uint64_t seed, int m, int K, int H, double lambda, double eta, int n_elite, float *nu_out,
                double *nu_out64, double *weights, mppi_stats *stats, unsigned flags, void *stream)
{
    if (!ctx || !scene || !costs || !nu_in || !sigma || !nu_out) return fail(MPPI_E_INVAL, "NULL argument");
    if (K < 1 || K > MPPI_MAX_K || H < 1 || H > MPPI_MAX_H || m < 0) return fail(MPPI_E_INVAL, "K, H or m out of range");
    if (!(lambda > 0) || !std::isfinite(lambda) || !std::isfinite(eta)) return fail(MPPI_E_INVAL, "bad lambda or eta");
    const bool dev = flags & MPPI_DEVICE_PTRS, sps = flags & MPPI_SIGMA_PER_STEP;
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const size_t nsig = sps ? (size_t)H * NU : NU;
    const void *dc, *dnu, *dsig;
    if ((rc = stage_in(ctx, S_IN0, costs, (size_t)K * sizeof(float), dev, s, &dc))) return rc;
    if ((rc = stage_in(ctx, S_IN1, nu_in, (size_t)H * NU * sizeof(float), dev, s, &dnu))) return rc;
    if ((rc = stage_in(ctx, S_SIGMA, sigma, nsig * sizeof(float), dev, s, &dsig))) return rc;
    void *dout, *dout64, *dw;
    if ((rc = out_ptr(ctx, S_OUT0, nu_out, (size_t)H * NU * sizeof(float), dev, &dout))) return rc;
    if ((rc = out_ptr(ctx, S_OUT1, nu_out64, (size_t)H * NU * sizeof(double), dev, &dout64))) return rc;
    if ((rc = out_ptr(ctx, S_OUT2, weights, (size_t)K * sizeof(double), dev, &dw))) return rc;
    if (!dw && (rc = ensure(ctx, S_W, (size_t)K * sizeof(double), &dw))) return rc;
    const int ne = (n_elite <= 0 || n_elite >= K) ? K : n_elite;
    launch_reset_stats(ctx->st, s);
    const int f32 = (flags & MPPI_FP32_WEIGHTS) ? 1 : 0;
    StatsArgs sa = {(const float *)dc, K, 1.0 / lambda, ne, (double *)dw, ctx->st, 0, nullptr, f32};
    launch_stats(sa, s);
    UpdateArgs ua = {(const double *)dw, K, H, (const float *)dnu, (const float *)dsig, sps, scene->host.u_max,
                     (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), m, eta, ctx->st, (float *)dout,
                     (double *)dout64, f32};
    launch_update(ua, s);
    HIPCHK(hipGetLastError());
    if ((rc = copy_out(nu_out, dout, (size_t)H * NU * sizeof(float), dev, s))) return rc;
    if ((rc = copy_out(nu_out64, dout64, (size_t)H * NU * sizeof(double), dev, s))) return rc;
    if ((rc = copy_out(weights, dw, (size_t)K * sizeof(double), dev, s))) return rc;
    PlanStats hs;
    HIPCHK(hipMemcpyAsync(&hs, ctx->st, sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->ess = hs.ess;
        stats->c_min = hs.cmin;
        stats->best = hs.best;
        stats->n_nonfinite = K - hs.n_finite;
        stats->diverged = hs.diverged;
        stats->iterations = 1;
        stats->cmin_iter[0] = hs.cmin;
    }
    if (hs.diverged) return fail(MPPI_E_DIVERGED, "no finite cost");
    return MPPI_OK;
}

int mppi_autotune(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *sigma, int K, int H,
                  int *mapping, float *ms)
{
    if (!ctx || !scene || !x0 || !sigma) return fail(MPPI_E_INVAL, "NULL argument");
    if (scene->ctx != ctx) return fail(MPPI_E_INVAL, "scene belongs to another context");
    if (K < 1 || K > MPPI_MAX_K || H < 1 || H > MPPI_MAX_H) return fail(MPPI_E_INVAL, "K=%d or H=%d out of range", K, H);
    if (!all_finite(x0, NX) || !all_finite(sigma, NU)) return fail(MPPI_E_INVAL, "non-finite input");
    if (scene->host.task_form)
        return fail(MPPI_E_INVAL, "the autotuner times ball scenes; scenes with a box object or the further task-cost "
                                  "terms follow the mapping it records for their size");
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto done = [&](int code) {
        // every launch below has completed (each is waited for), and with it
        // the context's earlier work that the stream waited for first
        (void)hipStreamSynchronize(s);
        ctx->has_last = false;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(s);
        return code;
    };
    // the scratch buffers below may still serve the context's previous call
    if (ctx->has_last && hipStreamWaitEvent(s, ctx->order_ev, 0) != hipSuccess)
        return done(fail(MPPI_E_DEVICE, "ordering after the previous call failed"));
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return done(fail(MPPI_E_DEVICE, "event creation failed"));
    const void *dx0, *dsig;
    void *dnu, *dcost, *ddist;
    if ((rc = stage_in(ctx, S_X0, x0, NX * sizeof(float), false, s, &dx0)) ||
        (rc = stage_in(ctx, S_SIGMA, sigma, NU * sizeof(float), false, s, &dsig)) ||
        (rc = ensure(ctx, S_NU, (size_t)H * NU * sizeof(float), &dnu)) ||
        (rc = ensure(ctx, S_COSTS, (size_t)K * sizeof(float), &dcost)) ||
        (rc = ensure(ctx, S_DIST, (size_t)K * MAXCOST * sizeof(float), &ddist)))
        return done(rc);
    if (hipMemsetAsync(dnu, 0, (size_t)H * NU * sizeof(float), s) != hipSuccess)
        return done(fail(MPPI_E_DEVICE, "clearing the mean failed"));
    RolloutArgs ra = {};
    ra.md = scene->dev;
    ra.x0 = (const float *)dx0;
    ra.x0_shared = 1;
    ra.nu = (const float *)dnu;
    ra.sigma = (const float *)dsig;
    ra.key0 = 0x5eed;
    ra.K = K;
    ra.H = H;
    ra.costs = (float *)dcost;
    ra.dist = (float *)ddist;
    const int maps[4] = {MAP_LANE, MAP_TEAM, MAP_WAVE, MAP_SPLIT};
    const unsigned flag_of[4] = {MPPI_MAP_LANE, MPPI_MAP_TEAM, MPPI_MAP_WAVE, MPPI_MAP_SPLIT};
    float best = 0.f;
    int bi = 0;
    for (int i = 0; i < 4; ++i) {
        float t = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
            ra.m = rep;
            if (hipEventRecord(e0, s) != hipSuccess) return done(fail(MPPI_E_DEVICE, "event record failed"));
            launch_rollout(ra, scene->host.n_cmax, s, maps[i]);
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return done(fail(MPPI_E_DEVICE, "timing launch failed"));
            float ms1 = 0.f;
            if (hipEventElapsedTime(&ms1, e0, e1) != hipSuccess) return done(fail(MPPI_E_DEVICE, "event timing failed"));
            if (rep > 0) t = rep == 1 ? ms1 : std::min(t, ms1);  // the first launch warms up
        }
        if (ms) ms[i] = t;
        if (i == 0 || t < best) {
            best = t;
            bi = i;
        }
    }
    if (hipGetLastError() != hipSuccess) return done(fail(MPPI_E_DEVICE, "rollout launch failed"));
    ctx->tuned_map[k_class(K)] = maps[bi];
    if (mapping) *mapping = (int)flag_of[bi];
    return done(MPPI_OK);
}

int mppi_broadphase(mppi_ctx *ctx, const mppi_scene *scene, const float *lo, const float *hi, int n, float margin,
                    int *flags, unsigned flags_in, void *stream)
{
    if (!ctx || !scene || !lo || !hi || !flags) return fail(MPPI_E_INVAL, "NULL argument");
    if (n < 1 || n > MPPI_MAX_K) return fail(MPPI_E_INVAL, "n out of range");
    const bool dev = flags_in & MPPI_DEVICE_PTRS;
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const int ng = G_BOX + scene->host.n_box, np = scene->host.n_pairs;
    const size_t nb = (size_t)n * ng * 3 * sizeof(float);
    const void *dlo, *dhi;
    if ((rc = stage_in(ctx, S_IN0, lo, nb, dev, s, &dlo))) return rc;
    if ((rc = stage_in(ctx, S_IN1, hi, nb, dev, s, &dhi))) return rc;
    void *df;
    if ((rc = out_ptr(ctx, S_OUT0, flags, (size_t)n * np * sizeof(int), dev, &df))) return rc;
    launch_broadphase(scene->dev, (const float *)dlo, (const float *)dhi, n, ng, margin, (int *)df, s);
    HIPCHK(hipGetLastError());
    if ((rc = copy_out(flags, df, (size_t)n * np * sizeof(int), dev, s))) return rc;
    if (!dev || (flags_in & MPPI_SYNC)) HIPCHK(hipStreamSynchronize(s));
    return MPPI_OK;
}

int mppi_narrowphase(mppi_ctx *ctx, const mppi_scene *scene, const float *X, int n, float *phi, float *normal,
                     float *point, float *lo, float *hi, unsigned flags, void *stream)
{
    if (!ctx || !scene || !X || !phi) return fail(MPPI_E_INVAL, "NULL argument");
    if (n < 1 || n > MPPI_MAX_K) return fail(MPPI_E_INVAL, "n out of range");
    if ((lo == nullptr) != (hi == nullptr)) return fail(MPPI_E_INVAL, "lo and hi go together");
    const bool dev = flags & MPPI_DEVICE_PTRS;
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    CtxStream order_guard(ctx, s);
    if ((rc = order_guard.begin())) return rc;
    const int np = scene->host.n_pairs, ng = G_BOX + scene->host.n_box;
    const void *dX;
    if ((rc = stage_in(ctx, S_IN0, X, (size_t)n * NX * sizeof(float), dev, s, &dX))) return rc;
    void *dphi, *dn, *dp, *dlo, *dhi;
    if ((rc = out_ptr(ctx, S_OUT0, phi, (size_t)n * np * sizeof(float), dev, &dphi))) return rc;
    if ((rc = out_ptr(ctx, S_OUT1, normal, (size_t)n * np * 3 * sizeof(float), dev, &dn))) return rc;
    if ((rc = out_ptr(ctx, S_OUT2, point, (size_t)n * np * 3 * sizeof(float), dev, &dp))) return rc;
    if ((rc = out_ptr(ctx, S_OUT3, lo, (size_t)2 * n * ng * 3 * sizeof(float), dev, &dlo))) return rc;
    dhi = nullptr;
    if (lo) dhi = dev ? (void *)hi : (void *)((float *)dlo + (size_t)n * ng * 3);
    launch_narrowphase(scene->dev, (const float *)dX, n, (float *)dphi, (float *)dn, (float *)dp, (float *)dlo,
                       (float *)dhi, s);
    HIPCHK(hipGetLastError());
    if ((rc = copy_out(phi, dphi, (size_t)n * np * sizeof(float), dev, s))) return rc;
    if ((rc = copy_out(normal, dn, (size_t)n * np * 3 * sizeof(float), dev, s))) return rc;
    if ((rc = copy_out(point, dp, (size_t)n * np * 3 * sizeof(float), dev, s))) return rc;
    if ((rc = copy_out(lo, dlo, (size_t)n * ng * 3 * sizeof(float), dev, s))) return rc;
    if ((rc = copy_out(hi, dhi, (size_t)n * ng * 3 * sizeof(float), dev, s))) return rc;
    if (!dev || (flags & MPPI_SYNC)) HIPCHK(hipStreamSynchronize(s));
    return MPPI_OK;
}

}  // extern "C"

int mppi_host::plan_with(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
                         double lambda, const float *sigma, const mppi_opts *opts, const mppi_qp *qp,
                         const mppi_cov *cov, float *U_new, float *U_best, float *costs, mppi_stats *stats,
                         void *stream)
{
    int rc;
    if (qp && (rc = qp_check(qp, H))) return rc;
    if (cov) {
        mppi_cov c = *cov;
        c.U_best = U_best;
        return mppi_plan_cov(ctx, scene, x0, nominal_U, K, H, lambda, sigma, opts, &c, qp, U_new, costs, stats,
                             stream);
    }
    return plan_impl(ctx, scene, x0, nominal_U, K, H, lambda, sigma, opts, qp, nullptr, U_new, costs, stats, stream,
                     U_best);
}
