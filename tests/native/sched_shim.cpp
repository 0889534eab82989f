// C wrappers over the host-only scheduling core (csrc/sched.h) so that the
// admission and arena logic of the serving loop is tested on the CPU.
#include <cstdint>
#include <vector>

#include "sched.h"

using namespace mppi;

extern "C" {

void *arena_new(uint64_t bytes) { return new Arena(bytes); }
void arena_free(void *a) { delete (Arena *)a; }
int64_t arena_alloc(void *a, uint64_t n)
{
    const size_t o = ((Arena *)a)->alloc(n);
    return o == NO_SPACE ? -1 : (int64_t)o;
}
int arena_release(void *a, uint64_t off) { return ((Arena *)a)->release(off) ? 1 : 0; }
uint64_t arena_used(void *a) { return ((Arena *)a)->used(); }
uint64_t arena_largest(void *a) { return ((Arena *)a)->largest_free(); }
uint64_t arena_nfree(void *a) { return ((Arena *)a)->n_free_ranges(); }
uint64_t arena_high(void *a) { return ((Arena *)a)->high_water(); }

void *sched_new(uint64_t dev, uint64_t host, int max_active, int max_pending)
{
    return new Scheduler(dev, host, max_active, max_pending);
}
void sched_free(void *s) { delete (Scheduler *)s; }
// returns the enqueue code; superseded ids are written to sup (count in *nsup)
int sched_enqueue(void *s, uint64_t id, int cell, int M, uint64_t dev, uint64_t host, int supersede, uint64_t *sup,
                  int *nsup)
{
    SchedReq r;
    r.id = id;
    r.cell = cell;
    r.M = M;
    r.dev_bytes = dev;
    r.host_bytes = host;
    std::vector<uint64_t> v;
    const int rc = ((Scheduler *)s)->enqueue(r, supersede != 0, &v);
    *nsup = (int)v.size();
    for (size_t i = 0; i < v.size(); ++i) sup[i] = v[i];
    return rc;
}
// enqueue with an absolute deadline (ms) and the work of one iteration
int sched_enqueue_dl(void *s, uint64_t id, int cell, int M, uint64_t dev, double deadline, double work)
{
    SchedReq r;
    r.id = id;
    r.cell = cell;
    r.M = M;
    r.dev_bytes = dev;
    r.host_bytes = 256;
    r.deadline = deadline;
    r.work = work;
    return ((Scheduler *)s)->enqueue(r, false, nullptr);
}
// admission at time `now` with the iteration model (base_ms + slope * W);
// shed ids in shed (count in *nshed)
int sched_admit_dl(void *s, double now, double base_ms, double slope, double floor_ms, int extra, uint64_t *ids,
                   uint64_t *shed, int *nshed)
{
    std::vector<uint64_t> sh;
    IterModel im;
    im.base_ms = base_ms;
    im.ms_per_work = slope;
    im.floor_ms = floor_ms;
    std::vector<uint64_t> v = ((Scheduler *)s)->admit(now, im, &sh, extra);
    for (size_t i = 0; i < v.size(); ++i) ids[i] = v[i];
    *nshed = (int)sh.size();
    for (size_t i = 0; i < sh.size(); ++i) shed[i] = sh[i];
    return (int)v.size();
}
int sched_admit(void *s, uint64_t *ids)
{
    std::vector<uint64_t> v = ((Scheduler *)s)->admit();
    for (size_t i = 0; i < v.size(); ++i) ids[i] = v[i];
    return (int)v.size();
}
int sched_cancel(void *s, uint64_t id) { return ((Scheduler *)s)->cancel(id); }
// active ids and their iteration index; dropped ids (cancelled) in drop
int sched_next(void *s, uint64_t *ids, int *m, uint64_t *drop, int *ndrop)
{
    std::vector<uint64_t> d;
    std::vector<const SchedReq *> v = ((Scheduler *)s)->next_iteration(&d);
    for (size_t i = 0; i < v.size(); ++i) {
        ids[i] = v[i]->id;
        m[i] = v[i]->m;
    }
    *ndrop = (int)d.size();
    for (size_t i = 0; i < d.size(); ++i) drop[i] = d[i];
    return (int)v.size();
}
int sched_advance(void *s, uint64_t *ids)
{
    std::vector<uint64_t> v = ((Scheduler *)s)->advance();
    for (size_t i = 0; i < v.size(); ++i) ids[i] = v[i];
    return (int)v.size();
}
int sched_release(void *s, uint64_t id) { return ((Scheduler *)s)->release(id) ? 1 : 0; }
void sched_forget(void *s, uint64_t id) { ((Scheduler *)s)->forget(id); }
int sched_cell_idle(void *s, int cell) { return ((Scheduler *)s)->cell_idle(cell) ? 1 : 0; }
int sched_counts(void *s, int *active, int *pending, uint64_t *dev_used, uint64_t *host_used)
{
    Scheduler *p = (Scheduler *)s;
    *active = p->n_active();
    *pending = p->n_pending();
    *dev_used = p->dev().used();
    *host_used = p->host().used();
    return 0;
}
}
