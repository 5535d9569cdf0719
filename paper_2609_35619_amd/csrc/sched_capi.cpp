// C entry points over the serving scheduler, for host-only tests: the caller
// plays the executor (plans steps and reports them done).  Built with the
// host compiler into libcsplat_sched.so; not part of the product ABI.
#include <cstddef>
#include <cstdint>

#include "sched.h"

using csplat::serve::Item;
using csplat::serve::ReqSpec;
using csplat::serve::Scheduler;
using csplat::serve::StepPlan;

extern "C" {

void *sched_new(uint64_t dev, uint64_t host, int32_t slots, int64_t step_pairs, int64_t max_items)
{
    return new Scheduler(dev, host, slots, step_pairs, max_items);
}

void sched_set_min_items(void *s, int64_t n) { static_cast<Scheduler *>(s)->set_min_items(n); }

void sched_free(void *s) { delete static_cast<Scheduler *>(s); }

int64_t sched_submit(void *s, int32_t tiles, int32_t splits, int32_t variant, int64_t item_pairs,
                     uint64_t dev_bytes, uint64_t host_bytes, double now)
{
    ReqSpec r;
    r.tiles = tiles;
    r.splits = splits;
    r.variant = variant;
    r.item_pairs = item_pairs;
    r.dev_bytes = dev_bytes;
    r.host_bytes = host_bytes;
    return static_cast<Scheduler *>(s)->submit(r, now);
}

int32_t sched_admit(void *s, double now, int64_t *out, int32_t cap)
{
    auto v = static_cast<Scheduler *>(s)->admit(now);
    int32_t n = 0;
    for (int64_t t : v)
        if (n < cap) out[n++] = t;
    return (int32_t)v.size();
}

// items: 4 int32 per item (slot, tile, split, variant); returns the step id
// (0 when there is nothing to issue)
int64_t sched_plan(void *s, int32_t *items, int32_t cap, int32_t *completing, int32_t ccap, int32_t *n_items,
                   int32_t *n_completing, int64_t *pairs)
{
    StepPlan p;
    if (!static_cast<Scheduler *>(s)->plan(&p)) {
        *n_items = *n_completing = 0;
        *pairs = 0;
        return 0;
    }
    *n_items = (int32_t)p.items.size();
    *n_completing = (int32_t)p.completing.size();
    *pairs = p.pairs;
    for (int32_t i = 0; i < *n_items && i < cap; ++i) {
        const Item &it = p.items[(size_t)i];
        items[4 * i] = it.slot;
        items[4 * i + 1] = it.tile;
        items[4 * i + 2] = it.split;
        items[4 * i + 3] = it.variant;
    }
    for (int32_t i = 0; i < *n_completing && i < ccap; ++i) completing[i] = p.completing[(size_t)i];
    return p.step;
}

int32_t sched_step_done(void *s, int64_t step, double now, int64_t *out, int32_t cap)
{
    auto v = static_cast<Scheduler *>(s)->step_done(step, now);
    int32_t n = 0;
    for (int64_t t : v)
        if (n < cap) out[n++] = t;
    return (int32_t)v.size();
}

int32_t sched_cancel(void *s, int64_t t, double now) { return static_cast<Scheduler *>(s)->cancel(t, now) ? 1 : 0; }
int32_t sched_finish(void *s, int64_t t) { return static_cast<Scheduler *>(s)->finish(t) ? 1 : 0; }

int32_t sched_state(void *s, int64_t t)
{
    auto *r = static_cast<Scheduler *>(s)->info(t);
    return r ? (int32_t)r->state : -1;
}

int32_t sched_slot(void *s, int64_t t)
{
    auto *r = static_cast<Scheduler *>(s)->info(t);
    return r ? r->slot : -1;
}

int32_t sched_active(void *s) { return static_cast<Scheduler *>(s)->active(); }
int32_t sched_queued(void *s) { return static_cast<Scheduler *>(s)->queued(); }
uint64_t sched_dev_free(void *s) { return static_cast<Scheduler *>(s)->dev_arena().free_bytes(); }
uint64_t sched_host_free(void *s) { return static_cast<Scheduler *>(s)->host_arena().free_bytes(); }
uint64_t sched_dev_largest(void *s) { return static_cast<Scheduler *>(s)->dev_arena().largest_free(); }
}
