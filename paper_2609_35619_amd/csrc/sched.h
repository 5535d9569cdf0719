// Host scheduler of the serving form: admission of requests by device and
// host memory budget and by slots, and continuous batching of their work
// items into bounded steps.  Pure C++ (no HIP): the GPU executor in
// serve.hip and the CPU tests (through sched_capi.cpp, with a fake executor
// that completes steps on command) drive the same code.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace csplat {
namespace serve {

// First-fit allocator over the offsets [0, size) of one preallocated buffer.
class Arena {
  public:
    explicit Arena(uint64_t size = 0, uint64_t align = 256);
    bool alloc(uint64_t bytes, uint64_t *off);
    void release(uint64_t off);
    uint64_t size() const { return size_; }
    uint64_t free_bytes() const;
    uint64_t largest_free() const;
    int used_blocks() const { return (int)used_.size(); }

  private:
    uint64_t size_, align_;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
    std::map<uint64_t, uint64_t> used_;
};

enum class State : int { Queued = 0, Active = 1, Done = 2, Cancelled = 3, Finished = 4 };

// What the scheduler needs to know about a request.
struct ReqSpec {
    int32_t tiles = 0;       // query tiles
    int32_t splits = 0;      // work items per query tile, each a group of Gaussian splits (fixed per
                             // request: results never depend on the mix)
    int32_t variant = 0;     // which step kernel evaluates its items
    int64_t item_pairs = 0;  // pair evaluations of one item (step budget accounting)
    uint64_t dev_bytes = 0;  // device arena bytes (inputs, partial reductions)
    uint64_t host_bytes = 0; // pinned host bytes (input staging, outputs)
};

struct Item {
    int32_t slot;    // request slot (index into the device descriptor table)
    int32_t tile;
    int32_t split;
    int32_t variant;
};

struct StepPlan {
    int64_t step = 0;
    std::vector<Item> items;            // sorted by variant
    std::vector<int32_t> completing;    // slots whose last items are in this step
    int64_t pairs = 0;
};

struct ReqInfo {
    State state = State::Queued;
    ReqSpec spec;
    int32_t slot = -1;
    uint64_t dev_off = 0, host_off = 0;
    int64_t next_item = 0;      // items issued so far
    int64_t inflight = 0;       // issued items whose step has not completed
    bool cancel_requested = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

class Scheduler {
  public:
    Scheduler(uint64_t dev_budget, uint64_t host_budget, int slots, int64_t step_pairs, int64_t max_items);

    // A new request; returns its ticket (> 0), or -1 if it can never fit the
    // budgets (device bytes, host bytes).
    int64_t submit(const ReqSpec &spec, double now);
    // Admit queued requests in arrival order while slots and memory allow
    // (a request that does not fit yet does not block smaller later ones).
    // Returns the tickets admitted by this call.
    std::vector<int64_t> admit(double now);
    // Plan the next step: round-robin over active requests, one item per
    // request per round, until the pair budget or the item cap is reached.
    // Returns false when there is nothing to issue.
    bool plan(StepPlan *out);
    // The GPU finished step `step`: requests whose every item has completed
    // become Done (or Cancelled).  Returns the tickets that changed state.
    std::vector<int64_t> step_done(int64_t step, double now);
    // Cancel: a queued request is dropped at once; an active one issues no
    // more items and becomes Cancelled when its in-flight items complete.
    bool cancel(int64_t ticket, double now);
    // The caller collected a Done/Cancelled request: free its host memory.
    bool finish(int64_t ticket);

    // The pair budget of a step (dense pairs, Q x N per item); the executor
    // steers it toward a target step duration.
    void set_step_pairs(int64_t pairs) { step_pairs_ = pairs; }
    int64_t step_pairs() const { return step_pairs_; }
    // A step takes at least this many items when that many are waiting,
    // whatever the pair budget (a step of a few long items would leave the
    // device idle while they run).
    void set_min_items(int64_t n) { min_items_ = n; }

    const ReqInfo *info(int64_t ticket) const;
    int active() const;
    int queued() const { return (int)queue_.size(); }
    int64_t inflight_steps() const { return (int64_t)steps_.size(); }
    const Arena &dev_arena() const { return dev_; }
    const Arena &host_arena() const { return host_; }

  private:
    void retire(int64_t ticket, ReqInfo &r, State s, double now);

    Arena dev_, host_;
    int slots_;
    int64_t step_pairs_, max_items_;
    int64_t min_items_ = 0;
    int64_t next_ticket_ = 1, next_step_ = 1;
    std::map<int64_t, ReqInfo> reqs_;
    std::deque<int64_t> queue_;
    std::vector<int64_t> slot_owner_;      // slot -> ticket (0: free)
    size_t rr_ = 0;                        // round-robin cursor over slots
    std::map<int64_t, std::vector<std::pair<int32_t, int64_t>>> steps_;  // step -> (slot, items)
};

}  // namespace serve
}  // namespace csplat
