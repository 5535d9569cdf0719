// Host scheduler of the serving form (see sched.h).
#include "sched.h"

#include <algorithm>

namespace csplat {
namespace serve {

Arena::Arena(uint64_t size, uint64_t align) : size_(size), align_(align ? align : 1)
{
    if (size_ > 0) free_[0] = size_;
}

bool Arena::alloc(uint64_t bytes, uint64_t *off)
{
    uint64_t need = (bytes + align_ - 1) / align_ * align_;
    if (need == 0) need = align_;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= need) {
            const uint64_t o = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[o + need] = len - need;
            used_[o] = need;
            *off = o;
            return true;
        }
    }
    return false;
}

void Arena::release(uint64_t off)
{
    auto u = used_.find(off);
    if (u == used_.end()) return;
    uint64_t o = u->first, len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(o);
    if (next != free_.end() && o + len == next->first) {  // merge with the following block
        len += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {  // merge with the preceding block
        auto prev = std::prev(next);
        if (prev->first + prev->second == o) {
            prev->second += len;
            return;
        }
    }
    free_[o] = len;
}

uint64_t Arena::free_bytes() const
{
    uint64_t s = 0;
    for (auto &kv : free_) s += kv.second;
    return s;
}

uint64_t Arena::largest_free() const
{
    uint64_t s = 0;
    for (auto &kv : free_) s = std::max(s, kv.second);
    return s;
}

Scheduler::Scheduler(uint64_t dev_budget, uint64_t host_budget, int slots, int64_t step_pairs,
                     int64_t max_items)
    : dev_(dev_budget), host_(host_budget), slots_(slots), step_pairs_(step_pairs),
      max_items_(max_items), slot_owner_((size_t)std::max(slots, 0), 0)
{
}

int64_t Scheduler::submit(const ReqSpec &spec, double now)
{
    if (spec.dev_bytes > dev_.size() || spec.host_bytes > host_.size()) return -1;
    const int64_t t = next_ticket_++;
    ReqInfo r;
    r.spec = spec;
    r.t_submit = now;
    reqs_[t] = r;
    queue_.push_back(t);
    return t;
}

std::vector<int64_t> Scheduler::admit(double now)
{
    std::vector<int64_t> out;
    for (auto it = queue_.begin(); it != queue_.end();) {
        int slot = -1;
        for (int s = 0; s < slots_; ++s)
            if (slot_owner_[(size_t)s] == 0) {
                slot = s;
                break;
            }
        if (slot < 0) break;  // no free slot: nothing more can be admitted now
        ReqInfo &r = reqs_[*it];
        uint64_t doff = 0, hoff = 0;
        if (!dev_.alloc(r.spec.dev_bytes, &doff)) {
            ++it;
            continue;
        }
        if (!host_.alloc(r.spec.host_bytes, &hoff)) {
            dev_.release(doff);
            ++it;
            continue;
        }
        r.state = State::Active;
        r.slot = slot;
        r.dev_off = doff;
        r.host_off = hoff;
        r.t_admit = now;
        slot_owner_[(size_t)slot] = *it;
        out.push_back(*it);
        it = queue_.erase(it);
    }
    return out;
}

int Scheduler::active() const
{
    int a = 0;
    for (int64_t t : slot_owner_) a += t != 0;
    return a;
}

bool Scheduler::plan(StepPlan *out)
{
    out->items.clear();
    out->completing.clear();
    out->pairs = 0;
    std::map<int32_t, int64_t> per_slot;
    const size_t ns = slot_owner_.size();
    bool progress = true;
    auto room = [&]() {
        const int64_t n = (int64_t)out->items.size();
        return n < max_items_ && (out->pairs < step_pairs_ || n < min_items_);
    };
    while (progress && room()) {
        progress = false;
        for (size_t k = 0; k < ns; ++k) {
            const size_t s = (rr_ + k) % ns;
            const int64_t t = slot_owner_[s];
            if (!t) continue;
            ReqInfo &r = reqs_[t];
            if (r.cancel_requested) continue;
            const int64_t total = (int64_t)r.spec.tiles * r.spec.splits;
            if (total == 0) {
                // nothing to evaluate (empty scene or no queries): only the final
                // reduction runs; book it once as a pseudo item
                if (r.next_item == 0) {
                    r.next_item = 1;
                    r.inflight += 1;
                    per_slot[(int32_t)s] += 1;
                    out->completing.push_back((int32_t)s);
                    progress = true;
                }
                continue;
            }
            if (r.next_item >= total) continue;
            if (!room()) break;
            const int64_t idx = r.next_item++;
            Item it;
            it.slot = (int32_t)s;
            it.split = (int32_t)(idx / r.spec.tiles);
            it.tile = (int32_t)(idx - (int64_t)it.split * r.spec.tiles);
            it.variant = r.spec.variant;
            out->items.push_back(it);
            out->pairs += r.spec.item_pairs;
            r.inflight += 1;
            per_slot[(int32_t)s] += 1;
            if (r.next_item == total) out->completing.push_back((int32_t)s);
            progress = true;
        }
    }
    if (ns) rr_ = (rr_ + 1) % ns;
    if (out->items.empty() && out->completing.empty()) return false;
    std::stable_sort(out->items.begin(), out->items.end(),
                     [](const Item &a, const Item &b) { return a.variant < b.variant; });
    out->step = next_step_++;
    auto &rec = steps_[out->step];
    for (auto &kv : per_slot) rec.emplace_back(kv.first, kv.second);
    return true;
}

void Scheduler::retire(int64_t ticket, ReqInfo &r, State s, double now)
{
    if (r.slot >= 0) {
        dev_.release(r.dev_off);
        slot_owner_[(size_t)r.slot] = 0;
    }
    r.state = s;
    r.t_done = now;
    (void)ticket;
}

std::vector<int64_t> Scheduler::step_done(int64_t step, double now)
{
    std::vector<int64_t> changed;
    auto it = steps_.find(step);
    if (it == steps_.end()) return changed;
    for (auto &sc : it->second) {
        const int64_t t = slot_owner_[(size_t)sc.first];
        if (!t) continue;
        ReqInfo &r = reqs_[t];
        r.inflight -= sc.second;
        if (r.inflight > 0) continue;
        const int64_t total = std::max<int64_t>((int64_t)r.spec.tiles * r.spec.splits, 1);
        if (r.cancel_requested) {
            retire(t, r, State::Cancelled, now);
            changed.push_back(t);
        } else if (r.next_item >= total) {
            retire(t, r, State::Done, now);
            changed.push_back(t);
        }
    }
    steps_.erase(it);
    return changed;
}

bool Scheduler::cancel(int64_t ticket, double now)
{
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return false;
    ReqInfo &r = it->second;
    if (r.state == State::Queued) {
        queue_.erase(std::remove(queue_.begin(), queue_.end(), ticket), queue_.end());
        r.state = State::Cancelled;
        r.t_done = now;
        return true;
    }
    if (r.state != State::Active) return false;
    r.cancel_requested = true;
    if (r.inflight == 0) retire(ticket, r, State::Cancelled, now);
    return true;
}

bool Scheduler::finish(int64_t ticket)
{
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return false;
    ReqInfo &r = it->second;
    if (r.state != State::Done && r.state != State::Cancelled) return false;
    if (r.slot >= 0) host_.release(r.host_off);
    reqs_.erase(it);
    return true;
}

const ReqInfo *Scheduler::info(int64_t ticket) const
{
    auto it = reqs_.find(ticket);
    return it == reqs_.end() ? nullptr : &it->second;
}

}  // namespace serve
}  // namespace csplat
