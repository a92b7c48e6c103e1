// Admission and grouping policy of the native request server (server.hip),
// written without HIP so that it is unit-tested on the host.
//
// Requests wait in arrival order.  When a builder thread is free, a group
// is formed from the front of the queue: as many requests as fit (at most
// max_group, their node counts summing below 2^31) are built together on
// one free slot (a library context plus its staging buffer) as one
// block-diagonal graph.
//
// Device memory is charged per slot, so that the sum of the charges bounds
// what the server really holds:
//   * an idle or running slot is charged the bytes its buffers hold now
//     (measured after its last build: its buffers keep their size for the
//     next group, so a slot holds its high-water mark between groups);
//   * a slot that is building is charged what it held before plus the
//     group's footprint (the most its build can add: server contexts grow
//     buffers to the exact size asked for, and a footprint bounds the sum of
//     the sizes a build asks for).
// A group is admitted only if the charges stay within the budget.  To make
// room, idle slots are trimmed (their buffers released), largest first,
// and the slot the group builds on last.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <stdexcept>
#include <vector>

namespace cleora {

struct AdmitDecision {
    int slot = -1;           // slot the group builds on
    int32_t count = 0;       // requests taken from the front of the queue
    int64_t footprint = 0;   // their summed footprint
    std::vector<int> trim;   // idle slots to release before the build (may include `slot`)
};

class Admission {
public:
    static constexpr int64_t kMaxNodes = 0x7fffffffLL;  // node ids of a group are int32

    Admission(int slots, int64_t budget, int32_t max_group)
        : budget_(budget), max_group_(max_group), held_(slots, 0), state_(slots, Idle)
    {
        if (slots < 1 || budget < 0 || max_group < 1)
            throw std::invalid_argument("bad admission parameters");
        for (int s = 0; s < slots; ++s) free_.push_back(s);
    }

    // A request joins the back of the queue.
    void push(int64_t footprint, int64_t n_nodes)
    {
        if (footprint < 0 || n_nodes < 1 || n_nodes > kMaxNodes)
            throw std::invalid_argument("bad request");
        queue_.push_back({footprint, n_nodes});
    }
    size_t waiting() const { return queue_.size(); }
    // Drop the first `n` waiting requests (they leave without a build).
    void drop_front(size_t n)
    {
        n = std::min(n, queue_.size());
        queue_.erase(queue_.begin(), queue_.begin() + (std::ptrdiff_t)n);
    }

    // Bytes a new group could be charged if every idle slot were trimmed.
    int64_t room() const
    {
        int64_t idle_held = 0;
        for (int s : free_) idle_held += held_[s];
        return budget_ - (used_ - idle_held);
    }

    // A free slot exists and the first waiting request fits.
    bool can_admit() const
    {
        return !queue_.empty() && !free_.empty() && queue_.front().footprint <= room();
    }

    // Form a group (call only when can_admit()).  The slot with the largest
    // holding is used (its buffers are the most likely to fit the group);
    // other idle slots are trimmed, largest first, only as far as needed,
    // and the build slot itself last.
    AdmitDecision admit()
    {
        if (!can_admit()) throw std::logic_error("admit() without can_admit()");
        AdmitDecision d;
        const int64_t avail = room();
        int64_t nodes = 0;
        while (d.count < max_group_ && (size_t)d.count < queue_.size()) {
            const Waiting &q = queue_[(size_t)d.count];
            if (d.footprint + q.footprint > avail) break;
            if (d.count > 0 && nodes + q.n_nodes > kMaxNodes) break;
            d.footprint += q.footprint;
            nodes += q.n_nodes;
            ++d.count;
        }
        auto slot_it = std::max_element(free_.begin(), free_.end(),
                                        [&](int a, int b) { return held_[a] < held_[b]; });
        d.slot = *slot_it;
        free_.erase(slot_it);
        // trim idle slots until the charges fit
        int64_t over = used_ + d.footprint - budget_;
        if (over > 0) {
            std::vector<int> idle(free_.begin(), free_.end());
            std::sort(idle.begin(), idle.end(), [&](int a, int b) { return held_[a] > held_[b]; });
            idle.push_back(d.slot);
            for (int s : idle) {
                if (over <= 0) break;
                if (held_[s] == 0) continue;
                over -= held_[s];
                used_ -= held_[s];
                held_[s] = 0;
                d.trim.push_back(s);
                if (s != d.slot) {
                    // the slot is busy while its buffers are released
                    free_.erase(std::find(free_.begin(), free_.end(), s));
                    state_[s] = Trimming;
                }
            }
        }
        queue_.erase(queue_.begin(), queue_.begin() + d.count);
        state_[d.slot] = Building;
        building_fp_.push_back({d.slot, d.footprint});
        used_ += d.footprint;
        peak_ = std::max(peak_, used_);
        ++groups_;
        return d;
    }

    // The bytes an idle slot holds (e.g. measured when it is created).
    void set_idle_held(int slot, int64_t bytes)
    {
        check(slot, Idle);
        used_ += bytes - held_[(size_t)slot];
        held_[(size_t)slot] = bytes;
        peak_ = std::max(peak_, used_);
    }

    // A trimmed slot (not the build slot) has released its buffers.
    void trimmed(int slot)
    {
        check(slot, Trimming);
        state_[slot] = Idle;
        free_.push_front(slot);
    }

    // A slot's build ended (successfully or not); `held_bytes` is what its
    // buffers hold now.  Returns false if that exceeds the charge of the
    // build (the footprint did not bound the build's allocations).
    bool built(int slot, int64_t held_bytes)
    {
        check(slot, Building);
        auto it = std::find_if(building_fp_.begin(), building_fp_.end(),
                               [&](const std::pair<int, int64_t> &p) { return p.first == slot; });
        const int64_t charge = held_[slot] + it->second;
        building_fp_.erase(it);
        used_ += held_bytes - charge;
        held_[slot] = held_bytes;
        peak_ = std::max(peak_, used_);
        state_[slot] = Running;
        return held_bytes <= charge;
    }

    // The slot's group is finished; the slot is free again and keeps its
    // buffers (and its charge).
    void release(int slot)
    {
        check(slot, Running);
        state_[slot] = Idle;
        free_.push_front(slot);
    }

    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }
    int64_t held(int slot) const { return held_.at((size_t)slot); }
    int64_t budget() const { return budget_; }
    int64_t groups() const { return groups_; }
    size_t free_slots() const { return free_.size(); }

private:
    enum State { Idle, Building, Running, Trimming };
    struct Waiting {
        int64_t footprint;
        int64_t n_nodes;
    };
    void check(int slot, State s) const
    {
        if (slot < 0 || (size_t)slot >= state_.size() || state_[(size_t)slot] != s)
            throw std::logic_error("slot not in the expected state");
    }

    int64_t budget_;
    int32_t max_group_;
    std::vector<int64_t> held_;
    std::vector<State> state_;
    std::deque<int> free_;
    std::deque<Waiting> queue_;
    std::vector<std::pair<int, int64_t>> building_fp_;
    int64_t used_ = 0, peak_ = 0, groups_ = 0;
};

}  // namespace cleora
