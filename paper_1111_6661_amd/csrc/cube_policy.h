// cube_policy.h -- the admission and batching policy of the query server,
// free of any GPU call so that it can be tested on a CPU.
//
// The paper's scheduler allocates tasks from status kept in shared memory
// (Section 2) and serves many users' batched and real-time requests
// (Abstract, Section 3).  Here the policy is continuous batching:
//   * queries wait in arrival order;
//   * a batch is formed whenever an execution slot is free: it takes the
//     oldest waiting queries while the batch stays within `max_batch`
//     queries and `max_batch_voxels` voxels (a single larger query is
//     taken alone), and while the bytes in flight over all slots stay
//     within `max_inflight_bytes` (admission by memory);
//   * batches on different slots run concurrently, so queries that arrive
//     while others are on the device are admitted as slots and memory free
//     up, without waiting for the running batches to finish.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <vector>

namespace cube {

struct PolicyLimits {
    int slots = 4;                          // concurrent batches (streams)
    int max_batch = 64;                     // queries per batch
    int64_t max_batch_voxels = 1ll << 33;   // voxels per batch (soft)
    int64_t max_inflight_bytes = 1ll << 30; // scratch bytes over all slots
    size_t max_queue = 1 << 16;             // waiting queries
};

struct PolicyQuery {
    uint64_t id;
    int64_t voxels;         // voxels the query reads
    int64_t scratch_bytes;  // device scratch the query needs while in flight
};

class Policy {
  public:
    explicit Policy(const PolicyLimits &lim) : lim_(lim), busy_(lim.slots, false),
                                               slot_bytes_(lim.slots, 0) {}

    // Queue a query; false when the queue is full (the caller reports EBUSY).
    bool submit(const PolicyQuery &q)
    {
        if (queue_.size() >= lim_.max_queue) return false;
        queue_.push_back(q);
        return true;
    }

    // Form the next batch for a free slot.  Returns the slot (and fills
    // `batch`), or -1 when no slot is free, nothing waits, or the oldest
    // waiting query does not fit the memory still free.
    int next_batch(std::vector<PolicyQuery> &batch)
    {
        batch.clear();
        if (queue_.empty()) return -1;
        int slot = -1;
        for (int s = 0; s < lim_.slots; ++s)
            if (!busy_[s]) {
                slot = s;
                break;
            }
        if (slot < 0) return -1;
        int64_t voxels = 0, bytes = 0;
        while (!queue_.empty() && (int)batch.size() < lim_.max_batch) {
            const PolicyQuery &q = queue_.front();
            const bool first = batch.empty();
            if (!first && voxels + q.voxels > lim_.max_batch_voxels) break;
            if (inflight_ + bytes + q.scratch_bytes > lim_.max_inflight_bytes) {
                // A query larger than the whole budget runs alone once the
                // device is otherwise idle.
                const bool alone_ok = first && inflight_ == 0;
                if (!alone_ok) break;
            }
            voxels += q.voxels;
            bytes += q.scratch_bytes;
            batch.push_back(q);
            queue_.pop_front();
        }
        if (batch.empty()) return -1;
        busy_[slot] = true;
        slot_bytes_[slot] = bytes;
        inflight_ += bytes;
        return slot;
    }

    // The batch on `slot` has completed.
    void complete(int slot)
    {
        if (slot < 0 || slot >= lim_.slots || !busy_[slot]) return;
        busy_[slot] = false;
        inflight_ -= slot_bytes_[slot];
        slot_bytes_[slot] = 0;
    }

    size_t waiting() const { return queue_.size(); }
    int64_t inflight_bytes() const { return inflight_; }
    int busy_slots() const
    {
        int n = 0;
        for (bool b : busy_) n += b;
        return n;
    }
    const PolicyLimits &limits() const { return lim_; }

  private:
    PolicyLimits lim_;
    std::deque<PolicyQuery> queue_;
    std::vector<bool> busy_;
    std::vector<int64_t> slot_bytes_;
    int64_t inflight_ = 0;
};

}  // namespace cube
