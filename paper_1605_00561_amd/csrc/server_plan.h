// server_plan.h -- host-side bookkeeping of the serving loop (dwt2_server_*):
// sets of byte ranges, the first-fit free list over the caller's arena, and
// the choice of the next batch.  Plain C++ with no HIP, so that the serving
// loop's scheduling can also be checked on a machine without a GPU.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace dwt2 {
namespace serve {

// Disjoint byte ranges [lo, hi); insert merges overlapping and touching
// ranges, so a query only needs the range that starts last before its end.
class RangeSet {
    std::map<uintptr_t, uintptr_t> r_;  // lo -> hi

public:
    bool overlaps(uintptr_t lo, uintptr_t hi) const
    {
        auto it = r_.lower_bound(hi);
        if (it == r_.begin()) return false;
        --it;
        return it->second > lo;
    }
    void insert(uintptr_t lo, uintptr_t hi)
    {
        auto it = r_.lower_bound(lo);
        if (it != r_.begin() && std::prev(it)->second >= lo) {
            --it;
            lo = it->first;
        }
        while (it != r_.end() && it->first <= hi) {
            hi = std::max(hi, it->second);
            it = r_.erase(it);
        }
        r_[lo] = hi;
    }
    size_t size() const { return r_.size(); }
};

// First-fit free list over [0, size) bytes; released blocks coalesce with
// their free neighbours.
class Arena {
    std::map<size_t, size_t> free_;  // offset -> bytes

public:
    explicit Arena(size_t size)
    {
        if (size) free_[0] = size;
    }
    bool fits(size_t bytes) const
    {
        for (const auto &f : free_)
            if (f.second >= bytes) return true;
        return false;
    }
    // The first free block that holds `bytes`, or SIZE_MAX (callers check fits()).
    size_t alloc(size_t bytes)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            return off;
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes)
    {
        if (!bytes) return;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t blocks() const { return free_.size(); }
};

// One pending request as the scheduler sees it: the byte ranges it reads and
// writes, its direction and depth, the bytes of its own part of a batched
// call's workspace (its LL buffers and tile-index entries), and its HBM
// footprint (the bytes of its input, its output and that part).
struct Item {
    uintptr_t src_lo, src_hi, dst_lo, dst_hi;
    int inverse, levels;
    size_t ll_bytes;
    size_t footprint;
};

// HBM footprint of a request: input span + output span + workspace part.
inline size_t footprint_of(const Item &it)
{
    return (size_t)(it.src_hi - it.src_lo) + (size_t)(it.dst_hi - it.dst_lo) + it.ll_bytes;
}

// Workspace of one direction's batched call: tables + the images' own parts.
struct Group {
    int count = 0, lmax = 0;
    size_t ll = 0;
};

template <typename Table>
size_t group_bytes(const Group &g, Table table)
{
    return g.count ? table(g.count, g.lmax) + g.ll : 0;
}

// The next batch: the longest prefix of the pending items, in submission
// order and of at most max_batch items, in which no item reads or writes a
// range that an earlier item of the prefix writes, nor writes a range that an
// earlier item reads (such an item must run after the batch), whose two
// direction groups fit one free block of the arena together, and whose
// footprints sum to at most `budget` bytes (the footprint cap less what the
// batches in flight hold).  item(i) gives the i-th pending item;
// table(count, lmax) the table bytes of a batched call.  Writes the groups
// and the batch's footprint and returns the prefix length (0: the first item
// does not fit the free arena or the budget).
template <typename ItemAt, typename Table>
size_t next_batch(ItemAt item, size_t pending, int max_batch, const Arena &arena, size_t budget,
                  Table table, Group g[2], size_t *footprint)
{
    g[0] = g[1] = Group{};
    *footprint = 0;
    RangeSet written, read;
    size_t n = 0;
    for (; n < pending && (long long)n < max_batch; n++) {
        const Item it = item(n);
        if (written.overlaps(it.src_lo, it.src_hi) || written.overlaps(it.dst_lo, it.dst_hi) ||
            read.overlaps(it.dst_lo, it.dst_hi))
            break;
        if (it.footprint > budget - *footprint) break;
        Group t[2] = {g[0], g[1]};
        Group &k = t[it.inverse ? 1 : 0];
        k.count++;
        k.lmax = std::max(k.lmax, it.levels);
        k.ll += it.ll_bytes;
        if (!arena.fits(group_bytes(t[0], table) + group_bytes(t[1], table))) break;
        g[0] = t[0];
        g[1] = t[1];
        *footprint += it.footprint;
        written.insert(it.dst_lo, it.dst_hi);
        read.insert(it.src_lo, it.src_hi);
    }
    return n;
}

}  // namespace serve
}  // namespace dwt2
