// First-fit device-memory arena over segments added on demand, bounded by a
// byte budget.  It manages offsets only: segment memory is obtained through
// the caller's grow callback, so this header has no device dependency (and is
// exercised on the host by the test suite).
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace rsf {

class Arena {
public:
    struct Block {
        int seg = -1;
        size_t off = 0, len = 0;
    };

    // budget: most bytes ever reserved; segment: default segment size;
    // align: every block offset and length is a multiple of it (a power of 2).
    Arena(size_t budget, size_t segment, size_t align)
        : budget_(budget), seg_(segment), align_(align) {}

    size_t round(size_t n) const { return (n + align_ - 1) & ~(align_ - 1); }

    // Reserve n bytes.  grow(len) must provide a new segment of len bytes
    // and return false if it cannot; it is called only when no free range
    // fits and the budget allows another segment.
    template <class Grow>
    bool alloc(size_t n, Block &out, Grow &&grow)
    {
        if (n == 0) n = 1;
        n = round(n);
        for (int s = 0; s < (int)free_.size(); ++s)
            if (take(s, n, out)) return true;
        size_t len = seg_ > n ? seg_ : n;
        if (reserved_ + len > budget_) len = budget_ - reserved_;
        len &= ~(align_ - 1);
        if (len < n || !grow(len)) return false;
        free_.emplace_back();
        free_.back()[0] = len;
        seg_len_.push_back(len);
        reserved_ += len;
        return take((int)free_.size() - 1, n, out);
    }

    // Return a block; adjacent free ranges merge.
    void release(const Block &b)
    {
        if (b.seg < 0 || b.len == 0) return;
        auto &fl = free_[b.seg];
        auto it = fl.emplace(b.off, b.len).first;
        if (it != fl.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                fl.erase(it);
                it = prev;
            }
        }
        auto next = std::next(it);
        if (next != fl.end() && it->first + it->second == next->first) {
            it->second += next->second;
            fl.erase(next);
        }
        used_ -= b.len;
    }

    size_t in_use() const { return used_; }
    size_t peak() const { return peak_; }
    size_t reserved() const { return reserved_; }
    size_t budget() const { return budget_; }
    int segments() const { return (int)seg_len_.size(); }
    size_t segment_bytes(int s) const { return seg_len_[s]; }
    // Largest free range of segment s (for checks).
    size_t largest_free(int s) const
    {
        size_t m = 0;
        for (const auto &kv : free_[s]) m = kv.second > m ? kv.second : m;
        return m;
    }

private:
    bool take(int s, size_t n, Block &out)
    {
        auto &fl = free_[s];
        for (auto it = fl.begin(); it != fl.end(); ++it) {
            if (it->second < n) continue;
            out.seg = s;
            out.off = it->first;
            out.len = n;
            const size_t rest = it->second - n, at = it->first + n;
            fl.erase(it);
            if (rest) fl[at] = rest;
            used_ += n;
            if (used_ > peak_) peak_ = used_;
            return true;
        }
        return false;
    }

    size_t budget_, seg_, align_;
    std::vector<size_t> seg_len_;
    std::vector<std::map<size_t, size_t>> free_;   // per segment: offset -> length
    size_t used_ = 0, peak_ = 0, reserved_ = 0;
};

}  // namespace rsf
