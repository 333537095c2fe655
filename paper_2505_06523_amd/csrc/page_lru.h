// Page replacement of a streamed scene: which clusters a cut pages in and
// which resident clusters give up their pages (host logic, no device calls).
//
// The pool has n_pages pages; a page holds one cluster.  Pages form a list in
// order of last use (head: most recent).  Planning a cut (the clusters that
// have slots in it, repeats allowed) opens a new paging frame:
// - a resident cluster of the cut moves its page to the head;
// - a missing one takes the page at the tail, the least recently used, which
//   is never a page of this cut (those were all moved to the head first);
//   the cluster that held it, if any, is evicted;
// - when the cut needs more clusters than the pool holds, nothing is assigned
//   and plan() returns false (the pages the cut touched stay at the head).
// Every page carries the frame of its last use; max_evicted_stamp is the
// latest such frame among evicted pages, so a selection planned in frame f is
// intact while f > max_evicted_stamp.
#pragma once

#include <cstdint>
#include <vector>

namespace v3dg {

class PageLRU {
public:
    static constexpr uint32_t kNone = 0xffffffffu;

    void init(uint32_t n_clusters, uint32_t n_pages)
    {
        page_of_.assign(n_clusters, kNone);
        miss_stamp_.assign(n_clusters, 0);
        cluster_of_.assign(n_pages, kNone);
        stamp_.assign(n_pages, 0);
        prev_.assign(n_pages, kNone);
        next_.assign(n_pages, kNone);
        head_ = tail_ = kNone;
        for (uint32_t p = 0; p < n_pages; ++p) push_front(p);
        frame = max_evicted_stamp = evictions = 0;
    }

    // Plans the cut ks[0 .. n): on success miss holds the clusters to page in
    // (first-seen order), each already assigned its page, and touched the
    // resident clusters the cut uses.
    bool plan(const uint32_t *ks, size_t n, std::vector<uint32_t> &miss, uint32_t &touched)
    {
        const uint64_t f = ++frame;
        miss.clear();
        touched = 0;
        for (size_t i = 0; i < n; ++i) {
            const uint32_t k = ks[i];
            const uint32_t p = page_of_[k];
            if (p != kNone) {
                if (stamp_[p] != f) {
                    stamp_[p] = f;
                    unlink(p);
                    push_front(p);
                    ++touched;
                }
            } else if (miss_stamp_[k] != f) {
                miss_stamp_[k] = f;
                miss.push_back(k);
            }
        }
        if ((uint64_t)touched + miss.size() > cluster_of_.size()) {
            miss.clear();
            return false;
        }
        for (uint32_t k : miss) {
            const uint32_t p = tail_;
            const uint32_t old = cluster_of_[p];
            if (old != kNone) {
                page_of_[old] = kNone;
                if (stamp_[p] > max_evicted_stamp) max_evicted_stamp = stamp_[p];
                ++evictions;
            }
            cluster_of_[p] = k;
            page_of_[k] = p;
            stamp_[p] = f;
            unlink(p);
            push_front(p);
        }
        return true;
    }

    // Gives up the page of cluster k (its contents never arrived); the free
    // page goes to the tail, so that the next miss takes it first.
    void release(uint32_t k)
    {
        const uint32_t p = page_of_[k];
        if (p == kNone) return;
        cluster_of_[p] = kNone;
        page_of_[k] = kNone;
        unlink(p);
        push_back(p);
    }

    uint32_t page_of(uint32_t k) const { return page_of_[k]; }
    uint32_t cluster_of(uint32_t p) const { return cluster_of_[p]; }
    uint32_t n_pages() const { return (uint32_t)cluster_of_.size(); }
    uint32_t resident() const
    {
        uint32_t r = 0;
        for (uint32_t c : cluster_of_) r += c != kNone ? 1u : 0u;
        return r;
    }

    uint64_t frame = 0, max_evicted_stamp = 0, evictions = 0;

private:
    void unlink(uint32_t p)
    {
        const uint32_t a = prev_[p], b = next_[p];
        if (a != kNone) next_[a] = b;
        else head_ = b;
        if (b != kNone) prev_[b] = a;
        else tail_ = a;
        prev_[p] = next_[p] = kNone;
    }
    void push_back(uint32_t p)
    {
        next_[p] = kNone;
        prev_[p] = tail_;
        if (tail_ != kNone) next_[tail_] = p;
        tail_ = p;
        if (head_ == kNone) head_ = p;
    }
    void push_front(uint32_t p)
    {
        prev_[p] = kNone;
        next_[p] = head_;
        if (head_ != kNone) prev_[head_] = p;
        head_ = p;
        if (tail_ == kNone) tail_ = p;
    }

    std::vector<uint32_t> page_of_, cluster_of_, prev_, next_;
    std::vector<uint64_t> stamp_, miss_stamp_;
    uint32_t head_ = kNone, tail_ = kNone;
};

}  // namespace v3dg
