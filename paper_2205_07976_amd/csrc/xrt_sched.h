// xrt_sched.h -- the shot server's scheduling logic, free of any device code:
// arena allocation, admission in arrival order by HBM footprint and resident
// slots, chunking of each shot's work, the order chunks are published in, and
// the bookkeeping that turns finished chunks into finished phases and shots.
// xrt_server.cpp drives it against the GPU (descriptors in pinned memory, a
// ring of chunk records, done flags written by the persistent kernel); the
// CPU tests drive it against a simulated device.  Not part of the public ABI.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

namespace xrt {
namespace sched {

constexpr uint64_t ALIGN = 256;
constexpr int TILE_PIXELS = 256;            // 16 x 16 pixels per tile
constexpr uint64_t CHUNK_TERMS = 1u << 20;  // pixel-terms a compute chunk aims at
constexpr int MAX_CHUNK = 64;               // work units per chunk
enum { PHASE_COMPUTE = 0, PHASE_REDUCE = 1, PHASE_BACKGROUND = 2 };
enum { POLICY_FAIR_SHARE = 0, POLICY_SHORTEST_REMAINING = 1 };
enum { QUEUED = 0, RUNNING = 1, DONE = 2 };

inline uint64_t align_up(uint64_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// Default pixel-terms of one segment of a unit's sums (two standard chunks,
// ~4 ms of a workgroup).  Measured on the served stream against 2^22 and
// 2^20: 8-13 % lower median latency than 2^22 at the same capacity; 2^20
// lowered it a little more at 0.8 x capacity but cost 1.6 % of capacity.
constexpr uint64_t SEGMENT_TERMS = 2 * CHUNK_TERMS;

// Segments of each work unit's outer iterations: a unit (a tile's sums, or
// one part of split sums) heavier than segment_terms pixel-terms runs as K
// consecutive segments of about equal length, the smallest K that keeps each
// below segment_terms, at most the shortest part's outer-iteration count (so
// no segment is empty).  A single tile-sized chunk otherwise holds its
// workgroup for up to ~0.1 s (a tile of 2.4e5 terms per pixel), and a shot
// that arrives meanwhile waits for workgroups to come free.
inline int32_t segments_of(uint64_t terms_per_pixel, int32_t split, int64_t n_outer, uint64_t segment_terms)
{
    if (split < 1 || n_outer < 1 || segment_terms < 1) return 1;
    const uint64_t per_unit = TILE_PIXELS * (terms_per_pixel / (uint64_t)split);
    uint64_t k = (per_unit + segment_terms - 1) / segment_terms;
    const uint64_t q_min = (uint64_t)(n_outer / split);
    k = std::min<uint64_t>({k, std::max<uint64_t>(q_min, 1), (uint64_t)1 << 20});
    return (int32_t)std::max<uint64_t>(k, 1);
}

// First-fit allocator over [0, size) with coalescing of freed neighbours.
class Arena {
  public:
    explicit Arena(uint64_t size) : size_(size) { free_[0] = size; }
    bool alloc(uint64_t n, uint64_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        if (n == 0) return;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }
    const std::map<uint64_t, uint64_t> &free_blocks() const { return free_; }

  private:
    uint64_t size_;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
};

// What the scheduler knows of a shot.  The caller fills the first block at
// submission; the scheduler owns the rest.
struct Work {
    uint64_t ticket = 0;
    uint64_t footprint = 0;        // device arena bytes (image, part sums, segment state)
    uint64_t desc_bytes = 0;       // host arena bytes (descriptor and tables)
    int32_t n_tiles = 0;           // 16 x 16 tiles of the region
    int32_t split = 1;             // parts per pixel sum (1: whole sums)
    int32_t n_seg = 1;             // consecutive segments of each unit's outer iterations
    uint64_t terms_per_pixel = 0;
    uint64_t bg_terms_per_pixel = 0;  // > 0: a background phase over the tiles
                                      // once the image is complete
    // owned by the scheduler
    int state = QUEUED;
    uint64_t dev_off = 0, host_off = 0;
    // current phase: PHASE_COMPUTE over units tile * split + part, then, for
    // split sums, PHASE_REDUCE over tiles once every part is done, then, with
    // a background, PHASE_BACKGROUND over tiles once the image is complete
    int32_t phase = PHASE_COMPUTE;
    int32_t n_units = 0, chunk_units = 1, next_unit = 0;
    int64_t chunks_total = 0, chunks_done = 0;
    // PHASE_COMPUTE with segments: chunks whose units finished segment k and
    // may run segment k + 1 (unit0, n_units, k + 1), published in that order
    // once every unit has started (the units with the most segments left go
    // first, so the phase ends with short chains, not with a few long ones)
    struct Ready {
        int32_t unit0, n_units, seg;
    };
    std::deque<Ready> ready;
    bool listed = false;           // in the scheduler's list of shots with work to publish
    double work_published = 0;     // fair share: the shot's level (its start level plus
                                   // the pixel-terms of its chunks published since)
    double work_left = 0;          // pixel-terms of every phase not yet published
};

// One published chunk: units [unit0, unit0 + n_units) of a shot's phase
// (and, for PHASE_COMPUTE, segment seg of their outer iterations).
struct Chunk {
    uint64_t seq;                  // publication number
    uint64_t ticket;
    int32_t kind;                  // PHASE_COMPUTE, PHASE_REDUCE or PHASE_BACKGROUND
    int32_t unit0, n_units;
    int32_t seg;
};

class Scheduler {
  public:
    // dev_bytes / host_bytes: arena sizes; n_wg: workgroups of the persistent
    // kernel (chunk sizing and the publication depth); ring: capacity of the
    // ring of chunk records.
    Scheduler(uint64_t dev_bytes, uint64_t host_bytes, int max_resident, int n_wg, uint32_t ring,
              int policy = POLICY_FAIR_SHARE)
        : dev_(dev_bytes), host_(host_bytes), max_resident_(max_resident), n_wg_(std::max(n_wg, 1)),
          depth_(std::min<size_t>(ring - 1, 2 * (size_t)std::max(n_wg, 1))), ring_(ring),
          slack_(0.5 * (double)std::max(n_wg, 1) * (double)CHUNK_TERMS), policy_(policy)
    {
    }

    // Queue a shot (footprint, desc_bytes, n_tiles, split, terms_per_pixel set).
    void submit(const Work &w)
    {
        Work &x = work_[w.ticket] = w;
        x.state = QUEUED;
        queue_.push_back(w.ticket);
    }

    // Admission in arrival order: while the head of the queue fits both arenas
    // and a resident slot is free, allocate its space, call
    // prepare(work) -> int (0: admitted; else the error, the space is freed
    // and admission stops) and start its first phase.  A head that does not
    // fit blocks the ones behind it (no overtaking).  Returns 0 or the error.
    template <class Prepare>
    int admit(Prepare prepare)
    {
        while (!queue_.empty() && resident_ < (uint64_t)max_resident_) {
            Work &w = work_[queue_.front()];
            uint64_t doff = 0, hoff = 0;
            if (!dev_.alloc(w.footprint, &doff)) break;
            if (!host_.alloc(w.desc_bytes, &hoff)) {
                dev_.release(doff, w.footprint);
                break;
            }
            w.dev_off = doff;
            w.host_off = hoff;
            const int st = prepare(w);
            if (st) {
                dev_.release(doff, w.footprint);
                host_.release(hoff, w.desc_bytes);
                return st;
            }
            w.state = RUNNING;
            start_phase(w, PHASE_COMPUTE);
            w.work_published = vtime_;  // it competes from now on, not from the start
            w.work_left = (double)w.n_tiles * TILE_PIXELS *
                          ((double)w.terms_per_pixel + (w.split > 1 ? (double)w.split : 0.0) +
                           (double)w.bg_terms_per_pixel);
            resident_++;
            list(w);
            queue_.pop_front();
        }
        return 0;
    }

    // Publication while fewer than `depth` chunks are in flight, the new
    // sequence number stays within `ring` of the oldest chunk still in flight
    // (records and done flags live at seq % ring: a slow chunk must not share
    // its slot with a later one), and the chunks waiting for a workgroup hold
    // less than `slack` pixel-terms (half a standard chunk per workgroup,
    // ~1 ms of the device: enough that no workgroup waits for the host
    // between two progress calls of a request loop that calls it often, few
    // enough that a chunk published now, which goes to the back of that
    // queue, is not held back long; with one or two per workgroup the
    // latency of served shots was up to 7 % or 15 % higher at the median and
    // up to 30 % or 2x higher in slowdown at p99, at the same capacity).  Workgroups claim chunks in publication order, so the
    // waiting ones are taken to be the in-flight chunks after the oldest
    // n_wg.  The next chunk comes, under POLICY_FAIR_SHARE, from the
    // admitted shot with the least work published so far (pixel-terms), so
    // resident shots share the device evenly by work whatever their chunk
    // sizes and a shot admitted later joins at the current level; under
    // POLICY_SHORTEST_REMAINING, from the admitted shot with the least work
    // left to publish, so a small shot overtakes the large ones in flight.
    // Ties go to the earlier ticket.  emit(const Chunk &, Work &) writes the
    // record.  Returns the number of chunks published.
    template <class Emit>
    size_t publish(Emit emit)
    {
        size_t n = 0;
        // inflight_ is in publication order: its front is the oldest chunk
        double waiting = 0;
        for (size_t i = (size_t)n_wg_; i < inflight_.size(); ++i) waiting += inflight_[i].work;
        while (inflight_.size() < depth_ && !admitted_.empty() &&
               (inflight_.empty() || tail_ - inflight_.front().seq < ring_) &&
               (inflight_.size() < (size_t)n_wg_ || waiting < slack_)) {
            size_t best = 0;
            for (size_t i = 1; i < admitted_.size(); ++i) {
                const Work &a = work_[admitted_[i]], &b = work_[admitted_[best]];
                const double ka = policy_ == POLICY_SHORTEST_REMAINING ? a.work_left : a.work_published;
                const double kb = policy_ == POLICY_SHORTEST_REMAINING ? b.work_left : b.work_published;
                if (ka < kb || (ka == kb && a.ticket < b.ticket)) best = i;
            }
            Work &w = work_[admitted_[best]];
            vtime_ = w.work_published;
            Chunk c;
            c.seq = tail_++;
            c.ticket = w.ticket;
            c.kind = w.phase;
            if (w.next_unit < w.n_units) {
                c.seg = 0;
                c.unit0 = w.next_unit;
                c.n_units = std::min(w.chunk_units, w.n_units - w.next_unit);
                w.next_unit += c.n_units;
            } else {  // a later segment of units whose last one is done
                c.unit0 = w.ready.front().unit0;
                c.n_units = w.ready.front().n_units;
                c.seg = w.ready.front().seg;
                w.ready.pop_front();
            }
            // a reduce chunk reads K values per pixel: count it as K terms
            const double cw = (double)c.n_units * TILE_PIXELS *
                              (w.phase == PHASE_COMPUTE  ? (double)w.terms_per_pixel / w.split / w.n_seg
                               : w.phase == PHASE_REDUCE ? (double)w.split
                                                         : (double)w.bg_terms_per_pixel);
            w.work_published += cw;
            w.work_left -= cw;
            inflight_.push_back({c.seq, c.ticket, cw, c.kind, c.unit0, c.n_units, c.seg});
            if (inflight_.size() > (size_t)n_wg_) waiting += cw;
            emit(c, w);
            ++n;
            if (w.next_unit >= w.n_units && w.ready.empty()) {
                w.listed = false;
                admitted_.erase(admitted_.begin() + best);
            }
        }
        return n;
    }

    // Finished chunks: is_done(seq) says whether chunk `seq` is done.  A
    // compute chunk of segment k < n_seg - 1 makes its units ready for
    // segment k + 1 (their running sums are in the arena); a compute phase
    // whose every unit finished its last segment starts, for split sums, the
    // reduce phase;
    // the phase that completes the image starts the background phase of a
    // shot that has one; any other completed phase finishes the shot, whose
    // ticket is appended to *finished.
    template <class IsDone>
    void collect(IsDone is_done, std::vector<uint64_t> *finished)
    {
        size_t k = 0;
        for (size_t i = 0; i < inflight_.size(); ++i) {
            const InFlight f = inflight_[i];
            if (!is_done(f.seq)) {
                inflight_[k++] = f;
                continue;
            }
            Work &w = work_[f.ticket];
            if (f.kind == PHASE_COMPUTE && f.seg + 1 < w.n_seg) {
                w.ready.push_back({f.unit0, f.n_units, f.seg + 1});
                list(w);
            }
            if (++w.chunks_done == w.chunks_total) {
                if (w.phase == PHASE_COMPUTE && w.split > 1) {
                    start_phase(w, PHASE_REDUCE);  // every part sum is in the arena
                    list(w);
                } else if (w.phase != PHASE_BACKGROUND && w.bg_terms_per_pixel > 0) {
                    start_phase(w, PHASE_BACKGROUND);  // the image is complete
                    list(w);
                } else {
                    w.state = DONE;
                    if (finished) finished->push_back(w.ticket);
                }
            }
        }
        inflight_.resize(k);
    }

    // Withdraw a shot that is still queued (it holds no space and no chunk
    // of it exists).  Returns false if the shot is unknown or was admitted.
    bool cancel(uint64_t ticket)
    {
        auto it = work_.find(ticket);
        if (it == work_.end() || it->second.state != QUEUED) return false;
        queue_.erase(std::find(queue_.begin(), queue_.end(), ticket));
        work_.erase(it);
        return true;
    }

    // Forget a finished shot and free its space.  Returns false if the shot
    // is unknown or not done.
    bool release(uint64_t ticket)
    {
        auto it = work_.find(ticket);
        if (it == work_.end() || it->second.state != DONE) return false;
        dev_.release(it->second.dev_off, it->second.footprint);
        host_.release(it->second.host_off, it->second.desc_bytes);
        resident_--;
        work_.erase(it);
        return true;
    }

    const Work *find(uint64_t ticket) const
    {
        auto it = work_.find(ticket);
        return it == work_.end() ? nullptr : &it->second;
    }
    size_t in_flight() const { return inflight_.size(); }
    size_t depth() const { return depth_; }
    int policy() const { return policy_; }
    double slack() const { return slack_; }
    // pixel-terms of the in-flight chunks after the oldest n_wg
    double waiting_work() const
    {
        double x = 0;
        for (size_t i = (size_t)n_wg_; i < inflight_.size(); ++i) x += inflight_[i].work;
        return x;
    }
    uint64_t resident() const { return resident_; }
    uint64_t published() const { return tail_; }
    const Arena &dev_arena() const { return dev_; }
    const Arena &host_arena() const { return host_; }

  private:
    struct InFlight {
        uint64_t seq, ticket;
        double work;  // pixel-terms
        int32_t kind, unit0, n_units, seg;
    };

    // Into the list of shots with work to publish (once).
    void list(Work &w)
    {
        if (!w.listed) {
            w.listed = true;
            admitted_.push_back(w.ticket);
        }
    }

    // Chunking of a phase: compute and background chunks hold about
    // CHUNK_TERMS pixel-terms (a few ms of one workgroup, so a shot admitted
    // later waits at most that long for a workgroup, and the last chunks of a
    // shot end close together) and no more units than spread the phase over
    // every workgroup; reduce chunks (K loads per pixel) are spread the same
    // way.
    void start_phase(Work &w, int32_t phase)
    {
        w.phase = phase;
        w.n_units = phase == PHASE_COMPUTE ? w.n_tiles * w.split : w.n_tiles;
        const uint64_t by_spread = ((uint64_t)w.n_units + n_wg_ - 1) / n_wg_;
        uint64_t by_cost = (uint64_t)MAX_CHUNK;
        if (phase != PHASE_REDUCE) {
            const uint64_t tpp = phase == PHASE_COMPUTE ? w.terms_per_pixel / (uint64_t)w.split / (uint64_t)w.n_seg
                                                        : w.bg_terms_per_pixel;
            const uint64_t per_unit = std::max<uint64_t>(1, TILE_PIXELS * tpp);
            by_cost = std::max<uint64_t>(1, CHUNK_TERMS / per_unit);
        }
        w.chunk_units = (int32_t)std::max<uint64_t>(1, std::min<uint64_t>({by_cost, by_spread, (uint64_t)MAX_CHUNK}));
        w.next_unit = 0;
        // segments: every chunk's units run each segment once, in order
        w.chunks_total = (int64_t)((w.n_units + w.chunk_units - 1) / w.chunk_units) *
                         (phase == PHASE_COMPUTE ? std::max(w.n_seg, 1) : 1);
        w.chunks_done = 0;
        w.ready.clear();
    }

    Arena dev_, host_;
    int max_resident_;
    int n_wg_;
    size_t depth_;
    uint64_t ring_;
    double slack_;  // pixel-terms allowed in chunks that wait for a workgroup
    int policy_;
    uint64_t resident_ = 0, tail_ = 0;
    double vtime_ = 0;  // published work of the shot served last
    std::deque<uint64_t> queue_;         // submitted, not admitted (FIFO)
    std::vector<uint64_t> admitted_;     // admitted, with units of the current phase left to publish
    std::vector<InFlight> inflight_;     // published, not done
    std::unordered_map<uint64_t, Work> work_;
};

}  // namespace sched
}  // namespace xrt
