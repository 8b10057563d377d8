// CPU checks of the shot server's scheduling logic (paper_2205_07976_amd/
// csrc/xrt_sched.h) against a simulated device: chunks are "run" by marking
// them done, in publication order or scrambled.  Each check prints its name;
// the first failure prints the condition and exits with status 1.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "../paper_2205_07976_amd/csrc/xrt_sched.h"

using namespace xrt::sched;

#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                              \
        }                                                                         \
    } while (0)

static Work shot(uint64_t ticket, uint64_t footprint, int32_t n_tiles, uint64_t tpp, int32_t split = 1,
                 uint64_t desc = 4096, uint64_t bg_tpp = 0, int32_t n_seg = 1)
{
    Work w;
    w.n_seg = n_seg;
    w.bg_terms_per_pixel = bg_tpp;
    w.ticket = ticket;
    w.footprint = footprint;
    w.desc_bytes = desc;
    w.n_tiles = n_tiles;
    w.terms_per_pixel = tpp;
    w.split = split;
    return w;
}

// A simulated device: published chunks wait in `pending`; run(n) finishes n
// of them (the oldest, or random ones), collect() hands the finished ones to
// the scheduler.
struct Device {
    Scheduler &s;
    std::vector<Chunk> pending;
    std::set<uint64_t> done;
    std::vector<Chunk> log;  // every chunk ever published
    std::mt19937_64 rng{7};
    explicit Device(Scheduler &sc) : s(sc) {}
    size_t publish()
    {
        return s.publish([&](const Chunk &c, const Work &) {
            // a reduce chunk comes only after every compute chunk of its shot
            // is done, a background chunk only after every compute and reduce
            // chunk
            // a compute chunk of segment k only after every compute chunk of
            // an earlier segment over any of its units is done;
            if (c.kind == PHASE_COMPUTE)
                for (const Chunk &x : log)
                    if (x.ticket == c.ticket && x.kind == PHASE_COMPUTE && x.seg < c.seg &&
                        x.unit0 < c.unit0 + c.n_units && c.unit0 < x.unit0 + x.n_units)
                        CHECK(done.count(x.seq));
            if (c.kind == PHASE_REDUCE)
                for (const Chunk &x : log)
                    if (x.ticket == c.ticket && x.kind == PHASE_COMPUTE) CHECK(done.count(x.seq));
            if (c.kind == PHASE_BACKGROUND)
                for (const Chunk &x : log)
                    if (x.ticket == c.ticket && x.kind != PHASE_BACKGROUND) CHECK(done.count(x.seq));
            pending.push_back(c);
            log.push_back(c);
        });
    }
    void run(size_t n, bool scrambled)
    {
        for (size_t i = 0; i < n && !pending.empty(); ++i) {
            size_t k = scrambled ? rng() % pending.size() : 0;
            done.insert(pending[k].seq);
            pending.erase(pending.begin() + k);
        }
    }
    std::vector<uint64_t> collect()
    {
        std::vector<uint64_t> fin;
        s.collect([&](uint64_t seq) { return done.count(seq) > 0; }, &fin);
        return fin;
    }
};

static void check_arena()
{
    printf("arena: first fit, coalescing, no overlap under random use\n");
    Arena a(1000);
    uint64_t o1, o2, o3, o4;
    CHECK(a.alloc(100, &o1) && o1 == 0);
    CHECK(a.alloc(200, &o2) && o2 == 100);
    CHECK(a.alloc(300, &o3) && o3 == 300);
    CHECK(!a.alloc(401, &o4));
    a.release(o2, 200);
    CHECK(a.alloc(150, &o4) && o4 == 100);  // first fit reuses the hole
    a.release(o4, 150);
    a.release(o1, 100);
    a.release(o3, 300);
    CHECK(a.free_blocks().size() == 1 && a.free_blocks().begin()->second == 1000);
    std::mt19937_64 rng(3);
    std::map<uint64_t, uint64_t> live;  // offset -> length
    Arena b(1 << 20);
    for (int it = 0; it < 20000; ++it) {
        if (!live.empty() && (rng() % 3 == 0 || live.size() > 200)) {
            auto p = live.begin();
            std::advance(p, rng() % live.size());
            b.release(p->first, p->second);
            live.erase(p);
        } else {
            uint64_t n = 1 + rng() % 20000, off;
            if (b.alloc(n, &off)) {
                CHECK(off + n <= b.size());
                auto nx = live.lower_bound(off);
                CHECK(nx == live.end() || off + n <= nx->first);
                if (nx != live.begin()) {
                    auto pv = std::prev(nx);
                    CHECK(pv->first + pv->second <= off);
                }
                live[off] = n;
            }
        }
        // free + live = everything, free blocks disjoint and coalesced
        uint64_t total = 0, end = 0;
        bool first = true;
        for (auto &f : b.free_blocks()) {
            CHECK(first || f.first > end);  // strictly after the previous block: coalesced
            total += f.second;
            end = f.first + f.second;
            first = false;
        }
        for (auto &l : live) total += l.second;
        CHECK(total == b.size());
    }
}

static void check_fifo_admission()
{
    printf("admission: arrival order, no overtaking, HBM budget and slots\n");
    Scheduler s(1000, 1 << 20, 3, 4, 1 << 16);
    Device d(s);
    s.submit(shot(1, 600, 4, 1000));
    s.submit(shot(2, 600, 4, 1000));  // does not fit beside 1
    s.submit(shot(3, 100, 4, 1000));  // would fit, but must not overtake 2
    CHECK(s.admit([](Work &) { return 0; }) == 0);
    CHECK(s.find(1)->state == RUNNING && s.find(2)->state == QUEUED && s.find(3)->state == QUEUED);
    // run shot 1 to completion
    for (int i = 0; i < 100 && s.find(1)->state != DONE; ++i) {
        d.publish();
        d.run(100, false);
        d.collect();
    }
    CHECK(s.find(1)->state == DONE);
    s.admit([](Work &) { return 0; });
    CHECK(s.find(2)->state == QUEUED);  // memory of 1 not yet released
    CHECK(s.release(1));
    s.admit([](Work &) { return 0; });
    CHECK(s.find(2)->state == RUNNING && s.find(3)->state == RUNNING);
    // the resident-slot limit
    Scheduler t(1 << 30, 1 << 20, 2, 4, 1 << 16);
    for (uint64_t k = 1; k <= 5; ++k) t.submit(shot(k, 100, 4, 1000));
    t.admit([](Work &) { return 0; });
    CHECK(t.resident() == 2 && t.find(3)->state == QUEUED);
    // a failing preparation frees the space and stops admission
    Scheduler u(1000, 1 << 20, 8, 4, 1 << 16);
    u.submit(shot(1, 500, 4, 1000));
    u.submit(shot(2, 500, 4, 1000));
    CHECK(u.admit([](Work &w) { return w.ticket == 1 ? -7 : 0; }) == -7);
    CHECK(u.find(1)->state == QUEUED && u.resident() == 0);
    CHECK(u.dev_arena().free_blocks().begin()->second == 1000);
}

static void check_units_and_depth()
{
    printf("chunks: every unit of every phase (and segment) exactly once, depth bound, phases in order\n");
    Scheduler s(1 << 30, 1 << 22, 64, 16, 1 << 16);
    Device d(s);
    std::map<uint64_t, Work> shots;
    std::mt19937_64 rng(11);
    for (uint64_t k = 1; k <= 40; ++k) {
        const int32_t tiles = 1 + (int32_t)(rng() % 300);
        const uint64_t tpp = 1 + rng() % 200000;
        const int32_t split = (rng() % 3 == 0) ? 1 + (int32_t)(rng() % 64) : 1;
        const uint64_t bg = (rng() % 2 == 0) ? 1 + rng() % 2000 : 0;
        const int32_t n_seg = (rng() % 3 == 0) ? 1 + (int32_t)(rng() % 7) : 1;
        shots[k] = shot(k, 4096, tiles, tpp, split, 4096, bg, n_seg);
        s.submit(shots[k]);
    }
    std::map<uint64_t, int> finished;
    for (int it = 0; it < 100000 && finished.size() < shots.size(); ++it) {
        s.admit([](Work &) { return 0; });
        d.publish();
        CHECK(s.in_flight() <= s.depth() && s.depth() == 32);
        d.run(1 + rng() % 40, true);
        for (uint64_t t : d.collect()) finished[t]++;
    }
    CHECK(finished.size() == shots.size());
    for (auto &f : finished) CHECK(f.second == 1);
    // coverage per (shot, phase); compute units once per segment, each
    // unit's segments in order
    std::map<std::pair<uint64_t, int>, std::vector<int>> cover;
    std::map<uint64_t, std::vector<int>> next_seg;  // per shot and compute unit
    std::map<uint64_t, uint64_t> last_compute, first_reduce, last_sums, first_bg;
    for (const Chunk &c : d.log) {
        auto &v = cover[{c.ticket, c.kind}];
        const Work &w = shots[c.ticket];
        const int n = c.kind == PHASE_COMPUTE ? w.n_tiles * w.split : w.n_tiles;
        if (c.kind != PHASE_BACKGROUND) last_sums[c.ticket] = std::max(last_sums[c.ticket], c.seq);
        if (c.kind == PHASE_BACKGROUND && !first_bg.count(c.ticket)) first_bg[c.ticket] = c.seq;
        if (v.empty()) v.assign(n, 0);
        CHECK(c.n_units >= 1 && c.n_units <= MAX_CHUNK && c.unit0 >= 0 && c.unit0 + c.n_units <= n);
        for (int u = c.unit0; u < c.unit0 + c.n_units; ++u) v[u]++;
        if (c.kind == PHASE_COMPUTE) {
            auto &ns = next_seg[c.ticket];
            if (ns.empty()) ns.assign(n, 0);
            CHECK(c.seg >= 0 && c.seg < w.n_seg);
            for (int u = c.unit0; u < c.unit0 + c.n_units; ++u) CHECK(ns[u]++ == c.seg);
        } else {
            CHECK(c.seg == 0);
        }
        if (c.kind == PHASE_COMPUTE) last_compute[c.ticket] = std::max(last_compute[c.ticket], c.seq);
        if (c.kind == PHASE_REDUCE && !first_reduce.count(c.ticket)) first_reduce[c.ticket] = c.seq;
    }
    for (auto &kv : shots) {
        const Work &w = kv.second;
        for (int x : cover[{w.ticket, PHASE_COMPUTE}]) CHECK(x == w.n_seg);
        for (int x : next_seg[w.ticket]) CHECK(x == w.n_seg);
        CHECK(std::abs(s.find(w.ticket)->work_left) < 1.0);
        if (w.split > 1) {
            CHECK(cover.count({w.ticket, PHASE_REDUCE}));
            for (int x : cover[{w.ticket, PHASE_REDUCE}]) CHECK(x == 1);
            CHECK(first_reduce[w.ticket] > last_compute[w.ticket]);
        } else {
            CHECK(!cover.count({w.ticket, PHASE_REDUCE}));
        }
        if (w.bg_terms_per_pixel > 0) {
            CHECK(cover.count({w.ticket, PHASE_BACKGROUND}));
            for (int x : cover[{w.ticket, PHASE_BACKGROUND}]) CHECK(x == 1);
            CHECK(first_bg[w.ticket] > last_sums[w.ticket]);
        } else {
            CHECK(!cover.count({w.ticket, PHASE_BACKGROUND}));
        }
    }
    for (auto &kv : shots) CHECK(s.release(kv.first));
    CHECK(s.dev_arena().free_blocks().size() == 1 && s.resident() == 0);
}

static void check_fair_share()
{
    printf("publication: backlogged shots share by work, a late shot joins at the current level\n");
    // shot 1: cheap units (tpp 1000: 64 tiles per chunk); shot 2: costly
    // units (tpp 100000: 1 tile per chunk)
    Scheduler s(1 << 30, 1 << 22, 8, 4, 1 << 16);
    Device d(s);
    s.submit(shot(1, 4096, 100000, 1000));
    s.submit(shot(2, 4096, 100000, 100000));
    s.admit([](Work &) { return 0; });
    double max_chunk = 0;
    for (int it = 0; it < 2000; ++it) {
        d.publish();
        d.run(8, false);
        d.collect();
        const double a = s.find(1)->work_published, b = s.find(2)->work_published;
        max_chunk = std::max(max_chunk, 256.0 * 100000);
        CHECK(std::abs(a - b) <= max_chunk + 1);  // within one chunk of each other
    }
    // a third shot arriving now starts at the current level: it does not get
    // the device alone until it catches up with the others
    s.submit(shot(3, 4096, 100000, 100000));
    s.admit([](Work &) { return 0; });
    const double w1 = s.find(1)->work_published, w2 = s.find(2)->work_published;
    CHECK(s.find(3)->work_published >= std::min(w1, w2) - max_chunk);
    CHECK(s.find(3)->work_published <= std::max(w1, w2));
    size_t n1 = 0, n2 = 0, n3 = 0;
    const size_t mark = d.log.size();
    for (int it = 0; it < 600; ++it) {
        d.publish();
        d.run(8, false);
        d.collect();
    }
    for (size_t i = mark; i < d.log.size(); ++i) {
        const Chunk &c = d.log[i];
        (c.ticket == 1 ? n1 : c.ticket == 2 ? n2 : n3) += 1;
    }
    CHECK(n2 > 0 && n3 > 0 && n1 > 0);
    CHECK(n2 * 10 >= n3 * 8 && n3 * 10 >= n2 * 8);  // equal-cost chunks: equal counts, within 20 %
}

static void check_waiting_bound()
{
    printf("publication: chunks waiting for a workgroup hold under the slack; a late shot is not queued behind them\n");
    const int n_wg = 16;
    const double big = 256.0 * 200000;  // one tile per chunk: 5.1e7 terms
    Scheduler s(1 << 30, 1 << 22, 8, n_wg, 1 << 16);
    Device d(s);
    CHECK(s.slack() == 0.5 * n_wg * CHUNK_TERMS && s.depth() == 2 * (size_t)n_wg);
    s.submit(shot(1, 4096, 100000, 200000));
    s.admit([](Work &) { return 0; });
    for (int it = 0; it < 50; ++it) {
        d.publish();
        // the chunk that crossed the slack is the only one past it
        CHECK(s.in_flight() <= (size_t)n_wg || s.waiting_work() < s.slack() + big);
        CHECK(s.in_flight() <= (size_t)n_wg + 1);
        d.run(3, false);
        d.collect();
    }
    // a small shot admitted now gets the next free workgroup: its first chunk
    // is published as soon as one of the in-flight chunks finishes
    d.publish();
    const size_t mark = d.log.size();
    s.submit(shot(2, 4096, 64, 100));
    s.admit([](Work &) { return 0; });
    d.run(1, false);
    d.collect();
    d.publish();
    bool seen = false;
    for (size_t i = mark; i < d.log.size(); ++i) seen = seen || d.log[i].ticket == 2;
    CHECK(seen);
    // with cheap chunks only, the count bound (depth) is the one that binds
    Scheduler t(1 << 30, 1 << 22, 8, n_wg, 1 << 16);
    Device e(t);
    t.submit(shot(3, 4096, 100000, 10));
    t.admit([](Work &) { return 0; });
    e.publish();
    CHECK(t.in_flight() == t.depth());
}

static void check_shortest_remaining()
{
    printf("publication, shortest remaining: the shot with the least work left goes first; a small late shot overtakes\n");
    const int n_wg = 8;
    Scheduler s(1 << 30, 1 << 22, 8, n_wg, 1 << 16, POLICY_SHORTEST_REMAINING);
    Device d(s);
    CHECK(s.policy() == POLICY_SHORTEST_REMAINING);
    s.submit(shot(1, 4096, 2000, 100000));  // large: 5.1e10 terms
    s.submit(shot(2, 4096, 300, 100000));   // medium
    s.admit([](Work &) { return 0; });
    // the medium shot, with less left, takes every chunk until it is all published
    for (int it = 0; it < 200 && s.find(2)->next_unit < s.find(2)->n_units; ++it) {
        d.publish();
        d.run(4, false);
        d.collect();
    }
    uint64_t last2 = 0, first1 = UINT64_MAX;
    for (const Chunk &c : d.log) {
        if (c.ticket == 2) last2 = std::max<uint64_t>(last2, c.seq);
        if (c.ticket == 1) first1 = std::min<uint64_t>(first1, c.seq);
    }
    CHECK(first1 > last2);
    // a small shot admitted now overtakes the large one at the next publication
    s.submit(shot(3, 4096, 16, 1000));
    s.admit([](Work &) { return 0; });
    const size_t mark = d.log.size();
    d.run(1, false);
    d.collect();
    d.publish();
    CHECK(d.log.size() > mark && d.log[mark].ticket == 3);
    // work left reaches zero exactly when the last chunk of every phase is out
    for (int it = 0; it < 100000 && (s.find(1)->state != DONE || s.find(3)->state != DONE ||
                                     s.find(2)->state != DONE); ++it) {
        d.publish();
        d.run(5, true);
        d.collect();
    }
    for (uint64_t t = 1; t <= 3; ++t) CHECK(s.find(t)->state == DONE && std::abs(s.find(t)->work_left) < 1.0);
    // split shots and backgrounds count their reduce and background phases
    Scheduler u(1 << 30, 1 << 22, 8, n_wg, 1 << 16, POLICY_SHORTEST_REMAINING);
    Device e(u);
    u.submit(shot(4, 4096, 40, 50000, 8, 4096, 500));
    u.admit([](Work &) { return 0; });
    CHECK(u.find(4)->work_left == 40.0 * 256 * (50000 + 8 + 500));
    for (int it = 0; it < 100000 && u.find(4)->state != DONE; ++it) {
        e.publish();
        e.run(3, true);
        e.collect();
    }
    CHECK(u.find(4)->state == DONE && std::abs(u.find(4)->work_left) < 1.0);
}

static void check_cancel()
{
    printf("cancel: queued shots only; the ones behind move up; space untouched\n");
    Scheduler s(1000, 1 << 20, 8, 4, 1 << 16);
    Device d(s);
    s.submit(shot(1, 600, 4, 1000));
    s.submit(shot(2, 600, 4, 1000));
    s.submit(shot(3, 300, 4, 1000));
    s.admit([](Work &) { return 0; });
    CHECK(s.find(1)->state == RUNNING && s.find(2)->state == QUEUED);
    CHECK(!s.cancel(1));                    // admitted: not cancellable
    CHECK(!s.cancel(99));                   // unknown
    CHECK(s.cancel(2));                     // queued head behind the running shot
    CHECK(s.find(2) == nullptr);
    s.admit([](Work &) { return 0; });
    CHECK(s.find(3)->state == RUNNING);     // moved up and fits beside shot 1
    for (int i = 0; i < 1000 && (s.find(1)->state != DONE || s.find(3)->state != DONE); ++i) {
        d.publish();
        d.run(10, true);
        d.collect();
    }
    for (const Chunk &c : d.log) CHECK(c.ticket != 2);
    CHECK(s.release(1) && s.release(3));
    CHECK(s.dev_arena().free_blocks().size() == 1 && s.dev_arena().free_blocks().begin()->second == 1000);
    CHECK(s.host_arena().free_blocks().begin()->second == (1u << 20));
}

static void check_ring_sequence()
{
    printf("ring: sequence numbers increase by one across many wraps\n");
    Scheduler s(1 << 30, 1 << 22, 4, 2, 16);  // tiny ring: depth min(15, 4)
    Device d(s);
    s.submit(shot(1, 4096, 20000, 10));
    s.admit([](Work &) { return 0; });
    CHECK(s.depth() == 4);
    for (int it = 0; it < 10000 && s.find(1)->state != DONE; ++it) {
        d.publish();
        CHECK(s.in_flight() <= 4);
        d.run(3, true);
        d.collect();
    }
    CHECK(s.find(1)->state == DONE);
    for (size_t i = 0; i < d.log.size(); ++i) CHECK(d.log[i].seq == i);
    CHECK(d.log.size() > 16 * 10);
}

static void check_ring_slot_reuse()
{
    printf("ring: a slow chunk held while many short ones finish never shares its slot\n");
    const uint32_t ring = 16;
    Scheduler s(1 << 30, 1 << 22, 4, 2, ring);  // depth min(15, 4)
    Device d(s);
    s.submit(shot(1, 4096, 20000, 10));
    s.admit([](Work &) { return 0; });
    d.publish();
    CHECK(!d.pending.empty());
    const Chunk slow = d.pending.front();  // held in flight throughout
    uint64_t max_seq = 0;
    for (int it = 0; it < 200; ++it) {
        d.publish();
        // every chunk in flight (the slow one and the pending ones) has its
        // own slot: sequence numbers within `ring` of the oldest
        std::set<uint64_t> slots;
        slots.insert(slow.seq % ring);
        for (const Chunk &c : d.pending) {
            if (c.seq == slow.seq) continue;
            CHECK(c.seq - slow.seq < ring);
            CHECK(slots.insert(c.seq % ring).second);
            max_seq = std::max<uint64_t>(max_seq, c.seq);
        }
        // finish everything but the slow chunk
        for (size_t k = 0; k < d.pending.size();) {
            if (d.pending[k].seq == slow.seq) {
                ++k;
                continue;
            }
            d.done.insert(d.pending[k].seq);
            d.pending.erase(d.pending.begin() + k);
        }
        d.collect();
    }
    CHECK(max_seq == slow.seq + ring - 1);  // publication stopped at the slot bound
    CHECK(s.find(1)->state == RUNNING);
    // once the slow chunk finishes, publication resumes and the shot completes
    d.done.insert(slow.seq);
    d.pending.erase(std::find_if(d.pending.begin(), d.pending.end(), [&](const Chunk &c) { return c.seq == slow.seq; }));
    for (int it = 0; it < 100000 && s.find(1)->state != DONE; ++it) {
        d.collect();
        d.publish();
        d.run(4, true);
    }
    d.collect();
    CHECK(s.find(1)->state == DONE);
}

// The segment rule: the fewest segments that keep a unit's pixel-terms
// within the budget, at most the shortest part's outer iterations.
static void check_segments_of()
{
    printf("segments: count from the unit's pixel-terms, bounded by its outer iterations\n");
    CHECK(SEGMENT_TERMS == 2 * CHUNK_TERMS);
    const uint64_t B = 4 * CHUNK_TERMS;  // a budget of 2^22 for the exact counts below
    CHECK(segments_of(100, 1, 1200, B) == 1);                  // 25600 pixel-terms
    CHECK(segments_of(240000, 1, 1200, B) == 15);              // 6.1e7 / 4.2e6 -> 14.6
    CHECK(segments_of(240000, 2, 1200, B) == 8);               // half per part
    CHECK(segments_of(16384, 1, 1200, B) == 1);                // exactly the budget
    CHECK(segments_of(16385, 1, 1200, B) == 2);
    CHECK(segments_of(240000, 1, 12, B) == 12);                // one outer iteration each
    CHECK(segments_of(240000, 5, 12, B) == 2);                 // parts of 2 or 3 iterations
    CHECK(segments_of(240000, 1, 1200, 1 << 10) == 1200);
    CHECK(segments_of(0, 1, 1, B) == 1);
    CHECK(segments_of(240000, 1, 1200, SEGMENT_TERMS) == 30);              // the default: 6.1e7 / 2.1e6
    for (uint64_t tpp : {1ull, 977ull, 60000ull, 240000ull, 6553600ull})
        for (int32_t split : {1, 3, 64})
            for (int64_t n_outer : {64ll, 1200ll, 51200ll}) {
                if (split > n_outer) continue;
                const int32_t k = segments_of(tpp, split, n_outer, SEGMENT_TERMS);
                const uint64_t per_unit = TILE_PIXELS * (tpp / split);
                CHECK(k >= 1 && k <= n_outer / split);
                // within the budget, unless the outer iterations ran out;
                // and no fewer would do
                CHECK((per_unit + k - 1) / k <= SEGMENT_TERMS || k == n_outer / split);
                CHECK(k == 1 || (per_unit + k - 2) / (k - 1) > SEGMENT_TERMS);
            }
}

int main()
{
    check_arena();
    check_segments_of();
    check_fifo_admission();
    check_units_and_depth();
    check_fair_share();
    check_waiting_bound();
    check_shortest_remaining();
    check_cancel();
    check_ring_sequence();
    check_ring_slot_reuse();
    printf("all scheduler checks passed\n");
    return 0;
}
